"""The allocation-free entry point pibm_conservation_noalloc, through the C
ABI: its FP64 mass and momentum equal pibm_conservation's bit for bit (the
same reduction kernels in the same order, with the partial sums in the
library's module-scope scratch instead of the workspace), on two calls in a
row, the second on a smaller context; and the first context still agrees
afterwards (the shared scratch keeps no state between calls)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1407_6704_amd import pibm
    pibm.load()
    return pibm


def _both(sim):
    m0, p0 = C.c_double(), (C.c_double * 3)()
    m1, p1 = C.c_double(), (C.c_double * 3)()
    assert sim.lib.pibm_conservation(sim.ctx, C.byref(m0), p0) == 0
    assert sim.lib.pibm_conservation_noalloc(sim.ctx, C.byref(m1), p1) == 0
    return (m0.value, list(p0)), (m1.value, list(p1))


def _sim(P, lat, n, npart, seed, steps):
    D = 2 if lat == 9 else 3
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(1.0, n[a] - 1.0, npart) for a in range(D)])
    keep = [0]
    for i in range(1, npart):
        r = np.sqrt(((X[:, keep] - X[:, i:i + 1]) ** 2).sum(axis=0))
        if np.all(r > 0.6):
            keep.append(i)
    X = X[:, keep].astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    U = (1e-4 * rng.standard_normal((D, npart))).astype(np.float32).astype(np.float64)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    cfg = P.make_config(lattice=lat, n=n, tau=0.7, gravity=g, n_sub=50, contact="lsd")
    sim = P.Sim(cfg, npart)
    sim.set_particles(X, U, np.full(npart, 0.5), np.full(npart, 2.5))
    sim.step(steps)
    return sim


def test_noalloc_conservation_equals_workspace_path(P):
    print("no-alloc conservation: D3Q19 40x36x32 then D2Q9 16x12", flush=True)
    big = _sim(P, 19, (40, 36, 32), 400, 3, 4)
    a, b = _both(big)
    print(f"  big:   mass {a[0]:.17g} / {b[0]:.17g}  momentum {a[1]} / {b[1]}", flush=True)
    assert a[0] == b[0] and a[1] == b[1]
    assert abs(a[0] - big.N) < 1e-6 * big.N and any(v != 0.0 for v in a[1])
    small = _sim(P, 9, (16, 12, 1), 12, 4, 2)
    a2, b2 = _both(small)
    print(f"  small: mass {a2[0]:.17g} / {b2[0]:.17g}  momentum {a2[1]} / {b2[1]}", flush=True)
    assert a2[0] == b2[0] and a2[1] == b2[1]
    assert abs(a2[0] - small.N) < 1e-6 * small.N
    # the larger context once more, after the smaller one used the scratch
    a3, b3 = _both(big)
    assert a3 == a and b3 == b
