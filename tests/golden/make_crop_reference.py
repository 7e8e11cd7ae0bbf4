"""Write the FP64 oracle's state after 100 coupled steps of the 64^3 crop
(D3Q19, 31,250 spheres with the lognormal diameters of the 256^3 case, seed
3), for the GPU parity test of the crop over 100 steps.

Calls only the oracle and the seeded input generator.  Stored, to keep the
file small: the fluid density deviation and velocity at 32,768 nodes drawn
with a fixed seed, and every particle's displacement and velocity.

    python tests/golden/make_crop_reference.py      # about 15 min, one core
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

STEPS = 100
NSAMPLE = 32768
OUT = os.path.join(HERE, "crop64_fp64_100steps.npz")


def main():
    from oracle import oracle as orc
    from paper_1407_6704_amd import workloads as W

    w = W.C3_CROP
    X, U, d, rp = W.make_particles(w)
    oc = orc.make_cfg(lattice=w.lattice, n=w.n, tau=w.tau, gravity=w.gravity_vec(), contact=w.contact,
                      kn=w.kn, restitution=w.restitution, k_soft=w.k_soft, skin=w.skin, n_sub=w.n_sub,
                      two_way=w.two_way, bin_log2=w.bin_log2)
    f = orc.rest_state(oc)
    Xo, Uo = X.copy(), U.copy()
    for k in range(STEPS):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
        assert out["nskin"] == 0
        print(f"step {k + 1}/{STEPS}", flush=True)
    N = orc.nnodes(oc)
    e, wq, _ = orc.tables(w.lattice)
    fq = f.reshape(-1, N)
    drho = (fq - wq[:, None]).sum(axis=0)
    j = e[:, :3].T.astype(np.float64) @ fq
    u = j / (1.0 + drho)
    nodes = np.sort(np.random.default_rng(12345).choice(N, size=NSAMPLE, replace=False))
    # FP32 keeps ~7 significant digits of each stored quantity, far below
    # the compared tolerances (1e-5 and up, relative)
    np.savez_compressed(OUT, steps=STEPS, nodes=nodes.astype(np.int32), drho=drho[nodes].astype(np.float32),
                        u=u[:, nodes].astype(np.float32), dx=(Xo - X).astype(np.float32),
                        v=Uo.astype(np.float32))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
