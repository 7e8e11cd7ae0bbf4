"""GPU parity of the Hertz-Mindlin contact with particle rotation (Sec. 2.3),
in its no-slip limit and with the Mindlin-Deresiewicz micro-slip factors,
against the FP64 oracle, through the C ABI: clusters of touching and
approaching particles with initial spins and wall contacts, one step and
then several more with the tangential-force history carried between steps;
an island larger than a wave; both island set-up paths.

Bounds, after one step and after five: fluid velocity 1e-5 relative (L2)
and density 1e-6; particle positions and velocities 1e-5 relative, angular
velocities 1e-5 relative (L2), as for the other contact models.
"""
import numpy as np
import pytest

from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1407_6704_amd import pibm
    pibm.load()
    return pibm


def _flush(msg):
    print(msg, flush=True)


def _clusters(D, n, seed, nclusters):
    rng = np.random.default_rng(seed)
    pts = []
    for c in range(nclusters):
        k = 2 + c % 5
        base = np.array([rng.uniform(3, n[a] - 3 - 0.5 * k) for a in range(D)])
        for i in range(k):
            p = base.copy()
            p[0] += 0.499 * i
            p[1] += 0.03 * (i % 2)
            pts.append(p)
    for i in range(6):                       # resting on the bottom wall (about the rest overlap)
        p = np.array([rng.uniform(2, n[a] - 2) for a in range(D)])
        p[D - 1] = 0.25 - 2e-6
        pts.append(p)
    X = np.array(pts).T.astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    U = (3e-4 * rng.standard_normal((D, npart))).astype(np.float32).astype(np.float64)
    U[D - 1, -6:] = 0.0                      # the wall particles slide and roll along the wall
    W = (2e-3 * rng.standard_normal((3, npart))).astype(np.float32).astype(np.float64)
    if D == 2:
        W[:2] = 0.0
    return X, U, W, np.full(npart, 0.5), np.full(npart, 2.5)


def _compare(P, orc, cfg, X, U, W, d, rp, steps_list):
    D = X.shape[0]
    sim = P.Sim(cfg, X.shape[1])
    sim.set_particles(X, U, d, rp)
    sim.set_rotation(W if D == 3 else W[2:3])
    oc = G.oracle_cfg(orc, cfg)
    f = G.to_oracle_f(orc, cfg.lattice, sim.read_populations())
    Xo, Uo, Wo, hist = X.copy(), U.copy(), W.copy(), None
    res = []
    for steps in steps_list:
        for _ in range(steps):
            out = orc.step_hm(oc, f, Xo, Uo, Wo, d, rp, hist)
            f, Xo, Uo, Wo, hist = out["f"], out["X"], out["U"], out["W"], out["hist"]
        sim.step(steps)
        sim.synchronize()
        got = sim.read_particles()
        w = sim.read_rotation()
        wref = Wo if D == 3 else Wo[2:3]
        eu, er, _ = G.field_errors(orc, cfg.lattice, sim.read_populations(), f, sim.N)
        disp = np.abs(Xo - X).max()
        ex = np.abs(got["x"] - Xo).max() / disp
        ev = np.linalg.norm(got["v"] - Uo) / np.linalg.norm(Uo)
        ew = np.linalg.norm(w - wref) / np.linalg.norm(wref)
        efc = np.linalg.norm(got["f_contact"] - out["fc"]) / max(np.linalg.norm(out["fc"]), 1e-30)
        _flush(f"  {steps} steps: eps_u={eu:.2e} eps_rho={er:.2e} dX={ex:.2e} dU={ev:.2e} dW={ew:.2e} "
               f"dFc={efc:.2e} contacts={len(hist[0])} active={sim.diagnostics()['active']}")
        res.append(dict(eu=eu, er=er, ex=ex, ev=ev, ew=ew, efc=efc, nh=len(hist[0]), sim=sim))
    return res


@pytest.mark.parametrize("contact", ["hertz_mindlin", "hertz_mindlin_microslip"])
@pytest.mark.parametrize("lat", [9, 19])
def test_mindlin_contacts_match_oracle(P, orc, lat, contact):
    _flush(f"Hertz-Mindlin contacts {lat} {contact}")
    D = 2 if lat == 9 else 3
    n = (40, 30, 1) if D == 2 else (16, 14, 18)
    X, U, W, d, rp = _clusters(D, n, 41, 12 if D == 2 else 10)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    cfg = P.make_config(lattice=lat, n=n, tau=0.8, gravity=g, n_sub=400, contact=contact, young=1e3,
                        poisson=0.33, friction=0.33)
    r1, r5 = _compare(P, orc, cfg, X, U, W, d, rp, [1, 4])
    assert r1["nh"] > 5 and r5["nh"] >= 4                # contacts carried between steps
    assert r1["eu"] <= 1e-5 and r1["er"] <= 1e-6
    assert r1["ex"] <= 1e-5 and r1["ev"] <= 1e-5 and r1["ew"] <= 1e-5
    assert r5["ex"] <= 1e-5 and r5["ev"] <= 1e-5 and r5["ew"] <= 1e-5 and r5["eu"] <= 1e-5


@pytest.mark.parametrize("contact", ["hertz_mindlin", "hertz_mindlin_microslip"])
def test_mindlin_big_island(P, orc, contact):
    """A chain of 120 particles in alternating contact: one island larger
    than a wave (the workgroup-per-island path)."""
    _flush(f"Hertz-Mindlin big island {contact}")
    k = 120
    x = [10.0]
    for i in range(1, k):
        x.append(x[-1] + 0.5 - (0.0004 if i % 2 == 1 else -0.004))
    X = np.zeros((2, k))
    X[0], X[1] = x, 6.0
    X = X.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(3)
    U = np.zeros((2, k))
    U[1] = 1e-4 * rng.standard_normal(k)
    U = U.astype(np.float32).astype(np.float64)
    W = np.zeros((3, k))
    W[2] = (1e-3 * rng.standard_normal(k)).astype(np.float32)
    cfg = P.make_config(lattice=9, n=(200, 12, 1), tau=0.8, gravity=(0, -1e-5, 0), n_sub=300,
                        contact=contact, young=1.0, poisson=0.33, friction=0.33)
    r1, r2 = _compare(P, orc, cfg, X, U, W, np.full(k, 0.5), np.full(k, 2.5), [1, 1])
    assert r1["sim"].diagnostics()["active"] == k
    assert r1["nh"] > 0 and r1["efc"] <= 1e-5           # the contacts acted in the first step
    for r in (r1, r2):
        assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["ew"] <= 1e-5 and r["eu"] <= 1e-5


@pytest.mark.parametrize("lat", [9, 19])
def test_mindlin_setup_paths_agree(P, lat):
    """One-workgroup and multi-kernel island set-up: bitwise identical
    states and spins over several steps."""
    _flush(f"Hertz-Mindlin set-up paths {lat}")
    D = 2 if lat == 9 else 3
    n = (40, 30, 1) if D == 2 else (16, 14, 18)
    X, U, W, d, rp = _clusters(D, n, 7, 14)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    out = []
    for mode in (1, 2):
        cfg = P.make_config(lattice=lat, n=n, tau=0.8, gravity=g, n_sub=200, contact="hertz_mindlin", young=1e3,
                            island_setup=mode)
        sim = P.Sim(cfg, X.shape[1])
        sim.set_particles(X, U, d, rp)
        sim.set_rotation(W if D == 3 else W[2:3])
        for k in (1, 3, 2):
            sim.step(k)
        p = sim.read_particles()
        out.append((p["x"], p["v"], p["f_contact"], sim.read_rotation(), sim.read_populations()))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_rotation_entry_points(P):
    """Rotation is refused for other contact models and after the first
    step; set_particles clears it."""
    cfg = P.make_config(lattice=9, n=(16, 16, 1), contact="lsd")
    sim = P.Sim(cfg, 2)
    X = np.array([[5.0, 9.0], [5.0, 9.0]])
    sim.set_particles(X, np.zeros((2, 2)), np.full(2, 0.5), np.full(2, 2.0))
    with pytest.raises(P.PibmError):
        sim.read_rotation()
    cfg = P.make_config(lattice=9, n=(16, 16, 1), contact="hertz_mindlin", young=1e3)
    sim = P.Sim(cfg, 2)
    sim.set_particles(X, np.zeros((2, 2)), np.full(2, 0.5), np.full(2, 2.0))
    sim.set_rotation(np.array([[1e-3, -2e-3]]))
    assert np.allclose(sim.read_rotation(), [[1e-3, -2e-3]])
    sim.step(2)
    # free particles keep their spin (no hydrodynamic torque)
    assert np.allclose(sim.read_rotation(), [[1e-3, -2e-3]])
    with pytest.raises(P.PibmError):
        sim.set_rotation(np.zeros((1, 2)))
    sim.set_particles(X, np.zeros((2, 2)), np.full(2, 0.5), np.full(2, 2.0))
    assert np.array_equal(sim.read_rotation(), np.zeros((1, 2)))
