"""Pins of the oracle's fixed obstacle points (the hybrid IBM-PIBM bodies of
Sec. 3.3): points of fixed bodies never move, and they act as external
supports, so over a coupled step the fluid plus moving-particle momentum
changes by the moving particles' buoyant weights minus every force the
fixed points take (hydrodynamic -A_l gbar_l, with each point's own area
A_l, plus the contact reactions).  Checked with the linear spring-dashpot,
Hertz and Hertz-Mindlin contacts, in 2D and 3D."""
import numpy as np
import pytest


def _scene(orc, D, contact):
    # walls far enough that no disturbance reaches them within the steps taken
    n = (24, 24, 1) if D == 2 else (24, 24, 24)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-4
    cfg = orc.make_cfg(lattice=9 if D == 2 else 19, n=n, tau=0.7, gravity=g, n_sub=60, contact=contact,
                       kn=1e-2, young=1e-2, poisson=0.33, friction=0.33, two_way=1, skin=0.05)
    rng = np.random.default_rng(9)
    c = np.array([n[a] / 2 for a in range(D)])
    # a fixed "sphere": 24 surface points of radius 1.5 with equal shares of its area,
    # and three fixed PIBM points in a row
    k = 24
    t = np.arange(k) + 0.5
    if D == 3:
        z = 1 - 2 * t / k
        ph = np.pi * (1 + 5 ** 0.5) * t
        S = np.stack([np.sqrt(1 - z * z) * np.cos(ph), np.sqrt(1 - z * z) * np.sin(ph), z])
        shell_area = 4 * np.pi * 1.5 ** 2 / k
    else:
        S = np.stack([np.cos(2 * np.pi * t / k), np.sin(2 * np.pi * t / k)])
        shell_area = 2 * np.pi * 1.5 / k
    Xs = c[:, None] + 1.5 * S
    Xc = c[:, None] + np.array([[3.0, 3.5, 4.0]] + [[0.0] * 3] * (D - 1))
    # moving particles: one resting on top of the shell, one touching a cube point, two free
    top = c.copy()
    top[D - 1] += 1.5 + 0.25 + 0.2 - 0.002
    nearc = Xc[:, 0].copy()
    nearc[D - 1] += 0.45
    Xm = np.stack([top, nearc, c + 5.0, c - 5.0], axis=1)
    X = np.concatenate([Xs, Xc, Xm], axis=1)
    npart = X.shape[1]
    d = np.concatenate([np.full(k, 0.4), np.full(3, 0.5), np.array([0.4, 0.5, 0.4, 0.6])])
    rp = np.concatenate([np.full(k + 3, 1.0), np.array([2.0, 2.5, 1.5, 2.0])])
    fixed = np.concatenate([np.ones(k + 3, np.int32), np.zeros(4, np.int32)])
    area = np.concatenate([np.full(k, shell_area), np.full(3, np.pi * 0.25 ** 2), np.zeros(4)])
    U = np.zeros((D, npart))
    U[:, k + 3:] = 1e-4 * rng.standard_normal((D, 4))
    return cfg, X, U, d, rp, fixed, area


@pytest.mark.parametrize("D,contact", [(2, "lsd"), (3, "lsd"), (3, "hertz"), (3, "hertz_mindlin"),
                                       (2, "hertz_mindlin"), (3, "hertz_mindlin_microslip")])
def test_fixed_points_are_supports(orc, D, contact):
    cfg, X, U, d, rp, fixed, area = _scene(orc, D, contact)
    N = orc.nnodes(cfg)
    e, w, _ = orc.tables(cfg.lattice)
    mv = fixed == 0
    m = np.array([orc.mass(D, d[i], rp[i]) for i in range(len(d))])
    g = np.array(list(cfg.gravity)[:D])
    Wp = ((1 - cfg.rho0 / rp[mv]) * m[mv])[None, :] * g[:, None]
    f = orc.rest_state(cfg)
    W = np.zeros((3, len(d)))
    W[2, mv] = 1e-3
    hist = None
    X0 = X.copy()
    touched = 0
    for step in range(3):
        P0 = e[:, :D].T.astype(float) @ (f.reshape(-1, N) - w[:, None]).sum(1) + (m[mv] * U[:, mv]).sum(1)
        out = orc.step_full(cfg, f, X, U, d, rp, W=W, hist=hist, fixed=fixed, area=area)
        f, X, U, W, hist = out["f"], out["X"], out["U"], out["W"], out["hist"]
        P1 = e[:, :D].T.astype(float) @ (f.reshape(-1, N) - w[:, None]).sum(1) + (m[mv] * U[:, mv]).sum(1)
        # forces on the fixed points: hydrodynamic and contact reactions
        on_fixed = (-(area[~mv] * out["gbar"][:, ~mv]) + out["fc"][:, ~mv]).sum(1)
        tol = 8 * 2.0 ** -53 * np.sqrt(N * len(w)) * w.max() + 1e-18
        assert np.allclose(P1 - P0, Wp.sum(1) - on_fixed, rtol=0, atol=tol), (step, P1 - P0, Wp.sum(1), on_fixed)
        touched += int(np.abs(out["fc"][:, ~mv]).max() > 0)
    # fixed points never move or spin
    assert np.array_equal(X[:, ~mv], X0[:, ~mv]) and np.all(U[:, ~mv] == 0) and np.all(W[:, ~mv] == 0)
    assert touched == 3                                   # the supports carried contacts every step


@pytest.mark.parametrize("contact", ["lsd", "hertz"])
def test_impact_on_a_fixed_point(orc, contact):
    """A fixed point is a partner of infinite mass: a head-on impact rebounds
    with the restitution 0.9 of the spring-dashpot (damping from the moving
    particle's own mass, as at a wall), or elastically for Hertz with the
    largest overlap of Hertz theory for m* = m and R* = R R_f / (R + R_f)."""
    import math
    from scipy.integrate import quad

    v, d, df = 1e-3, np.array([0.5, 0.3]), 0.3
    cfg = orc.make_cfg(lattice=19, n=(10, 10, 10), n_sub=400, contact=contact, kn=1e-2, restitution=0.9,
                       young=2e-3, poisson=0.33, two_way=0, skin=0.05)
    rc = 0.5 * (d[0] + d[1])
    X = np.array([[5.0 - rc - 0.02, 5.0], [5.0, 5.0], [5.0, 5.0]])
    U = np.array([[v, 0.0], [0.0, 0.0], [0.0, 0.0]])
    rp = np.array([2.0, 1.0])
    fixed = np.array([0, 1], np.int32)
    W = np.zeros((3, 2))
    rho_i, j_i = np.zeros(2), np.zeros((3, 2))
    ov = []
    for _ in range(400):
        X, U, W, gbar, fc, vmax, _h = orc.dem_hm(cfg, X, U, W, d, rp, rho_i, j_i, fixed=fixed)
        ov.append(rc - abs(X[0, 1] - X[0, 0]))
    assert X[0, 1] == 5.0 and U[0, 1] == 0.0
    if contact == "lsd":
        assert abs(-U[0, 0] / v - 0.9) < 2e-3
    else:
        m = orc.mass(3, d[0], rp[0])
        R, Rf = 0.5 * d[0], 0.5 * df
        Es = 2e-3 / (2 * (1 - 0.33 ** 2))
        dmax = (15 * m * v * v / (16 * Es * math.sqrt(R * Rf / (R + Rf)))) ** 0.4
        assert abs(-U[0, 0] / v - 1) < 1e-3
        assert abs(max(ov) / dmax - 1) < 5e-3
