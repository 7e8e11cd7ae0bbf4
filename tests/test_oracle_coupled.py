"""Pins of the oracle's whole coupled step (O1..O7).

* momentum bookkeeping (every lattice, both gathers): fluid plus particle
  momentum changes by exactly the buoyant weights sum_p (1 - rho0/rho_p) m_p g per step while the disturbance
  stays away from the walls (drag and contact forces are internal)
* mass conservation with particles and walls
* two-way settling consistency: the terminal speed of a single particle
  equals W' (1/(2 rho0 A_p) + M_self), where M_self is the fluid velocity at
  the particle per unit point force, measured in a separate run that applies
  a fixed spread force and moves no particle (linear response, Re << 1)
* the skin check counts particles whose speed exceeds skin/2
"""
import numpy as np
import pytest


def _buoyant_weight(orc, cfg, d, rp):
    D = orc.D(cfg)
    m = np.array([orc.mass(D, d[i], rp[i]) for i in range(len(d))])
    g = np.array([cfg.gravity[a] for a in range(D)])
    return ((1 - cfg.rho0 / rp) * m)[None, :] * g[:, None], m


@pytest.mark.parametrize("lat,interp", [(9, "delta"), (19, "delta"), (15, "delta"), (15, "lagrange"),
                                        (9, "lagrange")])
def test_momentum_bookkeeping(orc, lat, interp):
    D = 2 if lat == 9 else 3
    n = (28, 28, 1) if D == 2 else (22, 22, 22)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-4
    cfg = orc.make_cfg(lattice=lat, n=n, tau=0.7, gravity=g, n_sub=40, two_way=1, kn=1e-2, interp=interp)
    rng = np.random.default_rng(11)
    npart = 9 if D == 2 else 12
    c = np.array([n[a] / 2 for a in range(D)])
    grid = np.stack(np.meshgrid(*[np.arange(3) - 1.0] * D, indexing="ij")).reshape(D, -1)
    X = c[:, None] + 1.3 * grid[:, :npart] + rng.uniform(-0.1, 0.1, (D, npart))
    X[:, 1] = X[:, 0]
    X[0, 1] += 0.42                                   # one pair in contact
    U = 1e-4 * rng.standard_normal((D, npart))
    d = rng.uniform(0.4, 0.6, npart)
    d[0] = d[1] = 0.5
    rp = rng.uniform(1.5, 3.0, npart)
    Wp, m = _buoyant_weight(orc, cfg, d, rp)
    f = orc.rest_state(cfg)
    e, w, _ = orc.tables(lat)
    N = orc.nnodes(cfg)

    def totals(f):
        # deviations from the rest state keep the FP64 sums free of cancellation
        dev = f.reshape(-1, N) - w[:, None]
        return dev.sum(), e.T.astype(float) @ dev.sum(axis=1)

    for step in range(5):
        m0, P0 = totals(f)
        Pp0 = (m * U).sum(axis=1)
        out = orc.step(cfg, f, X, U, d, rp)
        m1, P1 = totals(out["f"])
        Pp1 = (m * out["U"]).sum(axis=1)
        dP = (P1[:D] - P0[:D]) + (Pp1 - Pp0)
        # rounding of the FP64 population updates: a random walk of N Q terms
        # of size 2^-53 max(w) (1e-15 .. 1e-14 here; the buoyant weight is 1e-4)
        tol = 8 * 2.0 ** -53 * np.sqrt(N * len(w)) * w.max()
        assert np.allclose(dP, Wp.sum(axis=1), rtol=0, atol=tol), (step, dP, Wp.sum(axis=1))
        assert abs(m1 - m0) < 10 * N * len(w) * 2.0 ** -53
        # the fluid received exactly the sub-step mean momentum exchange
        Fsum = out["F"].sum(axis=1)
        A = np.pi * d ** 2 / 4
        assert np.allclose(Fsum, (A * out["gbar"]).sum(axis=1), atol=1e-16)
        f, X, U = out["f"], out["X"], out["U"]
    assert np.abs(out["fc"]).max() > 0                # the contact did act


def test_mass_conservation_coupled(orc):
    cfg = orc.make_cfg(lattice=9, n=(24, 20, 1), tau=0.6, gravity=(0, -1e-4, 0), n_sub=20)
    rng = np.random.default_rng(12)
    npart = 30
    X = np.stack([rng.uniform(1, 23, npart), rng.uniform(1, 19, npart)])
    d = np.full(npart, 0.3)
    f = orc.rest_state(cfg)
    m0, _ = orc.fluid_totals(cfg, f)
    U = np.zeros((2, npart))
    for _ in range(50):
        out = orc.step(cfg, f, X, U, d, np.full(npart, 2.5))
        f, X, U = out["f"], out["X"], out["U"]
    m1, _ = orc.fluid_totals(cfg, f)
    assert abs(m1 - m0) < 10 * 50 * 9 * orc.nnodes(cfg) * 2.0 ** -53 * m0


def test_two_way_settling_consistency(orc):
    n = (48, 96, 1)
    d, rp, g, tau = 0.5, 2.5, -1e-6, 0.8
    steps = 2500
    cfg = orc.make_cfg(lattice=9, n=n, tau=tau, gravity=(0, g, 0), n_sub=20, two_way=1)
    X = np.array([[24.3], [48.2]])
    U = np.zeros((2, 1))
    f = orc.rest_state(cfg)
    for _ in range(steps):
        out = orc.step(cfg, f, X, U, np.array([d]), np.array([rp]))
        f, X, U = out["f"], out["X"], out["U"]
    m, A = orc.mass(2, d, rp), orc.area(d)
    W = (1 - 1 / rp) * m * g
    # run B: fixed point force W at the final position, no particle
    cfgB = orc.make_cfg(lattice=9, n=n, tau=tau, contact="none", two_way=1)
    FB = orc.spread(cfgB, X, np.array([[0.0], [W]]))
    fB = orc.rest_state(cfgB)
    for _ in range(steps):
        fB = orc.collide_stream(cfgB, fB, FB)
    rho, j = orc.moments(cfgB, fB)
    ri, ji = orc.interp(cfgB, X, rho, j)
    M_self = ji[1, 0] / ri[0] / W
    Ut = W * (1 / (2 * A) + M_self)
    assert abs(U[1, 0] - Ut) < 1e-3 * abs(Ut)
    # the self-induced part is a large share: this is not the one-way result
    assert abs(U[1, 0] - W / (2 * A)) > 0.3 * abs(Ut)


def test_skin_check_counts_fast_particles(orc):
    cfg = orc.make_cfg(lattice=9, n=(16, 16, 1), n_sub=10, skin=0.05)
    X = np.array([[4.0, 8.0, 12.0], [8.0, 8.0, 8.0]])
    U = np.array([[0.0, 0.03, 0.0], [0.0, 0.0, -0.024]])
    out = orc.step(cfg, orc.rest_state(cfg), X, U, np.full(3, 0.4), np.full(3, 2.5))
    assert out["nskin"] == 1


@pytest.mark.parametrize("lat", [9, 19])
def test_threads_do_not_change_results(orc, lat):
    """The node loops run on several threads; every node's arithmetic is the
    same and no sum crosses nodes, so a coupled step with contacts and
    walls is bitwise the same on one thread and on several."""
    D = 2 if lat == 9 else 3
    n = (37, 29, 1) if D == 2 else (15, 13, 11)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    cfg = orc.make_cfg(lattice=lat, n=n, tau=0.7, gravity=g, n_sub=50, two_way=1,
                       fluid_force=(1e-6, -2e-6, 5e-7 if D == 3 else 0.0))
    rng = np.random.default_rng(5)
    npart = 40
    X = np.stack([rng.uniform(0.4, n[a] - 0.4, npart) for a in range(D)])
    X[:, 1] = X[:, 0]
    X[0, 1] += 0.45                                     # a pair in contact
    X[D - 1, 2] = 0.2                                   # a wall contact
    U = 1e-4 * rng.standard_normal((D, npart))
    d = np.full(npart, 0.5)
    rp = np.full(npart, 2.5)
    _, w, _ = orc.tables(lat)
    N = orc.nnodes(cfg)
    f0 = (w[:, None] * (1.0 + 1e-3 * rng.standard_normal((len(w), N)))).reshape(-1)
    runs = []
    try:
        for t in (1, 3, max(orc.threads(), 2)):
            orc.set_threads(t)
            out = orc.step(cfg, f0, X, U, d, rp)
            rho, j = orc.moments(cfg, out["f"])
            runs.append((out["f"], out["X"], out["U"], out["F"], rho, j))
    finally:
        orc.set_threads(0)
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)
