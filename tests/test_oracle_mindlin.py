"""Pins of the oracle's Hertz-Mindlin contact with rotation (contact = 4,
Sec. 2.3, tangential law in its no-slip limit with the Coulomb bound)
against rigid-body mechanics that does not depend on the contact law's
details:

* a sphere (disk) launched sliding on a flat wall: while it slides the
  friction force is mu F_n against the motion; the angular momentum about
  the contact point, m R U + I W, is conserved exactly; it ends rolling at
  5/7 (2/3) of the launch speed, I = 2/5 m R^2 (1/2 m R^2);
* on an incline with tan(theta) < 7/2 mu (3 mu for a disk) it rolls with
  acceleration 5/7 g sin(theta) (2/3 for a disk); above that it slides with
  g (sin(theta) - mu cos(theta));
* an oblique impact of two spheres conserves linear momentum exactly and
  does not gain energy.
No fluid acts (zero interpolated moments), so the buoyant weight
(1 - rho0/rho_p) m g is the only body force."""
import math

import numpy as np
import pytest

E, NU, MU = 1e-3, 0.33, 0.33


def _cfg(orc, D, g, n_sub=10, n=None):
    n = n or ((60, 12, 1) if D == 2 else (60, 12, 12))
    return orc.make_cfg(lattice=9 if D == 2 else 19, n=n, n_sub=n_sub, contact="hertz_mindlin", young=E,
                        poisson=NU, friction=MU, two_way=0, skin=0.05, gravity=g)


def _rest_overlap(m_geff, R):
    """Overlap at which the Hertz wall force carries the buoyant weight."""
    kw = 4.0 / 3.0 * E / (2 * (1 - NU * NU)) * math.sqrt(R)
    return (m_geff / kw) ** (2.0 / 3.0)


def _run(orc, cfg, X, U, W, d, rp, steps):
    D = X.shape[0]
    hist = None
    rho_i, j_i = np.zeros(1), np.zeros((D, 1))
    out = []
    for _ in range(steps):
        X, U, W, gbar, fc, vmax, hist = orc.dem_hm(cfg, X, U, W, d, rp, rho_i, j_i, hist)
        out.append((X.copy(), U.copy(), W.copy(), fc.copy()))
    return out


@pytest.mark.parametrize("D", [3, 2])
def test_sliding_to_rolling(orc, D):
    g, rp, d, v0 = 1e-5, 2.0, 0.5, 1e-3
    R = 0.5 * d
    grav = [0.0, 0.0, 0.0]
    grav[D - 1] = -g
    cfg = _cfg(orc, D, grav)
    m = orc.mass(D, d, rp)
    I = (0.4 if D == 3 else 0.5) * m * R * R
    geff = (1 - 1 / rp) * g
    X = np.full((D, 1), 6.0)
    X[0, 0] = 10.0
    X[D - 1, 0] = R - _rest_overlap(m * geff, R)
    U = np.zeros((D, 1))
    U[0, 0] = v0
    W = np.zeros((3, 1))
    # the spin that rolls along +x: W_y (3D, W x (-R e_z) = -R W_y e_x) or W_z (2D, -R e_y)
    wi = 1 if D == 3 else 2
    sgn = 1.0 if D == 3 else -1.0
    hist = _run(orc, cfg, X, U, W, np.array([d]), np.array([rp]), 1500)
    L0 = m * R * v0
    Ls = np.array([m * R * h[1][0, 0] + sgn * I * h[2][wi, 0] for h in hist])
    assert np.abs(Ls - L0).max() < 1e-12 * L0
    # sliding phase: kinetic friction mu F_n against the motion
    t_stick = v0 / (geff * MU * (1 + m * R * R / I))
    fx, fn = hist[10][3][0, 0], hist[10][3][D - 1, 0]
    assert 10 < 0.5 * t_stick and abs(fx / fn + MU) < 1e-9
    # (the first ~2 steps load the tangential spring up to the bound)
    du = hist[30][1][0, 0] - hist[10][1][0, 0]
    assert abs(du / (-MU * geff * 20) - 1) < 1e-6
    # rolling: 5/7 (2/3) of v0, no mean slip
    ratio = 1.0 / (1.0 + I / (m * R * R))
    u = np.array([h[1][0, 0] for h in hist[800:]])
    slip = np.array([h[1][0, 0] - sgn * R * h[2][wi, 0] for h in hist[800:]])
    assert abs(u.mean() / (ratio * v0) - 1) < 2e-3
    # stuck: the contact point only oscillates on the tangential spring
    assert np.abs(slip).max() < 0.2 * v0 and abs(slip.mean()) < 0.05 * np.abs(slip).max()


@pytest.mark.parametrize("D", [3, 2])
@pytest.mark.parametrize("tan_over_mu", [1.0, 6.0])
def test_incline(orc, D, tan_over_mu):
    g, rp, d = 1e-5, 2.0, 0.5
    R = 0.5 * d
    th = math.atan(tan_over_mu * MU)
    grav = [0.0, 0.0, 0.0]
    grav[0], grav[D - 1] = g * math.sin(th), -g * math.cos(th)
    cfg = _cfg(orc, D, grav, n=(400, 12, 1) if D == 2 else (400, 12, 12))
    m = orc.mass(D, d, rp)
    I = (0.4 if D == 3 else 0.5) * m * R * R
    geff = (1 - 1 / rp) * g
    X = np.full((D, 1), 6.0)
    X[0, 0] = 10.0
    X[D - 1, 0] = R - _rest_overlap(m * geff * math.cos(th), R)
    hist = _run(orc, cfg, X, np.zeros((D, 1)), np.zeros((3, 1)), np.array([d]), np.array([rp]), 1200)
    t = np.arange(1, len(hist) + 1, dtype=float)
    u = np.array([h[1][0, 0] for h in hist])
    slope = np.polyfit(t[200:], u[200:], 1)[0]
    k = I / (m * R * R)
    if tan_over_mu * MU < (1 + k) / k * MU:      # rolls: a = g sin / (1 + I/(m R^2))
        expect = geff * math.sin(th) / (1 + k)
        assert abs(slope / expect - 1) < 5e-3
    else:                                          # slides
        expect = geff * (math.sin(th) - MU * math.cos(th))
        assert abs(slope / expect - 1) < 1e-6


def test_oblique_pair_impact(orc):
    rp, d, v = np.array([2.0, 3.0]), np.array([0.5, 0.4]), 1e-3
    cfg = _cfg(orc, 3, [0.0, 0.0, 0.0], n_sub=40, n=(12, 12, 12))
    m = np.array([orc.mass(3, d[i], rp[i]) for i in range(2)])
    I = 0.4 * m * (0.5 * d) ** 2
    rc = 0.5 * d.sum()
    X = np.array([[6.0 - 0.5 * rc - 0.01, 6.0 + 0.5 * rc + 0.01], [6.0, 6.0 + 0.3 * rc], [6.0, 6.0]])
    U = np.array([[v, -v * m[0] / m[1]], [0.0, 0.0], [2e-4, -2e-4 * m[0] / m[1]]])
    W = np.array([[0.0, 0.0], [0.0, 0.0], [3e-3, -1e-3]])
    ke0 = 0.5 * (m * (U ** 2).sum(0)).sum() + 0.5 * (I * (W ** 2).sum(0)).sum()
    rho_i, j_i = np.zeros(2), np.zeros((3, 2))
    hist = None
    P0 = (m * U).sum(1)
    touched = False
    for _ in range(300):
        X, U, W, gbar, fc, vmax, hist = orc.dem_hm(cfg, X, U, W, d, rp, rho_i, j_i, hist)
        touched = touched or len(hist[0]) > 0
        assert np.abs((m * U).sum(1) - P0).max() < 1e-18
    ke1 = 0.5 * (m * (U ** 2).sum(0)).sum() + 0.5 * (I * (W ** 2).sum(0)).sum()
    assert touched and len(hist[0]) == 0             # they met and separated
    assert ke1 <= ke0 * (1 + 1e-12)
    assert np.abs(W - np.array([[0, 0], [0, 0], [3e-3, -1e-3]])).max() > 1e-5   # friction spun them


def test_coupled_momentum_bookkeeping(orc):
    """Whole coupled steps with the Hertz-Mindlin contact: fluid plus
    particle momentum changes by exactly the buoyant weights (drag, normal
    and tangential contact forces are internal), and the history carries
    the touching pairs from step to step."""
    n = (20, 20, 20)
    cfg = orc.make_cfg(lattice=19, n=n, tau=0.7, gravity=(0, 0, -1e-4), n_sub=40, contact="hertz_mindlin",
                       young=1e-2, poisson=NU, friction=MU, two_way=1, skin=0.05)
    rng = np.random.default_rng(5)
    X = np.array([[10.0, 10.46, 10.2, 9.5], [10.0, 10.05, 10.42, 9.8], [10.0, 10.1, 10.0, 10.3]])
    U = 1e-4 * rng.standard_normal((3, 4))
    W = 1e-3 * rng.standard_normal((3, 4))
    d = np.array([0.5, 0.5, 0.45, 0.6])
    rp = np.array([2.0, 2.5, 1.5, 2.0])
    m = np.array([orc.mass(3, d[i], rp[i]) for i in range(4)])
    Wp = ((1 - 1 / rp) * m)[None, :] * np.array([0, 0, -1e-4])[:, None]
    f = orc.rest_state(cfg)
    e, w, _ = orc.tables(19)
    N = orc.nnodes(cfg)
    hist = None
    seen = 0
    for step in range(5):
        P0 = e.T.astype(float) @ (f.reshape(-1, N) - w[:, None]).sum(1) + np.r_[(m * U).sum(1)]
        out = orc.step_hm(cfg, f, X, U, W, d, rp, hist)
        f, X, U, W, hist = out["f"], out["X"], out["U"], out["W"], out["hist"]
        seen = max(seen, len(hist[0]))
        P1 = e.T.astype(float) @ (f.reshape(-1, N) - w[:, None]).sum(1) + np.r_[(m * U).sum(1)]
        tol = 8 * 2.0 ** -53 * np.sqrt(N * len(w)) * w.max()
        assert np.allclose(P1 - P0, Wp.sum(1), rtol=0, atol=tol), (step, P1 - P0, Wp.sum(1))
    assert seen >= 2
