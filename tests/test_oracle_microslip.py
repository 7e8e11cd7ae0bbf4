"""Pins of the oracle's Mindlin-Deresiewicz micro-slip law (contact = 5,
Sec. 2.3: dT = 8 G* r_a theta_k d(delta_t) + (-1)^k mu dF_n (1 - theta_k),
with k and theta_k read as in R27) against the closed forms of Mindlin and
Deresiewicz for a contact under a constant normal force P loaded
tangentially along one line (Johnson, Contact Mechanics, Sec. 7.3):

* monotonic loading: T(d) = mu P [1 - (1 - d / d*)^(3/2)], d* = 3 mu P / (16 G* a),
  full sliding (T = mu P) beyond d*;
* unloading from (d_A, T*): T = T* - 2 mu P [1 - (1 - (d_A - d) / (2 d*))^(3/2)];
* reloading from (d_B, T**): T = T** + 2 mu P [1 - (1 - (d - d_B) / (2 d*))^(3/2)],
  which closes the loop at (d_A, T*) and rejoins the loading curve;
* a contact loaded normally with no tangential motion carries no
  tangential force, and one whose normal force grows faster than the
  tangential load stays elastic (no slip zone);
* with mu -> infinity the law is the no-slip law of contact = 4;
* the law does not depend on the frame (a rotated loading gives the
  rotated force), so it is not tied to a coordinate axis;
* whole coupled steps: fluid plus particle momentum changes by exactly the
  buoyant weights (every contact force is internal).
The law is integrated in increments of the tangential displacement; the
closed forms are its limit, so the bounds are a small fraction of mu P set
by the increment count.
"""
import math

import numpy as np
import pytest

E, NU, MU = 1.0, 0.33, 0.33


def _cfg(orc, contact="hertz_mindlin_microslip", mu=MU):
    return orc.make_cfg(lattice=19, n=(12, 12, 12), contact=contact, young=E, poisson=NU, friction=mu,
                        n_sub=1, skin=0.05, two_way=0)


def _gstar():
    G = E / (2 * (1 + NU))
    return G / (2 * (1 - NU * NU))        # 1/G* = (1 - nu^2)/G + (1 - nu^2)/G, as printed


def _setup(P=2e-4, rstar=0.125, delta=None):
    # overlap of a Hertz contact carrying P: P = (4/3) E* sqrt(R*) delta^(3/2)
    Es = E / (2 * (1 - NU * NU))
    if delta is None:
        delta = (P / (4.0 / 3.0 * Es * math.sqrt(rstar))) ** (2.0 / 3.0)
    P = 4.0 / 3.0 * Es * math.sqrt(rstar) * delta ** 1.5
    a = math.sqrt(delta * rstar)
    dstar = 3.0 * MU * P / (16.0 * _gstar() * a)
    return P, rstar, delta, dstar


def _drive(orc, cfg, S, n, t, P, rstar, delta, dd, steps, h=1.0):
    """Tangential displacement increments dd along t (contact point of the
    particle moving by -dd relative to the partner, so the force grows along
    +t); returns the force along t after each increment."""
    out = []
    v = -np.asarray(t) * dd / h
    for _ in range(steps):
        S = orc.tangential_update(cfg, h, n, v, P, rstar, delta, S)
        out.append(float(np.dot(S[:3], t)))
    return S, np.array(out)


def _loading(d, P, dstar):
    return MU * P * (1.0 - np.clip(1.0 - d / dstar, 0.0, None) ** 1.5)


def test_monotonic_loading_and_sliding(orc):
    cfg = _cfg(orc)
    P, rstar, delta, dstar = _setup()
    n, t = np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0])
    S = np.zeros(orc.TS)
    S[9] = P                                   # loaded normally before the tangential load
    N = 20000
    dd = 1.2 * dstar / N
    S, T = _drive(orc, cfg, S, n, t, P, rstar, delta, dd, N)
    d = dd * np.arange(1, N + 1)
    err = np.abs(T - _loading(d, P, dstar)).max() / (MU * P)
    assert err < 2e-3, err
    # the secant stiffness at the start is the no-slip 8 G* a
    assert abs(T[0] / dd / (8 * _gstar() * math.sqrt(delta * rstar)) - 1) < 1e-12
    # full sliding beyond d*
    assert np.all(np.abs(T[d > 1.01 * dstar] / (MU * P) - 1) < 1e-12)
    assert S[6] == 0 and np.all(S[3:6] == t)


def test_unloading_reloading_loop(orc):
    cfg = _cfg(orc)
    P, rstar, delta, dstar = _setup()
    n, t = np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0])
    S = np.zeros(orc.TS)
    S[9] = P
    N = 20000
    dd = dstar / N
    nA = int(0.6 * N)
    S, T1 = _drive(orc, cfg, S, n, t, P, rstar, delta, dd, nA)
    Tstar = T1[-1]
    assert abs(Tstar - _loading(0.6 * dstar, P, dstar)) < 2e-3 * MU * P
    # unload by 1.2 d*
    nB = int(1.2 * N)
    S, T2 = _drive(orc, cfg, S, n, t, P, rstar, delta, -dd, nB)
    assert S[6] == 1 and S[7] == Tstar
    du = dd * np.arange(1, nB + 1)
    ref = Tstar - 2 * MU * P * (1.0 - (1.0 - du / (2 * dstar)) ** 1.5)
    assert np.abs(T2 - ref).max() < 2e-3 * MU * P
    Tss = T2[-1]
    # reload by 1.2 d* (back to d_A): the loop closes at T*
    S, T3 = _drive(orc, cfg, S, n, t, P, rstar, delta, dd, nB)
    assert S[8] == Tss
    dr = dd * np.arange(1, nB + 1)
    ref = Tss + 2 * MU * P * (1.0 - (1.0 - dr / (2 * dstar)) ** 1.5)
    assert np.abs(T3 - ref).max() < 2e-3 * MU * P
    assert abs(T3[-1] - Tstar) < 2e-3 * MU * P
    # further loading continues on the virgin curve (k back to 0)
    S, T4 = _drive(orc, cfg, S, n, t, P, rstar, delta, dd, int(0.2 * N))
    assert S[6] == 0
    assert abs(T4[-1] - _loading(0.8 * dstar, P, dstar)) < 3e-3 * MU * P
    # the loop is hysteretic: at the same displacement the reloading branch
    # lies above the unloading one, so the cycle dissipates energy
    mid = nB // 2
    assert T3[nB - 1 - mid] > T2[mid]
    work = dd * (T3.sum() - T2.sum())
    assert work > 0.01 * MU * P * dstar


def test_growing_normal_force(orc):
    cfg = _cfg(orc)
    n, t = np.array([0.0, 0.0, 1.0]), np.array([0.0, 1.0, 0.0])
    rstar = 0.125
    Es = E / (2 * (1 - NU * NU))
    S = np.zeros(orc.TS)
    # normal loading only: no tangential force ever
    for k in range(1, 200):
        dl = 1e-6 * k
        P = 4.0 / 3.0 * Es * math.sqrt(rstar) * dl ** 1.5
        S = orc.tangential_update(cfg, 1.0, n, np.zeros(3), P, rstar, dl, S)
        assert np.all(S[:3] == 0.0)
    # normal force growing faster than the tangential load: purely elastic
    S = np.zeros(orc.TS)
    T_el = 0.0
    for k in range(1, 200):
        dl = 1e-6 * k
        P = 4.0 / 3.0 * Es * math.sqrt(rstar) * dl ** 1.5
        kt = 8 * _gstar() * math.sqrt(dl * rstar)
        dd = 1e-3 * MU * (P - (4.0 / 3.0 * Es * math.sqrt(rstar) * (1e-6 * (k - 1)) ** 1.5)) / kt
        S = orc.tangential_update(cfg, 1.0, n, -t * dd, P, rstar, dl, S)
        T_el += kt * dd
        assert abs(float(np.dot(S[:3], t)) - T_el) <= 1e-12 * T_el


def test_infinite_friction_is_the_no_slip_law(orc):
    ms = _cfg(orc, mu=1e12)
    ns = _cfg(orc, contact="hertz_mindlin", mu=1e12)
    rng = np.random.default_rng(3)
    P, rstar, delta, dstar = _setup()
    S1, S2 = np.zeros(orc.TS), np.zeros(orc.TS)
    n = np.array([0.0, 0.0, 1.0])
    for _ in range(300):
        v = np.r_[rng.standard_normal(2) * 1e-3, 0.0]
        S1 = orc.tangential_update(ms, 1.0, n, v, P, rstar, delta, S1)
        S2 = orc.tangential_update(ns, 1.0, n, v, P, rstar, delta, S2)
    assert np.linalg.norm(S1[:3] - S2[:3]) <= 1e-9 * np.linalg.norm(S2[:3])


def test_frame_independence(orc):
    cfg = _cfg(orc)
    P, rstar, delta, dstar = _setup()
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    n0 = np.array([0.0, 0.0, 1.0])
    S0, S1 = np.zeros(orc.TS), np.zeros(orc.TS)
    S0[9] = S1[9] = P
    # a loading path that turns in the contact plane and reverses
    for k in range(3000):
        ang = 0.002 * k
        dirn = np.array([math.cos(ang), math.sin(ang), 0.0]) * (1.0 if k < 2000 else -1.0)
        v = -dirn * dstar / 1500
        S0 = orc.tangential_update(cfg, 1.0, n0, v, P, rstar, delta, S0)
        S1 = orc.tangential_update(cfg, 1.0, Q @ n0, Q @ v, P, rstar, delta, S1)
    assert np.linalg.norm(Q @ S0[:3] - S1[:3]) <= 1e-12 * MU * P
    assert S0[6] == S1[6] and abs(S0[7] - S1[7]) <= 1e-12 * MU * P
    assert 0 < np.linalg.norm(S0[:3]) <= MU * P * (1 + 1e-12)


def test_coupled_momentum_bookkeeping(orc):
    n = (20, 20, 20)
    cfg = orc.make_cfg(lattice=19, n=n, tau=0.7, gravity=(0, 0, -1e-4), n_sub=40,
                       contact="hertz_mindlin_microslip", young=1e-2, poisson=NU, friction=MU, two_way=1,
                       skin=0.05)
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
    # the carried state holds a loading direction and the previous normal force
    st = hist[1]
    assert np.all(np.abs(np.linalg.norm(st[:, 3:6], axis=1) - 1) < 1e-12) and np.all(st[:, 9] > 0)
