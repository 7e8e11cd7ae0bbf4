"""Pins of the oracle's lattice part (O1, O6, O7) against facts fixed by
lattice-Boltzmann theory and by closed forms, not by re-typing its formulas.

* velocity-set isotropy up to fourth order (fixes weights, velocities, c_s^2)
* equilibrium moments (Eq. lbm3): density, momentum, momentum flux
* Guo forcing (Eq. lbm9) plus the half-force velocity: exact momentum gain F
  per node and the second moment (1 - 1/2tau)(uF + Fu)
* body-force Poiseuille flow between halfway bounce-back walls: closed form
  u(y) = F/(2 nu) [y (H - y) + (16 Lambda - 3)/12], Lambda = (tau - 1/2)^2
* mass conservation with walls
"""

import numpy as np
import pytest


@pytest.mark.parametrize("lat", [9, 15, 19])
def test_lattice_isotropy(orc, lat):
    e, w, opp = orc.tables(lat)
    D = 2 if lat == 9 else 3
    e = e[:, :D].astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ e).max() < 1e-15
    M2 = np.einsum("q,qa,qb->ab", w, e, e)
    assert np.allclose(M2, np.eye(D) / 3, atol=1e-15)
    M3 = np.einsum("q,qa,qb,qc->abc", w, e, e, e)
    assert np.abs(M3).max() < 1e-15
    M4 = np.einsum("q,qa,qb,qc,qd->abcd", w, e, e, e, e)
    I = np.eye(D)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9
    assert np.allclose(M4, iso, atol=1e-15)
    # opposite directions
    assert np.all(e[opp] == -e)
    # integer velocities with components in {-1, 0, 1}, all distinct
    assert len({tuple(v) for v in e}) == len(e)


@pytest.mark.parametrize("lat", [9, 15, 19])
def test_equilibrium_moments(orc, lat):
    rng = np.random.default_rng(1)
    e, w, _ = orc.tables(lat)
    D = 2 if lat == 9 else 3
    for _ in range(5):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(D)
        feq = orc.equilibrium(lat, rho, u)
        ef = e[:, :D].astype(float)
        assert abs(feq.sum() - rho) < 1e-14
        assert np.allclose(feq @ ef, rho * u, atol=1e-15)
        Pi = np.einsum("q,qa,qb->ab", feq, ef, ef)
        assert np.allclose(Pi, rho * np.eye(D) / 3 + rho * np.outer(u, u), atol=1e-15)


@pytest.mark.parametrize("lat,tau", [(9, 0.8), (9, 0.55), (15, 0.65), (19, 0.6), (19, 1.3)])
def test_guo_forcing_moments(orc, lat, tau):
    """One node, all axes periodic: streaming returns every population to the
    node, so the step is the collision alone."""
    D = 2 if lat == 9 else 3
    cfg = orc.make_cfg(lattice=lat, n=(1, 1, 1), periodic=(1, 1, 1), tau=tau, contact="none")
    e, w, _ = orc.tables(lat)
    ef = e[:, :D].astype(float)
    rng = np.random.default_rng(2)
    f = w * (1 + 0.05 * rng.standard_normal(len(w)))
    F = 1e-3 * rng.standard_normal(D)
    fs = orc.collide_stream(cfg, f, F.reshape(D, 1))
    rho = f.sum()
    j = f @ ef
    assert abs(fs.sum() - rho) < 1e-15                       # mass
    assert np.allclose(fs @ ef, j + F, atol=1e-16)            # momentum gains F exactly
    # second moment: relaxation towards Pi_eq(rho, u) plus (1 - 1/2tau)(uF + Fu)
    u = (j + 0.5 * F) / rho
    Pi = np.einsum("q,qa,qb->ab", f, ef, ef)
    Pieq = rho * np.eye(D) / 3 + rho * np.outer(u, u)
    expect = Pi - (Pi - Pieq) / tau + (1 - 0.5 / tau) * (np.outer(u, F) + np.outer(F, u))
    got = np.einsum("q,qa,qb->ab", fs, ef, ef)
    assert np.allclose(got, expect, atol=1e-15)


@pytest.mark.parametrize("lat,tau", [(9, 0.8), (9, 0.6), (15, 0.85), (19, 0.8)])
def test_poiseuille_closed_form(orc, lat, tau):
    H, Fx = 8, 1e-6
    cfg = orc.make_cfg(lattice=lat, n=(1, H, 1), periodic=(1, 0, 1), tau=tau, contact="none")
    F = np.zeros((3, H))
    F[0] = Fx
    f = orc.rest_state(cfg)
    nu = (tau - 0.5) / 3
    steps = int(30 * H * H / (np.pi ** 2 * nu))
    for _ in range(steps):
        f = orc.collide_stream(cfg, f, F)
    rho, j = orc.moments(cfg, f)
    u = (j[0] + 0.5 * Fx) / rho
    y = np.arange(H) + 0.5
    lam = (tau - 0.5) ** 2
    ua = Fx / (2 * nu) * (y * (H - y) + (16 * lam - 3) / 12)
    assert np.abs(u - ua).max() / ua.max() < 1e-9
    # without the slip offset the profile is off by far more than the tolerance
    ub = Fx / (2 * nu) * y * (H - y)
    assert np.abs(u - ub).max() / ua.max() > 1e-4
    assert np.abs(j[1]).max() < 1e-8 * ua.max()


@pytest.mark.parametrize("lat", [9, 15, 19])
def test_mass_conservation_walls(orc, lat):
    n = (12, 10, 1) if lat == 9 else (6, 5, 7)
    cfg = orc.make_cfg(lattice=lat, n=n, tau=0.7, contact="none")
    rng = np.random.default_rng(3)
    f = orc.rest_state(cfg) * (1 + 0.01 * rng.standard_normal(orc.Q(cfg) * orc.nnodes(cfg)))
    D = orc.D(cfg)
    F = 1e-4 * rng.standard_normal((D, orc.nnodes(cfg)))
    m0, _ = orc.fluid_totals(cfg, f)
    steps = 200
    for _ in range(steps):
        f = orc.collide_stream(cfg, f, F)
    m1, _ = orc.fluid_totals(cfg, f)
    bound = 10 * steps * orc.nnodes(cfg) * orc.Q(cfg) * 2.0 ** -53 * m0
    assert abs(m1 - m0) < bound
