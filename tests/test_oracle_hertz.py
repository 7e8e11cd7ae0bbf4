"""Pins of the oracle's Hertz normal contact (Sec. 2.3) against the
classical theory of the elastic impact of spheres (Hertz; Johnson, Contact
Mechanics, Sec. 11.4): for relative approach speed v, effective mass m* and
effective radius R*, energy conservation gives the largest overlap

    delta_max = (15 m* v^2 / (16 E* sqrt(R*)))^(2/5)

and the contact lasts t_c = 2 (delta_max / v) I with
I = integral_0^1 (1 - x^(5/2))^(-1/2) dx (evaluated here by quadrature).
The rebound is elastic (no damping term in the paper's model).  A flat
wall is a body of infinite mass and radius (m* = m, R* = R).  With the
same E, halving E* (or dropping the 4/3) moves delta_max by 32 % (12 %)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

I_HERTZ = quad(lambda x: (1.0 - x ** 2.5) ** -0.5, 0.0, 1.0)[0]


def _estar(E, nu):
    return E / (2.0 * (1.0 - nu * nu))     # two bodies of one material


def _track(orc, cfg, X, U, d, rp, steps, gap_fn):
    """Run the DEM alone (no fluid moments) and record the overlap after
    every lattice step."""
    D = X.shape[0]
    rho_i = np.zeros(X.shape[1])
    j_i = np.zeros((D, X.shape[1]))
    ov = []
    for _ in range(steps):
        X, U, *_ = orc.dem(cfg, X, U, d, rp, rho_i, j_i)
        ov.append(gap_fn(X))
    return np.array(ov), X, U


def _contact_stats(ov, t0=0.0):
    """Largest overlap (parabola through the three samples at the peak) and
    the contact duration from linear interpolation of the sign changes."""
    i = int(np.argmax(ov))
    a, b, c = ov[i - 1], ov[i], ov[i + 1]
    den = a - 2 * b + c
    peak = b - 0.125 * (a - c) ** 2 / den if den != 0 else b
    pos = np.where(ov > 0)[0]
    i0, i1 = pos[0], pos[-1]
    # steps are recorded after step k + 1: sample k is at time k + 1
    ton = (i0 + 1) - ov[i0] / (ov[i0] - ov[i0 - 1])
    toff = (i1 + 1) + ov[i1] / (ov[i1] - ov[i1 + 1])
    return peak, toff - ton


@pytest.mark.parametrize("D,d,rp", [(3, (0.5, 0.5), (2.0, 2.0)), (3, (0.4, 0.7), (2.5, 1.5)),
                                    (2, (0.5, 0.5), (2.0, 2.0))])
def test_hertz_pair_impact(orc, D, d, rp):
    E, nu, v = 2e-3, 0.33, 1e-3
    n = (16, 16, 1) if D == 2 else (10, 10, 10)
    cfg = orc.make_cfg(lattice=9 if D == 2 else 19, n=n, n_sub=400, contact="hertz", young=E, poisson=nu,
                       two_way=0, skin=0.05)
    d, rp = np.array(d), np.array(rp)
    m = np.array([orc.mass(D, d[i], rp[i]) for i in range(2)])
    rc = 0.5 * (d[0] + d[1])
    X = np.full((D, 2), n[1] / 2.0)
    X[0, 0], X[0, 1] = 5.0 - 0.5 * rc - 0.02, 5.0 + 0.5 * rc + 0.02
    U = np.zeros((D, 2))
    # equal and opposite momenta: the centre of mass stays at rest
    U[0, 0], U[0, 1] = v * m[1] / m.sum(), -v * m[0] / m.sum()
    ov, X1, U1 = _track(orc, cfg, X, U, d, rp, 400, lambda X: rc - abs(X[0, 1] - X[0, 0]))
    mstar = m[0] * m[1] / m.sum()
    R = 0.5 * d
    Rstar = R[0] * R[1] / R.sum()
    Es = _estar(E, nu)
    dmax = (15 * mstar * v * v / (16 * Es * math.sqrt(Rstar))) ** 0.4
    tc = 2 * I_HERTZ * dmax / v
    peak, dur = _contact_stats(ov)
    assert 60 < tc < 200                                    # resolved by the lattice-step samples
    assert abs(peak / dmax - 1) < 2e-3, (peak, dmax)
    assert abs(dur / tc - 1) < 5e-3, (dur, tc)
    # elastic: the relative velocity reverses, momentum is conserved exactly
    e = (U1[0, 1] - U1[0, 0]) / v
    assert abs(e - 1) < 1e-3
    assert abs((m * U1[0]).sum()) < 1e-17
    assert np.all(U1[1:] == 0)


def test_hertz_wall_impact(orc):
    E, nu, v = 2e-3, 0.33, 1e-3
    cfg = orc.make_cfg(lattice=19, n=(10, 10, 10), n_sub=400, contact="hertz", young=E, poisson=nu,
                       two_way=0, skin=0.05)
    d, rp = np.array([0.5]), np.array([2.0])
    X = np.array([[5.0], [5.0], [0.25 + 0.02]])
    U = np.array([[0.0], [0.0], [-v]])
    ov, X1, U1 = _track(orc, cfg, X, U, d, rp, 400, lambda X: 0.25 - X[2, 0])
    m = orc.mass(3, 0.5, 2.0)
    dmax = (15 * m * v * v / (16 * _estar(E, nu) * math.sqrt(0.25))) ** 0.4
    tc = 2 * I_HERTZ * dmax / v
    peak, dur = _contact_stats(ov)
    assert abs(peak / dmax - 1) < 2e-3, (peak, dmax)
    assert abs(dur / tc - 1) < 5e-3, (dur, tc)
    assert abs(U1[2, 0] / v - 1) < 1e-3
