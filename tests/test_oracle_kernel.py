"""Pins of the oracle's coupling part (O2, O3, O5) and its cell list.

* Eq. lbm12 delta function: partition of unity, the closed-form first moment
  sum_k phi_k (X - x_k) = t - (sqrt 2 / 2) sin(pi t / 2) (t = offset of X from
  the midpoint of its two bracketing nodes), sum phi^2 = 3/8, C^1 at |a| = 2
* weights at walls: out-of-domain nodes carry no weight and every axis still
  sums to one (reading R6)
* interpolation and spreading are transposes: <a, I j> = <S a, j>
* total spread force equals the sum of particle coefficients, walls included
* interpolation of constant fields is exact
* cell list: sorted by (key, id), bin_start consistent with counts, and every
  particle lies geometrically inside its bin
"""
import numpy as np
import pytest


def test_delta_moments(orc):
    rng = np.random.default_rng(0)
    for t in np.concatenate([rng.uniform(-0.5, 0.5, 200), [-0.5, 0.0, 0.5]]):
        X = 10.0 + t                                  # midpoint of nodes 9.5 and 10.5
        nodes = np.array([8.5, 9.5, 10.5, 11.5])
        phi = np.array([orc.delta(X - x) for x in nodes])
        assert abs(phi.sum() - 1) < 1e-15
        m1 = (phi * (X - nodes)).sum()
        assert abs(m1 - (t - np.sqrt(2) / 2 * np.sin(np.pi * t / 2))) < 1e-15
        assert abs((phi ** 2).sum() - 3 / 8) < 1e-15
    # maximum of the first moment
    ts = np.linspace(-0.5, 0.5, 20001)
    m = ts - np.sqrt(2) / 2 * np.sin(np.pi * ts / 2)
    assert abs(np.abs(m).max() - 0.021088) < 1e-6
    # support and continuity of value and slope at |a| = 2
    assert orc.delta(2.0) == 0.0 and orc.delta(-2.0) == 0.0
    assert orc.delta(2.0000001) == 0.0
    eps = 1e-6
    assert abs(orc.delta(2 - eps)) < 1e-11
    assert abs((orc.delta(1.0 + eps) - orc.delta(1.0 - eps)) / (2 * eps) + np.pi / 8) < 1e-8


@pytest.mark.parametrize("lat", [9, 19])
def test_weights_interior_and_walls(orc, lat):
    n = (16, 12, 1) if lat == 9 else (10, 12, 9)
    cfg = orc.make_cfg(lattice=lat, n=n)
    D = orc.D(cfg)
    rng = np.random.default_rng(1)
    for _ in range(300):
        X = np.array([rng.uniform(0.0, n[a]) for a in range(D)])
        base, phi = orc.weights(cfg, X)
        for a in range(D):
            assert abs(phi[a].sum() - 1) < 1e-14
            for k in range(4):
                i = base[a] + k
                if i < 0 or i >= n[a]:
                    assert phi[a, k] == 0.0
                else:
                    assert abs(X[a] - (i + 0.5)) <= 2.0
            # the four nodes bracket X
            assert base[a] + 0.5 < X[a] + 1e-12 <= base[a] + 3.5 + 1.0


@pytest.mark.parametrize("lat", [9, 19])
def test_interp_spread_adjoint(orc, lat):
    n = (14, 11, 1) if lat == 9 else (9, 8, 10)
    cfg = orc.make_cfg(lattice=lat, n=n)
    D, N = orc.D(cfg), orc.nnodes(cfg)
    rng = np.random.default_rng(2)
    npart = 40
    X = np.stack([rng.uniform(0, n[a], npart) for a in range(D)])
    rho = rng.standard_normal(N)
    j = rng.standard_normal((D, N))
    a = rng.standard_normal((D, npart))
    rho_i, j_i = orc.interp(cfg, X, rho, j)
    F = orc.spread(cfg, X, a)
    lhs = (a * j_i).sum()
    rhs = (F * j).sum()
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)
    # scalar channel: spreading a unit coefficient on axis 0, read against rho
    a0 = np.zeros((D, npart))
    a0[0] = rng.standard_normal(npart)
    F0 = orc.spread(cfg, X, a0)
    assert abs((a0[0] * rho_i).sum() - (F0[0] * rho).sum()) < 1e-12 * (1 + abs((F0[0] * rho).sum()))


@pytest.mark.parametrize("lat", [9, 19])
def test_spread_total_and_constant_interp(orc, lat):
    n = (12, 10, 1) if lat == 9 else (7, 9, 8)
    cfg = orc.make_cfg(lattice=lat, n=n)
    D, N = orc.D(cfg), orc.nnodes(cfg)
    rng = np.random.default_rng(3)
    npart = 30
    X = np.stack([rng.uniform(0, n[a], npart) for a in range(D)])
    X[:, :5] = np.array([[0.05] * D, [n[0] - 0.01] + [0.3] * (D - 1),
                         [0.5] * D, [1.0] * D, [2.0] * D]).T[:D]
    coef = rng.standard_normal((D, npart))
    F = orc.spread(cfg, X, coef)
    assert np.allclose(F.sum(axis=1), coef.sum(axis=1), atol=1e-13)
    rho_i, j_i = orc.interp(cfg, X, np.full(N, 1.7), np.tile(np.arange(1, D + 1)[:, None], (1, N)))
    assert np.allclose(rho_i, 1.7, atol=1e-14)
    for a in range(D):
        assert np.allclose(j_i[a], a + 1, atol=1e-14)


@pytest.mark.parametrize("lat,bl", [(9, 1), (19, 1), (9, 0), (19, 2)])
def test_cell_list_properties(orc, lat, bl):
    n = (20, 16, 1) if lat == 9 else (12, 10, 14)
    cfg = orc.make_cfg(lattice=lat, n=n, bin_log2=bl)
    D = orc.D(cfg)
    rng = np.random.default_rng(4)
    npart = 300
    X = np.stack([rng.uniform(0, n[a], npart) for a in range(D)])
    # ties and bin edges: exact half-integers and node centres
    X[:, :10] = np.round(X[:, :10] * 2) / 2
    X[:, 10:20] = X[:, 0:10]
    keys, perm, bs = orc.cell_list(cfg, X)
    tot, nb = orc.nbins(cfg)
    assert sorted(perm.tolist()) == list(range(npart))
    pairs = list(zip(keys.tolist(), perm.tolist()))
    assert pairs == sorted(pairs)
    counts = np.bincount(keys, minlength=tot)
    assert np.array_equal(np.diff(bs), counts)
    assert bs[0] == 0 and bs[-1] == npart
    edge = 2.0 ** bl
    for s in range(npart):
        k = int(keys[s])
        b = [k % nb[0], (k // nb[0]) % nb[1], k // (nb[0] * nb[1])]
        for a in range(D):
            x = X[a, perm[s]]
            assert b[a] * edge - 0.5 <= x < (b[a] + 1) * edge - 0.5
