"""Pins of the oracle's Lagrange-polynomial interpolation (Eq. lbm5-lbm6),
the paper's own interpolation of the populations at a particle, on the four
nodes per axis the delta kernel also uses: exact reproduction of
polynomials up to the degree the in-domain nodes allow (cubic in the
interior, lower next to a wall), Kronecker property at the nodes, and exact
interpolation of a tensor-product cubic moment field."""
import numpy as np
import pytest


def _cfg(orc, lattice, n):
    return orc.make_cfg(lattice=lattice, n=n, contact="none", interp="lagrange")


@pytest.mark.parametrize("lattice,n", [(9, (16, 12, 1)), (15, (10, 9, 11)), (19, (10, 9, 11))])
def test_lagrange_reproduces_polynomials(orc, lattice, n):
    rng = np.random.default_rng(7)
    cfg = _cfg(orc, lattice, n)
    D = 2 if lattice == 9 else 3
    for trial in range(200):
        X = np.array([rng.uniform(0.0, n[a]) for a in range(D)])
        base, phi = orc.weights_lagrange(cfg, X)
        for a in range(D):
            nodes = base[a] + np.arange(4)
            inside = (nodes >= 0) & (nodes < n[a])
            xs = nodes + 0.5
            deg = int(inside.sum()) - 1
            assert np.all(phi[a][~inside] == 0.0)
            for p in range(deg + 1):
                assert abs(phi[a] @ xs ** p - X[a] ** p) <= 1e-12 * max(1.0, X[a] ** p)


def test_lagrange_kronecker_at_nodes(orc):
    cfg = _cfg(orc, 15, (8, 8, 8))
    for i in range(8):
        X = np.array([i + 0.5, 3.5, 4.5])
        base, phi = orc.weights_lagrange(cfg, X)
        k = i - base[0]
        expect = np.zeros(4)
        expect[k] = 1.0
        assert np.allclose(phi[0], expect, atol=1e-15)


@pytest.mark.parametrize("lattice", [15, 19])
def test_lagrange_interpolates_cubic_field_exactly(orc, lattice):
    n = (12, 11, 13)
    cfg = _cfg(orc, lattice, n)
    N = n[0] * n[1] * n[2]
    z, y, x = np.meshgrid(np.arange(n[2]) + 0.5, np.arange(n[1]) + 0.5, np.arange(n[0]) + 0.5, indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()

    def field(x, y, z):
        return 1 + 0.01 * x - 0.003 * x ** 3 / 100 + 0.02 * y ** 2 / 10 - 0.001 * z ** 3 / 50 + 1e-4 * x * y * z

    rho = field(x, y, z)
    j = np.stack([field(y, z, x), field(z, x, y), 0.5 * field(x, z, y)])
    rng = np.random.default_rng(3)
    X = np.stack([rng.uniform(2.0, n[a] - 2.0, 40) for a in range(3)])
    rho_i, j_i = orc.interp(cfg, X, rho, j)
    assert np.allclose(rho_i, field(*X), rtol=1e-12, atol=1e-12)
    assert np.allclose(j_i[0], field(X[1], X[2], X[0]), rtol=1e-12, atol=1e-12)
    assert np.allclose(j_i[2], 0.5 * field(X[0], X[2], X[1]), rtol=1e-12, atol=1e-12)
