"""Support facts that let the HIP path skip work, checked on the oracle.

* Interpolation and spreading (Eqs. lbm10-lbm12) touch, per axis, only the
  four nodes around a particle: node y takes part only for particles whose
  dual cell c' = floor(X - 1/2) + 1 lies in [y - 1, y + 2].  Checked by
  behaviour: moments replaced by garbage on every node row (y, z) that the
  rule leaves out do not change the gathered values (delta and Lagrange
  weights), and spreading writes nothing there.  With bins of 2^L dual
  cells the rule taken over whole bins keeps a superset of those rows.
* A particle of bin k lies in [k 2^L - 1/2, (k + 1) 2^L - 1/2): every bin
  below bin(X - r) or above bin(X + r) holds only particles farther than r
  from X along that axis (the neighbour scan visits only the bins between).
"""
import numpy as np
import pytest


def _dual_cell(X):
    return np.floor(X - 0.5).astype(np.int64) + 1


def _needed_rows(X, n, D, L=0):
    """Node rows (y, z) that some particle's stencil reaches, by the rule;
    with L > 0 taken over the bins of the particles' cells."""
    need = np.zeros((n[2], n[1]), bool)
    cy = _dual_cell(X[1]) >> L
    cz = (_dual_cell(X[2]) >> L) if D == 3 else np.zeros_like(cy)
    for z in range(n[2]):
        zl, zh = ((z - 1) >> L, (z + 2) >> L) if D == 3 else (0, 0)
        for y in range(n[1]):
            yl, yh = (y - 1) >> L, (y + 2) >> L
            if L == 0:
                yl, yh = y - 1, y + 2
                if D == 3:
                    zl, zh = z - 1, z + 2
            need[z, y] = np.any((cy >= yl) & (cy <= yh) & (cz >= zl) & (cz <= zh))
    return need


def _band(rng, D, n, npart):
    if D == 3:
        X = np.stack([rng.uniform(0.3, n[0] - 0.3, npart), rng.uniform(7.0, 10.0, npart),
                      rng.uniform(8.0, 11.0, npart)])
        X[1, :6] = [7.0, 10.0, 7.5, 9.5, 7.0, 10.0]
        X[2, :6] = [8.0, 11.0, 11.0, 8.0, 8.5, 10.5]
    else:
        X = np.stack([rng.uniform(0.3, n[0] - 0.3, npart), rng.uniform(12.0, 17.0, npart)])
        X[1, :4] = [12.0, 17.0, 12.5, 16.5]
    return X


@pytest.mark.parametrize("lattice,interp", [(19, "delta"), (19, "lagrange"), (9, "delta"), (9, "lagrange")])
def test_rows_outside_the_rule_are_neither_read_nor_written(orc, lattice, interp):
    D = 2 if lattice == 9 else 3
    n = (12, 20, 18) if D == 3 else (16, 30, 1)
    rng = np.random.default_rng(5)
    X = _band(rng, D, n, 40)
    cfg = orc.make_cfg(lattice=lattice, n=n, interp=interp)
    N = n[0] * n[1] * n[2]
    need = _needed_rows(X, n, D)
    assert need.any() and not need.all()
    rows_of_node = np.repeat(need.reshape(-1), n[0])            # node index = (z ny + y) nx + x
    rho = rng.normal(0.0, 1e-3, N)
    j = rng.normal(0.0, 1e-3, (D, N))
    rho2, j2 = rho.copy(), j.copy()
    rho2[~rows_of_node] = 1e3 * rng.standard_normal((~rows_of_node).sum())
    j2[:, ~rows_of_node] = 1e3 * rng.standard_normal((D, (~rows_of_node).sum()))
    r1, j1 = orc.interp(cfg, X, rho, j)
    r2, jb = orc.interp(cfg, X, rho2, j2)
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(j1, jb)
    F = orc.spread(cfg, X, rng.normal(0.0, 1.0, (D, X.shape[1])))
    assert np.all(F[:, ~rows_of_node] == 0.0)
    assert np.any(F[:, rows_of_node] != 0.0)
    # one row short on either side is not enough: the rule is tight
    lo_rows = np.argwhere(need)
    z0, y0 = lo_rows.min(axis=0)
    z1, y1 = lo_rows.max(axis=0)
    Fr = np.abs(F).sum(axis=0).reshape(n[2], n[1], n[0]).sum(axis=2)
    assert Fr[:, y0].any() and Fr[:, y1].any()
    if D == 3:
        assert Fr[z0, :].any() and Fr[z1, :].any()


@pytest.mark.parametrize("L", [1, 2])
def test_rows_by_whole_bins_cover_the_rule(L):
    rng = np.random.default_rng(6)
    for D, n in ((3, (12, 20, 18)), (2, (16, 30, 1))):
        X = _band(rng, D, n, 40)
        exact = _needed_rows(X, n, D, 0)
        coarse = _needed_rows(X, n, D, L)
        assert np.all(coarse[exact])


def _bin(orc, cfg, x, D, axis, n):
    """The oracle's bin coordinate of position x along one axis (the other
    coordinates at the box centre)."""
    P = np.array([[n[a] / 2.0] for a in range(D)])
    P[axis, 0] = x
    keys, _, _ = orc.cell_list(cfg, P)
    _, nb = orc.nbins(cfg)
    k = int(keys[0])
    return [k % nb[0], (k // nb[0]) % nb[1], k // (nb[0] * nb[1])][axis]


@pytest.mark.parametrize("L", [0, 1, 2])
def test_bins_outside_the_reach_hold_no_partner(orc, L):
    D, n = 3, (24, 20, 18)
    cfg = orc.make_cfg(lattice=19, n=n, bin_log2=L)
    rng = np.random.default_rng(8)
    for _ in range(300):
        axis = int(rng.integers(0, D))
        r = float(rng.choice([rng.uniform(0.2, 2.5), 0.5, 1.0, 1.5]))
        X = float(rng.uniform(r + 0.01, n[axis] - r - 0.01))
        if rng.random() < 0.3:
            X = np.round(X * 2) / 2                                 # half-integers and node centres
            X = min(max(X, r + 0.01), n[axis] - r - 0.01)
        lo, hi = _bin(orc, cfg, X - r, D, axis, n), _bin(orc, cfg, X + r, D, axis, n)
        for Y in np.concatenate([rng.uniform(0.01, n[axis] - 0.01, 8), [X - r, X + r, X]]):
            b = _bin(orc, cfg, Y, D, axis, n)
            if b < lo:
                assert X - Y > r
            elif b > hi:
                assert Y - X > r
            if abs(Y - X) <= r:
                assert lo <= b <= hi
