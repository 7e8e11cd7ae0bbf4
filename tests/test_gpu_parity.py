"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (floating point, per field; see tests/gpu_helpers.py):
  FP32 storage: eps_u <= 1e-5, eps_rho <= 1e-6 after one step from an
                identical state; particles: velocity L2-relative <= 1e-5,
                displacement max-relative <= 1e-5
  FP16 storage (deviations scaled by 2^14): eps_u <= 1e-3, eps_rho <= 1e-5
Integer results (cell-list keys, ids, bin ranges) are compared bit for bit.
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


@pytest.fixture(scope="module")
def W():
    from paper_1407_6704_amd import workloads
    return workloads


def _flush(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# lattice only
# ---------------------------------------------------------------------------
LATTICE_CASES = [
    (9, "fp32", (67, 45, 1), (0, 0, 0)),
    (9, "fp32", (64, 33, 1), (1, 0, 0)),
    (19, "fp32", (19, 13, 11), (0, 0, 0)),
    (19, "fp32", (16, 9, 12), (1, 0, 1)),
    (15, "fp32", (19, 13, 11), (0, 0, 0)),
    (15, "fp32", (16, 9, 12), (1, 0, 1)),
    (9, "fp16", (67, 45, 1), (0, 0, 0)),
    (19, "fp16", (19, 13, 11), (0, 0, 0)),
    (15, "fp16", (19, 13, 11), (0, 0, 0)),
]


@pytest.mark.parametrize("lat,storage,n,per", LATTICE_CASES)
def test_lattice_steps_match_oracle(P, W, orc, lat, storage, n, per):
    _flush(f"lattice {lat} {storage} {n} periodic={per}")
    cfg = P.make_config(lattice=lat, n=n, storage=storage, periodic=per, tau=0.7,
                        fluid_force=(2e-6, -1e-6, 5e-7 if lat != 9 else 0.0), contact="none")
    sim = P.Sim(cfg, 0)
    w = W.C0.replace(lattice=lat, n=n)
    h0 = G.perturbed_state(orc, sim, w, seed=5)
    oc = G.oracle_cfg(orc, cfg)
    N = sim.N
    F = np.tile(np.array(cfg.fluid_force)[: sim.D, None], (1, N))
    f = G.to_oracle_f(orc, lat, h0)
    tol_u, tol_rho = (1e-5, 1e-6) if storage == "fp32" else (1e-3, 1e-5)
    # element-wise population error against the largest deviation: FP32
    # arithmetic and storage leave a few units in the last place of the
    # largest |h| (2^-24 = 6e-8 each), bounded here by 16 of them; FP16
    # storage rounds each stored deviation once, to within 2^-11 of itself
    # (nearest-even, 11 significant bits), plus the FP32 part
    tol_h = 16 * 2.0 ** -24 if storage == "fp32" else 2.0 ** -11 + 16 * 2.0 ** -24
    # one step from an identical state
    sim.step(1)
    f1 = orc.collide_stream(oc, f, F)
    eu, er, eh = G.field_errors(orc, lat, sim.read_populations(), f1, N)
    _flush(f"  1 step: eps_u={eu:.2e} eps_rho={er:.2e} eps_h={eh:.2e} (bound {tol_h:.2e})")
    assert eu <= tol_u and er <= tol_rho and eh <= tol_h
    # ten more steps, same bounds
    sim.step(10)
    for _ in range(10):
        f1 = orc.collide_stream(oc, f1, F)
    eu, er, eh = G.field_errors(orc, lat, sim.read_populations(), f1, N)
    _flush(f"  11 steps: eps_u={eu:.2e} eps_rho={er:.2e} eps_h={eh:.2e}")
    assert eu <= tol_u and er <= tol_rho


@pytest.mark.parametrize("lat,storage", [(9, "fp32"), (19, "fp32"), (15, "fp32"), (9, "fp16"), (19, "fp16"),
                                         (15, "fp16")])
def test_poiseuille_gpu(P, lat, storage):
    _flush(f"poiseuille {lat} {storage}")
    H, Fx, tau = 16, 1e-6, 0.8
    cfg = P.make_config(lattice=lat, n=(1, H, 1), periodic=(1, 0, 1), storage=storage, tau=tau,
                        fluid_force=(Fx, 0, 0), contact="none")
    sim = P.Sim(cfg, 0)
    nu = (tau - 0.5) / 3
    sim.step(int(30 * H * H / (np.pi ** 2 * nu)))
    h = sim.read_populations().astype(np.float64)
    Q = h.shape[0]
    from oracle import oracle as orc
    e, w, _ = orc.tables(lat)
    dr = h.sum(axis=0)
    jx = e[:, 0].astype(float) @ h
    u = (jx + 0.5 * Fx) / (1 + dr)
    y = np.arange(H) + 0.5
    lam = (tau - 0.5) ** 2
    ua = Fx / (2 * nu) * (y * (H - y) + (16 * lam - 3) / 12)
    err = np.abs(u - ua).max() / ua.max()
    _flush(f"  max rel err {err:.2e}")
    # A steady state repeats the same roundings every step, so their bias adds
    # up over the slowest viscous time T = H^2/(pi^2 nu) (about 260 steps):
    # relative error <~ c T 2^-p with p = 24 (FP32) or 11 (FP16 storage) and
    # c = 2 for the two roundings of each stored value per step (relaxation
    # with forcing, then the store).  The FP64 oracle meets the same closed
    # form to 1e-9 on every lattice, so the excess is rounding alone.
    T = H * H / (np.pi ** 2 * nu)
    bound = 2 * T * 2.0 ** (-24 if storage == "fp32" else -11)
    assert err < bound


# ---------------------------------------------------------------------------
# particles
# ---------------------------------------------------------------------------
def _random_particles(rng, D, n, npart, dlo=0.3, dhi=0.6, margin=1.0):
    X = np.stack([rng.uniform(margin, n[a] - margin, npart) for a in range(D)])
    X = X.astype(np.float32).astype(np.float64)
    d = rng.uniform(dlo, dhi, npart).astype(np.float32).astype(np.float64)
    return X, d


@pytest.mark.parametrize("lat,n,npart", [(9, (40, 36, 1), 700), (19, (14, 12, 13), 900)])
def test_cell_list_bit_exact(P, W, orc, lat, n, npart):
    _flush(f"cell list {lat} {n} {npart}")
    rng = np.random.default_rng(21)
    D = 2 if lat == 9 else 3
    X, d = _random_particles(rng, D, n, npart, margin=0.3)
    # exact half-integers and node centres stress the floor of X - 1/2
    X[:, :40] = np.round(X[:, :40] * 2) / 2 + 0.0
    X[:, 40:60] = np.floor(X[:, 40:60]) + 0.5
    X[:, 60:70] = X[:, 0:10]                                  # coincident keys, ids decide
    X = np.clip(X, 0.25, np.array(n[:D])[:, None] - 0.25)
    cfg = P.make_config(lattice=lat, n=n, contact="none", two_way=0, bin_log2=1)
    sim = P.Sim(cfg, npart)
    sim.set_particles(X, np.zeros_like(X), d, np.full(npart, 2.0))
    sim.step(1)
    keys, ids, bs = sim.read_cell_list()
    oc = G.oracle_cfg(orc, cfg)
    k_ref, p_ref, b_ref = orc.cell_list(oc, X)
    assert np.array_equal(keys.astype(np.int64), k_ref)
    assert np.array_equal(ids, p_ref)
    assert np.array_equal(bs.astype(np.int64), b_ref)


def _coupled_compare(P, orc, cfg, X, U, d, rp, h0=None, steps=1, seed=0, tol=None, label=""):
    sim = P.Sim(cfg, X.shape[1])
    if h0 is not None:
        sim.write_populations(h0.astype(np.float32))
    h0 = sim.read_populations()
    sim.set_particles(X, U, d, rp)
    oc = G.oracle_cfg(orc, cfg)
    f = G.to_oracle_f(orc, cfg.lattice, h0)
    Xo, Uo = X.copy(), U.copy()
    for _ in range(steps):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
    sim.step(steps)
    sim.synchronize()
    got = sim.read_particles()
    eu, er, eh = G.field_errors(orc, cfg.lattice, sim.read_populations(), f, sim.N)
    disp = np.abs(Xo - X).max()
    ex = np.abs(got["x"] - Xo).max() / max(disp, 1e-30)
    ev = np.linalg.norm(got["v"] - Uo) / max(np.linalg.norm(Uo), 1e-30)
    fh_ref = -np.pi * d ** 2 / 4 * out["gbar"]
    efh = np.linalg.norm(got["f_hydro"] - fh_ref) / max(np.linalg.norm(fh_ref), 1e-30)
    _flush(f"  {label} eps_u={eu:.2e} eps_rho={er:.2e} eps_h={eh:.2e} dX={ex:.2e} (disp {disp:.2e}) "
           f"dU={ev:.2e} dFh={efh:.2e}")
    return dict(eu=eu, er=er, eh=eh, ex=ex, ev=ev, efh=efh, sim=sim, out=out, got=got)


FREE_CASES = [(9, "delta", 0), (19, "delta", 0), (15, "delta", 0), (9, "lagrange", 0), (15, "lagrange", 0),
              (19, "lagrange", 0), (15, "lagrange", 2), (9, "lagrange", 2)]


@pytest.mark.parametrize("lat,interp,bl", FREE_CASES)
def test_coupled_step_free_particles(P, W, orc, lat, interp, bl):
    """Particles away from each other (free: closed-form sub-steps), some
    near the walls (delta weights renormalised, Lagrange polynomials of lower
    order), on a perturbed fluid; both gathers, tiled (bins of one dual cell)
    and per-particle (bins of four)."""
    _flush(f"coupled free {lat} {interp} bin_log2={bl}")
    D = 2 if lat == 9 else 3
    n = (48, 40, 1) if D == 2 else (20, 18, 16)
    rng = np.random.default_rng(31)
    npart = 150 if D == 2 else 200
    X, d = _random_particles(rng, D, n, npart, 0.3, 0.5, margin=0.4)
    # push apart anything closer than contact + skin, so every particle is free
    keep = [0]
    for i in range(1, npart):
        r = np.sqrt(((X[:, keep] - X[:, i:i + 1]) ** 2).sum(axis=0))
        if np.all(r > 0.5 * (d[keep] + d[i]) + 0.2):
            keep.append(i)
    X, d = X[:, keep], d[keep]
    X = np.clip(X, 0.5 * d + 0.06, np.array(n[:D])[:, None] - 0.5 * d - 0.06)
    X = X.astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    U = (1e-4 * rng.standard_normal((D, npart))).astype(np.float32).astype(np.float64)
    rp = rng.uniform(1.5, 3.0, npart).astype(np.float32).astype(np.float64)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    cfg = P.make_config(lattice=lat, n=n, tau=0.7, gravity=g, n_sub=200, contact="lsd", interp=interp,
                        bin_log2=bl)
    w = W.C0.replace(lattice=lat, n=n)
    sim0 = P.Sim(P.make_config(lattice=lat, n=n, tau=0.7, contact="none"), 0)
    h0 = G.perturbed_state(orc, sim0, w, seed=7, amp=1e-4)
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, h0=h0, steps=1, label="1 step")
    assert r["eu"] <= 1e-5 and r["er"] <= 1e-6
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["efh"] <= 1e-5
    assert r["sim"].diagnostics()["active"] == 0
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, h0=h0, steps=5, label="5 steps")
    assert r["eu"] <= 1e-5 and r["er"] <= 1e-6 and r["ex"] <= 1e-5 and r["ev"] <= 1e-5


@pytest.mark.parametrize("lat,interp,bl", [(19, "delta", 0), (15, "lagrange", 0), (19, "delta", 2),
                                            (9, "delta", 2)])
def test_moments_only_where_gathered(P, W, orc, lat, interp, bl):
    """The moments pass of the coupled step skips the node rows that no
    particle's gather stencil reaches.  Particles confined to a band
    (3D: y in [6, 9], z in [9, 12]; 2D: y in [15, 20]) of a box whose x rows
    are long enough for a workgroup to span at most four rows, several
    exactly on the band's edges (their stencils end on the last rows
    computed): one step matches the oracle as in the free-particle case,
    also with bins of four cells (in 2D the only path with a moments pass)."""
    _flush(f"moments rows {lat} {interp} bin_log2={bl}")
    D = 2 if lat == 9 else 3
    rng = np.random.default_rng(77)
    if D == 3:
        n = (100, 16, 16)
        cand = np.stack([rng.uniform(1.0, 99.0, 400), rng.uniform(6.0, 9.0, 400), rng.uniform(9.0, 12.0, 400)])
        cand[1, :8] = [6.0, 9.0, 6.0, 9.0, 6.0, 9.0, 6.0, 9.0]
        cand[2, :8] = [9.0, 9.0, 12.0, 12.0, 9.0, 12.0, 9.0, 12.0]
    else:
        n = (100, 40, 1)
        cand = np.stack([rng.uniform(1.0, 99.0, 400), rng.uniform(15.0, 20.0, 400)])
        cand[1, :6] = [15.0, 20.0, 15.0, 20.0, 15.0, 20.0]
    d_all = rng.uniform(0.3, 0.5, 400)
    keep = [0]
    for i in range(1, 400):
        r = np.sqrt(((cand[:, keep] - cand[:, i:i + 1]) ** 2).sum(axis=0))
        if np.all(r > 0.5 * (d_all[keep] + d_all[i]) + 0.2):
            keep.append(i)
    X = cand[:, keep].astype(np.float32).astype(np.float64)
    d = d_all[keep].astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    assert npart > 60
    U = (1e-4 * rng.standard_normal((D, npart))).astype(np.float32).astype(np.float64)
    rp = rng.uniform(1.5, 3.0, npart).astype(np.float32).astype(np.float64)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    cfg = P.make_config(lattice=lat, n=n, tau=0.7, gravity=g, n_sub=200, contact="lsd",
                        interp=interp, bin_log2=bl)
    w = W.C0.replace(lattice=lat, n=n)
    sim0 = P.Sim(P.make_config(lattice=lat, n=n, tau=0.7, contact="none"), 0)
    h0 = G.perturbed_state(orc, sim0, w, seed=9, amp=1e-4)
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, h0=h0, steps=1, label="1 step")
    assert r["eu"] <= 1e-5 and r["er"] <= 1e-6
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["efh"] <= 1e-5
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, h0=h0, steps=3, label="3 steps")
    assert r["eu"] <= 1e-5 and r["er"] <= 1e-6 and r["ex"] <= 1e-5 and r["ev"] <= 1e-5


@pytest.mark.parametrize("lat,contact", [(9, "lsd"), (19, "lsd"), (15, "lsd"), (9, "hertz"), (19, "hertz")])
def test_coupled_step_with_contacts(P, orc, lat, contact):
    """Clusters of touching and approaching particles (islands of several
    sizes, wall contacts), linear spring-dashpot or Hertz, several steps."""
    _flush(f"coupled contacts {lat} {contact}")
    D = 2 if lat == 9 else 3
    n = (40, 30, 1) if D == 2 else (16, 14, 18)
    rng = np.random.default_rng(41)
    blocks = []
    ds = []
    # clusters: k particles on a jittered line with gaps ~0.01 (k = 2..6)
    for c in range(12 if D == 2 else 10):
        k = 2 + c % 5
        base = np.array([rng.uniform(3, n[a] - 3 - 0.5 * k) for a in range(D)])
        for i in range(k):
            p = base.copy()
            p[0] += 0.501 * i
            blocks.append(p)
            ds.append(0.5)
    # wall contacts: particles just touching the bottom wall
    for i in range(6):
        p = np.array([rng.uniform(2, n[a] - 2) for a in range(D)])
        p[D - 1] = 0.24999
        blocks.append(p)
        ds.append(0.5)
    X = np.array(blocks).T.astype(np.float32).astype(np.float64)
    d = np.array(ds)
    npart = X.shape[1]
    U = (3e-4 * rng.standard_normal((D, npart))).astype(np.float32).astype(np.float64)
    rp = np.full(npart, 2.5)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    cfg = P.make_config(lattice=lat, n=n, tau=0.8, gravity=g, n_sub=400, contact=contact, young=1e3)
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, steps=1, label="1 step")
    assert r["sim"].diagnostics()["active"] > 0
    assert r["eu"] <= 1e-5 and r["er"] <= 1e-6
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["efh"] <= 1e-5
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, steps=4, label="4 steps")
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["eu"] <= 1e-5 and r["er"] <= 1e-6


@pytest.mark.parametrize("lat,bl", [(9, 0), (19, 0), (9, 1), (19, 2)])
def test_contacts_of_particles_wider_than_a_bin(P, orc, lat, bl):
    """Polydisperse clusters with diameters up to 2.4 dual cells, some resting
    on the floor.  With bins of one dual cell a particle's neighbour reach
    spans up to seven bins per axis, so the counting scan takes its rows of
    bins in several batches (up to 49 rows in 3D, 7 in 2D); with bins of 2
    or 4 cells (bin_log2 1, 2) the same contacts are found in coarser rows.
    Every contact the scan misses would leave a particle on the free closed
    form."""
    _flush(f"wide particles {lat} bin_log2={bl}")
    D = 2 if lat == 9 else 3
    n = (48, 40, 1) if D == 2 else (24, 22, 26)
    rng = np.random.default_rng(57)
    sizes = [0.5, 1.6, 2.4, 0.8]
    pts, ds = [], []

    def fits(p, dd, floor=False):
        for q, e in zip(pts, ds):
            if np.sqrt(((p - q) ** 2).sum()) < 0.5 * (dd + e) + 0.3:
                return False
        return all((floor and a == D - 1) or dd / 2 + 1.0 <= p[a] <= n[a] - dd / 2 - 1.0 for a in range(D))

    clusters = 0
    for _ in range(4000):
        if clusters == (8 if D == 2 else 10):
            break
        k = 2 + clusters % 3
        axis = rng.standard_normal(D)
        axis /= np.linalg.norm(axis)
        dd = [sizes[(clusters + i) % 4] for i in range(k)]
        new = [np.array([rng.uniform(3, n[a] - 3) for a in range(D)])]
        for i in range(1, k):      # touching chain, gaps of 1e-3
            new.append(new[-1] + axis * (0.5 * (dd[i - 1] + dd[i]) + 1e-3))
        if all(fits(p, e) for p, e in zip(new, dd)):
            pts += new
            ds += dd
            clusters += 1
    assert clusters == (8 if D == 2 else 10)
    floor = 0
    for _ in range(4000):          # wide particles just touching the floor
        if floor == 3:
            break
        p = np.array([rng.uniform(3, n[a] - 3) for a in range(D)])
        p[D - 1] = 0.79999
        if fits(p, 1.6, floor=True):
            pts.append(p)
            ds.append(1.6)
            floor += 1
    assert floor == 3
    # both sides start from the same FP32-representable numbers: 1.6 rounded
    # to FP32 moves a radius by 1e-8, 1e-3 of the floor overlap
    X = np.array(pts).T.astype(np.float32).astype(np.float64)
    d = np.array(ds).astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    U = (3e-4 * rng.standard_normal((D, npart))).astype(np.float32).astype(np.float64)
    rp = np.full(npart, 2.5)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    cfg = P.make_config(lattice=lat, n=n, tau=0.8, gravity=g, n_sub=400, contact="lsd", bin_log2=bl)
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, steps=1, label="1 step")
    assert r["sim"].diagnostics()["active"] > 0
    assert r["eu"] <= 1e-5 and r["er"] <= 1e-6
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["efh"] <= 1e-5
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, steps=3, label="3 steps")
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["eu"] <= 1e-5 and r["er"] <= 1e-6


@pytest.mark.parametrize("k", [60, 150])
def test_big_island(P, orc, k):
    """150 particles linked by candidate pairs form one island larger than a
    wave.  Gaps alternate 2e-4 (pairs that collide head-on within the step)
    and 4e-3 (links that stay open), so the outcome is well conditioned.  (A
    chain of touching particles is not: a 1e-11 change of one position moves
    the FP64 result by 5e-4 within two steps.)"""
    _flush(f"island chain k={k}")
    n = (200, 12, 1)
    x = [10.0]
    for i in range(1, k):
        x.append(x[-1] + 0.5 + (0.0002 if i % 2 == 1 else 0.004))
    X = np.zeros((2, k))
    X[0] = x
    X[1] = 6.0
    X = X.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(3)
    U = np.zeros((2, k))
    U[0, 0::2], U[0, 1::2] = 1e-3, -1e-3
    U = (U + 1e-5 * rng.standard_normal((2, k))).astype(np.float32).astype(np.float64)
    d = np.full(k, 0.5)
    cfg = P.make_config(lattice=9, n=n, tau=0.8, gravity=(0, -1e-5, 0), n_sub=300, contact="lsd")
    r = _coupled_compare(P, orc, cfg, X, U, d, np.full(k, 2.5), steps=1, label="chain")
    dv = np.abs(r["got"]["v"] - r["out"]["U"]).max(axis=0)
    _flush(f"  worst particles {np.argsort(dv)[-5:].tolist()} dv {np.sort(dv)[-5:].tolist()}")
    assert r["sim"].diagnostics()["active"] == k
    assert np.abs(r["got"]["f_contact"]).max() > 0
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["eu"] <= 1e-5 and r["er"] <= 1e-6


@pytest.mark.parametrize("lat", [9, 19])
def test_resting_pile_lasting_contacts(P, orc, lat):
    """A small pile at rest on the floor: a bottom layer of touching
    candidates and a second layer in its hollows settle under gravity within
    a few steps and then stay in contact for the rest of the 60 steps, so
    the islands cannot jump over their sub-steps and the jump back-off runs
    step after step.  Every step has contact forces on the oracle's side.

    Particles: positions and velocities within the 1e-5 bound after 60
    steps.  Fluid: a resting particle's drag is the sub-step mean of a
    velocity that rattles in its contacts with an amplitude far above its
    mean, so the force it spreads is ill-conditioned; the oracle itself,
    started from positions moved by 1e-8 relative (below half an FP32 ulp),
    changes its fluid velocity by about 1e-3 (2D) and 4e-4 (3D) over the same
    60 steps.  The GPU's fluid error must stay below that change, measured
    here on the oracle alone."""
    _flush(f"resting pile {lat}")
    D = 2 if lat == 9 else 3
    pts = []
    if D == 2:
        n = (24, 12, 1)
        for k in range(10):
            pts.append((4.0 + 0.5002 * k, 0.2501))
        for k in range(9):
            pts.append((4.2501 + 0.5002 * k, 0.2501 + 0.4331 + 0.0003))
    else:
        n = (10, 10, 8)
        for i in range(3):
            for j in range(3):
                pts.append((3.5 + 0.5002 * i, 3.5 + 0.5002 * j, 0.2501))
        for i in range(2):
            for j in range(2):
                pts.append((3.7501 + 0.5002 * i, 3.7501 + 0.5002 * j, 0.2501 + 0.3536 + 0.0003))
    X = np.array(pts).T.astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    d = np.full(npart, 0.5)
    rp = np.full(npart, 2.5)
    U = np.zeros_like(X)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-4
    cfg = P.make_config(lattice=lat, n=n, tau=0.8, gravity=g, n_sub=400, contact="lsd")
    sim = P.Sim(cfg, npart)
    sim.set_particles(X, U, d, rp)
    oc = G.oracle_cfg(orc, cfg)
    sim0_h = sim.read_populations()
    f = G.to_oracle_f(orc, lat, sim0_h)
    Xo, Uo = X.copy(), U.copy()
    in_contact = []
    active = []
    for k in range(60):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
        in_contact.append(int((np.abs(out["fc"]).max(axis=0) > 0).sum()))
        sim.step(1)
        if k % 10 == 9:
            active.append(sim.diagnostics()["active"])
    sim.synchronize()
    got = sim.read_particles()
    eu, er, eh = G.field_errors(orc, lat, sim.read_populations(), f, sim.N)
    disp = np.abs(Xo - X).max()
    ex = np.abs(got["x"] - Xo).max() / disp
    ev = np.linalg.norm(got["v"] - Uo) / np.linalg.norm(Uo)
    # the oracle's own sensitivity: the same 60 steps from positions moved by
    # 1e-8 relative (seeded)
    Xp = X * (1.0 + 1e-8 * np.random.default_rng(1).standard_normal(X.shape))
    fp, Up = G.to_oracle_f(orc, lat, sim0_h), np.zeros_like(X)
    for k in range(60):
        outp = orc.step(oc, fp, Xp, Up, d, rp)
        fp, Xp, Up = outp["f"], outp["X"], outp["U"]
    wq = G.weights(orc, lat)
    eu_cond = G.field_errors(orc, lat, fp.reshape(-1, sim.N) - wq[:, None], f, sim.N)[0]
    _flush(f"  60 steps: eps_u={eu:.2e} (oracle's change under a 1e-8 input perturbation {eu_cond:.2e}) "
           f"eps_rho={er:.2e} eps_h={eh:.2e} dX={ex:.2e} (disp {disp:.2e}) dU={ev:.2e}; "
           f"particles in contact per step {in_contact[::10]}; active {active}")
    assert min(in_contact[5:]) >= npart // 2          # lasting contacts after the first few steps
    assert min(active) >= npart // 2
    assert eu <= eu_cond and eu <= 1e-3 and er <= 1e-6
    assert ex <= 1e-5 and ev <= 1e-5


@pytest.mark.parametrize("contact", ["lsd", "hertz"])
@pytest.mark.parametrize("lat", [9, 19])
def test_pairs_and_wall_singles_lasting_contact(P, orc, lat, contact):
    """Islands of one and two members, the ones the island kernel runs in
    its split form (four lanes per particle): pairs of touching particles
    stacked on the floor (gravity keeps them in contact), particles resting
    on the floor, and one pair whose members fly apart (its island jumps
    while the others sub-step).  40 steps against the oracle: particles
    within the 1e-5 bound;
    the fluid within the larger of 1e-5 and the oracle's own change under
    a 1e-8 relative move of the positions (resting contacts, as in the pile
    test)."""
    _flush(f"pairs and wall singles {lat} {contact}")
    D = 2 if lat == 9 else 3
    n = (32, 16, 1) if D == 2 else (16, 12, 12)
    rng = np.random.default_rng(8)
    pts, vel = [], []
    for k in range(5):                                    # pairs stacked on the floor
        base = np.array([3.0 + 2.5 * k, 6.0, 5.0][:D])
        if D == 3:
            base[1] = 3.0 + 1.5 * (k % 3)
        base[D - 1] = 0.2499
        for i in range(2):
            p = base.copy()
            p[D - 1] += 0.4999 * i
            p[0] += 0.01 * i
            pts.append(p)
            vel.append(np.zeros(D))
    for k in range(4):                                    # resting on the floor
        p = np.array([4.25 + 2.5 * k, 4.0, 7.0][:D])        # between the pairs
        p[D - 1] = 0.2499
        pts.append(p)
        vel.append(np.zeros(D))
    p = np.array([10.0, 10.0, 8.0][:D])                   # a pair flying apart
    for i, sgn in enumerate((-1.0, 1.0)):
        q = p.copy()
        q[0] += 0.4999 * i
        pts.append(q)
        v = np.zeros(D)
        v[0] = sgn * 2e-3
        vel.append(v)
    X = np.array(pts).T.astype(np.float32).astype(np.float64)
    U = np.array(vel).T.astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    d = np.full(npart, 0.5)
    rp = np.full(npart, 2.5)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-4
    cfg = P.make_config(lattice=lat, n=n, tau=0.8, gravity=g, n_sub=400, contact=contact, young=1e3)
    sim = P.Sim(cfg, npart)
    sim.set_particles(X, U, d, rp)
    oc = G.oracle_cfg(orc, cfg)
    h0 = sim.read_populations()
    f = G.to_oracle_f(orc, lat, h0)
    Xo, Uo = X.copy(), U.copy()
    touching = []
    for k in range(40):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
        touching.append(int((np.abs(out["fc"]).max(axis=0) > 0).sum()))
    sim.step(40)
    sim.synchronize()
    got = sim.read_particles()
    eu, er, eh = G.field_errors(orc, lat, sim.read_populations(), f, sim.N)
    disp = np.abs(Xo - X).max()
    ex = np.abs(got["x"] - Xo).max() / disp
    ev = np.linalg.norm(got["v"] - Uo) / np.linalg.norm(Uo)
    Xp = X * (1.0 + 1e-8 * np.random.default_rng(2).standard_normal(X.shape))
    fp, Up = G.to_oracle_f(orc, lat, h0), U.copy()
    for k in range(40):
        outp = orc.step(oc, fp, Xp, Up, d, rp)
        fp, Xp, Up = outp["f"], outp["X"], outp["U"]
    wq = G.weights(orc, lat)
    eu_cond = G.field_errors(orc, lat, fp.reshape(-1, sim.N) - wq[:, None], f, sim.N)[0]
    _flush(f"  40 steps: eps_u={eu:.2e} (oracle's own change {eu_cond:.2e}) eps_rho={er:.2e} dX={ex:.2e} "
           f"dU={ev:.2e}; particles in contact {touching[::8]}")
    # lasting contacts (the spring-dashpot pairs settle after a few bounces)
    assert min(touching[10:]) >= 10 if contact == "hertz" else np.mean(touching[20:]) >= 4
    assert ex <= 1e-5 and ev <= 1e-5
    assert eu <= max(1e-5, eu_cond) and er <= 1e-6


def test_soft_contact_parity(P, orc):
    _flush("soft contacts")
    n = (32, 32, 1)
    rng = np.random.default_rng(8)
    X = np.array([[10.0, 10.45, 20.0, 20.3, 15.0], [10.0, 10.05, 20.0, 20.2, 0.3]])
    X = X.astype(np.float32).astype(np.float64)
    U = (1e-3 * rng.standard_normal((2, 5))).astype(np.float32).astype(np.float64)
    cfg = P.make_config(lattice=9, n=n, tau=0.7, gravity=(0, -1e-5, 0), n_sub=1, contact="soft",
                        k_soft=1e-3)
    r = _coupled_compare(P, orc, cfg, X, U, np.full(5, 0.5), np.full(5, 2.5), steps=3, label="soft")
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5 and r["eu"] <= 1e-5


def test_c0_workload_100_steps(P, W, orc):
    """The 128^2 / 200-particle sedimentation case, 100 steps from rest."""
    _flush("c0 100 steps")
    w = W.C0
    X, U, d, rp = W.make_particles(w)
    cfg = P.config_from_workload(w)
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, steps=100, label="c0")
    assert r["eu"] <= 1e-5 and r["er"] <= 1e-6
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5


def test_deterministic_and_resume(P, W, orc):
    _flush("determinism + resume")
    w = W.C0.replace(n=(64, 64, 1), n_particles=300, region=(0.3, 1.0), seed=11)
    X, U, d, rp = W.make_particles(w)
    cfg = P.config_from_workload(w, n_sub=100)

    def run(steps, state=None):
        sim = P.Sim(cfg, X.shape[1])
        if state is None:
            sim.set_particles(X, U, d, rp)
        else:
            sim.write_populations(state[0])
            sim.set_particles(state[1], state[2], d, rp)
        sim.step(steps)
        p = sim.read_particles()
        return sim.read_populations(), p["x"], p["v"]

    a = run(20)
    b = run(20)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    mid = run(10)
    c = run(10, state=mid)
    assert np.array_equal(a[0], c[0])
    assert np.array_equal(a[1], c[1]) and np.array_equal(a[2], c[2])


def test_conservation_and_momentum(P, W, orc):
    """FP64 totals on the GPU against the oracle's, and the momentum balance
    while the disturbance stays away from the walls."""
    _flush("conservation")
    n = (48, 48, 1)
    rng = np.random.default_rng(12)
    npart = 40
    X = np.stack([rng.uniform(18, 30, npart), rng.uniform(18, 30, npart)])
    keep = [0]
    for i in range(1, npart):
        r = np.sqrt(((X[:, keep] - X[:, i:i + 1]) ** 2).sum(axis=0))
        if np.all(r > 0.5):
            keep.append(i)
    X = X[:, keep].astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    d = np.full(npart, 0.4)
    rp = np.full(npart, 2.5)
    U = np.zeros_like(X)
    cfg = P.make_config(lattice=9, n=n, tau=0.8, gravity=(0, -1e-5, 0), n_sub=50)
    sim = P.Sim(cfg, npart)
    sim.set_particles(X, U, d, rp)
    m0, p0 = sim.conservation()
    steps = 8
    sim.step(steps)
    m1, p1 = sim.conservation()
    N = sim.N
    assert abs(m0 - N) < 1e-9
    assert abs(m1 - m0) < steps * 9 * N * 2.0 ** -24 * 1e-4
    m = rp * np.pi * d ** 2 / 4
    Wsum = ((1 - 1 / rp) * m * cfg.gravity[1]).sum()
    assert abs((p1[1] - p0[1]) - steps * Wsum) < 1e-6 * abs(steps * Wsum)
    assert abs(p1[0] - p0[0]) < 1e-6 * abs(steps * Wsum)
    # the same totals from the oracle's state after the same steps
    oc = G.oracle_cfg(orc, cfg)
    f = orc.rest_state(oc)
    Xo, Uo = X.copy(), U.copy()
    for _ in range(steps):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
    e, w, _ = orc.tables(9)
    hdev = f.reshape(9, N) - w[:, None]
    p_ref = e[:, 1].astype(float) @ hdev.sum(axis=1) + (m * Uo[1]).sum()
    assert abs(p1[1] - p_ref) < 1e-5 * abs(p_ref)
    diag = sim.diagnostics()
    assert diag["nonfinite"] == 0 and diag["max_speed"] < 0.1


def test_skin_violation_is_reported(P):
    _flush("skin flag")
    cfg = P.make_config(lattice=9, n=(16, 16, 1), tau=0.8, n_sub=10, contact="lsd", skin=0.05)
    sim = P.Sim(cfg, 2)
    X = np.array([[4.0, 10.0], [8.0, 8.0]])
    U = np.array([[0.0, 0.04], [0.0, 0.0]])
    sim.set_particles(X, U, np.full(2, 0.4), np.full(2, 2.5))
    sim.step(1)
    with pytest.raises(P.PibmError) as ei:
        sim.synchronize()
    assert ei.value.name == "E_SKIN"
    sim.synchronize()                                           # latched flag was cleared


def test_particle_outside_box_rejected(P):
    cfg = P.make_config(lattice=9, n=(16, 16, 1))
    sim = P.Sim(cfg, 1)
    with pytest.raises(P.PibmError) as ei:
        sim.set_particles(np.array([[17.0], [3.0]]), None, np.array([0.4]), np.array([2.5]))
    assert ei.value.name == "E_ARG"


@pytest.mark.parametrize("lat", [9, 19])
def test_island_setup_paths_agree(P, lat):
    """The one-workgroup and the multi-kernel island set-up give bitwise
    identical steps (clusters, a large island, wall contacts)."""
    _flush(f"island set-up paths {lat}")
    D = 2 if lat == 9 else 3
    n = (48, 30, 1) if D == 2 else (20, 14, 18)
    rng = np.random.default_rng(43)
    pts = []
    for c in range(10):
        k = 2 + c % 6
        base = np.array([rng.uniform(3, n[a] - 3 - 0.5 * k) for a in range(D)])
        for i in range(k):
            p = base.copy()
            p[0] += 0.501 * i
            pts.append(p)
    base = np.array([4.0] * D)
    for i in range(9):                      # a 9 x 9 (x 1) sheet: one island of 81
        for j in range(9):
            p = base.copy()
            p[0] += 0.5005 * i
            p[1] += 0.5005 * j
            pts.append(p)
    X = np.array(pts).T.astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    d = np.full(npart, 0.5)
    U = (3e-4 * rng.standard_normal((D, npart))).astype(np.float32).astype(np.float64)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    out = []
    for mode in (1, 2):
        cfg = P.make_config(lattice=lat, n=n, tau=0.8, gravity=g, n_sub=200, contact="lsd", island_setup=mode)
        sim = P.Sim(cfg, npart)
        sim.set_particles(X, U, d, np.full(npart, 2.5))
        sim.step(3)
        sim.synchronize()
        p = sim.read_particles()
        out.append((sim.read_populations(), p["x"], p["v"], sim.diagnostics()["active"]))
    assert out[0][3] > 81
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)



@pytest.mark.parametrize("lat", [9, 19])
def test_dense_tile_spreads_unstaged(P, W, orc, lat):
    """More particles in one spreading tile's halo than it stages in LDS
    (384): those tiles read the particles from global memory instead; the
    coupled step must agree with the oracle all the same."""
    _flush(f"dense tile {lat}")
    D = 2 if lat == 9 else 3
    n = (48, 40, 1) if D == 2 else (20, 18, 16)
    rng = np.random.default_rng(77)
    npart = 900 if D == 2 else 700
    c = np.array([n[a] / 2 for a in range(D)])
    X = (c[:, None] + rng.uniform(-2.5 if D == 3 else -4.0, 2.5 if D == 3 else 4.0, (D, npart)))
    X = X.astype(np.float32).astype(np.float64)
    U = (1e-4 * rng.standard_normal((D, npart))).astype(np.float32).astype(np.float64)
    d = np.full(npart, 0.3)
    rp = np.full(npart, 2.5)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-5
    cfg = P.make_config(lattice=lat, n=n, tau=0.7, gravity=g, n_sub=20, contact="none")
    r = _coupled_compare(P, orc, cfg, X, U, d, rp, steps=2, label="dense")
    assert r["eu"] <= 1e-5 and r["er"] <= 1e-6 and r["efh"] <= 1e-5
    assert r["ex"] <= 1e-5 and r["ev"] <= 1e-5


def test_phase_times_sampled(P):
    """Phase events on every third step: 7 steps record 3 (the first, the
    fourth and the seventh), each phase non-negative."""
    _flush("phase times every 3")
    cfg = P.make_config(lattice=9, n=(32, 24, 1), tau=0.8, contact="lsd")
    sim = P.Sim(cfg, 2)
    X = np.array([[10.0, 20.0], [12.0, 12.5]])
    sim.set_particles(X, np.zeros((2, 2)), np.array([0.5, 0.5]), np.array([2.0, 2.0]))
    sim.set_profiling(True, every=3)
    sim.step(7)
    ph, n = sim.phase_times()
    assert n == 3
    assert all(v >= 0.0 for v in ph.values()) and ph["collide"] > 0.0
    sim.set_profiling(False)
    sim.step(2)
    ph, n = sim.phase_times()
    assert n == 0


@pytest.mark.parametrize("contact", ["lsd", "hertz"])
@pytest.mark.parametrize("lat", [9, 19])
def test_pairs_and_singles_closing_in(P, orc, lat, contact):
    """Islands of one and two that come into contact during the run, beside
    a pair resting on the floor in the same size class: particles settling
    onto the floor from small gaps, and particles settling onto a particle
    that rests on the floor (straight above it and off-centre).  Before the
    onset such an island jumps over contact-free stretches that shrink as
    the gap closes, checking again after each jump; after it, it sub-steps.
    30 steps against the oracle: particles within the 1e-5 bound, and every
    settling particle touches at some step."""
    _flush(f"pairs and singles closing in {lat} {contact}")
    D = 2 if lat == 9 else 3
    n = (32, 16, 1) if D == 2 else (16, 12, 12)
    r = 0.2499                                           # resting height (radius 0.25)

    def at(x, y, h):                                     # h along gravity (the last axis)
        return [x, h] if D == 2 else [x, y, h]

    pts = [at(2.0, 3.0, r + 2e-4), at(4.0, 5.0, r + 4e-4),            # settling onto the floor
           at(7.0, 3.0, r), at(7.0, 3.0, r + 0.5 + 2e-4),                # onto a resting particle
           at(10.0, 6.0, r), at(10.2, 6.0, r + np.sqrt(0.25 - 0.04) + 2e-4),   # off-centre
           at(13.0, 8.0, r), at(13.01, 8.0, r + 0.4999)]                 # resting pair
    X = np.array(pts).T.astype(np.float32).astype(np.float64)
    U = np.zeros_like(X)
    npart = X.shape[1]
    d = np.full(npart, 0.5)
    rp = np.full(npart, 2.5)
    g = [0.0, 0.0, 0.0]
    g[D - 1] = -1e-4
    cfg = P.make_config(lattice=lat, n=n, tau=0.8, gravity=g, n_sub=400, contact=contact, young=1e3)
    sim = P.Sim(cfg, npart)
    sim.set_particles(X, U, d, rp)
    oc = G.oracle_cfg(orc, cfg)
    f = G.to_oracle_f(orc, lat, sim.read_populations())
    Xo, Uo = X.copy(), U.copy()
    touched = np.zeros(npart, bool)
    for k in range(30):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
        touched |= np.abs(out["fc"]).max(axis=0) > 0
    sim.step(30)
    sim.synchronize()
    got = sim.read_particles()
    eu, er, eh = G.field_errors(orc, lat, sim.read_populations(), f, sim.N)
    disp = np.abs(Xo - X).max()
    ex = np.abs(got["x"] - Xo).max() / disp
    ev = np.linalg.norm(got["v"] - Uo) / np.linalg.norm(Uo)
    _flush(f"  30 steps: eps_u={eu:.2e} eps_rho={er:.2e} dX={ex:.2e} (disp {disp:.2e}) dU={ev:.2e}; "
           f"touched {touched.astype(int).tolist()}")
    assert touched[[0, 1, 3, 5]].all()         # every settling particle made contact
    assert ex <= 1e-5 and ev <= 1e-5
