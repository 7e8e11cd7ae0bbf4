"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (the same workload objects and default configuration).

The oracle cannot run these sizes for many steps, so the checks are:
  c1 (D2Q9 2048^2, 500k disks): two full coupled steps against the oracle
     (about 16 s of oracle time per step);
  c2/c3 (D3Q19 256^3, 2M spheres, FP32 and FP16 storage), one step from rest:
     - the cell list bit for bit against the oracle's,
     - a sample of free particles, integrated one by one by the oracle,
     - the whole force field against the oracle's spreading of the GPU's
       per-particle coefficients,
     - the whole collided and streamed lattice against the oracle's
       collision with the GPU's force field,
     - mass conservation;
  the 64^3 / 31,250-sphere crop with FP16 and FP32 storage against the oracle
  over three steps, and over its 100 steps against a stored oracle state;
  and the FP16 run of c2 against the FP32 run, ten steps.
Tolerances are the per-field bounds of the parity tests: FP32 velocity 1e-5
relative (L2), density 1e-6 absolute; FP16 storage 1e-3 and 1e-5.
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


def _particle_errors(got, Xo, Uo, X0, fh_ref=None):
    disp = np.abs(Xo - X0).max()
    ex = np.abs(got["x"] - Xo).max() / max(disp, 1e-30)
    ev = np.linalg.norm(got["v"] - Uo) / max(np.linalg.norm(Uo), 1e-30)
    efh = 0.0
    if fh_ref is not None:
        efh = np.linalg.norm(got["f_hydro"] - fh_ref) / max(np.linalg.norm(fh_ref), 1e-30)
    return ex, ev, efh


def test_c1_full_size_two_steps(P, W, orc):
    """D2Q9 2048^2 with 500k disks: every node and every particle after two
    coupled steps from rest against the oracle."""
    w = W.C1
    _flush(f"c1 full size: {w.n} {w.n_particles} particles, 2 steps")
    X, U, d, rp = W.make_particles(w)
    cfg = P.config_from_workload(w)
    sim = P.Sim(cfg, X.shape[1])
    h0 = sim.read_populations()
    sim.set_particles(X, U, d, rp)
    sim.step(1)
    x1 = sim.read_particles()["x"]
    sim.step(1)
    sim.synchronize()
    got = sim.read_particles()
    keys, ids, bs = sim.read_cell_list()
    h = sim.read_populations()

    oc = G.oracle_cfg(orc, cfg)
    # the cell list of the second step, from the GPU's positions after step
    # one (exact double-float values), bit for bit
    k_ref, p_ref, b_ref = orc.cell_list(oc, x1)
    f = G.to_oracle_f(orc, cfg.lattice, h0)
    Xo, Uo = X.copy(), U.copy()
    for k in range(2):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
    assert np.array_equal(keys.astype(np.int64), k_ref)
    assert np.array_equal(ids, p_ref)
    assert np.array_equal(bs.astype(np.int64), b_ref)
    eu, er, _ = G.field_errors(orc, cfg.lattice, h, f, sim.N)
    fh_ref = -np.pi * d ** 2 / 4 * out["gbar"]
    ex, ev, efh = _particle_errors(got, Xo, Uo, X, fh_ref)
    _flush(f"  eps_u={eu:.2e} eps_rho={er:.2e} dX={ex:.2e} dU={ev:.2e} dFh={efh:.2e} "
           f"active={sim.diagnostics()['active']}")
    assert eu <= 1e-5 and er <= 1e-6
    assert ex <= 1e-5 and ev <= 1e-5 and efh <= 1e-5


def _free_sample(X, d, n, k=400, clear=0.1, seed=0):
    """Indices of particles with every surface gap (to particles and walls)
    above `clear`: no contact can act on them within one step."""
    from scipy.spatial import cKDTree

    D = X.shape[0]
    tree = cKDTree(X.T)
    reach = float(d.max()) + clear
    dist, idx = tree.query(X.T, k=16, distance_upper_bound=reach)
    ok = np.ones(X.shape[1], bool)
    for c in range(1, 16):
        j = idx[:, c]
        valid = j < X.shape[1]
        jj = np.where(valid, j, 0)
        gap = dist[:, c] - 0.5 * (d + d[jj])
        ok &= ~(valid & (gap <= clear))
    for a in range(D):
        ok &= (X[a] - 0.5 * d > clear) & (n[a] - X[a] - 0.5 * d > clear)
    cand = np.flatnonzero(ok)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=min(k, cand.size), replace=False))


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_c2_full_size_one_step(P, W, orc, name):
    """D3Q19 256^3 with 2M spheres (FP32 and FP16 storage), one step from
    rest, in the benchmark's configuration."""
    w = W.WORKLOADS[name]
    _flush(f"{name} full size: {w.n} {w.n_particles} particles, storage {w.storage}")
    X, U, d, rp = W.make_particles(w)
    cfg = P.config_from_workload(w)
    sim = P.Sim(cfg, X.shape[1])
    h0 = sim.read_populations()
    m0, _ = sim.conservation()
    sim.set_particles(X, U, d, rp)
    sim.step(1)
    sim.synchronize()
    got = sim.read_particles()
    oc = G.oracle_cfg(orc, cfg)

    # cell list, bit for bit
    keys, ids, bs = sim.read_cell_list()
    k_ref, p_ref, b_ref = orc.cell_list(oc, X)
    assert np.array_equal(keys.astype(np.int64), k_ref)
    assert np.array_equal(ids, p_ref)
    assert np.array_equal(bs.astype(np.int64), b_ref)
    _flush("  cell list bit-exact")

    # free particles, one by one (from rest the interpolated moments are
    # exactly rho_i = 1, j_i = 0)
    s = _free_sample(X, d, w.n)
    assert s.size >= 200
    Xs, Us, gb, _, _ = orc.dem(oc, X[:, s], U[:, s], d[s], rp[s], np.ones(s.size), np.zeros((3, s.size)),
                               pairs=np.zeros((0, 2), np.int32))
    fh_ref = -np.pi * d[s] ** 2 / 4 * gb
    sub = {k: v[:, s] for k, v in got.items()}
    ex, ev, efh = _particle_errors(sub, Xs, Us, X[:, s], fh_ref)
    _flush(f"  {s.size} free particles: dX={ex:.2e} dU={ev:.2e} dFh={efh:.2e}")
    assert ex <= 1e-5 and ev <= 1e-5 and efh <= 1e-5

    # spreading: the GPU force field against the oracle's spreading of the
    # GPU's coefficients A_p gbar_p at the start-of-step positions
    F = sim.read_force().astype(np.float64)
    F_ref = orc.spread(oc, X, -got["f_hydro"]).reshape(3, -1)
    eF = np.abs(F - F_ref).max() / np.abs(F_ref).max()
    _flush(f"  force field: max rel {eF:.2e}  |F|max {np.abs(F_ref).max():.2e}")
    assert eF <= 1e-5
    del F_ref

    # collision and streaming of the whole lattice with the GPU's force
    f0 = G.to_oracle_f(orc, cfg.lattice, h0)
    del h0
    f1 = orc.collide_stream(oc, f0, F)
    del f0
    eu, er, _ = G.field_errors(orc, cfg.lattice, sim.read_populations(), f1, sim.N)
    tol_u, tol_r = (1e-5, 1e-6) if w.storage == "fp32" else (1e-3, 1e-5)
    _flush(f"  lattice: eps_u={eu:.2e} eps_rho={er:.2e}")
    assert eu <= tol_u and er <= tol_r
    del f1

    m1, _ = sim.conservation()
    bound = 1e-6 if w.storage == "fp32" else 1e-4
    _flush(f"  mass change {abs(m1 - m0) / m0:.2e}")
    assert abs(m1 - m0) / m0 <= bound


def test_fp16_crop_against_oracle(P, W, orc):
    """The 64^3 walled crop (31,250 spheres, same number density and
    diameters as c2), FP16 and FP32 storage, three steps from rest."""
    w = W.C3_CROP
    _flush(f"crop {w.n} {w.n_particles}")
    X, U, d, rp = W.make_particles(w)
    res = {}
    for storage in ("fp16", "fp32"):
        cfg = P.config_from_workload(w.replace(storage=storage))
        sim = P.Sim(cfg, X.shape[1])
        sim.set_particles(X, U, d, rp)
        sim.step(3)
        sim.synchronize()
        res[storage] = (sim.read_populations(), sim.read_particles(), sim.N)
    oc = G.oracle_cfg(orc, cfg)
    f = orc.rest_state(oc)
    Xo, Uo = X.copy(), U.copy()
    for _ in range(3):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
    for storage, (h, got, N) in res.items():
        eu, er, _ = G.field_errors(orc, w.lattice, h, f, N)
        ex, ev, _ = _particle_errors(got, Xo, Uo, X)
        _flush(f"  {storage}: eps_u={eu:.2e} eps_rho={er:.2e} dX={ex:.2e} dU={ev:.2e}")
        tol_u, tol_r, tol_p = (1e-5, 1e-6, 1e-5) if storage == "fp32" else (1e-3, 1e-5, 1e-3)
        assert eu <= tol_u and er <= tol_r
        assert ex <= tol_p and ev <= tol_p


def test_crop_100_steps_against_stored_oracle(P, W, orc):
    """The 64^3 crop over its full 100 steps, FP32 and FP16 storage, against
    the FP64 oracle's state after the same 100 steps, written beforehand by
    tests/golden/make_crop_reference.py (density deviation and velocity at
    32,768 sampled nodes, every particle's displacement and velocity).
    Bounds: the per-field bounds of the one-step tests, unchanged over the
    hundred steps (FP32: velocity 1e-5, density 1e-6, particles 1e-5; FP16
    storage: velocity 1e-3, density 1e-5, and particles 1e-3, since they
    follow a fluid known to 1e-3)."""
    import os

    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "crop64_fp64_100steps.npz"))
    steps = int(ref["steps"])
    nodes = ref["nodes"].astype(np.int64)
    w = W.C3_CROP
    _flush(f"crop {w.n} {w.n_particles}, {steps} steps against the stored oracle state")
    X, U, d, rp = W.make_particles(w)
    dx_ref, v_ref = ref["dx"].astype(np.float64), ref["v"].astype(np.float64)
    u_ref, dr_ref = ref["u"].astype(np.float64), ref["drho"].astype(np.float64)
    for storage in ("fp32", "fp16"):
        cfg = P.config_from_workload(w.replace(storage=storage))
        sim = P.Sim(cfg, X.shape[1])
        sim.set_particles(X, U, d, rp)
        sim.step(steps)
        sim.synchronize()
        h = sim.read_populations()[:, nodes]
        dr, j = G.moments_dev(orc, w.lattice, h)
        u = j / (1.0 + dr)
        eu = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        er = np.abs(dr - dr_ref).max()
        got = sim.read_particles()
        dx = got["x"] - X
        ex = np.abs(dx - dx_ref).max() / np.abs(dx_ref).max()
        ev = np.linalg.norm(got["v"] - v_ref) / np.linalg.norm(v_ref)
        _flush(f"  {storage}: eps_u={eu:.2e} eps_rho={er:.2e} dX={ex:.2e} dU={ev:.2e}")
        tu, tr, tp = (1e-5, 1e-6, 1e-5) if storage == "fp32" else (1e-3, 1e-5, 1e-3)
        assert eu <= tu and er <= tr
        assert ex <= tp and ev <= tp


def test_fp16_scale_reading(P, W, orc):
    """FP16 storage of f - w with the deviations scaled by 2^14 against the
    unscaled form (scale 2^0), on the 64^3 crop over three steps: slow-flow
    deviations of 1e-7..1e-5 fall in FP16's subnormal range without the
    scale, so the scaled form must be clearly more accurate."""
    w = W.C3_CROP
    X, U, d, rp = W.make_particles(w)
    res = {}
    for sl2 in (14, 0):
        cfg = P.config_from_workload(w, fp16_scale_log2=sl2)
        sim = P.Sim(cfg, X.shape[1])
        sim.set_particles(X, U, d, rp)
        sim.step(3)
        sim.synchronize()
        res[sl2] = (sim.read_populations(), sim.N)
    oc = G.oracle_cfg(orc, P.config_from_workload(w))
    f = orc.rest_state(oc)
    Xo, Uo = X.copy(), U.copy()
    for _ in range(3):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
    e = {sl2: G.field_errors(orc, w.lattice, h, f, N)[:2] for sl2, (h, N) in res.items()}
    _flush(f"  scale 2^14: eps_u={e[14][0]:.2e} eps_rho={e[14][1]:.2e};  scale 2^0: eps_u={e[0][0]:.2e} "
           f"eps_rho={e[0][1]:.2e}")
    assert e[14][0] <= 1e-3 and e[14][1] <= 1e-5
    assert e[0][0] > 10 * e[14][0]


def test_fp16_against_fp32_full_size(P, W, orc):
    """c3 (FP16 storage) against c2 (FP32) from the same initial state, ten
    steps, same error measures."""
    _flush("c3 vs c2, 10 steps")
    X, U, d, rp = W.make_particles(W.C2)
    out = {}
    for w in (W.C2, W.C3):
        sim = P.Sim(P.config_from_workload(w), X.shape[1])
        sim.set_particles(X, U, d, rp)
        sim.step(10)
        sim.synchronize()
        h = sim.read_populations()
        out[w.storage] = G.moments_dev(orc, w.lattice, h)
        del sim, h
    dr32, j32 = out["fp32"]
    dr16, j16 = out["fp16"]
    u32 = j32 / (1 + dr32)
    u16 = j16 / (1 + dr16)
    eu = np.linalg.norm(u16 - u32) / np.linalg.norm(u32)
    er = np.abs(dr16 - dr32).max()
    _flush(f"  fp16 vs fp32: eps_u={eu:.2e} eps_rho={er:.2e}")
    assert eu <= 1e-3 and er <= 1e-5
