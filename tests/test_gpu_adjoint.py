"""GPU parity of the hand-written adjoint (pibm_forward_ckpt + pibm_backward,
called through the C ABI) for J = mean particle height after T steps.

  - against autograd through the FP64 differentiable reference
    (oracle/torch_ref.py, itself pinned to the C oracle) on small cases with
    soft contacts engaged, a wall contact and particles near walls, in 2D
    and 3D: gradients with respect to tau, gravity, the initial velocities
    and the initial positions, 1e-4 relative;
  - on the 64^2 / 50-particle copy of the differentiation workload over 2000
    steps with checkpoints every 100 steps, against central differences of
    the FP64 C oracle, 1e-4 relative (dJ/dv0 as a vector: L2 over sampled
    components, and each component's error against the largest), and over
    300 steps against autograd through the FP64 reference, every component;
  - invariance of the gradients to the checkpoint interval (bitwise: the
    re-run reproduces the forward exactly, and the last segment, which the
    forward pass tapes as it runs it, equals its re-run; K >= T tapes the
    whole rollout), a second objective reversed on the same recording (whose
    last segment is then re-run), and the context's state after the rollout
    and after the backward pass.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1407_6704_amd import pibm
    pibm.load()
    return pibm


def _flush(msg):
    print(msg, flush=True)


def _small_case(lattice, seed):
    rng = np.random.default_rng(seed)
    if lattice == 9:
        n = (24, 20, 1)
        X = np.array([[6.0, 6.42, 12.0, 12.3, 18.0, 3.0, 20.0, 9.0],
                      [8.0, 8.1, 12.0, 12.38, 6.0, 0.2, 15.0, 17.0]])
        rp = rng.uniform(1.8, 3.0, X.shape[1])
    else:
        n = (12, 10, 9)
        X = np.array([[4.0, 4.45, 8.0, 6.0, 2.0],
                      [4.0, 4.05, 6.0, 7.0, 5.0],
                      [4.0, 4.1, 5.0, 0.22, 7.0]])
        rp = rng.uniform(7.0, 9.0, X.shape[1])      # explicit drag stable with one sub-step
    X = (X + 0.01 * rng.standard_normal(X.shape)).astype(np.float32).astype(np.float64)
    npart = X.shape[1]
    d = np.full(npart, 0.5)
    rp = rp.astype(np.float32).astype(np.float64)
    U = (1e-3 * rng.standard_normal(X.shape)).astype(np.float32).astype(np.float64)
    return n, X, U, d, rp


def _gpu_grads(P, lattice, n, X, U, d, rp, tau, g, steps, K, storage="fp32"):
    D = X.shape[0]
    grav = [0.0, 0.0, 0.0]
    grav[D - 1] = -g
    cfg = P.make_config(lattice=lattice, n=n, tau=tau, gravity=grav, contact="soft", k_soft=2e-3, skin=0.05,
                        n_sub=1, storage=storage)
    sim = P.Sim(cfg, X.shape[1])
    sim.set_particles(X, U, d, rp)
    sim.forward_ckpt(steps, K)
    xT = sim.read_particles()["x"]
    dJdx = np.zeros_like(X)
    dJdx[D - 1] = 1.0 / X.shape[1]
    r = sim.backward(dJ_dx=dJdx)
    r["xT"] = xT
    r["sim"] = sim
    return r


def _ref_grads(lattice, n, X, U, d, rp, tau, g, steps):
    import torch

    from oracle import torch_ref as TR

    D = X.shape[0]
    ref = TR.Ref(lattice, n, d, rp, k_soft=2e-3, contact="soft", n_sub=1)
    t_tau = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    t_g = torch.zeros(D, dtype=torch.float64)
    t_g[D - 1] = -g
    t_g.requires_grad_(True)
    t_U = torch.tensor(U, requires_grad=True)
    t_X = torch.tensor(X, requires_grad=True)
    _, XT, _ = ref.rollout(t_X, t_U, t_tau, t_g, steps)
    J = XT[D - 1].mean()
    J.backward()
    return {"dtau": t_tau.grad.item(), "dgravity": t_g.grad.numpy(), "dv0": t_U.grad.numpy(),
            "dx0": t_X.grad.numpy(), "xT": XT.detach().numpy()}


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("lattice", [9, 19, 15])
def test_adjoint_matches_autograd_reference(P, lattice):
    n, X, U, d, rp = _small_case(lattice, 5)
    tau, g, steps, K = 0.7, 1e-3, 15, 4
    _flush(f"adjoint vs autograd reference: lattice {lattice} n={n} np={X.shape[1]} T={steps} K={K}")
    gpu = _gpu_grads(P, lattice, n, X, U, d, rp, tau, g, steps, K)
    ref = _ref_grads(lattice, n, X, U, d, rp, tau, g, steps)
    D = X.shape[0]
    e = {"xT": np.abs(gpu["xT"] - ref["xT"]).max(),
         "dtau": _rel(gpu["dtau"], ref["dtau"]),
         "dg": _rel(gpu["dgravity"][:D], ref["dgravity"]),
         "dv0": _rel(gpu["dv0"], ref["dv0"]),
         "dx0": _rel(gpu["dx0"], ref["dx0"])}
    _flush("  " + " ".join(f"{k}={v:.2e}" for k, v in e.items()) +
           f"  (dJ/dtau {ref['dtau']:.4e}, dJ/dg {ref['dgravity'][D - 1]:.4e})")
    assert e["xT"] <= 1e-5
    assert e["dtau"] <= 1e-4 and e["dg"] <= 1e-4 and e["dv0"] <= 1e-4 and e["dx0"] <= 1e-4


def test_checkpoint_interval_invariance_and_state(P):
    lattice = 9
    n, X, U, d, rp = _small_case(lattice, 6)
    tau, g, steps = 0.7, 1e-3, 12
    _flush("checkpoint interval invariance")
    runs = [_gpu_grads(P, lattice, n, X, U, d, rp, tau, g, steps, K) for K in (1, 5, 12, 50)]
    for r in runs[1:]:
        assert r["dtau"] == runs[0]["dtau"]
        assert r["dgravity"] == runs[0]["dgravity"]
        assert np.array_equal(r["dv0"], runs[0]["dv0"])
        assert np.array_equal(r["dx0"], runs[0]["dx0"])
    # the recorded forward equals plain stepping, and backward leaves the
    # final state in place
    cfg = P.make_config(lattice=lattice, n=n, tau=tau, gravity=(0.0, -g, 0.0), contact="soft", k_soft=2e-3,
                        skin=0.05, n_sub=1)
    plain = P.Sim(cfg, X.shape[1])
    plain.set_particles(X, U, d, rp)
    plain.step(steps)
    sim = runs[1]["sim"]
    assert np.array_equal(sim.read_populations(), plain.read_populations())
    a, b = sim.read_particles(), plain.read_particles()
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["v"], b["v"])
    # a second objective on the same recording (dJ/dU_T only)
    r2 = sim.backward(dJ_dv=np.ones_like(X))
    assert np.isfinite(r2["dtau"]) and np.all(np.isfinite(r2["dv0"]))


def test_adjoint_fp16_storage_close_to_fp32(P):
    lattice = 9
    n, X, U, d, rp = _small_case(lattice, 7)
    tau, g, steps, K = 0.7, 1e-3, 10, 3
    a = _gpu_grads(P, lattice, n, X, U, d, rp, tau, g, steps, K, storage="fp32")
    b = _gpu_grads(P, lattice, n, X, U, d, rp, tau, g, steps, K, storage="fp16")
    e = (_rel(b["dtau"], a["dtau"]), _rel(b["dv0"], a["dv0"]), _rel(b["dgravity"], a["dgravity"]))
    _flush(f"fp16 vs fp32 adjoint: dtau {e[0]:.2e} dv0 {e[1]:.2e} dg {e[2]:.2e}")
    assert max(e) <= 1e-2


def test_adjoint_against_oracle_central_differences(P, orc):
    """The 64^2 / 50-particle copy of the differentiation workload, 2000
    steps, checkpoints every 100 steps."""
    from paper_1407_6704_amd import workloads as W

    w = W.C4_FD
    X, U, d, rp = W.make_particles(w)
    rng = np.random.default_rng(17)
    U = (2e-5 * rng.standard_normal(X.shape)).astype(np.float32).astype(np.float64)
    steps, K = w.steps, 100
    D = X.shape[0]
    g = w.gravity
    _flush(f"adjoint vs oracle central differences: {w.n} np={X.shape[1]} T={steps} K={K}")
    gpu = _gpu_grads(P, w.lattice, w.n, X, U, d, rp, w.tau, g, steps, K)

    def J(tau=w.tau, gg=g, U_=U):
        grav = [0.0, 0.0, 0.0]
        grav[D - 1] = -gg
        oc = orc.make_cfg(lattice=w.lattice, n=w.n, tau=tau, gravity=grav, contact="soft", k_soft=2e-3,
                          skin=0.05, n_sub=1, two_way=1)
        f = orc.rest_state(oc)
        Xo, Uo = X.copy(), U_.copy()
        for _ in range(steps):
            r = orc.step(oc, f, Xo, Uo, d, rp)
            f, Xo, Uo = r["f"], r["X"], r["U"]
        return (Xo[D - 1] - X[D - 1]).mean()

    h = 1e-4
    fd_tau = (J(tau=w.tau + h) - J(tau=w.tau - h)) / (2 * h)
    h = 1e-8
    fd_gy = -(J(gg=g + h) - J(gg=g - h)) / (2 * h)           # gravity_y = -g
    e_tau = _rel(gpu["dtau"], fd_tau)
    e_g = _rel(gpu["dgravity"][D - 1], fd_gy)
    _flush(f"  dJ/dtau gpu {gpu['dtau']:.6e} fd {fd_tau:.6e} rel {e_tau:.2e}")
    _flush(f"  dJ/dg_y gpu {gpu['dgravity'][D - 1]:.6e} fd {fd_gy:.6e} rel {e_g:.2e}")
    # dJ/dv0 is a vector: its error is measured relative to the vector's
    # size (L2 over the sampled components, each component against the
    # largest); single components can be small through cancellation
    h = 1e-6
    got, fds = [], []
    for (a, p) in ((1, 0), (1, 7), (0, 23), (1, 41), (0, 3), (1, 29)):
        Up, Um = U.copy(), U.copy()
        Up[a, p] += h
        Um[a, p] -= h
        fd = (J(U_=Up) - J(U_=Um)) / (2 * h)
        got.append(gpu["dv0"][a, p])
        fds.append(fd)
        _flush(f"  dJ/dv0[{a},{p}] gpu {gpu['dv0'][a, p]:.6e} fd {fd:.6e} rel {_rel(gpu['dv0'][a, p], fd):.2e}")
    got, fds = np.array(got), np.array(fds)
    e_v = _rel(got, fds)
    e_vmax = np.abs(got - fds).max() / np.abs(fds).max()
    _flush(f"  dJ/dv0 sampled: L2-relative {e_v:.2e}, max component error / max component {e_vmax:.2e}")
    assert e_tau <= 1e-4 and e_g <= 1e-4
    assert e_v <= 1e-4 and e_vmax <= 1e-4


def test_adjoint_c4_copy_against_autograd(P):
    """The 64^2 / 50-particle copy over 300 steps against autograd through
    the FP64 reference: every component of every gradient."""
    from paper_1407_6704_amd import workloads as W

    w = W.C4_FD
    X, U, d, rp = W.make_particles(w)
    rng = np.random.default_rng(17)
    U = (2e-5 * rng.standard_normal(X.shape)).astype(np.float32).astype(np.float64)
    steps, K = 300, 100
    _flush(f"adjoint vs autograd reference: {w.n} np={X.shape[1]} T={steps} K={K}")
    gpu = _gpu_grads(P, w.lattice, w.n, X, U, d, rp, w.tau, w.gravity, steps, K)
    ref = _ref_grads(w.lattice, w.n, X, U, d, rp, w.tau, w.gravity, steps)
    D = X.shape[0]
    e = {"xT": np.abs(gpu["xT"] - ref["xT"]).max(),
         "dtau": _rel(gpu["dtau"], ref["dtau"]),
         "dg": _rel(gpu["dgravity"][:D], ref["dgravity"]),
         "dv0": _rel(gpu["dv0"], ref["dv0"]),
         "dv0_max_comp": np.max(np.abs(gpu["dv0"] - ref["dv0"]) / np.abs(ref["dv0"])),
         "dx0": _rel(gpu["dx0"], ref["dx0"])}
    _flush("  " + " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert e["dtau"] <= 1e-4 and e["dg"] <= 1e-4 and e["dv0"] <= 1e-4 and e["dx0"] <= 1e-3


def test_adjoint_rejects_unsupported_and_edge_cases(P):
    """Unsupported forms are refused with PIBM_E_CONFIG; a rollout of zero
    steps returns the final-state adjoints unchanged; K larger than the
    rollout is one segment."""
    n, X, U, d, rp = _small_case(9, 8)
    for kw in (dict(contact="lsd", n_sub=1), dict(contact="soft", n_sub=4), dict(contact="soft", bin_log2=1),
               dict(contact="hertz", n_sub=1), dict(contact="soft", interp="lagrange"),
               dict(contact="soft", bodies=1), dict(contact="hertz_mindlin", young=1e-3)):
        cfg = P.make_config(lattice=9, n=n, tau=0.7, gravity=(0.0, -1e-3, 0.0), k_soft=2e-3, skin=0.05, **kw)
        sim = P.Sim(cfg, X.shape[1])
        sim.set_particles(X, U, d, rp)
        assert sim.lib.pibm_rollout_bytes(sim.ctx, 10, 5) == 0
        with pytest.raises(P.PibmError):
            sim.forward_ckpt(10, 5)
    cfg = P.make_config(lattice=9, n=n, tau=0.7, gravity=(0.0, -1e-3, 0.0), contact="soft", k_soft=2e-3,
                        skin=0.05, n_sub=1)
    sim = P.Sim(cfg, X.shape[1])
    sim.set_particles(X, U, d, rp)
    sim.forward_ckpt(0, 4)
    gx = np.arange(X.size, dtype=np.float64).reshape(X.shape) * 1e-3
    gv = -gx
    r = sim.backward(dJ_dx=gx, dJ_dv=gv)
    assert np.array_equal(r["dx0"], gx.astype(np.float32)) and np.array_equal(r["dv0"], gv.astype(np.float32))
    assert r["dtau"] == 0.0 and r["dgravity"] == [0.0, 0.0, 0.0]
    a = _gpu_grads(P, 9, n, X, U, d, rp, 0.7, 1e-3, 6, 50)
    b = _gpu_grads(P, 9, n, X, U, d, rp, 0.7, 1e-3, 6, 6)
    assert a["dtau"] == b["dtau"] and np.array_equal(a["dv0"], b["dv0"])

