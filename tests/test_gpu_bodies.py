"""GPU parity of fixed obstacle bodies (the hybrid IBM-PIBM case of Sec. 3.3)
against the FP64 oracle, through the C ABI: a sphere of IBM surface points
with their own areas and a row of fixed PIBM points, moving particles
resting on and touching them, with the spring-dashpot, Hertz and
Hertz-Mindlin contacts.  Compared after one and three steps: the fluid,
the moving particles, the per-body hydrodynamic and contact forces and
torques; fixed points must not move.

Bounds: fluid velocity 1e-5 relative (L2), density 1e-6; moving particles
1e-5 relative; body forces and torques 1e-5 relative (L2 over the bodies).
"""
import numpy as np
import pytest

from tests import gpu_helpers as G
from tests.test_oracle_bodies import _scene

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


def _body_sums(X, fh, fcn, body, nb):
    D = X.shape[0]
    out = {k: np.zeros((3, nb)) for k in ("f_hydro", "f_contact", "torque")}
    for b in range(nb):
        sel = body == b
        cen = X[:, sel].mean(1)
        out["f_hydro"][:D, b] = fh[:, sel].sum(1)
        out["f_contact"][:D, b] = fcn[:, sel].sum(1)
        r = np.zeros((3, sel.sum()))
        r[:D] = X[:, sel] - cen[:, None]
        ft = np.zeros((3, sel.sum()))
        ft[:D] = fh[:, sel] + fcn[:, sel]
        out["torque"][:, b] = np.cross(r.T, ft.T).sum(0)
    return out


@pytest.mark.parametrize("D,contact", [(2, "lsd"), (3, "lsd"), (3, "hertz"), (3, "hertz_mindlin"),
                                       (3, "hertz_mindlin_microslip")])
def test_fixed_bodies_match_oracle(P, orc, D, contact):
    _flush(f"fixed bodies {D}D {contact}")
    ocfg, X, U, d, rp, fixed, area = _scene(orc, D, contact)
    nshell = int((area > 0).sum()) - 3
    body = np.where(fixed == 1, 0, -1).astype(np.int32)
    body[nshell:nshell + 3] = 1                         # the row of PIBM points is body 1
    X = X.astype(np.float32).astype(np.float64)
    U = U.astype(np.float32).astype(np.float64)
    cfg = P.make_config(lattice=ocfg.lattice, n=tuple(ocfg.n), tau=ocfg.tau, gravity=tuple(ocfg.gravity),
                        n_sub=ocfg.n_sub, contact=contact, kn=ocfg.kn, restitution=ocfg.restitution,
                        young=ocfg.young, poisson=ocfg.poisson, friction=ocfg.friction, skin=ocfg.skin,
                        bodies=1)
    sim = P.Sim(cfg, X.shape[1])
    sim.set_particles(X, U, d, rp)
    sim.set_bodies(body, area=np.where(fixed == 1, area, 0.0))
    oc = G.oracle_cfg(orc, cfg)
    f = G.to_oracle_f(orc, cfg.lattice, sim.read_populations())
    Xo, Uo, Wo, hist = X.copy(), U.copy(), np.zeros((3, X.shape[1])), None
    mv = fixed == 0
    for steps in (1, 2):
        for _ in range(steps):
            out = orc.step_full(oc, f, Xo, Uo, d, rp, W=Wo, hist=hist, fixed=fixed, area=area)
            f, Xo, Uo, Wo, hist = out["f"], out["X"], out["U"], out["W"], out["hist"]
        sim.step(steps)
        sim.synchronize()
        got = sim.read_particles()
        bod = sim.read_bodies(2)
        ref = _body_sums(Xo, -(area * out["gbar"]), out["fc"], body, 2)
        eu, er, _ = G.field_errors(orc, cfg.lattice, sim.read_populations(), f, sim.N)
        ex = np.abs(got["x"][:, mv] - Xo[:, mv]).max() / np.abs(Xo[:, mv] - X[:, mv]).max()
        ev = np.linalg.norm(got["v"][:, mv] - Uo[:, mv]) / np.linalg.norm(Uo[:, mv])
        eb = {k: np.linalg.norm(bod[k] - ref[k]) / max(np.linalg.norm(ref[k]), 1e-30) for k in ref}
        _flush(f"  {steps} step(s): eps_u={eu:.2e} eps_rho={er:.2e} dX={ex:.2e} dU={ev:.2e} "
               + " ".join(f"{k}={v:.2e}" for k, v in eb.items())
               + f" |F_contact|={np.abs(ref['f_contact']).max():.2e}")
        assert np.array_equal(got["x"][:, ~mv], X[:, ~mv]) and np.all(got["v"][:, ~mv] == 0)
        assert eu <= 1e-5 and er <= 1e-6
        assert ex <= 1e-5 and ev <= 1e-5
        assert eb["f_hydro"] <= 1e-5 and eb["f_contact"] <= 1e-5 and eb["torque"] <= 1e-5
        assert np.abs(ref["f_contact"]).max() > 0


def test_bodies_need_the_option(P):
    cfg = P.make_config(lattice=9, n=(16, 16, 1), contact="lsd")
    sim = P.Sim(cfg, 2)
    X = np.array([[5.0, 9.0], [5.0, 9.0]])
    sim.set_particles(X, np.zeros((2, 2)), np.full(2, 0.5), np.full(2, 2.0))
    with pytest.raises(P.PibmError):
        sim.set_bodies(np.array([0, -1]))
    cfg = P.make_config(lattice=9, n=(16, 16, 1), contact="lsd", bodies=1)
    sim = P.Sim(cfg, 2)
    sim.set_particles(X, np.array([[1e-3, 0.0], [0.0, 0.0]]), np.full(2, 0.5), np.full(2, 2.0))
    sim.set_bodies(np.array([0, -1]))
    sim.step(3)
    p = sim.read_particles()
    assert np.array_equal(p["x"][:, 0], X[:, 0]) and np.all(p["v"][:, 0] == 0)   # velocity was cleared
    with pytest.raises(P.PibmError):
        sim.set_bodies(np.array([0, -1]))


def test_hybrid_workload_runs(P):
    """The hybrid workload at its full size (250k moving spheres above four
    IBM spheres and a 27-point cube, 128^3): a few steps in the benchmark's
    configuration; the obstacle points stay put, the step status is clean,
    and the bodies carry the settling load as it builds up."""
    from paper_1407_6704_amd import workloads as W

    w = W.HYBRID
    X, U, d, rp, body, area = W.make_hybrid(w)
    _flush(f"hybrid {w.n} {X.shape[1]} points, {(body >= 0).sum()} fixed")
    sim = P.Sim(P.config_from_workload(w), X.shape[1])
    sim.set_particles(X, U, d, rp)
    sim.set_bodies(body, area)
    sim.step(5)
    sim.synchronize()
    p = sim.read_particles()
    fx = body >= 0
    assert np.array_equal(p["x"][:, fx], X[:, fx]) and np.all(p["v"][:, fx] == 0)
    bf = sim.read_bodies(5)
    assert np.all(np.isfinite(bf["f_hydro"])) and np.all(np.isfinite(bf["torque"]))
    assert sim.diagnostics()["nonfinite"] == 0
