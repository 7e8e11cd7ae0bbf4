"""The single-particle settling study (Sec. 3.1, Table 2) on the GPU:
D3Q15, Lagrange-polynomial gather, 10 x 10 x 50 walled cavity, the four
diameters with their relaxation times and time steps.

* parity: the first 300 steps of the h/d = 1 and h/d = 4 rows against the
  FP64 oracle (fluid velocity and particle height and speed), with the
  bounds of the other parity tests: FP32 velocity 1e-5 relative (L2),
  particle speed 1e-5 relative;
* the settling speeds after 20,000 steps against the FP64 oracle's run of
  the same study (tests/golden/table2_oracle_settling.json), increasing with
  the diameter.  The paper's own numbers agree with Stokes' law (Eq. lbm14)
  to 1.5 % after a calibration it does not print; with this reading of the
  momentum exchange both the oracle and the GPU give 0.92 .. 1.22 times the
  Stokes speed.
"""
import numpy as np
import pytest

from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1407_6704_amd import pibm, settling
    pibm.load()
    return settling


def _flush(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("row", [0, 3])
@pytest.mark.parametrize("interp", ["lagrange", "delta"])
def test_settling_start_matches_oracle(S, orc, row, interp):
    from paper_1407_6704_amd import pibm

    steps = 300
    r = S.TABLE2[row]
    _flush(f"settling row {row} {interp}: {steps} steps against the oracle")
    cfg, X, U, d, rp, dt = S.case(r, interp=interp)
    sim = pibm.Sim(cfg, 1)
    sim.set_particles(X, U, d, rp)
    sim.step(steps)
    sim.synchronize()
    got = sim.read_particles()
    oc = G.oracle_cfg(orc, cfg)
    f = orc.rest_state(oc)
    Xo, Uo = X.copy(), U.copy()
    for _ in range(steps):
        out = orc.step(oc, f, Xo, Uo, d, rp)
        f, Xo, Uo = out["f"], out["X"], out["U"]
    eu, er, _ = G.field_errors(orc, cfg.lattice, sim.read_populations(), f, sim.N)
    ev = np.linalg.norm(got["v"] - Uo) / np.linalg.norm(Uo)
    ez = abs(got["x"][2, 0] - Xo[2, 0]) / abs(Xo[2, 0] - X[2, 0])
    _flush(f"  eps_u={eu:.2e} eps_rho={er:.2e} dU={ev:.2e} dZ={ez:.2e} (fall {X[2, 0] - Xo[2, 0]:.2e})")
    assert eu <= 1e-5 and er <= 1e-6
    assert ev <= 1e-5 and ez <= 1e-5


def test_settling_speeds_against_oracle(S):
    """20,000 steps of each Table 2 row: the settling speed (mean vertical
    speed over the last tenth of the run, sampled every 1000 steps) against
    the FP64 oracle's run of the same steps, stored by
    tests/golden/make_table2_reference.py (only the oracle runs there), to
    1e-3 relative; and the ratio to Stokes' law, which the paper reaches to
    1.5 % after a calibration of tau that it does not print, stays within the
    band this reading of the momentum exchange gives (0.9 .. 1.25)."""
    import json
    import os

    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "table2_oracle_settling.json")) as fh:
        ref = json.load(fh)
    assert ref["steps"] == 20000 and ref["sample_every"] == 1000 and ref["interp"] == "lagrange"
    speeds = []
    for r, o in zip(S.TABLE2, ref["rows"]):
        assert abs(r["tau"] - o["tau"]) < 1e-12
        res = S.run(r, steps=ref["steps"], chunk=ref["sample_every"])
        vs = S.stokes(r["d"])
        e = abs(res["settling"] - o["settling"]) / abs(o["settling"])
        _flush(f"h/d={r['h_over_d']:.3f}: {res['settling']:.6e} m/s, oracle {o['settling']:.6e} (rel {e:.1e}), "
               f"Stokes {vs:.3e}, ratio {res['settling'] / vs:.3f}, drift {res['drift']:.1e}")
        assert e <= 1e-3
        assert 0.9 <= res["settling"] / vs <= 1.25
        assert res["drift"] < 0.02
        speeds.append(res["settling"])
    assert all(a > b for a, b in zip(speeds, speeds[1:]))      # faster (more negative) with size
