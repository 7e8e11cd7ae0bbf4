"""Write tests/golden/table2_oracle_settling.json: the FP64 oracle's run of
the single-particle settling study (Sec. 3.1, Table 2 of the paper).

For each row of Table 2 (diameter and relaxation time, from
tests/golden/table2_settling.json) the oracle steps a 10 x 10 x 50 D3Q15
cavity with walls on every face (1 x 1 x 5 mm at h = 0.1 mm) and one
particle released at rest at (0.5, 0.5, 4.9) mm, with the Lagrange gather,
32 DEM sub-steps, for 20,000 steps.  Physical units follow Table 1: the time
step is dt = (tau - 1/2) h^2 / (3 nu) and gravity in lattice units is
g dt^2 / h.  The vertical particle speed is sampled every 1000 steps
(converted to m/s with h / dt); the settling speed is the mean of the last
tenth of the samples (with the start sample included, 21 samples: the last
two).  Only the oracle runs here.

    python tests/golden/make_table2_reference.py        (a few minutes)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc  # noqa: E402

STEPS, CHUNK, N_SUB = 20000, 1000, 32
CAVITY = (10, 10, 50)
START = (5.0, 5.0, 49.0)


def run_row(row, props):
    h, nu = props["h"], props["mu"] / props["rho_f"]
    dt = (row["tau"] - 0.5) * h * h / (3.0 * nu)
    g_lu = props["g"] * dt * dt / h
    oc = orc.make_cfg(lattice=15, n=CAVITY, tau=row["tau"], rho0=1.0, gravity=(0.0, 0.0, -g_lu), contact="lsd",
                      kn=1e3, restitution=0.9, skin=0.05, n_sub=N_SUB, two_way=1, bin_log2=0, interp="lagrange")
    f = orc.rest_state(oc)
    X = np.array(START, np.float64).reshape(3, 1)
    U = np.zeros((3, 1))
    d = np.array([row["d"] / h])
    rp = np.array([props["rho_p"] / props["rho_f"]])
    w = [0.0]
    for k in range(1, STEPS + 1):
        out = orc.step(oc, f, X, U, d, rp)
        f, X, U = out["f"], out["X"], out["U"]
        if k % CHUNK == 0:
            w.append(float(U[2, 0]) * h / dt)
    w = np.array(w)
    m = max(1, len(w) // 10)
    return dict(h_over_d=row["h_over_d"], tau=row["tau"], dt=dt, g_lattice=g_lu, samples=w.tolist(),
                settling=float(w[-m:].mean()), height_lattice=float(X[2, 0]))


def main():
    with open(os.path.join(HERE, "table2_settling.json")) as fh:
        spec = json.load(fh)
    rows = []
    for row in spec["rows"]:
        r = run_row(row, spec["properties"])
        print(f"h/d={r['h_over_d']:.3f}: oracle settling {r['settling']:.6e} m/s (Stokes {row['stokes']:.2e})",
              flush=True)
        rows.append(r)
    out = dict(source="FP64 oracle (oracle/pibm_oracle.c) via tests/golden/make_table2_reference.py; inputs from "
                      "table2_settling.json (Sec. 3.1, Tables 1-2 of the paper)",
               lattice="D3Q15", interp="lagrange", n_sub=N_SUB, steps=STEPS, sample_every=CHUNK, rows=rows)
    with open(os.path.join(HERE, "table2_oracle_settling.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
