"""Single-particle settling in a closed cuboid cavity (Sec. 3.1, Table 2).

The cavity is 1 mm x 1 mm x 5 mm with a lattice spacing of 0.1 mm, so
10 x 10 x 50 nodes of the D3Q15 lattice (Sec. 2.1), walls on every face.
One particle starts at rest at (0.5, 0.5, 4.9) mm and falls under gravity;
the fluid and particle properties are those of Table 1 (density ratio
1.01, water-like viscosity 1e-6 m^2/s, g = 9.8 m/s^2).  Each of the four
diameters of Table 2 comes with its own relaxation time; the physical time
step follows from tau through the lattice viscosity (tau - 1/2)/3:

    dt = (tau - 1/2) h^2 / (3 nu)            h = 1e-4 m, nu = 1e-6 m^2/s

and gravity in lattice units is g dt^2 / h.  Velocities convert back with
h / dt.  Stokes' law, Eq. lbm14, gives the reference settling speed.

    python -m paper_1407_6704_amd.settling [--steps N] [--interp lagrange|delta]

prints one line per diameter and, with --json PATH, writes the trajectories.
Everything runs on the GPU through the C ABI (pibm.Sim).
"""
import argparse
import json
import time

import numpy as np

# Table 1 properties and the lattice spacing of Sec. 3
RHO_F = 1000.0          # kg/m^3
RHO_P = 1010.0          # kg/m^3
MU = 1.0e-3             # Pa s
G = 9.8                 # m/s^2
H = 1.0e-4              # m, lattice spacing
NU = MU / RHO_F

# Table 2: diameter (m), tau, printed Stokes speed and printed numerical result (m/s)
TABLE2 = (
    dict(h_over_d=4.0, d=0.25e-4, tau=0.65, stokes=-3.40e-6, paper=-3.41e-6),
    dict(h_over_d=2.0, d=0.50e-4, tau=0.72, stokes=-1.36e-5, paper=-1.37e-5),
    dict(h_over_d=4.0 / 3.0, d=0.75e-4, tau=0.79, stokes=-3.06e-5, paper=-3.07e-5),
    dict(h_over_d=1.0, d=1.00e-4, tau=0.85, stokes=-5.44e-5, paper=-5.52e-5),
)

CAVITY = (10, 10, 50)            # nodes: 1 mm x 1 mm x 5 mm
START = (5.0, 5.0, 49.0)         # lattice units: (0.5, 0.5, 4.9) mm


def time_step(tau):
    """Physical time step (s) of one lattice step for relaxation time tau."""
    return (tau - 0.5) * H * H / (3.0 * NU)


def stokes(d):
    """Stokes settling velocity (m/s, downward negative), Eq. lbm14."""
    return -(RHO_P - RHO_F) * d * d * G / (18.0 * MU)


def case(row, lattice=15, interp="lagrange", n_sub=32, storage="fp32"):
    """Configuration and initial particle arrays of one Table 2 row."""
    from . import pibm

    dt = time_step(row["tau"])
    g_lu = G * dt * dt / H
    cfg = pibm.make_config(lattice=lattice, n=CAVITY, storage=storage, tau=row["tau"], rho0=1.0,
                           gravity=(0.0, 0.0, -g_lu), contact="lsd", kn=1e3, restitution=0.9,
                           n_sub=n_sub, skin=0.05, interp=interp)
    X = np.array(START, np.float64).reshape(3, 1)
    U = np.zeros((3, 1))
    d = np.array([row["d"] / H])
    rp = np.array([RHO_P / RHO_F])
    return cfg, X, U, d, rp, dt


def run(row, steps=20000, chunk=250, lattice=15, interp="lagrange", n_sub=32, device="cuda:0"):
    """Fall of one particle for `steps` lattice steps, sampled every `chunk`
    steps.  Returns the sampled times (s), heights (m) and vertical speeds
    (m/s) and the settling speed: the mean speed over the last tenth of the
    run, with the relative change against the tenth before it."""
    from . import pibm

    cfg, X, U, d, rp, dt = case(row, lattice, interp, n_sub)
    sim = pibm.Sim(cfg, 1, device=device)
    sim.set_particles(X, U, d, rp)
    t, z, w = [0.0], [X[2, 0] * H], [0.0]
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        done += k
        p = sim.read_particles()
        t.append(done * dt)
        z.append(float(p["x"][2, 0]) * H)
        w.append(float(p["v"][2, 0]) * H / dt)
    w = np.array(w)
    m = max(1, len(w) // 10)
    last, prev = w[-m:].mean(), w[-2 * m:-m].mean()
    return dict(t=t, z=z, w=w.tolist(), settling=float(last),
                drift=float(abs(last - prev) / max(abs(last), 1e-300)), dt=dt, steps=steps)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--interp", default="lagrange", choices=("lagrange", "delta"))
    ap.add_argument("--lattice", type=int, default=15, choices=(15, 19))
    ap.add_argument("--n-sub", type=int, default=32)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    out = []
    for row in TABLE2:
        t0 = time.perf_counter()
        r = run(row, a.steps, a.chunk, a.lattice, a.interp, a.n_sub)
        el = time.perf_counter() - t0
        vs = stokes(row["d"])
        print(f"h/d={row['h_over_d']:.3f} tau={row['tau']:.2f} dt={r['dt']:.2e}s: settling {r['settling']:.3e} m/s "
              f"(drift {r['drift']:.1e}) | Stokes {vs:.3e} ({r['settling'] / vs:.3f}x) | paper {row['paper']:.2e} "
              f"| {a.steps} steps in {el:.1f} s", flush=True)
        out.append(dict(row=row, stokes=vs, **r))
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(dict(lattice=a.lattice, interp=a.interp, n_sub=a.n_sub, cases=out), fh)
    return out


if __name__ == "__main__":
    main()
