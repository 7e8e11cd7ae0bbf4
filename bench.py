"""Benchmark of the coupled LBM-PIBM-DEM step on one MI355X.

Default workload: D2Q9 2048^2, tau 0.6, 500k disks (d ~ U[0.3, 0.8],
density ratio 2.5, upper 60 % of a closed cavity), FP32, linear
spring-dashpot contacts with 677 sub-steps.  A "step" is one full coupled
step: cell list, moments (3D), interpolation, DEM, spreading,
collision+streaming.
Inputs are seeded synthetic (no dataset); the timed region starts with all
state resident in HBM.

Prints ONE JSON line.  Besides the contract fields it carries
  roofline      - the dominant kernel against MI355X HBM peak (8 TB/s), from
                  HIP events recorded on the library's stream around every
                  phase of ten evenly spaced timed steps (algorithmic bytes / time)
  cpu_baseline  - the FP64 oracle on the host cores, on a bounded sample
  extra         - the same measurement for the D3Q19 256^3 / 2M-sphere case
                  in FP32 and with FP16 deviation storage, the FP16-vs-FP32
                  field errors, the D3Q15/Lagrange and Hertz-Mindlin variants
                  of that case, the hybrid obstacle case, and the
                  adjoint/forward cost ratio on the D2Q9 512^2 /
                  10k-particle differentiation workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_PROBE_BYTES = 1 << 30
PROFILE_SAMPLES = 10     # timed steps that record the phase events (evenly spaced)

# HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE, then
# WRITE_SIZE, each in its own run), scaled by the same counters over a plain
# device copy of known size (--copy-probe).  Keyed by (kernel, workload); the
# entry only applies while the kernel's source file hashes to `source_sha`.
MEASURED_TRAFFIC = {
    ("collide", "c1"): {"fetch_bytes": 90158.6 * 1024 * 1.9999, "write_bytes": 150214.1 * 1024,
                       "source_sha": "4ef8dfd1a49054f3"},
    ("spread", "c1"): {"fetch_bytes": 47517.5 * 1024 * 1.9999, "write_bytes": 32768.0 * 1024,
                      "source_sha": "7b3ffaebd410b3ee"},
    ("interp", "c1"): {"fetch_bytes": 98291.9 * 1024 * 1.9999, "write_bytes": 27474.0 * 1024,
                      "source_sha": "7b3ffaebd410b3ee"},
    ("collide", "c2"): {"fetch_bytes": 720974.5 * 1024 * 1.9999, "write_bytes": 1253280.8 * 1024,
                       "source_sha": "4ef8dfd1a49054f3"},
    ("moments", "c2"): {"fetch_bytes": 336723.5 * 1024 * 1.9999, "write_bytes": 133120.0 * 1024,
                       "source_sha": "4ef8dfd1a49054f3"},
    ("spread", "c2"): {"fetch_bytes": 704123.3 * 1024 * 1.9999, "write_bytes": 196608.0 * 1024,
                      "source_sha": "7b3ffaebd410b3ee"},
    ("interp", "c2"): {"fetch_bytes": 397785.0 * 1024 * 1.9999, "write_bytes": 180022.1 * 1024,
                      "source_sha": "7b3ffaebd410b3ee"},
}
METRIC = "coupled LBM-PIBM-DEM MLUPS + particle-updates/s; FP16 vs FP32; adjoint/fwd ratio"


def algorithmic_bytes(phase: str, w, np_: int) -> float:
    """Algorithmic bytes one launch of a phase moves (per step)."""
    Q = int(w.lattice)
    D = w.dim
    es = 2 if w.storage == "fp16" else 4
    N = w.nodes
    coupled = np_ > 0 and w.two_way
    if phase == "collide":
        return N * (2 * Q * es + (4 * D if coupled else 0))
    if phase == "moments":
        return N * (Q * es + 16)
    if phase == "spread":
        # force field write + per-particle weights, base and coefficients read
        return N * 4 * D + np_ * (8 + 16 * D + 4 * D)
    if phase == "interp":
        # particle position read, moments gathered once per node (dense), outputs
        return np_ * (8 * D + 4 + 4 * D + 8 + 16 * D) + N * 16
    if phase == "cell_list":
        return np_ * (2 * (12 * D + 12) + 16)
    if phase == "dem":
        return np_ * (2 * 12 * D + 8 + 4 * (1 + D) + 8 * D)
    return 0.0


def source_sha(kernel: str) -> str:
    import hashlib

    f = "lattice.hip" if kernel in ("collide", "moments") else "particles.hip"
    with open(os.path.join(ROOT, "paper_1407_6704_amd", "csrc", f), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None or rec["source_sha"] != source_sha(kernel):
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def copy_probe():
    """A plain device copy of COPY_PROBE_BYTES, for calibrating the HBM byte
    counters: FETCH_SIZE and WRITE_SIZE of this launch should read the size."""
    import torch

    n = COPY_PROBE_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    # a plain elementwise kernel over the same bytes (read once, write once):
    # what a simple streaming kernel reaches on this part
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(2):
        torch.mul(src, 2.0, out=dst)
    ev[0].record()
    for _ in range(5):
        torch.mul(src, 2.0, out=dst)
    ev[1].record()
    torch.cuda.synchronize()
    us = ev[0].elapsed_time(ev[1]) * 1e3 / 5
    print(json.dumps({"copy_probe_bytes_read": COPY_PROBE_BYTES, "copy_probe_bytes_written": COPY_PROBE_BYTES,
                      "launches": 3, "elementwise_us": us,
                      "elementwise_TBps": 2 * COPY_PROBE_BYTES / us / 1e6}), flush=True)


def run_gpu(w, steps: int, warmup: int, label: str, keep_fields: bool = False):
    import torch

    from paper_1407_6704_amd import pibm, workloads as W

    t0 = time.time()
    if w.obstacles:
        X, U, d, rp, body, area = W.make_hybrid(w)
    else:
        X, U, d, rp = W.make_particles(w)
    print(f"[bench] {label}: placed {X.shape[1]} particles in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    cfg = pibm.config_from_workload(w)
    sim = pibm.Sim(cfg, X.shape[1])
    sim.set_particles(X, U, d, rp)
    if w.obstacles:
        sim.set_bodies(body, area)
    sim.step(warmup)
    sim.synchronize()
    # phase events on PROFILE_SAMPLES evenly spaced timed steps: each recorded
    # step carries 7 event records, which add a few microseconds each
    sim.set_profiling(True, every=max(1, steps // PROFILE_SAMPLES))
    sim.phase_times()
    stream = sim.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    phases, nsteps = sim.phase_times()
    status = "ok"
    try:
        sim.synchronize()
    except pibm.PibmError as e:
        status = e.name
    diag = sim.diagnostics()
    sim.set_profiling(False)
    bodies = None
    if w.obstacles:
        nb = int(body.max()) + 1
        bf = sim.read_bodies(nb)
        bodies = {"points": int((body >= 0).sum()),
                  "f_hydro": bf["f_hydro"].T.tolist(), "f_contact": bf["f_contact"].T.tolist()}
    fields = sim.read_fields() if keep_fields else None
    np_ = X.shape[1]
    res = {
        "ms_per_step": ms / steps,
        "mlups": w.nodes * steps / (ms * 1e-3) / 1e6,
        "particle_updates_per_s": np_ * steps / (ms * 1e-3),
        "phases_ms_per_step": {k: v / max(nsteps, 1) for k, v in phases.items()},
        "active_particles": diag["active"],
        "status": status,
    }
    if bodies is not None:
        res["bodies"] = bodies
    # dominant kernel: the single-launch lattice phase with the most time (the
    # moments pass is left out: it skips the node rows no particle reaches, so
    # its bytes depend on where the particles are)
    single = {k: v for k, v in res["phases_ms_per_step"].items() if k in ("collide", "spread")}
    dom = max(single, key=single.get)
    b = algorithmic_bytes(dom, w, np_)
    t = single[dom] * 1e-3
    ach = b / t / 1e9
    res["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(dom, w.name),
                       "bytes_per_launch": b, "avg_launch_ms": single[dom]}
    if keep_fields:
        res["_fields"] = fields
    del sim
    torch.cuda.empty_cache()
    return res, (X, U, d, rp)


def run_adjoint(w, K: int = 100):
    """Adjoint/forward cost on the differentiation workload: plain FP32
    stepping of w.steps steps against the backward pass (segment re-runs plus
    the reverse steps) of a checkpointed rollout of the same steps, for
    J = mean particle height."""
    import numpy as np
    import torch

    from paper_1407_6704_amd import pibm, workloads as W

    X, U, d, rp = W.make_particles(w)
    cfg = pibm.config_from_workload(w)
    steps = w.steps

    def timed(fn, stream):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        out = fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1), out

    sim = pibm.Sim(cfg, X.shape[1])
    sim.set_particles(X, U, d, rp)
    sim.step(10)
    sim.synchronize()
    t_fwd, _ = timed(lambda: sim.step(steps), sim.stream)
    sim.synchronize()
    del sim
    rs = pibm.Sim(cfg, X.shape[1])
    rs.set_particles(X, U, d, rp)
    t_ck, _ = timed(lambda: rs.forward_ckpt(steps, K), rs.stream)
    dJdx = np.zeros_like(X)
    dJdx[w.dim - 1] = 1.0 / X.shape[1]
    t_bwd, r = timed(lambda: rs.backward(dJ_dx=dJdx), rs.stream)
    out = {"workload": f"{w.name}: D2Q9 {w.n[0]}x{w.n[1]}, {X.shape[1]} particles, soft contact, n_sub 1",
           "steps": steps, "checkpoint_every": K, "forward_ms": t_fwd, "forward_ckpt_ms": t_ck,
           "backward_ms": t_bwd, "ratio": t_bwd / t_fwd,
           "rollout_buffer_MB": rs.rollout_buf.numel() / 1e6,
           "dJ_dtau": r["dtau"], "dJ_dgravity_y": r["dgravity"][w.dim - 1],
           "dJ_dv0_norm": float(np.linalg.norm(r["dv0"]))}
    del rs
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, particles, budget_s=10.0, max_steps=4):
    """The FP64 oracle (single thread, as it stands) on full coupled steps of
    the same workload: steps are taken until about budget_s seconds of CPU
    work (at least one, at most max_steps)."""
    from oracle import oracle as orc

    X, U, d, rp = particles
    oc = orc.make_cfg(lattice=w.lattice, n=w.n, tau=w.tau, gravity=w.gravity_vec(), contact=w.contact,
                      kn=w.kn, restitution=w.restitution, k_soft=w.k_soft, skin=w.skin, n_sub=w.n_sub,
                      two_way=w.two_way, bin_log2=w.bin_log2)
    f = orc.rest_state(oc)
    t0 = time.time()
    steps = 0
    while steps < max_steps and (steps == 0 or time.time() - t0 < budget_s):
        out = orc.step(oc, f, X, U, d, rp)
        f, X, U = out["f"], out["X"], out["U"]
        steps += 1
    dt = time.time() - t0
    return {"value": w.nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "particle_updates_per_s": X.shape[1] * steps / dt,
            "sample": f"{steps} full coupled step(s) of the same workload ({w.nodes} nodes, {X.shape[1]} particles, "
                      f"{w.n_sub} sub-steps) from rest, FP64, single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--extra-steps", type=int, default=20)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this library runs on one GPU only; multi-GPU runs are not supported "
              "(the lattice would shard into slabs with a halo exchange, which is not built).",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe()
        return

    from paper_1407_6704_amd import pibm, workloads as W

    pibm.load()
    w = W.WORKLOADS[args.workload]
    res, parts = run_gpu(w, args.steps, args.warmup, w.name)
    line = {
        "metric": METRIC,
        "value": res["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.storage == "fp32" else "f16-storage/f32-compute",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: D2Q9 {w.n[0]}x{w.n[1]}" if w.dim == 2 else
                   f"{w.name}: D3Q{w.lattice} {w.n[0]}x{w.n[1]}x{w.n[2]}",
                   "particles": w.n_particles, "tau": w.tau, "n_sub": w.n_sub, "contact": w.contact,
                   "storage": w.storage, "seed": w.seed},
        "particle_updates_per_s": res["particle_updates_per_s"],
        "phases_ms_per_step": res["phases_ms_per_step"],
        "active_particles": res["active_particles"],
        "status": res["status"],
        "roofline": res["roofline"],
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, parts)
    if not args.no_extra:
        import numpy as np

        extra = {}
        for name in ("c2", "c3"):
            r, _ = run_gpu(W.WORKLOADS[name], args.extra_steps, 2, name, keep_fields=True)
            extra[name] = r
        extra["fp16_speedup"] = extra["c2"]["ms_per_step"] / extra["c3"]["ms_per_step"]
        # FP16 storage against FP32 from the same initial state, same steps
        (r32, u32), (r16, u16) = extra["c2"].pop("_fields"), extra["c3"].pop("_fields")
        # the paper's lattice and gather on the c2 particles
        r, _ = run_gpu(W.WORKLOADS["c2_d3q15"], args.extra_steps, 2, "c2_d3q15")
        extra["c2_d3q15_lagrange"] = r
        # the paper's contact law on the c2 particles
        r, _ = run_gpu(W.WORKLOADS["c2_hm"], args.extra_steps, 2, "c2_hm")
        extra["c2_hertz_mindlin"] = r
        # the hybrid IBM-PIBM case: particles above fixed obstacle bodies
        r, _ = run_gpu(W.WORKLOADS["hybrid"], args.extra_steps, 2, "hybrid")
        extra["hybrid_obstacles"] = r
        extra["c4_adjoint"] = run_adjoint(W.WORKLOADS["c4"])
        extra["fp16_vs_fp32"] = {
            "steps": args.extra_steps + 2,
            "eps_u": float(np.linalg.norm(u16.astype(np.float64) - u32) / np.linalg.norm(u32.astype(np.float64))),
            "eps_rho": float(np.abs(r16.astype(np.float64) - r32).max()),
        }
        line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
