"""Benchmark of the coupled LBM-PIBM-DEM step on one MI355X.

Default workload (the largest configuration that fits one GPU): D3Q19
256^3, tau 0.6, walls on every face, 2M spheres (diameters lognormal with
mean 0.5 and SD 0.2, truncated to [0.2, 1], density ratio 2.0, upper half of
the cavity), FP32, linear spring-dashpot contacts with 3109 sub-steps.  A
"step" is one full coupled step: cell list, moments, interpolation, DEM,
spreading, collision+streaming.  Inputs are seeded synthetic (no dataset);
the timed region starts with all state resident in HBM.

Prints ONE JSON line.  Besides the contract fields it carries
  roofline      - the dominant kernel (collision+streaming) against MI355X HBM
                  peak (8 TB/s), from HIP events recorded on the library's
                  stream around every phase of ten evenly spaced timed steps
                  (algorithmic bytes / time)
  cpu_baseline  - the FP64 oracle on the host cores, on a bounded sample of
                  the same workload (its 64^3 crop), one thread and all
  extra         - the D2Q9 2048^2 / 500k-disk case, the same 256^3 case with
                  FP16 deviation storage and the FP16-vs-FP32 field errors,
                  both cases timed again after contacts have formed (late
                  phase), the D3Q15/Lagrange and Hertz-Mindlin variants, the
                  hybrid obstacle case, and the adjoint/forward cost ratio on
                  the D2Q9 512^2 / 10k-particle differentiation workload
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
# device copy of known size (--copy-probe).  Keyed by (kernel, workload); an
# entry applies only while the kernel's own source (its __global__ function
# and the shared device header) hashes to `kernel_sha`: a changed kernel
# reports null until it is measured again.
MEASURED_TRAFFIC = {
    ("collide", "c1"): {"fetch_bytes": 184657106, "write_bytes": 153742632, "kernel_sha": "74c47c78842cd7f4"},
    ("collide", "c3"): {"fetch_bytes": 838978130, "write_bytes": 645541636, "kernel_sha": "74c47c78842cd7f4"},
    ("interp", "c1"): {"fetch_bytes": 147793950, "write_bytes": 35927872, "kernel_sha": "13550b2c69f29678"},
    ("interp", "c2"): {"fetch_bytes": 268623185, "write_bytes": 180321752, "kernel_sha": "13550b2c69f29678"},
    ("interp", "c3"): {"fetch_bytes": 268623185, "write_bytes": 180662947, "kernel_sha": "13550b2c69f29678"},
    ("moments", "c2"): {"fetch_bytes": 884715750, "write_bytes": 180287632, "kernel_sha": "3729ded843aba06f"},
    ("moments", "c3"): {"fetch_bytes": 365832693, "write_bytes": 136273430, "kernel_sha": "3729ded843aba06f"},
    ("spread", "c1"): {"fetch_bytes": 44522500, "write_bytes": 33539504, "kernel_sha": "f927fd0435b43768"},
    ("spread", "c3"): {"fetch_bytes": 212372739, "write_bytes": 201271147, "kernel_sha": "f927fd0435b43768"},
    ("spread_collide", "c2"): {"fetch_bytes": 1488861922, "write_bytes": 1296542399, "kernel_sha": "a6643ec0a5e65b86"},
}
# the source of each measured kernel: its __global__ function and the device
# routines of its own file that carry its arithmetic (pibm_internal.h, which
# holds the per-node collision, is hashed with every kernel)
KERNEL_SOURCES = {"collide": [("lattice.hip", "k_collide")], "moments": [("lattice.hip", "k_moments")],
                  "spread": [("particles.hip", "spread_tile"), ("particles.hip", "k_spread_csr")],
                  "spread_collide": [("particles.hip", "spread_tile"), ("particles.hip", "k_spread_collide")],
                  "interp": [("particles.hip", "k_interp_tile")]}
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
    rec = 4 * (16 if D == 3 else 12)       # a particle's spreading record: weights, x base, coefficients
    if phase == "spread":
        # force field write + each particle's record read once
        return N * 4 * D + np_ * rec
    if phase == "spread_collide":
        # 3D spreading fused into the collision: populations read and
        # written, each particle's record read once, no force field
        return N * 2 * Q * es + np_ * rec
    if phase == "interp":
        # moments read once per node; positions read; interpolated moments,
        # record and stencil bases written
        return N * 16 + np_ * (8 * D + 4 + 4 * D + rec + 8)
    if phase == "cell_list":
        return np_ * (2 * (12 * D + 12) + 16)
    if phase == "dem":
        return np_ * (2 * 12 * D + 8 + 4 * (1 + D) + 8 * D)
    return 0.0


def fused_spread(w, np_: int) -> bool:
    """3D steps with bins of one dual cell and FP32 storage spread into the
    collision."""
    return w.dim == 3 and w.bin_log2 == 0 and np_ > 0 and bool(w.two_way) and w.storage == "fp32"


def kernel_text(src: str, name: str) -> str:
    """The source text of kernel `name` in csrc/`src`: from the template line
    before its __global__ declaration to the closing brace in column 0."""
    with open(os.path.join(ROOT, "paper_1407_6704_amd", "csrc", src)) as fh:
        lines = fh.read().split("\n")
    start = next(i for i, ln in enumerate(lines)
                 if ("__global__" in ln or "__device__" in ln) and f" {name}(" in ln)
    if start > 0 and lines[start - 1].startswith("template"):
        start -= 1
    end = next(i for i in range(start + 1, len(lines)) if lines[i] == "}")
    return "\n".join(lines[start:end + 1])


def source_sha(kernel: str) -> str:
    """Hash of a kernel's own source and of the device header it includes."""
    import hashlib

    h = hashlib.sha256()
    for src, name in KERNEL_SOURCES[kernel]:
        h.update(kernel_text(src, name).encode())
    with open(os.path.join(ROOT, "paper_1407_6704_amd", "csrc", "pibm_internal.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None or rec["kernel_sha"] != source_sha(kernel):
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
    """Time `steps` coupled steps after `warmup` untimed ones (from rest)."""
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
    t_w = time.time()
    done = 0
    while done < warmup:                       # in chunks, printing progress on long warm-ups
        k = min(500, warmup - done)
        sim.step(k)
        torch.cuda.synchronize()
        done += k
        if warmup > 500:
            print(f"[bench] {label}: {done} of {warmup} untimed steps ({time.time() - t_w:.1f} s)",
                  file=sys.stderr, flush=True)
    # no phase events in the timed steps
    stream = sim.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    # the phase breakdown comes from the next `steps` steps, with events on
    # PROFILE_SAMPLES evenly spaced ones (each recorded step carries 7 event
    # records, which add a few microseconds each)
    sim.set_profiling(True, every=max(1, steps // PROFILE_SAMPLES))
    sim.phase_times()
    sim.step(steps)
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
    if fused_spread(w, np_):
        # the collision phase is the fused spreading and collision kernel
        single = {"spread_collide": single["collide"]}
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
    stepping of w.steps steps against the backward pass of a recorded rollout
    of the same steps, for J = mean particle height.  The forward pass tapes
    its last segment, so the backward pass re-runs every segment but the
    last before reversing it.  Two layouts: the whole rollout as one taped
    segment when it fits in a quarter of the free device memory (nothing is
    run twice), and checkpoints every K steps (one segment's tape)."""
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
    full_bytes = sim.lib.pibm_rollout_bytes(sim.ctx, int(steps), int(steps))
    del sim
    torch.cuda.empty_cache()
    dJdx = np.zeros_like(X)
    dJdx[w.dim - 1] = 1.0 / X.shape[1]

    def rollout(k):
        rs = pibm.Sim(cfg, X.shape[1])
        rs.set_particles(X, U, d, rp)
        t_ck, _ = timed(lambda: rs.forward_ckpt(steps, k), rs.stream)
        t_bwd, r = timed(lambda: rs.backward(dJ_dx=dJdx), rs.stream)
        res = {"checkpoint_every": k, "forward_ckpt_ms": t_ck, "backward_ms": t_bwd, "ratio": t_bwd / t_fwd,
               "rollout_buffer_MB": rs.rollout_buf.numel() / 1e6, "dJ_dtau": r["dtau"],
               "dJ_dgravity_y": r["dgravity"][w.dim - 1], "dJ_dv0_norm": float(np.linalg.norm(r["dv0"]))}
        del rs
        torch.cuda.empty_cache()
        return res

    ck = rollout(K)
    out = {"workload": f"{w.name}: D2Q9 {w.n[0]}x{w.n[1]}, {X.shape[1]} particles, soft contact, n_sub 1",
           "steps": steps, "forward_ms": t_fwd}
    free, _ = torch.cuda.mem_get_info()
    if 0 < full_bytes <= free // 4:
        out.update(rollout(steps))
        out["checkpointed"] = ck
    else:
        out.update(ck)
    return out


def host_cpu():
    """CPU model, physical and logical cores of this host, and the cores this
    process may run on."""
    model, phys = "unknown", set()
    try:
        cur = {}
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ":" not in ln:
                    if cur:
                        phys.add((cur.get("physical id"), cur.get("core id")))
                    cur = {}
                    continue
                k, v = (t.strip() for t in ln.split(":", 1))
                cur[k] = v
                if k == "model name":
                    model = v
        if cur:
            phys.add((cur.get("physical id"), cur.get("core id")))
    except OSError:
        pass
    return {"cpu_model": model, "physical_cores": len(phys) or None, "logical_cores": os.cpu_count(),
            "usable_cores": len(os.sched_getaffinity(0))}


def cpu_baseline(w, budget_s=8.0, max_steps=4):
    """The FP64 oracle as it stands, on host cores, on a bounded sample of the
    workload: its 64^3 crop (the same tau, walls, diameter distribution,
    density ratio, particle number density and sub-steps; 31,250 spheres),
    full coupled steps from rest until about budget_s seconds per run (at
    least one, at most max_steps).  Run once on one thread and once on all
    the threads the oracle's node loops get (OpenMP; particle, pair and
    spreading loops are serial in both).  value/cores: the all-thread run."""
    from oracle import oracle as orc
    from paper_1407_6704_amd import workloads as W

    s = w.replace(name=w.name + "_crop64", n=(64, 64, 64) if w.dim == 3 else (256, 256, 1),
                  n_particles=max(1, round(w.n_particles * (64 ** 3 if w.dim == 3 else 256 ** 2) / w.nodes)),
                  storage="fp32", seed=w.seed + 100)
    X0, U0, d, rp = W.make_particles(s)
    oc = orc.make_cfg(lattice=s.lattice, n=s.n, tau=s.tau, gravity=s.gravity_vec(), contact=s.contact,
                      kn=s.kn, restitution=s.restitution, k_soft=s.k_soft, skin=s.skin, n_sub=s.n_sub,
                      two_way=s.two_way, bin_log2=s.bin_log2, interp=s.interp)
    runs = {}
    all_threads = orc.threads()
    for label, th in (("single_thread", 1), ("all_threads", all_threads)):
        orc.set_threads(th)
        f, X, U = orc.rest_state(oc), X0.copy(), U0.copy()
        t0 = time.time()
        steps = 0
        while steps < max_steps and (steps == 0 or time.time() - t0 < budget_s):
            out = orc.step(oc, f, X, U, d, rp)
            f, X, U = out["f"], out["X"], out["U"]
            steps += 1
        dt = time.time() - t0
        runs[label] = {"threads": th, "steps": steps, "seconds": dt, "mlups": s.nodes * steps / dt / 1e6,
                       "particle_updates_per_s": X.shape[1] * steps / dt}
        print(f"[bench] cpu_baseline {label}: {steps} steps in {dt:.1f} s", file=sys.stderr, flush=True)
    orc.set_threads(0)
    best = runs["all_threads"]
    return {"value": best["mlups"], "unit": "MLUPS", "cores": best["threads"], "kind": "oracle",
            "particle_updates_per_s": best["particle_updates_per_s"], **host_cpu(),
            "single_thread": runs["single_thread"], "all_threads": runs["all_threads"],
            "sample": f"{s.name}: the workload's {'x'.join(map(str, s.n))} crop ({s.nodes} nodes, {X0.shape[1]} "
                      f"particles at the same number density, same tau, diameters, density ratio and "
                      f"{s.n_sub} sub-steps), full FP64 coupled steps from rest; MLUPS = crop nodes x steps / "
                      f"time; node loops on {best['threads']} threads (OpenMP), particle loops serial"}


def workload_name(w) -> str:
    return (f"{w.name}: D2Q9 {w.n[0]}x{w.n[1]}" if w.dim == 2 else
            f"{w.name}: D3Q{w.lattice} {w.n[0]}x{w.n[1]}x{w.n[2]}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--extra-steps", type=int, default=20)
    ap.add_argument("--late-c1", type=int, default=500, help="untimed steps before the late-phase c1 window")
    ap.add_argument("--late-c2", type=int, default=1900, help="untimed steps before the late-phase c2 window")
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
    fp16_twin = {"c2": "c3"}.get(w.name)
    res, parts = run_gpu(w, args.steps, args.warmup, w.name, keep_fields=fp16_twin is not None)
    fields32 = res.pop("_fields", None)
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
        "config": {"workload": workload_name(w), "particles": w.n_particles, "tau": w.tau, "n_sub": w.n_sub,
                   "contact": w.contact, "storage": w.storage, "seed": w.seed},
        "particle_updates_per_s": res["particle_updates_per_s"],
        "phases_ms_per_step": res["phases_ms_per_step"],
        "active_particles": res["active_particles"],
        "status": res["status"],
        "roofline": res["roofline"],
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w)
    if not args.no_extra:
        import numpy as np

        extra = {}
        if fp16_twin:
            # FP16 deviation storage from the same initial state over the same steps
            r16, _ = run_gpu(W.WORKLOADS[fp16_twin], args.steps, args.warmup, fp16_twin, keep_fields=True)
            (rho16, u16), (rho32, u32) = r16.pop("_fields"), fields32
            extra[fp16_twin] = r16
            extra["fp16_speedup"] = res["ms_per_step"] / r16["ms_per_step"]
            extra["fp16_vs_fp32"] = {
                "steps": args.steps + args.warmup,
                "eps_u": float(np.linalg.norm(u16.astype(np.float64) - u32) / np.linalg.norm(u32.astype(np.float64))),
                "eps_rho": float(np.abs(rho16.astype(np.float64) - rho32).max()),
            }
        if w.name != "c1":
            r, _ = run_gpu(W.C1, args.extra_steps, 5, "c1")
            r["workload"] = workload_name(W.C1)
            extra["c1"] = r
        # the step once contacts have formed and lasted: c1 after 500 steps
        # (lasting contacts from about step 300), c2 up to step 2000 (its
        # stated length), each timed over 100 more steps
        late = {}
        for name, before in (("c1", args.late_c1), ("c2", args.late_c2)):
            r, _ = run_gpu(W.WORKLOADS[name], 100, before, f"{name}_late")
            r["workload"] = workload_name(W.WORKLOADS[name])
            r["timed_steps"] = f"{before + 1}..{before + 100}"
            late[name] = r
        extra["late_phase"] = late
        # the paper's lattice and gather on the c2 particles
        r, _ = run_gpu(W.WORKLOADS["c2_d3q15"], args.extra_steps, 2, "c2_d3q15")
        extra["c2_d3q15_lagrange"] = r
        # the paper's contact law on the c2 particles
        r, _ = run_gpu(W.WORKLOADS["c2_hm"], args.extra_steps, 2, "c2_hm")
        extra["c2_hertz_mindlin"] = r
        r, _ = run_gpu(W.WORKLOADS["c2_hms"], args.extra_steps, 2, "c2_hms")
        extra["c2_hertz_mindlin_microslip"] = r
        # the hybrid IBM-PIBM case: particles above fixed obstacle bodies
        r, _ = run_gpu(W.WORKLOADS["hybrid"], args.extra_steps, 2, "hybrid")
        extra["hybrid_obstacles"] = r
        extra["c4_adjoint"] = run_adjoint(W.WORKLOADS["c4"])
        line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
