"""Python binding of libpibm (C ABI in include/pibm.h).

Argument marshalling only: every step of the coupled LBM-PIBM-DEM path runs
in the library's HIP kernels.  PyTorch provides the device workspace (one
uint8 tensor) and the HIP stream.  There is no fallback: if libpibm.so is not
built, importing this module's loader raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpibm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pibm.h")

ABI_VERSION = 6
D2Q9, D3Q15, D3Q19 = 9, 15, 19
STORE_FP32, STORE_FP16 = 0, 1
STAGE = {"collide_t": 1, "particles_t": 2, "interp": 3, "interp_t": 4}    # PIBM_STAGE_* in the header
CONTACT = {"none": 0, "lsd": 1, "soft": 2, "hertz": 3, "hertz_mindlin": 4, "hertz_mindlin_microslip": 5}
INTERP = {"delta": 0, "lagrange": 1}
STATUS = {0: "OK", 1: "E_ARG", 2: "E_CONFIG", 3: "E_HIP", 4: "E_STATE", 5: "E_UNSTABLE",
          6: "E_SKIN", 7: "E_CAPACITY"}


class Config(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("lattice", C.c_int32), ("storage", C.c_int32),
        ("fp16_scale_log2", C.c_int32), ("n", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
        ("tau", C.c_double), ("rho0", C.c_double), ("gravity", C.c_double * 3),
        ("fluid_force", C.c_double * 3), ("contact", C.c_int32), ("n_sub", C.c_int32),
        ("kn", C.c_double), ("restitution", C.c_double), ("k_soft", C.c_double),
        ("skin", C.c_double), ("two_way", C.c_int32), ("bin_log2", C.c_int32),
        ("max_candidates", C.c_int32), ("island_setup", C.c_int32), ("interp", C.c_int32),
        ("young", C.c_double), ("poisson", C.c_double), ("friction", C.c_double), ("bodies", C.c_int32),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("mass", C.c_double), ("momentum", C.c_double * 3), ("fluid_momentum", C.c_double * 3),
        ("max_speed", C.c_double), ("nonfinite", C.c_int64), ("active", C.c_int64),
        ("candidates", C.c_int64), ("min_height", C.c_double), ("mean_height", C.c_double),
    ]


class PibmError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {msg}")


_lib = None


def load():
    """Load libpibm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1407_6704_amd/build.py")
    # torch ships its own HIP runtime under the same soname as the system
    # one; loading torch first makes the library bind to that single copy,
    # so streams and device pointers from torch are valid in it.  Loading the
    # library first would put two different HIP/HSA runtimes in the process.
    import torch  # noqa: F401

    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    fp = C.POINTER(C.c_float)
    dp = C.POINTER(C.c_double)
    cp = C.POINTER(Config)
    sig = {
        "pibm_workspace_bytes": ([cp, C.c_int64], C.c_size_t),
        "pibm_create": ([cp, C.c_int64, vp, C.c_size_t, vp, C.POINTER(vp)], C.c_int),
        "pibm_destroy": ([vp], None),
        "pibm_last_error": ([vp], C.c_char_p),
        "pibm_set_stream": ([vp, vp], C.c_int),
        "pibm_init_equilibrium": ([vp, fp, fp], C.c_int),
        "pibm_write_populations": ([vp, fp], C.c_int),
        "pibm_read_populations": ([vp, fp], C.c_int),
        "pibm_set_particles": ([vp, dp, dp, dp, dp], C.c_int),
        "pibm_read_particles": ([vp, dp, dp, dp, dp], C.c_int),
        "pibm_set_rotation": ([vp, dp], C.c_int),
        "pibm_set_bodies": ([vp, C.POINTER(C.c_int32), dp], C.c_int),
        "pibm_read_bodies": ([vp, C.c_int32, dp, dp, dp], C.c_int),
        "pibm_read_rotation": ([vp, dp], C.c_int),
        "pibm_read_fields": ([vp, fp, fp], C.c_int),
        "pibm_read_force": ([vp, fp], C.c_int),
        "pibm_num_bins": ([vp], C.c_int64),
        "pibm_read_cell_list": ([vp, C.POINTER(C.c_uint32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
        "pibm_step": ([vp, C.c_int32], C.c_int),
        "pibm_synchronize": ([vp], C.c_int),
        "pibm_conservation": ([vp, dp, dp], C.c_int),
        "pibm_conservation_noalloc": ([vp, dp, dp], C.c_int),
        "pibm_diagnostics": ([vp, C.POINTER(Diag)], C.c_int),
        "pibm_set_profiling": ([vp, C.c_int], C.c_int),
        "pibm_phase_times": ([vp, dp, C.POINTER(C.c_int64)], C.c_int),
        "pibm_rollout_bytes": ([vp, C.c_int32, C.c_int32], C.c_size_t),
        "pibm_forward_ckpt": ([vp, C.c_int32, C.c_int32, vp, C.c_size_t], C.c_int),
        "pibm_backward": ([vp, fp, fp, fp, fp, dp, dp], C.c_int),
        "pibm_set_particles_device": ([vp, vp, vp, vp, vp, vp, C.c_double], C.c_int),
        "pibm_read_particles_device": ([vp, vp, vp, vp, vp, vp], C.c_int),
        "pibm_read_fields_device": ([vp, vp, vp], C.c_int),
        "pibm_read_force_device": ([vp, vp], C.c_int),
        "pibm_adjoint_stage": ([vp, C.c_int32, vp, vp, vp, vp, vp, vp, dp], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def header_symbols():
    """Names of the functions declared in include/pibm.h."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pibm_[a-z0-9_]+)\s*\(", txt)))


def make_config(lattice=9, n=(16, 16, 1), storage="fp32", fp16_scale_log2=14, periodic=(0, 0, 0),
                tau=0.8, rho0=1.0, gravity=(0.0, 0.0, 0.0), fluid_force=(0.0, 0.0, 0.0),
                contact="lsd", n_sub=1, kn=1e3, restitution=0.9, k_soft=1e-3, skin=0.05,
                two_way=1, bin_log2=0, max_candidates=16, island_setup=0, interp="delta", young=1e-3,
                poisson=0.33, friction=0.33, bodies=0) -> Config:
    c = Config()
    c.abi_version = ABI_VERSION
    c.lattice = int(lattice)
    c.storage = STORE_FP16 if storage in ("fp16", STORE_FP16) else STORE_FP32
    c.fp16_scale_log2 = int(fp16_scale_log2)
    for a in range(3):
        c.n[a] = int(n[a])
        c.periodic[a] = int(periodic[a])
        c.gravity[a] = float(gravity[a])
        c.fluid_force[a] = float(fluid_force[a])
    c.tau, c.rho0 = float(tau), float(rho0)
    c.contact = CONTACT[contact] if isinstance(contact, str) else int(contact)
    c.n_sub = int(n_sub)
    c.kn, c.restitution, c.k_soft, c.skin = float(kn), float(restitution), float(k_soft), float(skin)
    c.two_way, c.bin_log2, c.max_candidates = int(two_way), int(bin_log2), int(max_candidates)
    c.island_setup = int(island_setup)
    c.interp = INTERP[interp] if isinstance(interp, str) else int(interp)
    c.young, c.poisson, c.friction = float(young), float(poisson), float(friction)
    c.bodies = int(bodies)
    return c


def config_from_workload(w, **over) -> Config:
    kw = dict(lattice=w.lattice, n=w.n, storage=w.storage, fp16_scale_log2=w.fp16_scale_log2,
              tau=w.tau, gravity=w.gravity_vec(), contact=w.contact, n_sub=w.n_sub, kn=w.kn,
              restitution=w.restitution, k_soft=w.k_soft, skin=w.skin, two_way=w.two_way,
              bin_log2=w.bin_log2, interp=getattr(w, "interp", "delta"), young=w.young, poisson=w.poisson,
              friction=w.friction, bodies=int(w.obstacles))
    kw.update(over)
    return make_config(**kw)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


class Sim:
    """One coupled LBM-PIBM-DEM simulation on one GPU."""

    def __init__(self, cfg: Config, n_particles: int = 0, device="cuda:0", stream=None):
        import torch

        self.lib = load()
        self.cfg = cfg
        self.np = int(n_particles)
        self.Q = int(cfg.lattice)
        self.D = 2 if cfg.lattice == 9 else 3
        self.n = tuple(int(cfg.n[a]) for a in range(3))
        self.N = self.n[0] * self.n[1] * self.n[2]
        nbytes = self.lib.pibm_workspace_bytes(C.byref(cfg), self.np)
        if nbytes == 0:
            raise PibmError(2, "invalid configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        st = self.lib.pibm_create(C.byref(cfg), self.np, C.c_void_p(self.workspace.data_ptr()),
                                  int(nbytes), C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx))
        if st != 0:
            raise PibmError(st, "pibm_create failed")

    def _check(self, st):
        if st != 0:
            msg = self.lib.pibm_last_error(self.ctx)
            raise PibmError(st, msg.decode() if msg else "")

    def close(self):
        if self.ctx:
            self.lib.pibm_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- state -----------------------------------------------------------
    def init_equilibrium(self, rho=None, u=None):
        r = _f32(rho) if rho is not None else None
        uu = _f32(u) if u is not None else None
        self._check(self.lib.pibm_init_equilibrium(self.ctx, _fp(r), _fp(uu)))

    def write_populations(self, h):
        h = _f32(h).reshape(self.Q * self.N)
        self._check(self.lib.pibm_write_populations(self.ctx, _fp(h)))

    def read_populations(self):
        h = np.empty(self.Q * self.N, np.float32)
        self._check(self.lib.pibm_read_populations(self.ctx, _fp(h)))
        return h.reshape(self.Q, self.N)

    def set_particles(self, x, v=None, d=None, rho_p=None):
        x = _f64(x).reshape(self.D, self.np)
        v = _f64(v).reshape(self.D, self.np) if v is not None else None
        self._check(self.lib.pibm_set_particles(self.ctx, _dp(x), _dp(v), _dp(_f64(d)), _dp(_f64(rho_p))))

    # --- state in device tensors (no host round trip) ---------------------
    def _dev_f32(self, t):
        """A contiguous FP32 tensor on this simulation's device (marshalling)."""
        import torch

        return torch.as_tensor(t).to(device=self.device, dtype=torch.float32).contiguous()

    @staticmethod
    def _vp(t):
        return C.c_void_p(t.data_ptr()) if t is not None else None

    def set_particles_device(self, x_hi, d, rho_p, v=None, x_lo=None, d_max=None):
        """Particles from device tensors ((D, N) positions as x_hi + x_lo,
        velocities; (N,) diameters and densities), asynchronously on this
        simulation's stream.  d_max >= every diameter (None: taken from d,
        which waits for the device)."""
        xh = self._dev_f32(x_hi).reshape(self.D, self.np)
        xl = self._dev_f32(x_lo).reshape(self.D, self.np) if x_lo is not None else None
        vv = self._dev_f32(v).reshape(self.D, self.np) if v is not None else None
        dd = self._dev_f32(d).reshape(self.np)
        rp = self._dev_f32(rho_p).reshape(self.np)
        if d_max is None:
            d_max = float(dd.max().item()) if self.np else 1.0
        self._keep = (xh, xl, vv, dd, rp)          # alive until the stream has copied them
        self._check(self.lib.pibm_set_particles_device(self.ctx, self._vp(xh), self._vp(xl), self._vp(vv),
                                                       self._vp(dd), self._vp(rp), float(d_max)))

    def read_particles_device(self):
        """The particle state in id order as FP32 device tensors (D, N):
        x_hi, x_lo (position = x_hi + x_lo), v, f_hydro, f_contact."""
        import torch

        out = {k: torch.empty((self.D, self.np), dtype=torch.float32, device=self.device)
               for k in ("x_hi", "x_lo", "v", "f_hydro", "f_contact")}
        self._check(self.lib.pibm_read_particles_device(self.ctx, *(self._vp(out[k]) for k in
                                                                    ("x_hi", "x_lo", "v", "f_hydro", "f_contact"))))
        return out

    def read_fields_device(self):
        """Density (N,) and velocity (D, N) as FP32 device tensors."""
        import torch

        rho = torch.empty(self.N, dtype=torch.float32, device=self.device)
        u = torch.empty((self.D, self.N), dtype=torch.float32, device=self.device)
        self._check(self.lib.pibm_read_fields_device(self.ctx, self._vp(rho), self._vp(u)))
        return rho, u

    def read_force_device(self):
        """The force field of the last collision (D, N) as an FP32 device tensor."""
        import torch

        F = torch.empty((self.D, self.N), dtype=torch.float32, device=self.device)
        self._check(self.lib.pibm_read_force_device(self.ctx, self._vp(F)))
        return F

    def read_particles(self):
        out = {k: np.empty((self.D, self.np)) for k in ("x", "v", "f_hydro", "f_contact")}
        self._check(self.lib.pibm_read_particles(self.ctx, _dp(out["x"]), _dp(out["v"]),
                                                 _dp(out["f_hydro"]), _dp(out["f_contact"])))
        return out

    def set_rotation(self, w):
        """Angular velocities (3 x N in 3D, N in 2D), Hertz-Mindlin contact only,
        right after set_particles."""
        w = _f64(w).reshape(-1, self.np)
        self._check(self.lib.pibm_set_rotation(self.ctx, _dp(w)))

    def set_bodies(self, body, area=None):
        """Make particles points of fixed obstacle bodies (body index >= 0; -1
        moves); area: the area each fixed point spreads with (None: pi d^2/4).
        Needs make_config(bodies=1); right after set_particles."""
        body = np.ascontiguousarray(body, np.int32)
        self._check(self.lib.pibm_set_bodies(self.ctx, body.ctypes.data_as(C.POINTER(C.c_int32)),
                                             _dp(_f64(area)) if area is not None else None))

    def read_bodies(self, n_bodies):
        """Per body: hydrodynamic and contact force, torque about the centroid
        of its points (each 3 x n_bodies), from the last step."""
        out = {k: np.zeros((n_bodies, 3)) for k in ("f_hydro", "f_contact", "torque")}
        self._check(self.lib.pibm_read_bodies(self.ctx, int(n_bodies), _dp(out["f_hydro"]), _dp(out["f_contact"]),
                                              _dp(out["torque"])))
        return {k: v.T.copy() for k, v in out.items()}

    def read_rotation(self):
        w = np.empty((3 if self.D == 3 else 1, self.np))
        self._check(self.lib.pibm_read_rotation(self.ctx, _dp(w)))
        return w

    def read_fields(self):
        rho = np.empty(self.N, np.float32)
        u = np.empty((self.D, self.N), np.float32)
        self._check(self.lib.pibm_read_fields(self.ctx, _fp(rho), _fp(u)))
        return rho, u

    def read_force(self):
        F = np.empty((self.D, self.N), np.float32)
        self._check(self.lib.pibm_read_force(self.ctx, _fp(F)))
        return F

    def num_bins(self):
        return int(self.lib.pibm_num_bins(self.ctx))

    def read_cell_list(self):
        keys = np.empty(max(self.np, 1), np.uint32)
        ids = np.empty(max(self.np, 1), np.int32)
        bs = np.empty(self.num_bins() + 1, np.int32)
        self._check(self.lib.pibm_read_cell_list(
            self.ctx, keys.ctypes.data_as(C.POINTER(C.c_uint32)),
            ids.ctypes.data_as(C.POINTER(C.c_int32)), bs.ctypes.data_as(C.POINTER(C.c_int32))))
        return keys[: self.np], ids[: self.np], bs

    # --- stepping ----------------------------------------------------------
    def step(self, n=1):
        self._check(self.lib.pibm_step(self.ctx, int(n)))

    PHASES = ("cell_list", "moments", "interp", "dem", "spread", "collide")

    def set_profiling(self, on=True, every=1):
        """Phase events on every `every`-th step while on (see phase_times)."""
        self._check(self.lib.pibm_set_profiling(self.ctx, max(1, int(every)) if on else 0))

    def phase_times(self):
        """Milliseconds per phase summed over the recorded steps, and their
        number, since the last call."""
        ms = (C.c_double * 6)()
        steps = C.c_int64()
        self._check(self.lib.pibm_phase_times(self.ctx, ms, C.byref(steps)))
        return dict(zip(self.PHASES, list(ms))), steps.value

    def synchronize(self):
        self._check(self.lib.pibm_synchronize(self.ctx))

    def diagnostics(self):
        d = Diag()
        self._check(self.lib.pibm_diagnostics(self.ctx, C.byref(d)))
        return {"mass": d.mass, "momentum": list(d.momentum), "fluid_momentum": list(d.fluid_momentum),
                "max_speed": d.max_speed, "nonfinite": d.nonfinite, "active": d.active,
                "candidates": d.candidates, "min_height": d.min_height, "mean_height": d.mean_height}

    def conservation(self):
        m = C.c_double()
        p = (C.c_double * 3)()
        self._check(self.lib.pibm_conservation(self.ctx, C.byref(m), p))
        return m.value, list(p)

    # --- adjoint ---------------------------------------------------------
    def forward_ckpt(self, n_steps, K=100):
        """Run n_steps steps, recording checkpoints every K steps in a device
        buffer owned by this object (for backward).  The last segment is
        recorded step by step as it runs, and backward re-runs the others
        from their checkpoints: K >= n_steps records the whole rollout (the
        most memory, nothing run twice; see rollout_interval)."""
        import torch

        nbytes = self.lib.pibm_rollout_bytes(self.ctx, int(n_steps), int(K))
        if nbytes == 0:
            raise PibmError(2, "rollout not supported for this configuration")
        self.rollout_buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self._check(self.lib.pibm_forward_ckpt(self.ctx, int(n_steps), int(K),
                                               C.c_void_p(self.rollout_buf.data_ptr()), int(nbytes)))

    def rollout_interval(self, n_steps, share=0.25, K=100):
        """n_steps (the whole rollout recorded, no re-runs) when its buffer
        fits in `share` of the free device memory, else K."""
        import torch

        full = self.lib.pibm_rollout_bytes(self.ctx, int(n_steps), int(n_steps))
        free, _ = torch.cuda.mem_get_info(self.device)
        return int(n_steps) if 0 < full <= share * free else int(K)

    def backward_device(self, dJ_dx=None, dJ_dv=None):
        """Gradients of J given dJ/dX_T and dJ/dU_T ((D, N) arrays or tensors,
        id order) for the last forward_ckpt.  Returns dx0, dv0 as FP32 device
        tensors (D, N), dtau (float) and dgravity (3 floats)."""
        import torch

        def dev(a):
            return self._dev_f32(a).reshape(self.D, self.np) if a is not None else None

        gx, gv = dev(dJ_dx), dev(dJ_dv)
        dx0 = torch.empty((self.D, self.np), dtype=torch.float32, device=self.device)
        dv0 = torch.empty_like(dx0)
        dtau = C.c_double()
        dg = (C.c_double * 3)()

        def ptr(t):
            return C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_float)) if t is not None else None

        self._check(self.lib.pibm_backward(self.ctx, ptr(gx), ptr(gv), ptr(dx0), ptr(dv0), C.byref(dtau), dg))
        return {"dx0": dx0, "dv0": dv0, "dtau": dtau.value, "dgravity": list(dg)}

    def adjoint_stage(self, stage, in0, in1=None, in2=None):
        """One stage of the reverse step at the current state (see
        pibm_adjoint_stage; needs forward_ckpt first).  stage: "collide_t",
        "particles_t", "interp" or "interp_t"; inputs are arrays or tensors
        of the shapes the header gives.  Returns a dict of FP32 device
        tensors (and the stage's scalars as floats)."""
        import torch

        D, Q, N, n = self.D, self.cfg.lattice, self.N, self.np
        code = STAGE[stage]
        shapes = {"collide_t": ([(Q, N)], [(Q, N), (D, N)], 1),
                  "particles_t": ([(D, N), (D, n), (D, n)], [(D, n), (D, n), (1 + D, N)], 3),
                  "interp": ([(1 + D, N)], [(1 + D, n)], 0),
                  "interp_t": ([(1 + D, n)], [(1 + D, N)], 0)}[stage]
        ins = [self._dev_f32(a).reshape(sh) for a, sh in zip((in0, in1, in2), shapes[0])]
        outs = [torch.empty(sh, dtype=torch.float32, device=self.device) for sh in shapes[1]]
        nsc = shapes[2]
        sc = (C.c_double * 3)() if nsc else None
        vps = [self._vp(t) for t in ins] + [None] * (3 - len(ins))
        ops = [self._vp(t) for t in outs] + [None] * (3 - len(outs))
        self._check(self.lib.pibm_adjoint_stage(self.ctx, code, *vps, *ops, sc))
        names = {"collide_t": ("fbar", "Fbar"), "particles_t": ("xbar", "ubar", "mbar"),
                 "interp": ("out",), "interp_t": ("out",)}[stage]
        r = dict(zip(names, outs))
        if stage == "collide_t":
            r["dtau"] = sc[0]
        elif stage == "particles_t":
            r["dgravity"] = list(sc)
        return r

    def backward(self, dJ_dx=None, dJ_dv=None):
        """As backward_device, with dx0 and dv0 returned as numpy arrays."""
        r = self.backward_device(dJ_dx, dJ_dv)
        r["dx0"], r["dv0"] = r["dx0"].cpu().numpy(), r["dv0"].cpu().numpy()
        return r


def settling_rollout(cfg_kwargs, x0, d, rho_p, steps, K=None, device="cuda:0"):
    """A torch.autograd.Function over a checkpointed rollout of `steps`
    coupled steps, whose backward is the library's hand-written adjoint.

    Returns a callable f(tau, gravity, v0) -> X_T: tau a 0-d tensor, gravity
    a (3,) tensor (both small host parameters: they configure the step), v0
    a (D, N) tensor of initial velocities on the GPU.  X_T, the (D, N) final
    positions (FP64, the double-float state), stays on the GPU, and so do
    dJ/dv0 and the position data: the particle state moves in and out
    through the device-pointer calls, with no host copy.  x0 (D, N), d and
    rho_p (N) may be host arrays or device tensors.  Gradients of any
    J(X_T) with respect to tau, gravity and v0 come from pibm_backward.
    K: the checkpoint interval (None: Sim.rollout_interval, the whole
    rollout recorded when it fits)."""
    import torch

    dev = torch.device(device)
    x0 = torch.as_tensor(x0, dtype=torch.float64).to(dev)
    x_hi = x0.to(torch.float32)
    x_lo = (x0 - x_hi.to(torch.float64)).to(torch.float32)        # the exact double-float split
    d_t = torch.as_tensor(d).to(dev, torch.float32)
    rp_t = torch.as_tensor(rho_p).to(dev, torch.float32)
    d_max = float(np.max(np.asarray(d, np.float32))) if not torch.is_tensor(d) else float(d_t.max().item())
    npart = x0.shape[1]

    class Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, tau, gravity, v0):
            kw = dict(cfg_kwargs)
            kw["tau"] = float(tau)
            kw["gravity"] = tuple(float(g) for g in gravity.detach().cpu().tolist())
            sim = Sim(make_config(**kw), npart, device=dev)
            sim.set_particles_device(x_hi, d_t, rp_t, v=v0.detach(), x_lo=x_lo, d_max=d_max)
            sim.forward_ckpt(steps, sim.rollout_interval(steps) if K is None else K)
            p = sim.read_particles_device()
            ctx.sim = sim
            ctx.meta = (tau.dtype, tau.device, gravity.dtype, gravity.device, v0.dtype)
            return p["x_hi"].to(torch.float64) + p["x_lo"].to(torch.float64)

        @staticmethod
        def backward(ctx, gx):
            r = ctx.sim.backward_device(dJ_dx=gx.detach())
            t_dtype, t_dev, g_dtype, g_dev, v_dtype = ctx.meta
            return (torch.tensor(r["dtau"], dtype=t_dtype, device=t_dev),
                    torch.tensor(r["dgravity"], dtype=g_dtype, device=g_dev),
                    r["dv0"].to(v_dtype))

    return Rollout.apply
