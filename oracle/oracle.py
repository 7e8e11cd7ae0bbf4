"""ctypes wrapper of the FP64 CPU oracle (``pibm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the GPU library never does.  The C source is the
oracle; this file only marshals numpy arrays.  Every function names the part
of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pibm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2; OpenMP on the two node loops,
    whose results do not depend on the thread count)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Cfg(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("n", C.c_int * 3), ("periodic", C.c_int * 3),
        ("tau", C.c_double), ("rho0", C.c_double), ("gravity", C.c_double * 3),
        ("fluid_force", C.c_double * 3), ("contact", C.c_int), ("kn", C.c_double),
        ("restitution", C.c_double), ("k_soft", C.c_double), ("skin", C.c_double),
        ("n_sub", C.c_int), ("two_way", C.c_int), ("bin_log2", C.c_int), ("interp", C.c_int),
        ("young", C.c_double), ("poisson", C.c_double), ("friction", C.c_double),
    ]


CONTACT = {"none": 0, "lsd": 1, "soft": 2, "hertz": 3, "hertz_mindlin": 4, "hertz_mindlin_microslip": 5}
TS = 10     # doubles of tangential state per contact (ORC_TS in the C source)

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d = C.POINTER(C.c_double)
        i = C.POINTER(C.c_int)
        i64 = C.POINTER(C.c_int64)
        cp = C.POINTER(Cfg)
        sig = {
            "orc_q": ([C.c_int], C.c_int),
            "orc_threads": ([], C.c_int),
            "orc_set_threads": ([C.c_int], None),
            "orc_dim": ([C.c_int], C.c_int),
            "orc_tables": ([C.c_int, i, d, i], None),
            "orc_equilibrium": ([C.c_int, C.c_double, d, d], None),
            "orc_moments": ([cp, d, d, d], None),
            "orc_collide_stream": ([cp, d, d, d], None),
            "orc_delta": ([C.c_double], C.c_double),
            "orc_weights": ([cp, d, i, d], None),
            "orc_weights_lagrange": ([cp, d, i, d], None),
            "orc_interp": ([cp, C.c_int, d, d, d, d, d], None),
            "orc_spread": ([cp, C.c_int, d, d, d], None),
            "orc_nbins": ([cp, i64], C.c_int64),
            "orc_key": ([cp, d], C.c_int64),
            "orc_cell_list": ([cp, C.c_int, d, i64, i, i64], None),
            "orc_mass": ([C.c_int, C.c_double, C.c_double], C.c_double),
            "orc_area": ([C.c_double], C.c_double),
            "orc_zeta": ([C.c_double], C.c_double),
            "orc_candidate_pairs": ([cp, C.c_int, d, d, i, C.c_int64], C.c_int64),
            "orc_candidate_pairs_brute": ([cp, C.c_int, d, d, i, C.c_int64], C.c_int64),
            "orc_dem": ([cp, C.c_int, d, d, d, d, d, d, C.c_int64, i, d, d, d], None),
            "orc_dem_full": ([cp, C.c_int, d, d, d, d, d, i, d, d, C.c_int64, i, C.c_int64, i, d, i, d, d, d,
                              d], C.c_int64),
            "orc_step_full": ([cp, d, d, d, C.c_int, d, d, d, d, d, i, d, C.c_int64, i, d, i, d, i64, d, d, d,
                               d], C.c_int),
            "orc_step": ([cp, d, d, d, C.c_int, d, d, d, d, d, d, d, d], C.c_int),
            "orc_fluid_totals": ([cp, d, d, d], None),
            "orc_tangential_update": ([cp, C.c_double, d, d, C.c_double, C.c_double, C.c_double, d], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = res
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _i64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def make_cfg(lattice=9, n=(16, 16, 1), periodic=(0, 0, 0), tau=0.8, rho0=1.0,
             gravity=(0.0, 0.0, 0.0), fluid_force=(0.0, 0.0, 0.0), contact="lsd",
             kn=1e3, restitution=0.9, k_soft=1e-3, skin=0.05, n_sub=1, two_way=1,
             bin_log2=1, interp="delta", young=1e-3, poisson=0.33, friction=0.33) -> Cfg:
    c = Cfg()
    c.lattice = int(lattice)
    for a in range(3):
        c.n[a] = int(n[a])
        c.periodic[a] = int(periodic[a])
        c.gravity[a] = float(gravity[a])
        c.fluid_force[a] = float(fluid_force[a])
    c.tau, c.rho0 = float(tau), float(rho0)
    c.contact = CONTACT[contact] if isinstance(contact, str) else int(contact)
    c.kn, c.restitution, c.k_soft, c.skin = float(kn), float(restitution), float(k_soft), float(skin)
    c.n_sub, c.two_way, c.bin_log2 = int(n_sub), int(two_way), int(bin_log2)
    c.interp = {"delta": 0, "lagrange": 1}[interp] if isinstance(interp, str) else int(interp)
    c.young, c.poisson, c.friction = float(young), float(poisson), float(friction)
    return c


def threads() -> int:
    """Threads the node loops use."""
    return lib().orc_threads()


def set_threads(n: int) -> None:
    """Threads for the node loops; n < 1 restores the runtime's default."""
    lib().orc_set_threads(int(n))


def Q(cfg):
    return int(cfg.lattice)


def D(cfg):
    return 2 if cfg.lattice == 9 else 3


def nnodes(cfg):
    return cfg.n[0] * cfg.n[1] * cfg.n[2]


def tables(lattice):
    q = int(lattice)
    e = np.zeros((q, 3), np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, np.int32)
    lib().orc_tables(lattice, _i(e), _d(w), _i(opp))
    return e, w, opp


def equilibrium(lattice, rho, u):
    q = int(lattice)
    out = np.zeros(q)
    u3 = np.zeros(3)
    u3[: len(u)] = u
    lib().orc_equilibrium(lattice, float(rho), _d(u3), _d(out))
    return out


def moments(cfg, f):
    N = nnodes(cfg)
    f = _f64(f)
    rho = np.zeros(N)
    j = np.zeros(3 * N)
    lib().orc_moments(C.byref(cfg), _d(f), _d(rho), _d(j))
    return rho, j.reshape(3, N)


def collide_stream(cfg, f, F=None):
    N = nnodes(cfg)
    f = _f64(f)
    out = np.zeros_like(f)
    if F is None:
        lib().orc_collide_stream(C.byref(cfg), _d(f), None, _d(out))
    else:
        F3 = np.zeros((3, N))
        F = np.asarray(F, float).reshape(-1, N)
        F3[: F.shape[0]] = F
        lib().orc_collide_stream(C.byref(cfg), _d(f), _d(F3), _d(out))
    return out


def delta(a):
    return lib().orc_delta(float(a))


def weights(cfg, X):
    X3 = np.full(3, 0.5)
    X3[: len(X)] = X
    base = np.zeros(3, np.int32)
    phi = np.zeros(12)
    lib().orc_weights(C.byref(cfg), _d(X3), _i(base), _d(phi))
    return base, phi.reshape(3, 4)


def weights_lagrange(cfg, X):
    X3 = np.full(3, 0.5)
    X3[: len(X)] = X
    base = np.zeros(3, np.int32)
    phi = np.zeros(12)
    lib().orc_weights_lagrange(C.byref(cfg), _d(X3), _i(base), _d(phi))
    return base, phi.reshape(3, 4)


def interp(cfg, X, rho, j):
    X = _f64(X)
    np_ = X.shape[-1]
    rho_i = np.zeros(np_)
    j_i = np.zeros(3 * np_)
    j3 = np.zeros((3, nnodes(cfg)))
    jj = np.asarray(j, float).reshape(-1, nnodes(cfg))
    j3[: jj.shape[0]] = jj
    lib().orc_interp(C.byref(cfg), np_, _d(X), _d(_f64(rho)), _d(j3), _d(rho_i), _d(j_i))
    return rho_i, j_i.reshape(3, np_)[: D(cfg)]


def spread(cfg, X, coef):
    X = _f64(X)
    np_ = X.shape[-1]
    F = np.zeros((D(cfg), nnodes(cfg)))
    lib().orc_spread(C.byref(cfg), np_, _d(X), _d(_f64(coef)), _d(F))
    return F


def nbins(cfg):
    nb = np.zeros(3, np.int64)
    tot = lib().orc_nbins(C.byref(cfg), _i64(nb))
    return tot, nb


def cell_list(cfg, X):
    X = _f64(X)
    np_ = X.shape[-1]
    tot, _ = nbins(cfg)
    keys = np.zeros(max(np_, 1), np.int64)
    perm = np.zeros(max(np_, 1), np.int32)
    bs = np.zeros(tot + 1, np.int64)
    lib().orc_cell_list(C.byref(cfg), np_, _d(X), _i64(keys), _i(perm), _i64(bs))
    return keys[:np_], perm[:np_], bs


def mass(dim, d, rho_p):
    return lib().orc_mass(dim, float(d), float(rho_p))


def area(d):
    return lib().orc_area(float(d))


def zeta(e):
    return lib().orc_zeta(float(e))


def candidate_pairs(cfg, X, d, brute=False):
    X = _f64(X)
    d = _f64(d)
    np_ = X.shape[-1]
    fn = lib().orc_candidate_pairs_brute if brute else lib().orc_candidate_pairs
    n = fn(C.byref(cfg), np_, _d(X), _d(d), None, 0)
    pairs = np.zeros(2 * max(n, 1), np.int32)
    fn(C.byref(cfg), np_, _d(X), _d(d), _i(pairs), n)
    return pairs[: 2 * n].reshape(n, 2)


def dem(cfg, X, U, d, rho_p, rho_i, j_i, pairs=None):
    """O4 on copies of X, U; returns (X', U', gbar, fc_mean, vmax)."""
    dim = D(cfg)
    X = _f64(X).copy()
    U = _f64(U).copy()
    np_ = X.shape[-1]
    if pairs is None:
        pairs = candidate_pairs(cfg, X, d) if cfg.contact else np.zeros((0, 2), np.int32)
    pairs = np.ascontiguousarray(pairs, np.int32)
    j3 = np.zeros((3, np_))
    j3[:dim] = np.asarray(j_i, float).reshape(-1, np_)[:dim]
    gbar = np.zeros(3 * np_)
    fc = np.zeros(3 * np_)
    vmax = np.zeros(np_)
    lib().orc_dem(C.byref(cfg), np_, _d(X), _d(U), _d(_f64(d)), _d(_f64(rho_p)),
                  _d(_f64(rho_i)), _d(j3), len(pairs), _i(pairs), _d(gbar), _d(fc), _d(vmax))
    return X, U, gbar.reshape(3, np_)[:dim], fc.reshape(3, np_)[:dim], vmax


def _hist_arrays(hist):
    if hist is None:
        return np.zeros((1, 2), np.int32), np.zeros((1, TS)), 0
    keys, T = hist
    n = len(keys)
    k = np.ascontiguousarray(np.asarray(keys, np.int32).reshape(-1, 2)) if n else np.zeros((1, 2), np.int32)
    t = np.ascontiguousarray(np.asarray(T, np.float64).reshape(-1, TS)) if n else np.zeros((1, TS))
    return k, t, n


def tangential_update(cfg, h, n, vrel, Fn, rstar, delta, state):
    """One contact's tangential update (contact 4 or 5) on a copy of the
    state (TS doubles: T, loading direction, k, T*, T**, previous F_n)."""
    S = np.ascontiguousarray(np.asarray(state, np.float64).reshape(TS)).copy()
    nn = np.zeros(3)
    nn[: len(n)] = n
    vv = np.zeros(3)
    vv[: len(vrel)] = vrel
    lib().orc_tangential_update(C.byref(cfg), float(h), _d(nn), _d(vv), float(Fn), float(rstar), float(delta),
                                _d(S))
    return S


def dem_hm(cfg, X, U, W, d, rho_p, rho_i, j_i, hist=None, pairs=None, fixed=None):
    """O4 with the Hertz-Mindlin contact and rotation (contact = 4 or 5) on
    copies; W is (3, np) (2D: the z row only is used).  hist = (keys (n, 2),
    state (n, TS)) or None; fixed: np flags of fixed obstacle points or None.
    Returns (X', U', W', gbar, fc_mean, vmax, hist').  Works for every
    contact model (W and hist then stay unused)."""
    dim = D(cfg)
    X = _f64(X).copy()
    U = _f64(U).copy()
    np_ = X.shape[-1]
    W = np.ascontiguousarray(np.asarray(W, np.float64).reshape(3, np_)).copy()
    if pairs is None:
        pairs = candidate_pairs(cfg, X, d)
    pairs = np.ascontiguousarray(pairs, np.int32)
    j3 = np.zeros((3, np_))
    j3[:dim] = np.asarray(j_i, float).reshape(-1, np_)[:dim]
    gbar = np.zeros(3 * np_)
    fc = np.zeros(3 * np_)
    vmax = np.zeros(np_)
    kin, tin, hn = _hist_arrays(hist)
    cap = len(pairs) + 6 * np_ + 1
    kout = np.zeros((cap, 2), np.int32)
    tout = np.zeros((cap, TS))
    fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, np.int32))
    n = lib().orc_dem_full(C.byref(cfg), np_, _d(X), _d(U), _d(W), _d(_f64(d)), _d(_f64(rho_p)),
                           None if fx is None else _i(fx),
                           _d(_f64(rho_i)), _d(j3), len(pairs), _i(pairs), hn, _i(kin), _d(tin),
                           _i(kout), _d(tout), _d(gbar), _d(fc), _d(vmax))
    return (X, U, W, gbar.reshape(3, np_)[:dim], fc.reshape(3, np_)[:dim], vmax,
            (kout[:n].copy(), tout[:n].copy()))


def step_hm(cfg, f, X, U, W, d, rho_p, hist=None):
    """One coupled step with the Hertz-Mindlin contact and rotation; as
    step(), plus "W" and "hist" in the result."""
    return step_full(cfg, f, X, U, d, rho_p, W=W, hist=hist)


def step_full(cfg, f, X, U, d, rho_p, W=None, hist=None, fixed=None, area=None):
    """One coupled step with every option: angular velocities W (3, np) and
    the tangential history for the Hertz-Mindlin contact, and the points of
    fixed obstacle bodies (fixed: np flags; area: np areas used for the
    fixed points' spreading, None for pi d^2 / 4).  Returns step()'s dict
    plus "W" and "hist"."""
    dim = D(cfg)
    N = nnodes(cfg)
    f = _f64(f)
    X = _f64(X).copy()
    U = _f64(U).copy()
    np_ = X.shape[-1]
    W = np.zeros((3, np_)) if W is None else np.asarray(W, np.float64).reshape(3, np_)
    W = np.ascontiguousarray(W).copy()
    fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, np.int32))
    ar = None if area is None else _f64(area)
    fout = np.zeros_like(f)
    F = np.zeros(dim * N)
    gbar = np.zeros(3 * np_)
    fc = np.zeros(3 * np_)
    rho_i = np.zeros(np_)
    j_i = np.zeros(3 * np_)
    kin, tin, hn = _hist_arrays(hist)
    cap = 64 * np_ + 6 * np_ + 1
    kout = np.zeros((cap, 2), np.int32)
    tout = np.zeros((cap, TS))
    hout = np.zeros(1, np.int64)
    nskin = lib().orc_step_full(C.byref(cfg), _d(f), _d(fout), _d(F), np_, _d(X), _d(U), _d(W),
                                _d(_f64(d)), _d(_f64(rho_p)), None if fx is None else _i(fx),
                                None if ar is None else _d(ar), hn, _i(kin), _d(tin), _i(kout), _d(tout),
                                hout.ctypes.data_as(C.POINTER(C.c_int64)), _d(gbar), _d(fc), _d(rho_i),
                                _d(j_i))
    n = int(hout[0])
    return {
        "f": fout, "F": F.reshape(dim, N), "X": X, "U": U, "W": W,
        "gbar": gbar.reshape(3, np_)[:dim], "fc": fc.reshape(3, np_)[:dim],
        "rho_i": rho_i, "j_i": j_i.reshape(3, np_)[:dim], "nskin": nskin,
        "hist": (kout[:n].copy(), tout[:n].copy()),
    }


def step(cfg, f, X, U, d, rho_p):
    """One coupled step O1..O7.  Returns a dict with the new state and the
    by-products; inputs are not modified."""
    dim = D(cfg)
    N = nnodes(cfg)
    f = _f64(f)
    X = _f64(X).copy()
    U = _f64(U).copy()
    np_ = X.shape[-1] if X.size else 0
    fout = np.zeros_like(f)
    F = np.zeros(dim * N)
    gbar = np.zeros(3 * max(np_, 1))
    fc = np.zeros(3 * max(np_, 1))
    rho_i = np.zeros(max(np_, 1))
    j_i = np.zeros(3 * max(np_, 1))
    if np_ == 0:
        X = np.zeros((dim, 1))
        U = np.zeros((dim, 1))
        d = np.zeros(1)
        rho_p = np.ones(1)
    nskin = lib().orc_step(C.byref(cfg), _d(f), _d(fout), _d(F), np_, _d(X), _d(U),
                           _d(_f64(d)), _d(_f64(rho_p)), _d(gbar), _d(fc), _d(rho_i), _d(j_i))
    return {
        "f": fout, "F": F.reshape(dim, N), "X": X[:, :np_], "U": U[:, :np_],
        "gbar": gbar[: 3 * np_].reshape(3, np_)[:dim] if np_ else np.zeros((dim, 0)),
        "fc": fc[: 3 * np_].reshape(3, np_)[:dim] if np_ else np.zeros((dim, 0)),
        "rho_i": rho_i[:np_], "j_i": j_i[: 3 * np_].reshape(3, np_)[:dim] if np_ else np.zeros((dim, 0)),
        "nskin": nskin,
    }


def fluid_totals(cfg, f):
    m = C.c_double(0)
    mom = np.zeros(3)
    lib().orc_fluid_totals(C.byref(cfg), _d(_f64(f)), C.byref(m), _d(mom))
    return m.value, mom


def rest_state(cfg, rho=1.0):
    """Populations of fluid at rest with density rho: f_q = w_q rho."""
    _, w, _ = tables(cfg.lattice)
    return np.repeat(w[:, None] * rho, nnodes(cfg), axis=1).reshape(-1)
