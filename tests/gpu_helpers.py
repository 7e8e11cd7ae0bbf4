"""Shared plumbing of the GPU parity tests: build matching GPU and oracle
configurations, move states between them, and measure the per-field errors.

Error measures (floating point):
  eps_u   = ||u_gpu - u_ref||_2 / ||u_ref||_2 over all nodes and components,
            u = j / rho from the populations (FP64 on both sides)
  eps_rho = max |rho_gpu - rho_ref|
  particles: max |X_gpu - X_ref| relative to the step displacement, and
            ||U_gpu - U_ref||_2 / ||U_ref||_2
"""
import numpy as np


def oracle_cfg(orc, cfg):
    """The oracle configuration equal to a pibm.Config."""
    return orc.make_cfg(
        lattice=cfg.lattice, n=tuple(cfg.n), periodic=tuple(cfg.periodic), tau=cfg.tau,
        rho0=cfg.rho0, gravity=tuple(cfg.gravity), fluid_force=tuple(cfg.fluid_force),
        contact=cfg.contact, kn=cfg.kn, restitution=cfg.restitution, k_soft=cfg.k_soft,
        skin=cfg.skin, n_sub=cfg.n_sub, two_way=cfg.two_way, bin_log2=cfg.bin_log2,
        interp="lagrange" if cfg.interp == 1 else "delta", young=cfg.young, poisson=cfg.poisson,
        friction=cfg.friction)


def weights(orc, lattice):
    _, w, _ = orc.tables(lattice)
    return w


def to_oracle_f(orc, lattice, h):
    """FP64 populations f = w + h from the GPU deviations (Q, N)."""
    w = weights(orc, lattice)
    return (np.asarray(h, np.float64) + w[:, None]).reshape(-1)


def moments64(orc, lattice, f, N):
    e, _, _ = orc.tables(lattice)
    D = 2 if lattice == 9 else 3
    f = np.asarray(f, np.float64).reshape(-1, N)
    rho = f.sum(axis=0)
    j = e[:, :D].T.astype(np.float64) @ f
    return rho, j


def moments_dev(orc, lattice, h):
    """Density deviation and momentum from deviations h (sums of small
    numbers; exact enough to compare FP32 states)."""
    e, _, _ = orc.tables(lattice)
    D = 2 if lattice == 9 else 3
    h = np.asarray(h, np.float64)
    return h.sum(axis=0), e[:, :D].T.astype(np.float64) @ h


def field_errors(orc, lattice, h_gpu, f_ref, N):
    w = weights(orc, lattice)
    h_ref = np.asarray(f_ref, np.float64).reshape(-1, N) - w[:, None]
    dr_g, j_g = moments_dev(orc, lattice, h_gpu)
    dr_r, j_r = moments_dev(orc, lattice, h_ref)
    u_g = j_g / (1 + dr_g)
    u_r = j_r / (1 + dr_r)
    eps_u = np.linalg.norm(u_g - u_r) / max(np.linalg.norm(u_r), 1e-300)
    eps_rho = np.abs(dr_g - dr_r).max()
    eps_h = np.abs(np.asarray(h_gpu, np.float64) - h_ref).max() / max(np.abs(h_ref).max(), 1e-300)
    return eps_u, eps_rho, eps_h


def perturbed_state(orc, sim, w, seed, amp=1e-3, noneq=1e-2):
    """A smooth perturbed equilibrium plus a small non-equilibrium part,
    written to the GPU; returns the exact stored deviations (Q, N)."""
    from paper_1407_6704_amd import workloads as W

    rho, u = W.perturbed_fluid(w, seed, amp)
    sim.init_equilibrium(rho.astype(np.float32), u.astype(np.float32))
    h = sim.read_populations().astype(np.float64)
    rng = np.random.default_rng(seed + 1000)
    ww = weights(orc, w.lattice)
    h = h + noneq * amp * ww[:, None] * rng.standard_normal(h.shape)
    sim.write_populations(h.astype(np.float32))
    return sim.read_populations()
