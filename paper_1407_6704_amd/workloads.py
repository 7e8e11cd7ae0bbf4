"""Seeded synthetic workloads: lattice and particle set-ups of the paper's
sedimentation experiments, at the sizes the benchmark and the tests use.

This module only draws inputs.  It holds none of the method's arithmetic, so
both the GPU path and the CPU oracle may consume what it produces.

The paper's runs are cavities filled with fluid at rest and particles placed
at random in an upper part of the box (Sec. 3.2: 5000 disks in the upper
three fifths of a square cavity; Sec. 3.3: 8125 spheres in a closed cube),
released from rest, with no-slip walls on every face.  The workloads below
keep that structure at larger scale:

  c0  D2Q9 128^2, tau 0.8, 200 disks d = 0.4, rho_p/rho_f = 2.5, upper half
  c1  D2Q9 2048^2, tau 0.6, 500k disks d ~ U[0.3, 0.8], ratio 2.5, upper 60 %
  c2  D3Q19 256^3, tau 0.6, 2M spheres, d lognormal (mean 0.5, sd 0.2,
      truncated to [0.2, 1.0]), ratio 2.0, upper half
  c3  c2 with populations stored as FP16 deviations, from the same initial
      state (and a 64^3 crop with the same number density, 31,250 spheres)
  c4  D2Q9 512^2, tau 0.7, 10k disks d = 0.5, ratio 2.5, soft repulsion,
      dilute (gaps >= d, >= 3 from walls), objective = mean height
  hybrid  the hybrid IBM-PIBM case of Sec. 3.3 at scale: c2's particle
      statistics in a 128^3 cavity (250k spheres in the upper half) above
      five fixed obstacles (make_hybrid): four spheres of radius 10 made of
      conventional-IBM surface points and a cube of 27 fixed PIBM points

Gravity is 1e-5 lattice units along -y (2D) or -z (3D).  The candidate-list
skin is 0.01: a particle may move at most skin/2 per step, 100 times the
settling displacement per step of these flows.  The linear
spring-dashpot contact has k_n = 1e3 and restitution 0.9; the sub-step count
is the one that resolves the shortest contact (20 sub-steps per contact time
of the two smallest particles): 508, 677, 3109 for c0, c1, c2.

Positions and diameters are drawn in FP64 and rounded to FP32-representable
values, so that both sides of every comparison start from identical numbers.
Placement is random sequential addition in batches: candidates are drawn
uniformly in the region, and a candidate that overlaps an accepted particle
(or an earlier candidate of its batch) is redrawn.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    lattice: int                      # 9 (D2Q9) or 19 (D3Q19)
    n: tuple                          # nodes per axis (nz = 1 in 2D)
    tau: float
    n_particles: int
    diameter: tuple                   # ("const", d) | ("uniform", lo, hi) | ("lognormal", mean, sd, lo, hi)
    density_ratio: float
    region: tuple                     # fraction of the vertical axis: (lo, hi)
    gravity: float = 1e-5
    contact: str = "lsd"              # "lsd" | "soft" | "none"
    kn: float = 1e3
    restitution: float = 0.9
    k_soft: float = 1e-3
    skin: float = 0.01
    n_sub: int = 1
    steps: int = 100
    storage: str = "fp32"             # "fp32" | "fp16"
    fp16_scale_log2: int = 14
    seed: int = 0
    gap: float = 1e-3                 # minimum surface gap at placement
    wall_clear: float = 0.0           # extra clearance from walls beyond d/2
    bin_log2: int = 0                 # cell-list bins = dual cells
    two_way: int = 1
    interp: str = "delta"             # gather: "delta" (Eqs. lbm11-lbm12) | "lagrange" (Eqs. lbm5-lbm6)
    young: float = 1e3                # Hertz contacts: Young's modulus (lattice units)
    poisson: float = 0.33             # Hertz contacts: Poisson ratio (Table 1)
    friction: float = 0.33            # Hertz-Mindlin: Coulomb coefficient (Table 1)
    obstacles: bool = False           # fixed obstacle bodies below the particles (make_hybrid)
    extra: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return 2 if self.lattice == 9 else 3

    @property
    def nodes(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def gravity_vec(self):
        g = [0.0, 0.0, 0.0]
        g[self.dim - 1] = -self.gravity
        return tuple(g)

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


C0 = Workload("c0", 9, (128, 128, 1), 0.8, 200, ("const", 0.4), 2.5, (0.5, 1.0),
              n_sub=508, steps=1000, seed=0)
C1 = Workload("c1", 9, (2048, 2048, 1), 0.6, 500_000, ("uniform", 0.3, 0.8), 2.5, (0.4, 1.0),
              n_sub=677, steps=5000, seed=1)
C2 = Workload("c2", 19, (256, 256, 256), 0.6, 2_000_000, ("lognormal", 0.5, 0.2, 0.2, 1.0), 2.0,
              (0.5, 1.0), n_sub=3109, steps=2000, seed=2)
C3 = C2.replace(name="c3", storage="fp16")          # same initial state as c2
C3_CROP = C3.replace(name="c3_crop64", n=(64, 64, 64), n_particles=31_250, steps=100, seed=3)
# c2 on the paper's own lattice and gather: D3Q15 with Lagrange polynomials (same particles)
C2_D3Q15 = C2.replace(name="c2_d3q15", lattice=15, interp="lagrange")
# c2 particles with the paper's contact law: Hertz normal and Mindlin tangential
# forces with rotation (Table 1 Poisson ratio and friction)
C2_HM = C2.replace(name="c2_hm", contact="hertz_mindlin")
C2_HMS = C2.replace(name="c2_hms", contact="hertz_mindlin_microslip")
HYBRID = C2.replace(name="hybrid", n=(128, 128, 128), n_particles=250_000, steps=200, seed=6, obstacles=True)
C4 = Workload("c4", 9, (512, 512, 1), 0.7, 10_000, ("const", 0.5), 2.5, (0.5, 1.0),
              contact="soft", n_sub=1, steps=2000, seed=4, gap=0.5, wall_clear=3.0)
C4_FD = C4.replace(name="c4_fd", n=(64, 64, 1), n_particles=50, seed=40)

WORKLOADS = {w.name: w for w in (C0, C1, C2, C3, C3_CROP, C2_D3Q15, C2_HM, C2_HMS, HYBRID, C4, C4_FD)}


def draw_diameters(rng, spec, n):
    kind = spec[0]
    if kind == "const":
        d = np.full(n, float(spec[1]))
    elif kind == "uniform":
        d = rng.uniform(spec[1], spec[2], n)
    elif kind == "lognormal":
        mean, sd, lo, hi = spec[1:]
        s2 = np.log(1.0 + (sd / mean) ** 2)
        mu = np.log(mean) - 0.5 * s2
        d = np.empty(0)
        while d.size < n:          # truncation by resampling
            x = rng.lognormal(mu, np.sqrt(s2), 2 * (n - d.size) + 16)
            d = np.concatenate([d, x[(x >= lo) & (x <= hi)]])
        d = d[:n]
    else:
        raise ValueError(spec)
    return d.astype(np.float32).astype(np.float64)


def _overlapping(X_acc, d_acc, Xc, dc, gap):
    """Boolean mask over the candidates Xc (D, m): True where a candidate comes
    closer than gap (surface to surface) to an accepted particle or to an
    earlier candidate."""
    from scipy.spatial import cKDTree

    m = Xc.shape[1]
    bad = np.zeros(m, bool)
    if m == 0:
        return bad
    reach = float(max(dc.max(), d_acc.max() if d_acc.size else 0.0)) + gap
    tc = cKDTree(Xc.T)
    pairs = tc.query_pairs(reach, output_type="ndarray")
    if pairs.size:
        i, j = pairs[:, 0], pairs[:, 1]
        r2 = ((Xc[:, i] - Xc[:, j]) ** 2).sum(axis=0)
        lim = 0.5 * (dc[i] + dc[j]) + gap
        hit = r2 < lim * lim
        bad[np.maximum(i, j)[hit]] = True
    if d_acc.size:
        ta = cKDTree(X_acc.T)
        sdm = tc.sparse_distance_matrix(ta, reach, output_type="ndarray")
        if sdm.size:
            ci, ai = sdm["i"], sdm["j"]
            lim = 0.5 * (dc[ci] + d_acc[ai]) + gap
            hit = sdm["v"] < lim
            bad[ci[hit]] = True
    return bad


def place_particles(w: Workload, seed: int | None = None):
    """Random sequential addition (batched).  Returns X (D, N) float64 holding
    FP32-representable values, and the diameters (N,)."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    D = w.dim
    N = w.n_particles
    d_all = draw_diameters(rng, w.diameter, N)
    lo = np.zeros(D)
    hi = np.array([float(w.n[a]) for a in range(D)])
    lo[D - 1] = w.region[0] * w.n[D - 1]
    hi[D - 1] = w.region[1] * w.n[D - 1]
    X = np.zeros((D, 0))
    d_acc = np.zeros(0)
    todo = d_all.copy()
    it = 0
    while todo.size:
        it += 1
        if it > 200:
            raise RuntimeError("placement did not converge; region too dense")
        m = todo.size
        Xc = np.empty((D, m))
        for a in range(D):
            margin = 0.5 * todo + w.wall_clear
            lo_a = lo[a] + (margin if (lo[a] == 0 or a < D - 1) else 0.5 * todo)
            hi_a = hi[a] - margin
            Xc[a] = lo_a + rng.random(m) * (hi_a - lo_a)
        Xc = Xc.astype(np.float32).astype(np.float64)
        bad = _overlapping(X, d_acc, Xc, todo, w.gap)
        X = np.concatenate([X, Xc[:, ~bad]], axis=1)
        d_acc = np.concatenate([d_acc, todo[~bad]])
        todo = todo[bad]
    return X, d_acc


def make_particles(w: Workload, seed: int | None = None):
    """Initial particle state: positions, zero velocities, diameters, densities."""
    X, d = place_particles(w, seed)
    U = np.zeros_like(X)
    rho_p = np.full(d.shape, float(w.density_ratio))
    return X, U, d, rho_p


def sphere_points(k: int):
    """k nearly uniform unit vectors (Fibonacci sphere), (3, k)."""
    t = np.arange(k) + 0.5
    z = 1.0 - 2.0 * t / k
    phi = np.pi * (1.0 + 5.0 ** 0.5) * t
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z])


def make_hybrid(w: Workload, radius: float = 10.0, spacing: float = 0.8, cube_spacing: float = 1.0,
                cube_d: float = 1.0):
    """The moving particles of w (upper part) plus five fixed obstacles at a
    quarter of the height: four spheres of the given radius, each k surface
    points about `spacing` apart (contact diameter = spacing, area = the
    sphere's area / k), centred over the quarters of the floor, and a
    3 x 3 x 3 cube of PIBM points (diameter cube_d, area pi d^2/4) in the
    middle.  Returns X, U, d, rho_p, body (-1: moving; 0..3 spheres, 4 the
    cube), area (0 for the moving particles and the cube's points: pi d^2/4).
    Obstacle points come first."""
    Xm, Um, dm, rpm = make_particles(w)
    n = [float(v) for v in w.n]
    zc = 0.25 * n[2]
    k = int(round(4.0 * np.pi * radius * radius / (spacing * spacing)))
    S = sphere_points(k)
    pts, body, dd, area = [], [], [], []
    for b, (fx, fy) in enumerate([(0.25, 0.25), (0.75, 0.25), (0.25, 0.75), (0.75, 0.75)]):
        c = np.array([fx * n[0], fy * n[1], zc])
        pts.append(c[:, None] + radius * S)
        body += [b] * k
        dd += [spacing] * k
        area += [4.0 * np.pi * radius * radius / k] * k
    g = (np.arange(3) - 1.0) * cube_spacing
    cube = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1) + np.array([0.5 * n[0], 0.5 * n[1], zc])[:, None]
    pts.append(cube)
    body += [4] * 27
    dd += [cube_d] * 27
    area += [0.0] * 27
    Xf = np.concatenate(pts, axis=1).astype(np.float32).astype(np.float64)
    nf = Xf.shape[1]
    X = np.concatenate([Xf, Xm], axis=1)
    U = np.concatenate([np.zeros((3, nf)), Um], axis=1)
    d = np.concatenate([np.array(dd, np.float32).astype(np.float64), dm])
    rp = np.concatenate([np.ones(nf), rpm])
    return X, U, d, rp, np.array(body + [-1] * Xm.shape[1], np.int32), np.concatenate([np.array(area), np.zeros(Xm.shape[1])])


def perturbed_fluid(w: Workload, seed: int, amp: float = 1e-3):
    """A smooth random velocity and density perturbation of the rest state,
    for one-step comparisons: rho = 1 + amp * r0, u = amp * r_a, with r drawn
    per node and smoothed once along every axis.  Returns (rho (N,), u (D, N))."""
    rng = np.random.default_rng(seed)
    D = w.dim
    shape = (w.n[2], w.n[1], w.n[0])
    fields = []
    for _ in range(D + 1):
        r = rng.standard_normal(shape)
        for ax in range(3):
            if shape[ax] > 2:
                r = (np.roll(r, 1, ax) + 2 * r + np.roll(r, -1, ax)) / 4.0
        fields.append(r.reshape(-1))
    rho = 1.0 + amp * fields[0]
    u = np.stack([amp * f for f in fields[1:]])
    return rho, u
