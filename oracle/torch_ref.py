"""TEST INFRASTRUCTURE ONLY: a slow, differentiable FP64 PyTorch (CPU)
reference of the coupled LBM / PIBM / DEM step, for checking the GPU
library's hand-written adjoint.

Only the test suite may import this module.  It shares no code with the GPU
library or with the C oracle; the lattice tables are written out again from
the textbook definitions of D2Q9 and D3Q19.  Autograd through `step` gives
the exact gradient of the discrete map (up to FP64 rounding).  The tests pin
its forward against the C oracle step by step, and its gradient against
central differences of the C oracle.

Scope: every reading of the C oracle (Sec. 2 of the paper):
  Sec. 2.1   BGK collision with Guo forcing (Eq. lbm2, lbm9), push streaming,
             halfway bounce-back at walls, periodic axes
  Sec. 2.2   4-point cosine delta kernel (Eq. lbm11-lbm12), per-axis
             renormalisation at walls, interpolation of rho and j, momentum
             exchange g = 2 (rho_i U - j_i) (Eq. lbm7-lbm8, lbm13), spreading
             of A_p gbar (Eq. lbm10)
  Sec. 2.3   sub-stepped particle update (Eq. demgov) with no contact or the
             soft repulsion k_s (1 - r/r_c)^2 (pairs by brute force, walls as
             particles of infinite mass); the linear spring-dashpot is not
             included (its on/off switch at zero overlap has no gradient)
Particles: X, U of shape (D, np); populations f of shape (Q, N), node index
(z * ny + y) * nx + x.
"""
from __future__ import annotations

import math

import torch

_E9 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
       (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)]
_E19 = [(0, 0, 0),
        (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
        (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
        (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
        (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
_E15 = [(0, 0, 0),
        (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
        (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
        (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)]


def lattice_tables(lattice: int):
    """Velocities e (Q, 3), weights w (Q,) and opposite directions."""
    E = {19: _E19, 15: _E15}.get(lattice, _E9)
    e = torch.tensor(E, dtype=torch.float64)
    by_speed2 = {19: {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0},
                 15: {0: 2.0 / 9.0, 1: 1.0 / 9.0, 3: 1.0 / 72.0}}.get(lattice, {0: 4.0 / 9.0, 1: 1.0 / 9.0,
                                                                               2: 1.0 / 36.0})
    w = torch.tensor([by_speed2[sum(c * c for c in v)] for v in E], dtype=torch.float64)
    opp = [E.index(tuple(-c for c in v)) for v in E]
    return e, w, opp


class Ref:
    """Fixed geometry, particle sizes and physical constants of one case."""

    def __init__(self, lattice, n, d, rho_p, periodic=(0, 0, 0), rho0=1.0, k_soft=1e-3,
                 contact="soft", n_sub=1, two_way=True):
        self.lattice = lattice
        self.D = 2 if lattice == 9 else 3
        self.n = tuple(int(v) for v in n)
        self.periodic = tuple(int(v) for v in periodic)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.e, self.w, self.opp = lattice_tables(lattice)
        self.Q = self.e.shape[0]
        self.rho0 = float(rho0)
        self.k_soft = float(k_soft)
        assert contact in ("soft", "none")
        self.contact = contact
        self.n_sub = int(n_sub)
        self.two_way = bool(two_way)
        self.d = torch.as_tensor(d, dtype=torch.float64)
        self.rho_p = torch.as_tensor(rho_p, dtype=torch.float64)
        if self.D == 2:
            self.m = self.rho_p * math.pi * self.d ** 2 / 4.0      # disk of unit depth
        else:
            self.m = self.rho_p * math.pi * self.d ** 3 / 6.0
        self.A = math.pi * self.d ** 2 / 4.0
        self.src = self._pull_map()

    # --- lattice ------------------------------------------------------------
    def _pull_map(self):
        """src such that f_new.flatten() = f_star.flatten()[src]: the inverse
        of push streaming with halfway bounce-back (a permutation)."""
        nx, ny, nz = self.n
        idx = torch.arange(self.N)
        x = idx % nx
        y = (idx // nx) % ny
        z = idx // (nx * ny)
        dest = torch.empty(self.Q, self.N, dtype=torch.long)
        for q in range(self.Q):
            c = [int(v) for v in self.e[q]]
            tx, ty, tz = x + c[0], y + c[1], z + c[2]
            inside = torch.ones(self.N, dtype=torch.bool)
            coords = []
            for t, na, per in ((tx, nx, self.periodic[0]), (ty, ny, self.periodic[1]), (tz, nz, self.periodic[2])):
                if per:
                    t = t % na
                else:
                    inside &= (t >= 0) & (t < na)
                coords.append(t)
            tgt = (coords[2] * ny + coords[1]) * nx + coords[0]
            dest[q] = torch.where(inside, q * self.N + tgt, self.opp[q] * self.N + idx)
        src = torch.empty(self.Q * self.N, dtype=torch.long)
        src[dest.flatten()] = torch.arange(self.Q * self.N)
        return src

    def moments(self, f):
        rho = f.sum(0)
        j = self.e[:, : self.D].T @ f
        return rho, j

    def collide_stream(self, f, rho, j, F, tau):
        e = self.e[:, : self.D]
        u = (j + 0.5 * F) / rho
        eu = e @ u                                   # (Q, N)
        uu = (u * u).sum(0)
        feq = self.w[:, None] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu)
        eF = e @ F
        uF = (u * F).sum(0)
        S = (1.0 - 0.5 / tau) * self.w[:, None] * (3.0 * (eF - uF) + 9.0 * eu * eF)
        fs = f - (f - feq) / tau + S
        return fs.flatten()[self.src].reshape(self.Q, self.N)

    # --- delta kernel -------------------------------------------------------
    def stencil(self, X):
        """Node indices (np, 4^D) and weights (np, 4^D) of every particle,
        with per-axis renormalisation over in-domain nodes."""
        npart = X.shape[1]
        idx = torch.zeros(npart, 1, dtype=torch.long)
        W = torch.ones(npart, 1, dtype=torch.float64)
        stride = 1
        for a in range(self.D):
            b = torch.floor(X[a].detach() - 0.5).long() - 1
            k = torch.arange(4)
            i = b[:, None] + k[None, :]                       # (np, 4)
            r = X[a][:, None] - (i.to(torch.float64) + 0.5)
            phi = 0.25 * (1.0 + torch.cos(0.5 * math.pi * r))
            if self.periodic[a]:
                i = i % self.n[a]
            else:
                ok = (i >= 0) & (i < self.n[a])
                phi = torch.where(ok, phi, torch.zeros_like(phi))
                phi = phi / phi.sum(1, keepdim=True)
                i = i.clamp(0, self.n[a] - 1)
            idx = (idx[:, :, None] + stride * i[:, None, :]).reshape(npart, -1)
            W = (W[:, :, None] * phi[:, None, :]).reshape(npart, -1)
            stride *= self.n[a]
        return idx, W

    # --- particles ----------------------------------------------------------
    def contact_force(self, X):
        D = self.D
        F = torch.zeros_like(X)
        if self.contact == "none":
            return F
        npart = X.shape[1]
        if npart > 1:
            r = X[:, :, None] - X[:, None, :]                 # r[:, p, q] = X_p - X_q
            eye = torch.eye(npart, dtype=torch.bool)
            dist2 = (r * r).sum(0)
            dist = torch.sqrt(torch.where(eye, torch.ones_like(dist2), dist2))
            rc = 0.5 * (self.d[:, None] + self.d[None, :])
            s = 1.0 - dist / rc
            on = (~eye) & (dist < rc)
            mag = torch.where(on, self.k_soft * s * s / dist, torch.zeros_like(s))
            F = F + (mag[None] * r).sum(2)
        for a in range(D):
            if self.periodic[a]:
                continue
            rc = 0.5 * self.d
            for side, nrm in ((0, 1.0), (1, -1.0)):
                dist = X[a] if side == 0 else self.n[a] - X[a]
                s = 1.0 - dist / rc
                fa = torch.where(dist < rc, self.k_soft * s * s * nrm, torch.zeros_like(s))
                F = F.index_add(0, torch.tensor([a]), fa[None])
        return F

    def step(self, f, X, U, tau, gvec):
        """One coupled step; returns (f', X', U').  gvec: gravity (D,)."""
        rho, j = self.moments(f)
        X, U, F = self.particle_part(rho, j, X, U, gvec)
        f = self.collide_stream(f, rho, j, F, tau)
        return f, X, U

    def particle_part(self, rho, j, X, U, gvec):
        """The particle side of one step from the node moments (rho, j) of
        the populations: interpolation, the sub-stepped update and the
        spread force field.  Returns (X', U', F)."""
        idx, W = self.stencil(X)
        rho_i = (W * rho[idx]).sum(1)
        j_i = (W[None] * j[:, idx]).sum(2)
        h = 1.0 / self.n_sub
        bw = (1.0 - self.rho0 / self.rho_p)
        gsum = torch.zeros_like(U)
        for _ in range(self.n_sub):
            g = 2.0 * (rho_i * U - j_i)
            Fc = self.contact_force(X)
            acc = (-self.A * g + Fc) / self.m + bw * gvec[:, None]
            U = U + h * acc
            X = X + h * U
            gsum = gsum + g
        gbar = gsum / self.n_sub
        F = torch.zeros(self.D, self.N, dtype=torch.float64)
        if self.two_way:
            coef = self.A * gbar                                # (D, np)
            contrib = coef[:, :, None] * W[None]                # (D, np, 4^D)
            F = F.index_add(1, idx.flatten(), contrib.reshape(self.D, -1))
        return X, U, F

    def rest(self, rho=1.0):
        return (self.w[:, None] * rho).repeat(1, self.N)

    def rollout(self, X0, U0, tau, gvec, steps, f0=None):
        f = self.rest() if f0 is None else f0
        X, U = X0, U0
        for _ in range(steps):
            f, X, U = self.step(f, X, U, tau, gvec)
        return f, X, U
