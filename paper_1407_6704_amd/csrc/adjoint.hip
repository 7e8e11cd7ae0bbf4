// adjoint.hip -- reverse-mode derivative (adjoint) of the coupled step, for
// gradients of an objective of the final particle state with respect to the
// relaxation time, the gravity vector and the initial particle velocities and
// positions.
//
// Scope: one DEM sub-step per lattice step (the explicit update of Eq. demgov
// with the momentum-exchange drag of Eq. lbm7-lbm8 and lbm13), soft or no
// contact, bins equal to the dual cells.  The forward is re-run from
// checkpoints one segment at a time (the forward is bitwise reproducible, so
// the re-run is the recorded trajectory).  One reverse step goes back through
//   collision and streaming (Eq. lbm2, lbm9, bounce-back)  k_adj_collide, k_adj_assemble
//   spreading (Eq. lbm10-lbm11)                           k_adj_particles (gather of F-bar)
//   particle update and momentum exchange                 k_adj_particles
//   interpolation (Eq. lbm11-lbm12)                       k_adj_particles, then the adjoint
//                                                         moments are spread with k_spread_csr
//   moments                                               k_adj_assemble
// Notation: a-bar is the adjoint of a quantity.  All arithmetic is FP32; the
// parameter gradients are summed per block in FP32 and across blocks and
// steps in double-float (no FP64).
#include <algorithm>
#include <cmath>

#include "pibm_internal.h"

namespace pibm {

// Adjoint of push streaming with halfway bounce-back: the population that
// left node r in direction q arrived at r + e_q (or, across a wall, in the
// opposite direction at r); its adjoint is read from there.
template <int Q>
__device__ __forceinline__ float adj_pull(const float* __restrict__ abar, long long r, int q, int x, int y, int z,
                                          const Grid& g) {
    using L = Lattice<Q>;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const long long N = g.N, sx = 1, sy = nx, sz = (long long)nx * ny;
    const int ex = L::ex(q), ey = L::ey(q), ez = L::ez(q);
    long long src = r;
    bool out = false;
    if (ex > 0) { if (x == nx - 1) { if (g.periodic[0]) src -= (nx - 1) * sx; else out = true; } else src += sx; }
    if (ex < 0) { if (x == 0) { if (g.periodic[0]) src += (nx - 1) * sx; else out = true; } else src -= sx; }
    if (ey > 0) { if (y == ny - 1) { if (g.periodic[1]) src -= (ny - 1) * sy; else out = true; } else src += sy; }
    if (ey < 0) { if (y == 0) { if (g.periodic[1]) src += (ny - 1) * sy; else out = true; } else src -= sy; }
    if (ez > 0) { if (z == nz - 1) { if (g.periodic[2]) src -= (long long)(nz - 1) * sz; else out = true; } else src += sz; }
    if (ez < 0) { if (z == 0) { if (g.periodic[2]) src += (long long)(nz - 1) * sz; else out = true; } else src -= sz; }
    return out ? abar[(long long)L::opp(q) * N + r] : abar[(long long)q * N + src];
}

__device__ __forceinline__ void block_sum256(float* red, int t) {
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) red[t] += red[t + st];
        __syncthreads();
    }
}

// Reverse of the collision at every node.  In:  abar = adjoint of the
// populations after streaming; f_t and the force field F_t of the forward
// step.  Out: the moments of f_t (for the interpolation adjoint), F-bar, the
// collision's share of the moment adjoints (rho-bar, j-bar) and one partial
// sum of d/dtau per block.
//   f*_q = f_q - (f_q - feq_q(rho, u)) / tau + (1 - 1/(2 tau)) S_q(u, F),
//   u = (j + F/2) / rho;  d f*_q / d tau = (f_q - feq_q) / tau^2 + S_q / (2 tau^2)
template <int Q, class S>
__global__ __launch_bounds__(256) void k_adj_collide(const float* __restrict__ abar,
                                                     const typename S::T* __restrict__ ft,
                                                     const float* __restrict__ Ft, int hasF, float ffx, float ffy,
                                                     float ffz, Grid g, float tau, S st, float4* __restrict__ mom,
                                                     float* __restrict__ Fbar, float4* __restrict__ Mc,
                                                     float* __restrict__ tpart) {
    using L = Lattice<Q>;
    __shared__ float red[256];
    const long long N = g.N;
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    float tsum = 0.f;
    if (r < N) {
        const int nx = g.n[0], ny = g.n[1];
        const int x = (int)(r % nx);
        const long long tt = r / nx;
        const int y = (int)(tt % ny);
        const int z = (int)(tt / ny);
        float h[Q];
#pragma unroll
        for (int q = 0; q < Q; q++) h[q] = st.load(ft + (long long)q * N + r);
        float dr = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
        for (int q = 0; q < Q; q++) {
            dr += h[q];
            if (L::ex(q)) jx += L::ex(q) * h[q];
            if (L::ey(q)) jy += L::ey(q) * h[q];
            if (L::ez(q)) jz += L::ez(q) * h[q];
        }
        float Fx = ffx, Fy = ffy, Fz = ffz;
        if (hasF) {
            Fx += Ft[r];
            Fy += Ft[N + r];
            if (L::D == 3) Fz += Ft[2 * N + r];
        }
        const float rho = 1.0f + dr;
        const float ir = 1.0f / rho;
        const float ux = (jx + 0.5f * Fx) * ir, uy = (jy + 0.5f * Fy) * ir, uz = (jz + 0.5f * Fz) * ir;
        const float uu = ux * ux + uy * uy + uz * uz;
        const float uF = ux * Fx + uy * Fy + uz * Fz;
        const float it = 1.0f / tau, fpref = 1.0f - 0.5f * it;
        float rb = 0.f, ubx = 0.f, uby = 0.f, ubz = 0.f, fbx = 0.f, fby = 0.f, fbz = 0.f;
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const float a = adj_pull<Q>(abar, r, q, x, y, z, g);
            const float ex = (float)L::ex(q), ey = (float)L::ey(q), ez = (float)L::ez(q), w = L::w(q);
            const float eu = ex * ux + ey * uy + ez * uz;
            const float eF = ex * Fx + ey * Fy + ez * Fz;
            const float poly = 3.0f * eu + 4.5f * eu * eu - 1.5f * uu;
            const float heq = w * (dr + rho * poly);
            const float sraw = w * (3.0f * (eF - uF) + 9.0f * eu * eF);
            tsum += a * (it * it) * ((h[q] - heq) + 0.5f * sraw);
            rb += a * it * w * (1.0f + poly);
            // d feq / d u_b = 3 w rho (e_b (1 + 3 e.u) - u_b);  d S / d u_b = w (9 e_b e.F - 3 F_b)
            const float cf = a * it * 3.0f * w * rho, cs = a * fpref * w;
            const float k1 = 1.0f + 3.0f * eu;
            ubx += cf * (ex * k1 - ux) + cs * (9.0f * ex * eF - 3.0f * Fx);
            uby += cf * (ey * k1 - uy) + cs * (9.0f * ey * eF - 3.0f * Fy);
            ubz += cf * (ez * k1 - uz) + cs * (9.0f * ez * eF - 3.0f * Fz);
            // d S / d F_b = w (3 (e_b - u_b) + 9 e.u e_b)
            fbx += cs * (3.0f * (ex - ux) + 9.0f * eu * ex);
            fby += cs * (3.0f * (ey - uy) + 9.0f * eu * ey);
            fbz += cs * (3.0f * (ez - uz) + 9.0f * eu * ez);
        }
        // u = (j + F/2) / rho
        rb -= (ubx * ux + uby * uy + ubz * uz) * ir;
        fbx += 0.5f * ubx * ir;
        fby += 0.5f * uby * ir;
        fbz += 0.5f * ubz * ir;
        mom[r] = make_float4(dr, jx, jy, jz);
        Fbar[r] = fbx;
        Fbar[N + r] = fby;
        if (L::D == 3) Fbar[2 * N + r] = fbz;
        Mc[r] = make_float4(rb, ubx * ir, uby * ir, ubz * ir);
    }
    red[threadIdx.x] = tsum;
    block_sum256(red, threadIdx.x);
    if (threadIdx.x == 0) tpart[blockIdx.x] = red[0];
}

// The adjoint of the populations before the step: the direct term of the
// collision plus the moment adjoints (collision share Mc and the spread
// interpolation share Sf = (rho-bar, j-bar) fields).
template <int Q>
__global__ __launch_bounds__(256) void k_adj_assemble(const float* __restrict__ abar, const float4* __restrict__ Mc,
                                                      const float* __restrict__ Sf, int hasS, Grid g, float tau,
                                                      float* __restrict__ abar_out) {
    using L = Lattice<Q>;
    const long long N = g.N;
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= N) return;
    const int nx = g.n[0], ny = g.n[1];
    const int x = (int)(r % nx);
    const long long tt = r / nx;
    const int y = (int)(tt % ny);
    const int z = (int)(tt / ny);
    const float4 m = Mc[r];
    float rb = m.x, jbx = m.y, jby = m.z, jbz = m.w;
    if (hasS) {
        rb += Sf[r];
        jbx += Sf[N + r];
        jby += Sf[2 * N + r];
        if (L::D == 3) jbz += Sf[3 * N + r];
    }
    const float keep = 1.0f - 1.0f / tau;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const float a = adj_pull<Q>(abar, r, q, x, y, z, g);
        abar_out[(long long)q * N + r] = keep * a + rb + L::ex(q) * jbx + L::ey(q) * jby + L::ez(q) * jbz;
    }
}

// Weights of one axis (as in the forward: phi_k = delta(X - (i + 1/2)) on the
// four nodes i = floor(X - 1/2) - 1 + k, zero outside, renormalised) and
// their derivatives d phi_k / d X.  With fr the fractional dual offset the
// raw weights are (1 - sin, 1 + cos, 1 + sin, 1 - cos)(pi fr / 2) / 4, whose
// derivatives are (-cos, -sin, cos, sin)(pi fr / 2) pi / 8.
__device__ __forceinline__ void axis_weights_grad(float xh, float xl, int n, int& base, float* phi, float* dphi) {
    const int c = dual_cell(xh, xl);
    const float fr = dual_frac(xh, xl, c);
    float sv, cv;
    sincospif(0.5f * fr, &sv, &cv);
    base = c - 1;
    float w[4] = {0.25f * (1.0f - sv), 0.25f * (1.0f + cv), 0.25f * (1.0f + sv), 0.25f * (1.0f - cv)};
    const float k = 0.125f * PI_F;
    float dw[4] = {-k * cv, -k * sv, k * cv, k * sv};
    float S = 0.f, dS = 0.f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (base + i < 0 || base + i >= n) w[i] = dw[i] = 0.f;
        S += w[i];
        dS += dw[i];
    }
    const float inv = S > 0.f ? 1.0f / S : 0.f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        phi[i] = w[i] * inv;
        dphi[i] = (dw[i] - phi[i] * dS) * inv;
    }
}

// Soft repulsion f(s) = k_s (1 - s/r_c)^2 and its derivative.
__device__ __forceinline__ void soft_mag(float ks, float s, float rc, float& f, float& df) {
    const float t = 1.0f - s / rc;
    f = ks * t * t;
    df = -2.0f * ks * t / rc;
}

// Reverse of the particle side of one step, one thread per particle (sorted
// order of the step's cell list).  The forward, with h = 1:
//   g  = 2 (rho_i U - j_i),   Fc = contacts(X),
//   U' = U + (-A g + Fc) / m + (1 - rho0/rho_p) gvec,   X' = X + U',
//   F(r) += A g W(r; X),   rho_i = sum W rho,   j_i = sum W j.
// In: the adjoints of X', U' (id order; X-bar as double-float), the moments
// and F-bar fields.  Out: the adjoints of X, U (id order), the interpolation
// adjoints (rho_i-bar, j_i-bar) with their weights for spreading, and one
// partial sum of d/dgvec per block.
template <int D>
__global__ __launch_bounds__(256) void k_adj_particles(PState A, int np, Grid g, PCfg c, int two_way,
                                                       const uint32_t* __restrict__ start,
                                                       const uint32_t* __restrict__ keys_sorted,
                                                       const float4* __restrict__ mom, const float* __restrict__ Fbar,
                                                       const float* __restrict__ xbh, const float* __restrict__ xbl,
                                                       const float* __restrict__ ub, float* __restrict__ xbh_o,
                                                       float* __restrict__ xbl_o, float* __restrict__ ub_o,
                                                       float* __restrict__ coefS, float* __restrict__ srec,
                                                       short4* __restrict__ wbase, float* __restrict__ gpart) {
    __shared__ float red[3][256];
    const int s = blockIdx.x * 256 + threadIdx.x;
    float gacc[3] = {0.f, 0.f, 0.f};
    if (s < np) {
        const int id = A.id[s];
        const float d = A.d[s], rp = A.rp[s];
        const float m = particle_mass(D, d, rp);
        const float Ap = 0.25f * PI_F * d * d;
        const float bw = 1.0f - c.rho0 / rp;
        int base[3] = {0, 0, 0};
        float phi[3][4], dphi[3][4], U[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (a < D) {
                axis_weights_grad(A.xh[a][s], A.xl[a][s], g.n[a], base[a], phi[a], dphi[a]);
                U[a] = A.u[a][s];
            } else {
                phi[a][0] = 1.f;
                phi[a][1] = phi[a][2] = phi[a][3] = 0.f;
                dphi[a][0] = dphi[a][1] = dphi[a][2] = dphi[a][3] = 0.f;
            }
        }
        // gather the moments and F-bar with the weights and their derivatives
        float dri = 0.f, ji[3] = {0.f, 0.f, 0.f}, Phi[3] = {0.f, 0.f, 0.f};
        float ddri[3] = {0.f, 0.f, 0.f}, dji[3][3] = {}, dPhi[3][3] = {};
#pragma unroll
        for (int kz = 0; kz < (D == 3 ? 4 : 1); kz++)
#pragma unroll
            for (int ky = 0; ky < 4; ky++)
#pragma unroll
                for (int kx = 0; kx < 4; kx++) {
                    const int x = base[0] + kx, y = base[1] + ky, z = (D == 3) ? base[2] + kz : 0;
                    if (x < 0 || x >= g.n[0] || y < 0 || y >= g.n[1] || z < 0 || z >= g.n[2]) continue;
                    const long long node = ((long long)z * g.n[1] + y) * g.n[0] + x;
                    const float W = phi[0][kx] * phi[1][ky] * phi[2][kz];
                    const float dW[3] = {dphi[0][kx] * phi[1][ky] * phi[2][kz], phi[0][kx] * dphi[1][ky] * phi[2][kz],
                                         phi[0][kx] * phi[1][ky] * dphi[2][kz]};
                    const float4 mm = mom[node];
                    const float mj[3] = {mm.y, mm.z, mm.w};
                    float fb[3] = {0.f, 0.f, 0.f};
                    if (two_way)
#pragma unroll
                        for (int b = 0; b < D; b++) fb[b] = Fbar[(long long)b * g.N + node];
                    dri += W * mm.x;
#pragma unroll
                    for (int b = 0; b < D; b++) {
                        ji[b] += W * mj[b];
                        Phi[b] += W * fb[b];
                    }
#pragma unroll
                    for (int a = 0; a < D; a++) {
                        ddri[a] += dW[a] * mm.x;
#pragma unroll
                        for (int b = 0; b < D; b++) {
                            dji[a][b] += dW[a] * mj[b];
                            dPhi[a][b] += dW[a] * fb[b];
                        }
                    }
                }
        const float ri = 1.0f + dri;
        float gg[3], Ut[3], gb[3], Fcb[3];
#pragma unroll
        for (int b = 0; b < D; b++) {
            gg[b] = 2.0f * (ri * U[b] - ji[b]);
            Ut[b] = ub[(long long)b * np + id] + (xbh[(long long)b * np + id] + xbl[(long long)b * np + id]);
            gb[b] = (two_way ? Ap * Phi[b] : 0.f) - (Ap / m) * Ut[b];
            Fcb[b] = Ut[b] / m;
            gacc[b] = bw * Ut[b];
        }
        float rib = 0.f;
#pragma unroll
        for (int b = 0; b < D; b++) rib += 2.0f * U[b] * gb[b];
        float dX[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < D; a++) {
            float v = rib * ddri[a];
#pragma unroll
            for (int b = 0; b < D; b++) {
                v += (-2.0f * gb[b]) * dji[a][b];
                if (two_way) v += Ap * gg[b] * dPhi[a][b];
            }
            dX[a] = v;
        }
        if (c.contact == PIBM_CONTACT_SOFT) {
            // pairs: d Fc_p / d X_p = J_pq, d Fc_q / d X_p = -J_pq (central force)
            const uint32_t key = keys_sorted[s];
            int bc[3];
            bc[0] = (int)(key % (uint32_t)c.nb[0]);
            bc[1] = (int)((key / (uint32_t)c.nb[0]) % (uint32_t)c.nb[1]);
            bc[2] = (int)(key / ((uint32_t)c.nb[0] * (uint32_t)c.nb[1]));
            const int H = c.H;
            const int zl = (D == 3) ? max(bc[2] - H, 0) : 0, zh = (D == 3) ? min(bc[2] + H, c.nb[2] - 1) : 0;
            for (int bz = zl; bz <= zh; bz++)
                for (int by = max(bc[1] - H, 0); by <= min(bc[1] + H, c.nb[1] - 1); by++) {
                    const int bxl = max(bc[0] - H, 0), bxh = min(bc[0] + H, c.nb[0] - 1);
                    const uint32_t row = (uint32_t)(((long long)bz * c.nb[1] + by) * c.nb[0]);
                    const uint32_t t0 = start[row + bxl], t1 = start[row + bxh + 1];
                    for (uint32_t t = t0; t < t1; t++) {
                        if ((int)t == s) continue;
                        float rv[3] = {0.f, 0.f, 0.f}, r2 = 0.f;
#pragma unroll
                        for (int a = 0; a < D; a++) {
                            rv[a] = (A.xh[a][s] - A.xh[a][t]) + (A.xl[a][s] - A.xl[a][t]);
                            r2 += rv[a] * rv[a];
                        }
                        const float rc = 0.5f * (d + A.d[t]);
                        if (!(r2 < rc * rc)) continue;
                        const float dist = sqrtf(r2);
                        float f, df;
                        soft_mag(c.ks, dist, rc, f, df);
                        const int idq = A.id[t];
                        const float mq = particle_mass(D, A.d[t], A.rp[t]);
                        float diff[3], nv[3];
#pragma unroll
                        for (int b = 0; b < D; b++) {
                            const float utq = ub[(long long)b * np + idq] +
                                              (xbh[(long long)b * np + idq] + xbl[(long long)b * np + idq]);
                            diff[b] = Fcb[b] - utq / mq;
                            nv[b] = rv[b] / dist;
                        }
                        float nd = 0.f;
#pragma unroll
                        for (int b = 0; b < D; b++) nd += nv[b] * diff[b];
                        const float fo = f / dist;
                        // J = df n n^T + (f / s) (I - n n^T)
#pragma unroll
                        for (int a = 0; a < D; a++) dX[a] += (df - fo) * nv[a] * nd + fo * diff[a];
                    }
                }
            // walls at 0 and n_a: d Fw_a / d X_a = f'(distance) on both sides
#pragma unroll
            for (int a = 0; a < D; a++) {
                const float xa = A.xh[a][s] + A.xl[a][s];
                const float rcw = 0.5f * d;
                float f, df;
                if (xa < rcw) {
                    soft_mag(c.ks, xa, rcw, f, df);
                    dX[a] += df * Fcb[a];
                }
                const float up = (float)g.n[a] - xa;
                if (up < rcw) {
                    soft_mag(c.ks, up, rcw, f, df);
                    dX[a] += df * Fcb[a];
                }
            }
        }
#pragma unroll
        for (int b = 0; b < D; b++) {
            float hi = xbh[(long long)b * np + id], lo = xbl[(long long)b * np + id];
            df_add(hi, lo, dX[b]);
            xbh_o[(long long)b * np + id] = hi;
            xbl_o[(long long)b * np + id] = lo;
            ub_o[(long long)b * np + id] = Ut[b] + 2.0f * ri * gb[b];
            coefS[(long long)(1 + b) * np + s] = -2.0f * gb[b];
        }
        coefS[s] = rib;
#pragma unroll
        for (int a = 0; a < D; a++)
#pragma unroll
            for (int k = 0; k < 4; k++) srec[(long long)s * SRec<D>::STRIDE + 4 * a + k] = phi[a][k];
        srec[(long long)s * SRec<D>::STRIDE + SRec<D>::BASE] = __int_as_float(base[0]);
        wbase[s] = make_short4((short)base[0], (short)base[1], (short)base[2], 0);
    }
#pragma unroll
    for (int b = 0; b < 3; b++) red[b][threadIdx.x] = gacc[b];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
#pragma unroll
            for (int b = 0; b < 3; b++) red[b][threadIdx.x] += red[b][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int b = 0; b < 3; b++) gpart[blockIdx.x * 3 + b] = red[b][0];
}

// (ahi, alo) += (bhi, blo), double-float.
__device__ __forceinline__ void df_add_df(float& ahi, float& alo, float bhi, float blo) {
#pragma clang fp contract(off)
    float s, e;
    two_sum(ahi, bhi, s, e);
    e += alo + blo;
    fast_two_sum(s, e, ahi, alo);
}

// Sum the per-block partials of one reverse step in a fixed order and add
// them to the running double-float totals acc = [tau, g_x, g_y, g_z] x (hi, lo).
__global__ __launch_bounds__(256) void k_adj_accumulate(const float* __restrict__ tpart, int ntb,
                                                        const float* __restrict__ gpart, int ngb,
                                                        float* __restrict__ acc) {
    __shared__ float sh[4][256], sl[4][256];
    const int t = threadIdx.x;
    float hi[4] = {0.f, 0.f, 0.f, 0.f}, lo[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i = t; i < ntb; i += 256) df_add(hi[0], lo[0], tpart[i]);
    for (int i = t; i < ngb; i += 256)
#pragma unroll
        for (int b = 0; b < 3; b++) df_add(hi[1 + b], lo[1 + b], gpart[i * 3 + b]);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        sh[k][t] = hi[k];
        sl[k][t] = lo[k];
    }
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st)
#pragma unroll
            for (int k = 0; k < 4; k++) df_add_df(sh[k][t], sl[k][t], sh[k][t + st], sl[k][t + st]);
        __syncthreads();
    }
    if (t < 4) {
        float h = acc[2 * t], l = acc[2 * t + 1];
        df_add_df(h, l, sh[t][0], sl[t][0]);
        acc[2 * t] = h;
        acc[2 * t + 1] = l;
    }
}

__global__ void k_fill_f32(float* __restrict__ p, long long n, float v) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// Particle state in sorted order -> id order: [xh D][xl D][u D] x np.
__global__ __launch_bounds__(256) void k_save_state(PState A, int np, int D, float* __restrict__ out) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= np) return;
    const int id = A.id[s];
    for (int a = 0; a < D; a++) {
        out[(long long)a * np + id] = A.xh[a][s];
        out[(long long)(D + a) * np + id] = A.xl[a][s];
        out[(long long)(2 * D + a) * np + id] = A.u[a][s];
    }
}

// Diameters and densities in id order.
__global__ __launch_bounds__(256) void k_save_const(PState A, int np, float* __restrict__ d, float* __restrict__ rp) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= np) return;
    const int id = A.id[s];
    d[id] = A.d[s];
    rp[id] = A.rp[s];
}

// Id-order state -> PState A in id order (the next sort orders it).
__global__ __launch_bounds__(256) void k_load_state(const float* __restrict__ in, const float* __restrict__ d,
                                                    const float* __restrict__ rp, int np, int D, PState A) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= np) return;
    for (int a = 0; a < D; a++) {
        A.xh[a][i] = in[(long long)a * np + i];
        A.xl[a][i] = in[(long long)(D + a) * np + i];
        A.u[a][i] = in[(long long)(2 * D + a) * np + i];
    }
    A.d[i] = d[i];
    A.rp[i] = rp[i];
    A.id[i] = i;
}

// out = hi + lo (the position adjoint as one FP32 value)
__global__ void k_df_collapse(const float* __restrict__ hi, const float* __restrict__ lo, float* __restrict__ out,
                              long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = hi[i] + lo[i];
}

// Node fields in planes (comps planes of n) to the float4 moments layout
// read by the interpolation (components past comps are zero).
__global__ __launch_bounds__(256) void k_pack_mom(const float* __restrict__ in, int comps, long long n,
                                                  float4* __restrict__ out) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < comps && k < 4; k++) v[k] = in[(long long)k * n + i];
    out[i] = make_float4(v[0], v[1], v[2], v[3]);
}

static inline unsigned blocks256(long long n) { return (unsigned)std::max<long long>((n + 255) / 256, 1); }

// ---------------------------------------------------------------------------
// launchers (called from runtime.hip)
// ---------------------------------------------------------------------------
void adj_fill(float* p, long long n, float v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks256(n)), dim3(256), 0, s, p, n, v);
}

void adj_save_state(int D, const PBuf& b, int np, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_save_state, dim3(blocks256(np)), dim3(256), 0, s, b.A, np, D, out);
}

void adj_save_const(const PBuf& b, int np, float* d, float* rp, hipStream_t s) {
    hipLaunchKernelGGL(k_save_const, dim3(blocks256(np)), dim3(256), 0, s, b.A, np, d, rp);
}

void adj_load_state(int D, PBuf& b, int np, const float* in, const float* d, const float* rp, hipStream_t s) {
    hipLaunchKernelGGL(k_load_state, dim3(blocks256(np)), dim3(256), 0, s, in, d, rp, np, D, b.A);
}

void adj_df_collapse(const float* hi, const float* lo, float* out, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_df_collapse, dim3(blocks256(n)), dim3(256), 0, s, hi, lo, out, n);
}

int adj_collide_blocks(long long N) { return (int)blocks256(N); }
int adj_particle_blocks(int np) { return (int)blocks256(np); }

template <int Q, class S>
static void collide_launch(const float* abar, const void* ft, const float* Ft, int hasF, const float* ff,
                           const Grid& g, float tau, S st, float4* mom, float* Fbar, float4* Mc, float* tpart,
                           hipStream_t s) {
    hipLaunchKernelGGL((k_adj_collide<Q, S>), dim3(blocks256(g.N)), dim3(256), 0, s, abar,
                       (const typename S::T*)ft, Ft, hasF, ff[0], ff[1], ff[2], g, tau, st, mom, Fbar, Mc, tpart);
}

void adj_collide(int Q, int fp16, int sl2, const float* abar, const void* ft, const float* Ft, int hasF,
                 const float* ff, const Grid& g, float tau, float4* mom, float* Fbar, float4* Mc, float* tpart,
                 hipStream_t s) {
    const float sc = std::ldexp(1.0f, sl2), isc = std::ldexp(1.0f, -sl2);
    if (Q == 19) {
        if (fp16) collide_launch<19>(abar, ft, Ft, hasF, ff, g, tau, StoreF16{sc, isc}, mom, Fbar, Mc, tpart, s);
        else collide_launch<19>(abar, ft, Ft, hasF, ff, g, tau, StoreF32{1.f, 1.f}, mom, Fbar, Mc, tpart, s);
    } else if (Q == 15) {
        if (fp16) collide_launch<15>(abar, ft, Ft, hasF, ff, g, tau, StoreF16{sc, isc}, mom, Fbar, Mc, tpart, s);
        else collide_launch<15>(abar, ft, Ft, hasF, ff, g, tau, StoreF32{1.f, 1.f}, mom, Fbar, Mc, tpart, s);
    } else {
        if (fp16) collide_launch<9>(abar, ft, Ft, hasF, ff, g, tau, StoreF16{sc, isc}, mom, Fbar, Mc, tpart, s);
        else collide_launch<9>(abar, ft, Ft, hasF, ff, g, tau, StoreF32{1.f, 1.f}, mom, Fbar, Mc, tpart, s);
    }
}

void adj_assemble(int Q, const float* abar, const float4* Mc, const float* Sf, int hasS, const Grid& g, float tau,
                  float* abar_out, hipStream_t s) {
    if (Q == 19)
        hipLaunchKernelGGL(k_adj_assemble<19>, dim3(blocks256(g.N)), dim3(256), 0, s, abar, Mc, Sf, hasS, g, tau,
                           abar_out);
    else if (Q == 15)
        hipLaunchKernelGGL(k_adj_assemble<15>, dim3(blocks256(g.N)), dim3(256), 0, s, abar, Mc, Sf, hasS, g, tau,
                           abar_out);
    else
        hipLaunchKernelGGL(k_adj_assemble<9>, dim3(blocks256(g.N)), dim3(256), 0, s, abar, Mc, Sf, hasS, g, tau,
                           abar_out);
}

void adj_particles(int D, PBuf& b, int np, const Grid& g, const PCfg& c, int two_way, const float4* mom,
                   const float* Fbar, const float* xbh, const float* xbl, const float* ub, float* xbh_o,
                   float* xbl_o, float* ub_o, float* coefS, float* gpart, hipStream_t s) {
    if (D == 3)
        hipLaunchKernelGGL(k_adj_particles<3>, dim3(blocks256(np)), dim3(256), 0, s, b.A, np, g, c, two_way, b.start,
                           b.keys_sorted, mom, Fbar, xbh, xbl, ub, xbh_o, xbl_o, ub_o, coefS, b.srec, b.wbase, gpart);
    else
        hipLaunchKernelGGL(k_adj_particles<2>, dim3(blocks256(np)), dim3(256), 0, s, b.A, np, g, c, two_way, b.start,
                           b.keys_sorted, mom, Fbar, xbh, xbl, ub, xbh_o, xbl_o, ub_o, coefS, b.srec, b.wbase, gpart);
}

void adj_accumulate(const float* tpart, int ntb, const float* gpart, int ngb, float* acc, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_accumulate, dim3(1), dim3(256), 0, s, tpart, ntb, gpart, ngb, acc);
}

void adj_pack_mom(const float* in, int comps, long long n, float4* out, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_mom, dim3(blocks256(n)), dim3(256), 0, s, in, comps, n, out);
}

}  // namespace pibm
