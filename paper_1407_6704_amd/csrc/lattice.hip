// lattice.hip -- lattice-Boltzmann kernels of the coupled step (gfx950).
//
//  k_moments  : density deviation and momentum of the stored populations
//               (moment definitions of Sec. 2.1), one float4 per node; in
//               the coupled step only on the node rows that some particle's
//               4-node gather stencil reaches (the others are never read).
//  k_collide  : BGK collision, Eq. lbm2, towards the equilibrium of Eq. lbm3,
//               with the forcing term of Eq. lbm9 and the half-force velocity
//               rho u = sum f e + F/2 (end of Sec. 2.2); the post-collision
//               value is pushed to its neighbour, or reflected into the
//               opposite direction at the same node when the link crosses a
//               wall (halfway bounce-back; walls at 0 and n).
//
// Both are streaming node loops bound by HBM bandwidth: structure of arrays
// f[q][node], one node per lane, 64 consecutive x-nodes per wave, so every
// population load is one contiguous 256 B (FP32) or 128 B (FP16) segment.
// All arithmetic is FP32 on deviations h = f - w, which keeps the small
// velocities of sedimentation (1e-6 .. 1e-4) resolved; FP64 appears only in
// the conservation reductions.
#include "pibm_internal.h"

namespace pibm {

// Node y of an axis is a gather node of the particles whose dual cell
// c' = floor(X - 1/2) + 1 lies in [y - 1, y + 2] (stencil c' - 2 .. c' + 1).
// A row of nodes (y, z) along x is needed when the bins of those cells hold
// a particle: 16 bin rows (4 in 2D), each a contiguous run of the sorted
// order.  A workgroup whose nodes span at most ROWS_MAX rows decides for
// all of them together and skips when none is needed; otherwise it computes.
constexpr int ROWS_MAX = 4;
__device__ __forceinline__ bool rows_needed(const RowMask& m, long long r0, long long r1) {
    const long long R0 = r0 / m.n[0], R1 = r1 / m.n[0];
    if (R1 - R0 >= ROWS_MAX) return true;
    uint32_t cnt = 0;
    const int t = threadIdx.x;
    if (t < 16 * (int)(R1 - R0 + 1)) {
        const long long R = R0 + t / 16;
        const int y = (int)(R % m.n[1]), z = (int)(R / m.n[1]);
        const int cy = y - 1 + (t & 3), cz = z - 1 + ((t >> 2) & 3);
        if (cy >= 0 && cz >= 0) {
            const int by = cy >> m.L, bz = cz >> m.L;
            if (by < m.nb[1] && bz < m.nb[2]) {
                const long long row = ((long long)bz * m.nb[1] + by) * m.nb[0];
                cnt = m.start[row + m.nb[0]] - m.start[row];
            }
        }
    }
    return __syncthreads_or(cnt != 0u) != 0;
}

template <int Q, class S>
__global__ __launch_bounds__(256) void k_moments(const typename S::T* __restrict__ f,
                                                 float4* __restrict__ mom, long long N, S st, RowMask m) {
    using L = Lattice<Q>;
    const long long r0 = (long long)blockIdx.x * 256;
    if (m.start && !rows_needed(m, r0, min(r0 + 255, N - 1))) return;   // uniform over the block
    long long r = r0 + threadIdx.x;
    if (r >= N) return;
    float dr = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        // non-temporal: the populations outgrow the last-level cache, and
        // the collision reads them again only after the particle phases
        float h = st.load_stream(f + (long long)q * N + r);
        dr += h;
        if (L::ex(q)) jx += L::ex(q) * h;
        if (L::ey(q)) jy += L::ey(q) * h;
        if (L::ez(q)) jz += L::ez(q) * h;
    }
    mom[r] = make_float4(dr, jx, jy, jz);
}

// Workgroup size: 512 lanes for the 3D lattices in FP32 (256^3 D3Q19: 480
// against 492 us in the coupled step), 256 for D2Q9 (2048^2: 59 against
// 60 us) and for FP16 storage (266 against 269 us); 128 and 64 are far slower.
template <int Q, class S>
constexpr int collide_bs() { return (Q >= 15 && sizeof(typename S::T) == 4) ? 512 : 256; }

template <int Q, class S>
__global__ __launch_bounds__((collide_bs<Q, S>())) void k_collide(const typename S::T* __restrict__ fin,
                                                 typename S::T* __restrict__ fout,
                                                 const float* __restrict__ F, int hasF,
                                                 float ffx, float ffy, float ffz, Grid g,
                                                 float omega, float fpref, S st) {
    using L = Lattice<Q>;
    const long long N = g.N;
    long long r = (long long)blockIdx.x * collide_bs<Q, S>() + threadIdx.x;
    if (r >= N) return;
    const int nx = g.n[0], ny = g.n[1];
    const int x = (int)(r % nx);
    const long long t = r / nx;
    const int y = (int)(t % ny);
    const int z = (int)(t / ny);
    float Fx = ffx, Fy = ffy, Fz = ffz;
    if (hasF) {
        Fx += F[r];
        Fy += F[N + r];
        if (L::D == 3) Fz += F[2 * N + r];
    }
    collide_node<Q, S>(fin, fout, r, x, y, z, g, Fx, Fy, Fz, omega, fpref, st);
}

// Equilibrium populations (Eq. lbm3) from density and velocity fields.
template <int Q, class S>
__global__ __launch_bounds__(256) void k_init_eq(typename S::T* __restrict__ f, const float* __restrict__ rho,
                                                 const float* __restrict__ u, long long N, S st) {
    using L = Lattice<Q>;
    long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= N) return;
    float ro = rho ? rho[r] : 1.0f;
    float ux = u ? u[r] : 0.f, uy = u ? u[N + r] : 0.f, uz = (u && L::D == 3) ? u[2 * N + r] : 0.f;
    float uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        float eu = L::ex(q) * ux + L::ey(q) * uy + L::ez(q) * uz;
        float h = L::w(q) * ((ro - 1.0f) + ro * (3.0f * eu + 4.5f * eu * eu - 1.5f * uu));
        st.store(f + (long long)q * N + r, h);
    }
}

template <class S>
__global__ void k_decode(const typename S::T* __restrict__ f, float* __restrict__ out, long long n, S st) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = st.load(f + i);
}
template <class S>
__global__ void k_encode(typename S::T* __restrict__ f, const float* __restrict__ in, long long n, S st) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) st.store(f + i, in[i]);
}

// rho and u = j / rho of the stored state (from the float4 moments).
__global__ void k_fields(const float4* __restrict__ mom, float* __restrict__ rho, float* __restrict__ u,
                         long long N, int D) {
    long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= N) return;
    float4 m = mom[r];
    float ro = 1.0f + m.x;
    if (rho) rho[r] = ro;
    if (u) {
        u[r] = m.y / ro;
        u[N + r] = m.z / ro;
        if (D == 3) u[2 * N + r] = m.w / ro;
    }
}

// FP64 totals of the fluid: per block partial sums in a fixed tree, then a
// single block adds the partials in order (deterministic).
// part[b*8 + 0] = sum h, 1..3 = sum e h, 4 = max |u|^2, 5 = nonfinite count.
template <int Q, class S>
__global__ __launch_bounds__(256) void k_fluid_totals(const typename S::T* __restrict__ f, long long N,
                                                      double* __restrict__ part, S st) {
    using L = Lattice<Q>;
    __shared__ double sm[4][256];
    __shared__ float smax[256];
    __shared__ unsigned sbad[256];
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    float mx = 0.f;
    unsigned bad = 0;
    for (long long r = (long long)blockIdx.x * 256 + threadIdx.x; r < N; r += (long long)gridDim.x * 256) {
        double dr = 0, jx = 0, jy = 0, jz = 0;
        bool fin = true;
#pragma unroll
        for (int q = 0; q < Q; q++) {
            float hf = st.load(f + (long long)q * N + r);
            fin = fin && isfinite(hf);
            double hq = (double)hf;
            dr += hq;
            jx += L::ex(q) * hq;
            jy += L::ey(q) * hq;
            jz += L::ez(q) * hq;
        }
        a0 += dr; a1 += jx; a2 += jy; a3 += jz;
        float ro = 1.0f + (float)dr;
        float ux = (float)jx / ro, uy = (float)jy / ro, uz = (float)jz / ro;
        float s2 = ux * ux + uy * uy + uz * uz;
        if (!fin || !isfinite(s2)) bad++;
        else mx = fmaxf(mx, s2);
    }
    int t = threadIdx.x;
    sm[0][t] = a0; sm[1][t] = a1; sm[2][t] = a2; sm[3][t] = a3;
    smax[t] = mx; sbad[t] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            for (int k = 0; k < 4; k++) sm[k][t] += sm[k][t + s];
            smax[t] = fmaxf(smax[t], smax[t + s]);
            sbad[t] += sbad[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int k = 0; k < 4; k++) part[blockIdx.x * 8 + k] = sm[k][0];
        part[blockIdx.x * 8 + 4] = smax[0];
        part[blockIdx.x * 8 + 5] = sbad[0];
    }
}

__global__ void k_sum_partials(const double* __restrict__ part, int nblocks, double* __restrict__ out) {
    // one thread per output slot, blocks added in order
    int k = threadIdx.x;
    if (k >= 8) return;
    double acc = 0;
    for (int b = 0; b < nblocks; b++) {
        double v = part[b * 8 + k];
        if (k == 4) acc = fmax(acc, v);
        else acc += v;
    }
    out[k] = acc;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

template <int Q, class S>
static void launch_lattice_moments(const void* f, float4* mom, long long N, S st, const RowMask& m,
                                   hipStream_t s) {
    hipLaunchKernelGGL((k_moments<Q, S>), dim3(nblk(N)), dim3(256), 0, s, (const typename S::T*)f, mom, N, st, m);
}

template <int Q, class S>
static void launch_lattice_collide(const void* fin, void* fout, const float* F, int hasF, const float* ff,
                                   const Grid& g, float tau, S st, hipStream_t s) {
    constexpr int BS = collide_bs<Q, S>();
    hipLaunchKernelGGL((k_collide<Q, S>), dim3((unsigned)((g.N + BS - 1) / BS)), dim3(BS), 0, s,
                       (const typename S::T*)fin,
                       (typename S::T*)fout, F, hasF, ff[0], ff[1], ff[2], g, 1.0f / tau,
                       1.0f - 0.5f / tau, st);
}

#define PIBM_DISPATCH(Q, FP16, ...)                                   \
    do {                                                              \
        if ((Q) == 9 && !(FP16)) { constexpr int QQ = 9; using SS = StoreF32; __VA_ARGS__; }        \
        else if ((Q) == 9) { constexpr int QQ = 9; using SS = StoreF16; __VA_ARGS__; }              \
        else if ((Q) == 15 && !(FP16)) { constexpr int QQ = 15; using SS = StoreF32; __VA_ARGS__; } \
        else if ((Q) == 15) { constexpr int QQ = 15; using SS = StoreF16; __VA_ARGS__; }            \
        else if (!(FP16)) { constexpr int QQ = 19; using SS = StoreF32; __VA_ARGS__; }              \
        else { constexpr int QQ = 19; using SS = StoreF16; __VA_ARGS__; }                           \
    } while (0)

template <class S> static S make_store(int scale_log2) {
    S st;
    st.scale = ldexpf(1.0f, scale_log2);
    st.inv_scale = ldexpf(1.0f, -scale_log2);
    return st;
}

void lattice_moments(int Q, int fp16, int sl2, const void* f, float4* mom, long long N, const RowMask& m,
                     hipStream_t s) {
    PIBM_DISPATCH(Q, fp16, launch_lattice_moments<QQ, SS>(f, mom, N, make_store<SS>(sl2), m, s));
}

void lattice_collide(int Q, int fp16, int sl2, const void* fin, void* fout, const float* F, int hasF,
                     const float* ff, const Grid& g, float tau, hipStream_t s) {
    PIBM_DISPATCH(Q, fp16, launch_lattice_collide<QQ, SS>(fin, fout, F, hasF, ff, g, tau, make_store<SS>(sl2), s));
}

void lattice_init_eq(int Q, int fp16, int sl2, void* f, const float* rho, const float* u, long long N,
                     hipStream_t s) {
    PIBM_DISPATCH(Q, fp16,
                  hipLaunchKernelGGL((k_init_eq<QQ, SS>), dim3(nblk(N)), dim3(256), 0, s,
                                     (typename SS::T*)f, rho, u, N, make_store<SS>(sl2)));
}

void lattice_decode(int fp16, int sl2, const void* f, float* out, long long n, hipStream_t s) {
    if (fp16)
        hipLaunchKernelGGL((k_decode<StoreF16>), dim3(nblk(n)), dim3(256), 0, s, (const _Float16*)f, out, n,
                           make_store<StoreF16>(sl2));
    else
        hipLaunchKernelGGL((k_decode<StoreF32>), dim3(nblk(n)), dim3(256), 0, s, (const float*)f, out, n,
                           make_store<StoreF32>(sl2));
}

void lattice_encode(int fp16, int sl2, void* f, const float* in, long long n, hipStream_t s) {
    if (fp16)
        hipLaunchKernelGGL((k_encode<StoreF16>), dim3(nblk(n)), dim3(256), 0, s, (_Float16*)f, in, n,
                           make_store<StoreF16>(sl2));
    else
        hipLaunchKernelGGL((k_encode<StoreF32>), dim3(nblk(n)), dim3(256), 0, s, (float*)f, in, n,
                           make_store<StoreF32>(sl2));
}

void lattice_fields(const float4* mom, float* rho, float* u, long long N, int D, hipStream_t s) {
    hipLaunchKernelGGL(k_fields, dim3(nblk(N)), dim3(256), 0, s, mom, rho, u, N, D);
}

// out[a N + r] = in[a N + r] + c[a] for a < D: the spread force field plus
// the uniform fluid force, as the collision uses it.
__global__ __launch_bounds__(256) void k_add_const(const float* __restrict__ in, float* __restrict__ out,
                                                   long long N, int D, float c0, float c1, float c2) {
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= N) return;
    const float c[3] = {c0, c1, c2};
    for (int a = 0; a < D; a++) out[a * N + r] = c[a] != 0.0f ? in[a * N + r] + c[a] : in[a * N + r];
}

void lattice_add_const(const float* in, float* out, long long N, int D, const float* c, hipStream_t s) {
    hipLaunchKernelGGL(k_add_const, dim3(nblk(N)), dim3(256), 0, s, in, out, N, D, c[0], c[1], c[2]);
}

int lattice_totals_blocks() { return 1024; }

void lattice_totals(int Q, int fp16, int sl2, const void* f, long long N, double* part, double* out,
                    hipStream_t s) {
    int nb = lattice_totals_blocks();
    PIBM_DISPATCH(Q, fp16,
                  hipLaunchKernelGGL((k_fluid_totals<QQ, SS>), dim3(nb), dim3(256), 0, s,
                                     (const typename SS::T*)f, N, part, make_store<SS>(sl2)));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, nb, out);
}

}  // namespace pibm
