// particles.hip -- particle side of the coupled step (gfx950, wave64).
//
// Cell list (the paper is silent on neighbour search): every particle gets
// the bin of its dual cell floor(X - 1/2) (bins of 2^L dual cells per axis);
// a counting sort over bins (one radix digit = the bin index) with integer
// atomics gives the bin ranges, and the slot of each particle inside its bin
// is its rank by id, so the order (bin, id) is unique and the result is
// bit-identical from run to run.  The particle state is kept in that order.
//
// Interpolation (Eqs. lbm11-lbm12): 4^D support nodes per particle; one
// group of 4^(D-1) lanes per particle, each lane one x-row of 4 nodes, a
// float4 (drho, j) load per node and a shuffle reduction.
//
// DEM (Eq. demgov with the reaction force of Eq. lbm13 and the momentum
// exchange of Eqs. lbm7-lbm8, g = 2 (rho_i U - j_i)): n_sub sub-steps with
// the fluid moments frozen.  A particle with no neighbour and no wall within
// contact distance + skin has a linear sub-step recurrence and takes its
// closed form; the others are grouped into islands (connected components of
// the candidate graph, union-find with integer CAS) packed into waves, and
// iterate their sub-steps in LDS with one barrier per sub-step.
//
// Spreading (Eq. lbm10): gathered per node over the bins whose particles
// can reach it, in (bin, id) order: deterministic, no float atomics.
#include <algorithm>
#include <utility>

#include "pibm_internal.h"

namespace pibm {


__device__ __forceinline__ int bin_of(const PCfg& c, float xh, float xl, int a) {
    int ci = dual_cell(xh, xl);
    int b = (ci + 1) >> c.L;
    return min(max(b, 0), c.nb[a] - 1);
}

// ---------------------------------------------------------------------------
// generic helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, long long n, uint32_t v) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// fill p[0 .. count*mult) where count is read on the device
__global__ void k_fill_dyn(uint32_t* p, const uint32_t* count, int mult, uint32_t v, long long cap) {
    long long n = (long long)(*count) * mult;
    if (n > cap) n = cap;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        p[i] = v;
}

// Three-phase exclusive scan (u32 or u64).  A tile is 256 threads x 16
// consecutive items; within a block the thread sums are scanned with wave
// shuffles (64 lanes) and the four wave totals through LDS.
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;

template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

// Exclusive scan of one value per thread over a block of NW waves (sh holds
// NW entries of LDS).
template <class T, int NW = 4>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh, T& total) {
    const int t = threadIdx.x, w = t >> 6;
    const T inc = wave_inclusive_scan<T>(v);
    if ((t & 63) == 63) sh[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) {
        if (k < w) before += sh[k];
        all += sh[k];
    }
    total = all;
    __syncthreads();
    return before + inc - v;
}

// Largest number of blocks for which every block adds up the totals of the
// blocks before it itself (the sum costs O(blocks^2) reads over the grid).
constexpr long long RAW_MAX_BLOCKS = 2048;

// Sum of x[0, n) over one block of NT threads, returned to every thread
// (sh: NT / 64 entries of LDS).  Integer sums: exact in any order.
template <class T, int NT>
__device__ __forceinline__ T block_sum(const T* __restrict__ x, long long n, T* sh) {
    T s = 0;
    for (long long i = threadIdx.x; i < n; i += NT) s += x[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    T t = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; k++) t += sh[k];
    __syncthreads();
    return t;
}

// Items [base, base + SCAN_ITEMS) of `in`, zero past n; full tiles are read
// with 16-byte loads (the arrays are 256-byte aligned, base a multiple of 16).
template <class T>
__device__ __forceinline__ void load_items(const T* __restrict__ in, long long base, long long n, T* v) {
    if (base + SCAN_ITEMS <= n) {
        constexpr int PER = 16 / sizeof(T);
        const uint4* p = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS / PER; k++) {
            uint4 q = p[k];
            T tmp[PER];
            __builtin_memcpy(tmp, &q, 16);
#pragma unroll
            for (int i = 0; i < PER; i++) v[k * PER + i] = tmp[i];
        }
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; k++) v[k] = (base + k < n) ? in[base + k] : (T)0;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_scan_reduce(const T* __restrict__ in, long long n, T* __restrict__ bsum) {
    __shared__ T sh4[4];
    const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    load_items<T>(in, base, n, v);
    T s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) s += v[k];
    T tot;
    block_exclusive_scan<T>(s, sh4, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One block of 1024 threads: exclusive scan of the nb tile sums in place
// (each thread takes a run of consecutive sums), grand total to *total.
constexpr int TOP_THREADS = 1024;
constexpr int TOP_ITEMS = 16;      // sums per thread held in registers (up to 16384 blocks)
template <class T>
__global__ __launch_bounds__(TOP_THREADS) void k_scan_top(T* __restrict__ bsum, long long nb, T* __restrict__ total) {
    __shared__ T sh[TOP_THREADS / 64];
    const long long per = (nb + TOP_THREADS - 1) / TOP_THREADS;
    const long long b0 = (long long)threadIdx.x * per;
    const long long b1 = b0 + per < nb ? b0 + per : nb;
    T s = 0, tot;
    if (per <= TOP_ITEMS) {
        // the usual case: a thread's sums loaded together into registers
        T v[TOP_ITEMS];
#pragma unroll
        for (int k = 0; k < TOP_ITEMS; k++) {
            v[k] = b0 + k < b1 ? bsum[b0 + k] : (T)0;
            s += v[k];
        }
        T run = block_exclusive_scan<T, TOP_THREADS / 64>(s, sh, tot);
#pragma unroll
        for (int k = 0; k < TOP_ITEMS; k++)
            if (b0 + k < b1) {
                bsum[b0 + k] = run;
                run += v[k];
            }
    } else {
        for (long long i = b0; i < b1; i++) s += bsum[i];
        T run = block_exclusive_scan<T, TOP_THREADS / 64>(s, sh, tot);
        for (long long i = b0; i < b1; i++) {
            const T x = bsum[i];
            bsum[i] = run;
            run += x;
        }
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

// With zero_in the input is cleared after it has been read (the bin counts
// then start from zero at the next sort without a separate fill).  With RAW
// the tile sums in bsum are not scanned yet: each block adds up those of
// the tiles before it itself (no one-block pass in between).
template <class T, bool RAW>
__global__ __launch_bounds__(256) void k_scan_down(T* __restrict__ in, T* __restrict__ out, long long n,
                                                   const T* __restrict__ bsum, int zero_in) {
    __shared__ T sh4[4];
    const T before = RAW ? block_sum<T, 256>(bsum, (long long)blockIdx.x, sh4) : bsum[blockIdx.x];
    const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    load_items<T>(in, base, n, v);
    if (zero_in) {
        if (base + SCAN_ITEMS <= n) {
            // items that are all zero stay as they are (the bin counts of
            // the empty parts of the box cost no writes)
            T any = 0;
#pragma unroll
            for (int k = 0; k < SCAN_ITEMS; k++) any |= v[k];
            if (any != 0) {
                uint4* p = reinterpret_cast<uint4*>(in + base);
#pragma unroll
                for (int k = 0; k < (int)(SCAN_ITEMS * sizeof(T) / 16); k++) p[k] = make_uint4(0u, 0u, 0u, 0u);
            }
        } else {
            for (int k = 0; k < SCAN_ITEMS; k++)
                if (base + k < n) in[base + k] = (T)0;
        }
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) s += v[k];
    T tot;
    T ex = block_exclusive_scan<T>(s, sh4, tot) + before;
    if (base + SCAN_ITEMS <= n) {
        constexpr int PER = 16 / sizeof(T);
        uint4* p = reinterpret_cast<uint4*>(out + base);
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS / PER; k++) {
            T tmp[PER];
#pragma unroll
            for (int i = 0; i < PER; i++) {
                tmp[i] = ex;
                ex += v[k * PER + i];
            }
            uint4 q;
            __builtin_memcpy(&q, tmp, 16);
            p[k] = q;
        }
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; k++) {
            if (base + k < n) out[base + k] = ex;
            ex += v[k];
        }
    }
}

// Exclusive scan of in[0, n) into out; the input is cleared afterwards when
// zero_in is set.
// Without a total, two passes (tile sums, then tiles adding up their
// predecessors' sums themselves); with one, three (the tile sums scanned by
// one block, which also writes the total).
template <class T>
void scan_exclusive(T* in, T* out, long long n, T* bsum, T* total, bool zero_in, hipStream_t s) {
    long long nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL((k_scan_reduce<T>), dim3((unsigned)nb), dim3(256), 0, s, in, n, bsum);
    if (total || nb > 2 * RAW_MAX_BLOCKS) {
        hipLaunchKernelGGL((k_scan_top<T>), dim3(1), dim3(TOP_THREADS), 0, s, bsum, nb, total);
        hipLaunchKernelGGL((k_scan_down<T, false>), dim3((unsigned)nb), dim3(256), 0, s, in, out, n, bsum,
                           zero_in ? 1 : 0);
    } else {
        hipLaunchKernelGGL((k_scan_down<T, true>), dim3((unsigned)nb), dim3(256), 0, s, in, out, n, bsum,
                           zero_in ? 1 : 0);
    }
}

long long scan_blocks(long long n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

// ---------------------------------------------------------------------------
// cell list
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_bin_count(PState A, int np, PCfg c, uint32_t* __restrict__ cnt,
                                                   uint32_t* __restrict__ keys, uint32_t* __restrict__ slot,
                                                   uint32_t* __restrict__ flags) {
    int s = xcd_block() * 256 + threadIdx.x;
    if (s >= np) return;
    int b[3] = {0, 0, 0};
    bool inside = true;
#pragma unroll
    for (int a = 0; a < D; a++) {
        float xh = A.xh[a][s], xl = A.xl[a][s];
        inside = inside && (xh > 0.0f) && (xh < (float)c.n[a]) && isfinite(xh);
        b[a] = bin_of(c, xh, xl, a);
    }
    if (!inside) atomicOr(flags, FLAG_UNSTABLE);
    uint32_t key = (uint32_t)(((long long)b[2] * c.nb[1] + b[1]) * c.nb[0] + b[0]);
    keys[s] = key;
    slot[s] = atomicAdd(&cnt[key], 1u);
}

// The id of each particle to its place among its bin (in the order the
// counts were taken), so that ranking reads the ids of a bin from
// consecutive words.
__global__ void k_scatter(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ slot,
                          const uint32_t* __restrict__ start, const int* __restrict__ id,
                          int* __restrict__ tmpid, int np) {
    int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= np) return;
    tmpid[start[keys[s]] + slot[s]] = id[s];
}

// Final slot = bin start + rank of the particle's id among its bin.
template <int D>
__global__ __launch_bounds__(256) void k_reorder(PState A, PState B, const uint32_t* __restrict__ keys,
                                                 const uint32_t* __restrict__ start,
                                                 const int* __restrict__ tmpid,
                                                 uint32_t* __restrict__ keys_sorted, float4* __restrict__ pos4,
                                                 int np) {
    int s = xcd_block() * 256 + threadIdx.x;
    if (s >= np) return;
    uint32_t k = keys[s];
    uint32_t b0 = start[k], b1 = start[k + 1];
    int myid = A.id[s];
    uint32_t rank = 0;
    for (uint32_t t = b0; t < b1; t++) rank += (tmpid[t] < myid) ? 1u : 0u;
    uint32_t o = b0 + rank;
#pragma unroll
    for (int a = 0; a < D; a++) {
        B.xh[a][o] = A.xh[a][s];
        B.xl[a][o] = A.xl[a][s];
        B.u[a][o] = A.u[a][s];
    }
    B.d[o] = A.d[s];
    B.rp[o] = A.rp[s];
    B.id[o] = myid;
#pragma unroll
    for (int a = 0; a < 3; a++)
        if (A.w[a]) B.w[a][o] = A.w[a][s];
    if (A.fixa) B.fixa[o] = A.fixa[s];
    keys_sorted[o] = k;
    // leading parts of the position and the diameter, for neighbour screening
    pos4[o] = make_float4(A.xh[0][s], A.xh[1][s], D == 3 ? A.xh[2][s] : 0.f, A.d[s]);
}

// ---------------------------------------------------------------------------
// interpolation (Eqs. lbm11-lbm12 weights, moments gathered): phi_k = delta(X - (i + 1/2)) of the four
// nodes i = floor(X - 1/2) - 1 + k, zero outside the domain, divided by
// their sum.  With fr = X - 1/2 - floor(X - 1/2) the four cosines are
// -sin, cos, sin, -cos of (pi fr / 2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void axis_weights(float xh, float xl, int n, int& base, float* phi) {
    int c = dual_cell(xh, xl);
    float fr = dual_frac(xh, xl, c);
    float sv, cv;
    sincospif(0.5f * fr, &sv, &cv);
    base = c - 1;
    float w0 = 0.25f * (1.0f - sv), w1 = 0.25f * (1.0f + cv), w2 = 0.25f * (1.0f + sv), w3 = 0.25f * (1.0f - cv);
    if (base < 0 || base >= n) w0 = 0.f;
    if (base + 1 < 0 || base + 1 >= n) w1 = 0.f;
    if (base + 2 < 0 || base + 2 >= n) w2 = 0.f;
    if (base + 3 < 0 || base + 3 >= n) w3 = 0.f;
    float sum = w0 + w1 + w2 + w3;
    float inv = sum > 0.f ? 1.0f / sum : 0.f;
    phi[0] = w0 * inv; phi[1] = w1 * inv; phi[2] = w2 * inv; phi[3] = w3 * inv;
}

// Lagrange form of the gather (Eq. lbm5-lbm6) on the same four nodes: the
// basis polynomial of node k through the in-domain nodes of the axis,
// l_k = prod_{m != k, in domain} (t - m) / (k - m), with the particle at
// t = fr + 1 in node units from node 0 of the stencil.  Cubic in the
// interior, of lower order next to a wall; zero for nodes outside.
__device__ __forceinline__ void axis_lagrange(float xh, float xl, int n, float* lag) {
    const int c = dual_cell(xh, xl);
    const float t = dual_frac(xh, xl, c) + 1.0f;
    const int base = c - 1;
    bool in[4];
#pragma unroll
    for (int k = 0; k < 4; k++) in[k] = base + k >= 0 && base + k < n;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        float v = in[k] ? 1.0f : 0.0f;
#pragma unroll
        for (int m = 0; m < 4; m++)
            if (m != k && in[m]) v *= (t - (float)m) * (1.0f / (float)(k - m));
        lag[k] = v;
    }
}

// Gather weights of one axis: the delta-kernel weights phi (always: the
// spreading pass reuses them) and, with LAG, the Lagrange weights in gw.
template <bool LAG>
__device__ __forceinline__ void axis_gather(float xh, float xl, int n, int& base, float* phi, float* gw) {
    axis_weights(xh, xl, n, base, phi);
    if (LAG) axis_lagrange(xh, xl, n, gw);
    else
#pragma unroll
        for (int k = 0; k < 4; k++) gw[k] = phi[k];
}

template <int D, bool LAG>
__global__ __launch_bounds__(256) void k_interp(PState A, int np, Grid g, const float4* __restrict__ mom,
                                                float* __restrict__ drho_i, float* __restrict__ j_i,
                                                short4* __restrict__ wbase, float* __restrict__ srec) {
    constexpr int LP = (D == 3) ? 16 : 4;   // lanes per particle
    long long gt = (long long)xcd_block() * 256 + threadIdx.x;
    int s = (int)(gt / LP);
    int l = (int)(gt % LP);
    bool valid = s < np;
    int sc = valid ? s : np - 1;
    int base[3] = {0, 0, 0};
    float phi[3][4], gw[3][4];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (a < D) axis_gather<LAG>(A.xh[a][sc], A.xl[a][sc], g.n[a], base[a], phi[a], gw[a]);
        else {
            phi[a][0] = gw[a][0] = 1.f;
            phi[a][1] = phi[a][2] = phi[a][3] = gw[a][1] = gw[a][2] = gw[a][3] = 0.f;
        }
    }
    int ky = l & 3, kz = (D == 3) ? (l >> 2) : 0;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (valid) {
        int y = base[1] + ky, z = base[2] + kz;
        float wyz = gw[1][ky] * gw[2][kz];
        if (wyz != 0.f) {
            long long row = ((long long)z * g.n[1] + y) * g.n[0];
#pragma unroll
            for (int kx = 0; kx < 4; kx++) {
                float W = gw[0][kx] * gw[1][ky] * gw[2][kz];
                if (W != 0.f) {
                    float4 m = mom[row + base[0] + kx];
                    acc[0] += W * m.x; acc[1] += W * m.y; acc[2] += W * m.z; acc[3] += W * m.w;
                }
            }
        }
    }
#pragma unroll
    for (int off = 1; off < LP; off <<= 1)
#pragma unroll
        for (int k = 0; k < 4; k++) acc[k] += __shfl_xor(acc[k], off, LP);
    if (!valid) return;
    if (l == 0) {
        drho_i[s] = acc[0];
        j_i[s] = acc[1];
        j_i[(long long)np + s] = acc[2];
        if (D == 3) j_i[2LL * np + s] = acc[3];
        wbase[s] = make_short4((short)base[0], (short)base[1], (short)base[2], 0);
        srec[(long long)s * SRec<D>::STRIDE + SRec<D>::BASE] = __int_as_float(base[0]);
    }
    // weights for the spreading pass: 4 D floats per particle
    if (D == 3) {
        if (l < 12) srec[(long long)s * SRec<D>::STRIDE + l] = phi[l >> 2][l & 3];
    } else {
        srec[(long long)s * SRec<D>::STRIDE + l] = phi[0][l];
        srec[(long long)s * SRec<D>::STRIDE + 4 + l] = phi[1][l];
    }
}

// Interpolation by tiles: a workgroup owns a box of bins; the sorted
// particles of those bins are contiguous per bin row.  It stages the moment
// field of every node those particles can reach (the box of nodes plus a
// halo of 2 below and 1 above, in dual-cell terms) in LDS once, then each
// thread gathers one particle's 4^D support from LDS.  Tiles without
// particles return before loading anything.
// tile extent in dual cells (bins hold 2^L cells per axis)
template <int D> struct InterpTile;
template <> struct InterpTile<3> { static constexpr int CX = 32, CY = 4, CZ = 4; };
template <> struct InterpTile<2> { static constexpr int CX = 128, CY = 8, CZ = 1; };

// Node moments (density deviation, momentum) staged into LDS either from
// the moments pass (MomSrc) or, in D2Q9, straight from the stored
// populations (PopSrc): only tiles holding particles read the lattice.
struct MomSrc {
    const float4* mom;
    __device__ __forceinline__ float4 at(long long r, long long) const { return mom[r]; }
};
template <class S>
struct PopSrc {
    const typename S::T* f;
    S st;
    __device__ __forceinline__ float4 at(long long r, long long N) const {
        using L = Lattice<9>;
        float dr = 0.f, jx = 0.f, jy = 0.f;
#pragma unroll
        for (int q = 0; q < 9; q++) {
            const float h = st.load(f + (long long)q * N + r);
            dr += h;
            if (L::ex(q)) jx += L::ex(q) * h;
            if (L::ey(q)) jy += L::ey(q) * h;
        }
        return make_float4(dr, jx, jy, 0.f);
    }
};

template <int D, class Src, bool LAG>
__global__ __launch_bounds__(256) void k_interp_tile(PState A, int np, Grid g, PCfg c,
                                                     const uint32_t* __restrict__ start,
                                                     Src src,
                                                     float* __restrict__ drho_i, float* __restrict__ j_i,
                                                     short4* __restrict__ wbase, float* __restrict__ srec,
                                                     int ntx, int nty) {
    using T0 = InterpTile<D>;
    constexpr int NX = T0::CX + 3, NY = T0::CY + 3, NZ = (D == 3) ? T0::CZ + 3 : 1;
    constexpr int MAXR = T0::CY * T0::CZ;                // bin rows per tile at most (L = 0)
    struct TB { int TBX, TBY, TBZ; };
    const int E = 1 << c.L;                               // dual cells per bin edge
    const TB T{T0::CX / E, T0::CY / E, (D == 3) ? T0::CZ / E : 1};
    __shared__ float4 sm[NX * NY * NZ];
    __shared__ uint32_t rs[MAXR], re[MAXR], roff[MAXR + 1];
    __shared__ uint32_t scan4[4];
    int tx, ty, tz;
    banded_tile(ntx, nty, (int)gridDim.x / (ntx * nty), D == 3 ? 1 : 0, tx, ty, tz);
    const int B0x = tx * T.TBX, B0y = ty * T.TBY, B0z = tz * T.TBZ;
    const int t = threadIdx.x;
    if (t < T.TBY * T.TBZ) {
        const int by = B0y + t % T.TBY, bz = B0z + t / T.TBY;
        uint32_t s0 = 0, s1 = 0;
        if (by < c.nb[1] && bz < c.nb[2] && B0x < c.nb[0]) {
            const int bx1 = min(B0x + T.TBX, c.nb[0]) - 1;
            const uint32_t row = (uint32_t)(((long long)bz * c.nb[1] + by) * c.nb[0]);
            s0 = start[row + B0x];
            s1 = start[row + bx1 + 1];
        }
        rs[t] = s0;
        re[t] = s1;
    }
    {
        // row offsets: exclusive scan of the row counts over the block
        const uint32_t n = (t < T.TBY * T.TBZ) ? re[t] - rs[t] : 0u;
        uint32_t all;
        const uint32_t ex = block_exclusive_scan<uint32_t>(n, scan4, all);
        if (t < T.TBY * T.TBZ) roff[t] = ex;
        if (t == 0) roff[T.TBY * T.TBZ] = all;
    }
    __syncthreads();
    const uint32_t total = roff[T.TBY * T.TBZ];
    if (total == 0) return;
    // sorted slot of entry k: row r is the largest with roff[r] <= k
    auto slot_of = [&](uint32_t k) {
        int r = 0, rh = T.TBY * T.TBZ;
        while (rh - r > 1) {
            const int mid = (r + rh) >> 1;
            if (roff[mid] <= k) r = mid;
            else rh = mid;
        }
        return rs[r] + (k - roff[r]);
    };
    // the positions of the thread's first particle are loaded together with
    // the halo (a tile holds fewer than 256 particles as a rule)
    const uint32_t s_first = t < total ? slot_of((uint32_t)t) : 0u;
    float xh0[3] = {0.f, 0.f, 0.f}, xl0[3] = {0.f, 0.f, 0.f};
    if ((uint32_t)t < total) {
#pragma unroll
        for (int a = 0; a < D; a++) {
            xh0[a] = A.xh[a][s_first];
            xl0[a] = A.xl[a][s_first];
        }
    }
    // node box: dual cells of the tile are [B0 E - 1, (B0 + TB) E - 2], reaching nodes
    // [B0 E - 2, (B0 + TB) E]
    const int nx0 = B0x * E - 2, ny0 = B0y * E - 2, nz0 = (D == 3) ? B0z * E - 2 : 0;
    const int lx = T.TBX * E + 3, ly = T.TBY * E + 3, lz = (D == 3) ? T.TBZ * E + 3 : 1;
    {
        // every thread issues all of its halo loads before using any (nodes
        // outside the lattice read node 0 and are zeroed)
        constexpr int IT = (NX * NY * NZ + 255) / 256;
        const int nh = lx * ly * lz;
        float4 v[IT];
#pragma unroll
        for (int k = 0; k < IT; k++) {
            const int i = t + k * 256;
            const int ix = i % lx, iy = (i / lx) % ly, iz = i / (lx * ly);
            const int x = nx0 + ix, y = ny0 + iy, z = nz0 + iz;
            const bool ok = i < nh && x >= 0 && x < g.n[0] && y >= 0 && y < g.n[1] && z >= 0 && z < g.n[2];
            v[k] = src.at(ok ? ((long long)z * g.n[1] + y) * g.n[0] + x : 0LL, g.N);
            if (!ok) v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < IT; k++)
            if (t + k * 256 < nh) sm[t + k * 256] = v[k];
    }
    __syncthreads();
    for (uint32_t k = t; k < total; k += 256) {
        const bool first = k == (uint32_t)t;
        const uint32_t s = first ? s_first : slot_of(k);
        int base[3] = {0, 0, 0};
        float phi[3][4], gw[3][4];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (a < D)
                axis_gather<LAG>(first ? xh0[a] : A.xh[a][s], first ? xl0[a] : A.xl[a][s], g.n[a], base[a], phi[a],
                                 gw[a]);
            else {
                phi[a][0] = gw[a][0] = 1.f;
                phi[a][1] = phi[a][2] = phi[a][3] = gw[a][1] = gw[a][2] = gw[a][3] = 0.f;
            }
        }
        float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
        const int ox = base[0] - nx0, oy = base[1] - ny0, oz = (D == 3) ? base[2] - nz0 : 0;
#pragma unroll
        for (int kz = 0; kz < (D == 3 ? 4 : 1); kz++)
#pragma unroll
            for (int ky = 0; ky < 4; ky++)
#pragma unroll
                for (int kx = 0; kx < 4; kx++) {
                    const float W = gw[0][kx] * gw[1][ky] * gw[2][kz];
                    if (W != 0.f) {
                        const float4 m = sm[((oz + kz) * ly + (oy + ky)) * lx + (ox + kx)];
                        acc0 += W * m.x; acc1 += W * m.y; acc2 += W * m.z; acc3 += W * m.w;
                    }
                }
        drho_i[s] = acc0;
        j_i[s] = acc1;
        j_i[(long long)np + s] = acc2;
        if (D == 3) j_i[2LL * np + s] = acc3;
        wbase[s] = make_short4((short)base[0], (short)base[1], (short)base[2], 0);
        float* rec = srec + (long long)s * SRec<D>::STRIDE;
#pragma unroll
        for (int a = 0; a < D; a++)
#pragma unroll
            for (int q = 0; q < 4; q++) rec[4 * a + q] = phi[a][q];
        rec[SRec<D>::BASE] = __int_as_float(base[0]);
    }
}

// ---------------------------------------------------------------------------
// DEM: classification and the free-particle closed form
// ---------------------------------------------------------------------------
// The bins around particle s that its reach meets: at most (2H + 1)^D,
// usually 2 or 3 per axis.  A partner within (d_s + d_t)/2 + skin + eps
// <= r_s lies at most ceil(r_s / edge) bins away (bin = (floor(X - 1/2) + 1)
// >> L).  Per axis, only the bins that meet [X - r_s, X + r_s]: a particle
// of bin k lies in [k - 1/2, k + 1/2) (edge 1), so every bin beyond
// bin(X + r_s) or below bin(X - r_s) is farther than r_s along that axis.
// The 1/64 margin covers the rounding of X +- r_s against the bin keys.
// The range never excludes the own bin, so a stray position cannot widen it.
template <int D>
__device__ __forceinline__ void neighbour_bins(const float4& me, uint32_t key, const PCfg& c, int lo[3], int hi[3]) {
    int b[3];
    b[0] = (int)(key % (uint32_t)c.nb[0]);
    b[1] = (int)((key / (uint32_t)c.nb[0]) % (uint32_t)c.nb[1]);
    b[2] = (int)(key / ((uint32_t)c.nb[0] * (uint32_t)c.nb[1]));
    const float r_s = (0.5f * (me.w + c.dmax) + c.skin + c.eps) * (1.0f + 1e-6f);
    const int H = min(c.H, max(1, (int)ceilf(r_s * ldexpf(1.0f, -c.L))));
    const float rr = r_s + 0.015625f;
    lo[1] = lo[2] = hi[1] = hi[2] = 0;
#pragma unroll
    for (int a = 0; a < D; a++) {
        const float xa = a == 0 ? me.x : (a == 1 ? me.y : me.z);
        const int l = ((int)floorf(xa - rr - 0.5f) + 1) >> c.L;
        const int h = ((int)floorf(xa + rr - 0.5f) + 1) >> c.L;
        lo[a] = min(max(max(l, b[a] - H), 0), b[a]);
        hi[a] = max(min(min(h, b[a] + H), c.nb[a] - 1), b[a]);
    }
}

// Screening uses the leading FP32 parts of the positions; c.eps bounds the
// neglected trailing parts, and every test is widened by it (more candidates
// or more active particles only cost time).  Points of fixed bodies do not
// interact with each other.

// Counting scan: the number of candidates within (d_s + d_t)/2 + skin, and
// whether any lies within (d_s + d_t)/2 + thr.  The order of the visits does
// not matter here, so the scan is laid out for memory-level parallelism:
// the start and end of up to R rows of bins (bins of one row are contiguous
// in the sorted order) are loaded together, their particles are numbered
// 0..tot-1 across the rows, and the positions are fetched four at a time.
template <int D>
__device__ __forceinline__ int count_neighbours(const float4* __restrict__ pos4, const uint32_t* __restrict__ start,
                                                const float4& me, uint32_t key, const PCfg& c, int s, float thr,
                                                bool& close, bool mefix, const float* __restrict__ fixa) {
    constexpr int R = (D == 3) ? 9 : 3;          // rows per batch: every row of a reach of 3 bins per axis
    int lo[3], hi[3];
    neighbour_bins<D>(me, key, c, lo, hi);
    const int ny = hi[1] - lo[1] + 1;
    const int nr = ny * (hi[2] - lo[2] + 1);
    int cnt = 0;
    int cy = lo[1], cz = lo[2];                  // next row to load
    for (int r0 = 0; r0 < nr; r0 += R) {
        // particle k (pre[i] <= k < pre[i + 1]) of this batch is t = k + off[i]
        uint32_t pre[R + 1], off[R];
        pre[0] = 0u;
#pragma unroll
        for (int i = 0; i < R; i++) {
            uint32_t t0 = 0u, t1 = 0u;
            if (r0 + i < nr) {
                const uint32_t row = (uint32_t)(((long long)cz * c.nb[1] + cy) * c.nb[0]);
                t0 = start[row + lo[0]];
                t1 = start[row + hi[0] + 1];
                if (++cy > hi[1]) {
                    cy = lo[1];
                    cz++;
                }
            }
            off[i] = t0 - pre[i];
            pre[i + 1] = pre[i] + (t1 - t0);
        }
        const uint32_t tot = pre[R];
        for (uint32_t k = 0; k < tot; k += 4) {
            int t[4];
            float4 o[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t kk = k + j;
                uint32_t tt = kk + off[0];
#pragma unroll
                for (int i = 1; i < R; i++) tt = kk >= pre[i] ? kk + off[i] : tt;
                t[j] = kk < tot ? (int)tt : s;   // past the end: the particle itself, skipped
                o[j] = pos4[t[j]];
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                bool ok = t[j] != s;
                if (mefix) ok = ok && !(fixa[t[j]] > 0.f);
                const float dx = me.x - o[j].x, dy = me.y - o[j].y, dz = (D == 3) ? me.z - o[j].z : 0.f;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rc = 0.5f * (me.w + o[j].w);
                const float cut = rc + c.skin + c.eps;
                const float lim = rc + thr + c.eps;
                ok = ok && r2 < cut * cut;
                cnt += ok ? 1 : 0;
                close = close || (ok && r2 <= lim * lim);
            }
        }
    }
    return cnt;
}

// Collecting scan: the candidates within (d_s + d_t)/2 + skin that are
// active, in scan order (bins ascending, sorted order within a bin).
template <int D>
__device__ __forceinline__ int collect_neighbours(const float4* __restrict__ pos4, const uint32_t* __restrict__ start,
                                                  const uint32_t* __restrict__ keys_sorted, const PCfg& c, int s,
                                                  const unsigned long long* __restrict__ actcc, uint32_t* list,
                                                  int cap, const float* __restrict__ fixa) {
    const bool mefix = fixa && fixa[s] > 0.f;
    const float4 me = pos4[s];
    int lo[3], hi[3];
    neighbour_bins<D>(me, keys_sorted[s], c, lo, hi);
    int cnt = 0;
    for (int bz = lo[2]; bz <= hi[2]; bz++)
        for (int by = lo[1]; by <= hi[1]; by++) {
            const uint32_t row = (uint32_t)(((long long)bz * c.nb[1] + by) * c.nb[0]);
            const uint32_t t0 = start[row + lo[0]], t1 = start[row + hi[0] + 1];
            for (uint32_t t = t0; t < t1; t++) {
                if ((int)t == s) continue;
                if (mefix && fixa[t] > 0.f) continue;
                const float4 o = pos4[t];
                const float dx = me.x - o.x, dy = me.y - o.y, dz = (D == 3) ? me.z - o.z : 0.f;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float cut = 0.5f * (me.w + o.w) + c.skin + c.eps;
                if (r2 < cut * cut && actcc[t] != 0ULL) {
                    if (cnt < cap) list[cnt] = t;
                    cnt++;
                }
            }
        }
    return cnt;
}

// Classification and the free-particle closed form.  With the fluid moments
// frozen and no contact force, the sub-step recurrence
//   U^{k+1} = U^k + h [cc (u* - U^k) + a],  cc = 2 A_p rho_i / m,  u* = j_i / rho_i
// has the solution U^k = U_eq + (U^0 - U_eq) q^k, q = 1 - h cc.  The free
// path then stays within B = max(|U^0|, |U^n|) (|U^k| is convex along the
// segment), and every particle moves at most skin/2 (else E_SKIN).  So a
// particle is provably free when every neighbour gap exceeds B + skin/2 and
// every wall gap exceeds B; the others are active and run the sub-steps.
// Active particles get a compact index and a candidate range in particle
// order: each block's totals of (active, candidates) go to bsum, one small
// scan turns them into block offsets, and k_collect adds the offsets within
// the block.
template <int D>
__global__ __launch_bounds__(256, 8) void k_classify(PState A, PState Bn, int np, PCfg c,
                                                  const uint32_t* __restrict__ start,
                                                  const float4* __restrict__ pos4,
                                                  const uint32_t* __restrict__ keys_sorted,
                                                  const float* __restrict__ drho_i, const float* __restrict__ j_i,
                                                  float* __restrict__ srec, float* __restrict__ fc,
                                                  unsigned long long* __restrict__ actcc,
                                                  unsigned long long* __restrict__ bsum,
                                                  uint32_t* __restrict__ counters, uint32_t* __restrict__ flags,
                                                  uint32_t* __restrict__ hcnt) {
    __shared__ unsigned long long sh4[4];
    const unsigned lb = xcd_block();
    const int s = lb * 256 + threadIdx.x;
    const bool valid = s < np;
    if (lb == 0 && threadIdx.x < CNT_SIZE) counters[threadIdx.x] = 0u;   // this step's counters
    bool active = false;
    uint32_t ncand = 0;
    if (valid) {
        // pos4 holds the leading position parts and the diameter of the
        // sorted particles (k_reorder): every per-particle load is issued here
        const float4 me = pos4[s];
        const uint32_t key = keys_sorted[s];
        float xl[3], jv[3], u0v[3];
#pragma unroll
        for (int a = 0; a < D; a++) {
            xl[a] = A.xl[a][s];
            jv[a] = j_i[(long long)a * np + s];
            u0v[a] = A.u[a][s];
        }
        const float d = me.w, rp = A.rp[s];
        float m = particle_mass(D, d, rp);
        float Ap = 0.25f * PI_F * d * d;
        float ri = 1.0f + drho_i[s];
        float cc = 2.0f * Ap * ri / m;
        float hc = cc * c.h;
        const bool fixedp = A.fixa && A.fixa[s] > 0.f;     // a point of a fixed body
        if (!(hc < 2.0f) && !fixedp) atomicOr(flags, FLAG_UNSTABLE);   // explicit drag diverges
        float qn, omq;                       // q^n, 1 - q^n
        drag_power(hc, c.n_sub, qn, omq);
        float geo = omq / hc;                // sum_{k<n} q^k
        float q = 1.0f - hc;
        float bw = 1.0f - c.rho0 / rp;
        float v0s = 0.f, vns = 0.f, ves = 0.f, dvs = 0.f;
        float un[3], dx[3], gb[3];
#pragma unroll
        for (int a = 0; a < D; a++) {
            float ustar = jv[a] / ri;
            float slip = bw * c.g[a] / cc;   // U_eq - u*
            float ueq = ustar + slip;
            float u0 = u0v[a];
            un[a] = ueq + (u0 - ueq) * qn;
            dx[a] = ueq + (u0 - ueq) * (c.h * q * geo);
            gb[a] = 2.0f * ri * (slip + (u0 - ueq) * (geo * c.h));
            v0s += u0 * u0;
            vns += un[a] * un[a];
            ves += ueq * ueq;
            dvs += (u0 - ueq) * (u0 - ueq);
        }
        if (fixedp) {
            // at rest: g = 2 (rho_i 0 - j_i) at every sub-step, spread with the point's own area
#pragma unroll
            for (int a = 0; a < D; a++) {
                un[a] = 0.f;
                dx[a] = 0.f;
                gb[a] = -2.0f * jv[a];
            }
            v0s = vns = ves = dvs = 0.f;
            Ap = A.fixa[s];
        }
        // q > 0: U^k moves along the segment from U^0 to U^n; q < 0: it
        // alternates around U_eq within |U^0 - U_eq|
        const float B = (q > 0.f) ? sqrtf(fmaxf(v0s, vns)) : sqrtf(ves) + sqrtf(dvs);
        const bool skin_out = B > 0.5f * c.skin;
        // The free result is written for every particle before the scan (the
        // island kernels overwrite it for the active ones), so that none of
        // it stays live across the scan.
        bool wall = false;
#pragma unroll
        for (int a = 0; a < D; a++) {
            float xh = a == 0 ? me.x : (a == 1 ? me.y : me.z), xla = xl[a];
            const float x = xh + xla;
            wall = wall || (x - 0.5f * d <= B) || (((float)c.n[a] - x) - 0.5f * d <= B);
            df_add(xh, xla, dx[a]);
            Bn.xh[a][s] = xh;
            Bn.xl[a][s] = xla;
            Bn.u[a][s] = un[a];
            srec[(long long)s * SRec<D>::STRIDE + SRec<D>::COEF + a] = Ap * gb[a];
            fc[(long long)a * np + s] = 0.f;
        }
        wall = wall && !fixedp;                             // fixed points feel no wall
        if (c.contact != PIBM_CONTACT_NONE) {
            bool close = false;
            const int cnt = count_neighbours<D>(pos4, start, me, key, c, s, B + 0.5f * c.skin, close, fixedp, A.fixa);
            if (close || wall) {
                if (cnt > c.maxc) atomicOr(flags, FLAG_CAPACITY);
                active = true;
                ncand = (uint32_t)min(cnt, c.maxc);
            }
        }
        if (!active) {
            if (hcnt) {
                // no contact: the spin is unchanged and no tangential force is carried
#pragma unroll
                for (int a = 0; a < 3; a++)
                    if (A.w[a]) Bn.w[a][s] = A.w[a][s];
                hcnt[A.id[s]] = 0u;
            }
            if (skin_out) atomicOr(flags, FLAG_SKIN);
        }
        actcc[s] = active ? ((1ULL << 32) | (unsigned long long)ncand) : 0ULL;
    }
    // block totals (every thread of the block takes part)
    const unsigned long long v = active ? ((1ULL << 32) | (unsigned long long)ncand) : 0ULL;
    unsigned long long tot;
    block_exclusive_scan<unsigned long long>(v, sh4, tot);
    if (threadIdx.x == 0) bsum[lb] = tot;
}

// active particles: compact index, candidate list (active partners only; a
// free partner provably never touches), union-find init.  RAW: bsum holds
// the blocks' unscanned totals and each block adds up those before it (for
// up to RAW_MAX_BLOCKS blocks; beyond, a one-block scan runs first).
template <int D, bool RAW>
__global__ __launch_bounds__(256) void k_collect(PState A, int np, PCfg c, const uint32_t* __restrict__ start,
                                                 const float4* __restrict__ pos4,
                                                 const uint32_t* __restrict__ keys_sorted,
                                                 const unsigned long long* __restrict__ actcc,
                                                 const unsigned long long* __restrict__ bsum,
                                                 unsigned long long* __restrict__ prefix,
                                                 uint32_t* __restrict__ alist, uint32_t* __restrict__ aidx,
                                                 uint32_t* __restrict__ cand, uint32_t* __restrict__ ccount,
                                                 uint32_t* __restrict__ parent, uint32_t* __restrict__ isize,
                                                 uint32_t* __restrict__ fill, uint32_t* __restrict__ counters) {
    __shared__ unsigned long long sh4[4];
    const unsigned lb = xcd_block();
    int s = lb * 256 + threadIdx.x;
    // A block without active particles has nothing to do (active particles
    // are a small share: those near walls or near each other).  RAW: bsum[lb]
    // is the block's total (block 0 still writes the grand totals below);
    // else bsum is scanned and the total is the step to the next block's
    // offset (the last block's: to the grand total in counters[0..1]).
    if (RAW) {
        if (lb != 0 && bsum[lb] == 0ULL) return;
    } else {
        const unsigned long long next = lb + 1 < gridDim.x ? bsum[lb + 1]
                                                            : *(const unsigned long long*)counters;
        if (next == bsum[lb]) return;
    }
    // bsum holds the blocks' (active << 32 | candidates) totals of k_classify:
    // this block's offset is the sum of those before it; block 0 also writes
    // the grand totals (candidates, active) to counters[0..1]
    const unsigned long long before = RAW ? block_sum<unsigned long long, 256>(bsum, (long long)lb, sh4) : bsum[lb];
    if (RAW && lb == 0) {
        const unsigned long long all = block_sum<unsigned long long, 256>(bsum, (long long)gridDim.x, sh4);
        if (threadIdx.x == 0) {
            counters[CNT_CAND] = (uint32_t)(all & 0xffffffffULL);
            counters[CNT_ACTIVE] = (uint32_t)(all >> 32);
        }
    }
    const unsigned long long v = s < np ? actcc[s] : 0ULL;
    unsigned long long tot;
    const unsigned long long p = block_exclusive_scan<unsigned long long>(v, sh4, tot) + before;
    if (s >= np || v == 0ULL) return;
    prefix[s] = p;
    uint32_t a = (uint32_t)(p >> 32), off = (uint32_t)(p & 0xffffffffULL);
    int cap = (int)(v & 0xffffffffULL);
    alist[a] = s;
    aidx[s] = a;
    parent[a] = a;
    isize[a] = 0;
    fill[a] = 0;
    int n = cap > 0 ? collect_neighbours<D>(pos4, start, keys_sorted, c, s, actcc, cand + off, cap, A.fixa) : 0;
    ccount[s] = (uint32_t)min(n, cap);
}

__device__ __forceinline__ uint32_t uf_find(uint32_t* parent, uint32_t x) {
    uint32_t p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
    while (p != x) {
        x = p;
        p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
    }
    return x;
}

// Union active particle a with its later candidates (the larger root is
// hooked under the smaller, so every island's root is its smallest index).
__device__ __forceinline__ void uf_hook_one(uint32_t a, const uint32_t* __restrict__ alist,
                                            const uint32_t* __restrict__ ccount,
                                            const unsigned long long* __restrict__ prefix,
                                            const uint32_t* __restrict__ cand, const uint32_t* __restrict__ aidx,
                                            uint32_t* parent) {
    uint32_t s = alist[a];
    uint32_t off = (uint32_t)(prefix[s] & 0xffffffffULL);
    int cnt = (int)ccount[s];
    for (int k = 0; k < cnt; k++) {
        uint32_t b = aidx[cand[off + k]];
        if (b <= a) continue;
        while (true) {
            uint32_t ra = uf_find(parent, a), rb = uf_find(parent, b);
            if (ra == rb) break;
            if (ra > rb) { uint32_t t = ra; ra = rb; rb = t; }
            if (atomicCAS(&parent[rb], rb, ra) == rb) break;
        }
    }
}

__global__ __launch_bounds__(256) void k_uf_hook(const uint32_t* __restrict__ alist,
                                                 const uint32_t* __restrict__ ccount,
                                                 const unsigned long long* __restrict__ prefix,
                                                 const uint32_t* __restrict__ cand, const uint32_t* __restrict__ aidx,
                                                 uint32_t* parent, const uint32_t* __restrict__ counters) {
    uint32_t na = counters[CNT_ACTIVE];
    for (uint32_t a = blockIdx.x * 256 + threadIdx.x; a < na; a += gridDim.x * 256)
        uf_hook_one(a, alist, ccount, prefix, cand, aidx, parent);
}

__global__ __launch_bounds__(256) void k_uf_flatten(uint32_t* parent, uint32_t* __restrict__ isize,
                                                    const uint32_t* __restrict__ counters) {
    uint32_t na = counters[CNT_ACTIVE];
    for (uint32_t a = blockIdx.x * 256 + threadIdx.x; a < na; a += gridDim.x * 256) {
        uint32_t r = uf_find(parent, a);
        parent[a] = r;
        atomicAdd(&isize[r], 1u);
    }
}

// Wave plan of the small-island size classes, computed by wave 0 of the
// block (one class per lane, then a wave scan): wb[s] = first wave of class
// s = 1..64 (a wave holds 64 / s islands of size s), wb[0] = all waves.
// cls[s] is the number of islands of size s.  The caller synchronises.
__device__ __forceinline__ void wave_plan(const uint32_t* cls, uint32_t* wb) {
    if (threadIdx.x < WAVE) {
        const uint32_t s = threadIdx.x + 1;
        const uint32_t per = WAVE / s;
        const uint32_t v = (cls[s] + per - 1) / per;
        const uint32_t inc = wave_inclusive_scan<uint32_t>(v);
        wb[s] = inc - v;
        if (s == WAVE) wb[0] = inc;
    }
}

// An island of two (root a) whose members touch at the start of the step,
// or would close their gap within the step at their present speeds: such a
// pair is likely to be in contact for most of the step, and so to take
// every sub-step.  These pairs are ranked apart (rank | TOUCH_BIT) and
// packed into the first waves of the class, so that they fill few waves;
// the pairs that can jump fill the rest.  (Only the packing depends on this
// test: an island's result does not depend on its wave.)
constexpr uint32_t TOUCH_BIT = 0x80000000u;
template <int D>
__device__ __forceinline__ bool pair_touching(uint32_t a, const PState& A, const uint32_t* __restrict__ alist,
                                              const uint32_t* __restrict__ ccount,
                                              const unsigned long long* __restrict__ prefix,
                                              const uint32_t* __restrict__ cand) {
    const uint32_t s = alist[a];
    if (ccount[s] == 0) return false;
    const uint32_t t = cand[(uint32_t)(prefix[s] & 0xffffffffULL)];
    float r2 = 0.f, us = 0.f, ut = 0.f;
#pragma unroll
    for (int ax = 0; ax < D; ax++) {
        const float e = (A.xh[ax][s] - A.xh[ax][t]) + (A.xl[ax][s] - A.xl[ax][t]);
        r2 += e * e;
        us += A.u[ax][s] * A.u[ax][s];
        ut += A.u[ax][t] * A.u[ax][t];
    }
    const float reach = 0.5f * (A.d[s] + A.d[t]) + sqrtf(us) + sqrtf(ut);
    return r2 < reach * reach;
}

// islands by size class: 1..64 packed into waves, 65 = larger than a wave
// (ranks within a class are counted in LDS per chunk of 256 and reserved
// with one global atomic per class and chunk: no contended counter)
template <int D>
__global__ __launch_bounds__(256) void k_island_class(PState A, const uint32_t* __restrict__ alist,
                                                      const uint32_t* __restrict__ ccount,
                                                      const unsigned long long* __restrict__ prefix,
                                                      const uint32_t* __restrict__ cand,
                                                      const uint32_t* __restrict__ parent,
                                                      const uint32_t* __restrict__ isize, uint32_t* __restrict__ irank,
                                                      uint32_t* __restrict__ bigroot, uint32_t* counters) {
    __shared__ uint32_t lc[WAVE + 3], gbase[WAVE + 3];     // [WAVE + 2]: touching pairs
    const uint32_t t = threadIdx.x;
    const uint32_t na = counters[CNT_ACTIVE];
    for (uint32_t c0 = blockIdx.x * 256; c0 < na; c0 += gridDim.x * 256) {
        if (t < WAVE + 3) lc[t] = 0;
        __syncthreads();
        const uint32_t a = c0 + t;
        uint32_t cls = 0, lr = 0;
        const bool root = a < na && parent[a] == a;
        if (root) {
            const uint32_t sz = isize[a];
            cls = sz <= WAVE ? sz : WAVE + 1;
            if (cls == 2 && pair_touching<D>(a, A, alist, ccount, prefix, cand)) cls = WAVE + 2;
            lr = atomicAdd(&lc[cls], 1u);
        }
        __syncthreads();
        if (t < WAVE + 2 && lc[t] > 0) gbase[t] = atomicAdd(&counters[CNT_CLASS + t], lc[t]);
        if (t == WAVE + 2 && lc[t] > 0) gbase[t] = atomicAdd(&counters[CNT_PAIRC], lc[t]);
        __syncthreads();
        if (root) {
            const uint32_t r = gbase[cls] + lr;
            irank[a] = cls == WAVE + 2 ? (r | TOUCH_BIT) : r;
            if (cls == WAVE + 1) bigroot[r] = a;
        }
        __syncthreads();
    }
}



// Lane (small islands, packed by size into waves) or slot (large islands)
// of active particle a; wavebase[s] = first wave of size class s.
__device__ __forceinline__ void island_place_one(uint32_t a, const uint32_t* __restrict__ parent,
                                                 const uint32_t* __restrict__ isize,
                                                 const uint32_t* __restrict__ irank, uint32_t* __restrict__ fill,
                                                 int* __restrict__ lanemember, uint32_t* __restrict__ loc,
                                                 const uint32_t* __restrict__ bigoff,
                                                 uint32_t* __restrict__ bigmember, const uint32_t* wavebase,
                                                 uint32_t ntouch) {
    uint32_t r = parent[a];
    uint32_t pos = atomicAdd(&fill[r], 1u);
    uint32_t sz = isize[r];
    if (sz <= WAVE) {
        // islands of two: the ntouch touching pairs first
        uint32_t ir = irank[r];
        if (sz == 2) ir = (ir & TOUCH_BIT) ? (ir & ~TOUCH_BIT) : ir + ntouch;
        uint32_t per = WAVE / sz;
        uint32_t w = wavebase[sz] + ir / per;
        uint32_t lane = (ir % per) * sz + pos;
        lanemember[(long long)w * WAVE + lane] = (int)a;
        loc[a] = lane;
    } else {
        bigmember[bigoff[irank[r]] + pos] = a;
        loc[a] = a;
    }
}

// Every block first forms the wave plan and the large-island offsets itself
// (a few hundred loads; it saves a one-block launch); block 0 stores the
// plan for the sub-step kernels, and every block writes the same offsets.
__global__ __launch_bounds__(256) void k_island_place(const uint32_t* __restrict__ parent,
                                                      const uint32_t* __restrict__ isize,
                                                      const uint32_t* __restrict__ irank, uint32_t* __restrict__ fill,
                                                      int* __restrict__ lanemember, uint32_t* __restrict__ loc,
                                                      uint32_t* __restrict__ bigoff,
                                                      uint32_t* __restrict__ bigmember,
                                                      const uint32_t* __restrict__ bigroot,
                                                      uint32_t* __restrict__ counters) {
    __shared__ uint32_t wb[WAVE + 1];
    __shared__ uint32_t scan4[4];
    __shared__ uint32_t cls[WAVE + 1];
    const uint32_t ntouch = counters[CNT_PAIRC];
    if (threadIdx.x <= WAVE) cls[threadIdx.x] = counters[CNT_CLASS + threadIdx.x] + (threadIdx.x == 2 ? ntouch : 0u);
    __syncthreads();
    wave_plan(cls, wb);
    const uint32_t nbig = counters[CNT_CLASS + WAVE + 1];
    uint32_t run = 0;
    for (uint32_t k0 = 0; k0 < nbig; k0 += 256) {
        const uint32_t k = k0 + threadIdx.x;
        const uint32_t v = k < nbig ? isize[bigroot[k]] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<uint32_t>(v, scan4, tot);
        if (k < nbig) bigoff[k] = run + ex;
        run += tot;
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int s = 1; s <= WAVE; s++) counters[CNT_WAVEBASE + s] = wb[s];
        counters[CNT_WAVES] = wb[0];
        counters[CNT_BIG] = nbig;
    }
    const uint32_t na = counters[CNT_ACTIVE];
    for (uint32_t a = blockIdx.x * 256 + threadIdx.x; a < na; a += gridDim.x * 256)
        island_place_one(a, parent, isize, irank, fill, lanemember, loc, bigoff, bigmember, wb, ntouch);
}

// Candidate constants for the sub-steps.  K0 = r_c^2 - |r0|^2 is formed in
// double-float so that overlaps far below the FP32 spacing of positions
// (1e-9 .. 1e-6 for stiff springs and slow particles) stay resolved.
template <int D>
__device__ __forceinline__ void cand_prep_one(uint32_t a, const PState& A, const PCfg& c,
                                              const uint32_t* __restrict__ alist,
                                              const uint32_t* __restrict__ ccount,
                                              const unsigned long long* __restrict__ prefix,
                                              const uint32_t* __restrict__ cand, const uint32_t* __restrict__ aidx,
                                              const uint32_t* __restrict__ loc, CandData* __restrict__ cdata,
                                              MdBuf md) {
#pragma clang fp contract(off)
    uint32_t s = alist[a];
    uint32_t off = (uint32_t)(prefix[s] & 0xffffffffULL);
    int cnt = (int)ccount[s];
    float ms = particle_mass(D, A.d[s], A.rp[s]);
    for (int k = 0; k < cnt; k++) {
        uint32_t t = cand[off + k];
        CandData cd;
        cd.local = (int)loc[aidx[t]];
        // r0 = X_s - X_t in double-float, |r0|^2 in double-float
        float sh = 0.f, sl = 0.f;
        float r0[3] = {0, 0, 0};
#pragma unroll
        for (int ax = 0; ax < D; ax++) {
            float hi, e;
            two_sum(A.xh[ax][s], -A.xh[ax][t], hi, e);
            float lo = e + (A.xl[ax][s] - A.xl[ax][t]);
            float rh, rl;
            fast_two_sum(hi, lo, rh, rl);
            r0[ax] = rh;
            // (rh + rl)^2 = rh^2 + 2 rh rl (+ rl^2, negligible)
            float p = rh * rh;
            float pe = fmaf(rh, rh, -p);
            pe = fmaf(2.0f * rh, rl, pe);
            float ns, ne;
            two_sum(sh, p, ns, ne);
            sl += ne + pe;
            sh = ns;
        }
        // r_c = (d_s + d_t)/2 exactly as a double-float, then r_c^2
        float dsum, derr;
        two_sum(A.d[s], A.d[t], dsum, derr);
        float rch = 0.5f * dsum, rcl = 0.5f * derr;
        float q = rch * rch;
        float qe = fmaf(rch, rch, -q);
        qe = fmaf(2.0f * rch, rcl, qe);
        // K0 = (q + qe) - (sh + sl)
        float k0h, k0e;
        two_sum(q, -sh, k0h, k0e);
        cd.K0 = k0h + (k0e + (qe - sl));
        cd.rc = rch;
        cd.r0[0] = r0[0]; cd.r0[1] = r0[1]; cd.r0[2] = r0[2];
        if (c.contact == PIBM_CONTACT_HERTZ || c.contact >= PIBM_CONTACT_HERTZ_MINDLIN) {
            // Hertz: gam holds the pair's stiffness (4/3) E* sqrt(R*)
            const float rs = 0.5f * A.d[s], rt = 0.5f * A.d[t];
            const float rstar = rs * rt / (rs + rt);
            cd.gam = c.hk * sqrtf(rstar);
            if (md.cmd) {
                // the tangential force this pair carried at the end of the last step
                const int pid = A.id[t];
                const long long base = (long long)A.id[s] * c.hmax;
                const uint32_t hn = md.hcnt[A.id[s]];
                float S[TSN];
#pragma unroll
                for (int q = 0; q < TSN; q++) S[q] = 0.f;
                for (uint32_t e = 0; e < hn; e++)
                    if (md.hkey[base + e] == pid) {
#pragma unroll
                        for (int q = 0; q < TSN; q++) S[q] = md.hT[TSN * (base + e) + q];
                        break;
                    }
                md.cmd[off + k] = make_float4(S[0], S[1], S[2], c.kt8 * sqrtf(rstar));
                md.cms[2 * (off + k)] = make_float4(S[3], S[4], S[5], S[9]);
                md.cms[2 * (off + k) + 1] = make_float4(S[6], S[7], S[8], 0.f);
                md.cpid[off + k] = pid;
            }
        } else {
            float mt = particle_mass(D, A.d[t], A.rp[t]);
            float meff = ms * mt / (ms + mt);
            if (A.fixa) {                            // a fixed partner has infinite mass
                if (A.fixa[t] > 0.f) meff = ms;
                else if (A.fixa[s] > 0.f) meff = mt;
            }
            cd.gam = 2.0f * c.zeta * sqrtf(c.kn * meff);
        }
        cdata[off + k] = cd;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_cand_prep(PState A, PCfg c, const uint32_t* __restrict__ alist,
                                                   const uint32_t* __restrict__ ccount,
                                                   const unsigned long long* __restrict__ prefix,
                                                   const uint32_t* __restrict__ cand, const uint32_t* __restrict__ aidx,
                                                   const uint32_t* __restrict__ loc, CandData* __restrict__ cdata,
                                                   MdBuf md, const uint32_t* __restrict__ counters) {
    uint32_t na = counters[CNT_ACTIVE];
    for (uint32_t a = blockIdx.x * 256 + threadIdx.x; a < na; a += gridDim.x * 256)
        cand_prep_one<D>(a, A, c, alist, ccount, prefix, cand, aidx, loc, cdata, md);
}

// The whole island set-up of one step in one 1024-thread workgroup, phase
// after phase (for a few active particles this replaces five short
// launches): union the candidates, flatten
// and size the islands, class them by size, plan the waves, place every
// member, and prepare the candidate constants.  Same results as the
// multi-kernel chain (roots are the smallest index; sub-step results do not
// depend on lane placement).
constexpr int SETUP_THREADS = 1024;
template <int D>
__global__ __launch_bounds__(SETUP_THREADS) void k_island_setup(
    PState A, PCfg c, const uint32_t* __restrict__ alist, const uint32_t* __restrict__ ccount,
    const unsigned long long* __restrict__ prefix, const uint32_t* __restrict__ cand,
    const uint32_t* __restrict__ aidx, uint32_t* parent, uint32_t* isize, uint32_t* irank, uint32_t* fill,
    int* lanemember, uint32_t* loc, uint32_t* bigroot, uint32_t* bigoff, uint32_t* bigmember, CandData* cdata, MdBuf md,
    uint32_t* counters, long long lane_cap) {
    __shared__ uint32_t ccls[WAVE + 3];     // [WAVE + 2]: touching pairs
    __shared__ uint32_t wbase[WAVE + 1];
    __shared__ uint32_t nwaves;
    const uint32_t t = threadIdx.x;
    const uint32_t na = counters[CNT_ACTIVE];
    if (t < WAVE + 3) ccls[t] = 0;
    __syncthreads();
    for (uint32_t a = t; a < na; a += SETUP_THREADS) uf_hook_one(a, alist, ccount, prefix, cand, aidx, parent);
    __syncthreads();
    for (uint32_t a = t; a < na; a += SETUP_THREADS) {
        uint32_t r = uf_find(parent, a);
        parent[a] = r;
        atomicAdd(&isize[r], 1u);
    }
    __syncthreads();
    for (uint32_t a = t; a < na; a += SETUP_THREADS) {
        if (parent[a] != a) continue;
        uint32_t sz = isize[a];
        uint32_t cls = sz <= WAVE ? sz : WAVE + 1;
        if (cls == 2 && pair_touching<D>(a, A, alist, ccount, prefix, cand)) cls = WAVE + 2;
        uint32_t r = atomicAdd(&ccls[cls], 1u);
        irank[a] = cls == WAVE + 2 ? (r | TOUCH_BIT) : r;
        if (cls == WAVE + 1) bigroot[r] = a;
    }
    __syncthreads();
    const uint32_t ntouch = ccls[WAVE + 2];
    if (t == 0) ccls[2] += ntouch;
    __syncthreads();
    wave_plan(ccls, wbase);
    __syncthreads();
    if (t < WAVE) {
        counters[CNT_WAVEBASE + t + 1] = wbase[t + 1];
        counters[CNT_CLASS + t + 1] = ccls[t + 1];
    }
    if (t == 0) {
        nwaves = wbase[0];
        counters[CNT_WAVES] = wbase[0];
        const uint32_t nbig = ccls[WAVE + 1];
        counters[CNT_CLASS + WAVE + 1] = nbig;
        counters[CNT_BIG] = nbig;
        uint32_t off = 0;
        for (uint32_t k = 0; k < nbig; k++) {
            bigoff[k] = off;
            off += isize[bigroot[k]];
        }
    }
    __syncthreads();
    for (uint32_t a = t; a < na; a += SETUP_THREADS)
        island_place_one(a, parent, isize, irank, fill, lanemember, loc, bigoff, bigmember, wbase, ntouch);
    __syncthreads();
    for (uint32_t a = t; a < na; a += SETUP_THREADS)
        cand_prep_one<D>(a, A, c, alist, ccount, prefix, cand, aidx, loc, cdata, md);
}

// ---------------------------------------------------------------------------
// Active sub-steps.  Jacobi: every force of sub-step k uses the state at k.
// ---------------------------------------------------------------------------
template <int D>
struct Active {
    float xh[3], xl[3];     // start-of-step position
    float dx[3], cdx[3];    // displacement in the step and its compensation
    float u[3], cu[3];      // velocity and its compensation
    float ri, j[3];
    float m, Ap, bw[3], d, gw;
    float hm, hbw[3];       // h / m and h (1 - rho0/rho_p) g: the update without a division
    float lq, ihc;          // log(1 - hc) (when hc < 1) and 1 / hc, for the closed-form jumps
    float gs[3], fs[3];     // sums of g and of the contact force
    float vmax2;
    uint32_t off;
    int cnt;
    bool wall;              // a wall lies within contact distance + skin
    // contact-free closed form: U_eq = u* + slip, q = 1 - hc
    float ueq[3], slip[3], hc, veq;
    // Hertz-Mindlin only: angular velocity (2D: z), the tangential force of
    // the wall contact of each axis (bit a of wside: the upper wall), moment
    // of inertia, radius, id
    float W[3];
    float wT[3][TSN];       // tangential state of the wall contact of each axis
    uint32_t wside;
    float I, R, hI;         // hI = h / I
    int id;
    // a point of a fixed body: never moves, spreads with its own area Af
    bool fixed;
    float Af;
};

__device__ __forceinline__ void cross3(const float* x, const float* y, float* z) {
    z[0] = x[1] * y[2] - x[2] * y[1];
    z[1] = x[2] * y[0] - x[0] * y[2];
    z[2] = x[0] * y[1] - x[1] * y[0];
}

// Turn v into the contact plane of unit normal n, keeping its length.
__device__ __forceinline__ void into_plane(const float* n, float* v) {
    const float vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
    const float old = sqrt_fast(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    float P[3];
#pragma unroll
    for (int a = 0; a < 3; a++) P[a] = v[a] - vn * n[a];
    const float pl2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
    const float sp = pl2 > 0.f ? old * rsq_fast(pl2) : 0.f;
#pragma unroll
    for (int a = 0; a < 3; a++) v[a] = P[a] * sp;
}

// Tangential state of one contact, one sub-step (Sec. 2.3).  n: unit normal
// from the partner to the particle; vrel: contact-point velocity relative to
// the partner's; S: the TSN-float state (T first).  The elastic trial
// increment is E = -k_t h v_t.  No-slip limit (theta_k = 1): T += E.  With
// micro-slip: dT = theta_k E + (-1)^k mu dF_n (1 - theta_k) t along the
// contact's loading direction t (set by its first tangential increment):
// the part e = E.t along t grows by theta_k e + (-1)^k mu dF_n (1 - theta_k),
// the part across t elastically, with theta_k^3 = 1 - (T_t + mu dF_n)/(mu F_n)
// when loading (k = 0), 1 - (T* - T_t + 2 mu dF_n)/(2 mu F_n) unloading
// (k = 1), 1 - (T_t - T** + 2 mu dF_n)/(2 mu F_n) reloading (k = 2), clamped
// to [0, 1]; k turns where e changes sign, a reloading that reaches T* is
// loading again, and the step is elastic while |e| <= mu dF_n.  Finally
// |T| <= mu F_n.
__device__ __forceinline__ void tangential_update(const PCfg& c, const float* n, const float* vrel, float Fn,
                                                  float kt, float* S) {
    float* T = S;
    into_plane(n, T);
    const float vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    float E[3];
#pragma unroll
    for (int a = 0; a < 3; a++) E[a] = -kt * c.h * (vrel[a] - vn * n[a]);
    if (c.microslip) {
        float* t = S + 3;
        // the loading direction is turned into the plane and kept at unit
        // length: carrying its length like T's would let FP32 rounding
        // random-walk it, and the law weighs every increment by it
        {
            const float tn = t[0] * n[0] + t[1] * n[1] + t[2] * n[2];
#pragma unroll
            for (int a = 0; a < 3; a++) t[a] -= tn * n[a];
            const float q2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
            const float iq = q2 > 0.f ? rsq_fast(q2) : 0.f;
#pragma unroll
            for (int a = 0; a < 3; a++) t[a] *= iq;
        }
        const float dFn = Fn - S[9];
        S[9] = Fn;
        const float el2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
        float tl2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        if (tl2 == 0.f && el2 > 0.f) {                   // the first tangential increment sets t
            const float ie = rsq_fast(el2);
#pragma unroll
            for (int a = 0; a < 3; a++) t[a] = E[a] * ie;
            S[6] = S[7] = S[8] = 0.f;
            tl2 = 1.f;
        }
        if (tl2 > 0.f) {
            const float Tt = T[0] * t[0] + T[1] * t[1] + T[2] * t[2];
            const float e = E[0] * t[0] + E[1] * t[1] + E[2] * t[2];
            int k = (int)S[6];
            if (k == 0 && e < 0.f) {
                k = 1;
                S[7] = Tt;
            } else if (k == 1 && e > 0.f) {
                k = 2;
                S[8] = Tt;
            } else if (k == 2) {
                if (e < 0.f) {
                    k = 1;
                    S[7] = Tt;
                } else if (Tt >= S[7]) {
                    k = 0;
                }
            }
            S[6] = (float)k;
            const float mdf = c.mu * dFn;
            if (dFn > 0.f && fabsf(e) <= mdf) {
#pragma unroll
                for (int a = 0; a < 3; a++) T[a] += E[a];
            } else {
                const float num = k == 0 ? Tt + mdf : (k == 1 ? S[7] - Tt + 2.0f * mdf : Tt - S[8] + 2.0f * mdf);
                const float den = (k == 0 ? 1.0f : 2.0f) * c.mu * Fn;
                const float arg = fminf(fmaxf(1.0f - num / den, 0.0f), 1.0f);
                const float th = cbrtf(arg);
                const float sg = k == 1 ? -mdf : mdf;
                const float dt = th * e + sg * (1.0f - th);          // along t
#pragma unroll
                for (int a = 0; a < 3; a++) T[a] += dt * t[a] + (E[a] - e * t[a]);
            }
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; a++) T[a] += E[a];
    }
    const float tl2 = T[0] * T[0] + T[1] * T[1] + T[2] * T[2];
    const float lim = c.mu * Fn;
    if (tl2 > lim * lim) {
        const float sc = lim * rsq_fast(tl2);
#pragma unroll
        for (int a = 0; a < 3; a++) T[a] *= sc;
    }
}

template <int D, bool MD>
__device__ __forceinline__ void active_load(Active<D>& P, const PState& A, const PCfg& c, uint32_t s,
                                            const float* drho_i, const float* j_i, int np,
                                            const uint32_t* ccount, const unsigned long long* prefix,
                                            const MdBuf& md) {
    P.d = A.d[s];
    float rp = A.rp[s];
    P.m = particle_mass(D, P.d, rp);
    P.Ap = 0.25f * PI_F * P.d * P.d;
    P.ri = 1.0f + drho_i[s];
    // wall dashpot coefficient, or the Hertz wall stiffness (4/3) E* sqrt(R_p)
    const bool hertz = c.contact == PIBM_CONTACT_HERTZ || c.contact >= PIBM_CONTACT_HERTZ_MINDLIN;
    P.gw = hertz ? c.hk * sqrtf(0.5f * P.d) : 2.0f * c.zeta * sqrtf(c.kn * P.m);
    float v2 = 0.f;
    bool wall = false;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        bool on = a < D;
        P.xh[a] = on ? A.xh[a][s] : 0.f;
        P.xl[a] = on ? A.xl[a][s] : 0.f;
        P.u[a] = on ? A.u[a][s] : 0.f;
        P.j[a] = on ? j_i[(long long)a * np + s] : 0.f;
        P.bw[a] = on ? (1.0f - c.rho0 / rp) * c.g[a] : 0.f;
        P.dx[a] = P.cdx[a] = P.cu[a] = 0.f;
        P.gs[a] = P.fs[a] = 0.f;
        v2 += P.u[a] * P.u[a];
        if (on) {
            float x = P.xh[a] + P.xl[a];
            wall = wall || (x - 0.5f * P.d < c.skin) || (((float)c.n[a] - x) - 0.5f * P.d < c.skin);
        }
    }
    // a wall farther than skin cannot be reached (displacement <= skin/2)
    P.wall = wall && c.contact != PIBM_CONTACT_NONE;
    const float cc = 2.0f * P.Ap * P.ri / P.m;
    P.hc = cc * c.h;
    float ve = 0.f;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        P.slip[a] = P.bw[a] / cc;
        P.ueq[a] = (a < D ? P.j[a] / P.ri : 0.f) + P.slip[a];
        ve += P.ueq[a] * P.ueq[a];
    }
    P.veq = sqrtf(ve);
    P.vmax2 = v2;
    P.hm = c.h / P.m;
#pragma unroll
    for (int a = 0; a < 3; a++) P.hbw[a] = c.h * P.bw[a];
    P.lq = P.hc < 1.0f ? log1pf(-P.hc) : 0.f;
    P.ihc = 1.0f / P.hc;
    P.off = (uint32_t)(prefix[s] & 0xffffffffULL);
    P.cnt = c.contact != PIBM_CONTACT_NONE ? (int)ccount[s] : 0;
    P.fixed = A.fixa && A.fixa[s] > 0.f;
    P.Af = P.fixed ? A.fixa[s] : P.Ap;
    if (P.fixed) {
        // at rest for good: no wall, no drift, no contact-free motion
        P.wall = false;
        P.hc = 0.f;
        P.veq = 0.f;
#pragma unroll
        for (int a = 0; a < 3; a++) P.ueq[a] = P.slip[a] = P.u[a] = 0.f;
        P.vmax2 = 0.f;
    }
    if (MD) {
        P.R = 0.5f * P.d;
        P.I = (D == 3 ? 0.4f : 0.5f) * P.m * P.R * P.R;
        P.hI = c.h / P.I;
        P.W[0] = D == 3 ? A.w[0][s] : 0.f;
        P.W[1] = D == 3 ? A.w[1][s] : 0.f;
        P.W[2] = D == 3 ? A.w[2][s] : A.w[0][s];
        P.id = A.id[s];
        P.wside = 0u;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int q = 0; q < TSN; q++) P.wT[a][q] = 0.f;
        // wall contacts carried over from the last step
        const long long base = (long long)P.id * c.hmax;
        const uint32_t hn = md.hcnt[P.id];
        for (uint32_t e = 0; e < hn; e++) {
            const int key = md.hkey[base + e];
            if (key >= 0) continue;
            const int code = -1 - key, a = code >> 1;
#pragma unroll
            for (int ax = 0; ax < D; ax++)
                if (ax == a) {
#pragma unroll
                    for (int q = 0; q < TSN; q++) P.wT[ax][q] = md.hT[TSN * (base + e) + q];
                    P.wside |= (uint32_t)(code & 1) << ax;
                }
        }
    }
}

// Hertz-Mindlin wall contacts: Hertz normal force with R* = R, tangential
// force on the contact point at -R n, its torque.
template <int D>
__device__ __forceinline__ void wall_force_md(Active<D>& P, const PCfg& c, float* F, float* tq) {
    const float rc = 0.5f * P.d;
#pragma unroll
    for (int a = 0; a < D; a++) {
        const float dlo = ((rc - P.xh[a]) - P.xl[a]) - P.dx[a];
        const float dhi = ((rc - ((float)c.n[a] - P.xh[a])) + P.xl[a]) + P.dx[a];
        const bool lo = dlo > 0.f, hi = !lo && dhi > 0.f;
        if (!lo && !hi) {
#pragma unroll
            for (int q = 0; q < TSN; q++) P.wT[a][q] = 0.f;       // out of contact: no state
            continue;
        }
        const uint32_t side = hi ? 1u : 0u;
        if (((P.wside >> a) & 1u) != side) {
#pragma unroll
            for (int q = 0; q < TSN; q++) P.wT[a][q] = 0.f;
            P.wside ^= 1u << a;
        }
        const float delta = lo ? dlo : dhi;
        float n[3] = {0.f, 0.f, 0.f};
        n[a] = lo ? 1.0f : -1.0f;              // from the wall to the particle
        const float Fn = P.gw * delta * sqrt_fast(delta);
        float arm[3], wr[3], vrel[3];
#pragma unroll
        for (int b = 0; b < 3; b++) arm[b] = -P.R * n[b];
        cross3(P.W, arm, wr);
#pragma unroll
        for (int b = 0; b < 3; b++) vrel[b] = (b < D ? P.u[b] : 0.f) + wr[b];
        tangential_update(c, n, vrel, Fn, c.kt8 * sqrt_fast(delta * P.R), P.wT[a]);
        float t[3];
        cross3(arm, P.wT[a], t);
#pragma unroll
        for (int b = 0; b < 3; b++) {
            if (b < D) F[b] += Fn * n[b] + P.wT[a][b];
            tq[b] += t[b];
        }
    }
}

// The wall force along one axis on a particle of diameter d (wall
// coefficient gw) with velocity u along it, from the overlaps dlo with the
// lower wall at 0 (d/2 - X) and dhi with the upper wall at n (d/2 - (n - X)).
// CT: the contact model when known at compile time (-1: read from c).
template <int CT>
__device__ __forceinline__ float wall_axis(const PCfg& c, float gw, float d, float dlo, float dhi, float u, float F) {
    const int ct = CT < 0 ? c.contact : CT;
    if (ct == PIBM_CONTACT_LSD) {
        if (dlo > 0.f) F += c.kn * dlo - gw * u;
        if (dhi > 0.f) F -= c.kn * dhi + gw * u;
    } else if (ct == PIBM_CONTACT_HERTZ) {
        if (dlo > 0.f) F += gw * dlo * sqrt_fast(dlo);
        if (dhi > 0.f) F -= gw * dhi * sqrt_fast(dhi);
    } else {
        const float irc = rcp_fast(0.5f * d);
        if (dlo > 0.f) { float q = dlo * irc; F += c.ks * q * q; }
        if (dhi > 0.f) { float q = dhi * irc; F -= c.ks * q * q; }
    }
    return F;
}

// The overlap offsets of the lower and upper wall along axis a: the
// overlaps at displacement dx are elo - dx and ehi + dx.
template <int D>
__device__ __forceinline__ void wall_offsets(const Active<D>& P, const PCfg& c, int a, float& elo, float& ehi) {
    const float rc = 0.5f * P.d;
    elo = (rc - P.xh[a]) - P.xl[a];
    ehi = (rc - ((float)c.n[a] - P.xh[a])) + P.xl[a];
}

template <int D, int CT = -1>
__device__ __forceinline__ void wall_force(const Active<D>& P, const PCfg& c, float* F) {
#pragma unroll
    for (int a = 0; a < D; a++) {
        float elo, ehi;
        wall_offsets<D>(P, c, a, elo, ehi);
        F[a] = wall_axis<CT>(c, P.gw, P.d, elo - P.dx[a], ehi + P.dx[a], P.u[a], F[a]);
    }
}

// The sum of a vector's D components in the fixed order (x + y) + z.
template <int D>
__device__ __forceinline__ float sum_d(const float* p) {
#pragma clang fp contract(off)
    float v = p[0] + p[1];
    if (D == 3) v = v + p[2];
    return v;
}

// The geometry of a pair contact: del is this particle's displacement in
// the step minus the candidate's.  Out of contact: false.  Otherwise
// r = r0 + del, inv = 1/|r| and delta = r_c - |r| (the overlap).  FLAT: no
// early return (the outputs are then meaningless out of contact).
template <int D, bool FLAT = false>
__device__ __forceinline__ bool pair_geom(const CandData& cd, const float* del, float* r, float& inv, float& delta) {
    float rd = 0.f, dd = 0.f;
#pragma unroll
    for (int a = 0; a < D; a++) {
        r[a] = cd.r0[a] + del[a];
        rd += cd.r0[a] * del[a];
        dd += del[a] * del[a];
    }
    float num = cd.K0 - (2.0f * rd + dd);        // r_c^2 - |r|^2
    if (!FLAT && !(num > 0.f)) return false;
    float r2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; a++) r2 += r[a] * r[a];
    inv = rsq_fast(r2);                          // 1 / |r|
    const float dist = r2 * inv;
    delta = num * rcp_fast(cd.rc + dist);        // r_c - |r|
    return num > 0.f;
}

// The normal force magnitude at overlap delta; vn (read by the dashpot
// only) is the normal component of this particle's velocity relative to
// the candidate's, sum_d of (u - u_c)_a n_a.
template <int CT>
__device__ __forceinline__ float pair_mag(const CandData& cd, const PCfg& c, float delta, float vn) {
    const int ct = CT < 0 ? c.contact : CT;
    if (ct == PIBM_CONTACT_LSD) return c.kn * delta - cd.gam * vn;
    if (ct == PIBM_CONTACT_HERTZ) return cd.gam * delta * sqrt_fast(delta);
    const float q = delta * rcp_fast(cd.rc);
    return c.ks * q * q;
}

template <int D, int CT = -1>
__device__ __forceinline__ void pair_force(const Active<D>& P, const CandData& cd, const float* odx,
                                           const float* ou, const PCfg& c, float* F) {
    const int ct = CT < 0 ? c.contact : CT;
    float del[3] = {0, 0, 0}, r[3], inv, delta;
#pragma unroll
    for (int a = 0; a < D; a++) del[a] = P.dx[a] - odx[a];
    if (!pair_geom<D>(cd, del, r, inv, delta)) return;
    float n[3] = {0, 0, 0}, p[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; a++) n[a] = r[a] * inv;
    float vn = 0.f;
    if (ct == PIBM_CONTACT_LSD) {
#pragma unroll
        for (int a = 0; a < D; a++) p[a] = (P.u[a] - ou[a]) * n[a];
        vn = sum_d<D>(p);
    }
    const float mag = pair_mag<CT>(cd, c, delta, vn);
#pragma unroll
    for (int a = 0; a < D; a++) F[a] += mag * n[a];
}

// Hertz-Mindlin pair contact: Hertz normal force, tangential force T
// (carried in cmd, the force on this particle), torque of T about the
// centre.  Partner spin ow; contact point at -R_self n from this centre and
// at +R_partner n from the partner's.
template <int D>
__device__ __forceinline__ void pair_force_md(const Active<D>& P, const CandData& cd, float4* __restrict__ cmd,
                                              float4* __restrict__ cms, const float* odx, const float* ou,
                                              const float* ow, const PCfg& c, float* F, float* tq) {
    float r[3] = {0, 0, 0};
    float rd = 0.f, dd = 0.f;
#pragma unroll
    for (int a = 0; a < D; a++) {
        const float del = P.dx[a] - odx[a];
        r[a] = cd.r0[a] + del;
        rd += cd.r0[a] * del;
        dd += del * del;
    }
    const float num = cd.K0 - (2.0f * rd + dd);          // r_c^2 - |r|^2
    float4 m = *cmd;
    if (!(num > 0.f)) {
        // out of contact: no tangential state
        if (m.x != 0.f || m.y != 0.f || m.z != 0.f) *cmd = make_float4(0.f, 0.f, 0.f, m.w);
        if (c.microslip) {
            cms[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            cms[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        return;
    }
    float r2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; a++) r2 += r[a] * r[a];
    const float inv = rsq_fast(r2);                      // 1 / |r|
    const float dist = r2 * inv;
    const float delta = num * rcp_fast(cd.rc + dist);    // r_c - |r|
    float n[3], as[3], at[3], ws[3], wt[3], vrel[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        n[a] = r[a] * inv;
        as[a] = -P.R * n[a];
        at[a] = (cd.rc - P.R) * n[a];
    }
    cross3(P.W, as, ws);
    cross3(ow, at, wt);
#pragma unroll
    for (int a = 0; a < 3; a++) vrel[a] = (((a < D ? P.u[a] : 0.f) - ou[a]) + ws[a]) - wt[a];
    const float sd = sqrt_fast(delta);
    const float Fn = cd.gam * delta * sd;
    float T[TSN] = {m.x, m.y, m.z, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (c.microslip) {
        const float4 s0 = cms[0], s1 = cms[1];
        T[3] = s0.x; T[4] = s0.y; T[5] = s0.z; T[9] = s0.w;
        T[6] = s1.x; T[7] = s1.y; T[8] = s1.z;
    }
    tangential_update(c, n, vrel, Fn, m.w * sd, T);
    *cmd = make_float4(T[0], T[1], T[2], m.w);
    if (c.microslip) {
        cms[0] = make_float4(T[3], T[4], T[5], T[9]);
        cms[1] = make_float4(T[6], T[7], T[8], 0.f);
    }
    float t[3];
    cross3(as, T, t);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (a < D) F[a] += Fn * n[a] + T[a];
        tq[a] += t[a];
    }
}

// Candidate k of a particle: the first n1 from `first`, the rest from global
// memory.  With LDS (the small-island waves cache their first candidates in
// LDS) the first ones are read through an LDS pointer: a select between an
// LDS and a global pointer would turn every read into a much slower
// generic-address one.
template <bool LDS>
__device__ __forceinline__ CandData cand_at(const CandData* first, int n1, const CandData* __restrict__ rest,
                                            int k) {
    if constexpr (LDS) {
        using LC = const __attribute__((address_space(3))) CandData;
        LC* f = (LC*)first;
        const int i = k < n1 ? k : 0;
        CandData v;
        v.local = f[i].local;
        v.r0[0] = f[i].r0[0];
        v.r0[1] = f[i].r0[1];
        v.r0[2] = f[i].r0[2];
        v.K0 = f[i].K0;
        v.rc = f[i].rc;
        v.gam = f[i].gam;
        if (k >= n1) v = rest[k];
        return v;
    } else {
        return k < n1 ? first[k] : rest[k];
    }
}

// One sub-step for particle P.  Partner states are read through arrays
// (sdx, su, and with MD the spins sw) of stride `stride` indexed by the
// candidate's local index; the first nfirst candidates come from `first`
// (an LDS copy), the rest from `rest` (global).
template <int D, bool MD>
__device__ __forceinline__ void substep_update(Active<D>& P, const PCfg& c, const float* F, const float* tq);

template <int D, bool MD, bool LDS = false>
__device__ __forceinline__ void active_substep(Active<D>& P, const PCfg& c, const CandData* first, int nfirst,
                                               const CandData* __restrict__ rest, const float* sdx,
                                               const float* su, const float* sw, int stride, const MdBuf& md) {
    float F[3] = {0.f, 0.f, 0.f}, tq[3] = {0.f, 0.f, 0.f};
    if (P.wall) {
        if (MD) wall_force_md<D>(P, c, F, tq);
        else wall_force<D>(P, c, F);
    }
    const int n1 = min(P.cnt, nfirst);
    // the next candidate and its partner's state are loaded while the
    // current one is evaluated (a sub-step is a serial latency chain when few
    // islands are left); the partner states do not change within a sub-step
    CandData nx{};
    float ndx[3] = {0, 0, 0}, nu[3] = {0, 0, 0}, nw[3] = {0, 0, 0};
    auto fetch = [&](int k) {
        nx = cand_at<LDS>(first, n1, rest, k);
#pragma unroll
        for (int a = 0; a < D; a++) {
            ndx[a] = sdx[a * stride + nx.local];
            nu[a] = su[a * stride + nx.local];
        }
        if (MD) {
#pragma unroll
            for (int a = 0; a < 3; a++) nw[a] = sw[a * stride + nx.local];
        }
    };
    if (P.cnt > 0) fetch(0);
    for (int k = 0; k < P.cnt; k++) {
        const CandData cd = nx;
        float odx[3], ou[3], ow[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            odx[a] = ndx[a];
            ou[a] = nu[a];
            ow[a] = nw[a];
        }
        if (k + 1 < P.cnt) fetch(k + 1);
        if (MD) {
            pair_force_md<D>(P, cd, md.cmd + P.off + k, md.cms + 2 * (P.off + k), odx, ou, ow, c, F, tq);
        } else {
            pair_force<D>(P, cd, odx, ou, c, F);
        }
    }
    substep_update<D, MD>(P, c, F, tq);
}

// One axis of a sub-step (Eq. demgov, Jacobi) from the contact force F
// along it: drag from the momentum exchange j, buoyant weight (hbw = h bw),
// compensated velocity and displacement sums.
template <int D>
__device__ __forceinline__ void axis_update(const Active<D>& P, const PCfg& c, float F, float j, float hbw, float& u,
                                            float& cu, float& dx, float& cdx, float& gs, float& fs) {
#pragma clang fp contract(off)
    // (the products enter their sums fused, each rounded once)
    float g = 2.0f * fmaf(P.ri, u, -j);
    gs += g;
    fs += F;
    float incr = fmaf(fmaf(-P.Ap, g, F), P.hm, hbw);
    // compensated sums keep the many tiny increments exact to FP32
    float y = incr - cu;
    float t = u + y;
    cu = (t - u) - y;
    u = t;
    float yx = fmaf(c.h, u, -cdx);
    float tx = dx + yx;
    cdx = (tx - dx) - yx;
    dx = tx;
}

// |u|^2: the squares summed by sum_d
template <int D>
__device__ __forceinline__ float speed2(const float* u) {
    float sq[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < D; a++) sq[a] = u[a] * u[a];
    return sum_d<D>(sq);
}

// The update of one sub-step from the contact force F and torque tq
// (Eq. demgov, Jacobi).
template <int D, bool MD>
__device__ __forceinline__ void substep_update(Active<D>& P, const PCfg& c, const float* F, const float* tq) {
    if (P.fixed) {
        // a fixed point keeps its state; g = -2 j_i with U = 0, contact reactions summed
#pragma unroll
        for (int a = 0; a < D; a++) {
            P.gs[a] += -2.0f * P.j[a];
            P.fs[a] += F[a];
        }
        return;
    }
    if (MD) {
        // I dW/dt = torque (second line of Eq. demgov)
#pragma unroll
        for (int a = (D == 3 ? 0 : 2); a < 3; a++) P.W[a] += tq[a] * P.hI;
    }
#pragma unroll
    for (int a = 0; a < D; a++)
        axis_update(P, c, F[a], P.j[a], P.hbw[a], P.u[a], P.cu[a], P.dx[a], P.cdx[a], P.gs[a], P.fs[a]);
    P.vmax2 = fmaxf(P.vmax2, speed2<D>(P.u));
}

template <int D, bool MD>
__device__ __forceinline__ void active_store(const Active<D>& P, PState& Bn, const PCfg& c, uint32_t s, int np,
                                             float* srec, float* fc, uint32_t* flags, const MdBuf& md) {
    float invn = 1.0f / (float)c.n_sub;
#pragma unroll
    for (int a = 0; a < D; a++) {
        float xh = P.xh[a], xl = P.xl[a];
        df_add(xh, xl, P.dx[a]);
        Bn.xh[a][s] = xh;
        Bn.xl[a][s] = xl;
        Bn.u[a][s] = P.u[a];
        srec[(long long)s * SRec<D>::STRIDE + SRec<D>::COEF + a] = P.Af * (P.gs[a] * invn);
        fc[(long long)a * np + s] = P.fs[a] * invn;
    }
    if (sqrtf(P.vmax2) > 0.5f * c.skin) atomicOr(flags, FLAG_SKIN);
    if (MD) {
        if (D == 3) {
            Bn.w[0][s] = P.W[0];
            Bn.w[1][s] = P.W[1];
            Bn.w[2][s] = P.W[2];
        } else {
            Bn.w[0][s] = P.W[2];
        }
        // the history for the next step: every contact that carries a force
        const long long base = (long long)P.id * c.hmax;
        uint32_t n = 0;
        // (a contact is kept while any of its state is not zero; the
        // no-slip form carries T only)
        for (int k = 0; k < P.cnt; k++) {
            const float4 m = md.cmd[P.off + k];
            float S[TSN] = {m.x, m.y, m.z, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (c.microslip) {
                const float4 s0 = md.cms[2 * (P.off + k)], s1 = md.cms[2 * (P.off + k) + 1];
                S[3] = s0.x; S[4] = s0.y; S[5] = s0.z; S[9] = s0.w;
                S[6] = s1.x; S[7] = s1.y; S[8] = s1.z;
            }
            bool any = false;
#pragma unroll
            for (int q = 0; q < TSN; q++) any = any || S[q] != 0.f;
            if (!any) continue;
            md.hkey[base + n] = md.cpid[P.off + k];
#pragma unroll
            for (int q = 0; q < TSN; q++) md.hT[TSN * (base + n) + q] = S[q];
            n++;
        }
#pragma unroll
        for (int a = 0; a < D; a++) {
            bool any = false;
#pragma unroll
            for (int q = 0; q < TSN; q++) any = any || P.wT[a][q] != 0.f;
            if (!any) continue;
            md.hkey[base + n] = -1 - (2 * a + (int)((P.wside >> a) & 1u));
#pragma unroll
            for (int q = 0; q < TSN; q++) md.hT[TSN * (base + n) + q] = P.wT[a][q];
            n++;
        }
        md.hcnt[P.id] = n;
    }
}

constexpr int CAND_LDS = 8;   // candidates per lane cached in LDS

// The walls' bound on the contact-free sub-steps (remaining if none is
// near), for a particle moving at most V per unit time.
template <int D>
__device__ __forceinline__ float wall_allowance(const Active<D>& P, const PCfg& c, float V, int remaining) {
    float allow = (float)remaining;
    const float rc = 0.5f * P.d;
    if (P.wall) {
        // (the bounds below carry a 1e-5 margin, far above the reciprocal's rounding)
        const float iv = rcp_fast(V * c.h) * (1.0f - 1e-5f);
#pragma unroll
        for (int a = 0; a < D; a++) {
            float glo = P.dx[a] - ((rc - P.xh[a]) - P.xl[a]);
            float ghi = -(((rc - ((float)c.n[a] - P.xh[a])) + P.xl[a]) + P.dx[a]);
            allow = fminf(allow, fminf(glo, ghi) * iv);
        }
    }
    return allow;
}

// One candidate's bound: the gap closes by at most (V + Vt) h per sub-step,
// Vt from the partner's speed |ou| and equilibrium speed oveq.
template <int D>
__device__ __forceinline__ float cand_allowance(const Active<D>& P, const PCfg& c, const CandData& cd,
                                                const float* odx, const float* ou, float oveq, float V) {
    float rd = 0.f, dd = 0.f, r2 = 0.f, ou2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; a++) {
        float del = P.dx[a] - odx[a];
        float r = cd.r0[a] + del;
        rd += cd.r0[a] * del;
        dd += del * del;
        r2 += r * r;
        ou2 += ou[a] * ou[a];
    }
    float num = cd.K0 - (2.0f * rd + dd);             // r_c^2 - |r|^2
    float gap = -num * rcp_fast(cd.rc + sqrt_fast(r2));   // |r| - r_c
    float Vt = fmaxf(sqrt_fast(ou2), oveq) * (1.0f + 1e-5f);
    return (gap * (1.0f - 2e-5f)) * rcp_fast((V + Vt) * c.h);
}

// Number of sub-steps (<= remaining) that particle P can advance with no
// contact: along a contact-free stretch U^{k+i} is a convex combination of
// U^k and U_eq, so every particle moves at most V = max(|U^k|, |U_eq|) per
// unit time, and a gap g closes by at most (V_p + V_q) i h after i sub-steps.
template <int D, bool LDS = false>
__device__ __forceinline__ int free_allowance(const Active<D>& P, const PCfg& c, const CandData* first, int nfirst,
                                              const CandData* __restrict__ rest, const float* sdx, const float* su,
                                              const float* sveq, int stride, int remaining) {
    // the convexity bound needs q = 1 - hc > 0; otherwise take sub-steps
    if (!(P.hc < 1.0f)) return 0;
    float u2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; a++) {
        float ut = P.u[a] - P.cu[a];
        u2 += ut * ut;
    }
    const float V = fmaxf(sqrt_fast(u2), P.veq) * (1.0f + 1e-5f) + 1e-30f;
    float allow = wall_allowance<D>(P, c, V, remaining);
    const int n1 = min(P.cnt, nfirst);
    for (int k = 0; k < P.cnt; k++) {
        CandData cd = cand_at<LDS>(first, n1, rest, k);
        float odx[3], ou[3];
#pragma unroll
        for (int a = 0; a < D; a++) {
            odx[a] = sdx[a * stride + cd.local];
            ou[a] = su[a * stride + cd.local];
        }
        allow = fminf(allow, cand_allowance<D>(P, c, cd, odx, ou, sveq[cd.local], V));
    }
    if (!(allow > 0.f)) return 0;
    return allow >= (float)remaining ? remaining : (int)allow;
}

// The same for a particle whose only candidate's state at this sub-step is
// odx, ou (equilibrium speed oveq).
template <int D>
__device__ __forceinline__ int free_allowance_one(const Active<D>& P, const PCfg& c, const CandData& cd,
                                                  const float* odx, const float* ou, float oveq, int remaining) {
    if (!(P.hc < 1.0f)) return 0;
    float u2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; a++) {
        float ut = P.u[a] - P.cu[a];
        u2 += ut * ut;
    }
    const float V = fmaxf(sqrt_fast(u2), P.veq) * (1.0f + 1e-5f) + 1e-30f;
    float allow = wall_allowance<D>(P, c, V, remaining);
    allow = fminf(allow, cand_allowance<D>(P, c, cd, odx, ou, oveq, V));
    if (!(allow > 0.f)) return 0;
    return allow >= (float)remaining ? remaining : (int)allow;
}

// Advance P by m contact-free sub-steps in closed form:
//   U^{k+m} = U_eq + (U^k - U_eq) q^m,  sum_{i=1..m} U^{k+i} = m U_eq + (U^k - U_eq) q S,
//   sum_{i<m} g^{k+i} = 2 rho_i (m slip + (U^k - U_eq) S),  S = (1 - q^m)/(1 - q).
template <int D, bool MD>
__device__ __forceinline__ void active_jump(Active<D>& P, const PCfg& c, int m, const MdBuf& md) {
    if (MD) {
        // no contact along the stretch: every tangential force lapses, the
        // spin is unchanged
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int q = 0; q < TSN; q++) P.wT[a][q] = 0.f;
        for (int k = 0; k < P.cnt; k++) {
            const float4 q = md.cmd[P.off + k];
            if (q.x != 0.f || q.y != 0.f || q.z != 0.f) md.cmd[P.off + k] = make_float4(0.f, 0.f, 0.f, q.w);
            if (c.microslip) {
                md.cms[2 * (P.off + k)] = make_float4(0.f, 0.f, 0.f, 0.f);
                md.cms[2 * (P.off + k) + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    }
    if (P.fixed) {
#pragma unroll
        for (int a = 0; a < D; a++) P.gs[a] += (float)m * (-2.0f * P.j[a]);
        return;
    }
    const float mm = (float)m;
    float qm, omq;
    if (P.hc < 1.0f) {
        const float l = mm * P.lq;                   // m log(1 - hc)
        qm = expf(l);
        omq = -expm1f(l);
    } else {
        drag_power(P.hc, m, qm, omq);
    }
    const float S = omq * P.ihc;
    const float q = 1.0f - P.hc;
    float v2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; a++) {
#pragma clang fp contract(off)
        const float diff = (P.u[a] - P.ueq[a]) - P.cu[a];
        const float incx = c.h * (mm * P.ueq[a] + diff * (q * S));
        float yx = incx - P.cdx[a];
        float tx = P.dx[a] + yx;
        P.cdx[a] = (tx - P.dx[a]) - yx;
        P.dx[a] = tx;
        P.gs[a] += 2.0f * P.ri * (mm * P.slip[a] + diff * S);
        P.u[a] = P.ueq[a] + diff * qm;
        P.cu[a] = 0.f;
        v2 += P.u[a] * P.u[a];
    }
    P.vmax2 = fmaxf(P.vmax2, v2);
}

// Small islands: one 64-lane workgroup per packed wave, states in LDS.  A
// wave holds islands of one size s at lanes [i s, (i+1) s).  Each island
// advances on its own clock: per iteration it either jumps over a
// contact-free stretch (all of its members agree on the shortest allowance)
// or takes one Jacobi sub-step; so the result of an island does not depend
// on which other islands share its wave.
//
// Islands of one and two without fixed points take the split form below:
// a wave holds 16 particles, four lanes each.  Lane l updates axis l & 3 of
// its particle (with D = 2, lanes 2 and 3 repeat axis 1) and holds a copy
// of the particle's other state; the two members of an island of two sit
// eight lanes apart in one row of 16 lanes.  Cross-lane reads are DPP moves
// within the VALU: a broadcast from lane b of the quad, a rotation of the
// row by 8.  The lanes a move reads from belong to the reading lane's own
// island, which takes the same branches, so they are active whenever the
// reader is.
extern "C" __device__ int __ockl_wfred_min_i32(int);   // minimum over the wave's active lanes

template <int B>
__device__ __forceinline__ float quad_get(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), B * 0x55, 0xF, 0xF, false));
}
__device__ __forceinline__ float row_swap8(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, false));
}
__device__ __forceinline__ int row_swap8(int v) { return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false); }

// The full vector of a per-axis value (axis b from lane b of the quad).
template <int D>
__device__ __forceinline__ void quad_gather(float v, float* out) {
    out[0] = quad_get<0>(v);
    out[1] = quad_get<1>(v);
    if (D == 3) out[2] = quad_get<2>(v);
}

__device__ __forceinline__ float pick3(const float* v, int a) { return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]); }

// All sub-steps of a split wave of islands of one (NC = 0: a particle near
// a wall with no candidate) or of two (NC = 1: each member the other's only
// candidate), contact model CT; the partner's state by a row rotation, the
// candidate in registers.  The decisions and arithmetic are those of the
// general island loop: every lane of a quad holds the same copy of the
// particle's scalars and takes the same decisions.
template <int D, int CT, int NC>
__device__ __forceinline__ void split_wave(Active<D>& P, const PCfg& c, bool valid, const CandData& cd,
                                           const MdBuf& md) {
    const int ax = min((int)(threadIdx.x & 3u), D - 1);
    const int ct = CT < 0 ? c.contact : CT;
    if (!valid) P = Active<D>{};      // padding lanes: a zero state, never stored
    const float oveq = NC ? row_swap8(P.veq) : 0.f;
    // this lane's axis: the running state and the step's constants
    float u = pick3(P.u, ax), cu = pick3(P.cu, ax), dx = pick3(P.dx, ax), cdx = pick3(P.cdx, ax);
    float gs = pick3(P.gs, ax), fs = pick3(P.fs, ax);
    const float j = pick3(P.j, ax), hbw = pick3(P.hbw, ax), r0 = pick3(cd.r0, ax);
    float elo = 0.f, ehi = 0.f;
    {
        float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < D; a++) wall_offsets<D>(P, c, a, lo[a], hi[a]);
        elo = pick3(lo, ax);
        ehi = pick3(hi, ax);
    }
    // one sub-step of this lane's axis
    auto substep = [&](float& u, float& cu, float& dx, float& cdx, float& gs, float& fs, float& vm) {
        float F = 0.f;
        if (P.wall) F = wall_axis<CT>(c, P.gw, P.d, elo - dx, ehi + dx, u, F);
        if (NC) {
            // (every member of a split pair wave has its partner as only candidate)
            // the relative displacement and velocity, axis by axis
            // (this lane's component of r = r0 + del is r0 + its own del)
            float del[3] = {0.f, 0.f, 0.f}, r[3], inv, delta;
            const float dl = dx - row_swap8(dx);
            quad_gather<D>(dl, del);
            const bool on = pair_geom<D, true>(cd, del, r, inv, delta);
            const float n = (r0 + dl) * inv;
            float vn = 0.f;
            if (ct == PIBM_CONTACT_LSD) {
                float pv[3] = {0.f, 0.f, 0.f};
                quad_gather<D>((u - row_swap8(u)) * n, pv);
                vn = sum_d<D>(pv);
            }
            const float Fp = F + pair_mag<CT>(cd, c, delta, vn) * n;
            F = on ? Fp : F;
        }
        axis_update<D>(P, c, F, j, hbw, u, cu, dx, cdx, gs, fs);
        float sq[3] = {0.f, 0.f, 0.f};
        quad_gather<D>(u * u, sq);
        vm = fmaxf(vm, sum_d<D>(sq));
    };
    // Each island keeps its own trip count (its sub-steps and jumps so far),
    // back-off and k, and takes the decisions of the general loop in the
    // same order; only the interleaving of islands within the wave differs.
    int k = 0, backoff = 1, trip = 0;
    while (__any(valid && k < c.n_sub)) {
        // Checks, and the jumps they allow: an island that jumps checks again
        // on its next trip (back-off 1), taken here at once.
        bool more, check;
        int m;
        for (;;) {
            more = valid && k < c.n_sub;
            check = more && (trip & (backoff - 1)) == 0;
            m = 0;
            if (__any(check)) {
                // the full vectors of this particle and of its partner
                Active<D> Q = P;
                quad_gather<D>(u, Q.u);
                quad_gather<D>(cu, Q.cu);
                quad_gather<D>(dx, Q.dx);
                float odx[3] = {0.f, 0.f, 0.f}, ou[3] = {0.f, 0.f, 0.f};
                if (NC) {
#pragma unroll
                    for (int a = 0; a < D; a++) {
                        odx[a] = row_swap8(Q.dx[a]);
                        ou[a] = row_swap8(Q.u[a]);
                    }
                }
                int allow = 0;
                if (check) {
                    if (NC) allow = free_allowance_one<D>(Q, c, cd, odx, ou, oveq, c.n_sub - k);
                    else allow = free_allowance<D>(Q, c, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, c.n_sub - k);
                }
                const int other = NC ? row_swap8(allow) : allow;
                m = check ? min(allow, other) : 0;
            }
            const bool jump = more && m >= 2;
            if (!__any(jump)) break;
            if (jump) {
                quad_gather<D>(u, P.u);
                quad_gather<D>(cu, P.cu);
                quad_gather<D>(dx, P.dx);
                quad_gather<D>(cdx, P.cdx);
                quad_gather<D>(gs, P.gs);
                active_jump<D, false>(P, c, m, md);
                u = pick3(P.u, ax);
                cu = pick3(P.cu, ax);
                dx = pick3(P.dx, ax);
                cdx = pick3(P.cdx, ax);
                gs = pick3(P.gs, ax);
                k += m;
                backoff = 1;
                trip += 1;
            }
        }
        // a sub-step for every island left, computed on every lane and kept where it steps
        {
            float u1 = u, cu1 = cu, dx1 = dx, cdx1 = cdx, gs1 = gs, fs1 = fs, vm1 = P.vmax2;
            substep(u1, cu1, dx1, cdx1, gs1, fs1, vm1);
            u = more ? u1 : u;
            cu = more ? cu1 : cu;
            dx = more ? dx1 : dx;
            cdx = more ? cdx1 : cdx;
            gs = more ? gs1 : gs;
            fs = more ? fs1 : fs;
            P.vmax2 = more ? vm1 : P.vmax2;
        }
        if (more) {
            k += 1;
            trip += 1;
            if (check) backoff = min(2 * backoff, 64);
        }
        // The trips before the next check of any island, and before any
        // island ends, hold plain sub-steps only: run them with no decision.
        const bool run = valid && k < c.n_sub;
        int T = __ockl_wfred_min_i32(run ? min((-trip) & (backoff - 1), c.n_sub - k) : INT_MAX);
        if (T == INT_MAX) T = 0;
        if (run) {
            float vm = P.vmax2;
            for (int t = 0; t < T; t++) substep(u, cu, dx, cdx, gs, fs, vm);
            P.vmax2 = vm;
            k += T;
            trip += T;
        }
    }
    quad_gather<D>(u, P.u);
    quad_gather<D>(cu, P.cu);
    quad_gather<D>(dx, P.dx);
    quad_gather<D>(cdx, P.cdx);
    quad_gather<D>(gs, P.gs);
    quad_gather<D>(fs, P.fs);
}

template <int D, bool MD>
__global__ __launch_bounds__(64) void k_island_small(PState A, PState Bn, int np, PCfg c,
                                                     const int* __restrict__ lanemember,
                                                     const uint32_t* __restrict__ alist,
                                                     const uint32_t* __restrict__ ccount,
                                                     const unsigned long long* __restrict__ prefix,
                                                     const uint32_t* __restrict__ parent,
                                                     const uint32_t* __restrict__ isize,
                                                     const CandData* __restrict__ cdata,
                                                     const float* __restrict__ drho_i, const float* __restrict__ j_i,
                                                     float* __restrict__ srec, float* __restrict__ fc,
                                                     uint32_t* __restrict__ flags,
                                                     const uint32_t* __restrict__ counters, MdBuf md) {
    __shared__ float sdx[2][3 * WAVE];
    __shared__ float su[2][3 * WAVE];
    __shared__ float sw[MD ? 2 : 1][MD ? 3 * WAVE : 1];
    __shared__ float sveq[WAVE];
    __shared__ int sallow[WAVE];
    __shared__ CandData scd[WAVE * CAND_LDS];
    const uint32_t nw = counters[CNT_WAVES];
    const int lane = threadIdx.x;
    // first wave of size class lane + 1 (non-decreasing in the class)
    const uint32_t wb_lane = counters[CNT_WAVEBASE + 1 + lane];
    // Without Mindlin, each packed wave is worked by QUARTERS workgroups:
    // quarter q takes the islands of one or two at its lanes
    // [16 q, 16 q + 16) in the split form (or in the general loop below,
    // restricted to those lanes, when one of them does not qualify); a wave
    // of larger islands is worked by quarter 0 alone.
    constexpr uint32_t QUARTERS = MD ? 1u : 4u;
    for (uint32_t v = blockIdx.x; v < nw * QUARTERS; v += gridDim.x) {
        const uint32_t w = v / QUARTERS, part = v % QUARTERS;
        // the wave's size class is the largest whose first wave is <= w;
        // its islands fill lanes [0, islands_here * size)
        const unsigned long long le = __ballot(wb_lane <= w);
        const int sz = 64 - __clzll(le);
        const uint32_t per = WAVE / sz;
        const uint32_t nisl = counters[CNT_CLASS + sz] + (sz == 2 ? counters[CNT_PAIRC] : 0u);
        const uint32_t idx = w - counters[CNT_WAVEBASE + sz];
        const uint32_t here = min(per, nisl - idx * per);
        const bool quartered = !MD && sz <= 2;
        if (!quartered && part != 0) continue;
        if (quartered) {
            // the split form: original lane ol of this quarter for each group of four lanes
            const int ol = (int)part * 16 +
                           (sz == 2 ? (((lane >> 4) << 2) | (((lane >> 2) & 1) << 1) | ((lane >> 3) & 1)) : (lane >> 2));
            const bool sv = (uint32_t)ol < here * (uint32_t)sz;
            const uint32_t ss = sv ? alist[lanemember[(long long)w * WAVE + ol]] : 0;
            Active<D> P;
            CandData cd{};
            if (sv) {
                active_load<D, MD>(P, A, c, ss, drho_i, j_i, np, ccount, prefix, md);
                if (sz == 2 && P.cnt > 0) cd = cdata[P.off];
            }
            const bool ok = sv && (sz == 1 ? (P.cnt == 0 && !P.fixed)
                                           : (P.cnt == 1 && !P.fixed && cd.local == (ol ^ 1)));
            if (__all(!sv || ok)) {
                if (sz == 1) {
                    if (c.contact == PIBM_CONTACT_LSD) split_wave<D, PIBM_CONTACT_LSD, 0>(P, c, sv, cd, md);
                    else if (c.contact == PIBM_CONTACT_HERTZ) split_wave<D, PIBM_CONTACT_HERTZ, 0>(P, c, sv, cd, md);
                    else split_wave<D, -1, 0>(P, c, sv, cd, md);
                } else {
                    if (c.contact == PIBM_CONTACT_LSD) split_wave<D, PIBM_CONTACT_LSD, 1>(P, c, sv, cd, md);
                    else if (c.contact == PIBM_CONTACT_HERTZ) split_wave<D, PIBM_CONTACT_HERTZ, 1>(P, c, sv, cd, md);
                    else split_wave<D, -1, 1>(P, c, sv, cd, md);
                }
                if (sv && (lane & 3) == 0) active_store<D, MD>(P, Bn, c, ss, np, srec, fc, flags, md);
                continue;
            }
        }
        // the general loop: the whole wave, or this quarter's lanes of it
        bool valid = (uint32_t)lane < here * (uint32_t)sz && (!quartered || (uint32_t)(lane >> 4) == part);
        int a = valid ? lanemember[(long long)w * WAVE + lane] : -1;
        uint32_t s = valid ? alist[a] : 0;
        Active<D> P;
        int nfirst = 0, isz = 1;
        if (valid) {
            active_load<D, MD>(P, A, c, s, drho_i, j_i, np, ccount, prefix, md);
            nfirst = min(P.cnt, CAND_LDS);
            for (int k = 0; k < nfirst; k++) scd[lane * CAND_LDS + k] = cdata[P.off + k];
            isz = (int)isize[parent[a]];
        }
        const int ibase = (lane / isz) * isz;
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            sdx[0][ax * WAVE + lane] = 0.f;
            su[0][ax * WAVE + lane] = valid ? P.u[ax] : 0.f;
            if (MD) sw[0][ax * WAVE + lane] = valid ? P.W[ax] : 0.f;
        }
        sveq[lane] = valid ? P.veq : 0.f;
        __syncthreads();
        const CandData* rest = cdata + (valid ? P.off : 0);
        int k = 0, cur = 0;
        // An island checks for a contact-free stretch to jump over on the
        // trips (iterations of this loop, counted from 0 for every island)
        // that are multiples of its back-off b: 1 after a jump, doubled by
        // every check that finds none, up to 64 (a pair in lasting contact
        // fails every check).  The check trips of all islands in a wave thus
        // coincide, and the trips in between cost no check at all.  Every
        // member of an island takes the same decisions (they share k, b and
        // the island minimum), an island's decisions depend on its own state
        // and the trip count only, and plain sub-steps are always valid.
        // A wave whose members have no partner (islands of one particle in
        // wall contact) exchanges nothing.
        int backoff = 1;
        const bool xchg = __any(valid && P.cnt > 0);        // some member has a partner
        for (int trip = 0; __any(valid && k < c.n_sub); trip++) {
            const bool more = valid && k < c.n_sub;
            const bool check = more && (trip & (backoff - 1)) == 0;
            int m = 0;
            if (__any(check)) {
                int allow = 0;
                if (check)
                    allow = free_allowance<D, true>(P, c, scd + lane * CAND_LDS, nfirst, rest, sdx[cur], su[cur],
                                                    sveq, WAVE, c.n_sub - k);
                m = allow;
                if (xchg) {
                    sallow[lane] = allow;
                    __syncthreads();
                    if (check)
                        for (int i = 0; i < isz; i++) m = min(m, sallow[ibase + i]);
                    __syncthreads();
                }
            }
            if (more) {
                if (m >= 2) {
                    active_jump<D, MD>(P, c, m, md);
                    k += m;
                    backoff = 1;
                } else {
                    active_substep<D, MD, true>(P, c, scd + lane * CAND_LDS, nfirst, rest, sdx[cur], su[cur],
                                                MD ? sw[cur] : nullptr, WAVE, md);
                    k += 1;
                    if (check) backoff = min(2 * backoff, 64);
                }
            }
            if (xchg) {
#pragma unroll
                for (int ax = 0; ax < 3; ax++) {
                    sdx[cur ^ 1][ax * WAVE + lane] = valid ? P.dx[ax] : 0.f;
                    su[cur ^ 1][ax * WAVE + lane] = valid ? P.u[ax] : 0.f;
                    if (MD) sw[cur ^ 1][ax * WAVE + lane] = valid ? P.W[ax] : 0.f;
                }
                __syncthreads();
                cur ^= 1;
            }
        }
        if (valid) active_store<D, MD>(P, Bn, c, s, np, srec, fc, flags, md);
        __syncthreads();
    }
}

// Islands larger than a wave: one 256-lane workgroup per island, states in
// global scratch indexed by the active index (gdx, gu: [2][3][cap]; the
// compensations and running sums follow gdx at 6 cap .. 19 cap).
template <int D, bool MD>
__global__ __launch_bounds__(256) void k_island_big(PState A, PState Bn, int np, PCfg c,
                                                    const uint32_t* __restrict__ bigmember,
                                                    const uint32_t* __restrict__ bigoff,
                                                    const uint32_t* __restrict__ bigroot,
                                                    const uint32_t* __restrict__ isize,
                                                    const uint32_t* __restrict__ alist,
                                                    const uint32_t* __restrict__ ccount,
                                                    const unsigned long long* __restrict__ prefix,
                                                    const CandData* __restrict__ cdata,
                                                    const float* __restrict__ drho_i, const float* __restrict__ j_i,
                                                    float* __restrict__ srec, float* __restrict__ fc,
                                                    float* gdx, float* gu, long long cap,
                                                    uint32_t* __restrict__ flags,
                                                    const uint32_t* __restrict__ counters, MdBuf md) {
    // MD scratch: spin [2][3][cap], wall tangential states [3 TSN][cap], wall sides [cap]
    float* gw = md.gmd;
    float* gwt = md.gmd + 6 * cap;
    uint32_t* gside = (uint32_t*)(md.gmd + (6 + 3 * TSN) * cap);
    const uint32_t nbig = counters[CNT_BIG];
    for (uint32_t ib = blockIdx.x; ib < nbig; ib += gridDim.x) {
        uint32_t base = bigoff[ib];
        uint32_t sz = isize[bigroot[ib]];
        for (uint32_t i = threadIdx.x; i < sz; i += 256) {
            uint32_t a = bigmember[base + i];
            uint32_t s = alist[a];
#pragma unroll
            for (int ax = 0; ax < 3; ax++) {
                gdx[(0 * 3 + ax) * cap + a] = 0.f;
                gu[(0 * 3 + ax) * cap + a] = ax < D ? A.u[ax][s] : 0.f;
            }
            if (MD) {
                gw[(0 * 3 + 0) * cap + a] = D == 3 ? A.w[0][s] : 0.f;
                gw[(0 * 3 + 1) * cap + a] = D == 3 ? A.w[1][s] : 0.f;
                gw[(0 * 3 + 2) * cap + a] = D == 3 ? A.w[2][s] : A.w[0][s];
            }
        }
        __syncthreads();
        // per-member state is re-read from scratch each sub-step (a lane may own several members)
        for (int k = 0; k < c.n_sub; k++) {
            int cur = k & 1;
            for (uint32_t i = threadIdx.x; i < sz; i += 256) {
                uint32_t a = bigmember[base + i];
                uint32_t s = alist[a];
                Active<D> P;
                active_load<D, MD>(P, A, c, s, drho_i, j_i, np, ccount, prefix, md);
#pragma unroll
                for (int ax = 0; ax < D; ax++) {
                    P.dx[ax] = gdx[(cur * 3 + ax) * cap + a];
                    P.u[ax] = gu[(cur * 3 + ax) * cap + a];
                }
                if (MD) {
#pragma unroll
                    for (int ax = 0; ax < 3; ax++) P.W[ax] = gw[(cur * 3 + ax) * cap + a];
                    if (k > 0) {
#pragma unroll
                        for (int ax = 0; ax < 3; ax++)
#pragma unroll
                            for (int b = 0; b < TSN; b++) P.wT[ax][b] = gwt[(TSN * ax + b) * cap + a];
                        P.wside = gside[a];
                    }
                }
                float* aux = gdx + 6 * cap;
                if (k > 0) {
#pragma unroll
                    for (int ax = 0; ax < D; ax++) {
                        P.cdx[ax] = aux[(0 * 3 + ax) * cap + a];
                        P.cu[ax] = aux[(1 * 3 + ax) * cap + a];
                        P.gs[ax] = aux[(2 * 3 + ax) * cap + a];
                        P.fs[ax] = aux[(3 * 3 + ax) * cap + a];
                    }
                    P.vmax2 = aux[12 * cap + a];
                }
                active_substep<D, MD>(P, c, cdata + P.off, P.cnt, cdata + P.off, gdx + cur * 3 * cap,
                                      gu + cur * 3 * cap, MD ? gw + cur * 3 * cap : nullptr, (int)cap, md);
                if (MD) {
#pragma unroll
                    for (int ax = 0; ax < 3; ax++) {
                        gw[((cur ^ 1) * 3 + ax) * cap + a] = P.W[ax];
#pragma unroll
                        for (int b = 0; b < TSN; b++) gwt[(TSN * ax + b) * cap + a] = P.wT[ax][b];
                    }
                    gside[a] = P.wside;
                }
#pragma unroll
                for (int ax = 0; ax < D; ax++) {
                    gdx[((cur ^ 1) * 3 + ax) * cap + a] = P.dx[ax];
                    gu[((cur ^ 1) * 3 + ax) * cap + a] = P.u[ax];
                    aux[(0 * 3 + ax) * cap + a] = P.cdx[ax];
                    aux[(1 * 3 + ax) * cap + a] = P.cu[ax];
                    aux[(2 * 3 + ax) * cap + a] = P.gs[ax];
                    aux[(3 * 3 + ax) * cap + a] = P.fs[ax];
                }
                aux[12 * cap + a] = P.vmax2;
                if (k == c.n_sub - 1) active_store<D, MD>(P, Bn, c, s, np, srec, fc, flags, md);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// spreading (Eq. lbm10): F(r) = sum_p A_p gbar_p W_p(r) with the start-of-step
// weights.
// ---------------------------------------------------------------------------
// Spreading with dual-cell bins (bin edge 1): cell c' = floor(X - 1/2) + 1.
// Node r receives exactly the particles of cells c' in [r - 1, r + 2] per
// axis, with support offset k = r + 2 - c'.  A workgroup owns a tile of
// nodes; it stages, for the tile's halo of cells, the LDS position of each
// cell's first particle, and the particles' weights and coefficients; each
// thread then sums, for its nodes, the particles of its 4^D cells in a fixed
// order (rows of cells by kz, ky; cells by kx; particles in sorted order).
// No atomics, no wasted candidate checks.  A tile holding more than MAXP
// particles reads them from global memory instead of LDS (same order, same
// result); a tile that no particle reaches writes zeros at once.
template <int D> struct CsrTile;
// MAXP: particles staged in LDS per tile (the halo of a 3D tile holds about
// 200 at 0.24 particles per cell; 256 slots leave room for 8 workgroups per
// CU, and a fuller halo takes the unstaged path)
template <> struct CsrTile<3> { static constexpr int TX = 8, TY = 8, TZ = 4, MAXP = 256; };
template <> struct CsrTile<2> { static constexpr int TX = 32, TY = 16, TZ = 1, MAXP = 384; };

// C components are spread: REC, C = D: the force field, with the
// coefficients in the spreading records; the adjoint spreads C = D + 1
// components (density and momentum adjoints) from the planes coef[a np + s]
// with the same kernel.  Each staged particle is its record (and the
// adjoint's planes after it).
//
// The halo's cell starts are loaded by one thread per halo row (one batch of
// independent loads each), and that thread turns them into the row's table
// pk: for each node column lx of the tile, the LDS index of the first
// particle of the four cells that reach it and the index one past the last,
// packed in one word (tile positions < 2^16).  A node then reads one word per
// halo row.
template <int D, int C, bool REC, class T, class Sink>
__device__ __forceinline__ void spread_tile(const Grid& g, const PCfg& c, const uint32_t* __restrict__ start,
                                            const float* __restrict__ srec, const float* __restrict__ coef, int np,
                                            int ntx, int nty, Sink& sink) {
    using RS = SRec<D>;
    constexpr int TX = T::TX, TY = T::TY, TZ = T::TZ;
    constexpr int HX = TX + 3, HY = TY + 3, HZ = (D == 3) ? TZ + 3 : 1;
    constexpr int NR = HY * HZ;                  // halo rows of cells
    // staged floats per particle: the record (and the adjoint's planes), to
    // an odd stride so that lanes reading different particles hit different
    // LDS banks
    constexpr int PW = (REC ? RS::STRIDE : RS::STRIDE + C) | 1;
    constexpr int CO = REC ? RS::COEF : RS::STRIDE;                    // the coefficients in a staged particle
    constexpr int MAXP = T::MAXP;
    static_assert(!REC || C == D, "records carry D coefficients");
    static_assert(NR <= 256 && NR <= 255, "one thread per halo row; rows fit the row table");
    static_assert(MAXP < 65536, "tile positions fit 16 bits");
    __shared__ uint32_t pk[NR * TX];             // per row and node column: first | end << 16
    __shared__ uint32_t rowbase[NR + 1], rowg0[NR];
    __shared__ float sp[MAXP * PW];
    __shared__ uint8_t rowof[MAXP];              // halo row of each staged particle
    __shared__ uint32_t scan4[4];
    const int t = threadIdx.x;
    int tx, ty, tz;
    banded_tile(ntx, nty, (int)gridDim.x / (ntx * nty), D == 3 ? 1 : 0, tx, ty, tz);
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int cx0 = x0 - 1, cy0 = y0 - 1, cz0 = (D == 3) ? z0 - 1 : 0;
    const int lo = max(cx0, 0), hi = min(cx0 + HX - 1, c.nb[0] - 1);
    // row t: the starts of its cells cx0 .. cx0 + HX, clamped to the bins
    // [lo, hi + 1] (so v[0] is the row's first start and v[HX] its end)
    uint32_t v[HX + 1];
    uint32_t cnt_row = 0;
    if (t < NR) {
        const int cy = cy0 + t % HY, cz = cz0 + t / HY;
        const bool ok = cy >= 0 && cy < c.nb[1] && cz >= 0 && cz < c.nb[2] && lo <= hi;
        const uint32_t* row = start + (ok ? ((long long)cz * c.nb[1] + cy) * c.nb[0] : 0);
#pragma unroll
        for (int ix = 0; ix <= HX; ix++) v[ix] = row[ok ? min(max(cx0 + ix, lo), hi + 1) : 0];
        if (!ok)
#pragma unroll
            for (int ix = 0; ix <= HX; ix++) v[ix] = 0;
        cnt_row = v[HX] - v[0];
    }
    uint32_t rb;
    {
        // row offsets: exclusive scan of the row counts over the block
        uint32_t all;
        rb = block_exclusive_scan<uint32_t>(cnt_row, scan4, all);
        if (t < NR) {
            rowbase[t] = rb;
            rowg0[t] = v[0];
#pragma unroll
            for (int lx = 0; lx < TX; lx++)
                pk[t * TX + lx] = (rb + (v[lx] - v[0])) | ((rb + (v[lx + 4] - v[0])) << 16);
        }
        if (t == 0) rowbase[NR] = all;
    }
    __syncthreads();
    const uint32_t total = rowbase[NR];
    if (total == 0) {
        // no particle reaches the tile (the same for the whole workgroup)
        for (int node = t; node < TX * TY * TZ; node += 256) {
            const int x = x0 + node % TX, y = y0 + (node / TX) % TY, z = z0 + node / (TX * TY);
            if (x >= g.n[0] || y >= g.n[1] || z >= g.n[2]) continue;
            const long long rn = ((long long)z * g.n[1] + y) * g.n[0] + x;
            float acc[C];
#pragma unroll
            for (int a = 0; a < C; a++) acc[a] = 0.f;
            sink(x, y, z, rn, acc);
        }
        return;
    }
    const bool staged = total <= (uint32_t)MAXP;
    if (staged) {
        if (t < NR)
            for (uint32_t k = rb; k < rb + cnt_row; k++) rowof[k] = (uint8_t)t;
        __syncthreads();
        for (uint32_t k = t; k < total; k += 256) {
            const int r = rowof[k];
            const uint32_t gsl = rowg0[r] + (k - rowbase[r]);
            const float4* rec = (const float4*)(srec + (long long)gsl * RS::STRIDE);
#pragma unroll
            for (int i = 0; i < RS::STRIDE / 4; i++) {
                const float4 w = rec[i];
                sp[__umul24(k, PW) + 4 * i] = w.x;
                sp[__umul24(k, PW) + 4 * i + 1] = w.y;
                sp[__umul24(k, PW) + 4 * i + 2] = w.z;
                sp[__umul24(k, PW) + 4 * i + 3] = w.w;
            }
            if (!REC) {
#pragma unroll
                for (int a = 0; a < C; a++) sp[__umul24(k, PW) + CO + a] = coef[(long long)a * np + gsl];
            }
        }
        __syncthreads();
    }
    for (int node = t; node < TX * TY * TZ; node += 256) {
        const int lx = node % TX, ly = (node / TX) % TY, lz = node / (TX * TY);
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (x >= g.n[0] || y >= g.n[1] || z >= g.n[2]) continue;
        float acc[C];
#pragma unroll
        for (int a = 0; a < C; a++) acc[a] = 0.f;
        // the particle ranges of the node's 4^(D-1) halo rows (i = ky + 4 kz:
        // row (ly + 3 - ky, lz + 3 - kz)); each particle's x weight index is
        // x - base_x
        constexpr int NRW = (D == 3 ? 16 : 4);
        auto row_of = [&](int i) { return (D == 3 ? (lz + 3 - (i >> 2)) * HY : 0) + (ly + 3 - (i & 3)); };
        if (staged && D == 2) {
#pragma unroll
            for (int i = 0; i < NRW; i++) {
                const uint32_t pr = pk[row_of(i) * TX + lx];
                for (uint32_t k = pr & 0xffffu; k < (pr >> 16); k++) {
                    const float* q = sp + __umul24(k, PW);
                    const float W = q[x - __float_as_int(q[RS::BASE])] * q[4 + i];
#pragma unroll
                    for (int a = 0; a < C; a++) acc[a] += W * q[CO + a];
                }
            }
        } else if (staged) {
            // 3D: one flat loop over the lane's particles, rows in order: a
            // wave then runs as many trips as its busiest lane has particles,
            // not the sum over the 16 rows of each row's busiest lane
            uint32_t mask = 0;
#pragma unroll
            for (int i = 0; i < NRW; i++) {
                const uint32_t pr = pk[row_of(i) * TX + lx];
                if ((pr >> 16) > (pr & 0xffffu)) mask |= 1u << i;
            }
            uint32_t k = 0, e = 0;
            int ky = 0, kz = 0;
            while (true) {
                if (k == e) {
                    if (!mask) break;
                    const int i = __builtin_ctz(mask);
                    mask &= mask - 1u;
                    ky = i & 3;
                    kz = i >> 2;
                    const uint32_t pr = pk[row_of(i) * TX + lx];
                    k = pr & 0xffffu;
                    e = pr >> 16;
                }
                // (k < 2^16: the 24-bit multiply, full rate, not the 32-bit one)
                const float* q = sp + __umul24(k, PW);
                const float W = q[x - __float_as_int(q[RS::BASE])] * q[4 + ky] * q[8 % (4 * D) + kz];
#pragma unroll
                for (int a = 0; a < C; a++) acc[a] += W * q[CO + a];
                k++;
            }
        } else {
#pragma unroll 1
            for (int i = 0; i < NRW; i++) {
                const int ky = i & 3, kz = i >> 2;
                const int r = row_of(i);
                const uint32_t pr = pk[r * TX + lx];
                for (uint32_t k = pr & 0xffffu; k < (pr >> 16); k++) {
                    // particle k of halo row r sits at sorted slot rowg0[r] + (k - rowbase[r])
                    const uint32_t gsl = rowg0[r] + (k - rowbase[r]);
                    const float* q = srec + (long long)gsl * RS::STRIDE;
                    const float W = q[x - __float_as_int(q[RS::BASE])] * q[4 + ky] *
                                    (D == 3 ? q[8 % (4 * D) + kz] : 1.f);
#pragma unroll
                    for (int a = 0; a < C; a++)
                        acc[a] += W * (REC ? q[CO + a] : coef[(long long)a * np + gsl]);
                }
            }
        }
        const long long rn = ((long long)z * g.n[1] + y) * g.n[0] + x;
        sink(x, y, z, rn, acc);
    }
}

template <int D, int C, bool REC>
__global__ __launch_bounds__(256) void k_spread_csr(Grid g, PCfg c, const uint32_t* __restrict__ start,
                                                    const float* __restrict__ srec, const float* __restrict__ coef,
                                                    int np, float* __restrict__ F, int ntx, int nty) {
    auto sink = [&](int, int, int, long long rn, const float* acc) {
#pragma unroll
        for (int a = 0; a < C; a++) F[(long long)a * g.N + rn] = acc[a];
    };
    spread_tile<D, C, REC, CsrTile<D>>(g, c, start, srec, coef, np, ntx, nty, sink);
}

// Spreading fused with the collision (3D, spreading records): each node's
// spread force goes straight into its collision and streaming, so the force
// field never goes to HBM, and the spreading's instruction-bound work runs
// beside the collision's memory traffic.  The tile spans 32 nodes in x so
// that the collision's reads and writes of each population plane are whole
// 128-byte rows; even so the tiled order streams slower than the collision's
// own row order (c2: 600 against 477 us for the collision alone), so the
// fusion pays only where the collision moves 4-byte populations.  Per node
// the same sums in the same order as k_spread_csr followed by k_collide:
// bitwise the same result.
struct FusedTile { static constexpr int TX = 32, TY = 4, TZ = 2, MAXP = 384; };

template <int Q, class S>
__global__ __launch_bounds__(256) void k_spread_collide(Grid g, PCfg c, const uint32_t* __restrict__ start,
                                                        const float* __restrict__ srec, int np,
                                                        const typename S::T* __restrict__ fin,
                                                        typename S::T* __restrict__ fout, float ffx, float ffy,
                                                        float ffz, float omega, float fpref, S st, int ntx, int nty) {
    using T = FusedTile;
    static_assert(T::TX * T::TY * T::TZ == 256, "one node per thread");
    // this thread's node (the one spread_tile hands to the sink): its
    // populations are loaded first, so that the loads are in flight while
    // the spreading prologue and sums run
    int tx, ty, tz;
    banded_tile(ntx, nty, (int)gridDim.x / (ntx * nty), 1, tx, ty, tz);
    const int t = threadIdx.x;
    const int x0 = tx * T::TX + t % T::TX, y0 = ty * T::TY + (t / T::TX) % T::TY, z0 = tz * T::TZ + t / (T::TX * T::TY);
    float h[Q];
    if (x0 < g.n[0] && y0 < g.n[1] && z0 < g.n[2])
        collide_load<Q, S>(fin, ((long long)z0 * g.n[1] + y0) * g.n[0] + x0, g, h, st);
    auto sink = [&](int x, int y, int z, long long rn, const float* acc) {
        collide_finish<Q, S>(h, fout, rn, x, y, z, g, ffx + acc[0], ffy + acc[1], ffz + acc[2], omega, fpref, st);
    };
    spread_tile<3, 3, true, T>(g, c, start, srec, nullptr, np, ntx, nty, sink);
}

// Spread C per-particle components with the weights of the spreading records
// of the same slots onto C node fields (L = 0 only): the records' own
// coefficients (coef == nullptr, C = D), or the planes coef[a * np + s].
template <int D, int C>
void spread_fields(const PBuf& b, int np, const PCfg& c, const Grid& g, const float* coef, float* out,
                   hipStream_t s) {
    using T = CsrTile<D>;
    int ntx = (g.n[0] + T::TX - 1) / T::TX, nty = (g.n[1] + T::TY - 1) / T::TY;
    int ntz = (D == 3) ? (g.n[2] + T::TZ - 1) / T::TZ : 1;
    const dim3 grid((unsigned)((long long)ntx * nty * ntz));
    if (coef == nullptr) {
        if constexpr (C == D)
            hipLaunchKernelGGL((k_spread_csr<D, C, true>), grid, dim3(256), 0, s, g, c, b.start, b.srec, nullptr, np,
                               out, ntx, nty);
    } else {
        hipLaunchKernelGGL((k_spread_csr<D, C, false>), grid, dim3(256), 0, s, g, c, b.start, b.srec, coef, np, out,
                           ntx, nty);
    }
}

template <int Q, class S>
static void spread_collide_launch(const PBuf& b, int np, const PCfg& c, const Grid& g, const void* fin, void* fout,
                                  const float* ff, float tau, S st, hipStream_t s) {
    using T = FusedTile;
    const int ntx = (g.n[0] + T::TX - 1) / T::TX, nty = (g.n[1] + T::TY - 1) / T::TY;
    const int ntz = (g.n[2] + T::TZ - 1) / T::TZ;
    const dim3 grid((unsigned)((long long)ntx * nty * ntz));
    hipLaunchKernelGGL((k_spread_collide<Q, S>), grid, dim3(256), 0, s, g, c, b.start, b.srec, np,
                       (const typename S::T*)fin, (typename S::T*)fout, ff[0], ff[1], ff[2], 1.0f / tau,
                       1.0f - 0.5f / tau, st, ntx, nty);
}

void particles_spread_collide(int Q, int fp16, int sl2, const PBuf& b, int np, const PCfg& c, const Grid& g,
                              const void* fin, void* fout, const float* ff, float tau, hipStream_t s) {
    StoreF32 s32{ldexpf(1.0f, sl2), ldexpf(1.0f, -sl2)};
    StoreF16 s16{ldexpf(1.0f, sl2), ldexpf(1.0f, -sl2)};
    if (Q == 15) {
        if (fp16) spread_collide_launch<15>(b, np, c, g, fin, fout, ff, tau, s16, s);
        else spread_collide_launch<15>(b, np, c, g, fin, fout, ff, tau, s32, s);
    } else {
        if (fp16) spread_collide_launch<19>(b, np, c, g, fin, fout, ff, tau, s16, s);
        else spread_collide_launch<19>(b, np, c, g, fin, fout, ff, tau, s32, s);
    }
}

void particles_spread_adjoint(int D, PBuf& b, int np, const PCfg& c, const Grid& g, const float* coef, float* out,
                              hipStream_t s) {
    if (D == 3) spread_fields<3, 4>(b, np, c, g, coef, out, s);
    else spread_fields<2, 3>(b, np, c, g, coef, out, s);
}

template <int D> struct SpreadBlock;
template <> struct SpreadBlock<3> { static constexpr int BX = 4, BY = 4, BZ = 4; };
template <> struct SpreadBlock<2> { static constexpr int BX = 8, BY = 8, BZ = 1; };

__device__ __forceinline__ float pick4(int k, float a, float b, float c, float d) {
    const float lo = (k & 1) ? b : a, hi = (k & 1) ? d : c;
    return (k & 2) ? hi : lo;
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int D>
__global__ __launch_bounds__(256) void k_spread(Grid g, PCfg c, const uint32_t* __restrict__ start,
                                                const short4* __restrict__ wbase, const float* __restrict__ srec,
                                                int np, float* __restrict__ F,
                                                int nbx, int nby, int nbz) {
    using B = SpreadBlock<D>;
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int blk = uni((int)blockIdx.x * 4 + wave);      // 4 waves per workgroup, neighbours along x
    if (blk >= nbx * nby * nbz) return;                   // uniform per wave
    const int bxi = blk % nbx, t2 = blk / nbx;
    const int byi = t2 % nby, bzi = t2 / nby;
    const int x0 = bxi * B::BX, y0 = byi * B::BY, z0 = bzi * B::BZ;
    const int x = x0 + (D == 3 ? (lane & 3) : (lane & 7));
    const int y = y0 + (D == 3 ? ((lane >> 2) & 3) : (lane >> 3));
    const int z = z0 + (D == 3 ? (lane >> 4) : 0);

    const int b0x = max((x0 - 1) >> c.L, 0), b1x = min((x0 + B::BX + 1) >> c.L, c.nb[0] - 1);
    const int b0y = max((y0 - 1) >> c.L, 0), b1y = min((y0 + B::BY + 1) >> c.L, c.nb[1] - 1);
    const int b0z = (D == 3) ? max((z0 - 1) >> c.L, 0) : 0;
    const int b1z = (D == 3) ? min((z0 + B::BZ + 1) >> c.L, c.nb[2] - 1) : 0;
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (int bz = b0z; bz <= b1z; bz++)
        for (int by = b0y; by <= b1y; by++) {
            const uint32_t row = (uint32_t)(((long long)bz * c.nb[1] + by) * c.nb[0]);
            const uint32_t s0 = (uint32_t)uni((int)start[row + b0x]);
            const uint32_t s1 = (uint32_t)uni((int)start[row + b1x + 1]);
            for (uint32_t s = s0; s < s1; s++) {
                const short4 b = wbase[s];
                const int kx = x - b.x, ky = y - b.y, kz = (D == 3) ? z - b.z : 0;
                const float* ph = srec + (long long)s * SRec<D>::STRIDE;
                const float cx = ph[SRec<D>::COEF], cy = ph[SRec<D>::COEF + 1];
                const float cz = (D == 3) ? ph[SRec<D>::COEF + 2 - (D == 3 ? 0 : 1)] : 0.f;
                const float p0 = ph[0], p1 = ph[1], p2 = ph[2], p3 = ph[3];
                const float q0 = ph[4], q1 = ph[5], q2 = ph[6], q3 = ph[7];
                float r0 = 1.f, r1 = 0.f, r2 = 0.f, r3 = 0.f;
                if (D == 3) { r0 = ph[8 % (4 * D)]; r1 = ph[9 % (4 * D)]; r2 = ph[10 % (4 * D)]; r3 = ph[11 % (4 * D)]; }
                if ((unsigned)kx < 4u && (unsigned)ky < 4u && (unsigned)kz < 4u) {
                    float W = pick4(kx, p0, p1, p2, p3) * pick4(ky, q0, q1, q2, q3);
                    if (D == 3) W *= pick4(kz, r0, r1, r2, r3);
                    ax += W * cx;
                    ay += W * cy;
                    az += W * cz;
                }
            }
        }
    if (x < g.n[0] && y < g.n[1] && z < g.n[2]) {
        const long long r = ((long long)z * g.n[1] + y) * g.n[0] + x;
        F[r] = ax;
        F[g.N + r] = ay;
        if (D == 3) F[2 * g.N + r] = az;
    }
}

// ---------------------------------------------------------------------------
// FP64 particle totals: momentum sum m U, min and sum of the last coordinate
// part[b*8 + 0..2] momentum, 3 min height, 4 sum height
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_particle_totals(PState A, int np, double* __restrict__ part) {
    __shared__ double sm[5][256];
    double p0 = 0, p1 = 0, p2 = 0, mn = 1e300, sh = 0;
    for (int s = blockIdx.x * 256 + threadIdx.x; s < np; s += gridDim.x * 256) {
        double m = (double)particle_mass(D, A.d[s], A.rp[s]);
        p0 += m * (double)A.u[0][s];
        p1 += m * (double)A.u[1][s];
        if (D == 3) p2 += m * (double)A.u[2][s];
        double hgt = (double)A.xh[D - 1][s] + (double)A.xl[D - 1][s];
        mn = fmin(mn, hgt);
        sh += hgt;
    }
    int t = threadIdx.x;
    sm[0][t] = p0; sm[1][t] = p1; sm[2][t] = p2; sm[3][t] = mn; sm[4][t] = sh;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) {
            sm[0][t] += sm[0][t + st];
            sm[1][t] += sm[1][t + st];
            sm[2][t] += sm[2][t + st];
            sm[3][t] = fmin(sm[3][t], sm[3][t + st]);
            sm[4][t] += sm[4][t + st];
        }
        __syncthreads();
    }
    if (t == 0)
        for (int k = 0; k < 5; k++) part[blockIdx.x * 8 + k] = sm[k][0];
}

__global__ void k_particle_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    int k = threadIdx.x;
    if (k >= 5) return;
    double acc = (k == 3) ? 1e300 : 0.0;
    for (int b = 0; b < nb; b++) acc = (k == 3) ? fmin(acc, part[b * 8 + k]) : acc + part[b * 8 + k];
    out[k] = acc;
}

// state in sorted order -> staging arrays in id order
template <int D>
__global__ __launch_bounds__(256) void k_unpermute(PState A, int np, const float* __restrict__ srec,
                                                   const float* __restrict__ fc, float* __restrict__ out) {
    // out layout: [xh D][xl D][u D][fh D][fc D] x np
    int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= np) return;
    int id = A.id[s];
#pragma unroll
    for (int a = 0; a < D; a++) {
        out[(long long)(0 * D + a) * np + id] = A.xh[a][s];
        out[(long long)(1 * D + a) * np + id] = A.xl[a][s];
        out[(long long)(2 * D + a) * np + id] = A.u[a][s];
        out[(long long)(3 * D + a) * np + id] =
            srec ? -srec[(long long)s * SRec<D>::STRIDE + SRec<D>::COEF + a] : 0.f;
        out[(long long)(4 * D + a) * np + id] = fc ? fc[(long long)a * np + s] : 0.f;
    }
}

// Angular velocities in id order: [component][id], 3 components in 3D, the
// z component in 2D.
template <int D>
__global__ __launch_bounds__(256) void k_unpermute_spin(PState A, int np, float* __restrict__ out) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= np) return;
    const int id = A.id[s];
#pragma unroll
    for (int a = 0; a < (D == 3 ? 3 : 1); a++) out[(long long)a * np + id] = A.w[a][s];
}

// Particle state from caller-owned device arrays in id order (positions as
// leading and trailing FP32 parts): PState A in id order (the first sort
// orders it).  (hi, lo) is renormalised with an error-free sum, so any split
// of the same value gives the same state.  Invalid input (a position outside
// the open box, a diameter <= 0, above dmax or above the limits of the host
// path, a density <= 0, anything not finite) raises FLAG_ARG.
template <int D>
__global__ __launch_bounds__(256) void k_set_state(const float* __restrict__ xh, const float* __restrict__ xl,
                                                   const float* __restrict__ v, const float* __restrict__ d,
                                                   const float* __restrict__ rp, int np, Grid g, float dmax,
                                                   PState A, uint32_t* flags) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= np) return;
    bool bad = false;
    const float di = d[i], ri = rp[i];
    bad |= !(di > 0.0f) || !(di <= dmax) || !(di <= 0.5f * (float)g.n[0]) || !(di <= 64.0f) || !(ri > 0.0f) ||
           !isfinite(ri);
#pragma unroll
    for (int a = 0; a < D; a++) {
        const long long k = (long long)a * np + i;
        float hi, lo;
        two_sum(xh[k], xl ? xl[k] : 0.0f, hi, lo);
        const float ua = v ? v[k] : 0.0f;
        // strictly inside (0, n): the leading part decides except on the walls
        bad |= !(hi >= 0.0f) || !(hi <= (float)g.n[a]) || (hi == 0.0f && !(lo > 0.0f)) ||
               (hi == (float)g.n[a] && !(lo < 0.0f)) || !isfinite(lo) || !isfinite(ua);
        A.xh[a][i] = hi;
        A.xl[a][i] = lo;
        A.u[a][i] = ua;
    }
    A.d[i] = di;
    A.rp[i] = ri;
    A.id[i] = i;
    if (A.fixa) A.fixa[i] = 0.0f;
    if (bad) atomicOr(flags, FLAG_ARG);
}

// ---------------------------------------------------------------------------
// launchers (called from runtime.hip)
// ---------------------------------------------------------------------------
static inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

void particles_sort(int D, PBuf& b, int np, const PCfg& c, hipStream_t s) {
    // the bin counts are zero here: cleared at creation and by the scan of
    // the previous sort
    long long nbins = c.nbins;
    if (D == 3)
        hipLaunchKernelGGL(k_bin_count<3>, dim3(nb256(np)), dim3(256), 0, s, b.A, np, c, b.cnt, b.keys, b.slot, b.flags);
    else
        hipLaunchKernelGGL(k_bin_count<2>, dim3(nb256(np)), dim3(256), 0, s, b.A, np, c, b.cnt, b.keys, b.slot, b.flags);
    scan_exclusive<uint32_t>(b.cnt, b.start, nbins + 1, b.scan_u32, nullptr, true, s);
    hipLaunchKernelGGL(k_scatter, dim3(nb256(np)), dim3(256), 0, s, b.keys, b.slot, b.start, b.A.id, b.tmpid, np);
    if (D == 3)
        hipLaunchKernelGGL(k_reorder<3>, dim3(nb256(np)), dim3(256), 0, s, b.A, b.B, b.keys, b.start, b.tmpid,
                           b.keys_sorted, b.pos4, np);
    else
        hipLaunchKernelGGL(k_reorder<2>, dim3(nb256(np)), dim3(256), 0, s, b.A, b.B, b.keys, b.start, b.tmpid,
                           b.keys_sorted, b.pos4, np);
    PState t = b.A;
    b.A = b.B;
    b.B = t;
}

template <class Src>
static void interp_tile_2d(PBuf& b, int np, const Grid& g, const PCfg& c, Src src, hipStream_t s) {
    using T = InterpTile<2>;
    const int E = 1 << c.L;
    const int bx = T::CX / E, by = T::CY / E;
    int ntx = (c.nb[0] + bx - 1) / bx, nty = (c.nb[1] + by - 1) / by;
    const dim3 grid((unsigned)((long long)ntx * nty));
    if (c.lagrange)
        hipLaunchKernelGGL((k_interp_tile<2, Src, true>), grid, dim3(256), 0, s, b.A, np, g, c, b.start, src,
                           b.drho_i, b.j_i, b.wbase, b.srec, ntx, nty);
    else
        hipLaunchKernelGGL((k_interp_tile<2, Src, false>), grid, dim3(256), 0, s, b.A, np, g, c, b.start, src,
                           b.drho_i, b.j_i, b.wbase, b.srec, ntx, nty);
}

// D2Q9 with bins of edge 1 or 2: moments straight from the populations f
// (storage FP32 or FP16 with scale 2^sl2); no separate moments pass.
void particles_interp_from_populations(PBuf& b, int np, const Grid& g, const PCfg& c, const void* f, int fp16,
                                       int sl2, hipStream_t s) {
    if (fp16) {
        StoreF16 st{ldexpf(1.0f, sl2), ldexpf(1.0f, -sl2)};
        interp_tile_2d(b, np, g, c, PopSrc<StoreF16>{(const _Float16*)f, st}, s);
    } else {
        interp_tile_2d(b, np, g, c, PopSrc<StoreF32>{(const float*)f, StoreF32{1.f, 1.f}}, s);
    }
}

void particles_interp(int D, PBuf& b, int np, const Grid& g, const PCfg& c, const float4* mom, hipStream_t s) {
    if (c.L <= 1) {
        const int E = 1 << c.L;
        if (D == 3) {
            using T = InterpTile<3>;
            const int bx = T::CX / E, by = T::CY / E, bz = T::CZ / E;
            int ntx = (c.nb[0] + bx - 1) / bx, nty = (c.nb[1] + by - 1) / by, ntz = (c.nb[2] + bz - 1) / bz;
            const dim3 grid((unsigned)((long long)ntx * nty * ntz));
            if (c.lagrange)
                hipLaunchKernelGGL((k_interp_tile<3, MomSrc, true>), grid, dim3(256), 0, s, b.A, np, g, c, b.start,
                                   MomSrc{mom}, b.drho_i, b.j_i, b.wbase, b.srec, ntx, nty);
            else
                hipLaunchKernelGGL((k_interp_tile<3, MomSrc, false>), grid, dim3(256), 0, s, b.A, np, g, c, b.start,
                                   MomSrc{mom}, b.drho_i, b.j_i, b.wbase, b.srec, ntx, nty);
        } else {
            interp_tile_2d(b, np, g, c, MomSrc{mom}, s);
        }
        return;
    }
    long long threads = (long long)np * (D == 3 ? 16 : 4);
    const dim3 grid(nb256(threads));
    if (D == 3 && c.lagrange)
        hipLaunchKernelGGL((k_interp<3, true>), grid, dim3(256), 0, s, b.A, np, g, mom, b.drho_i, b.j_i, b.wbase, b.srec);
    else if (D == 3)
        hipLaunchKernelGGL((k_interp<3, false>), grid, dim3(256), 0, s, b.A, np, g, mom, b.drho_i, b.j_i, b.wbase, b.srec);
    else if (c.lagrange)
        hipLaunchKernelGGL((k_interp<2, true>), grid, dim3(256), 0, s, b.A, np, g, mom, b.drho_i, b.j_i, b.wbase, b.srec);
    else
        hipLaunchKernelGGL((k_interp<2, false>), grid, dim3(256), 0, s, b.A, np, g, mom, b.drho_i, b.j_i, b.wbase, b.srec);
}

template <int D>
static void dem_impl(PBuf& b, int np, const PCfg& c, bool one_group, hipStream_t s) {
    // the island chain works on the active particles only (grid-stride)
    const unsigned grid_act = std::min<unsigned>(nb256(np), 128u);
    const MdBuf md{b.cmd, b.cpid, b.hcnt, b.hkey, b.hT, b.gmd, b.cms};
    hipLaunchKernelGGL(k_classify<D>, dim3(nb256(np)), dim3(256), 0, s, b.A, b.Bn, np, c, b.start, b.pos4,
                       b.keys_sorted, b.drho_i, b.j_i, b.srec, b.fc, b.actcc, b.bsum64, b.counters, b.flags,
                       b.hcnt);
    // block offsets and the totals (candidates, active) -> counters[0..1]
    if ((long long)nb256(np) <= RAW_MAX_BLOCKS) {
        hipLaunchKernelGGL((k_collect<D, true>), dim3(nb256(np)), dim3(256), 0, s, b.A, np, c, b.start, b.pos4,
                           b.keys_sorted, b.actcc, b.bsum64, b.prefix, b.alist, b.aidx, b.cand, b.ccount, b.parent,
                           b.isize, b.fill, b.counters);
    } else {
        hipLaunchKernelGGL((k_scan_top<unsigned long long>), dim3(1), dim3(TOP_THREADS), 0, s, b.bsum64,
                           (long long)nb256(np), (unsigned long long*)(void*)b.counters);
        hipLaunchKernelGGL((k_collect<D, false>), dim3(nb256(np)), dim3(256), 0, s, b.A, np, c, b.start, b.pos4,
                           b.keys_sorted, b.actcc, b.bsum64, b.prefix, b.alist, b.aidx, b.cand, b.ccount, b.parent,
                           b.isize, b.fill, b.counters);
    }
    if (one_group) {
        hipLaunchKernelGGL(k_island_setup<D>, dim3(1), dim3(SETUP_THREADS), 0, s, b.A, c, b.alist, b.ccount, b.prefix,
                           b.cand, b.aidx, b.parent, b.isize, b.irank, b.fill, b.lanemember, b.loc, b.bigroot,
                           b.bigoff, b.bigmember, b.cdata, md, b.counters, b.lane_cap);
    } else {
        hipLaunchKernelGGL(k_uf_hook, dim3(grid_act), dim3(256), 0, s, b.alist, b.ccount, b.prefix, b.cand, b.aidx, b.parent,
                           b.counters);
        hipLaunchKernelGGL(k_uf_flatten, dim3(grid_act), dim3(256), 0, s, b.parent, b.isize, b.counters);
        hipLaunchKernelGGL(k_island_class<D>, dim3(grid_act), dim3(256), 0, s, b.A, b.alist, b.ccount, b.prefix,
                           b.cand, b.parent, b.isize, b.irank, b.bigroot,
                           b.counters);
        hipLaunchKernelGGL(k_island_place, dim3(grid_act), dim3(256), 0, s, b.parent, b.isize, b.irank, b.fill,
                           b.lanemember, b.loc, b.bigoff, b.bigmember, b.bigroot, b.counters);
        hipLaunchKernelGGL(k_cand_prep<D>, dim3(grid_act), dim3(256), 0, s, b.A, c, b.alist, b.ccount, b.prefix, b.cand,
                           b.aidx, b.loc, b.cdata, md, b.counters);
    }
    // (a workgroup per packed wave, four per wave of islands of one or two without Mindlin)
    const dim3 gsmall(std::max<unsigned>(grid_act * 4, 256u));
    const dim3 gsplit(4 * gsmall.x);
    if (c.contact >= PIBM_CONTACT_HERTZ_MINDLIN) {
        hipLaunchKernelGGL((k_island_small<D, true>), gsmall, dim3(64), 0, s, b.A, b.Bn, np, c, b.lanemember, b.alist,
                           b.ccount, b.prefix, b.parent, b.isize, b.cdata, b.drho_i, b.j_i, b.srec, b.fc, b.flags,
                           b.counters, md);
        hipLaunchKernelGGL((k_island_big<D, true>), dim3(256), dim3(256), 0, s, b.A, b.Bn, np, c, b.bigmember,
                           b.bigoff, b.bigroot, b.isize, b.alist, b.ccount, b.prefix, b.cdata, b.drho_i, b.j_i,
                           b.srec, b.fc, b.gdx, b.gu, (long long)np, b.flags, b.counters, md);
    } else {
        hipLaunchKernelGGL((k_island_small<D, false>), gsplit, dim3(64), 0, s, b.A, b.Bn, np, c, b.lanemember, b.alist,
                           b.ccount, b.prefix, b.parent, b.isize, b.cdata, b.drho_i, b.j_i, b.srec, b.fc, b.flags,
                           b.counters, md);
        hipLaunchKernelGGL((k_island_big<D, false>), dim3(256), dim3(256), 0, s, b.A, b.Bn, np, c, b.bigmember,
                           b.bigoff, b.bigroot, b.isize, b.alist, b.ccount, b.prefix, b.cdata, b.drho_i, b.j_i,
                           b.srec, b.fc, b.gdx, b.gu, (long long)np, b.flags, b.counters, md);
    }
}

void particles_dem(int D, PBuf& b, int np, const PCfg& c, bool one_group, hipStream_t s) {
    if (D == 3) dem_impl<3>(b, np, c, one_group, s);
    else dem_impl<2>(b, np, c, one_group, s);
    // the new positions, velocities and spins become the current ones
    for (int a = 0; a < 3; a++) {
        std::swap(b.A.xh[a], b.Bn.xh[a]);
        std::swap(b.A.xl[a], b.Bn.xl[a]);
        std::swap(b.A.u[a], b.Bn.u[a]);
        std::swap(b.A.w[a], b.Bn.w[a]);
    }
}

void particles_spread(int D, PBuf& b, int np, const PCfg& c, const Grid& g, float* F, hipStream_t s) {
    if (c.L == 0) {
        if (D == 3) spread_fields<3, 3>(b, np, c, g, nullptr, F, s);
        else spread_fields<2, 2>(b, np, c, g, nullptr, F, s);
        return;
    }

    if (D == 3) {
        using B = SpreadBlock<3>;
        int nbx = (g.n[0] + B::BX - 1) / B::BX, nby = (g.n[1] + B::BY - 1) / B::BY, nbz = (g.n[2] + B::BZ - 1) / B::BZ;
        long long nblk = (long long)nbx * nby * nbz;
        hipLaunchKernelGGL(k_spread<3>, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, s, g, c, b.start, b.wbase,
                           b.srec, np, F, nbx, nby, nbz);
    } else {
        using B = SpreadBlock<2>;
        int nbx = (g.n[0] + B::BX - 1) / B::BX, nby = (g.n[1] + B::BY - 1) / B::BY;
        long long nblk = (long long)nbx * nby;
        hipLaunchKernelGGL(k_spread<2>, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, s, g, c, b.start, b.wbase,
                           b.srec, np, F, nbx, nby, 1);
    }
}

int particles_totals_blocks() { return 256; }

void particles_totals(int D, PBuf& b, int np, double* part, double* out, hipStream_t s) {
    int nb = particles_totals_blocks();
    if (D == 3) hipLaunchKernelGGL(k_particle_totals<3>, dim3(nb), dim3(256), 0, s, b.A, np, part);
    else hipLaunchKernelGGL(k_particle_totals<2>, dim3(nb), dim3(256), 0, s, b.A, np, part);
    hipLaunchKernelGGL(k_particle_final, dim3(1), dim3(64), 0, s, part, nb, out);
}

void particles_unpermute_spin(int D, PBuf& b, int np, float* out, hipStream_t s) {
    if (D == 3) hipLaunchKernelGGL(k_unpermute_spin<3>, dim3(nb256(np)), dim3(256), 0, s, b.A, np, out);
    else hipLaunchKernelGGL(k_unpermute_spin<2>, dim3(nb256(np)), dim3(256), 0, s, b.A, np, out);
}

void particles_set_state(int D, PBuf& b, int np, const Grid& g, const float* xh, const float* xl, const float* v,
                         const float* d, const float* rp, float dmax, hipStream_t s) {
    if (D == 3)
        hipLaunchKernelGGL(k_set_state<3>, dim3(nb256(np)), dim3(256), 0, s, xh, xl, v, d, rp, np, g, dmax, b.A, b.flags);
    else
        hipLaunchKernelGGL(k_set_state<2>, dim3(nb256(np)), dim3(256), 0, s, xh, xl, v, d, rp, np, g, dmax, b.A, b.flags);
}

void particles_unpermute(int D, PBuf& b, int np, bool have_forces, float* out, hipStream_t s) {
    const float* coef = have_forces ? b.srec : nullptr;
    const float* fc = have_forces ? b.fc : nullptr;
    if (D == 3) hipLaunchKernelGGL(k_unpermute<3>, dim3(nb256(np)), dim3(256), 0, s, b.A, np, coef, fc, out);
    else hipLaunchKernelGGL(k_unpermute<2>, dim3(nb256(np)), dim3(256), 0, s, b.A, np, coef, fc, out);
}

}  // namespace pibm
