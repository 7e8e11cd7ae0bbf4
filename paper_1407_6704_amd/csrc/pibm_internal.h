// pibm_internal.h -- device-side definitions shared by the HIP sources of
// libpibm (gfx950, wave64).  Not part of the public ABI (include/pibm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pibm.h"

namespace pibm {

// ---------------------------------------------------------------------------
// Lattices: D2Q9, D3Q15 and D3Q19 (c = 1, c_s^2 = 1/3), direction order of
// the ABI.
// ---------------------------------------------------------------------------
template <int Q> struct Lattice;

template <> struct Lattice<9> {
    static constexpr int D = 2;
    __host__ __device__ static constexpr int ex(int q) {
        constexpr int t[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
        return t[q];
    }
    __host__ __device__ static constexpr int ey(int q) {
        constexpr int t[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
        return t[q];
    }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr float w(int q) {
        return q == 0 ? 4.0f / 9.0f : (q < 5 ? 1.0f / 9.0f : 1.0f / 36.0f);
    }
    __host__ __device__ static constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
};

// D3Q15, the three-dimensional lattice of Sec. 2.1: rest, 6 faces, 8 corners.
template <> struct Lattice<15> {
    static constexpr int D = 3;
    __host__ __device__ static constexpr int ex(int q) {
        constexpr int t[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
        return t[q];
    }
    __host__ __device__ static constexpr int ey(int q) {
        constexpr int t[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
        return t[q];
    }
    __host__ __device__ static constexpr int ez(int q) {
        constexpr int t[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};
        return t[q];
    }
    __host__ __device__ static constexpr float w(int q) {
        return q == 0 ? 2.0f / 9.0f : (q < 7 ? 1.0f / 9.0f : 1.0f / 72.0f);
    }
    __host__ __device__ static constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
};

template <> struct Lattice<19> {
    static constexpr int D = 3;
    __host__ __device__ static constexpr int ex(int q) {
        constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        return t[q];
    }
    __host__ __device__ static constexpr int ey(int q) {
        constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        return t[q];
    }
    __host__ __device__ static constexpr int ez(int q) {
        constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        return t[q];
    }
    __host__ __device__ static constexpr float w(int q) {
        return q == 0 ? 1.0f / 3.0f : (q < 7 ? 1.0f / 18.0f : 1.0f / 36.0f);
    }
    __host__ __device__ static constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
};

// Storage codecs: the stored quantity is the deviation h = f - w, in FP32,
// or scaled by 2^s and rounded to FP16 (nearest-even).  Arithmetic is FP32.
// load_stream/store_stream mark accesses that are used once per pass
// (non-temporal), for the streaming lattice kernels.
struct StoreF32 {
    using T = float;
    float scale, inv_scale;
    __device__ __forceinline__ float load(const T* p) const { return *p; }
    __device__ __forceinline__ void store(T* p, float v) const { *p = v; }
    __device__ __forceinline__ float load_stream(const T* p) const { return __builtin_nontemporal_load(p); }
    __device__ __forceinline__ void store_stream(T* p, float v) const { __builtin_nontemporal_store(v, p); }
};
struct StoreF16 {
    using T = _Float16;
    float scale, inv_scale;
    __device__ __forceinline__ float load(const T* p) const { return (float)(*p) * inv_scale; }
    __device__ __forceinline__ void store(T* p, float v) const { *p = (_Float16)(v * scale); }
    __device__ __forceinline__ float load_stream(const T* p) const {
        return (float)__builtin_nontemporal_load(p) * inv_scale;
    }
    __device__ __forceinline__ void store_stream(T* p, float v) const {
        __builtin_nontemporal_store((_Float16)(v * scale), p);
    }
};

struct Grid {
    int n[3];
    int periodic[3];
    long long N;       // nodes
};

// BGK collision with Guo forcing (Eq. lbm2, lbm9) of node r = (x, y, z) and
// push streaming into fout, with halfway bounce-back on wall links (Sec. 3.3)
// and wrap-around on periodic axes.  F: the force density at the node (the
// spread field plus any constant body force).  omega = 1/tau, fpref =
// 1 - 1/(2 tau).  The stored populations are deviations from the rest state.
// In two parts, so that a caller can issue the loads early: collide_load
// reads the node's populations, collide_finish does the rest.
template <int Q, class S>
__device__ __forceinline__ void collide_load(const typename S::T* __restrict__ fin, long long r, const Grid& g,
                                             float* h, const S& st) {
#pragma unroll
    for (int q = 0; q < Q; q++) h[q] = st.load_stream(fin + (long long)q * g.N + r);
}

template <int Q, class S>
__device__ __forceinline__ void collide_finish(const float* h, typename S::T* __restrict__ fout, long long r, int x,
                                               int y, int z, const Grid& g, float Fx, float Fy, float Fz,
                                               float omega, float fpref, const S& st) {
    using L = Lattice<Q>;
    const long long N = g.N;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    float dr = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        dr += h[q];
        if (L::ex(q)) jx += L::ex(q) * h[q];
        if (L::ey(q)) jy += L::ey(q) * h[q];
        if (L::ez(q)) jz += L::ez(q) * h[q];
    }
    const float rho = 1.0f + dr;
    const float ir = 1.0f / rho;
    const float ux = (jx + 0.5f * Fx) * ir, uy = (jy + 0.5f * Fy) * ir, uz = (jz + 0.5f * Fz) * ir;
    const float uu = ux * ux + uy * uy + uz * uz;
    const float uF = ux * Fx + uy * Fy + uz * Fz;

    // neighbour offsets with wrap (periodic) or a bounce flag (wall)
    const long long sx = 1, sy = nx, sz = (long long)nx * ny;
    const bool xlo = (x == 0), xhi = (x == nx - 1);
    const bool ylo = (y == 0), yhi = (y == ny - 1);
    const bool zlo = (z == 0), zhi = (z == nz - 1);

#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int ex = L::ex(q), ey = L::ey(q), ez = L::ez(q);
        const float eu = ex * ux + ey * uy + ez * uz;
        const float eF = ex * Fx + ey * Fy + ez * Fz;
        const float heq = L::w(q) * (dr + rho * (3.0f * eu + 4.5f * eu * eu - 1.5f * uu));
        const float src = fpref * L::w(q) * (3.0f * (eF - uF) + 9.0f * eu * eF);
        const float hs = h[q] - omega * (h[q] - heq) + src;

        long long dst = r;
        bool out = false;
        if (ex > 0) { if (xhi) { if (g.periodic[0]) dst -= (nx - 1) * sx; else out = true; } else dst += sx; }
        if (ex < 0) { if (xlo) { if (g.periodic[0]) dst += (nx - 1) * sx; else out = true; } else dst -= sx; }
        if (ey > 0) { if (yhi) { if (g.periodic[1]) dst -= (ny - 1) * sy; else out = true; } else dst += sy; }
        if (ey < 0) { if (ylo) { if (g.periodic[1]) dst += (ny - 1) * sy; else out = true; } else dst -= sy; }
        if (ez > 0) { if (zhi) { if (g.periodic[2]) dst -= (long long)(nz - 1) * sz; else out = true; } else dst += sz; }
        if (ez < 0) { if (zlo) { if (g.periodic[2]) dst += (long long)(nz - 1) * sz; else out = true; } else dst -= sz; }
        if (out)
            st.store(fout + (long long)L::opp(q) * N + r, hs);
        else
            st.store(fout + (long long)q * N + dst, hs);
    }
}

template <int Q, class S>
__device__ __forceinline__ void collide_node(const typename S::T* __restrict__ fin, typename S::T* __restrict__ fout,
                                             long long r, int x, int y, int z, const Grid& g, float Fx, float Fy,
                                             float Fz, float omega, float fpref, const S& st) {
    float h[Q];
    collide_load<Q, S>(fin, r, g, h, st);
    collide_finish<Q, S>(h, fout, r, x, y, z, g, Fx, Fy, Fz, omega, fpref, st);
}

// Which node rows the particle gather can reach: the cell list's bin starts
// (start == nullptr: every row), the grid and the binning.
struct RowMask {
    const uint32_t* start;
    int n[3];
    int nb[3];
    int L;
};

// ---------------------------------------------------------------------------
// Double-float helpers (value = hi + lo, |lo| <= ulp(hi)/2), FP32 only.
// Error-free transformations must not be contracted into FMAs, hence the
// contract(off) pragmas here and wherever such sequences appear.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__host__ __device__ __forceinline__ void fast_two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
    s = a + b;
    e = b - (s - a);
}
// (hi, lo) += d
__host__ __device__ __forceinline__ void df_add(float& hi, float& lo, float d) {
#pragma clang fp contract(off)
    float s, e;
    two_sum(hi, d, s, e);
    e += lo;
    fast_two_sum(s, e, hi, lo);
}

// Dual cell floor(X - 1/2) of X = hi + lo, exactly (hi - 1/2 is exact for
// hi >= 1/4 and cannot reach an integer below; lo only matters when
// hi - 1/2 is an integer).
__device__ __forceinline__ int dual_cell(float hi, float lo) {
    float t = hi - 0.5f;
    float c = floorf(t);
    int ci = (int)c;
    if (t == c && lo < 0.0f) ci -= 1;
    return ci;
}
// X - 1/2 - floor(X - 1/2), in [0, 1) up to rounding of the last add.
__device__ __forceinline__ float dual_frac(float hi, float lo, int c) {
    float f = ((hi - 0.5f) - (float)c) + lo;
    return fminf(fmaxf(f, 0.0f), 0.99999994f);
}

// Particle state, structure of arrays in sorted (bin, id) order.
struct PState {
    float* xh[3];
    float* xl[3];
    float* u[3];
    float* w[3];        // angular velocity (Hertz-Mindlin only, else null): x, y, z in 3D; z in 2D
    float* fixa;        // fixed obstacle points (bodies only, else null): their area; 0 for moving ones
    float* d;
    float* rp;
    int* id;
};

// Device-side error flags (bit mask), latched until read by the host.
enum : unsigned {
    FLAG_SKIN = 1u,
    FLAG_CAPACITY = 2u,
    FLAG_UNSTABLE = 4u,
    FLAG_ARG = 8u,       // a particle array handed over in device memory was invalid
};

// Counters written by the particle kernels (one small device array).
enum {
    CNT_CAND = 0,        // directed candidate entries (low word of the scan total)
    CNT_ACTIVE = 1,      // active particles of the current step (high word)
    CNT_WAVES = 2,       // packed waves of small islands
    CNT_BIG = 3,         // islands larger than one wave
    CNT_PAIRC = 4,       // islands of two whose members touch at the start of the step
    CNT_CLASS = 8,       // 65 class counters (index 1..64 sizes, 65 big) at 8..73
    CNT_WAVEBASE = 80,   // 66 prefix entries at 80..145
    CNT_SIZE = 160
};

constexpr int WAVE = 64;
constexpr unsigned NUM_XCD = 8;

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Map dispatch index b (on XCD b % 8) to a logical block so that every
// XCD works on one contiguous eighth of the index space: neighbouring nodes
// and neighbouring sorted particles then share an L2.  A bijection.
__device__ __forceinline__ unsigned xcd_block() {
    const unsigned n = gridDim.x, b = blockIdx.x;
    const unsigned per = n / NUM_XCD, rem = n % NUM_XCD;
    const unsigned x = b % NUM_XCD, i = b / NUM_XCD;
    return x * per + min(x, rem) + i;
}
// Tile coordinates for tile kernels whose tiles read a halo shared with
// their neighbours.  The tile grid is cut into NUM_XCD bands along axis A
// (one that gravity does not point along, so the particles spread evenly over
// the bands) and each XCD walks its own band, a row of tiles at a time,
// layer after layer: the halo a tile reads in the neighbouring rows and
// layers was then fetched into the same L2 shortly before, and every XCD
// has about the same work.  A bijection of the dispatch indices onto the
// tiles (the logical index from xcd_block() is read band-major).
__device__ __forceinline__ void banded_tile(int ntx, int nty, int ntz, int A, int& tx, int& ty, int& tz) {
    const int L = (int)xcd_block();
    const int nA = A == 0 ? ntx : nty;                   // tiles along the banded axis
    const int other = (A == 0 ? nty : ntx) * ntz;        // tiles of one band position
    const int q = nA / (int)NUM_XCD, r = nA % (int)NUM_XCD;
    int b = 0;
    for (int k = 1; k < (int)NUM_XCD; k++)
        if ((k * q + min(k, r)) * other <= L) b = k;
    const int a0 = b * q + min(b, r), nb = q + (b < r ? 1 : 0);
    const int off = L - a0 * other;
    if (A == 1) {                                        // rows of x tiles, band rows, then layers
        tx = off % ntx;
        const int rest = off / ntx;
        ty = a0 + rest % nb;
        tz = rest / nb;
    } else {                                             // band columns, then rows, then layers
        tx = a0 + off % nb;
        const int rest = off / nb;
        ty = rest % nty;
        tz = rest / nty;
    }
}
constexpr float PI_F = 3.14159265358979323846f;

// Powers of the drag recurrence factor q = 1 - hc for 0 < hc < 2 (|q| < 1):
// qm = q^m and omq = 1 - q^m.  For q > 0 through log1p/expm1, accurate when
// hc is small; for q <= 0 the powers alternate in sign and 1 - q^m has no
// cancellation.
__device__ __forceinline__ void drag_power(float hc, int m, float& qm, float& omq) {
    if (hc < 1.0f) {
        const float l = (float)m * log1pf(-hc);
        qm = expf(l);
        omq = -expm1f(l);
    } else {
        const float p = m == 0 ? 1.0f : powf(hc - 1.0f, (float)m);
        qm = (m & 1) ? -p : p;
        omq = 1.0f - qm;
    }
}

// Hardware reciprocal, square root and reciprocal square root (about one
// unit in the last place).  The DEM sub-step runs thousands of times per
// lattice step as one wave's serial chain of instructions, where a correctly
// rounded division or square root expands into a dozen instructions; these
// are single instructions.  Their extra rounding is of the order of FP32's.
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsq_fast(float x) { return __builtin_amdgcn_rsqf(x); }

// Particle mass: sphere (3D) or disk of unit depth (2D).
__device__ __forceinline__ float particle_mass(int D, float d, float rp) {
    return D == 3 ? rp * (PI_F / 6.0f) * d * d * d : rp * 0.25f * PI_F * d * d;
}

// Particle-side constants of one configuration.
struct PCfg {
    int D;
    int n[3];
    int L;              // bin edge 2^L dual cells
    int nb[3];          // bins per axis
    long long nbins;
    float skin;
    int contact;
    float kn, zeta, ks;
    int n_sub;
    float h;            // 1 / n_sub
    float rho0;
    float g[3];
    int maxc;
    float eps;          // bound on the trailing position parts left out by screening
    int H;              // neighbour-search half-width in bins: ceil((d_max + skin + eps) / 2^L)
    float dmax;         // largest diameter present
    int lagrange;       // 1: gather with the Lagrange polynomials of Eq. lbm5-lbm6
    float hk;           // Hertz: (4/3) E*, so that F_n = hk sqrt(R*) delta^(3/2)
    float kt8;          // Mindlin: 8 G*, so that k_t = kt8 sqrt(delta R*)
    float mu;           // Coulomb friction coefficient
    int microslip;      // 1: the Mindlin-Deresiewicz micro-slip factors (contact model 5)
    int hmax;           // tangential-history entries per particle: max candidates + D walls
};

// Per-candidate constants of the active sub-steps.
struct CandData {
    int local;      // partner index in the island's state array
    float r0[3];    // X_self - X_partner at the start of the step
    float K0;       // r_c^2 - |r0|^2, accurate to FP32 relative precision
    float rc;       // (d_self + d_partner) / 2
    float gam;      // dashpot coefficient 2 zeta sqrt(kn m_eff)
};

// Tangential state of one Hertz-Mindlin contact, TSN floats: the force T on
// the particle (3), then for the micro-slip form the loading direction (3),
// k (0 loading, 1 unloading, 2 reloading), T*, T** and the normal force of
// the previous sub-step.  The history slots and the big-island scratch keep
// it in this order.
constexpr int TSN = 10;

// The Hertz-Mindlin buffers handed to the DEM kernels (all null for the
// other contact models); see PBuf.
struct MdBuf {
    float4* cmd;        // per candidate entry: tangential force on the particle (xyz), 8 G* sqrt(R*) (w)
    int* cpid;          // per candidate entry: partner id
    uint32_t* hcnt;     // per particle id: history entries
    int* hkey;          // per particle id, hmax slots: partner id, or -1 - (2 axis + side) for a wall
    float* hT;          // per slot: tangential state (TSN floats)
    float* gmd;         // big islands: spin [2][3][cap], wall states [3 TSN][cap], wall sides [cap]
    float4* cms;        // per candidate entry, two float4: the rest of the tangential state
                        // (loading direction, previous F_n), (k, T*, T**, 0)
};

// Spreading record of one sorted particle slot: the 4 D one-dimensional
// delta-kernel weights of Eq. lbm11 (4 per axis), the x index of the first
// stencil node (int bits), then the D spreading coefficients A_p gbar of the
// forward step, padded to whole float4s.  Interpolation writes the weights
// and the base, the DEM kernels the coefficients; spreading reads each
// record as one contiguous run.
template <int D> struct SRec {
    static constexpr int STRIDE = D == 3 ? 16 : 12;   // floats per slot
    static constexpr int BASE = 4 * D;
    static constexpr int COEF = 4 * D + 1;
};

// Device buffers of the particle side (carved from the workspace).
struct PBuf {
    PState A, B, Bn;             // current, reorder target, next (after DEM)
    uint32_t *cnt, *start, *keys, *slot, *keys_sorted;
    int* tmpid;                  // particle ids grouped by bin (unranked within a bin)
    float4* pos4;                // (x, y, z) leading parts and d, sorted order
    uint32_t* scan_u32;          // scan block sums
    unsigned long long *actcc, *prefix, *bsum64;   // bsum64: per-block totals of actcc
    float *drho_i, *j_i, *srec, *fc;     // srec: spreading records (SRec), per sorted slot
    short4* wbase;
    uint32_t *alist, *aidx, *cand, *ccount, *parent, *isize, *irank, *fill, *loc, *bigroot, *bigoff, *bigmember;
    int* lanemember;
    CandData* cdata;
    float *gdx, *gu;
    // Hertz-Mindlin: per-candidate tangential force (xyz) and 8 G* sqrt(R*) (w),
    // partner id; per-particle-id history (count, partner ids or wall codes
    // -1 - (2 axis + side), forces); spin and wall scratch of big islands
    float4* cmd;
    int* cpid;
    uint32_t* hcnt;
    int* hkey;
    float* hT;
    float* gmd;
    float4* cms;
    uint32_t* counters;
    uint32_t* flags;
    long long cand_cap, lane_cap;
};

}  // namespace pibm
