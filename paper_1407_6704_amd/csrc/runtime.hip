// runtime.hip -- C ABI of libpibm (include/pibm.h): configuration checks,
// workspace carving, host I/O and the launch sequence of one coupled step.
// Every launch goes to the context's stream; only I/O, diagnostics and
// pibm_synchronize wait for it.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pibm_internal.h"

namespace pibm {
constexpr size_t CAND_BYTES = sizeof(CandData);

void lattice_moments(int Q, int fp16, int sl2, const void* f, float4* mom, long long N, const RowMask& m,
                     hipStream_t s);
void lattice_collide(int Q, int fp16, int sl2, const void* fin, void* fout, const float* F, int hasF,
                     const float* ff, const Grid& g, float tau, hipStream_t s);
void lattice_init_eq(int Q, int fp16, int sl2, void* f, const float* rho, const float* u, long long N,
                     hipStream_t s);
void lattice_decode(int fp16, int sl2, const void* f, float* out, long long n, hipStream_t s);
void lattice_encode(int fp16, int sl2, void* f, const float* in, long long n, hipStream_t s);
void lattice_fields(const float4* mom, float* rho, float* u, long long N, int D, hipStream_t s);
int lattice_totals_blocks();
void lattice_totals(int Q, int fp16, int sl2, const void* f, long long N, double* part, double* out,
                    hipStream_t s);
long long scan_blocks(long long n);
void particles_sort(int D, PBuf& b, int np, const PCfg& c, hipStream_t s);
void particles_interp(int D, PBuf& b, int np, const Grid& g, const PCfg& c, const float4* mom, hipStream_t s);
void particles_unpermute_spin(int D, PBuf& b, int np, float* out, hipStream_t s);
void particles_interp_from_populations(PBuf& b, int np, const Grid& g, const PCfg& c, const void* f, int fp16,
                                       int sl2, hipStream_t s);
void particles_dem(int D, PBuf& b, int np, const PCfg& c, bool one_group, hipStream_t s);
void particles_spread(int D, PBuf& b, int np, const PCfg& c, const Grid& g, float* F, hipStream_t s);
void particles_spread_collide(int Q, int fp16, int sl2, const PBuf& b, int np, const PCfg& c, const Grid& g,
                              const void* fin, void* fout, const float* ff, float tau, hipStream_t s);
int particles_totals_blocks();
void particles_totals(int D, PBuf& b, int np, double* part, double* out, hipStream_t s);
void particles_unpermute(int D, PBuf& b, int np, bool have_forces, float* out, hipStream_t s);
void particles_set_state(int D, PBuf& b, int np, const Grid& g, const float* xh, const float* xl, const float* v,
                         const float* d, const float* rp, float dmax, hipStream_t s);
void lattice_add_const(const float* in, float* out, long long N, int D, const float* c, hipStream_t s);
void particles_spread_adjoint(int D, PBuf& b, int np, const PCfg& c, const Grid& g, const float* coef, float* out,
                              hipStream_t s);
void adj_fill(float* p, long long n, float v, hipStream_t s);
void adj_save_state(int D, const PBuf& b, int np, float* out, hipStream_t s);
void adj_save_const(const PBuf& b, int np, float* d, float* rp, hipStream_t s);
void adj_load_state(int D, PBuf& b, int np, const float* in, const float* d, const float* rp, hipStream_t s);
void adj_df_collapse(const float* hi, const float* lo, float* out, long long n, hipStream_t s);
int adj_collide_blocks(long long N);
int adj_particle_blocks(int np);
void adj_collide(int Q, int fp16, int sl2, const float* abar, const void* ft, const float* Ft, int hasF,
                 const float* ff, const Grid& g, float tau, float4* mom, float* Fbar, float4* Mc, float* tpart,
                 hipStream_t s);
void adj_assemble(int Q, const float* abar, const float4* Mc, const float* Sf, int hasS, const Grid& g, float tau,
                  float* abar_out, hipStream_t s);
void adj_particles(int D, PBuf& b, int np, const Grid& g, const PCfg& c, int two_way, const float4* mom,
                   const float* Fbar, const float* xbh, const float* xbl, const float* ub, float* xbh_o,
                   float* xbl_o, float* ub_o, float* coefS, float* gpart, hipStream_t s);
void adj_accumulate(const float* tpart, int ntb, const float* gpart, int ngb, float* acc, hipStream_t s);
void adj_pack_mom(const float* in, int comps, long long n, float4* out, hipStream_t s);

// Layout of the caller's rollout buffer (see pibm_rollout_bytes).
struct Rollout {
    int steps = 0, K = 0, nck = 0;
    bool valid = false;
    int taped = -1;               // the segment whose steps the tape holds (-1: none)
    std::vector<char*> ck_f;      // populations (storage format) at steps 0, K, 2K, ... and the final step
    std::vector<float*> ck_p;     // particle state [xh D][xl D][u D] x np, id order
    float *d_id = nullptr, *rp_id = nullptr;
    char* tape_f = nullptr;       // populations at the start of each step of one segment
    float* tape_F = nullptr;      // force field of each step of one segment
    float* tape_p = nullptr;      // particle state at the start of each step of one segment
    float* abar[2] = {nullptr, nullptr};
    float* Fbar = nullptr;
    float4* Mc = nullptr;
    float* Sf = nullptr;
    float *xbh[2] = {nullptr, nullptr}, *xbl[2] = {nullptr, nullptr}, *ub[2] = {nullptr, nullptr};
    float* coefS = nullptr;
    float *tpart = nullptr, *gpart = nullptr, *acc = nullptr;
};
}  // namespace pibm

using namespace pibm;

struct pibm_ctx {
    pibm_config cfg;
    int Q = 9, D = 2, fp16 = 0, sl2 = 0;
    long long N = 0;
    int np = 0;
    hipStream_t stream = nullptr;
    void* fA = nullptr;
    void* fB = nullptr;
    float4* mom = nullptr;
    float* F = nullptr;
    float* stage = nullptr;
    long long stage_floats = 0;
    double* part = nullptr;
    double* totals = nullptr;
    PBuf pb{};
    PCfg pc{};
    Grid grid{};
    Rollout ro{};
    bool particles_set = false;
    bool stepped = false;
    // the spreading records change with every step, particle hand-over and
    // particle adjoint stage; PIBM_STAGE_INTERP_T needs those of the last
    // PIBM_STAGE_INTERP
    uint64_t srec_epoch = 0, interp_stage_epoch = ~0ull;
    // the last step spread its force straight into the collision: the field
    // in F is recomputed from the spreading records when someone needs it
    bool F_stale = false;
    // particles handed over in device memory whose validity the device has
    // reported but the host has not read yet: the first step waits for it
    bool device_input_unchecked = false;
    std::string err;
    // phase timing: a ring of event rows, PIBM_NUM_PHASES + 1 events per step
    bool prof = false;
    int prof_every = 1;          // events on every n-th step
    int64_t prof_tick = 0;
    std::vector<hipEvent_t> ev;
    int ev_rows = 0, ev_used = 0;
    double phase_ms[PIBM_NUM_PHASES] = {0, 0, 0, 0, 0, 0};
    int64_t prof_steps = 0;
    // active-particle count of a recent step, copied to pinned host memory
    // every few steps; selects the single-workgroup island set-up
    uint32_t* host_active = nullptr;
    uint64_t steps_done = 0;
    // fixed obstacle bodies: the body of each particle id (-1: moving)
    std::vector<int> body_of;
    // device address of the module-scope reduction scratch on this
    // context's GPU (for pibm_conservation_noalloc), resolved at creation
    double* scratch = nullptr;
    ~pibm_ctx() {
        // nothing to report from a destructor: failures are dropped on purpose
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        if (host_active) (void)hipHostFree(host_active);
    }
};

namespace {

struct Carver {
    char* base;
    size_t off = 0;
    template <class T> T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

pibm_status fail(pibm_ctx* c, pibm_status st, const std::string& msg) {
    if (c) c->err = msg;
    return st;
}

pibm_status check_hip(pibm_ctx* c, hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(c, PIBM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return PIBM_OK;
}

// Return from the calling entry point with PIBM_E_HIP on the first failed
// HIP call.
#define HIP_TRY(c, call, what)                                            \
    do {                                                                  \
        if (pibm_status st_ = check_hip((c), (call), (what))) return st_; \
    } while (0)

// Keeps the first failure of a sequence of enqueued HIP calls.
struct HipSeq {
    hipError_t e = hipSuccess;
    void operator()(hipError_t r) {
        if (e == hipSuccess) e = r;
    }
};

// Reduction scratch of pibm_conservation_noalloc: the per-block FP64 partial
// sums of the mass/momentum reductions (8 per block) and their totals.
// Module-scope device memory, so that entry point allocates nothing; each
// GPU the library runs on holds its own copy until the process ends.  In
// host code the name is only a host-side stand-in: device code gets the
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t SCRATCH_DOUBLES = 8 * 1040 + 16;     // 66.7 KB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
double* scratch_addr[MAX_DEVICES] = {};          // per device, resolved once

// The device address of `scratch` on the current device (resolved once per
// device, with that device current).
hipError_t scratch_for_current_device(double** out) {
    int dev = -1;
    if (hipError_t e = hipGetDevice(&dev)) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_addr[dev]) {
        void* p = nullptr;
        if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) return e;
        scratch_addr[dev] = (double*)p;
    }
    *out = scratch_addr[dev];
    return hipSuccess;
}

int dimension(int lattice) { return lattice == PIBM_D2Q9 ? 2 : 3; }

// angular-velocity components: 3 in 3D, the z component in 2D
int spin_components(int D) { return D == 3 ? 3 : 1; }

std::string validate(const pibm_config* cfg, int64_t np) {
    if (!cfg) return "null config";
    if (cfg->abi_version != PIBM_ABI_VERSION) return "ABI version mismatch";
    if (cfg->lattice != PIBM_D2Q9 && cfg->lattice != PIBM_D3Q15 && cfg->lattice != PIBM_D3Q19)
        return "lattice must be D2Q9 (9), D3Q15 (15) or D3Q19 (19)";
    if (cfg->storage != PIBM_STORE_FP32 && cfg->storage != PIBM_STORE_FP16) return "unknown storage";
    if (cfg->fp16_scale_log2 < 0 || cfg->fp16_scale_log2 > 24) return "fp16_scale_log2 out of range";
    int D = dimension(cfg->lattice);
    for (int a = 0; a < 3; a++) {
        if (cfg->n[a] < 1) return "lattice extent < 1";
        if (a >= D && cfg->n[a] != 1) return "n[2] must be 1 for D2Q9";
    }
    long long N = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
    if (N > (1LL << 31) - 1) return "too many nodes";
    for (int a = 0; a < D; a++)
        if (cfg->n[a] > 30000) return "axis longer than 30000 nodes";
    if (!(cfg->tau > 0.5)) return "tau must exceed 1/2";
    if (cfg->n_sub < 1) return "n_sub must be >= 1";
    if (cfg->contact < 0 || cfg->contact > 5) return "unknown contact model";
    if ((cfg->contact == PIBM_CONTACT_HERTZ || cfg->contact >= PIBM_CONTACT_HERTZ_MINDLIN) &&
        (!(cfg->young > 0) || !(cfg->poisson >= 0) || !(cfg->poisson < 0.5)))
        return "Hertz contact needs young > 0 and 0 <= poisson < 1/2";
    if (cfg->contact >= PIBM_CONTACT_HERTZ_MINDLIN && !(cfg->friction >= 0)) return "friction must be >= 0";
    if (cfg->bodies != 0 && cfg->bodies != 1) return "bodies must be 0 or 1";
    if (cfg->bin_log2 < 0 || cfg->bin_log2 > 3) return "bin_log2 must be 0..3";
    if (cfg->max_candidates < 1 || cfg->max_candidates > 64) return "max_candidates must be 1..64";
    if (cfg->island_setup < 0 || cfg->island_setup > 2) return "island_setup must be 0, 1 or 2";
    if (cfg->interp != PIBM_INTERP_DELTA && cfg->interp != PIBM_INTERP_LAGRANGE) return "unknown interpolation";
    if (cfg->contact == PIBM_CONTACT_LSD && (!(cfg->kn > 0) || !(cfg->restitution > 0) || cfg->restitution > 1))
        return "linear spring-dashpot needs kn > 0 and 0 < restitution <= 1";
    if (!(cfg->skin >= 0)) return "skin must be >= 0";
    if (np < 0 || np > (1LL << 30)) return "particle count out of range";
    if (np > 0)
        for (int a = 0; a < D; a++)
            if (cfg->periodic[a]) return "particles need walls on every axis";
    return "";
}

// Lay out the workspace; with base == nullptr only the size is computed.
size_t carve(pibm_ctx& c, char* base) {
    Carver cv{base};
    const long long N = c.N;
    const size_t es = c.fp16 ? 2 : 4;
    c.fA = cv.take<char>((size_t)c.Q * N * es);
    c.fB = cv.take<char>((size_t)c.Q * N * es);
    c.mom = cv.take<float4>(N);
    c.F = cv.take<float>((size_t)c.D * N);
    long long np = c.np;
    const bool md = c.cfg.contact >= PIBM_CONTACT_HERTZ_MINDLIN;
    c.stage_floats = std::max<long long>((long long)(c.D + 1) * N, 5LL * c.D * np);
    c.stage = cv.take<float>(c.stage_floats);
    c.part = cv.take<double>(8 * (std::max(lattice_totals_blocks(), particles_totals_blocks()) + 2));
    c.totals = cv.take<double>(16);
    PBuf& b = c.pb;
    b.flags = cv.take<uint32_t>(4);
    b.counters = cv.take<uint32_t>(CNT_SIZE);
    if (np > 0) {
        PState* S[3] = {&b.A, &b.B, &b.Bn};
        for (int k = 0; k < 3; k++) {
            for (int a = 0; a < 3; a++) {
                S[k]->xh[a] = a < c.D ? cv.take<float>(np) : nullptr;
                S[k]->xl[a] = a < c.D ? cv.take<float>(np) : nullptr;
                S[k]->u[a] = a < c.D ? cv.take<float>(np) : nullptr;
                S[k]->w[a] = (md && a < spin_components(c.D)) ? cv.take<float>(np) : nullptr;
            }
            S[k]->d = k < 2 ? cv.take<float>(np) : nullptr;
            S[k]->rp = k < 2 ? cv.take<float>(np) : nullptr;
            S[k]->id = k < 2 ? cv.take<int>(np) : nullptr;
            S[k]->fixa = (k < 2 && c.cfg.bodies) ? cv.take<float>(np) : nullptr;
        }
        long long nb1 = c.pc.nbins + 1;
        b.cnt = cv.take<uint32_t>(nb1);
        b.start = cv.take<uint32_t>(nb1);
        b.keys = cv.take<uint32_t>(np);
        b.slot = cv.take<uint32_t>(np);
        b.tmpid = cv.take<int>(np);
        b.keys_sorted = cv.take<uint32_t>(np);
        b.pos4 = cv.take<float4>(np);
        b.scan_u32 = cv.take<uint32_t>(scan_blocks(nb1) + 1);
        b.actcc = cv.take<unsigned long long>(np);
        b.prefix = cv.take<unsigned long long>(np);
        b.bsum64 = cv.take<unsigned long long>(np / 256 + 2);
        b.drho_i = cv.take<float>(np);
        b.j_i = cv.take<float>((size_t)c.D * np);
        b.srec = cv.take<float>((size_t)(c.D == 3 ? SRec<3>::STRIDE : SRec<2>::STRIDE) * np);
        b.fc = cv.take<float>((size_t)c.D * np);
        b.wbase = cv.take<short4>(np);
        b.alist = cv.take<uint32_t>(np);
        b.aidx = cv.take<uint32_t>(np);
        b.ccount = cv.take<uint32_t>(np);
        b.parent = cv.take<uint32_t>(np);
        b.isize = cv.take<uint32_t>(np);
        b.irank = cv.take<uint32_t>(np);
        b.fill = cv.take<uint32_t>(np);
        b.loc = cv.take<uint32_t>(np);
        b.bigroot = cv.take<uint32_t>(np);
        b.bigoff = cv.take<uint32_t>(np);
        b.bigmember = cv.take<uint32_t>(np);
        b.cand_cap = np * (long long)c.cfg.max_candidates;
        b.cand = cv.take<uint32_t>(b.cand_cap);
        b.cdata = (CandData*)cv.take<char>(b.cand_cap * CAND_BYTES);
        b.lane_cap = 2 * np + (long long)(WAVE + 2) * WAVE;
        b.lanemember = cv.take<int>(b.lane_cap);
        b.gdx = cv.take<float>(19 * np);
        b.gu = cv.take<float>(6 * np);
        if (md) {
            const long long hmax = (long long)c.cfg.max_candidates + c.D;
            b.cmd = cv.take<float4>(b.cand_cap);
            b.cpid = cv.take<int>(b.cand_cap);
            b.hcnt = cv.take<uint32_t>(np);
            b.hkey = cv.take<int>(np * hmax);
            b.hT = cv.take<float>((long long)TSN * np * hmax);
            b.gmd = cv.take<float>((6 + 3 * TSN + 1) * np);
            b.cms = cv.take<float4>(2 * b.cand_cap);
        } else {
            b.cmd = nullptr;
            b.cpid = nullptr;
            b.hcnt = nullptr;
            b.hkey = nullptr;
            b.hT = nullptr;
            b.gmd = nullptr;
            b.cms = nullptr;
        }
    }
    return cv.off + 256;
}

void fill_pcfg(pibm_ctx& c) {
    PCfg& p = c.pc;
    p.D = c.D;
    for (int a = 0; a < 3; a++) p.n[a] = c.cfg.n[a];
    p.L = c.cfg.bin_log2;
    p.nbins = 1;
    for (int a = 0; a < 3; a++) {
        p.nb[a] = a < c.D ? (c.cfg.n[a] >> p.L) + 1 : 1;
        p.nbins *= p.nb[a];
    }
    p.skin = (float)c.cfg.skin;
    p.contact = c.cfg.contact;
    p.kn = (float)c.cfg.kn;
    double e = c.cfg.restitution > 0 ? c.cfg.restitution : 1.0;
    double l = std::log(e);
    p.zeta = (float)(-l / std::sqrt(M_PI * M_PI + l * l));
    p.ks = (float)c.cfg.k_soft;
    p.n_sub = c.cfg.n_sub;
    p.h = (float)(1.0 / c.cfg.n_sub);
    p.rho0 = (float)c.cfg.rho0;
    for (int a = 0; a < 3; a++) p.g[a] = (float)c.cfg.gravity[a];
    p.maxc = c.cfg.max_candidates;
    p.lagrange = c.cfg.interp == PIBM_INTERP_LAGRANGE;
    p.hk = (float)(4.0 / 3.0 * c.cfg.young / (2.0 * (1.0 - c.cfg.poisson * c.cfg.poisson)));
    // G* as printed: 1/G* = 2 (1 - nu^2) / G, G = E / (2 (1 + nu))
    const double G = c.cfg.young / (2.0 * (1.0 + c.cfg.poisson));
    p.kt8 = (float)(8.0 * G / (2.0 * (1.0 - c.cfg.poisson * c.cfg.poisson)));
    p.mu = (float)c.cfg.friction;
    p.microslip = c.cfg.contact == PIBM_CONTACT_HERTZ_MINDLIN_MICROSLIP;
    p.hmax = c.cfg.max_candidates + c.D;
    // trailing parts are at most half an ulp of the leading ones; the
    // screened distance is off by at most sqrt(D) ulp(max extent)
    int nmax = std::max(c.cfg.n[0], std::max(c.cfg.n[1], c.cfg.n[2]));
    p.eps = (float)(std::sqrt((double)c.D) * std::ldexp(1.0, (int)std::ceil(std::log2((double)nmax + 1.0)) - 23));
    p.H = 1;
}

// Neighbour-search half-width for the largest diameter present.
void set_stencil(pibm_ctx& c, double dmax) {
    const double edge = std::ldexp(1.0, c.cfg.bin_log2);
    c.pc.H = std::max(1, (int)std::ceil((dmax + c.cfg.skin + (double)c.pc.eps) / edge));
    c.pc.dmax = (float)dmax;
}

// Why the adjoint cannot run on this context ("" if it can).
std::string adjoint_unsupported(const pibm_ctx& c) {
    if (c.np < 1) return "the adjoint needs at least one particle";
    if (c.cfg.n_sub != 1) return "the adjoint supports n_sub = 1 only";
    if (c.cfg.contact == PIBM_CONTACT_LSD || c.cfg.contact == PIBM_CONTACT_HERTZ ||
        c.cfg.contact >= PIBM_CONTACT_HERTZ_MINDLIN)
        return "the adjoint supports no contact or soft contact only";
    if (c.cfg.bin_log2 != 0) return "the adjoint needs bin_log2 = 0";
    if (c.cfg.bodies) return "the adjoint supports no fixed bodies";
    if (c.cfg.interp != PIBM_INTERP_DELTA) return "the adjoint supports delta-kernel interpolation only";
    return "";
}

size_t carve_rollout(const pibm_ctx& c, int steps, int K, char* base, Rollout& R) {
    Carver cv{base};
    const size_t es = c.fp16 ? 2 : 4;
    const size_t fbytes = (size_t)c.Q * c.N * es;
    const long long np = c.np, N = c.N, D = c.D;
    const size_t pf = (size_t)3 * D * np;
    R.nck = (steps + K - 1) / K + 1;
    R.ck_f.assign(R.nck, nullptr);
    R.ck_p.assign(R.nck, nullptr);
    for (int i = 0; i < R.nck; i++) {
        R.ck_f[i] = cv.take<char>(fbytes);
        R.ck_p[i] = cv.take<float>(pf);
    }
    R.d_id = cv.take<float>(np);
    R.rp_id = cv.take<float>(np);
    const long long len = std::max(1, std::min(K, steps));
    R.tape_f = cv.take<char>(len * fbytes);
    R.tape_F = cv.take<float>(len * D * N);
    R.tape_p = cv.take<float>(len * pf);
    for (int k = 0; k < 2; k++) R.abar[k] = cv.take<float>((size_t)c.Q * N);
    R.Fbar = cv.take<float>(D * N);
    R.Mc = cv.take<float4>(N);
    R.Sf = cv.take<float>((D + 1) * N);
    for (int k = 0; k < 2; k++) {
        R.xbh[k] = cv.take<float>(D * np);
        R.xbl[k] = cv.take<float>(D * np);
        R.ub[k] = cv.take<float>(D * np);
    }
    R.coefS = cv.take<float>((D + 1) * np);
    R.tpart = cv.take<float>(adj_collide_blocks(N));
    R.gpart = cv.take<float>(3LL * adj_particle_blocks((int)np));
    R.acc = cv.take<float>(8);
    return cv.off + 256;
}

bool init_ctx(pibm_ctx& c, const pibm_config* cfg, int64_t np) {
    c.cfg = *cfg;
    c.Q = cfg->lattice;
    c.D = dimension(cfg->lattice);
    c.fp16 = cfg->storage == PIBM_STORE_FP16;
    c.sl2 = c.fp16 ? cfg->fp16_scale_log2 : 0;
    c.N = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
    c.np = (int)np;
    for (int a = 0; a < 3; a++) {
        c.grid.n[a] = cfg->n[a];
        c.grid.periodic[a] = cfg->periodic[a] ? 1 : 0;
    }
    c.grid.N = c.N;
    fill_pcfg(c);
    return true;
}

// Zero angular velocities and the tangential-force history (Hertz-Mindlin
// contexts only): the state of freshly set particles.
hipError_t clear_spin_history(pibm_ctx* c) {
    if (!c->pb.hcnt) return hipSuccess;
    HipSeq q;
    for (int a = 0; a < spin_components(c->D); a++) q(hipMemsetAsync(c->pb.A.w[a], 0, 4 * (size_t)c->np, c->stream));
    q(hipMemsetAsync(c->pb.hcnt, 0, 4 * (size_t)c->np, c->stream));
    return q.e;
}

// The force field of the last step in F, spread again from the records the
// step left (the same sums in the same order: bitwise the field the fused
// collision used).  Before anything that rewrites the records.
void ensure_force(pibm_ctx* c) {
    if (!c->F_stale) return;
    particles_spread(c->D, c->pb, c->np, c->pc, c->grid, c->F, c->stream);
    c->F_stale = false;
}

pibm_status sync_and_flags(pibm_ctx* c) {
    pibm_status st = check_hip(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (st) return st;
    uint32_t flags = 0;
    st = check_hip(c, hipMemcpy(&flags, c->pb.flags, 4, hipMemcpyDeviceToHost), "read flags");
    if (st) return st;
    if (flags) {
        uint32_t z = 0;
        st = check_hip(c, hipMemcpy(c->pb.flags, &z, 4, hipMemcpyHostToDevice), "clear flags");
        if (st) return st;
        if (flags & FLAG_ARG) {
            // the particle state handed over in device memory is invalid: no
            // step may run on it until valid particles are set
            c->particles_set = false;
            c->device_input_unchecked = false;
            return fail(c, PIBM_E_ARG, "a particle array passed in device memory was invalid (position outside the box, "
                                       "diameter <= 0 or above d_max, density <= 0, or not finite)");
        }
        if (flags & FLAG_UNSTABLE) return fail(c, PIBM_E_UNSTABLE, "unstable: a particle left the box or a drag sub-step had h c >= 2");
        if (flags & FLAG_CAPACITY) return fail(c, PIBM_E_CAPACITY, "a particle had more candidates than max_candidates");
        if (flags & FLAG_SKIN) return fail(c, PIBM_E_SKIN, "a particle moved more than skin/2 within one step");
    }
    return PIBM_OK;
}

// Before the first step on particles handed over in device memory, wait for
// the device's check of them: no kernel ever runs on an invalid state.
pibm_status check_device_input(pibm_ctx* c) {
    if (!c->device_input_unchecked) return PIBM_OK;
    pibm_status st = sync_and_flags(c);
    if (st == PIBM_OK) c->device_input_unchecked = false;
    return st;
}

constexpr int PROF_ROWS = 256;

// Sum the elapsed times of the recorded rows and empty the ring.
pibm_status drain_events(pibm_ctx* c) {
    if (c->ev_used == 0) return PIBM_OK;
    if (pibm_status s = check_hip(c, hipStreamSynchronize(c->stream), "sync")) return s;
    const int E = PIBM_NUM_PHASES + 1;
    for (int r = 0; r < c->ev_used; r++)
        for (int p = 0; p < PIBM_NUM_PHASES; p++) {
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[r * E + p], c->ev[r * E + p + 1]), "hipEventElapsedTime");
            c->phase_ms[p] += ms;
        }
    c->prof_steps += c->ev_used;
    c->ev_used = 0;
    return PIBM_OK;
}

inline hipError_t mark(pibm_ctx* c, int row, int p) {
    return row >= 0 ? hipEventRecord(c->ev[row * (PIBM_NUM_PHASES + 1) + p], c->stream) : hipSuccess;
}

}  // namespace

extern "C" {

size_t pibm_workspace_bytes(const pibm_config* cfg, int64_t n_particles) {
    if (!validate(cfg, n_particles).empty()) return 0;
    pibm_ctx c;
    init_ctx(c, cfg, n_particles);
    return carve(c, nullptr);
}

pibm_status pibm_create(const pibm_config* cfg, int64_t n_particles, void* dev_ws, size_t ws_bytes,
                        void* hip_stream, pibm_ctx** out) {
    if (!out) return PIBM_E_ARG;
    *out = nullptr;
    std::string v = validate(cfg, n_particles);
    if (!v.empty()) return PIBM_E_CONFIG;
    pibm_ctx* c = new pibm_ctx();
    init_ctx(*c, cfg, n_particles);
    size_t need = carve(*c, nullptr);
    if (!dev_ws || ws_bytes < need) {
        delete c;
        return PIBM_E_ARG;
    }
    char* base = (char*)(((uintptr_t)dev_ws + 255) & ~(uintptr_t)255);
    if ((size_t)(base - (char*)dev_ws) + need - 256 > ws_bytes) {
        delete c;
        return PIBM_E_ARG;
    }
    carve(*c, base);
    c->stream = (hipStream_t)hip_stream;
    if (hipHostMalloc((void**)&c->host_active, 64, hipHostMallocDefault) != hipSuccess) {
        c->host_active = nullptr;
        delete c;
        return PIBM_E_HIP;
    }
    *(volatile uint32_t*)c->host_active = 0xffffffffu;   // unknown: multi-kernel set-up
    if (scratch_for_current_device(&c->scratch) != hipSuccess) {
        delete c;
        return PIBM_E_HIP;
    }
    HipSeq q;
    q(hipMemsetAsync(c->F, 0, sizeof(float) * c->D * c->N, c->stream));
    if (c->np > 0) q(hipMemsetAsync(c->pb.cnt, 0, sizeof(uint32_t) * (c->pc.nbins + 1), c->stream));
    q(hipMemsetAsync(c->pb.flags, 0, 16, c->stream));
    lattice_init_eq(c->Q, c->fp16, c->sl2, c->fA, nullptr, nullptr, c->N, c->stream);
    q(hipGetLastError());
    q(hipStreamSynchronize(c->stream));
    if (q.e != hipSuccess) {
        delete c;
        return PIBM_E_HIP;
    }
    *out = c;
    return PIBM_OK;
}

void pibm_destroy(pibm_ctx* ctx) { delete ctx; }

const char* pibm_last_error(const pibm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

pibm_status pibm_set_stream(pibm_ctx* ctx, void* hip_stream) {
    if (!ctx) return PIBM_E_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return PIBM_OK;
}

pibm_status pibm_init_equilibrium(pibm_ctx* c, const float* rho, const float* u) {
    if (!c) return PIBM_E_ARG;
    float* drho = nullptr;
    float* du = nullptr;
    if (rho) {
        drho = c->stage;
        if (pibm_status s = check_hip(c, hipMemcpyAsync(drho, rho, sizeof(float) * c->N, hipMemcpyHostToDevice, c->stream), "copy rho")) return s;
    }
    if (u) {
        du = c->stage + c->N;
        if (pibm_status s = check_hip(c, hipMemcpyAsync(du, u, sizeof(float) * c->D * c->N, hipMemcpyHostToDevice, c->stream), "copy u")) return s;
    }
    lattice_init_eq(c->Q, c->fp16, c->sl2, c->fA, drho, du, c->N, c->stream);
    if (pibm_status s = check_hip(c, hipGetLastError(), "init_eq launch")) return s;
    return check_hip(c, hipStreamSynchronize(c->stream), "sync");
}

pibm_status pibm_write_populations(pibm_ctx* c, const float* h) {
    if (!c || !h) return fail(c, PIBM_E_ARG, "null argument");
    const size_t es = c->fp16 ? 2 : 4;
    for (int q = 0; q < c->Q; q++) {
        if (pibm_status s = check_hip(c, hipMemcpyAsync(c->stage, h + (size_t)q * c->N, sizeof(float) * c->N,
                                                         hipMemcpyHostToDevice, c->stream), "copy populations")) return s;
        lattice_encode(c->fp16, c->sl2, (char*)c->fA + (size_t)q * c->N * es, c->stage, c->N, c->stream);
    }
    if (pibm_status s = check_hip(c, hipGetLastError(), "encode launch")) return s;
    return check_hip(c, hipStreamSynchronize(c->stream), "sync");
}

pibm_status pibm_read_populations(pibm_ctx* c, float* h) {
    if (!c || !h) return fail(c, PIBM_E_ARG, "null argument");
    const size_t es = c->fp16 ? 2 : 4;
    for (int q = 0; q < c->Q; q++) {
        lattice_decode(c->fp16, c->sl2, (char*)c->fA + (size_t)q * c->N * es, c->stage, c->N, c->stream);
        if (pibm_status s = check_hip(c, hipMemcpyAsync(h + (size_t)q * c->N, c->stage, sizeof(float) * c->N,
                                                         hipMemcpyDeviceToHost, c->stream), "copy populations")) return s;
        if (pibm_status s = check_hip(c, hipStreamSynchronize(c->stream), "sync")) return s;
    }
    return check_hip(c, hipGetLastError(), "decode launch");
}

pibm_status pibm_set_particles(pibm_ctx* c, const double* x, const double* v, const double* d,
                               const double* rho_p) {
    if (!c) return PIBM_E_ARG;
    ensure_force(c);
    if (c->np == 0) {
        c->particles_set = true;
        c->srec_epoch++;
        return PIBM_OK;
    }
    if (!x || !d || !rho_p) return fail(c, PIBM_E_ARG, "null particle array");
    const int D = c->D, np = c->np;
    std::vector<float> buf((size_t)(3 * D + 3) * np);
    double dmax = 0;
    float* xh = buf.data();
    float* xl = xh + (size_t)D * np;
    float* u = xl + (size_t)D * np;
    float* dd = u + (size_t)D * np;
    float* rp = dd + np;
    int* id = (int*)(rp + np);
    for (int i = 0; i < np; i++) {
        if (!(d[i] > 0) || !(rho_p[i] > 0)) return fail(c, PIBM_E_ARG, "diameter and density must be positive");
        if (d[i] > 0.5 * c->cfg.n[0] || d[i] > 64.0) return fail(c, PIBM_E_ARG, "diameter too large");
        dmax = std::max(dmax, (double)(float)d[i]);
        dd[i] = (float)d[i];
        rp[i] = (float)rho_p[i];
        id[i] = i;
        for (int a = 0; a < D; a++) {
            double xa = x[(size_t)a * np + i];
            if (!(xa > 0.0 && xa < (double)c->cfg.n[a])) return fail(c, PIBM_E_ARG, "particle outside the box");
            float h = (float)xa;
            xh[(size_t)a * np + i] = h;
            xl[(size_t)a * np + i] = (float)(xa - (double)h);
            u[(size_t)a * np + i] = v ? (float)v[(size_t)a * np + i] : 0.0f;
        }
    }
    PState& A = c->pb.A;
    HipSeq q;
    for (int a = 0; a < D; a++) {
        q(hipMemcpyAsync(A.xh[a], xh + (size_t)a * np, 4 * np, hipMemcpyHostToDevice, c->stream));
        q(hipMemcpyAsync(A.xl[a], xl + (size_t)a * np, 4 * np, hipMemcpyHostToDevice, c->stream));
        q(hipMemcpyAsync(A.u[a], u + (size_t)a * np, 4 * np, hipMemcpyHostToDevice, c->stream));
    }
    q(hipMemcpyAsync(A.d, dd, 4 * np, hipMemcpyHostToDevice, c->stream));
    q(hipMemcpyAsync(A.rp, rp, 4 * np, hipMemcpyHostToDevice, c->stream));
    q(hipMemcpyAsync(A.id, id, 4 * np, hipMemcpyHostToDevice, c->stream));
    if (A.fixa) q(hipMemsetAsync(A.fixa, 0, 4 * (size_t)np, c->stream));   // every particle moves
    q(clear_spin_history(c));
    // the staging vector must outlive the copies: wait before returning
    q(hipStreamSynchronize(c->stream));
    HIP_TRY(c, q.e, "copy particles");
    c->body_of.assign(np, -1);
    set_stencil(*c, dmax);
    c->particles_set = true;
    c->srec_epoch++;
    c->stepped = false;
    c->device_input_unchecked = false;
    return PIBM_OK;
}

pibm_status pibm_set_particles_device(pibm_ctx* c, const float* x_hi, const float* x_lo, const float* v,
                                      const float* d, const float* rho_p, double d_max) {
    if (!c) return PIBM_E_ARG;
    ensure_force(c);
    if (c->np == 0) {
        c->particles_set = true;
        c->srec_epoch++;
        return PIBM_OK;
    }
    if (!x_hi || !d || !rho_p) return fail(c, PIBM_E_ARG, "null particle array");
    if (!(d_max > 0.0) || d_max > 64.0 || d_max > 0.5 * c->cfg.n[0])
        return fail(c, PIBM_E_ARG, "d_max must be positive and within the diameter limits");
    const float dmax = (float)d_max;
    particles_set_state(c->D, c->pb, c->np, c->grid, x_hi, x_lo, v, d, rho_p, dmax, c->stream);
    HIP_TRY(c, hipGetLastError(), "set particles launch");
    HIP_TRY(c, clear_spin_history(c), "clear rotation");
    c->body_of.assign(c->np, -1);
    set_stencil(*c, (double)dmax);
    c->particles_set = true;
    c->srec_epoch++;
    c->stepped = false;
    c->device_input_unchecked = true;
    return PIBM_OK;
}

pibm_status pibm_set_rotation(pibm_ctx* c, const double* w) {
    if (!c || !w) return PIBM_E_ARG;
    if (c->cfg.contact < PIBM_CONTACT_HERTZ_MINDLIN) return fail(c, PIBM_E_CONFIG, "no rotation without Hertz-Mindlin contact");
    if (c->np == 0) return PIBM_OK;
    if (!c->particles_set || c->stepped) return fail(c, PIBM_E_STATE, "set the rotation right after the particles");
    const int nw = spin_components(c->D), np = c->np;
    std::vector<float> buf((size_t)nw * np);
    for (size_t k = 0; k < buf.size(); k++) buf[k] = (float)w[k];
    // before the first step the state is in id order
    HipSeq q;
    for (int a = 0; a < nw; a++)
        q(hipMemcpyAsync(c->pb.A.w[a], buf.data() + (size_t)a * np, 4 * (size_t)np, hipMemcpyHostToDevice, c->stream));
    q(hipStreamSynchronize(c->stream));
    return check_hip(c, q.e, "copy rotation");
}

pibm_status pibm_set_bodies(pibm_ctx* c, const int32_t* body, const double* area) {
    if (!c || !body) return PIBM_E_ARG;
    if (!c->cfg.bodies) return fail(c, PIBM_E_CONFIG, "fixed bodies need cfg.bodies = 1");
    if (c->np == 0) return PIBM_OK;
    if (!c->particles_set || c->stepped) return fail(c, PIBM_E_STATE, "set the bodies right after the particles");
    const int D = c->D, np = c->np;
    // before the first step the state is in id order
    std::vector<float> d(np), fa(np, 0.0f), u((size_t)D * np);
    HipSeq q;
    q(hipMemcpyAsync(d.data(), c->pb.A.d, 4 * (size_t)np, hipMemcpyDeviceToHost, c->stream));
    for (int a = 0; a < D; a++)
        q(hipMemcpyAsync(u.data() + (size_t)a * np, c->pb.A.u[a], 4 * (size_t)np, hipMemcpyDeviceToHost, c->stream));
    q(hipStreamSynchronize(c->stream));
    HIP_TRY(c, q.e, "read particles");
    for (int i = 0; i < np; i++) {
        if (body[i] < -1) return fail(c, PIBM_E_ARG, "body index must be >= -1");
        if (body[i] < 0) continue;
        const double ar = (area && area[i] > 0) ? area[i] : 0.25 * M_PI * (double)d[i] * d[i];
        fa[i] = (float)ar;
        for (int a = 0; a < D; a++) u[(size_t)a * np + i] = 0.0f;      // fixed points are at rest
    }
    q(hipMemcpyAsync(c->pb.A.fixa, fa.data(), 4 * (size_t)np, hipMemcpyHostToDevice, c->stream));
    for (int a = 0; a < D; a++)
        q(hipMemcpyAsync(c->pb.A.u[a], u.data() + (size_t)a * np, 4 * (size_t)np, hipMemcpyHostToDevice, c->stream));
    q(hipStreamSynchronize(c->stream));
    HIP_TRY(c, q.e, "copy bodies");
    c->body_of.assign(body, body + np);
    return PIBM_OK;
}

pibm_status pibm_read_bodies(pibm_ctx* c, int32_t n_bodies, double* f_hydro, double* f_contact, double* torque) {
    if (!c || n_bodies < 0) return PIBM_E_ARG;
    if (!c->cfg.bodies) return fail(c, PIBM_E_CONFIG, "fixed bodies need cfg.bodies = 1");
    for (int32_t b = 0; b < 3 * n_bodies; b++) {
        if (f_hydro) f_hydro[b] = 0.0;
        if (f_contact) f_contact[b] = 0.0;
        if (torque) torque[b] = 0.0;
    }
    if (c->np == 0 || n_bodies == 0) return PIBM_OK;
    if (!c->particles_set) return fail(c, PIBM_E_STATE, "particles not set");
    const int D = c->D, np = c->np;
    particles_unpermute(D, c->pb, np, c->stepped, c->stage, c->stream);
    HIP_TRY(c, hipGetLastError(), "unpermute launch");
    std::vector<float> buf((size_t)5 * D * np);
    if (pibm_status s = check_hip(c, hipMemcpyAsync(buf.data(), c->stage, buf.size() * 4, hipMemcpyDeviceToHost, c->stream), "copy particles")) return s;
    if (pibm_status s = check_hip(c, hipStreamSynchronize(c->stream), "sync")) return s;
    // centroids, then forces and torques, summed in id order in FP64
    std::vector<double> cen((size_t)3 * n_bodies, 0.0), cnt(n_bodies, 0.0);
    auto pos = [&](int a, int i) { return (double)buf[(size_t)a * np + i] + (double)buf[(size_t)(D + a) * np + i]; };
    for (int i = 0; i < np; i++) {
        const int b = c->body_of[i];
        if (b < 0 || b >= n_bodies) continue;
        cnt[b] += 1.0;
        for (int a = 0; a < D; a++) cen[3 * b + a] += pos(a, i);
    }
    for (int b = 0; b < n_bodies; b++)
        for (int a = 0; a < 3; a++) cen[3 * b + a] = cnt[b] > 0 ? cen[3 * b + a] / cnt[b] : 0.0;
    for (int i = 0; i < np; i++) {
        const int b = c->body_of[i];
        if (b < 0 || b >= n_bodies) continue;
        double fh[3] = {0, 0, 0}, fcn[3] = {0, 0, 0}, r[3] = {0, 0, 0};
        for (int a = 0; a < D; a++) {
            fh[a] = buf[(size_t)(3 * D + a) * np + i];
            fcn[a] = buf[(size_t)(4 * D + a) * np + i];
            r[a] = pos(a, i) - cen[3 * b + a];
        }
        const double ft[3] = {fh[0] + fcn[0], fh[1] + fcn[1], fh[2] + fcn[2]};
        for (int a = 0; a < 3; a++) {
            if (f_hydro) f_hydro[3 * b + a] += fh[a];
            if (f_contact) f_contact[3 * b + a] += fcn[a];
        }
        if (torque) {
            torque[3 * b + 0] += D == 3 ? r[1] * ft[2] - r[2] * ft[1] : 0.0;
            torque[3 * b + 1] += D == 3 ? r[2] * ft[0] - r[0] * ft[2] : 0.0;
            torque[3 * b + 2] += r[0] * ft[1] - r[1] * ft[0];
        }
    }
    return PIBM_OK;
}

pibm_status pibm_read_rotation(pibm_ctx* c, double* w) {
    if (!c || !w) return PIBM_E_ARG;
    if (c->cfg.contact < PIBM_CONTACT_HERTZ_MINDLIN) return fail(c, PIBM_E_CONFIG, "no rotation without Hertz-Mindlin contact");
    if (c->np == 0) return PIBM_OK;
    if (!c->particles_set) return fail(c, PIBM_E_STATE, "particles not set");
    const int nw = spin_components(c->D), np = c->np;
    particles_unpermute_spin(c->D, c->pb, np, c->stage, c->stream);
    HIP_TRY(c, hipGetLastError(), "unpermute launch");
    std::vector<float> buf((size_t)nw * np);
    if (pibm_status s = check_hip(c, hipMemcpyAsync(buf.data(), c->stage, buf.size() * 4, hipMemcpyDeviceToHost, c->stream), "copy rotation")) return s;
    if (pibm_status s = check_hip(c, hipStreamSynchronize(c->stream), "sync")) return s;
    for (size_t k = 0; k < buf.size(); k++) w[k] = buf[k];
    return PIBM_OK;
}

pibm_status pibm_read_particles_device(pibm_ctx* c, float* x_hi, float* x_lo, float* v, float* f_hydro,
                                       float* f_contact) {
    if (!c) return PIBM_E_ARG;
    if (c->np == 0) return PIBM_OK;
    if (!c->particles_set) return fail(c, PIBM_E_STATE, "particles not set");
    const int D = c->D, np = c->np;
    particles_unpermute(D, c->pb, np, c->stepped, c->stage, c->stream);
    HIP_TRY(c, hipGetLastError(), "unpermute launch");
    // staging layout [x_hi D][x_lo D][v D][f_hydro D][f_contact D] x np
    float* out[5] = {x_hi, x_lo, v, f_hydro, f_contact};
    const size_t plane = sizeof(float) * (size_t)D * np;
    HipSeq q;
    for (int k = 0; k < 5; k++)
        if (out[k]) q(hipMemcpyAsync(out[k], c->stage + (size_t)k * D * np, plane, hipMemcpyDeviceToDevice, c->stream));
    return check_hip(c, q.e, "copy particles");
}

pibm_status pibm_read_particles(pibm_ctx* c, double* x, double* v, double* f_hydro, double* f_contact) {
    if (!c) return PIBM_E_ARG;
    if (c->np == 0) return PIBM_OK;
    if (!c->particles_set) return fail(c, PIBM_E_STATE, "particles not set");
    const int D = c->D, np = c->np;
    particles_unpermute(D, c->pb, np, c->stepped, c->stage, c->stream);
    HIP_TRY(c, hipGetLastError(), "unpermute launch");
    std::vector<float> buf((size_t)5 * D * np);
    if (pibm_status s = check_hip(c, hipMemcpyAsync(buf.data(), c->stage, buf.size() * 4, hipMemcpyDeviceToHost, c->stream), "copy particles")) return s;
    if (pibm_status s = check_hip(c, hipStreamSynchronize(c->stream), "sync")) return s;
    for (int a = 0; a < D; a++)
        for (int i = 0; i < np; i++) {
            size_t k = (size_t)a * np + i;
            if (x) x[k] = (double)buf[k] + (double)buf[(size_t)D * np + k];
            if (v) v[k] = buf[(size_t)2 * D * np + k];
            if (f_hydro) f_hydro[k] = buf[(size_t)3 * D * np + k];
            if (f_contact) f_contact[k] = buf[(size_t)4 * D * np + k];
        }
    return PIBM_OK;
}

// Density and velocity of the stored populations into device arrays (the
// caller's, or the staging area).
hipError_t fields_to(pibm_ctx* c, float* rho, float* u) {
    lattice_moments(c->Q, c->fp16, c->sl2, c->fA, c->mom, c->N, RowMask{}, c->stream);   // every node
    lattice_fields(c->mom, rho, u, c->N, c->D, c->stream);
    return hipGetLastError();
}

pibm_status pibm_read_fields(pibm_ctx* c, float* rho, float* u) {
    if (!c) return PIBM_E_ARG;
    HIP_TRY(c, fields_to(c, c->stage, c->stage + c->N), "fields launch");
    HipSeq q;
    if (rho) q(hipMemcpyAsync(rho, c->stage, sizeof(float) * c->N, hipMemcpyDeviceToHost, c->stream));
    if (u) q(hipMemcpyAsync(u, c->stage + c->N, sizeof(float) * c->D * c->N, hipMemcpyDeviceToHost, c->stream));
    q(hipStreamSynchronize(c->stream));
    return check_hip(c, q.e, "read fields");
}

pibm_status pibm_read_fields_device(pibm_ctx* c, float* rho, float* u) {
    if (!c || !rho || !u) return fail(c, PIBM_E_ARG, "null field array");
    return check_hip(c, fields_to(c, rho, u), "fields launch");
}

pibm_status pibm_read_force(pibm_ctx* c, float* F) {
    if (!c || !F) return PIBM_E_ARG;
    ensure_force(c);
    HipSeq q;
    q(hipMemcpyAsync(F, c->F, sizeof(float) * c->D * c->N, hipMemcpyDeviceToHost, c->stream));
    q(hipStreamSynchronize(c->stream));
    HIP_TRY(c, q.e, "copy F");
    for (int a = 0; a < c->D; a++) {
        float ff = (float)c->cfg.fluid_force[a];
        if (ff != 0.0f)
            for (long long r = 0; r < c->N; r++) F[(size_t)a * c->N + r] += ff;
    }
    return PIBM_OK;
}

pibm_status pibm_read_force_device(pibm_ctx* c, float* F) {
    if (!c || !F) return PIBM_E_ARG;
    ensure_force(c);
    const float ff[3] = {(float)c->cfg.fluid_force[0], (float)c->cfg.fluid_force[1], (float)c->cfg.fluid_force[2]};
    lattice_add_const(c->F, F, c->N, c->D, ff, c->stream);
    return check_hip(c, hipGetLastError(), "force launch");
}

int64_t pibm_num_bins(const pibm_ctx* c) { return c ? c->pc.nbins : 0; }

pibm_status pibm_read_cell_list(pibm_ctx* c, uint32_t* keys, int32_t* ids, int32_t* bin_start) {
    if (!c) return PIBM_E_ARG;
    if (c->np == 0) return PIBM_OK;
    if (!c->stepped) return fail(c, PIBM_E_STATE, "no step taken yet");
    HipSeq q;
    if (keys) q(hipMemcpyAsync(keys, c->pb.keys_sorted, 4 * (size_t)c->np, hipMemcpyDeviceToHost, c->stream));
    if (ids) q(hipMemcpyAsync(ids, c->pb.A.id, 4 * (size_t)c->np, hipMemcpyDeviceToHost, c->stream));
    if (bin_start) q(hipMemcpyAsync(bin_start, c->pb.start, 4 * (size_t)(c->pc.nbins + 1), hipMemcpyDeviceToHost, c->stream));
    q(hipStreamSynchronize(c->stream));
    return check_hip(c, q.e, "read cell list");
}

}  // extern "C"

namespace {
constexpr uint32_t ONE_GROUP_MAX = 1024;   // one pass per phase: faster than nine launches

// One coupled step from populations fin to fout, with the force field in F.
// Returns the first failure of the enqueued event records and copies (kernel
// launch errors are read by the caller with hipGetLastError).
// One coupled step from fin into fout.  want_F: the force field must be
// written to F (a rollout records it); otherwise 3D spreading with bins of
// one dual cell and FP32 storage is fused into the collision (with FP16
// storage the collision is short enough that the fused tile order costs
// more than the force field's traffic saves).
hipError_t launch_step(pibm_ctx* c, const void* fin, void* fout, float* F, int row, bool want_F) {
    HipSeq q;
    c->srec_epoch++;
    const float ff[3] = {(float)c->cfg.fluid_force[0], (float)c->cfg.fluid_force[1], (float)c->cfg.fluid_force[2]};
    const bool spread = c->np > 0 && c->cfg.two_way;
    const bool fuse_sc = spread && !want_F && c->D == 3 && c->pc.L == 0 && !c->fp16;
    // D2Q9 interpolation takes the moments straight from the populations of
    // the tiles that hold particles; 3D (15 or 19 planes, a larger halo) and
    // the coarse-bin path read them from a moments pass, which the cell list
    // restricts to the node rows that the particles' stencils reach
    const bool fused = c->D == 2 && c->pc.L <= 1;
    q(mark(c, row, 0));
    if (c->np > 0) particles_sort(c->D, c->pb, c->np, c->pc, c->stream);
    q(mark(c, row, 1));
    if (c->np > 0 && !fused) {
        RowMask m{c->pb.start, {c->pc.n[0], c->pc.n[1], c->pc.n[2]}, {c->pc.nb[0], c->pc.nb[1], c->pc.nb[2]},
                  c->pc.L};
        lattice_moments(c->Q, c->fp16, c->sl2, fin, c->mom, c->N, m, c->stream);
    }
    q(mark(c, row, 2));
    if (c->np > 0) {
        if (fused) particles_interp_from_populations(c->pb, c->np, c->grid, c->pc, fin, c->fp16, c->sl2, c->stream);
        else particles_interp(c->D, c->pb, c->np, c->grid, c->pc, c->mom, c->stream);
    }
    q(mark(c, row, 3));
    if (c->np > 0) {
        // island set-up in one workgroup while a recent step had at most
        // ONE_GROUP_MAX active particles (both paths give the same result)
        const uint32_t recent = *(volatile uint32_t*)c->host_active;
        const bool one = c->cfg.island_setup == 1 || (c->cfg.island_setup == 0 && recent <= ONE_GROUP_MAX);
        particles_dem(c->D, c->pb, c->np, c->pc, one, c->stream);
        if (c->steps_done % 8 == 0)
            q(hipMemcpyAsync(c->host_active, c->pb.counters + CNT_ACTIVE, 4, hipMemcpyDeviceToHost, c->stream));
    }
    c->steps_done++;
    q(mark(c, row, 4));
    if (spread && !fuse_sc) particles_spread(c->D, c->pb, c->np, c->pc, c->grid, F, c->stream);
    q(mark(c, row, 5));
    if (fuse_sc) {
        particles_spread_collide(c->Q, c->fp16, c->sl2, c->pb, c->np, c->pc, c->grid, fin, fout, ff,
                                 (float)c->cfg.tau, c->stream);
        if (F == c->F) c->F_stale = true;
    } else {
        lattice_collide(c->Q, c->fp16, c->sl2, fin, fout, F, spread ? 1 : 0, ff, c->grid, (float)c->cfg.tau,
                        c->stream);
        if (F == c->F) c->F_stale = false;
    }
    q(mark(c, row, 6));
    return q.e;
}

size_t pop_bytes(const pibm_ctx* c) { return (size_t)c->Q * c->N * (c->fp16 ? 2 : 4); }

hipError_t save_checkpoint(pibm_ctx* c, int i) {
    hipError_t e = hipMemcpyAsync(c->ro.ck_f[i], c->fA, pop_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    adj_save_state(c->D, c->pb, c->np, c->ro.ck_p[i], c->stream);
    return e;
}
}  // namespace

extern "C" {

pibm_status pibm_step(pibm_ctx* c, int32_t n_steps) {
    if (!c) return PIBM_E_ARG;
    if (n_steps < 0) return fail(c, PIBM_E_ARG, "negative step count");
    if (c->np > 0 && !c->particles_set) return fail(c, PIBM_E_STATE, "particles not set");
    if (n_steps > 0)
        if (pibm_status st = check_device_input(c)) return st;
    for (int it = 0; it < n_steps; it++) {
        int row = -1;
        if (c->prof && c->prof_tick++ % c->prof_every == 0) {
            if (c->ev_used == c->ev_rows)
                if (pibm_status s = drain_events(c)) return s;
            row = c->ev_used++;
        }
        const hipError_t e = launch_step(c, c->fA, c->fB, c->F, row, false);
        std::swap(c->fA, c->fB);
        c->stepped = true;
        HIP_TRY(c, e, "step: event record or copy");
    }
    return check_hip(c, hipGetLastError(), "step launch");
}

size_t pibm_rollout_bytes(const pibm_ctx* c, int32_t n_steps, int32_t K) {
    if (!c || n_steps < 0 || K < 1 || !adjoint_unsupported(*c).empty()) return 0;
    Rollout R;
    return carve_rollout(*c, n_steps, K, nullptr, R);
}

pibm_status pibm_forward_ckpt(pibm_ctx* c, int32_t n_steps, int32_t K, void* dev_buf, size_t buf_bytes) {
    if (!c) return PIBM_E_ARG;
    c->ro.valid = false;
    if (n_steps < 0 || K < 1) return fail(c, PIBM_E_ARG, "need n_steps >= 0 and K >= 1");
    std::string why = adjoint_unsupported(*c);
    if (!why.empty()) return fail(c, PIBM_E_CONFIG, why);
    if (!c->particles_set) return fail(c, PIBM_E_STATE, "particles not set");
    if (pibm_status st = check_device_input(c)) return st;
    Rollout plan;
    const size_t need = carve_rollout(*c, n_steps, K, nullptr, plan);
    if (!dev_buf || buf_bytes < need) return fail(c, PIBM_E_ARG, "rollout buffer too small");
    char* base = (char*)(((uintptr_t)dev_buf + 255) & ~(uintptr_t)255);
    if ((size_t)(base - (char*)dev_buf) + need - 256 > buf_bytes) return fail(c, PIBM_E_ARG, "rollout buffer too small");
    carve_rollout(*c, n_steps, K, base, c->ro);
    c->ro.steps = n_steps;
    c->ro.K = K;
    adj_save_const(c->pb, c->np, c->ro.d_id, c->ro.rp_id, c->stream);
    Rollout& R = c->ro;
    R.taped = -1;
    const int last = n_steps > 0 ? (n_steps - 1) / K : -1;    // the last segment
    const size_t fbytes = pop_bytes(c), pf = (size_t)3 * c->D * c->np;
    HipSeq q;
    for (int t = 0; t < n_steps; t++) {
        if (t % K == 0) q(save_checkpoint(c, t / K));
        if (t / K != last) {
            q(launch_step(c, c->fA, c->fB, c->F, -1, true));
        } else {
            // The last segment runs on the tape, as the backward pass would
            // re-run it (same steps, same buffers): the backward pass then
            // starts reversing at once.  One segment (K >= n_steps) tapes
            // the whole rollout and nothing is run twice.
            const int k = t - last * K, len = n_steps - last * K;
            if (k == 0) q(hipMemcpyAsync(R.tape_f, c->fA, fbytes, hipMemcpyDeviceToDevice, c->stream));
            adj_save_state(c->D, c->pb, c->np, R.tape_p + k * pf, c->stream);
            void* fout = (k + 1 < len) ? (void*)(R.tape_f + (k + 1) * fbytes) : c->fB;
            q(launch_step(c, R.tape_f + k * fbytes, fout, R.tape_F + (size_t)k * c->D * c->N, -1, true));
        }
        std::swap(c->fA, c->fB);
    }
    if (last >= 0) {
        R.taped = last;
        // the last force field went to the tape: F is spread again when read
        if (c->np > 0 && c->cfg.two_way) c->F_stale = true;
    }
    q(save_checkpoint(c, c->ro.nck - 1));
    if (n_steps > 0) c->stepped = true;
    HIP_TRY(c, q.e, "forward: copy");
    if (pibm_status s = check_hip(c, hipGetLastError(), "forward launch")) return s;
    c->ro.valid = true;
    return PIBM_OK;
}

pibm_status pibm_backward(pibm_ctx* c, const float* dJ_dx_T, const float* dJ_dv_T, float* dJ_dx0, float* dJ_dv0,
                          double* dJ_dtau, double* dJ_dgravity) {
    if (!c) return PIBM_E_ARG;
    ensure_force(c);
    Rollout& R = c->ro;
    if (!R.valid) return fail(c, PIBM_E_STATE, "no recorded rollout (call pibm_forward_ckpt first)");
    const int D = c->D, np = c->np, Q = c->Q;
    const long long N = c->N, DN = (long long)D * np;
    const size_t fbytes = pop_bytes(c), pf = (size_t)3 * D * np;
    hipStream_t s = c->stream;
    const float ff[3] = {(float)c->cfg.fluid_force[0], (float)c->cfg.fluid_force[1], (float)c->cfg.fluid_force[2]};
    const int spread = c->cfg.two_way ? 1 : 0;
    const float tau = (float)c->cfg.tau;
    int cur = 0;
    HipSeq q;
    adj_fill(R.abar[0], (long long)Q * N, 0.f, s);
    if (dJ_dx_T) q(hipMemcpyAsync(R.xbh[0], dJ_dx_T, 4 * DN, hipMemcpyDeviceToDevice, s));
    else adj_fill(R.xbh[0], DN, 0.f, s);
    adj_fill(R.xbl[0], DN, 0.f, s);
    if (dJ_dv_T) q(hipMemcpyAsync(R.ub[0], dJ_dv_T, 4 * DN, hipMemcpyDeviceToDevice, s));
    else adj_fill(R.ub[0], DN, 0.f, s);
    adj_fill(R.acc, 8, 0.f, s);
    const int nseg = (R.steps + R.K - 1) / R.K;
    for (int seg = nseg - 1; seg >= 0; seg--) {
        const int t0 = seg * R.K, len = std::min(R.K, R.steps - t0);
        // re-run the segment, recording the state at the start of every step
        // (the last one was taped by the forward pass)
        if (seg != R.taped) {
            q(hipMemcpyAsync(R.tape_f, R.ck_f[seg], fbytes, hipMemcpyDeviceToDevice, s));
            adj_load_state(D, c->pb, np, R.ck_p[seg], R.d_id, R.rp_id, s);
            for (int k = 0; k < len; k++) {
                adj_save_state(D, c->pb, np, R.tape_p + k * pf, s);
                void* fout = (k + 1 < len) ? (void*)(R.tape_f + (k + 1) * fbytes) : c->fB;
                q(launch_step(c, R.tape_f + k * fbytes, fout, R.tape_F + (size_t)k * D * N, -1, true));
            }
            R.taped = seg;
        }
        // reverse it
        for (int k = len - 1; k >= 0; k--) {
            adj_load_state(D, c->pb, np, R.tape_p + k * pf, R.d_id, R.rp_id, s);
            particles_sort(D, c->pb, np, c->pc, s);
            adj_collide(Q, c->fp16, c->sl2, R.abar[cur], R.tape_f + k * fbytes, R.tape_F + (size_t)k * D * N, spread,
                        ff, c->grid, tau, c->mom, R.Fbar, R.Mc, R.tpart, s);
            adj_particles(D, c->pb, np, c->grid, c->pc, spread, c->mom, R.Fbar, R.xbh[cur], R.xbl[cur], R.ub[cur],
                          R.xbh[1 - cur], R.xbl[1 - cur], R.ub[1 - cur], R.coefS, R.gpart, s);
            particles_spread_adjoint(D, c->pb, np, c->pc, c->grid, R.coefS, R.Sf, s);
            adj_assemble(Q, R.abar[cur], R.Mc, R.Sf, 1, c->grid, tau, R.abar[1 - cur], s);
            adj_accumulate(R.tpart, adj_collide_blocks(N), R.gpart, adj_particle_blocks(np), R.acc, s);
            cur ^= 1;
        }
    }
    if (dJ_dx0) adj_df_collapse(R.xbh[cur], R.xbl[cur], dJ_dx0, DN, s);
    if (dJ_dv0) q(hipMemcpyAsync(dJ_dv0, R.ub[cur], 4 * DN, hipMemcpyDeviceToDevice, s));
    float acc[8];
    q(hipMemcpyAsync(acc, R.acc, sizeof(acc), hipMemcpyDeviceToHost, s));
    // leave the context in the final state of the rollout
    q(hipMemcpyAsync(c->fA, R.ck_f[R.nck - 1], fbytes, hipMemcpyDeviceToDevice, s));
    adj_load_state(D, c->pb, np, R.ck_p[R.nck - 1], R.d_id, R.rp_id, s);
    if (q.e != hipSuccess) {
        (void)hipStreamSynchronize(s);          // acc is written by the copy above
        return check_hip(c, q.e, "backward: copy");
    }
    if (pibm_status st = check_hip(c, hipGetLastError(), "backward launch")) {
        (void)hipStreamSynchronize(s);
        return st;
    }
    if (pibm_status st = sync_and_flags(c)) return st;
    if (dJ_dtau) *dJ_dtau = (double)acc[0] + (double)acc[1];
    if (dJ_dgravity)
        for (int a = 0; a < 3; a++) dJ_dgravity[a] = a < D ? (double)acc[2 + 2 * a] + (double)acc[3 + 2 * a] : 0.0;
    return PIBM_OK;
}

pibm_status pibm_adjoint_stage(pibm_ctx* c, int32_t stage, const float* in0, const float* in1, const float* in2,
                               float* out0, float* out1, float* out2, double* scalars) {
    if (!c) return PIBM_E_ARG;
    ensure_force(c);
    Rollout& R = c->ro;
    if (!R.valid) return fail(c, PIBM_E_STATE, "adjoint stages need a recorded rollout (pibm_forward_ckpt)");
    const int D = c->D, np = c->np, Q = c->Q;
    const long long N = c->N, DN = (long long)D * np;
    hipStream_t s = c->stream;
    const float tau = (float)c->cfg.tau;
    const int spread = c->cfg.two_way ? 1 : 0;
    HipSeq q;
    int nsc = 0;
    float acc[8];
    switch (stage) {
    case PIBM_STAGE_COLLIDE_T: {
        if (!in0 || !out0 || !out1) return fail(c, PIBM_E_ARG, "collide stage: null array");
        const float ff[3] = {(float)c->cfg.fluid_force[0], (float)c->cfg.fluid_force[1],
                             (float)c->cfg.fluid_force[2]};
        adj_fill(R.acc, 8, 0.f, s);
        adj_collide(Q, c->fp16, c->sl2, in0, c->fA, c->F, np > 0 && spread, ff, c->grid, tau, c->mom, out1, R.Mc,
                    R.tpart, s);
        adj_assemble(Q, in0, R.Mc, nullptr, 0, c->grid, tau, out0, s);
        adj_accumulate(R.tpart, adj_collide_blocks(N), nullptr, 0, R.acc, s);
        nsc = 1;
        break;
    }
    case PIBM_STAGE_PARTICLES_T: {
        if (!in0 || !in1 || !in2 || !out0 || !out1 || !out2)
            return fail(c, PIBM_E_ARG, "particle stage: null array");
        if (np == 0) return fail(c, PIBM_E_STATE, "particle stage: no particles");
        particles_sort(D, c->pb, np, c->pc, s);
        lattice_moments(Q, c->fp16, c->sl2, c->fA, c->mom, N, RowMask{}, s);
        adj_fill(R.acc, 8, 0.f, s);
        adj_fill(R.xbl[0], DN, 0.f, s);
        adj_particles(D, c->pb, np, c->grid, c->pc, spread, c->mom, in0, in1, R.xbl[0], in2, R.xbh[1], R.xbl[1],
                      out1, R.coefS, R.gpart, s);
        particles_spread_adjoint(D, c->pb, np, c->pc, c->grid, R.coefS, out2, s);
        adj_df_collapse(R.xbh[1], R.xbl[1], out0, DN, s);
        adj_accumulate(nullptr, 0, R.gpart, adj_particle_blocks(np), R.acc, s);
        c->srec_epoch++;
        nsc = 3;
        break;
    }
    case PIBM_STAGE_INTERP: {
        if (!in0 || !out0) return fail(c, PIBM_E_ARG, "interpolation stage: null array");
        if (np == 0) return fail(c, PIBM_E_STATE, "interpolation stage: no particles");
        particles_sort(D, c->pb, np, c->pc, s);
        adj_pack_mom(in0, 1 + D, N, c->mom, s);
        particles_interp(D, c->pb, np, c->grid, c->pc, c->mom, s);
        q(hipMemcpyAsync(out0, c->pb.drho_i, 4 * (size_t)np, hipMemcpyDeviceToDevice, s));
        q(hipMemcpyAsync(out0 + np, c->pb.j_i, 4 * (size_t)DN, hipMemcpyDeviceToDevice, s));
        c->interp_stage_epoch = ++c->srec_epoch;
        break;
    }
    case PIBM_STAGE_INTERP_T: {
        if (!in0 || !out0) return fail(c, PIBM_E_ARG, "interpolation transpose: null array");
        if (c->interp_stage_epoch != c->srec_epoch)
            return fail(c, PIBM_E_STATE, "interpolation transpose: PIBM_STAGE_INTERP must come first");
        particles_spread_adjoint(D, c->pb, np, c->pc, c->grid, in0, out0, s);
        break;
    }
    default:
        return fail(c, PIBM_E_ARG, "unknown adjoint stage");
    }
    if (scalars && nsc > 0) q(hipMemcpyAsync(acc, R.acc, sizeof(acc), hipMemcpyDeviceToHost, s));
    if (q.e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        return check_hip(c, q.e, "adjoint stage: copy");
    }
    if (pibm_status st = check_hip(c, hipGetLastError(), "adjoint stage launch")) return st;
    if (scalars && nsc > 0) {
        if (pibm_status st = sync_and_flags(c)) return st;
        if (stage == PIBM_STAGE_COLLIDE_T) scalars[0] = (double)acc[0] + (double)acc[1];
        else
            for (int a = 0; a < 3; a++) scalars[a] = a < D ? (double)acc[2 + 2 * a] + (double)acc[3 + 2 * a] : 0.0;
    }
    return PIBM_OK;
}

pibm_status pibm_set_profiling(pibm_ctx* c, int enable) {
    if (!c) return PIBM_E_ARG;
    if (enable && c->ev.empty()) {
        c->ev.resize((size_t)PROF_ROWS * (PIBM_NUM_PHASES + 1));
        for (hipEvent_t& e : c->ev)
            if (pibm_status s = check_hip(c, hipEventCreate(&e), "hipEventCreate")) return s;
        c->ev_rows = PROF_ROWS;
    }
    if (enable <= 0 && c->prof)
        if (pibm_status s = drain_events(c)) return s;
    c->prof = enable > 0;
    c->prof_every = enable > 0 ? enable : 1;
    c->prof_tick = 0;
    return PIBM_OK;
}

pibm_status pibm_phase_times(pibm_ctx* c, double* ms, int64_t* steps) {
    if (!c) return PIBM_E_ARG;
    if (pibm_status s = drain_events(c)) return s;
    for (int p = 0; p < PIBM_NUM_PHASES; p++) {
        if (ms) ms[p] = c->phase_ms[p];
        c->phase_ms[p] = 0;
    }
    if (steps) *steps = c->prof_steps;
    c->prof_steps = 0;
    return PIBM_OK;
}

pibm_status pibm_synchronize(pibm_ctx* c) {
    if (!c) return PIBM_E_ARG;
    return sync_and_flags(c);
}

}  // extern "C"

namespace {
// Diagnostics with the reductions' partial sums in `part` (8 doubles per
// block) and their totals in `totals` (16 doubles).  Every slot read is
// written first by the same call, so neither needs clearing.
pibm_status diagnostics_with(pibm_ctx* c, double* part, double* totals, pibm_diag* out) {
    std::memset(out, 0, sizeof(*out));
    lattice_totals(c->Q, c->fp16, c->sl2, c->fA, c->N, part, totals, c->stream);
    double fl[8];
    double pt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t cnt[2] = {0, 0};
    HipSeq q;
    q(hipGetLastError());
    q(hipMemcpyAsync(fl, totals, sizeof(fl), hipMemcpyDeviceToHost, c->stream));
    if (c->np > 0 && c->particles_set) {
        particles_totals(c->D, c->pb, c->np, part, totals + 8, c->stream);
        q(hipGetLastError());
        q(hipMemcpyAsync(pt, totals + 8, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        q(hipMemcpyAsync(cnt, c->pb.counters, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    }
    // the host buffers above are written by the stream: wait before any return
    q(hipStreamSynchronize(c->stream));
    HIP_TRY(c, q.e, "totals");
    out->mass = (double)c->N + fl[0];
    for (int a = 0; a < 3; a++) {
        out->fluid_momentum[a] = fl[1 + a];
        out->momentum[a] = fl[1 + a] + pt[a];
    }
    out->max_speed = std::sqrt(fl[4]);
    out->nonfinite = (int64_t)fl[5];
    out->candidates = cnt[CNT_CAND];
    out->active = cnt[CNT_ACTIVE];
    if (c->np > 0) {
        out->min_height = pt[3];
        out->mean_height = pt[4] / c->np;
    }
    pibm_status st = sync_and_flags(c);
    if (st) return st;
    if (out->nonfinite > 0 || out->max_speed > 0.1)
        return fail(c, PIBM_E_UNSTABLE, "non-finite populations or |u| > 0.1");
    return PIBM_OK;
}

// Scratch doubles the reductions need: partial sums of the larger of the
// two block counts, then 16 totals.
size_t reduction_scratch_doubles() {
    return 8 * ((size_t)std::max(lattice_totals_blocks(), particles_totals_blocks()) + 2) + 16;
}
}  // namespace

extern "C" {

pibm_status pibm_diagnostics(pibm_ctx* c, pibm_diag* out) {
    if (!c || !out) return PIBM_E_ARG;
    return diagnostics_with(c, c->part, c->totals, out);
}

pibm_status pibm_conservation(pibm_ctx* c, double* mass, double* momentum) {
    pibm_diag dg;
    pibm_status st = pibm_diagnostics(c, &dg);
    if (mass) *mass = dg.mass;
    if (momentum)
        for (int a = 0; a < 3; a++) momentum[a] = dg.momentum[a];
    return st;
}

pibm_status pibm_conservation_noalloc(pibm_ctx* c, double* mass, double* momentum) {
    if (!c) return PIBM_E_ARG;
    if (!c->scratch) return fail(c, PIBM_E_STATE, "static reduction scratch not resolved for this context's GPU");
    const size_t need = reduction_scratch_doubles();
    if (need > SCRATCH_DOUBLES)
        return fail(c, PIBM_E_CONFIG, "the reductions need " + std::to_string(need) +
                                          " doubles of scratch, above the static maximum of " +
                                          std::to_string(SCRATCH_DOUBLES));
    pibm_diag dg;
    pibm_status st = diagnostics_with(c, c->scratch, c->scratch + (need - 16), &dg);
    if (mass) *mass = dg.mass;
    if (momentum)
        for (int a = 0; a < 3; a++) momentum[a] = dg.momentum[a];
    return st;
}

}  // extern "C"
