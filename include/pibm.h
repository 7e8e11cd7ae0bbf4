/*
 * pibm.h -- C ABI of the MI355X (gfx950) library for one coupled
 * lattice-Boltzmann / particulate immersed boundary (PIBM) / DEM time step,
 * after Zhang et al., "PIBM: Particulate immersed boundary method for
 * fluid-particle interaction problems" (arXiv:1407.6704).
 *
 * One step n -> n+1 (Sec. 2 of the paper, in this order):
 *   1. density and momentum of the stored populations (Sec. 2.1);
 *   2. cell list of the particles (bins of 2^bin_log2 dual cells);
 *   3. interpolation of density and momentum to every particle with the
 *      delta-kernel weights of Eqs. lbm11-lbm12, or with the Lagrange
 *      polynomials of Eqs. lbm5-lbm6 on the same four nodes per axis;
 *   4. momentum-exchange force g = 2 (rho_i U - j_i) (Eqs. lbm7-lbm8), its
 *      reaction -A_p g on the particle (Eq. lbm13), contacts and buoyant
 *      weight (Eq. demgov), integrated over n_sub sub-steps;
 *   5. spreading of A_p * mean(g) back to the lattice (Eq. lbm10);
 *   6. BGK collision with the forcing term (Eqs. lbm2, lbm3, lbm9) and
 *      streaming with halfway bounce-back at the walls.
 *
 * Units are lattice units (node spacing 1, time step 1).  Node (x, y, z)
 * sits at (x + 1/2, y + 1/2, z + 1/2); a non-periodic axis a has walls at 0
 * and n[a].  Fields are laid out [component][z][y][x] with x fastest
 * (nz = 1 for D2Q9).  Particle arrays are [axis][N] in the caller's id order,
 * which every call preserves.
 *
 * Memory ownership: the caller owns all device memory.  pibm_create carves
 * its buffers from one device workspace of pibm_workspace_bytes() bytes that
 * the caller allocates (for instance as a torch uint8 tensor) and keeps alive
 * until pibm_destroy.  The library never allocates or frees device memory;
 * the context itself owns only host bookkeeping.  All GPU work goes to the
 * HIP stream given at creation (or by pibm_set_stream), asynchronously.
 *
 * I/O calls come in two forms.  pibm_set_*, pibm_read_* and pibm_write_*
 * take HOST arrays, copy through the workspace and synchronise the stream
 * before returning (convenient for tests and small cases).  The *_device
 * forms take caller-owned DEVICE arrays (for instance torch tensors on the
 * context's GPU), only enqueue work on the context's stream and never wait
 * for it, so state moves between the caller's tensors and the library with
 * no host round trip; the caller orders its own use of those arrays after
 * the stream (as with any asynchronous HIP call).  pibm_step only enqueues
 * work.  Numerical trouble found on the device (skin violation, NaN, a full
 * candidate list, an unstable drag sub-step, an invalid particle array handed
 * over in device memory) is latched in a device flag and reported by the
 * next synchronising call.
 *
 * Error behaviour: every call returns a pibm_status; nothing throws across
 * the ABI.  pibm_last_error() gives a message for the last failure on that
 * context.  A context must be used by one host thread at a time.
 */
#ifndef PIBM_H
#define PIBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIBM_ABI_VERSION 6

typedef enum {
    PIBM_OK = 0,
    PIBM_E_ARG = 1,       /* bad pointer, size, particle outside the box, ... */
    PIBM_E_CONFIG = 2,    /* tau <= 1/2, n_sub < 1, unknown lattice, ABI mismatch */
    PIBM_E_HIP = 3,       /* a HIP runtime call failed */
    PIBM_E_STATE = 4,     /* call order (e.g. step before particles are set) */
    PIBM_E_UNSTABLE = 5,  /* NaN/Inf, |u| > 0.1, or a drag sub-step with h c >= 2 */
    PIBM_E_SKIN = 6,      /* a particle moved more than skin/2 within one step */
    PIBM_E_CAPACITY = 7   /* more candidates per particle than max_candidates */
} pibm_status;

enum { PIBM_D2Q9 = 9, PIBM_D3Q15 = 15, PIBM_D3Q19 = 19 };
enum { PIBM_STORE_FP32 = 0, PIBM_STORE_FP16 = 1 };
enum {
    PIBM_CONTACT_NONE = 0,
    PIBM_CONTACT_LSD = 1,
    PIBM_CONTACT_SOFT = 2,
    PIBM_CONTACT_HERTZ = 3,
    PIBM_CONTACT_HERTZ_MINDLIN = 4,
    PIBM_CONTACT_HERTZ_MINDLIN_MICROSLIP = 5
};
enum { PIBM_INTERP_DELTA = 0, PIBM_INTERP_LAGRANGE = 1 };

/* Lattice velocity order used by pibm_read_populations/pibm_write_populations:
 *   D2Q9 : 0 (0,0); 1 (1,0); 2 (-1,0); 3 (0,1); 4 (0,-1);
 *          5 (1,1); 6 (-1,-1); 7 (1,-1); 8 (-1,1)
 *   D3Q19: 0 rest; 1..6 (+-x, +-y, +-z) as (1,0,0),(-1,0,0),(0,1,0),(0,-1,0),
 *          (0,0,1),(0,0,-1); 7..18 edges (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),
 *          (1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),(0,1,1),(0,-1,-1),(0,1,-1),
 *          (0,-1,1).
 *   D3Q15 (Sec. 2.1): 0 rest; 1..6 faces in the D3Q19 order; 7..14 corners
 *          (1,1,1),(-1,-1,-1),(1,1,-1),(-1,-1,1),(1,-1,1),(-1,1,-1),(-1,1,1),
 *          (1,-1,-1).
 * Weights: D2Q9 4/9, 1/9, 1/36; D3Q15 2/9, 1/9, 1/72; D3Q19 1/3, 1/18, 1/36
 * (c_s^2 = 1/3). */

typedef struct {
    int32_t abi_version;      /* PIBM_ABI_VERSION */
    int32_t lattice;          /* PIBM_D2Q9, PIBM_D3Q15 or PIBM_D3Q19 */
    int32_t storage;          /* PIBM_STORE_FP32: f - w in FP32;
                                 PIBM_STORE_FP16: (f - w) * 2^fp16_scale_log2 in FP16 */
    int32_t fp16_scale_log2;  /* 0 .. 24 */
    int32_t n[3];             /* nodes per axis; n[2] = 1 for D2Q9 */
    int32_t periodic[3];      /* 1: periodic axis (lattice only; then no particles) */
    double tau;               /* BGK relaxation time, > 1/2 (Eq. lbm2) */
    double rho0;              /* fluid density in the buoyancy term (Eq. demgov) */
    double gravity[3];        /* acceleration on particles */
    double fluid_force[3];    /* uniform body force density on the fluid */
    int32_t contact;          /* PIBM_CONTACT_*: none, linear spring-dashpot, soft repulsion,
                                 Hertz, or Hertz with the Mindlin tangential force and particle
                                 rotation (Sec. 2.3; young, poisson, friction below), in its
                                 no-slip limit (HERTZ_MINDLIN) or with the Mindlin-Deresiewicz
                                 micro-slip factors (HERTZ_MINDLIN_MICROSLIP): the increment
                                 dT = 8 G* r_a theta_k d(delta_t) + (-1)^k mu dF_n (1 - theta_k)
                                 along the contact's loading direction, with theta_k of loading
                                 (k = 0), unloading (1) and reloading (2) from the turning points
                                 T*, T** (Thornton's incremental form), elastic while the normal
                                 force grows faster than the tangential load */
    int32_t n_sub;            /* DEM sub-steps per lattice step, >= 1 */
    double kn;                /* linear spring stiffness */
    double restitution;       /* normal restitution of the linear spring-dashpot, (0, 1] */
    double k_soft;            /* soft repulsion k_s (1 - r/r_c)^2 */
    double skin;              /* candidate-list skin: particles may move <= skin/2 per step */
    int32_t two_way;          /* 1: spread the particle forces onto the fluid */
    int32_t bin_log2;         /* cell-list bin edge 2^bin_log2 node spacings, 0 .. 3 (0: fastest spreading) */
    int32_t max_candidates;   /* per-particle candidate capacity, 1 .. 64 */
    int32_t island_setup;     /* set-up of the active islands: 0 automatic, 1 one workgroup,
                                 2 one launch per phase (identical results; 0 picks 1 while a
                                 recent step had at most 1024 active particles) */
    int32_t interp;           /* PIBM_INTERP_DELTA: gather with the delta-kernel weights;
                                 PIBM_INTERP_LAGRANGE: gather with the Lagrange polynomials
                                 through the in-domain nodes of the same four per axis (cubic
                                 in the interior, Eqs. lbm5-lbm6).  Spreading always uses
                                 the delta kernel (Eq. lbm10) */
    double young;             /* PIBM_CONTACT_HERTZ: Young's modulus E of the particles and the
                                 walls (one material), lattice units; > 0 */
    double poisson;           /* PIBM_CONTACT_HERTZ: Poisson ratio nu, 0 <= nu < 1/2.  The normal
                                 force is (4/3) E* sqrt(R*) delta^(3/2) with E* = E / (2 (1 - nu^2)),
                                 1/R* = 1/R_p + 1/R_q (R* = R_p at a wall), undamped (Sec. 2.3) */
    double friction;          /* PIBM_CONTACT_HERTZ_MINDLIN: Coulomb coefficient mu >= 0.  The
                                 tangential force T on a particle grows by -8 G* r_a h v_t per
                                 sub-step (v_t: tangential contact-point velocity relative to the
                                 partner, r_a = sqrt(delta R*), 1/G* = 2 (1 - nu^2)/G as printed in
                                 the paper, G = E / (2 (1 + nu))), is turned into the current
                                 contact plane, capped at mu F_n, and carried between steps per
                                 pair of particle ids; spheres (disks) spin with I = 2/5 m R^2
                                 (1/2 m R^2) under the torque (-R n) x T.  No hydrodynamic torque */
    int32_t bodies;           /* 1: particles may be made points of fixed obstacle bodies
                                 (pibm_set_bodies); 0: all particles move */
} pibm_config;

typedef struct {
    double mass;              /* sum over nodes and directions of f */
    double momentum[3];       /* fluid sum f e plus particle sum m U */
    double fluid_momentum[3];
    double max_speed;         /* max over nodes of |u| */
    int64_t nonfinite;        /* nodes with a NaN/Inf population */
    int64_t active;           /* particles with a candidate neighbour or wall, last step */
    int64_t candidates;       /* directed candidate entries, last step */
    double min_height;        /* min over particles of the last coordinate */
    double mean_height;       /* mean over particles of the last coordinate */
} pibm_diag;

typedef struct pibm_ctx pibm_ctx;

/* Bytes of device workspace for this configuration and particle count. */
size_t pibm_workspace_bytes(const pibm_config* cfg, int64_t n_particles);

/* Validate cfg, carve the workspace (device pointer dev_ws, ws_bytes bytes),
 * bind the HIP stream (hipStream_t, may be NULL for the default stream) and
 * set the fluid to rest (f = w).  On success *out owns host bookkeeping only. */
pibm_status pibm_create(const pibm_config* cfg, int64_t n_particles, void* dev_ws,
                        size_t ws_bytes, void* hip_stream, pibm_ctx** out);
void pibm_destroy(pibm_ctx* ctx);
const char* pibm_last_error(const pibm_ctx* ctx);
pibm_status pibm_set_stream(pibm_ctx* ctx, void* hip_stream);

/* Fluid at equilibrium (Eq. lbm3) with density rho and velocity u (host
 * arrays of N and D x N floats); NULL means rho = 1, u = 0. */
pibm_status pibm_init_equilibrium(pibm_ctx* ctx, const float* rho, const float* u);

/* Populations as deviations from the rest state, h_q = f_q - w_q, Q x N FP32
 * host arrays in the direction order above.  Writing rounds to the storage
 * format; reading is exact for both storage formats. */
pibm_status pibm_write_populations(pibm_ctx* ctx, const float* h);
pibm_status pibm_read_populations(pibm_ctx* ctx, float* h);

/* Particles: positions x (D x N, strictly inside the box), velocities v
 * (D x N), diameters d and densities rho_p (N), host FP64 arrays.
 * Positions are kept as an unevaluated sum of two FP32 numbers (about 48
 * significant bits), velocities, diameters and densities in FP32. */
pibm_status pibm_set_particles(pibm_ctx* ctx, const double* x, const double* v,
                               const double* d, const double* rho_p);
/* Any output may be NULL.  f_hydro = -A_p mean(g) (Eq. lbm13) and
 * f_contact = sub-step mean of the contact force, both of the last step. */
pibm_status pibm_read_particles(pibm_ctx* ctx, double* x, double* v, double* f_hydro,
                                double* f_contact);

/* The same particle state (Sec. 2.2-2.3: position X, velocity U, diameter d,
 * density rho_p of each Lagrangian point) in caller-owned DEVICE FP32 arrays,
 * id order, [axis][N] for vectors.  A position is x_hi + x_lo (x_lo may be
 * NULL: zero); the pair is renormalised, so the split does not matter.  v may
 * be NULL (at rest).  d_max (host) must be >= every diameter: it sizes the
 * neighbour search (a larger value is correct but slower).  Asynchronous on
 * the context's stream: the arrays must stay valid until the stream has run
 * the copy.  Host-side checks (null arrays, d_max) return PIBM_E_ARG at once;
 * a position outside the open box, a diameter <= 0 or > d_max, a density
 * <= 0 or a non-finite value is found on the device and returned as
 * PIBM_E_ARG by the next synchronising call.  Resets rotation and tangential
 * history like pibm_set_particles. */
pibm_status pibm_set_particles_device(pibm_ctx* ctx, const float* x_hi, const float* x_lo, const float* v,
                                      const float* d, const float* rho_p, double d_max);
/* The particle state after the last step into caller-owned DEVICE FP32
 * arrays (D x N, id order; any may be NULL): position as x_hi + x_lo (the
 * exact double-float state), velocity, f_hydro = -A_p mean(g) (Eq. lbm13) and
 * the sub-step mean contact force.  Asynchronous on the context's stream. */
pibm_status pibm_read_particles_device(pibm_ctx* ctx, float* x_hi, float* x_lo, float* v,
                                       float* f_hydro, float* f_contact);
/* Angular velocities for PIBM_CONTACT_HERTZ_MINDLIN(_MICROSLIP) (the second line of
 * Eq. demgov), host FP64 arrays in id order: 3 x N (x, y, z) in 3D, N (the
 * z component) in 2D.  pibm_set_particles sets them to zero and clears the
 * tangential-force history; pibm_set_rotation may follow it before the first
 * step (PIBM_E_STATE afterwards).  Other contact models: PIBM_E_CONFIG. */
pibm_status pibm_set_rotation(pibm_ctx* ctx, const double* w);
pibm_status pibm_read_rotation(pibm_ctx* ctx, double* w);

/* Fixed obstacle bodies (the hybrid IBM-PIBM case of Sec. 3.3; needs
 * cfg.bodies = 1).  body (N int32, host): -1 for a moving particle, else
 * the index (0 .. n_bodies-1) of the fixed body the point belongs to.  area
 * (N doubles, host, may be NULL): the area a fixed point spreads with, e.g.
 * a conventional-IBM surface element (sphere area / point count); NULL or a
 * value <= 0 means pi d^2 / 4.  Fixed points keep their position, have zero
 * velocity and spin, exchange momentum with the fluid with U = 0
 * (Eqs. lbm7-lbm8, g = -2 j_i), and act on moving particles as contact
 * partners of infinite mass at rest; they feel neither walls nor each
 * other.  Call after pibm_set_particles and before the first step
 * (PIBM_E_STATE otherwise); pibm_set_particles makes every particle move
 * again. */
pibm_status pibm_set_bodies(pibm_ctx* ctx, const int32_t* body, const double* area);
/* Per body, from the last step (host FP64 arrays of 3 x n_bodies, any may be
 * NULL; z is zero in 2D): f_hydro = sum over the body's points of
 * -A_l mean(g_l) (Eq. lbm13), f_contact = sum of the contact reactions from
 * moving particles, torque of both about the centroid of the body's points
 * (in 2D only its z component is set).  Sums in id order, deterministic. */
pibm_status pibm_read_bodies(pibm_ctx* ctx, int32_t n_bodies, double* f_hydro, double* f_contact,
                             double* torque);

/* Density (N) and velocity u = j / rho (D x N) of the stored populations
 * (the moments after Eq. lbm3: rho = sum f, rho u = sum e f). */
pibm_status pibm_read_fields(pibm_ctx* ctx, float* rho, float* u);
/* Force field F (D x N) used by the last collision (spread + fluid_force). */
pibm_status pibm_read_force(pibm_ctx* ctx, float* F);
/* The same two outputs into caller-owned DEVICE FP32 arrays of the same
 * layout, asynchronously on the context's stream.  Both arrays of
 * pibm_read_fields_device are required; the force is the field F of Eq. lbm9
 * (spreading of Eq. lbm10 plus the uniform fluid force). */
pibm_status pibm_read_fields_device(pibm_ctx* ctx, float* rho, float* u);
pibm_status pibm_read_force_device(pibm_ctx* ctx, float* F);
/* Cell list built at the start of the last step: per sorted slot the bin key
 * and particle id (N each), and bin_start (n_bins + 1 entries); bins are
 * x-fastest over ((n_a >> bin_log2) + 1) per axis, a particle's bin being
 * (floor(X_a - 1/2) + 1) >> bin_log2.  Order: (key, id). */
int64_t pibm_num_bins(const pibm_ctx* ctx);
pibm_status pibm_read_cell_list(pibm_ctx* ctx, uint32_t* keys, int32_t* ids,
                                int32_t* bin_start);

/* Enqueue n_steps coupled steps on the context's stream (no host sync). */
pibm_status pibm_step(pibm_ctx* ctx, int32_t n_steps);

/* Phase timing.  pibm_set_profiling(ctx, n) with n >= 1 makes pibm_step
 * record HIP events on the context's stream between the phases of every
 * n-th step (the first step after the call included); n <= 0 turns it off.
 * pibm_phase_times synchronises and returns the milliseconds spent in each
 * phase, summed over the recorded steps, and their number, since profiling
 * was enabled or last read, then resets the sums.  Phases: 0 cell list,
 * 1 moments, 2 interpolation, 3 DEM, 4 spreading, 5 collision and
 * streaming.  A recorded step carries 7 event records, which cost a few
 * microseconds each on the stream. */
#define PIBM_NUM_PHASES 6
pibm_status pibm_set_profiling(pibm_ctx* ctx, int enable);
pibm_status pibm_phase_times(pibm_ctx* ctx, double* ms, int64_t* steps);

/* Wait for the stream; return the first latched device error, if any. */
pibm_status pibm_synchronize(pibm_ctx* ctx);

/* FP64 totals (synchronising): fluid mass and total momentum
 * (fluid sum f e + particle sum m U). */
pibm_status pibm_conservation(pibm_ctx* ctx, double* mass, double* momentum);
pibm_status pibm_diagnostics(pibm_ctx* ctx, pibm_diag* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as pibm_conservation, bit for bit (same kernels, same order), with
 * the reductions' partial sums in a module-scope device array of the library
 * (66.7 KB per GPU, held until the process ends) instead of the context's
 * workspace.  It allocates nothing and calls no allocating routine.  Nothing
 * in the array needs clearing (every slot read is first written by the same
 * call).  Every call on one GPU shares that array: calls that overlap on one
 * GPU (several streams or host threads at once) race and may return each
 * other's sums.  A reduction needing more scratch than the array holds is
 * rejected with PIBM_E_CONFIG.  Synchronising, like pibm_conservation. */
pibm_status pibm_conservation_noalloc(pibm_ctx* ctx, double* mass, double* momentum);

/* ---- Adjoint of a rollout (reverse-mode gradients) ----------------------
 * Gradients of a scalar objective J(X_T, U_T) of the particle state after
 * n_steps coupled steps with respect to the relaxation time tau (Eq. lbm2),
 * the gravity vector of the buoyant weight (Eq. demgov) and the initial
 * particle velocities and positions.  The backward pass is the exact reverse
 * of every operation of the step (collision and streaming, spreading,
 * momentum exchange, particle update, interpolation, moments), in FP32 with
 * double-float sums of the parameter gradients.
 * Supported: any lattice, no fixed bodies, delta-kernel interpolation, n_sub = 1 (the
 * explicit update of Eq. demgov), contact NONE or SOFT, bin_log2 = 0, FP32
 * or FP16 storage; other configurations return
 * PIBM_E_CONFIG.  Memory stays bounded by checkpointing: the state is saved
 * every K steps and each K-step segment is re-run before it is reversed,
 * except the last, which the forward pass records as it runs it (with
 * K >= n_steps the whole rollout is recorded once and nothing runs twice).
 *
 * Bytes of the caller-owned device buffer for a rollout of n_steps steps with
 * checkpoints every K steps (checkpoints, one segment's recorded states and
 * the adjoint fields); 0 for invalid arguments or an unsupported context. */
size_t pibm_rollout_bytes(const pibm_ctx* ctx, int32_t n_steps, int32_t K);
/* Run n_steps steps from the current state (as pibm_step) and record the
 * checkpoints in dev_buf (device memory of at least pibm_rollout_bytes bytes,
 * owned by the caller and kept alive until pibm_backward).  Asynchronous. */
pibm_status pibm_forward_ckpt(pibm_ctx* ctx, int32_t n_steps, int32_t K, void* dev_buf,
                              size_t buf_bytes);
/* Reverse the last recorded rollout.  Inputs dJ_dx_T, dJ_dv_T: DEVICE FP32
 * arrays D x N (id order), dJ/dX and dJ/dU at the final state; NULL means 0.
 * Outputs (each may be NULL): dJ_dx0, dJ_dv0 DEVICE FP32 D x N; dJ_dtau one
 * HOST double; dJ_dgravity three HOST doubles (components beyond D are 0).
 * Synchronises.  The context is left in the final state of the rollout, as
 * after pibm_forward_ckpt; the recorded rollout stays valid until the next
 * pibm_forward_ckpt, so several objectives may be reversed. */
pibm_status pibm_backward(pibm_ctx* ctx, const float* dJ_dx_T, const float* dJ_dv_T, float* dJ_dx0,
                          float* dJ_dv0, double* dJ_dtau, double* dJ_dgravity);

/* ---- Stages of the reverse step, one at a time --------------------------
 * For checking each part of the adjoint on its own (a vector-Jacobian
 * product against an independent derivative of the same stage, or a
 * transpose against the forward operator it transposes), and for callers
 * composing objectives of their own.  Each call applies one stage at the
 * context's current state and leaves that state unchanged (the particles may
 * be re-sorted, which no output depends on).  Needs a recorded rollout
 * (pibm_forward_ckpt), whose buffer provides the scratch; the recording stays
 * valid.  Arrays are DEVICE FP32; n = nodes, np = particles.  Asynchronous,
 * except that `scalars` (HOST doubles, may be NULL) makes the call
 * synchronise.  Unknown stages and NULL arrays return PIBM_E_ARG.
 *
 * PIBM_STAGE_COLLIDE_T (Eq. lbm2 and lbm9 with push streaming and
 *   bounce-back, Sec. 2.1): in0 = adjoint of the populations after collision
 *   and streaming (Q x n, canonical order); out0 = adjoint of the populations
 *   before the collision, the force field held fixed (Q x n); out1 = adjoint
 *   of the force field (D x n); scalars[0] = derivative with respect to tau.
 *   At the current populations and the force field of the last step.
 * PIBM_STAGE_PARTICLES_T (Eq. lbm7-lbm8, lbm10-lbm13 and demgov, as in
 *   pibm_backward): in0 = adjoint of the spread force field (D x n), in1 and
 *   in2 = adjoints of the positions and velocities after the particle update
 *   (D x np, id order); out0 and out1 = the adjoints of the positions and
 *   velocities before it (D x np, id order), out2 = adjoint of the node
 *   moments that were interpolated (delta rho, j: (1 + D) x n);
 *   scalars[0 .. 2] = derivative with respect to gravity.  At the current
 *   particle state and the moments of the current populations.
 * PIBM_STAGE_INTERP (Eq. lbm11-lbm12): in0 = node fields ((1 + D) x n);
 *   out0 = their interpolation at the particles ((1 + D) x np, in the
 *   library's sorted order, as pibm_read_cell_list reports it), with the
 *   delta-kernel weights of the current positions.
 * PIBM_STAGE_INTERP_T: in0 = (1 + D) x np in the same order; out0 = the
 *   transpose of the last PIBM_STAGE_INTERP, (1 + D) x n: each particle
 *   value spread with the same weights (Eq. lbm10-lbm11).  PIBM_E_STATE
 *   unless PIBM_STAGE_INTERP came first. */
enum { PIBM_STAGE_COLLIDE_T = 1, PIBM_STAGE_PARTICLES_T = 2, PIBM_STAGE_INTERP = 3, PIBM_STAGE_INTERP_T = 4 };
pibm_status pibm_adjoint_stage(pibm_ctx* ctx, int32_t stage, const float* in0, const float* in1,
                               const float* in2, float* out0, float* out1, float* out2, double* scalars);

#ifdef __cplusplus
}
#endif
#endif /* PIBM_H */
