/*
 * pibm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference of one coupled lattice-Boltzmann /
 * particulate immersed boundary (PIBM) / discrete-element time step, written
 * from Zhang et al., "PIBM: Particulate immersed boundary method for
 * fluid-particle interaction problems" (arXiv:1407.6704).  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no source, header, table or helper with the GPU library;
 * the lattice tables below are written out again from the textbook
 * definitions of D2Q9, D3Q15 and D3Q19.
 *
 * Every loop is the definition, in the paper's order: no blocking, no
 * fusion, no shortcut.  Where the paper is silent or garbled the reading
 * taken is stated at the function, tagged R1..R26.
 *
 * Threads: built with OpenMP, the two node loops whose iterations are
 * independent (the moments and the collision-streaming) are split over
 * threads with a static schedule.  Each node's arithmetic is unchanged and
 * no sum crosses nodes, so results are bitwise the same for any thread
 * count.  Every particle, pair, spreading and reduction loop stays serial.
 *
 * Pins (tests/test_oracle_*.py) tie each function to something other than
 * itself: body-force Poiseuille closed form, delta-kernel moments, equilibrium
 * moments, mass and momentum bookkeeping, interpolation/spreading adjointness,
 * one-way terminal settling, brute-force contact lists, restitution,
 * Lagrange polynomial reproduction, Hertz impact theory, rolling and
 * sliding with friction, obstacles as momentum supports.
 * Parity unpinned: long multi-particle trajectories (chaotic; compared by
 * statistics only).
 *
 * Layouts: populations f[q][z][y][x] (x fastest, z = 0 in 2D), vector fields
 * v[a][z][y][x], particle arrays p[a*np + i] (axis-major).  Node (x,y,z) sits
 * at (x+1/2, y+1/2, z+1/2); non-periodic axes have walls at 0 and n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int lattice;            /* 9 = D2Q9, 15 = D3Q15, 19 = D3Q19 */
    int n[3];               /* nodes per axis; n[2] == 1 for D2Q9 */
    int periodic[3];        /* 1: periodic lattice axis (no particles allowed) */
    double tau;             /* BGK relaxation time, Eq. lbm2 */
    double rho0;            /* fluid density used in the buoyancy term */
    double gravity[3];      /* gravitational acceleration, Eq. demgov */
    double fluid_force[3];  /* uniform body force density on the fluid */
    int contact;            /* 0 none, 1 linear spring-dashpot, 2 soft, 3 Hertz, 4 Hertz-Mindlin
                               (no-slip limit), 5 Hertz-Mindlin with micro-slip */
    double kn, restitution; /* linear spring-dashpot parameters */
    double k_soft;          /* soft repulsion stiffness */
    double skin;            /* candidate-list skin */
    int n_sub;              /* DEM sub-steps per lattice step */
    int two_way;            /* 1: spread the particle force onto the fluid */
    int bin_log2;           /* cell-list bin edge, in node spacings, = 2^bin_log2 */
    int interp;             /* 0: cosine delta kernel (Eq. lbm11-lbm12); 1: Lagrange
                               polynomials (Eq. lbm5-lbm6) for the interpolation, the
                               delta kernel still spreads (Eq. lbm10-lbm11) */
    double young, poisson;  /* Hertz contact (contact = 3, 4): Young's modulus and Poisson
                               ratio of the particles and the walls (one material) */
    double friction;        /* contact = 4, 5: Coulomb friction coefficient mu */
} orc_cfg;

/* ------------------------------------------------------------------ */
/* Lattices (R1).  D2Q9, D3Q15 (the paper's lattice, Sec. 2.1) and D3Q19,  */
/* c = 1, c_s^2 = 1/3.  Direction order is                                  */
/* the exchange order of the public interface: rest, then opposite pairs.   */
/* ------------------------------------------------------------------ */

static const int E9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const int E19[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static const int E15[15][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

int orc_q(int lattice) { return lattice == 19 ? 19 : (lattice == 15 ? 15 : 9); }
int orc_dim(int lattice) { return lattice == 9 ? 2 : 3; }

/* Threads used by the node loops (1 without OpenMP).  n < 1 restores the
 * default (all the threads the runtime offers). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n >= 1 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

static const int *lattice_vector(int Q, int q)
{
    return Q == 19 ? E19[q] : (Q == 15 ? E15[q] : E9[q]);
}

/* Velocity set, weights and opposite directions.  Weights are the textbook
 * values for the second-order equilibrium of Eq. lbm3 with c_s^2 = 1/3:
 * D2Q9 4/9, 1/9, 1/36; D3Q15 2/9, 1/9, 1/72 (as listed in Sec. 2.1);
 * D3Q19 1/3, 1/18, 1/36. */
void orc_tables(int lattice, int *e, double *w, int *opp)
{
    int Q = orc_q(lattice);
    for (int q = 0; q < Q; q++) {
        const int *v = lattice_vector(Q, q);
        int s = abs(v[0]) + abs(v[1]) + abs(v[2]);
        for (int a = 0; a < 3; a++) e[3 * q + a] = v[a];
        if (Q == 19)
            w[q] = (s == 0) ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        else if (Q == 15)
            w[q] = (s == 0) ? 2.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 72.0);
        else
            w[q] = (s == 0) ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        /* opposite: search for -e_q */
        for (int r = 0; r < Q; r++) {
            const int *u = lattice_vector(Q, r);
            if (u[0] == -v[0] && u[1] == -v[1] && u[2] == -v[2]) opp[q] = r;
        }
    }
}

/* Equilibrium distribution, Eq. lbm3 (c = 1). */
void orc_equilibrium(int lattice, double rho, const double *u, double *feq)
{
    int Q = orc_q(lattice), e[19 * 3], opp[19];
    double w[19];
    orc_tables(lattice, e, w, opp);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < Q; q++) {
        double eu = e[3 * q] * u[0] + e[3 * q + 1] * u[1] + e[3 * q + 2] * u[2];
        feq[q] = rho * w[q] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

static size_t nnodes(const orc_cfg *c) { return (size_t)c->n[0] * c->n[1] * c->n[2]; }

/* O1.  Density and momentum of the stored (post-stream, pre-collision)
 * populations: rho = sum_q f_q, j = sum_q e_q f_q (Sec. 2.1, the moment
 * definitions after Eq. lbm3). */
void orc_moments(const orc_cfg *c, const double *f, double *rho, double *j)
{
    int Q = orc_q(c->lattice), e[19 * 3], opp[19];
    double w[19];
    orc_tables(c->lattice, e, w, opp);
    size_t N = nnodes(c);
#pragma omp parallel for schedule(static)
    for (size_t r = 0; r < N; r++) {
        double s = 0, m[3] = {0, 0, 0};
        for (int q = 0; q < Q; q++) {
            double v = f[q * N + r];
            s += v;
            for (int a = 0; a < 3; a++) m[a] += e[3 * q + a] * v;
        }
        rho[r] = s;
        for (int a = 0; a < 3; a++) j[a * N + r] = m[a];
    }
}

/* O6 + O7.  BGK collision with the body-force term of Eq. lbm9 (Guo form)
 * and the half-force velocity rho u = sum f e + F/2 (end of Sec. 2.2),
 * Eq. lbm2, followed by streaming.  F may be NULL (no force).  Streaming
 * wraps on periodic axes; a link leaving the domain through a wall is
 * reflected into the opposite direction at the same node (halfway
 * bounce-back; R7: the paper's no-slip walls, nodes at i+1/2, walls at 0 and
 * n).  A diagonal link counts as leaving if any of its components does. */
void orc_collide_stream(const orc_cfg *c, const double *f, const double *F, double *fout)
{
    int Q = orc_q(c->lattice), e[19 * 3], opp[19];
    double w[19];
    orc_tables(c->lattice, e, w, opp);
    size_t N = nnodes(c);
    const double tau = c->tau;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < c->n[2]; z++)
        for (int y = 0; y < c->n[1]; y++)
            for (int x = 0; x < c->n[0]; x++) {
                size_t r = ((size_t)z * c->n[1] + y) * c->n[0] + x;
                double rho = 0, jm[3] = {0, 0, 0}, Fr[3] = {0, 0, 0};
                for (int q = 0; q < Q; q++) {
                    rho += f[q * N + r];
                    for (int a = 0; a < 3; a++) jm[a] += e[3 * q + a] * f[q * N + r];
                }
                if (F)
                    for (int a = 0; a < 3; a++) Fr[a] = F[a * N + r];
                double u[3];
                for (int a = 0; a < 3; a++) u[a] = (jm[a] + 0.5 * Fr[a]) / rho;
                double feq[19];
                orc_equilibrium(c->lattice, rho, u, feq);
                int pos[3] = {x, y, z};
                for (int q = 0; q < Q; q++) {
                    double eu = 0, eF = 0, uF = 0;
                    for (int a = 0; a < 3; a++) {
                        eu += e[3 * q + a] * u[a];
                        eF += e[3 * q + a] * Fr[a];
                        uF += u[a] * Fr[a];
                    }
                    /* Eq. lbm9: (1 - 1/2tau) w [3 (e - u) + 9 (e.u) e] . F */
                    double S = (1.0 - 0.5 / tau) * w[q] * (3.0 * (eF - uF) + 9.0 * eu * eF);
                    double fs = f[q * N + r] - (f[q * N + r] - feq[q]) / tau + S;
                    int t[3], out = 0;
                    for (int a = 0; a < 3; a++) {
                        t[a] = pos[a] + e[3 * q + a];
                        if (t[a] < 0 || t[a] >= c->n[a]) {
                            if (c->periodic[a])
                                t[a] = (t[a] + c->n[a]) % c->n[a];
                            else
                                out = 1;
                        }
                    }
                    if (out)
                        fout[opp[q] * N + r] = fs;
                    else
                        fout[q * N + ((size_t)t[2] * c->n[1] + t[1]) * c->n[0] + t[0]] = fs;
                }
            }
}

/* Eq. lbm12: the four-point cosine regularised delta function. */
double orc_delta(double a)
{
    if (fabs(a) <= 2.0) return 0.25 * (1.0 + cos(M_PI * a / 2.0));
    return 0.0;
}

/* O2.  One-dimensional weights of Eq. lbm11 (h = 1) for the four nodes
 * base_a .. base_a+3 around X_a, base_a = floor(X_a - 1/2) - 1.  Nodes outside
 * the domain get weight zero and the remaining weights of that axis are
 * divided by their sum (R6), which keeps the partition of unity at walls. */
void orc_weights(const orc_cfg *c, const double *X, int *base, double *phi)
{
    int D = orc_dim(c->lattice);
    for (int a = 0; a < D; a++) {
        base[a] = (int)floor(X[a] - 0.5) - 1;
        double s = 0;
        for (int k = 0; k < 4; k++) {
            int i = base[a] + k;
            double v = (i >= 0 && i < c->n[a]) ? orc_delta(X[a] - (i + 0.5)) : 0.0;
            phi[4 * a + k] = v;
            s += v;
        }
        for (int k = 0; k < 4; k++) phi[4 * a + k] /= s;
    }
    for (int a = D; a < 3; a++) {
        base[a] = 0;
        phi[4 * a] = 1.0;
        phi[4 * a + 1] = phi[4 * a + 2] = phi[4 * a + 3] = 0.0;
    }
}

/* O2 with the Lagrange polynomials of Eq. lbm5-lbm6 instead: on the same
 * four nodes per axis, the basis polynomial of node k through the in-domain
 * nodes of that axis (four in the interior: cubic; fewer next to a wall),
 *   l_k(X) = prod over in-domain m != k of (X - x_m) / (x_k - x_m),
 * x_m = base_a + m + 1/2, and zero for nodes outside the domain. */
void orc_weights_lagrange(const orc_cfg *c, const double *X, int *base, double *phi)
{
    int D = orc_dim(c->lattice);
    for (int a = 0; a < D; a++) {
        base[a] = (int)floor(X[a] - 0.5) - 1;
        int in[4];
        for (int k = 0; k < 4; k++) {
            int i = base[a] + k;
            in[k] = (i >= 0 && i < c->n[a]);
        }
        for (int k = 0; k < 4; k++) {
            double v = 0.0;
            if (in[k]) {
                v = 1.0;
                double xk = base[a] + k + 0.5;
                for (int m = 0; m < 4; m++) {
                    if (m == k || !in[m]) continue;
                    double xm = base[a] + m + 0.5;
                    v *= (X[a] - xm) / (xk - xm);
                }
            }
            phi[4 * a + k] = v;
        }
    }
    for (int a = D; a < 3; a++) {
        base[a] = 0;
        phi[4 * a] = 1.0;
        phi[4 * a + 1] = phi[4 * a + 2] = phi[4 * a + 3] = 0.0;
    }
}

/* O3.  Interpolation of density and momentum to each particle with the
 * weights of O2 (or their Lagrange form when interp = 1): rho_i = sum_r W
 * rho, j_i = sum_r W j (R3: moments of the pre-collision state; by linearity
 * this equals interpolating every f_alpha as Eq. lbm5 does and taking
 * moments). */
void orc_interp(const orc_cfg *c, int np, const double *X, const double *rho,
                const double *j, double *rho_i, double *j_i)
{
    int D = orc_dim(c->lattice);
    size_t N = nnodes(c);
    for (int p = 0; p < np; p++) {
        double Xp[3] = {0.5, 0.5, 0.5}, phi[12];
        int base[3];
        for (int a = 0; a < D; a++) Xp[a] = X[a * np + p];
        if (c->interp == 1)
            orc_weights_lagrange(c, Xp, base, phi);
        else
            orc_weights(c, Xp, base, phi);
        double sr = 0, sj[3] = {0, 0, 0};
        int kz_n = (D == 3) ? 4 : 1;
        for (int kz = 0; kz < kz_n; kz++)
            for (int ky = 0; ky < 4; ky++)
                for (int kx = 0; kx < 4; kx++) {
                    double W = phi[kx] * phi[4 + ky] * phi[8 + kz];
                    if (W == 0.0) continue;
                    int x = base[0] + kx, y = base[1] + ky, z = base[2] + kz;
                    size_t r = ((size_t)z * c->n[1] + y) * c->n[0] + x;
                    sr += W * rho[r];
                    for (int a = 0; a < 3; a++) sj[a] += W * j[a * N + r];
                }
        rho_i[p] = sr;
        for (int a = 0; a < 3; a++) j_i[a * np + p] = sj[a];
    }
}

/* O5.  Spreading, Eq. lbm10: F(r) += sum_l coef_l D(r - X_l), where the
 * caller passes coef_l = A_p g_l.  Adds into F (which the caller clears). */
void orc_spread(const orc_cfg *c, int np, const double *X, const double *coef, double *F)
{
    int D = orc_dim(c->lattice);
    size_t N = nnodes(c);
    for (int p = 0; p < np; p++) {
        double Xp[3] = {0.5, 0.5, 0.5}, phi[12];
        int base[3];
        for (int a = 0; a < D; a++) Xp[a] = X[a * np + p];
        orc_weights(c, Xp, base, phi);
        int kz_n = (D == 3) ? 4 : 1;
        for (int kz = 0; kz < kz_n; kz++)
            for (int ky = 0; ky < 4; ky++)
                for (int kx = 0; kx < 4; kx++) {
                    double W = phi[kx] * phi[4 + ky] * phi[8 + kz];
                    if (W == 0.0) continue;
                    int x = base[0] + kx, y = base[1] + ky, z = base[2] + kz;
                    size_t r = ((size_t)z * c->n[1] + y) * c->n[0] + x;
                    for (int a = 0; a < D; a++) F[a * N + r] += W * coef[a * np + p];
                }
    }
}

/* ------------------------------------------------------------------ */
/* Cell list (the paper is silent on neighbour search).  A particle's     */
/* dual cell along axis a is c_a = floor(X_a - 1/2) in [-1, n_a - 1], its   */
/* bin b_a = (c_a + 1) >> bin_log2, and its key the x-fastest linear index  */
/* of the bin.  Particles are ordered by (key, id); bin_start[k] is the     */
/* first sorted slot of bin k, bin_start[nbins] = np.                       */
/* ------------------------------------------------------------------ */

int64_t orc_nbins(const orc_cfg *c, int64_t *nb)
{
    int D = orc_dim(c->lattice);
    int64_t total = 1;
    for (int a = 0; a < 3; a++) {
        nb[a] = (a < D) ? ((int64_t)c->n[a] >> c->bin_log2) + 1 : 1;
        total *= nb[a];
    }
    return total;
}

static int64_t bin_coord(const orc_cfg *c, double x)
{
    int64_t cell = (int64_t)floor(x - 0.5);
    return (cell + 1) >> c->bin_log2;
}

int64_t orc_key(const orc_cfg *c, const double *Xp)
{
    int D = orc_dim(c->lattice);
    int64_t nb[3];
    orc_nbins(c, nb);
    int64_t b[3] = {0, 0, 0};
    for (int a = 0; a < D; a++) b[a] = bin_coord(c, Xp[a]);
    return (b[2] * nb[1] + b[1]) * nb[0] + b[0];
}

typedef struct { int64_t key; int id; } kv_t;
static int kv_cmp(const void *pa, const void *pb)
{
    const kv_t *a = pa, *b = pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* keys[s] and perm[s] are the key and id of sorted slot s. */
void orc_cell_list(const orc_cfg *c, int np, const double *X, int64_t *keys,
                   int *perm, int64_t *bin_start)
{
    int D = orc_dim(c->lattice);
    int64_t nb[3];
    int64_t nbins = orc_nbins(c, nb);
    kv_t *kv = malloc(sizeof(kv_t) * (np > 0 ? np : 1));
    for (int p = 0; p < np; p++) {
        double Xp[3] = {0.5, 0.5, 0.5};
        for (int a = 0; a < D; a++) Xp[a] = X[a * np + p];
        kv[p].key = orc_key(c, Xp);
        kv[p].id = p;
    }
    qsort(kv, np, sizeof(kv_t), kv_cmp);
    for (int s = 0; s < np; s++) {
        keys[s] = kv[s].key;
        perm[s] = kv[s].id;
    }
    /* bin_start by counting */
    for (int64_t k = 0; k <= nbins; k++) bin_start[k] = 0;
    for (int s = 0; s < np; s++) bin_start[kv[s].key + 1]++;
    for (int64_t k = 0; k < nbins; k++) bin_start[k + 1] += bin_start[k];
    free(kv);
}

/* ------------------------------------------------------------------ */
/* Particles and contacts.                                                */
/* ------------------------------------------------------------------ */

/* Particle volume: a disk of unit depth in 2D, a sphere in 3D (R5). */
double orc_mass(int D, double d, double rho_p)
{
    return D == 3 ? rho_p * M_PI * d * d * d / 6.0 : rho_p * 0.25 * M_PI * d * d;
}

/* Cross-sectional area of Eq. lbm10. */
double orc_area(double d) { return 0.25 * M_PI * d * d; }

/* Damping ratio from the coefficient of restitution of a linear
 * spring-dashpot (R10). */
double orc_zeta(double e)
{
    double l = log(e);
    return -l / sqrt(M_PI * M_PI + l * l);
}

/* Hertz normal force of Sec. 2.3 for overlap delta > 0:
 *   F_n = (4/3) E* sqrt(R*) delta^(3/2),
 *   1/E* = (1 - nu^2)/E + (1 - nu^2)/E  (both bodies of the one material),
 *   1/R* = 1/R_p + 1/R_q, or R* = R_p against a flat wall.
 * The paper gives no damping term, so none is added (R24). */
static double hertz_estar(const orc_cfg *c)
{
    return c->young / (2.0 * (1.0 - c->poisson * c->poisson));
}

static double hertz_force(const orc_cfg *c, double rstar, double delta)
{
    return 4.0 / 3.0 * hertz_estar(c) * sqrt(rstar) * delta * sqrt(delta);
}

/* Contact force on particle p from particle q (R10).  r = X_p - X_q,
 * du = U_p - U_q.  Linear spring-dashpot, normal only, no clamp, force only
 * for strictly positive overlap; soft repulsion k_s (1 - r/r_c)^2; or the
 * Hertz force above. */
static void pair_force(const orc_cfg *c, int D, const double *r, const double *du,
                       double dp, double dq, double meff, double *Fout)
{
    double dist2 = 0;
    for (int a = 0; a < D; a++) dist2 += r[a] * r[a];
    double dist = sqrt(dist2);
    double rc = 0.5 * (dp + dq);
    for (int a = 0; a < 3; a++) Fout[a] = 0;
    if (c->contact == 1) {
        double delta = rc - dist;
        if (!(delta > 0.0)) return;
        double vn = 0;
        for (int a = 0; a < D; a++) vn += du[a] * r[a] / dist;
        double gam = 2.0 * orc_zeta(c->restitution) * sqrt(c->kn * meff);
        double mag = c->kn * delta - gam * vn;
        for (int a = 0; a < D; a++) Fout[a] = mag * r[a] / dist;
    } else if (c->contact == 2) {
        if (!(dist < rc)) return;
        double s = 1.0 - dist / rc;
        for (int a = 0; a < D; a++) Fout[a] = c->k_soft * s * s * r[a] / dist;
    } else if (c->contact == 3) {
        double delta = rc - dist;
        if (!(delta > 0.0)) return;
        double Rp = 0.5 * dp, Rq = 0.5 * dq;
        double mag = hertz_force(c, Rp * Rq / (Rp + Rq), delta);
        for (int a = 0; a < D; a++) Fout[a] = mag * r[a] / dist;
    }
}

/* Contact with the walls at 0 and n_a of every non-periodic axis: the wall
 * acts as a particle of infinite mass (and, for Hertz, infinite radius) at
 * distance dist along the inward normal, with r_c = d/2. */
static void wall_force(const orc_cfg *c, int D, const double *X, const double *U,
                       double dp, double mp, double *Fout)
{
    for (int a = 0; a < 3; a++) Fout[a] = 0;
    if (c->contact == 0) return;
    for (int a = 0; a < D; a++) {
        if (c->periodic[a]) continue;
        for (int side = 0; side < 2; side++) {
            double nrm = side == 0 ? 1.0 : -1.0;         /* inward normal */
            double dist = side == 0 ? X[a] : c->n[a] - X[a];
            double vn = U[a] * nrm;
            double rc = 0.5 * dp;
            if (c->contact == 1) {
                double delta = rc - dist;
                if (!(delta > 0.0)) continue;
                double gam = 2.0 * orc_zeta(c->restitution) * sqrt(c->kn * mp);
                Fout[a] += (c->kn * delta - gam * vn) * nrm;
            } else if (c->contact == 3) {
                double delta = rc - dist;
                if (!(delta > 0.0)) continue;
                Fout[a] += hertz_force(c, 0.5 * dp, delta) * nrm;
            } else {
                if (!(dist < rc)) continue;
                double s = 1.0 - dist / rc;
                Fout[a] += c->k_soft * s * s * nrm;
            }
        }
    }
}

/* Candidate pairs: every unordered pair with |X_p - X_q| < (d_p+d_q)/2 + skin,
 * found through the bins of orc_cell_list: the (2H+1)^D bins around a
 * particle, H = ceil((d_max + skin) / bin edge), hold every particle within
 * the largest cutoff.  Writes up to cap pairs (p < q) and returns the total
 * count. */
int64_t orc_candidate_pairs(const orc_cfg *c, int np, const double *X, const double *d,
                            int *pairs, int64_t cap)
{
    int D = orc_dim(c->lattice);
    int64_t nb[3];
    int64_t nbins = orc_nbins(c, nb);
    int64_t *keys = malloc(sizeof(int64_t) * (np > 0 ? np : 1));
    int *perm = malloc(sizeof(int) * (np > 0 ? np : 1));
    int64_t *bs = malloc(sizeof(int64_t) * (nbins + 1));
    orc_cell_list(c, np, X, keys, perm, bs);
    /* the neighbouring bins must cover the largest cutoff */
    double dmax = 0;
    for (int p = 0; p < np; p++)
        if (d[p] > dmax) dmax = d[p];
    int H = (int)ceil((dmax + c->skin) / (double)(1 << c->bin_log2));
    if (H < 1) H = 1;
    int64_t count = 0;
    for (int p = 0; p < np; p++) {
        int64_t b[3] = {0, 0, 0};
        for (int a = 0; a < D; a++) b[a] = bin_coord(c, X[a * np + p]);
        int lo[3], hi[3];
        for (int a = 0; a < 3; a++) {
            lo[a] = (a < D) ? -H : 0;
            hi[a] = (a < D) ? H : 0;
        }
        for (int oz = lo[2]; oz <= hi[2]; oz++)
            for (int oy = lo[1]; oy <= hi[1]; oy++)
                for (int ox = lo[0]; ox <= hi[0]; ox++) {
                    int64_t bb[3] = {b[0] + ox, b[1] + oy, b[2] + oz};
                    int ok = 1;
                    for (int a = 0; a < 3; a++)
                        if (bb[a] < 0 || bb[a] >= nb[a]) ok = 0;
                    if (!ok) continue;
                    int64_t k = (bb[2] * nb[1] + bb[1]) * nb[0] + bb[0];
                    for (int64_t s = bs[k]; s < bs[k + 1]; s++) {
                        int q = perm[s];
                        if (q <= p) continue;
                        double d2 = 0;
                        for (int a = 0; a < D; a++) {
                            double t = X[a * np + p] - X[a * np + q];
                            d2 += t * t;
                        }
                        double cut = 0.5 * (d[p] + d[q]) + c->skin;
                        if (d2 < cut * cut) {
                            if (count < cap) {
                                pairs[2 * count] = p;
                                pairs[2 * count + 1] = q;
                            }
                            count++;
                        }
                    }
                }
    }
    free(keys);
    free(perm);
    free(bs);
    return count;
}

/* Brute-force O(N^2) version of the same list (for pinning the cell list). */
int64_t orc_candidate_pairs_brute(const orc_cfg *c, int np, const double *X, const double *d,
                                  int *pairs, int64_t cap)
{
    int D = orc_dim(c->lattice);
    int64_t count = 0;
    for (int p = 0; p < np; p++)
        for (int q = p + 1; q < np; q++) {
            double d2 = 0;
            for (int a = 0; a < D; a++) {
                double t = X[a * np + p] - X[a * np + q];
                d2 += t * t;
            }
            double cut = 0.5 * (d[p] + d[q]) + c->skin;
            if (d2 < cut * cut) {
                if (count < cap) {
                    pairs[2 * count] = p;
                    pairs[2 * count + 1] = q;
                }
                count++;
            }
        }
    return count;
}

/* Mindlin tangential force and rotation (contact = 4, Sec. 2.3, R25; with
 * the micro-slip factor of R27 for contact = 5).
 * The paper's increment dT = 8 G* r_a theta_k d(delta_t) + (-1)^k mu dF_n (1 - theta_k)
 * is taken in its no-slip limit theta_k = 1, dT = 8 G* r_a d(delta_t), with
 * r_a = sqrt(delta_n R*) and, as printed, 1/G* = (1 - nu^2)/G + (1 - nu^2)/G,
 * G = E / (2 (1 + nu)); the Coulomb bound |T| <= mu F_n caps it (sliding).
 * Per sub-step and contact, with n the unit normal from the partner to the
 * particle and v_t the tangential part of the velocity of the particle's
 * contact point relative to the partner's:
 *   T <- T - (T.n) n, rescaled to its former length (the contact plane turns)
 *   T <- T - 8 G* r_a h v_t,   then |T| <= mu F_n
 * T is the tangential force on the particle; it is zero while the bodies do
 * not overlap.  Moments of inertia: 2/5 m R^2 (sphere), 1/2 m R^2 (disk);
 * torque (-R n) x T on each body; I dW/dt = torque (Eq. demgov, second line). */
static double mindlin_gstar(const orc_cfg *c)
{
    double G = c->young / (2.0 * (1.0 + c->poisson));
    return G / (2.0 * (1.0 - c->poisson * c->poisson));
}

static double inertia(int D, double m, double d)
{
    return (D == 3 ? 0.4 : 0.5) * m * 0.25 * d * d;
}

/* z = x cross y; in 2D vectors lie in the plane and angular quantities are
 * stored in component 2 (the z axis). */
static void cross3(const double *x, const double *y, double *z)
{
    z[0] = x[1] * y[2] - x[2] * y[1];
    z[1] = x[2] * y[0] - x[0] * y[2];
    z[2] = x[0] * y[1] - x[1] * y[0];
}

/* Tangential state of one contact, ORC_TS doubles:
 *   [0..2] T, the tangential force on the particle;
 *   [3..5] the contact's loading direction (a unit vector in the contact
 *          plane; zero until the first tangential increment), micro-slip only;
 *   [6] k: 0 loading, 1 unloading, 2 reloading;  [7] T*, [8] T**: the
 *   tangential force along the loading direction where the last unloading
 *   and reloading began;  [9] the normal force of the previous sub-step. */
#define ORC_TS 10

/* Turn a vector into the contact plane of normal n, keeping its length. */
static void into_plane(const double *n, double *v)
{
    double vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
    double old = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double P[3];
    for (int a = 0; a < 3; a++) P[a] = v[a] - vn * n[a];
    double pl = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
    for (int a = 0; a < 3; a++) v[a] = pl > 0.0 ? P[a] * (old / pl) : 0.0;
}

/* One contact's tangential update.  n: unit normal (3 components, z = 0 in
 * 2D); vrel: contact-point velocity of the particle minus the partner's;
 * Fn: Hertz normal force; rstar: effective radius; delta: overlap.
 * S (in/out, ORC_TS doubles): the tangential state above.
 *
 * The elastic trial increment is E = -8 G* r_a h v_t, r_a = sqrt(delta R*)
 * (v_t: the tangential part of vrel, so h v_t is the increment of the
 * tangential surface displacement).  contact = 4 takes the no-slip limit
 * theta_k = 1 of the paper's increment: T += E.  contact = 5 (R27) applies
 * the paper's increment to the part of E along the contact's loading
 * direction t (the direction of its first tangential increment, turned with
 * the contact plane), e = E.t:
 *   dT = [theta_k e + (-1)^k mu dF_n (1 - theta_k)] t + (E - e t)
 * (the part of E across t is taken elastically), with the
 * Mindlin-Deresiewicz factors in the incremental form of Thornton:
 *   loading   (k = 0): theta^3 = 1 - (T_t + mu dF_n) / (mu F_n)
 *   unloading (k = 1): theta^3 = 1 - (T* - T_t + 2 mu dF_n) / (2 mu F_n)
 *   reloading (k = 2): theta^3 = 1 - (T_t - T** + 2 mu dF_n) / (2 mu F_n)
 * where T_t = T.t, dF_n is the change of the normal force since the last
 * sub-step and theta is clamped to [0, 1] (0: the whole contact slides).
 * k changes where the increment along t, e = E.t, changes sign: loading
 * with e < 0 starts unloading (T* = T_t), unloading with e > 0 starts
 * reloading (T** = T_t), reloading with e < 0 unloads again (T* = T_t) and
 * reloading that reaches T* is back on the loading curve (k = 0).  While the
 * normal force grows faster than the tangential load, |e| <= mu dF_n, no
 * slip zone grows and dT = E.  Along one line (E parallel to t) this is
 * Mindlin-Deresiewicz's law; splitting off the cross part keeps the
 * increment continuous where k changes (e = 0) and where the slip zone
 * starts to grow (|e| = mu dF_n).  Both forms finally cap |T| at mu F_n
 * (Coulomb sliding). */
static void tangential_update(const orc_cfg *c, double h, const double *n, const double *vrel,
                              double Fn, double rstar, double delta, double *S)
{
    double *T = S, *t = S + 3;
    into_plane(n, T);
    double vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    double kt = 8.0 * mindlin_gstar(c) * sqrt(delta * rstar);
    double E[3];
    for (int a = 0; a < 3; a++) E[a] = -kt * h * (vrel[a] - vn * n[a]);
    double mu = c->friction;
    if (c->contact == 5) {
        into_plane(n, t);
        double dFn = Fn - S[9];
        S[9] = Fn;
        double el = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
        double tl = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        if (tl == 0.0 && el > 0.0) {                  /* the first tangential increment sets t */
            for (int a = 0; a < 3; a++) t[a] = E[a] / el;
            S[6] = 0.0;
            S[7] = S[8] = 0.0;
            tl = 1.0;
        }
        if (tl > 0.0) {
            double Tt = T[0] * t[0] + T[1] * t[1] + T[2] * t[2];
            double e = E[0] * t[0] + E[1] * t[1] + E[2] * t[2];
            int k = (int)S[6];
            if (k == 0 && e < 0.0) {
                k = 1;
                S[7] = Tt;
            } else if (k == 1 && e > 0.0) {
                k = 2;
                S[8] = Tt;
            } else if (k == 2) {
                if (e < 0.0) {
                    k = 1;
                    S[7] = Tt;
                } else if (Tt >= S[7]) {
                    k = 0;
                }
            }
            S[6] = k;
            if (dFn > 0.0 && fabs(e) <= mu * dFn) {
                for (int a = 0; a < 3; a++) T[a] += E[a];
            } else {
                double arg;
                if (k == 0)
                    arg = 1.0 - (Tt + mu * dFn) / (mu * Fn);
                else if (k == 1)
                    arg = 1.0 - (S[7] - Tt + 2.0 * mu * dFn) / (2.0 * mu * Fn);
                else
                    arg = 1.0 - (Tt - S[8] + 2.0 * mu * dFn) / (2.0 * mu * Fn);
                arg = arg < 0.0 ? 0.0 : (arg > 1.0 ? 1.0 : arg);
                double th = cbrt(arg);
                double sg = k == 1 ? -1.0 : 1.0;
                double dt = th * e + sg * mu * dFn * (1.0 - th);     /* along t */
                for (int a = 0; a < 3; a++) T[a] += dt * t[a] + (E[a] - e * t[a]);
            }
        }
    } else {
        for (int a = 0; a < 3; a++) T[a] += E[a];
    }
    double tl = sqrt(T[0] * T[0] + T[1] * T[1] + T[2] * T[2]);
    double lim = mu * Fn;
    if (tl > lim)
        for (int a = 0; a < 3; a++) T[a] *= lim / tl;
}

/* The tangential update alone, for the tests (same arguments). */
void orc_tangential_update(const orc_cfg *c, double h, const double *n, const double *vrel, double Fn,
                           double rstar, double delta, double *S)
{
    tangential_update(c, h, n, vrel, Fn, rstar, delta, S);
}

/* History of the tangential forces between steps: entry i is the pair
 * key[2i], key[2i+1] (particle indices p < q, or p and -1 - (2 a + side) for
 * the wall at side 0 / n of axis a) with the state S[ORC_TS i ..] of p. */
static int64_t hist_find(int64_t hn, const int *key, int p, int q)
{
    for (int64_t i = 0; i < hn; i++)
        if (key[2 * i] == p && key[2 * i + 1] == q) return i;
    return -1;
}

/* O4.  Particle sub-steps (R4, R8, R9).  For k = 0 .. n_sub-1 with h = 1/n_sub,
 * every force uses the state at sub-step k (Jacobi):
 *   g^k   = 2 (rho_i U^k - j_i)                (R2: momentum exchange, Eqs. lbm7-lbm8)
 *   F_h^k = -A_p g^k                           (Eq. lbm13)
 *   F_c^k = sum over candidate pairs and walls
 *   U^{k+1} = U^k + h (F_h^k + F_c^k + (1 - rho0/rho_p) m g) / m   (Eq. demgov)
 *   X^{k+1} = X^k + h U^{k+1}
 *   W^{k+1} = W^k + h torque^k / I             (contact = 4, 5 only)
 * Outputs the final X, U, the sub-step mean gbar of g (what the fluid
 * receives), the sub-step mean contact force, and vmax_p = max_k |U^k|
 * over k = 0..n_sub (the skin check: displacement <= vmax * one step).
 * pairs: candidate pairs at the start of the step (orc_candidate_pairs).
 * With contact = 4 or 5: W (3 x np, angular velocities) is updated, and the
 * tangential history (hn_in entries of ORC_TS doubles each) is read and
 * rewritten to key_out / T_out (capacity npairs + 2 D np entries),
 * returning the entry count.
 * fixed (nullable): points of fixed obstacle bodies (R26), which keep X,
 * U = 0 and W = 0, exchange momentum with the fluid like any point (g with
 * U = 0), act on moving particles with infinite mass, and feel neither the
 * walls nor each other. */
static double pair_meff(const int *fixed, int p, int q, const double *m)
{
    if (fixed && fixed[p]) return m[q];
    if (fixed && fixed[q]) return m[p];
    return m[p] * m[q] / (m[p] + m[q]);
}

int64_t orc_dem_full(const orc_cfg *c, int np, double *X, double *U, double *W, const double *d,
                     const double *rho_p, const int *fixed, const double *rho_i, const double *j_i,
                     int64_t npairs, const int *pairs, int64_t hn_in, const int *key_in,
                     const double *T_in, int *key_out, double *T_out,
                     double *gbar, double *fc_mean, double *vmax)
{
    int D = orc_dim(c->lattice);
    int n_sub = c->n_sub;
    double h = 1.0 / n_sub;
    int mind = c->contact == 4 || c->contact == 5;
    int npp = np > 0 ? np : 1;
    double *m = malloc(sizeof(double) * npp);
    double *g = malloc(sizeof(double) * 3 * npp);
    double *Fc = malloc(sizeof(double) * 3 * npp);
    double *tq = malloc(sizeof(double) * 3 * npp);
    double *Tp = malloc(sizeof(double) * ORC_TS * (npairs > 0 ? npairs : 1));
    double *Tw = malloc(sizeof(double) * ORC_TS * 6 * npp);
    /* tangential forces carried over from the previous step */
    for (int64_t i = 0; i < npairs; i++) {
        int64_t e = mind ? hist_find(hn_in, key_in, pairs[2 * i], pairs[2 * i + 1]) : -1;
        for (int a = 0; a < ORC_TS; a++) Tp[ORC_TS * i + a] = e >= 0 ? T_in[ORC_TS * e + a] : 0.0;
    }
    for (int p = 0; p < np; p++)
        for (int w = 0; w < 6; w++) {
            int64_t e = mind ? hist_find(hn_in, key_in, p, -1 - w) : -1;
            for (int a = 0; a < ORC_TS; a++) Tw[ORC_TS * (6 * p + w) + a] = e >= 0 ? T_in[ORC_TS * e + a] : 0.0;
        }
    for (int p = 0; p < np; p++) {
        m[p] = orc_mass(D, d[p], rho_p[p]);
        for (int a = 0; a < 3; a++) {
            gbar[a * np + p] = 0;
            fc_mean[a * np + p] = 0;
        }
        double s = 0;
        for (int a = 0; a < D; a++) s += U[a * np + p] * U[a * np + p];
        vmax[p] = sqrt(s);
    }
    for (int k = 0; k < n_sub; k++) {
        /* forces at sub-step k */
        for (int p = 0; p < np; p++) {
            for (int a = 0; a < 3; a++) {
                g[3 * p + a] = (a < D) ? 2.0 * (rho_i[p] * U[a * np + p] - j_i[a * np + p]) : 0.0;
                Fc[3 * p + a] = 0;
                tq[3 * p + a] = 0;
            }
            double Xp[3] = {0, 0, 0}, Up[3] = {0, 0, 0}, Fw[3];
            for (int a = 0; a < D; a++) {
                Xp[a] = X[a * np + p];
                Up[a] = U[a * np + p];
            }
            if (fixed && fixed[p]) continue;
            if (!mind) {
                wall_force(c, D, Xp, Up, d[p], m[p], Fw);
                for (int a = 0; a < D; a++) Fc[3 * p + a] += Fw[a];
                continue;
            }
            /* Hertz-Mindlin walls: infinite radius and mass, at rest */
            double R = 0.5 * d[p];
            for (int a = 0; a < D; a++) {
                if (c->periodic[a]) continue;
                for (int side = 0; side < 2; side++) {
                    double *T = Tw + ORC_TS * (6 * p + 2 * a + side);
                    double dist = side == 0 ? Xp[a] : c->n[a] - Xp[a];
                    double delta = R - dist;
                    if (!(delta > 0.0)) {
                        memset(T, 0, sizeof(double) * ORC_TS);     /* out of contact: no state */
                        continue;
                    }
                    double n[3] = {0, 0, 0};
                    n[a] = side == 0 ? 1.0 : -1.0;          /* from the wall to the particle */
                    double Fn = hertz_force(c, R, delta);
                    double arm[3], wr[3], vrel[3];
                    for (int b = 0; b < 3; b++) arm[b] = -R * n[b];
                    double Wp[3] = {0, 0, W[2 * np + p]};
                    if (D == 3) { Wp[0] = W[p]; Wp[1] = W[np + p]; }
                    cross3(Wp, arm, wr);
                    for (int b = 0; b < 3; b++) vrel[b] = Up[b] + wr[b];
                    tangential_update(c, h, n, vrel, Fn, R, delta, T);
                    double t[3];
                    cross3(arm, T, t);
                    for (int b = 0; b < 3; b++) {
                        Fc[3 * p + b] += Fn * n[b] + T[b];
                        tq[3 * p + b] += t[b];
                    }
                }
            }
        }
        if (c->contact != 0)
            for (int64_t i = 0; i < npairs; i++) {
                int p = pairs[2 * i], q = pairs[2 * i + 1];
                if (fixed && fixed[p] && fixed[q]) continue;
                double r[3] = {0, 0, 0}, du[3] = {0, 0, 0}, Fpq[3];
                for (int a = 0; a < D; a++) {
                    r[a] = X[a * np + p] - X[a * np + q];
                    du[a] = U[a * np + p] - U[a * np + q];
                }
                if (!mind) {
                    pair_force(c, D, r, du, d[p], d[q], pair_meff(fixed, p, q, m), Fpq);
                    for (int a = 0; a < D; a++) {
                        Fc[3 * p + a] += Fpq[a];
                        Fc[3 * q + a] -= Fpq[a];
                    }
                    continue;
                }
                double *T = Tp + ORC_TS * i;
                double dist = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                double Rp = 0.5 * d[p], Rq = 0.5 * d[q];
                double delta = Rp + Rq - dist;
                if (!(delta > 0.0)) {
                    memset(T, 0, sizeof(double) * ORC_TS);
                    continue;
                }
                double rstar = Rp * Rq / (Rp + Rq);
                double Fn = hertz_force(c, rstar, delta);
                double n[3], ap[3], aq[3], wp[3], wq[3], vrel[3];
                for (int a = 0; a < 3; a++) {
                    n[a] = r[a] / dist;                     /* from q to p */
                    ap[a] = -Rp * n[a];                      /* contact point from p's centre */
                    aq[a] = Rq * n[a];                       /* contact point from q's centre */
                }
                double Wp[3] = {0, 0, W[2 * np + p]}, Wq[3] = {0, 0, W[2 * np + q]};
                if (D == 3) {
                    Wp[0] = W[p]; Wp[1] = W[np + p];
                    Wq[0] = W[q]; Wq[1] = W[np + q];
                }
                cross3(Wp, ap, wp);
                cross3(Wq, aq, wq);
                for (int a = 0; a < 3; a++) vrel[a] = (du[a] + wp[a]) - wq[a];
                tangential_update(c, h, n, vrel, Fn, rstar, delta, T);
                double tp[3], tqq[3], mT[3] = {-T[0], -T[1], -T[2]};
                cross3(ap, T, tp);
                cross3(aq, mT, tqq);
                for (int a = 0; a < 3; a++) {
                    Fc[3 * p + a] += Fn * n[a] + T[a];
                    Fc[3 * q + a] -= Fn * n[a] + T[a];
                    tq[3 * p + a] += tp[a];
                    tq[3 * q + a] += tqq[a];
                }
            }
        /* symplectic Euler update */
        for (int p = 0; p < np; p++) {
            double A = orc_area(d[p]);
            double s = 0;
            if (fixed && fixed[p]) {
                for (int a = 0; a < D; a++) {
                    gbar[a * np + p] += g[3 * p + a];
                    fc_mean[a * np + p] += Fc[3 * p + a];
                }
                continue;
            }
            for (int a = 0; a < D; a++) {
                double Wg = (1.0 - c->rho0 / rho_p[p]) * m[p] * c->gravity[a];
                double Fh = -A * g[3 * p + a];
                U[a * np + p] += h * (Fh + Fc[3 * p + a] + Wg) / m[p];
                X[a * np + p] += h * U[a * np + p];
                gbar[a * np + p] += g[3 * p + a];
                fc_mean[a * np + p] += Fc[3 * p + a];
                s += U[a * np + p] * U[a * np + p];
            }
            if (mind) {
                double I = inertia(D, m[p], d[p]);
                for (int a = (D == 3 ? 0 : 2); a < 3; a++) W[a * np + p] += h * tq[3 * p + a] / I;
            }
            if (sqrt(s) > vmax[p]) vmax[p] = sqrt(s);
        }
    }
    for (int p = 0; p < np; p++)
        for (int a = 0; a < 3; a++) {
            gbar[a * np + p] /= n_sub;
            fc_mean[a * np + p] /= n_sub;
        }
    /* the new history: every contact whose tangential state is not zero
     * (the no-slip form carries only T, so a contact carries a force) */
    int64_t hn = 0;
    if (mind) {
        for (int64_t i = 0; i < npairs; i++) {
            double *T = Tp + ORC_TS * i;
            int any = 0;
            for (int a = 0; a < ORC_TS; a++) any |= T[a] != 0.0;
            if (!any) continue;
            key_out[2 * hn] = pairs[2 * i];
            key_out[2 * hn + 1] = pairs[2 * i + 1];
            for (int a = 0; a < ORC_TS; a++) T_out[ORC_TS * hn + a] = T[a];
            hn++;
        }
        for (int p = 0; p < np; p++)
            for (int w = 0; w < 6; w++) {
                double *T = Tw + ORC_TS * (6 * p + w);
                int any = 0;
                for (int a = 0; a < ORC_TS; a++) any |= T[a] != 0.0;
                if (!any) continue;
                key_out[2 * hn] = p;
                key_out[2 * hn + 1] = -1 - w;
                for (int a = 0; a < ORC_TS; a++) T_out[ORC_TS * hn + a] = T[a];
                hn++;
            }
    }
    free(m);
    free(g);
    free(Fc);
    free(tq);
    free(Tp);
    free(Tw);
    return hn;
}

void orc_dem(const orc_cfg *c, int np, double *X, double *U, const double *d,
             const double *rho_p, const double *rho_i, const double *j_i,
             int64_t npairs, const int *pairs, double *gbar, double *fc_mean, double *vmax)
{
    orc_dem_full(c, np, X, U, NULL, d, rho_p, NULL, rho_i, j_i, npairs, pairs, 0, NULL, NULL, NULL, NULL,
                 gbar, fc_mean, vmax);
}

/* One coupled step n -> n+1, O1..O7 (R9):
 *   O1 moments of f;  O2-O3 weights and interpolation at the start-of-step
 *   positions;  O4 particle sub-steps;  O5 spreading of A_p gbar with the
 *   start-of-step weights (if two_way);  O6-O7 collision with
 *   F = fluid_force + spread, and streaming.
 * Particle state X, U (and, with contact = 4 or 5, W and the tangential
 * history of orc_dem_full) is updated in place.  Outputs: fout; F (D x N,
 * the force field used by the collision); gbar, fc_mean (D x np); returns
 * the number of particles whose vmax exceeds skin/2 (the skin check). */
int orc_step_full(const orc_cfg *c, const double *f, double *fout, double *F,
                  int np, double *X, double *U, double *W, const double *d, const double *rho_p,
                  const int *fixed, const double *area,
                  int64_t hn_in, const int *key_in, const double *T_in, int *key_out, double *T_out,
                  int64_t *hn_out, double *gbar, double *fc_mean, double *rho_i_out, double *j_i_out)
{
    int D = orc_dim(c->lattice);
    size_t N = nnodes(c);
    double *rho = malloc(sizeof(double) * N);
    double *j = malloc(sizeof(double) * 3 * N);
    orc_moments(c, f, rho, j);

    int npp = np > 0 ? np : 1;
    double *X0 = malloc(sizeof(double) * 3 * npp);
    double *rho_i = malloc(sizeof(double) * npp);
    double *j_i = malloc(sizeof(double) * 3 * npp);
    double *vmax = malloc(sizeof(double) * npp);
    memcpy(X0, X, sizeof(double) * D * np);
    orc_interp(c, np, X0, rho, j, rho_i, j_i);

    int64_t npairs = 0;
    int *pairs = NULL;
    if (c->contact != 0 && np > 1) {
        npairs = orc_candidate_pairs(c, np, X0, d, NULL, 0);
        pairs = malloc(sizeof(int) * 2 * (npairs > 0 ? npairs : 1));
        orc_candidate_pairs(c, np, X0, d, pairs, npairs);
    }
    int64_t hn = orc_dem_full(c, np, X, U, W, d, rho_p, fixed, rho_i, j_i, npairs, pairs, hn_in, key_in, T_in,
                              key_out, T_out, gbar, fc_mean, vmax);
    if (hn_out) *hn_out = hn;

    for (int a = 0; a < D; a++)
        for (size_t r = 0; r < N; r++) F[a * N + r] = c->fluid_force[a];
    if (c->two_way && np > 0) {
        double *coef = malloc(sizeof(double) * 3 * npp);
        for (int p = 0; p < np; p++)
            for (int a = 0; a < D; a++) {
                /* a fixed point may carry its own area (an IBM surface element, R26) */
                double A = (fixed && fixed[p] && area) ? area[p] : orc_area(d[p]);
                coef[a * np + p] = A * gbar[a * np + p];
            }
        orc_spread(c, np, X0, coef, F);
        free(coef);
    }
    /* the collision takes a 3-component field; pad the 2D case */
    double *F3 = malloc(sizeof(double) * 3 * N);
    for (int a = 0; a < 3; a++)
        for (size_t r = 0; r < N; r++) F3[a * N + r] = (a < D) ? F[a * N + r] : 0.0;
    orc_collide_stream(c, f, F3, fout);

    int nskin = 0;
    for (int p = 0; p < np; p++)
        if (vmax[p] > 0.5 * c->skin) nskin++;
    if (rho_i_out) memcpy(rho_i_out, rho_i, sizeof(double) * np);
    if (j_i_out)
        for (int a = 0; a < D; a++)
            for (int p = 0; p < np; p++) j_i_out[a * np + p] = j_i[a * np + p];
    free(F3);
    free(rho);
    free(j);
    free(X0);
    free(rho_i);
    free(j_i);
    free(vmax);
    free(pairs);
    return nskin;
}

int orc_step(const orc_cfg *c, const double *f, double *fout, double *F,
             int np, double *X, double *U, const double *d, const double *rho_p,
             double *gbar, double *fc_mean, double *rho_i_out, double *j_i_out)
{
    return orc_step_full(c, f, fout, F, np, X, U, NULL, d, rho_p, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL,
                         gbar, fc_mean, rho_i_out, j_i_out);
}

/* Total fluid mass sum_r sum_q f and momentum sum_r sum_q e_q f. */
void orc_fluid_totals(const orc_cfg *c, const double *f, double *mass, double *mom)
{
    int Q = orc_q(c->lattice), e[19 * 3], opp[19];
    double w[19];
    orc_tables(c->lattice, e, w, opp);
    size_t N = nnodes(c);
    *mass = 0;
    mom[0] = mom[1] = mom[2] = 0;
    for (int q = 0; q < Q; q++)
        for (size_t r = 0; r < N; r++) {
            *mass += f[q * N + r];
            for (int a = 0; a < 3; a++) mom[a] += e[3 * q + a] * f[q * N + r];
        }
}
