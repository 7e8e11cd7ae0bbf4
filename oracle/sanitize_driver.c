/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A stand-alone program that drives every entry point of the FP64 oracle
 * (pibm_oracle.c, included below as one translation unit) through coupled
 * steps with contacts, so that the test suite can build it with the
 * compiler's address and undefined-behaviour sanitizers and run it: every
 * heap access, every integer and float-to-int conversion along the
 * paths the parity tests use is then checked.
 *
 * Cases: D2Q9 with the linear spring-dashpot and the Lagrange gather;
 * D3Q19 with Hertz-Mindlin contacts (no-slip and micro-slip forms),
 * rotation, the tangential history carried over three steps, and points of
 * fixed obstacle bodies with their own areas; D3Q15 with soft repulsion and bins of four cells; and the
 * brute-force and cell-list candidate searches.  It prints one line per
 * case and "sanitize_driver: ok" at the end; a sanitizer finding aborts
 * with a report and a non-zero exit status.
 */
#include <stdio.h>

#include "pibm_oracle.c"

static unsigned long long rng_state = 88172645463325252ULL;

/* xorshift64 (Marsaglia 2003) mapped to [0, 1) */
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static orc_cfg base_cfg(int lattice, int nx, int ny, int nz)
{
    orc_cfg c;
    memset(&c, 0, sizeof c);
    c.lattice = lattice;
    c.n[0] = nx;
    c.n[1] = ny;
    c.n[2] = nz;
    c.tau = 0.7;
    c.rho0 = 1.0;
    c.gravity[orc_dim(lattice) - 1] = -1e-5;
    c.contact = 1;
    c.kn = 1e3;
    c.restitution = 0.9;
    c.k_soft = 1e-3;
    c.skin = 0.05;
    c.n_sub = 40;
    c.two_way = 1;
    c.bin_log2 = 1;
    c.young = 1.0;
    c.poisson = 0.33;
    c.friction = 0.33;
    return c;
}

/* Particles in touching clusters, one on a wall and one in a corner. */
static void place(const orc_cfg *c, int np, double *X, double *U, double *d, double *rp)
{
    int D = orc_dim(c->lattice);
    for (int p = 0; p < np; p++) {
        d[p] = 0.4 + 0.2 * urand();
        rp[p] = 1.5 + urand();
        for (int a = 0; a < D; a++) {
            X[a * np + p] = 0.6 + (c->n[a] - 1.2) * urand();
            U[a * np + p] = 1e-5 * (urand() - 0.5);
        }
        if (p % 3 == 1) {                                  /* touching the previous one */
            for (int a = 0; a < D; a++) X[a * np + p] = X[a * np + p - 1];
            X[p] += 0.999 * 0.5 * (d[p] + d[p - 1]);
            if (X[p] > c->n[0] - 0.3) X[p] -= 2.0 * 0.999 * 0.5 * (d[p] + d[p - 1]);
        }
    }
    X[(D - 1) * np + 2] = 0.499 * d[2];                     /* overlapping the floor */
    for (int a = 0; a < D; a++) X[a * np + 5] = 0.499 * d[5];   /* in a corner */
}

static int run_case(const char *name, orc_cfg c, int np, int steps, int with_bodies)
{
    int D = orc_dim(c.lattice), Q = orc_q(c.lattice);
    size_t N = (size_t)c.n[0] * c.n[1] * c.n[2];
    double *f = malloc(sizeof(double) * Q * N), *fo = malloc(sizeof(double) * Q * N);
    double *F = malloc(sizeof(double) * D * N);
    double *X = calloc(3 * np, sizeof(double)), *U = calloc(3 * np, sizeof(double));
    double *W = calloc(3 * np, sizeof(double)), *d = malloc(sizeof(double) * np);
    double *rp = malloc(sizeof(double) * np), *area = malloc(sizeof(double) * np);
    double *gbar = malloc(sizeof(double) * 3 * np), *fc = malloc(sizeof(double) * 3 * np);
    double *rho_i = malloc(sizeof(double) * np), *j_i = malloc(sizeof(double) * 3 * np);
    int *fixed = calloc(np, sizeof(int));
    int64_t cap = 64 * (int64_t)np + 6 * (int64_t)np + 1, hn = 0, hn_out = 0;
    int *key_in = calloc(2 * cap, sizeof(int)), *key_out = calloc(2 * cap, sizeof(int));
    double *T_in = calloc(3 * cap, sizeof(double)), *T_out = calloc(3 * cap, sizeof(double));
    int e[19 * 3], opp[19];
    double w[19];
    orc_tables(c.lattice, e, w, opp);
    for (int q = 0; q < Q; q++)
        for (size_t r = 0; r < N; r++) f[q * N + r] = w[q] * (1.0 + 1e-3 * (urand() - 0.5));
    if (np > 5) place(&c, np, X, U, d, rp);
    for (int p = 0; p < np; p++) {
        W[2 * np + p] = 1e-3 * (urand() - 0.5);
        if (D == 3) {
            W[p] = 1e-3 * (urand() - 0.5);
            W[np + p] = 1e-3 * (urand() - 0.5);
        }
        area[p] = 0.0;
        if (with_bodies && p % 7 == 3) {                   /* a point of a fixed body */
            fixed[p] = 1;
            area[p] = p % 2 ? 0.3 : -1.0;
            for (int a = 0; a < 3; a++) {
                U[a * np + p] = 0.0;
                W[a * np + p] = 0.0;
            }
        }
    }
    int nskin = 0;
    for (int s = 0; s < steps; s++) {
        nskin += orc_step_full(&c, f, fo, F, np, X, U, W, d, rp, with_bodies ? fixed : NULL,
                               with_bodies ? area : NULL, hn, key_in, T_in, key_out, T_out, &hn_out,
                               gbar, fc, rho_i, j_i);
        memcpy(f, fo, sizeof(double) * Q * N);
        hn = hn_out;
        memcpy(key_in, key_out, sizeof(int) * 2 * hn);
        memcpy(T_in, T_out, sizeof(double) * 3 * hn);
    }
    double mass, mom[3];
    orc_fluid_totals(&c, f, &mass, mom);
    int64_t npair = orc_candidate_pairs(&c, np, X, d, NULL, 0);
    int *pairs = malloc(sizeof(int) * 2 * (npair > 0 ? npair : 1));
    int *pairs_b = malloc(sizeof(int) * 2 * (npair > 0 ? npair : 1));
    orc_candidate_pairs(&c, np, X, d, pairs, npair);
    int64_t nb = orc_candidate_pairs_brute(&c, np, X, d, pairs_b, npair);
    printf("%s: mass %.12f, %lld candidate pairs (brute force %lld), history %lld, skin %d\n", name, mass,
           (long long)npair, (long long)nb, (long long)hn, nskin);
    int bad = nb != npair || !(mass > 0.0);
    free(f); free(fo); free(F); free(X); free(U); free(W); free(d); free(rp); free(area);
    free(gbar); free(fc); free(rho_i); free(j_i); free(fixed); free(key_in); free(key_out);
    free(T_in); free(T_out); free(pairs); free(pairs_b);
    return bad;
}

int main(void)
{
    int bad = 0;
    orc_cfg c = base_cfg(9, 23, 19, 1);
    c.interp = 1;
    bad |= run_case("D2Q9 spring-dashpot, Lagrange gather", c, 60, 3, 0);

    c = base_cfg(19, 11, 10, 9);
    c.contact = 4;
    bad |= run_case("D3Q19 Hertz-Mindlin, rotation, fixed bodies", c, 70, 3, 1);

    c = base_cfg(19, 11, 10, 9);
    c.contact = 5;
    bad |= run_case("D3Q19 Hertz-Mindlin with micro-slip, rotation, fixed bodies", c, 70, 3, 1);

    c = base_cfg(9, 17, 15, 1);
    c.contact = 3;
    bad |= run_case("D2Q9 Hertz, fixed bodies", c, 40, 2, 1);

    c = base_cfg(15, 12, 9, 10);
    c.contact = 2;
    c.n_sub = 1;
    c.bin_log2 = 2;
    bad |= run_case("D3Q15 soft repulsion, bins of four", c, 50, 2, 0);

    c = base_cfg(19, 8, 8, 8);
    c.contact = 0;
    c.periodic[0] = c.periodic[1] = c.periodic[2] = 1;
    c.fluid_force[0] = 1e-6;
    bad |= run_case("D3Q19 periodic lattice", c, 0, 2, 0);
    if (bad) {
        printf("sanitize_driver: FAILED\n");
        return 1;
    }
    printf("sanitize_driver: ok\n");
    return 0;
}
