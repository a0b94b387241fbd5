/*
 * Driver for the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure; built and run by tests/test_oracle_sanitized.py on
 * the CPU).  It includes the oracle's source as one translation unit and
 * calls every exported entry point on small seeded inputs: each scheme,
 * limiter, system, dimension count and boundary rule, the sampled entry
 * points, the building blocks, invalid arguments and the non-finite gamma
 * sum.  Any invalid access or undefined operation aborts the run; the exit
 * status is 0 only when every call also returned what it should.
 */
#include "../oracle/tenom_oracle.c"

#include <stdio.h>

static uint64_t g_rng = 0x2010132890ull;

/* splitmix64, uniform in [0, 1) */
static double urand(void) {
    uint64_t z = (g_rng += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int g_fail = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
            g_fail = 1;                                               \
        }                                                             \
    } while (0)

/* A positive Euler state (rho, momenta, E) with waves and one jump, or
 * scalar data of the same kind. */
static void fill_state(const or_grid* g, double* U) {
    int nf = or_nfields(g);
    size_t N = or_ncells(g);
    for (size_t i = 0; i < N; i++) {
        double jump = (i % 7 < 3) ? 1.0 : 0.3;
        if (g->system == 0) {
            U[i] = jump + 0.2 * urand();
            continue;
        }
        double rho = jump * (0.8 + 0.2 * urand());
        double e = 1.0 + 0.5 * urand();
        double ke = 0.0;
        for (int d = 0; d < g->ndim; d++) {
            double u = 0.3 * (urand() - 0.5);
            U[(size_t)(1 + d) * N + i] = rho * u;
            ke += 0.5 * rho * u * u;
        }
        U[i] = rho;
        U[(size_t)(nf - 1) * N + i] = e / 0.4 + ke;
    }
}

static void run_grid(int ndim, int system, int bc, int scheme, int lim) {
    static const int sizes[3][3] = {{13, 1, 1}, {9, 8, 1}, {7, 5, 6}};
    or_grid g;
    memset(&g, 0, sizeof(g));
    g.ndim = ndim;
    g.system = system;
    for (int d = 0; d < 3; d++) {
        g.n[d] = sizes[ndim - 1][d];
        g.dx[d] = 0.1 + 0.01 * d;
        g.bc[d] = (bc + d) & 1;
        g.adv[d] = (d & 1) ? -0.7 : 1.1;
    }
    int nf = or_nfields(&g);
    size_t N = or_ncells(&g);
    double C_T = (scheme & 0xff) == 6 ? 1e-5 : 1e-7;
    double* U = malloc(sizeof(double) * nf * N);
    double* D = malloc(sizeof(double) * nf * N);
    fill_state(&g, U);
    for (int ax = 0; ax < ndim; ax++) {
        size_t nfaces = N / (size_t)g.n[ax] * (size_t)(g.n[ax] + 1);
        double* F = malloc(sizeof(double) * nf * nfaces);
        uint8_t* fl = malloc(2 * (size_t)nf * nfaces);
        uint8_t* bd = malloc(2 * (size_t)nf * nfaces);
        CHECK(or_reconstruct_faces(&g, scheme, lim, C_T, 1.4, ax, U, F, fl, bd) == 0);
        long idx[3] = {0, (long)nfaces / 2, (long)nfaces - 1};
        double Fp[3 * 5];
        uint8_t flp[3 * 10], bdp[3 * 10];
        CHECK(or_faces_points(&g, scheme, lim, C_T, 1.4, ax, U, 3, idx, Fp, flp, bdp) == 0);
        for (int t = 0; t < 3; t++)
            for (int f = 0; f < nf; f++) CHECK(Fp[t * nf + f] == F[(size_t)f * nfaces + idx[t]]);
        free(F);
        free(fl);
        free(bd);
    }
    CHECK(or_flux_divergence(&g, scheme, lim, C_T, 1.4, U, D) == 0);
    long cells[2] = {0, (long)N - 1};
    double Dp[2 * 5], Up[2 * 5];
    long bh[2];
    CHECK(or_dudt_points(&g, scheme, lim, C_T, 1.4, U, 2, cells, Dp, bh) == 0);
    double rate = or_max_wave_speed(&g, 1.4, U);
    CHECK(isfinite(rate) && rate > 0.0);
    double dt = 0.4 / rate;
    CHECK(or_rk3_points(&g, scheme, lim, C_T, 1.4, dt, U, 2, cells, Up, bh) == 0);
    CHECK(or_rk3_step(&g, scheme, lim, C_T, 1.4, dt, U) == 0);
    for (int t = 0; t < 2; t++)
        for (int f = 0; f < nf; f++) CHECK(Up[t * nf + f] == U[(size_t)f * N + cells[t]]);
    free(U);
    free(D);
}

int main(void) {
    CHECK(or_init() == 0);
    CHECK(or_trace_size() == (int)sizeof(or_trace));
    double d[6], c[8];
    CHECK(or_get_weights(6, d) == 0 && or_get_weights(8, d) == 0);
    CHECK(or_get_poly_face(-2, 3, c) == 0);
    CHECK(isnan(or_beta_stencil(3, 1, c)) && isnan(or_beta_stencil(-4, 5, c)));
    CHECK(or_param("mp_alpha") == 1.25 && isnan(or_param("")));

    /* building blocks on random data */
    for (int t = 0; t < 2000; t++) {
        double f[8];
        for (int m = 0; m < 8; m++) f[m] = 4.0 * urand() - 2.0;
        double lo, hi;
        or_mp_bounds(f[0], f[1], f[2], f[3], f[4], t & 1, (t & 2) ? 4.0 : 2.0, &lo, &hi);
        CHECK(lo <= f[2] && f[2] <= hi);
        (void)or_tvd5(f[0], f[1], f[2], f[3], f[4]);
        (void)or_van_albada(f[1], f[2], f[3]);
        (void)or_tvd_minmod(f[1], f[2], f[3]);
        (void)or_median(f[0], f[1], f[2]);
        (void)or_minmod4(f[0], f[1], f[2], f[3]);
        static const int schemes[3] = {6, 8, 8 | OR_SCHEME_ADAPTIVE};
        or_trace tr;
        double out = or_teno_m(schemes[t % 3], t % 9, (t % 9) ? 1e-5 : 0.1, f, &tr);
        CHECK(isfinite(out) && tr.status == 0);
    }
    /* degenerate slopes of the TVD-type fluxes */
    CHECK(or_tvd5(1.0, 1.0, 1.0, 2.0, 3.0) == 1.0);
    CHECK(or_van_albada(1.0, 1.0, 2.0) == 1.0);
    /* the non-finite gamma sum is reported */
    {
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 1e12};
        or_trace tr;
        CHECK(isnan(or_teno_m(6, OR_LIM_MP, 1e-5, v, &tr)) && tr.status == OR_ENONFINITE);
        or_grid g;
        memset(&g, 0, sizeof(g));
        g.ndim = 1;
        g.n[0] = 12;
        g.dx[0] = 0.1;
        g.bc[0] = 1;
        g.adv[0] = 1.0;
        double U[12] = {0}, F[13];
        U[10] = U[11] = 1e12;
        CHECK(or_reconstruct_faces(&g, 6, OR_LIM_MP, 1e-5, 1.4, 0, U, F, NULL, NULL) == OR_ENONFINITE);
    }
    /* invalid arguments */
    {
        or_trace tr;
        double v[8] = {0};
        CHECK(isnan(or_teno_m(7, OR_LIM_MP, 1e-5, v, &tr)));
        CHECK(isnan(or_teno_m(6 | OR_SCHEME_ADAPTIVE, OR_LIM_MP, 1e-5, v, &tr)));
        CHECK(isnan(or_teno_m(6, 42, 1e-5, v, &tr)));
        or_grid g;
        memset(&g, 0, sizeof(g));
        g.ndim = 4;
        CHECK(or_reconstruct_faces(&g, 6, 1, 1e-5, 1.4, 0, v, v, NULL, NULL) == -1);
        g.ndim = 1;
        g.n[0] = 8;
        g.dx[0] = 1.0;
        g.system = 1;
        CHECK(or_reconstruct_faces(&g, 6, 1, 1e-5, 1.4, 1, v, v, NULL, NULL) == -1);
        CHECK(or_rk3_step(&g, 5, 1, 1e-5, 1.4, 0.1, v) == -2);
    }
    /* Roe eigenvectors: L R = I */
    for (int nd = 1; nd <= 3; nd++)
        for (int ax = 0; ax < nd; ax++) {
            double UL[5] = {1.0, 0.1, -0.2, 0.05, 2.7}, UR[5] = {0.5, -0.05, 0.1, 0.2, 1.9};
            UL[nd + 1] = 2.7;
            UR[nd + 1] = 1.9;
            double R[25], L[25];
            CHECK(or_roe_eigenvectors(nd, 1.4, ax, UL, UR, R, L) == 0);
            int nf = nd + 2;
            for (int i = 0; i < nf; i++)
                for (int j = 0; j < nf; j++) {
                    double s = 0.0;
                    for (int k = 0; k < nf; k++) s += L[i * nf + k] * R[k * nf + j];
                    CHECK(fabs(s - (i == j)) < 1e-12);
                }
        }
    /* whole grids: every scheme, limiter, system, dimension count and
     * boundary pattern */
    static const int schemes[3] = {6, 8, 8 | OR_SCHEME_ADAPTIVE};
    for (int nd = 1; nd <= 3; nd++)
        for (int sys = 0; sys <= 1; sys++)
            for (int s = 0; s < 3; s++)
                for (int lim = 0; lim <= 8; lim++) {
                    if (nd >= 2 && (lim % 3) != s) continue; /* keep the run short */
                    run_grid(nd, sys, (lim + s) & 1, schemes[s], lim);
                }
    if (g_fail) return 1;
    printf("sanitized oracle run: ok\n");
    return 0;
}
