/*
 * Plain FP64 CPU oracle of the TENO-M per-face reconstruction (Li, Fu &
 * Adams, "A low-dissipation shock-capturing framework with flexible
 * nonlinear dissipation control", arXiv 2010.13289).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product path
 * (the HIP library) never calls it, and the two share no code, header or
 * constant table: every constant below is either printed in the paper
 * (Table 1, the parameters of Sec. 2-3) or derived here at start-up from the
 * paper's definitions.
 *
 * The code follows the paper's steps in its order and notation and is meant
 * to be read against it; it is deliberately slow (no blocking, no fusion,
 * IEEE division and sqrt everywhere, pow() for the q-th power).  Build with
 * -O2 -ffp-contract=off so that no multiply-add contraction happens.
 *
 * Readings where the paper is silent or ambiguous (each one is also listed
 * in the design notes of the repository):
 *  - optimal weights d_k: the maximum-order weights, obtained by matching
 *    the K-point linear reconstruction on the full stencil (Sec. 3.3 leaves
 *    the choice open);
 *  - stencil widths for K = 8 follow Table 1 (S0..S5 with 3,3,3,4,4,5
 *    points), where the general width formula of Sec. 2.1 is garbled;
 *  - beta_K is the Jiang-Shu measure (Sec. 2.2) of the degree K-1 polynomial
 *    on the full K-point stencil; tau uses the central 3-point stencil S0
 *    with weight 4 as printed (Eq. taukTENO);
 *  - chi_k == C_T counts as smooth (Eq. cut-off: 0 only if chi < C_T);
 *  - MP limiter: bounds once per face, applied to each nonsmooth candidate
 *    (Sec. 3.2.3); TVD-type limiters: one limited flux on the fixed stencil
 *    centred at i replaces every nonsmooth candidate (Sec. 3.2.3);
 *  - "TVD (minmod)": Eq. TVDbeta with phi(r) = max(0, min(1, r)), i.e.
 *    f_i + minmod(delta-, delta+)/2;
 *  - TVD5 / Van Albada slope ratios: the literal formulas wherever their
 *    denominators are nonzero, otherwise their continuous limit (the slope
 *    term vanishes with delta- since phi is bounded);
 *  - Rusanov splitting: one alpha per face, the maximum of |u_n| + c over
 *    the K stencil cells (scalar advection: |a|);
 *  - the f- side is the mirror image of the f+ side about the face;
 *  - transmissive boundaries clamp cell indices (zero-gradient ghosts).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Parameters printed in the paper                                           */
/* ------------------------------------------------------------------------ */

/* Eq. measureTENO: gamma_k = (C + tau_K / (beta_k + eps))^q */
static const double OR_C = 1.0;
static const double OR_Q = 6.0;
static const double OR_EPS = 1e-40;

/* Eq. upper_limiter: alpha = 1.25; Eq. large_curvature: beta = 4 (the
 * recommended value; Secs. 4.2.5 and 4.4 also run beta = 2 and 1) */
static const double OR_MP_ALPHA = 1.25;
static const double OR_MP_BETA = 4.0;
/* Eq. high order TVD: alpha = 2 */
static const double OR_TVD5_ALPHA = 2.0;
/* Sec. 3.2.1: kappa = 1/3 restores third order for the Van Albada flux */
static const double OR_VA_KAPPA = 1.0 / 3.0;

/* Sec. 2.4 (adaptive cutoff of the eight-point schemes): Ren-type indicator
 * with xi = 1e-3, C_r = 0.23 (Eq. shock_indicator), alpha_1 = 10.5,
 * alpha_2 = 3.5 (Eq. cut-off_adjust). */
static const double OR_REN_XI = 1e-3;
static const double OR_REN_CR = 0.23;
static const double OR_ADAPT_A1 = 10.5;
static const double OR_ADAPT_A2 = 3.5;

/* Relative width of the cutoff band reported next to the flags. */
static const double OR_BAND = 1e-10;

/* Status of a reconstruction whose gamma sum is not finite (Eq. normalize
 * is then undefined); the whole-grid entry points return it as well. */
#define OR_ENONFINITE (-5)

/* The printed constants by name, so that a test can hold them against the
 * paper's text; NaN for an unknown name. */
double or_param(const char* name) {
    const struct { const char* name; double value; } tab[] = {
        {"C", OR_C},
        {"q", OR_Q},
        {"epsilon", OR_EPS},
        {"mp_alpha", OR_MP_ALPHA},
        {"mp_beta", OR_MP_BETA},
        {"tvd5_alpha", OR_TVD5_ALPHA},
        {"va_kappa", OR_VA_KAPPA},
        {"ren_xi", OR_REN_XI},
        {"ren_cr", OR_REN_CR},
        {"adapt_alpha1", OR_ADAPT_A1},
        {"adapt_alpha2", OR_ADAPT_A2},
    };
    for (size_t i = 0; i < sizeof(tab) / sizeof(tab[0]); i++)
        if (strcmp(tab[i].name, name) == 0) return tab[i].value;
    return NAN;
}

/* Scheme identifiers: the number of points K, optionally with the adaptive
 * cutoff flag (the eight-point TENO8A scheme of Sec. 2.4). */
#define OR_SCHEME_ADAPTIVE 0x100

/* Table 1: f_k = sum_m c_m f_m, columns c_{i-3} .. c_{i+4}.  Stored as the
 * printed numerators over the printed denominators. */
static const int TAB1_NUM[6][8] = {
    /*        i-3  i-2  i-1    i  i+1  i+2  i+3  i+4 */
    /* k=0 */ {0, 0, -1, 5, 2, 0, 0, 0},
    /* k=1 */ {0, 0, 0, 2, 5, -1, 0, 0},
    /* k=2 */ {0, 2, -7, 11, 0, 0, 0, 0},
    /* k=3 */ {0, 0, 0, 3, 13, -5, 1, 0},
    /* k=4 */ {-3, 13, -23, 25, 0, 0, 0, 0},
    /* k=5 */ {0, 0, 0, 12, 77, -43, 17, -3},
};
static const int TAB1_DEN[6] = {6, 6, 6, 12, 12, 60};
/* point range [lo, hi] of candidate S_k relative to i (Fig. 1 / Table 1) */
static const int CAND_LO[6] = {-1, 0, -2, 0, -3, 0};
static const int CAND_HI[6] = {1, 2, 0, 3, 0, 4};

/* ------------------------------------------------------------------------ */
/* Limiter identifiers (the oracle's own numbering)                         */
/* ------------------------------------------------------------------------ */
enum {
    OR_LIM_TENO = 0,      /* classic TENO: discard nonsmooth, renormalise */
    OR_LIM_MP = 1,        /* MP, d^M4, beta = 4 */
    OR_LIM_TVD_MINMOD = 2,
    OR_LIM_TVD5 = 3,
    OR_LIM_VA = 4,
    OR_LIM_MP_M4_B2 = 5,  /* MP, d^M4, beta = 2 */
    OR_LIM_MP_MM_B4 = 6,  /* MP, d^MM, beta = 4 */
    OR_LIM_MP_MM_B2 = 7,  /* MP, d^MM, beta = 2 */
    OR_LIM_MP_MM_B1 = 8,  /* MP, d^MM, beta = 1 */
};

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra (Gauss-Jordan with partial pivoting)          */
/* ------------------------------------------------------------------------ */

/* Invert the n x n matrix a (row-major, n <= 8) into inv.  Returns 0, or -1
 * if a pivot vanishes.  The elimination runs in long double so that the
 * derived tables are accurate to the last bit of a double. */
static int or_invert_ld(int n, const long double* a, long double* inv) {
    long double m[8][16];
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < n; j++) {
            m[i][j] = a[i * n + j];
            m[i][n + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
                if (fabsl(m[r][c]) > fabsl(m[p][c])) p = r;
        if (m[p][c] == 0.0L) return -1;
        if (p != c)
            for (int j = 0; j < 2 * n; j++) {
                long double t = m[c][j];
                m[c][j] = m[p][j];
                m[p][j] = t;
            }
        long double piv = m[c][c];
        for (int j = 0; j < 2 * n; j++) m[c][j] /= piv;
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            long double f = m[r][c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; j++) m[r][j] -= f * m[c][j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) inv[i * n + j] = m[i][n + j];
    return 0;
}

static int or_invert(int n, const double* a, double* inv) {
    long double al[64] = {0}, il[64];
    for (int i = 0; i < n * n; i++) al[i] = a[i];
    if (or_invert_ld(n, al, il) != 0) return -1;
    for (int i = 0; i < n * n; i++) inv[i] = (double)il[i];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Polynomial reconstruction on a stencil (Sec. 2, Eqs. definitionEq and     */
/* approximatepolynomial)                                                    */
/* ------------------------------------------------------------------------ */

/* A stencil [lo, hi] of r = hi - lo + 1 points around cell i.  With
 * xi = (x - x_i)/dx the candidate polynomial is p(xi) = sum_l a_l xi^l, and
 * its averages over the cells [m - 1/2, m + 1/2] equal the point values v_m
 * (Eq. definitionEq).  ainv maps v to a; dmap maps the differences
 * D_j = v_{lo+j+1} - v_{lo+j} to a_1..a_{r-1} (a constant shift of v only
 * moves a_0, so the derivatives of p see differences only).  face holds the
 * coefficients of p(1/2) on v: the linear reconstruction at x_{i+1/2}. */
typedef struct {
    int lo, hi, r;
    double ainv[8][8];
    double dmap[8][8];
    double face[8];
    long double face_ld[8];
} or_poly;

static int or_poly_init(or_poly* s, int lo, int hi) {
    int r = hi - lo + 1;
    long double A[64] = {0}, inv[64];
    s->lo = lo;
    s->hi = hi;
    s->r = r;
    for (int row = 0; row < r; row++) {
        long double m = (long double)(lo + row);
        for (int l = 0; l < r; l++) {
            /* integral of xi^l over [m-1/2, m+1/2] */
            A[row * r + l] = (powl(m + 0.5L, l + 1) - powl(m - 0.5L, l + 1)) / (long double)(l + 1);
        }
    }
    if (or_invert_ld(r, A, inv) != 0) return -1;
    for (int l = 0; l < r; l++)
        for (int j = 0; j < r; j++) s->ainv[l][j] = (double)inv[l * r + j];
    /* a_l = sum_m ainv[l][m] v_m,  v_m = v_lo + sum_{j < m-lo} D_j
     *     => a_l = sum_j D_j sum_{m > j} ainv[l][m]   (l >= 1) */
    for (int l = 0; l < r; l++)
        for (int j = 0; j < r - 1; j++) {
            long double acc = 0.0L;
            for (int m = j + 1; m < r; m++) acc += inv[l * r + m];
            s->dmap[l][j] = (double)acc;
        }
    for (int j = 0; j < r; j++) {
        long double acc = 0.0L;
        for (int l = 0; l < r; l++) acc += inv[l * r + j] * powl(0.5L, l);
        s->face[j] = (double)acc;
        s->face_ld[j] = acc;
    }
    return 0;
}

/* Eq. measureTENO (second form): beta = sum_{j=1}^{r-1} dx^{2j-1}
 * int_{x_{i-1/2}}^{x_{i+1/2}} (d^j p / dx^j)^2 dx.  In xi = (x - x_i)/dx the
 * powers of dx cancel: beta = sum_j int_{-1/2}^{1/2} (p^{(j)}(xi))^2 dxi.
 * vs[0..r-1] are the values on [lo, hi]. */
static double or_beta(const or_poly* s, const double* vs) {
    int r = s->r;
    double D[8], a[8];
    for (int j = 0; j < r - 1; j++) D[j] = vs[j + 1] - vs[j];
    a[0] = 0.0; /* never used: no derivative sees a_0 */
    for (int l = 1; l < r; l++) {
        double acc = 0.0;
        for (int j = 0; j < r - 1; j++) acc += s->dmap[l][j] * D[j];
        a[l] = acc;
    }
    double beta = 0.0;
    for (int j = 1; j < r; j++) {
        /* p^{(j)}(xi) = sum_e c_e xi^e with c_e = a_{e+j} (e+j)!/e! */
        double c[8];
        int deg = r - 1 - j;
        for (int e = 0; e <= deg; e++) {
            double ff = 1.0;
            for (int t = e + 1; t <= e + j; t++) ff *= (double)t;
            c[e] = a[e + j] * ff;
        }
        double integral = 0.0;
        for (int e1 = 0; e1 <= deg; e1++)
            for (int e2 = 0; e2 <= deg; e2++) {
                int e = e1 + e2;
                if (e % 2) continue; /* odd moments of [-1/2, 1/2] vanish */
                integral += c[e1] * c[e2] * 2.0 * pow(0.5, e + 1) / (double)(e + 1);
            }
        beta += integral;
    }
    return beta;
}

/* ------------------------------------------------------------------------ */
/* Derived tables: filled once by or_init()                                  */
/* ------------------------------------------------------------------------ */
static or_poly g_cand[6];     /* the candidate stencils S0..S5 */
static or_poly g_full[2];     /* full stencils: K=6 [-2,3], K=8 [-3,4] */
static double g_d[2][6];      /* optimal weights d_k for K = 6, 8 */
static double g_tab1[6][8];   /* Table 1 as doubles */
static int g_ready = 0;

static int full_lo(int K) { return -(K / 2) + 1; }
static int full_hi(int K) { return K / 2; }

/* Optimal (maximum-order) weights: sum_k d_k c_{k,m} = full-stencil linear
 * coefficient at m, for every m of the K-point stencil (K equations in K-2
 * unknowns, consistent).  Gaussian elimination with the pivot row chosen
 * among all remaining equations; the equations left over must then hold. */
static int or_derive_weights(int K, double* d) {
    int nk = K - 2, lo = full_lo(K);
    const or_poly* F = &g_full[K == 6 ? 0 : 1];
    long double M[8][7], dl[6];
    for (int m = 0; m < K; m++) {
        int off = lo + m; /* offset relative to i */
        for (int k = 0; k < nk; k++)
            M[m][k] = (long double)TAB1_NUM[k][off + 3] / (long double)TAB1_DEN[k];
        M[m][nk] = F->face_ld[m];
    }
    for (int c = 0; c < nk; c++) {
        int p = c;
        for (int r = c + 1; r < K; r++)
            if (fabsl(M[r][c]) > fabsl(M[p][c])) p = r;
        if (M[p][c] == 0.0L) return -1;
        for (int j = 0; j <= nk; j++) {
            long double t = M[c][j];
            M[c][j] = M[p][j];
            M[p][j] = t;
        }
        for (int r = c + 1; r < K; r++) {
            long double f = M[r][c] / M[c][c];
            for (int j = c; j <= nk; j++) M[r][j] -= f * M[c][j];
        }
    }
    for (int c = nk - 1; c >= 0; c--) {
        long double acc = M[c][nk];
        for (int j = c + 1; j < nk; j++) acc -= M[c][j] * dl[j];
        dl[c] = acc / M[c][c];
    }
    /* the system must be consistent: the eliminated rows must vanish */
    for (int r = nk; r < K; r++)
        if (fabsl(M[r][nk]) > 1e-14L) return -2;
    for (int c = 0; c < nk; c++) d[c] = (double)dl[c];
    return 0;
}

int or_init(void) {
    if (g_ready) return 0;
    for (int k = 0; k < 6; k++) {
        for (int c = 0; c < 8; c++) g_tab1[k][c] = (double)TAB1_NUM[k][c] / (double)TAB1_DEN[k];
        if (or_poly_init(&g_cand[k], CAND_LO[k], CAND_HI[k]) != 0) return -1;
    }
    if (or_poly_init(&g_full[0], full_lo(6), full_hi(6)) != 0) return -1;
    if (or_poly_init(&g_full[1], full_lo(8), full_hi(8)) != 0) return -1;
    if (or_derive_weights(6, g_d[0]) != 0) return -2;
    if (or_derive_weights(8, g_d[1]) != 0) return -2;
    g_ready = 1;
    return 0;
}

/* Accessors used by the pin tests. */
int or_get_weights(int K, double* d) {
    if (or_init() != 0 || (K != 6 && K != 8)) return -1;
    for (int k = 0; k < K - 2; k++) d[k] = g_d[K == 6 ? 0 : 1][k];
    return 0;
}

/* Linear face-value coefficients of the polynomial through the averages on
 * [lo, hi] (relative to i), evaluated at x_{i+1/2}. */
int or_get_poly_face(int lo, int hi, double* coef) {
    or_poly s;
    if (hi < lo || hi - lo + 1 > 8) return -1;
    if (or_poly_init(&s, lo, hi) != 0) return -1;
    for (int j = 0; j < s.r; j++) coef[j] = s.face[j];
    return 0;
}

/* beta of the polynomial through the r values vs on [lo, hi]. */
double or_beta_stencil(int lo, int hi, const double* vs) {
    or_poly s;
    if (hi < lo || hi - lo + 1 > 8 || or_poly_init(&s, lo, hi) != 0) return NAN;
    return or_beta(&s, vs);
}

/* ------------------------------------------------------------------------ */
/* Limiter building blocks (Sec. 3.2)                                        */
/* ------------------------------------------------------------------------ */

static double or_sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

/* Eq. minmod222 */
double or_minmod2(double x, double y) {
    return 0.5 * (or_sgn(x) + or_sgn(y)) * fmin(fabs(x), fabs(y));
}

/* Eq. minmod444 */
double or_minmod4(double a, double b, double c, double d) {
    return 0.125 * (or_sgn(a) + or_sgn(b)) *
           fabs((or_sgn(a) + or_sgn(c)) * (or_sgn(a) + or_sgn(d))) *
           fmin(fmin(fabs(a), fabs(b)), fmin(fabs(c), fabs(d)));
}

/* Eq. median */
double or_median(double x, double y, double z) { return x + or_minmod2(y - x, z - x); }

/* MP bounds of Sec. 3.2.2 at x_{i+1/2} from f_{i-2..i+2} (fm2..fp2).
 * curv: 0 = d^M4 (Eq. maximal_curvature), 1 = d^MM (Eq. maximal_curvature1);
 * bet is the beta of Eq. large_curvature. */
void or_mp_bounds(double fm2, double fm1, double f0, double fp1, double fp2, int curv,
                  double bet, double* fmin_out, double* fmax_out) {
    /* Eq. curvature */
    double d_im1 = f0 - 2.0 * fm1 + fm2;
    double d_i = fp1 - 2.0 * f0 + fm1;
    double d_ip1 = fp2 - 2.0 * fp1 + f0;
    double d_iph, d_imh;
    if (curv == 0) {
        d_iph = or_minmod4(4.0 * d_i - d_ip1, 4.0 * d_ip1 - d_i, d_i, d_ip1);
        d_imh = or_minmod4(4.0 * d_im1 - d_i, 4.0 * d_i - d_im1, d_im1, d_i);
    } else {
        d_iph = or_minmod2(d_i, d_ip1);
        d_imh = or_minmod2(d_im1, d_i);
    }
    /* Eq. upper_limiter */
    double f_ul = f0 + OR_MP_ALPHA * (f0 - fm1);
    /* Eq. median_value */
    double f_md = 0.5 * (f0 + fp1) - 0.5 * d_iph;
    /* Eq. large_curvature */
    double f_lc = f0 + 0.5 * (f0 - fm1) + (bet / 3.0) * d_imh;
    /* Eq. value_min_max */
    double f_lo = fmax(fmin(fmin(f0, fp1), f_md), fmin(fmin(f0, f_ul), f_lc));
    double f_hi = fmin(fmax(fmax(f0, fp1), f_md), fmax(fmax(f0, f_ul), f_lc));
    *fmin_out = f_lo;
    *fmax_out = f_hi;
}

/* TVD flux on the fixed stencil centred at i (Sec. 3.2.1). */
double or_tvd_minmod(double fm1, double f0, double fp1) {
    /* Eq. TVDbeta with phi = max(0, min(1, r)): f_i + minmod(d-, d+)/2 */
    return f0 + 0.5 * or_minmod2(f0 - fm1, fp1 - f0);
}

double or_tvd5(double fm2, double fm1, double f0, double fp1, double fp2) {
    double dm = f0 - fm1;   /* delta^- at i */
    double dp = fp1 - f0;   /* delta^+ at i */
    double dmm = fm1 - fm2; /* delta^- at i-1 */
    double dpp = fp2 - fp1; /* delta^+ at i+1 */
    if (dm != 0.0 && dp != 0.0 && dmm != 0.0) {
        /* Eq. slop_ratio at i-1, i, i+1 */
        double r_jm1 = dm / dmm;
        double r_j = dp / dm;
        double r_jp1 = dpp / dp;
        /* Eq. TVDhighorder2 */
        double beta = (-2.0 / r_jm1 + 11.0 + 24.0 * r_j - 3.0 * r_j * r_jp1) / 30.0;
        /* Eq. high order TVD */
        double phi = fmax(0.0, fmin(fmin(OR_TVD5_ALPHA, OR_TVD5_ALPHA * r_j), beta));
        /* Eq. TVDbeta */
        return f0 + 0.5 * phi * dm;
    }
    if (dm == 0.0) return f0; /* phi is bounded, the slope term vanishes */
    /* one of r_{j-1}, r_{j+1} is degenerate: continuous limit of phi * dm */
    double B = (-2.0 * dmm + 11.0 * dm + 24.0 * dp - 3.0 * dpp) / 30.0;
    double s;
    if (dm > 0.0)
        s = fmax(0.0, fmin(fmin(OR_TVD5_ALPHA * dm, OR_TVD5_ALPHA * dp), B));
    else
        s = fmin(0.0, fmax(fmax(OR_TVD5_ALPHA * dm, OR_TVD5_ALPHA * dp), B));
    return f0 + 0.5 * s;
}

double or_van_albada(double fm1, double f0, double fp1) {
    double dm = f0 - fm1, dp = fp1 - f0;
    double phi = 0.0;
    if (dm != 0.0) {
        double r = dp / dm;                 /* Eq. slop_ratio */
        phi = 2.0 * r / (r * r + 1.0);      /* Eq. van_Albada_limiter */
    }
    /* Eq. vAflux */
    return f0 + 0.25 * phi * ((1.0 - OR_VA_KAPPA * phi) * dm + (1.0 + OR_VA_KAPPA * phi) * dp);
}

/* ------------------------------------------------------------------------ */
/* One TENO-M reconstruction: one face, one component, the + orientation     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double cand[6];  /* candidate fluxes f_k (Table 1) */
    double beta[6];  /* beta_{k,r} */
    double betaK;    /* beta on the full stencil */
    double tau;      /* Eq. taukTENO */
    double gam[6];   /* Eq. measureTENO */
    double chi[6];   /* Eq. normalize */
    int delta[6];    /* Eq. cut-off */
    int band[6];     /* |chi/C_T - 1| <= 1e-10 */
    double fmin, fmax; /* MP bounds */
    double ftvd;     /* TVD-type flux on the fixed stencil */
    double fM[6];    /* Eq. mp_flux */
    double out;
    double eta;      /* adaptive cutoff: eta_{i+1/2} of Eq. shock_indicator */
    double m;        /* adaptive cutoff: m */
    double ct;       /* the C_T actually used */
    int ct_band;     /* adaptive cutoff: beta within 1e-10 of an integer */
    int status;      /* 0, or OR_ENONFINITE when sum_k gamma_k is not finite */
} or_trace;

/* Eqs. shock_indicator and cut-off_adjust: the cutoff of one face from
 * f_{i-2} .. f_{i+3} (fv points at f_i). */
static double or_adaptive_ct(const double* fv, or_trace* tr) {
    double eps = 0.9 * OR_REN_CR / (1.0 - 0.9 * OR_REN_CR) * OR_REN_XI * OR_REN_XI;
    double eta_face = 0.0;
    for (int j = -1; j <= 2; j++) {
        double dp = fv[j + 1] - fv[j]; /* Delta f_{j+1/2} */
        double dm = fv[j] - fv[j - 1]; /* Delta f_{j-1/2} */
        double eta = (fabs(2.0 * dp * dm) + eps) / (dp * dp + dm * dm + eps);
        eta_face = (j == -1) ? eta : fmin(eta_face, eta);
    }
    double m = 1.0 - fmin(1.0, eta_face / OR_REN_CR);
    double g = pow(1.0 - m, 4.0) * (1.0 + 4.0 * m);
    double beta = OR_ADAPT_A1 - OR_ADAPT_A2 * (1.0 - g);
    double fl = floor(beta);
    tr->eta = eta_face;
    tr->m = m;
    /* Rounding can move floor(beta) only where beta is close to one of the
     * interior integers 8, 9, 10: g lies in [0, 1], so beta >= alpha_1 -
     * alpha_2 = 7 holds exactly in any rounding and floor(beta) = 7 at the
     * bottom of the range. */
    double nb = nearbyint(beta);
    tr->ct_band = (nb >= 8.0 && nb <= 10.0 && fabs(beta - nb) <= 1e-10) ? 1 : 0;
    return pow(10.0, -fl);
}

/* v[0..K-1] hold f at i-K/2+1 .. i+K/2; the result approximates the flux at
 * x_{i+1/2}.  `scheme` is K, or 8 | OR_SCHEME_ADAPTIVE for the adaptive
 * cutoff of Sec. 2.4 (C_T is then ignored). */
double or_teno_m(int scheme, int lim, double C_T, const double* v, or_trace* tr) {
    or_trace loc;
    if (!tr) tr = &loc;
    memset(tr, 0, sizeof(*tr));
    int K = scheme & 0xff;
    int adaptive = (scheme & OR_SCHEME_ADAPTIVE) != 0;
    if (or_init() != 0 || (K != 6 && K != 8) || (adaptive && K != 8)) return NAN;
    if (adaptive) C_T = or_adaptive_ct(v + K / 2 - 1, tr);
    tr->ct = C_T;
    int nk = K - 2;
    int c0 = K / 2 - 1; /* index of f_i in v */
    const double* dk = g_d[K == 6 ? 0 : 1];

    /* Sec. 3.1, Table 1: candidate fluxes */
    for (int k = 0; k < nk; k++) {
        double acc = 0.0;
        for (int off = CAND_LO[k]; off <= CAND_HI[k]; off++) acc += g_tab1[k][off + 3] * v[c0 + off];
        tr->cand[k] = acc;
    }
    /* Eq. measureTENO: smoothness indicators of the candidates */
    for (int k = 0; k < nk; k++) tr->beta[k] = or_beta(&g_cand[k], v + c0 + CAND_LO[k]);
    /* ... and of the full stencil */
    tr->betaK = or_beta(&g_full[K == 6 ? 0 : 1], v);
    /* Eq. taukTENO */
    tr->tau = fabs(tr->betaK - (tr->beta[1] + tr->beta[2] + 4.0 * tr->beta[0]) / 6.0);
    /* Eq. measureTENO */
    double sum = 0.0;
    for (int k = 0; k < nk; k++) {
        tr->gam[k] = pow(OR_C + tr->tau / (tr->beta[k] + OR_EPS), OR_Q);
        sum += tr->gam[k];
    }
    /* The literal gamma_k overflows once tau / (beta_k + eps) exceeds about
     * 1e51 (a jump of about 1e6 beside exactly constant data); chi_k is then
     * undefined, so the reconstruction reports it instead of guessing. */
    if (!isfinite(sum)) {
        tr->status = OR_ENONFINITE;
        tr->out = NAN;
        return NAN;
    }
    /* Eq. normalize and Eq. cut-off */
    for (int k = 0; k < nk; k++) {
        tr->chi[k] = tr->gam[k] / sum;
        tr->delta[k] = (tr->chi[k] < C_T) ? 0 : 1;
        tr->band[k] = (C_T > 0.0 && fabs(tr->chi[k] / C_T - 1.0) <= OR_BAND) ? 1 : 0;
    }

    double fm2 = v[c0 - 2], fm1 = v[c0 - 1], f0 = v[c0], fp1 = v[c0 + 1], fp2 = v[c0 + 2];
    if (lim == OR_LIM_TENO) {
        /* Eq. weight_renormalize and the first Eq. reconstuction */
        double den = 0.0, acc = 0.0;
        for (int k = 0; k < nk; k++) den += dk[k] * tr->delta[k];
        for (int k = 0; k < nk; k++) {
            tr->fM[k] = tr->cand[k];
            acc += (dk[k] * tr->delta[k] / den) * tr->cand[k];
        }
        tr->out = acc;
        return acc;
    }
    int is_mp = (lim == OR_LIM_MP || (lim >= OR_LIM_MP_M4_B2 && lim <= OR_LIM_MP_MM_B1));
    if (is_mp) {
        int curv = (lim == OR_LIM_MP || lim == OR_LIM_MP_M4_B2) ? 0 : 1;
        double bet = (lim == OR_LIM_MP || lim == OR_LIM_MP_MM_B4) ? OR_MP_BETA
                     : (lim == OR_LIM_MP_MM_B1) ? 1.0 : 2.0;
        or_mp_bounds(fm2, fm1, f0, fp1, fp2, curv, bet, &tr->fmin, &tr->fmax);
    } else if (lim == OR_LIM_TVD_MINMOD) {
        tr->ftvd = or_tvd_minmod(fm1, f0, fp1);
    } else if (lim == OR_LIM_TVD5) {
        tr->ftvd = or_tvd5(fm2, fm1, f0, fp1, fp2);
    } else if (lim == OR_LIM_VA) {
        tr->ftvd = or_van_albada(fm1, f0, fp1);
    } else {
        return NAN;
    }
    /* Eq. mp_flux, then Eq. reconstuction with w_k = d_k */
    double acc = 0.0;
    for (int k = 0; k < nk; k++) {
        double flim;
        if (is_mp)
            flim = or_median(tr->cand[k], tr->fmin, tr->fmax); /* Eq. value_monotonicity_preserving */
        else
            flim = tr->ftvd;
        tr->fM[k] = tr->delta[k] ? tr->cand[k] : flim;
        acc += dk[k] * tr->fM[k];
    }
    tr->out = acc;
    return acc;
}

/* Flat-array view of a trace for the Python tests. */
int or_trace_size(void) { return (int)sizeof(or_trace); }

/* ------------------------------------------------------------------------ */
/* Grid, state access and boundary conditions                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t ndim;
    int32_t n[3];
    double dx[3];
    int32_t bc[3];     /* 0 periodic, 1 transmissive */
    int32_t system;    /* 0 scalar advection, 1 Euler */
    double adv[3];     /* advection velocity (scalar system) */
} or_grid;

static int or_nfields(const or_grid* g) { return g->system == 0 ? 1 : g->ndim + 2; }
static size_t or_ncells(const or_grid* g) {
    size_t c = 1;
    for (int d = 0; d < g->ndim; d++) c *= (size_t)g->n[d];
    return c;
}

/* Map an unwrapped coordinate into [0, n) by the boundary rule. */
static int or_bc_index(int i, int n, int bc) {
    if (bc == 0) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* A readable state: either the whole grid (coordinates are wrapped or
 * clamped) or a box of precomputed cells addressed by unwrapped coordinates
 * relative to an origin. */
typedef struct {
    const or_grid* g;
    const double* base;
    int is_box;
    int org[3];
    int bn[3];
} or_state;

static double or_get(const or_state* s, int f, const int* p) {
    const or_grid* g = s->g;
    if (!s->is_box) {
        size_t idx = 0, stride = 1;
        for (int d = 0; d < g->ndim; d++) {
            idx += (size_t)or_bc_index(p[d], g->n[d], g->bc[d]) * stride;
            stride *= (size_t)g->n[d];
        }
        return s->base[(size_t)f * or_ncells(g) + idx];
    }
    size_t idx = 0, stride = 1, tot = 1;
    for (int d = 0; d < g->ndim; d++) tot *= (size_t)s->bn[d];
    for (int d = 0; d < g->ndim; d++) {
        int l = p[d] - s->org[d];
        idx += (size_t)l * stride;
        stride *= (size_t)s->bn[d];
    }
    return s->base[(size_t)f * tot + idx];
}

/* ------------------------------------------------------------------------ */
/* Euler equations: fluxes and Roe-average eigenvectors (Sec. 4)             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int K, lim;
    double C_T, gamma;
} or_scheme;

/* Physical flux along axis `ax` and the signal speed |u_n| + c of one cell. */
static void or_euler_flux(int ndim, double gamma, int ax, const double* U, double* F, double* lam) {
    double rho = U[0], E = U[ndim + 1];
    double vel[3] = {0, 0, 0}, q2 = 0.0;
    for (int d = 0; d < ndim; d++) {
        vel[d] = U[1 + d] / rho;
        q2 += vel[d] * vel[d];
    }
    double p = (gamma - 1.0) * (E - 0.5 * rho * q2);
    double un = vel[ax];
    F[0] = rho * un;
    for (int d = 0; d < ndim; d++) F[1 + d] = rho * vel[d] * un + (d == ax ? p : 0.0);
    F[ndim + 1] = (E + p) * un;
    double c = sqrt(gamma * p / rho);
    *lam = fabs(un) + c;
}

/* Right eigenvectors of the flux Jacobian along `ax` at the Roe average of
 * the states UL, UR (columns: u_n - c, entropy, shear waves, u_n + c). */
static void or_roe_right(int ndim, double gamma, int ax, const double* UL, const double* UR, double* R) {
    int nf = ndim + 2;
    double rl = UL[0], rr = UR[0];
    double vl[3] = {0, 0, 0}, vr[3] = {0, 0, 0}, ql = 0.0, qr = 0.0;
    for (int d = 0; d < ndim; d++) {
        vl[d] = UL[1 + d] / rl;
        vr[d] = UR[1 + d] / rr;
        ql += vl[d] * vl[d];
        qr += vr[d] * vr[d];
    }
    double pl = (gamma - 1.0) * (UL[nf - 1] - 0.5 * rl * ql);
    double pr = (gamma - 1.0) * (UR[nf - 1] - 0.5 * rr * qr);
    double Hl = (UL[nf - 1] + pl) / rl, Hr = (UR[nf - 1] + pr) / rr;
    double sl = sqrt(rl), sr = sqrt(rr);
    double u[3] = {0, 0, 0}, q2 = 0.0;
    for (int d = 0; d < ndim; d++) {
        u[d] = (sl * vl[d] + sr * vr[d]) / (sl + sr);
        q2 += u[d] * u[d];
    }
    double H = (sl * Hl + sr * Hr) / (sl + sr);
    double c = sqrt((gamma - 1.0) * (H - 0.5 * q2));
    double un = u[ax];
    memset(R, 0, sizeof(double) * nf * nf);
    /* column 0: u_n - c */
    R[0 * nf + 0] = 1.0;
    for (int d = 0; d < ndim; d++) R[(1 + d) * nf + 0] = u[d] - (d == ax ? c : 0.0);
    R[(nf - 1) * nf + 0] = H - un * c;
    /* column 1: entropy wave */
    R[0 * nf + 1] = 1.0;
    for (int d = 0; d < ndim; d++) R[(1 + d) * nf + 1] = u[d];
    R[(nf - 1) * nf + 1] = 0.5 * q2;
    /* shear waves, one per tangential direction in increasing order */
    int col = 2;
    for (int t = 0; t < ndim; t++) {
        if (t == ax) continue;
        R[(1 + t) * nf + col] = 1.0;
        R[(nf - 1) * nf + col] = u[t];
        col++;
    }
    /* last column: u_n + c */
    R[0 * nf + nf - 1] = 1.0;
    for (int d = 0; d < ndim; d++) R[(1 + d) * nf + nf - 1] = u[d] + (d == ax ? c : 0.0);
    R[(nf - 1) * nf + nf - 1] = H + un * c;
}

int or_roe_eigenvectors(int ndim, double gamma, int ax, const double* UL, const double* UR,
                        double* R, double* L) {
    int nf = ndim + 2;
    or_roe_right(ndim, gamma, ax, UL, UR, R);
    return or_invert(nf, R, L);
}

/* Numerical flux at the face between cell p and p + e_ax (all fields),
 * evaluated on the state s.  flags/band (nullable) receive, per side
 * (0 = +, 1 = -) and component, the bit mask of delta_k / band hits. */
static int or_face_flux(const or_grid* g, const or_scheme* sc, const or_state* s, int ax, const int* p,
                        double* Fout, uint8_t* flags, uint8_t* band) {
    int K = sc->K & 0xff, h = K / 2, nf = or_nfields(g);
    double Uc[8][5], Fc[8][5], lam[8];
    for (int m = 0; m < K; m++) {
        int q[3] = {p[0], p[1], p[2]};
        q[ax] += m - h + 1; /* cells i-K/2+1 .. i+K/2 */
        for (int f = 0; f < nf; f++) Uc[m][f] = or_get(s, f, q);
    }
    double gp[5][8], gm[5][8];
    double R[25], L[25];
    if (g->system == 0) {
        double a = g->adv[ax], alpha = fabs(a);
        for (int m = 0; m < K; m++) {
            double u = Uc[m][0], f = a * u;
            gp[0][m] = 0.5 * (f + alpha * u); /* Rusanov splitting */
            gm[0][m] = 0.5 * (f - alpha * u);
        }
    } else {
        double alpha = 0.0;
        for (int m = 0; m < K; m++) {
            or_euler_flux(g->ndim, sc->gamma, ax, Uc[m], Fc[m], &lam[m]);
            if (lam[m] > alpha) alpha = lam[m];
        }
        if (or_roe_eigenvectors(g->ndim, sc->gamma, ax, Uc[h - 1], Uc[h], R, L) != 0) return -1;
        for (int c = 0; c < nf; c++)
            for (int m = 0; m < K; m++) {
                double w = 0.0, gg = 0.0;
                for (int r = 0; r < nf; r++) {
                    w += L[c * nf + r] * Uc[m][r];
                    gg += L[c * nf + r] * Fc[m][r];
                }
                gp[c][m] = 0.5 * (gg + alpha * w);
                gm[c][m] = 0.5 * (gg - alpha * w);
            }
    }
    double fc[5];
    for (int c = 0; c < nf; c++) {
        or_trace tp, tm;
        double mir[8];
        for (int m = 0; m < K; m++) mir[m] = gm[c][K - 1 - m];
        double fplus = or_teno_m(sc->K, sc->lim, sc->C_T, gp[c], &tp);
        double fminus = or_teno_m(sc->K, sc->lim, sc->C_T, mir, &tm);
        if (tp.status || tm.status) return OR_ENONFINITE;
        fc[c] = fplus + fminus;
        if (flags || band) {
            uint8_t bp = 0, bm = 0, np = 0, nm = 0;
            for (int k = 0; k < K - 2; k++) {
                bp |= (uint8_t)(tp.delta[k] << k);
                bm |= (uint8_t)(tm.delta[k] << k);
                np |= (uint8_t)((tp.band[k] | tp.ct_band) << k);
                nm |= (uint8_t)((tm.band[k] | tm.ct_band) << k);
            }
            if (flags) {
                flags[c] = bp;
                flags[nf + c] = bm;
            }
            if (band) {
                band[c] = np;
                band[nf + c] = nm;
            }
        }
    }
    if (g->system == 0) {
        Fout[0] = fc[0];
    } else {
        for (int r = 0; r < nf; r++) {
            double acc = 0.0;
            for (int c = 0; c < nf; c++) acc += R[r * nf + c] * fc[c];
            Fout[r] = acc;
        }
    }
    return 0;
}

/* dU/dt at cell p: -sum_axis (F_{p+1/2} - F_{p-1/2}) / dx_axis, axes in
 * the order x, y, z (Eq. approximateEq, dimension by dimension).
 * *bandhit is incremented for every band hit met on the way. */
static int or_dudt_cell(const or_grid* g, const or_scheme* sc, const or_state* s, const int* p, double* dU,
                        long* bandhit) {
    int nf = or_nfields(g);
    for (int f = 0; f < nf; f++) dU[f] = 0.0;
    for (int ax = 0; ax < g->ndim; ax++) {
        double Fr[5], Fl[5];
        uint8_t br[10], bl[10];
        int pl[3] = {p[0], p[1], p[2]};
        pl[ax] -= 1;
        int rc = or_face_flux(g, sc, s, ax, p, Fr, NULL, br);
        if (rc == 0) rc = or_face_flux(g, sc, s, ax, pl, Fl, NULL, bl);
        if (rc) return rc;
        if (bandhit)
            for (int t = 0; t < 2 * nf; t++) *bandhit += (br[t] != 0) + (bl[t] != 0);
        for (int f = 0; f < nf; f++) dU[f] = dU[f] - (Fr[f] - Fl[f]) / g->dx[ax];
    }
    return 0;
}

static int or_check(const or_grid* g, const or_scheme* sc) {
    if (or_init() != 0) return -10;
    if (!g || g->ndim < 1 || g->ndim > 3) return -1;
    int k = sc->K & 0xff;
    if (k != 6 && k != 8) return -2;
    if ((sc->K & ~(0xff | OR_SCHEME_ADAPTIVE)) || ((sc->K & OR_SCHEME_ADAPTIVE) && k != 8)) return -2;
    for (int d = 0; d < g->ndim; d++)
        if (g->n[d] < 1) return -1;
    if (g->system != 0 && g->system != 1) return -2;
    return 0;
}

/* Error bits of the parallel loops: 1 = a face failed (Roe average),
 * 2 = a gamma sum was not finite (OR_ENONFINITE). */
static int or_err_bit(int rc) { return rc == 0 ? 0 : (rc == OR_ENONFINITE ? 2 : 1); }
static int or_err_code(int err) { return (err & 2) ? OR_ENONFINITE : (err ? -3 : 0); }

/* ------------------------------------------------------------------------ */
/* Whole-grid entry points (host arrays, same layouts as the C-ABI)          */
/* ------------------------------------------------------------------------ */

/* Face fluxes along `ax`: Fhat[field][..][n_ax + 1][..], face j between
 * cells j-1 and j.  flags/band (nullable): [2][nf][faces]. */
int or_reconstruct_faces(const or_grid* g, int K, int lim, double C_T, double gamma, int ax,
                         const double* U, double* Fhat, uint8_t* flags, uint8_t* band) {
    or_scheme sc = {K, lim, C_T, gamma};
    int rc = or_check(g, &sc);
    if (rc) return rc;
    if (ax < 0 || ax >= g->ndim) return -1;
    int nf = or_nfields(g);
    int fn[3] = {1, 1, 1};
    for (int d = 0; d < g->ndim; d++) fn[d] = g->n[d];
    fn[ax] += 1;
    long nfaces = (long)fn[0] * fn[1] * fn[2];
    or_state s = {g, U, 0, {0, 0, 0}, {0, 0, 0}};
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (long idx = 0; idx < nfaces; idx++) {
        int c[3] = {(int)(idx % fn[0]), (int)((idx / fn[0]) % fn[1]), (int)(idx / ((long)fn[0] * fn[1]))};
        int p[3] = {c[0], c[1], c[2]};
        p[ax] -= 1; /* face j sits between cells j-1 and j */
        double F[5];
        uint8_t fl[10], bd[10];
        int frc = or_face_flux(g, &sc, &s, ax, p, F, fl, bd);
        if (frc) {
            err |= or_err_bit(frc);
            continue;
        }
        for (int f = 0; f < nf; f++) {
            Fhat[(size_t)f * nfaces + idx] = F[f];
            if (flags) {
                flags[(size_t)f * nfaces + idx] = fl[f];
                flags[(size_t)(nf + f) * nfaces + idx] = fl[nf + f];
            }
            if (band) {
                band[(size_t)f * nfaces + idx] = bd[f];
                band[(size_t)(nf + f) * nfaces + idx] = bd[nf + f];
            }
        }
    }
    return or_err_code(err);
}

/* dU/dt on the whole grid, computed from the face fluxes of each axis. */
int or_flux_divergence(const or_grid* g, int K, int lim, double C_T, double gamma, const double* U,
                       double* dUdt) {
    or_scheme sc = {K, lim, C_T, gamma};
    int rc = or_check(g, &sc);
    if (rc) return rc;
    int nf = or_nfields(g);
    size_t N = or_ncells(g);
    for (size_t i = 0; i < (size_t)nf * N; i++) dUdt[i] = 0.0;
    for (int ax = 0; ax < g->ndim; ax++) {
        int fn[3] = {1, 1, 1}, cn[3] = {1, 1, 1};
        for (int d = 0; d < g->ndim; d++) fn[d] = cn[d] = g->n[d];
        fn[ax] += 1;
        size_t nfaces = (size_t)fn[0] * fn[1] * fn[2];
        double* F = (double*)malloc(sizeof(double) * nf * nfaces);
        if (!F) return -4;
        rc = or_reconstruct_faces(g, K, lim, C_T, gamma, ax, U, F, NULL, NULL);
        if (rc) {
            free(F);
            return rc;
        }
#pragma omp parallel for schedule(static)
        for (long idx = 0; idx < (long)N; idx++) {
            int c[3] = {(int)(idx % cn[0]), (int)((idx / cn[0]) % cn[1]), (int)(idx / ((long)cn[0] * cn[1]))};
            int r[3] = {c[0], c[1], c[2]};
            r[ax] += 1;
            size_t il = (size_t)c[0] + (size_t)fn[0] * ((size_t)c[1] + (size_t)fn[1] * c[2]);
            size_t ir = (size_t)r[0] + (size_t)fn[0] * ((size_t)r[1] + (size_t)fn[1] * r[2]);
            for (int f = 0; f < nf; f++)
                dUdt[(size_t)f * N + idx] =
                    dUdt[(size_t)f * N + idx] - (F[(size_t)f * nfaces + ir] - F[(size_t)f * nfaces + il]) / g->dx[ax];
        }
        free(F);
    }
    return 0;
}

/* One third-order SSP Runge-Kutta step (Gottlieb & Shu), in place:
 *   U1 = U + dt L(U);  U2 = 3/4 U + 1/4 (U1 + dt L(U1));
 *   U  = 1/3 U + 2/3 (U2 + dt L(U2)). */
int or_rk3_step(const or_grid* g, int K, int lim, double C_T, double gamma, double dt, double* U) {
    or_scheme sc = {K, lim, C_T, gamma};
    int rc = or_check(g, &sc);
    if (rc) return rc;
    size_t M = (size_t)or_nfields(g) * or_ncells(g);
    double* U1 = (double*)malloc(sizeof(double) * M);
    double* U2 = (double*)malloc(sizeof(double) * M);
    double* L = (double*)malloc(sizeof(double) * M);
    if (!U1 || !U2 || !L) {
        free(U1);
        free(U2);
        free(L);
        return -4;
    }
    rc = or_flux_divergence(g, K, lim, C_T, gamma, U, L);
    for (size_t i = 0; !rc && i < M; i++) U1[i] = U[i] + dt * L[i];
    if (!rc) rc = or_flux_divergence(g, K, lim, C_T, gamma, U1, L);
    for (size_t i = 0; !rc && i < M; i++) U2[i] = 0.75 * U[i] + 0.25 * (U1[i] + dt * L[i]);
    if (!rc) rc = or_flux_divergence(g, K, lim, C_T, gamma, U2, L);
    for (size_t i = 0; !rc && i < M; i++) U[i] = (1.0 / 3.0) * U[i] + (2.0 / 3.0) * (U2[i] + dt * L[i]);
    free(U1);
    free(U2);
    free(L);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Sampled entry points for grids too large to process whole on the CPU     */
/* ------------------------------------------------------------------------ */

static void or_unflatten(const or_grid* g, long idx, int* c) {
    c[0] = c[1] = c[2] = 0;
    for (int d = 0; d < g->ndim; d++) {
        c[d] = (int)(idx % g->n[d]);
        idx /= g->n[d];
    }
}

/* Face fluxes at selected faces of axis `ax`; face index uses the layout of
 * or_reconstruct_faces.  out: [npts][nf]; flags/band: [npts][2*nf]. */
int or_faces_points(const or_grid* g, int K, int lim, double C_T, double gamma, int ax, const double* U,
                    long npts, const long* face_idx, double* out, uint8_t* flags, uint8_t* band) {
    or_scheme sc = {K, lim, C_T, gamma};
    int rc = or_check(g, &sc);
    if (rc) return rc;
    int nf = or_nfields(g);
    int fn[3] = {1, 1, 1};
    for (int d = 0; d < g->ndim; d++) fn[d] = g->n[d];
    fn[ax] += 1;
    or_state s = {g, U, 0, {0, 0, 0}, {0, 0, 0}};
    int err = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : err)
    for (long t = 0; t < npts; t++) {
        long idx = face_idx[t];
        int p[3] = {(int)(idx % fn[0]), (int)((idx / fn[0]) % fn[1]), (int)(idx / ((long)fn[0] * fn[1]))};
        p[ax] -= 1;
        err |= or_err_bit(or_face_flux(g, &sc, &s, ax, p, out + t * nf, flags ? flags + t * 2 * nf : NULL,
                                       band ? band + t * 2 * nf : NULL));
    }
    return or_err_code(err);
}

/* dU/dt at selected cells (flat cell indices). out: [npts][nf]. */
int or_dudt_points(const or_grid* g, int K, int lim, double C_T, double gamma, const double* U, long npts,
                   const long* cell_idx, double* out, long* bandhits) {
    or_scheme sc = {K, lim, C_T, gamma};
    int rc = or_check(g, &sc);
    if (rc) return rc;
    int nf = or_nfields(g);
    or_state s = {g, U, 0, {0, 0, 0}, {0, 0, 0}};
    int err = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : err)
    for (long t = 0; t < npts; t++) {
        int p[3];
        long bh = 0;
        or_unflatten(g, cell_idx[t], p);
        err |= or_err_bit(or_dudt_cell(g, &sc, &s, p, out + t * nf, &bh));
        if (bandhits) bandhits[t] = bh;
    }
    return or_err_code(err);
}

/* Fill one RK stage on a box of cells around `ctr` with half-width rad
 * (in the grid's dimensions): out(Q) = a*U0(Qc) + b*(Us(Qc) + dt*L(Us)(Qc)),
 * where Qc is Q with transmissive coordinates clamped into the grid. */
static int or_stage_box(const or_grid* g, const or_scheme* sc, const or_state* s0, const or_state* ss,
                        const int* ctr, int rad, double a, double b, double dt, double* out, int* bn,
                        int* org, long* bandhit) {
    int nf = or_nfields(g);
    size_t tot = 1;
    for (int d = 0; d < 3; d++) {
        bn[d] = (d < g->ndim) ? 2 * rad + 1 : 1;
        org[d] = (d < g->ndim) ? ctr[d] - rad : 0;
        tot *= (size_t)bn[d];
    }
    for (size_t t = 0; t < tot; t++) {
        int Q[3] = {org[0] + (int)(t % bn[0]), org[1] + (int)((t / bn[0]) % bn[1]),
                    org[2] + (int)(t / ((size_t)bn[0] * bn[1]))};
        for (int d = 0; d < g->ndim; d++)
            if (g->bc[d] == 1) Q[d] = or_bc_index(Q[d], g->n[d], 1);
        double dU[5];
        int rc = or_dudt_cell(g, sc, ss, Q, dU, bandhit);
        if (rc) return rc;
        for (int f = 0; f < nf; f++) {
            double u0 = or_get(s0, f, Q), us = or_get(ss, f, Q);
            out[(size_t)f * tot + t] = a * u0 + b * (us + dt * dU[f]);
        }
    }
    return 0;
}

/* One SSP-RK3 step evaluated only at the selected cells, from the dependency
 * cone of each one (boxes of half-width 2K/2 and K/2 for the first two
 * stages).  out: [npts][nf]; bandhits[t] counts band hits in the cone. */
int or_rk3_points(const or_grid* g, int K, int lim, double C_T, double gamma, double dt, const double* U,
                  long npts, const long* cell_idx, double* out, long* bandhits) {
    or_scheme sc = {K, lim, C_T, gamma};
    int rc = or_check(g, &sc);
    if (rc) return rc;
    int nf = or_nfields(g), h = (K & 0xff) / 2;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (long t = 0; t < npts; t++) {
        int ctr[3];
        long bh = 0;
        or_unflatten(g, cell_idx[t], ctr);
        size_t n1 = 1, n2 = 1;
        for (int d = 0; d < g->ndim; d++) {
            n1 *= (size_t)(4 * h + 1);
            n2 *= (size_t)(2 * h + 1);
        }
        double* B1 = (double*)malloc(sizeof(double) * nf * n1);
        double* B2 = (double*)malloc(sizeof(double) * nf * n2);
        if (!B1 || !B2) {
            free(B1);
            free(B2);
            err |= 1;
            continue;
        }
        or_state s0 = {g, U, 0, {0, 0, 0}, {0, 0, 0}};
        or_state s1 = {g, B1, 1, {0, 0, 0}, {0, 0, 0}};
        or_state s2 = {g, B2, 1, {0, 0, 0}, {0, 0, 0}};
        int src = or_stage_box(g, &sc, &s0, &s0, ctr, 2 * h, 0.0, 1.0, dt, B1, s1.bn, s1.org, &bh);
        if (src == 0) src = or_stage_box(g, &sc, &s0, &s1, ctr, h, 0.75, 0.25, dt, B2, s2.bn, s2.org, &bh);
        if (src == 0) {
            double dU[5];
            src = or_dudt_cell(g, &sc, &s2, ctr, dU, &bh);
            for (int f = 0; src == 0 && f < nf; f++)
                out[t * nf + f] = (1.0 / 3.0) * or_get(&s0, f, ctr) + (2.0 / 3.0) * (or_get(&s2, f, ctr) + dt * dU[f]);
        }
        err |= or_err_bit(src);
        if (bandhits) bandhits[t] = bh;
        free(B1);
        free(B2);
    }
    return or_err_code(err);
}

/* max over cells of sum_d (|u_d| + c) / dx_d (scalar: sum_d |a_d| / dx_d);
 * a stable step is dt = CFL / this value. */
double or_max_wave_speed(const or_grid* g, double gamma, const double* U) {
    size_t N = or_ncells(g);
    double best = 0.0;
    for (size_t i = 0; i < N; i++) {
        double s = 0.0;
        if (g->system == 0) {
            for (int d = 0; d < g->ndim; d++) s += fabs(g->adv[d]) / g->dx[d];
        } else {
            int nf = g->ndim + 2;
            double rho = U[i], E = U[(size_t)(nf - 1) * N + i], q2 = 0.0, vel[3] = {0, 0, 0};
            for (int d = 0; d < g->ndim; d++) {
                vel[d] = U[(size_t)(1 + d) * N + i] / rho;
                q2 += vel[d] * vel[d];
            }
            double p = (gamma - 1.0) * (E - 0.5 * rho * q2);
            double c = sqrt(gamma * p / rho);
            for (int d = 0; d < g->ndim; d++) s += (fabs(vel[d]) + c) / g->dx[d];
        }
        if (!(s <= best)) best = s; /* a NaN propagates */
    }
    return best;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel regions (n >= 1); timing only. */
void or_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
