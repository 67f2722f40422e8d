/*
 * Drives every entry point of the C oracle on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py
 * compiles it with gcc; nothing else uses it).  It includes the oracle's
 * source so that its internal types are visible, and prints "OK" when every
 * check passes.  Any out-of-bounds access, leak of a freed block or undefined
 * operation aborts the run under the sanitizers.
 *
 * Besides running the code, it checks properties the paper's definitions fix:
 *   - the residual is f minus the stencil of eq. 2.2 applied to x;
 *   - full weighting and bilinear prolongation (eq. 2.9) are adjoint up to
 *     the factor 4 (P = 4 R^T), also on grids whose size is not a power of 2;
 *   - the banded direct solve leaves a residual at rounding level;
 *   - FGMRES with the built-in V-cycle and with the same V-cycle passed as a
 *     callback gives the same iterates, and both reach the tolerance in the
 *     true residual;
 *   - a run cut off by maxit reports non-convergence with the step count;
 *   - invalid hierarchies and arguments are rejected.
 */
#include "helm_oracle.c"

#include <stdio.h>

static unsigned long long rng_s = 0x9E3779B97F4A7C15ULL;

/* xorshift64*, uniform in [0, 1) */
static double urand(void)
{
    rng_s ^= rng_s >> 12;
    rng_s ^= rng_s << 25;
    rng_s ^= rng_s >> 27;
    return (double)((rng_s * 0x2545F4914F6CDD1DULL) >> 11) * (1.0 / 9007199254740992.0);
}

static void fill_medium(int n, double *kap, double *gam)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double x = (i + 0.5) / n, y = (j + 0.5) / n;
            kap[(size_t)i * n + j] = 0.6 + 0.3 * sin(3.0 * x) * cos(2.0 * y);
            int d = i < j ? i : j;
            int e = (n - 1 - i) < (n - 1 - j) ? (n - 1 - i) : (n - 1 - j);
            if (e < d) d = e;
            gam[(size_t)i * n + j] = 0.01 + (d < 4 ? 0.5 * (4 - d) / 4.0 : 0.0);
        }
}

static void fill_field(size_t N, cplx *u)
{
    for (size_t p = 0; p < N; p++)
        u[p] = (urand() - 0.5) + I * (urand() - 0.5);
}

static int fails = 0;
#define CHECK(cond, ...)                              \
    do {                                              \
        if (!(cond)) {                                \
            fails++;                                  \
            printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            printf(__VA_ARGS__);                      \
            printf("\n");                             \
        }                                             \
    } while (0)

static void vcycle_prec(void *ctx, const cplx *in, cplx *out)
{
    orc_vcycle((const orc_hier *)ctx, in, out);
}

static void grid_operators(int n, double omega)
{
    size_t N = (size_t)n * n, Nc = N / 4;
    double h = 1.0 / n;
    double *kap = malloc(N * sizeof(double)), *gam = malloc(N * sizeof(double));
    double *kc = malloc(Nc * sizeof(double));
    cplx *x = malloc(N * sizeof(cplx)), *f = malloc(N * sizeof(cplx));
    cplx *y = malloc(N * sizeof(cplx)), *r = malloc(N * sizeof(cplx));
    cplx *g = malloc(Nc * sizeof(cplx)), *fc = malloc(Nc * sizeof(cplx));
    cplx *pg = calloc(N, sizeof(cplx));
    fill_medium(n, kap, gam);
    fill_field(N, x);
    fill_field(N, f);
    fill_field(Nc, g);

    orc_apply(n, h, omega, kap, gam, 0.5, x, y);
    orc_residual(n, h, omega, kap, gam, 0.5, f, x, r);
    double d = 0.0;
    for (size_t p = 0; p < N; p++) d = fmax(d, cabs(r[p] - (f[p] - y[p])));
    CHECK(d == 0.0, "n=%d residual differs from f - M x by %g", n, d);

    orc_jacobi(n, h, omega, kap, gam, 0.5, 0.8, f, x);
    for (size_t p = 0; p < N; p++) CHECK(isfinite(creal(x[p])) && isfinite(cimag(x[p])), "jacobi nan");

    /* <R f, g> * 4 = <f, P g> */
    orc_restrict(n, f, fc);
    orc_prolong_add(n, g, pg);
    cplx a = 0.0, b = 0.0;
    double s = 0.0;
    for (size_t p = 0; p < Nc; p++) { a += conj(fc[p]) * g[p]; s += cabs(fc[p]) * cabs(g[p]); }
    for (size_t p = 0; p < N; p++) b += conj(f[p]) * pg[p];
    CHECK(cabs(4.0 * a - b) <= 1e-13 * (4.0 * s + 1.0), "n=%d adjoint mismatch %g", n, cabs(4.0 * a - b));

    orc_inject(n, kap, kc);
    for (int i = 0; i < n / 2; i++)
        for (int j = 0; j < n / 2; j++)
            CHECK(kc[(size_t)i * (n / 2) + j] == kap[(size_t)(2 * i) * n + 2 * j], "inject (%d,%d)", i, j);

    /* banded direct solve of the shifted operator */
    memcpy(y, f, N * sizeof(cplx));
    CHECK(orc_band_solve(n, h, omega, kap, gam, 0.5, y) == 0, "band solve failed n=%d", n);
    orc_residual(n, h, omega, kap, gam, 0.5, f, y, r);
    CHECK(vnorm(r, N) <= 1e-10 * vnorm(f, N), "band solve residual %g", vnorm(r, N) / vnorm(f, N));

    free(kap); free(gam); free(kc); free(x); free(f); free(y); free(r); free(g); free(fc); free(pg);
}

static void solve(int n, int levels, double omega, int coarse_k)
{
    size_t N = (size_t)n * n;
    double *kap = malloc(N * sizeof(double)), *gam = malloc(N * sizeof(double));
    cplx *b = calloc(N, sizeof(cplx)), *x1 = malloc(N * sizeof(cplx));
    cplx *x2 = malloc(N * sizeof(cplx)), *r = malloc(N * sizeof(cplx));
    double *hist = malloc(401 * sizeof(double));
    fill_medium(n, kap, gam);
    b[(size_t)(n / 2) * n + n / 3] = 1.0;
    b[(size_t)(n / 4) * n + n / 2] = 0.5 * I;

    orc_hier *H = orc_hier_create(n, levels, omega, kap, gam, 0.5, 0.8);
    CHECK(H != NULL, "hierarchy n=%d levels=%d", n, levels);
    if (!H) goto out;
    CHECK(orc_hier_level_n(H, levels - 1) == n >> (levels - 1), "level size");
    CHECK(orc_hier_level_kappa(H, 0)[5] == kap[5] && orc_hier_level_gamma(H, 0)[7] == gam[7], "level 0 fields");
    CHECK(orc_hier_set_coarse_gmres(H, coarse_k) == 0, "set coarse gmres");

    orc_fgmres_stats s1, s2;
    int rc1 = orc_fgmres(H, NULL, NULL, 10, 1e-8, 400, b, x1, hist, &s1);
    int rc2 = orc_fgmres(H, vcycle_prec, H, 10, 1e-8, 400, b, x2, NULL, &s2);
    CHECK(rc1 == 0 && s1.converged, "n=%d levels=%d k=%d not converged (%d its, %g)", n, levels, coarse_k,
          s1.iterations, s1.true_relres);
    orc_hier_residual_A(H, b, x1, r);
    CHECK(vnorm(r, N) / vnorm(b, N) <= 1e-8 && fabs(vnorm(r, N) / vnorm(b, N) - s1.true_relres) <= 1e-12,
          "true residual %g reported %g", vnorm(r, N) / vnorm(b, N), s1.true_relres);
    CHECK(hist[0] == 1.0 && hist[s1.iterations] <= hist[0], "history");
    double d = 0.0;
    for (size_t p = 0; p < N; p++) d = fmax(d, cabs(x1[p] - x2[p]));
    CHECK(rc2 == 0 && s2.iterations == s1.iterations && d == 0.0,
          "callback V-cycle differs: its %d vs %d, max diff %g", s2.iterations, s1.iterations, d);

    /* cut off by maxit: three steps, tolerance out of reach */
    int rc3 = orc_fgmres(H, NULL, NULL, 10, 1e-30, 3, b, x2, hist, &s2);
    CHECK(rc3 == 1 && !s2.converged && s2.iterations == 3, "maxit: rc %d its %d", rc3, s2.iterations);
    orc_hier_free(H);
out:
    free(kap); free(gam); free(b); free(x1); free(x2); free(r); free(hist);
}

int main(void)
{
    grid_operators(24, 30.0);   /* not a power of 2 */
    grid_operators(32, 60.0);
    solve(32, 3, 30.0, 0);      /* exact coarsest solve on 8 x 8 */
    solve(48, 4, 40.0, 0);      /* coarsest 6 x 6 */
    solve(32, 3, 30.0, 4);      /* GMRES(4) + Jacobi on the coarsest level */
    solve(16, 1, 20.0, 0);      /* one level: the direct solve preconditions */

    double k1[16] = {1.0}, g1[16] = {0.0};
    CHECK(orc_hier_create(4, 0, 1.0, k1, g1, 0.5, 0.8) == NULL, "levels 0 accepted");
    CHECK(orc_hier_create(6, 3, 1.0, k1, g1, 0.5, 0.8) == NULL, "n not divisible accepted");
    CHECK(orc_hier_set_coarse_gmres(NULL, 1) == -1, "null hierarchy accepted");
    CHECK(orc_vcycle(NULL, NULL, NULL) == -1, "null V-cycle accepted");

    if (fails) {
        printf("%d check(s) failed\n", fails);
        return 1;
    }
    printf("OK\n");
    return 0;
}
