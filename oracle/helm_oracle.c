/*
 * CPU oracle for the shifted-Laplacian (SL) preconditioned FGMRES solver of
 * the discrete heterogeneous 2D Helmholtz equation (Azulay & Treister,
 * "Multigrid-augmented deep learning preconditioners for the Helmholtz
 * equation").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg load it; the product path never does.
 * It shares no code, header or table with the GPU library.
 *
 * Everything here is double precision (complex double for fields), written
 * as direct loops in the order the paper states the method.
 *
 * Grid convention: unknowns u[i*n + j], i, j = 0..n-1, mesh width h = 1/n;
 * values outside the array are zero (zero padding of the convolution form,
 * i.e. the Dirichlet condition of section 2.4).  Coarse point (I, J) of a
 * level sits on fine point (2I, 2J).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Value of field u at (i, j), zero outside the n x n array. */
static cplx at(const cplx *u, int n, int i, int j)
{
    if (i < 0 || j < 0 || i >= n || j >= n)
        return 0.0;
    return u[(size_t)i * n + j];
}

/*
 * Mass coefficient of the operator at one point.
 * Eq. 2.1 gives the Helmholtz term -omega^2 kappa^2 (1 - gamma i) u; the
 * shifted Laplacian of eq. 2.4 uses (alpha - beta i) with alpha = 1, so with
 * attenuation present the shift adds beta to gamma.  `shift` = 0 gives A,
 * `shift` = beta gives M.  The operator is  (5-point Laplacian) - mass * u.
 */
static cplx mass_coef(double omega, double kappa, double gamma, double shift)
{
    return omega * omega * kappa * kappa * (1.0 - I * (gamma + shift));
}

/*
 * y = Op x, the 5-point finite-difference stencil of eq. 2.2 with the
 * attenuated mass term of eq. 2.1:
 *   (Op x)(i,j) = (4x(i,j) - x(i-1,j) - x(i+1,j) - x(i,j-1) - x(i,j+1)) / h^2
 *                 - omega^2 kappa(i,j)^2 (1 - i(gamma(i,j) + shift)) x(i,j)
 */
void orc_apply(int n, double h, double omega, const double *kappa,
               const double *gamma, double shift, const cplx *x, cplx *y)
{
    double ih2 = 1.0 / (h * h);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            size_t p = (size_t)i * n + j;
            cplx lap = (4.0 * x[p] - at(x, n, i - 1, j) - at(x, n, i + 1, j)
                        - at(x, n, i, j - 1) - at(x, n, i, j + 1)) * ih2;
            y[p] = lap - mass_coef(omega, kappa[p], gamma[p], shift) * x[p];
        }
}

/* r = f - Op x */
void orc_residual(int n, double h, double omega, const double *kappa,
                  const double *gamma, double shift, const cplx *f,
                  const cplx *x, cplx *r)
{
    orc_apply(n, h, omega, kappa, gamma, shift, x, r);
    for (size_t p = 0; p < (size_t)n * n; p++)
        r[p] = f[p] - r[p];
}

/*
 * One damped Jacobi sweep on Op x = f (section 2.2 footnote; weight 0.8 in
 * section 4):  x <- x + w D^{-1} (f - Op x),  D = diag(Op) = 4/h^2 - mass.
 */
void orc_jacobi(int n, double h, double omega, const double *kappa,
                const double *gamma, double shift, double weight,
                const cplx *f, cplx *x)
{
    size_t N = (size_t)n * n;
    cplx *r = malloc(N * sizeof(cplx));
    orc_residual(n, h, omega, kappa, gamma, shift, f, x, r);
    for (size_t p = 0; p < N; p++) {
        cplx d = 4.0 / (h * h) - mass_coef(omega, kappa[p], gamma[p], shift);
        x[p] += weight * r[p] / d;
    }
    free(r);
}

/*
 * Full-weighting restriction (eq. 2.9): a stride-2 convolution with the
 * kernel (1/16)[1 2 1; 2 4 2; 1 2 1] and zero padding 1.
 *   fc(I,J) = sum_{a,b in {-1,0,1}} w(a) w(b) f(2I+a, 2J+b),  w = (1/4,1/2,1/4)
 * n is the fine size (even); the coarse size is n/2.
 */
void orc_restrict(int n, const cplx *f, cplx *fc)
{
    static const double w[3] = {0.25, 0.5, 0.25};
    int nc = n / 2;
    for (int ic = 0; ic < nc; ic++)
        for (int jc = 0; jc < nc; jc++) {
            cplx s = 0.0;
            for (int a = -1; a <= 1; a++)
                for (int b = -1; b <= 1; b++)
                    s += w[a + 1] * w[b + 1] * at(f, n, 2 * ic + a, 2 * jc + b);
            fc[(size_t)ic * nc + jc] = s;
        }
}

/*
 * Bilinear prolongation added into the fine field (eq. 2.9): the transposed
 * stride-2 convolution with (1/4)[1 2 1; 2 4 2; 1 2 1]: every coarse value
 * is scattered to the 3 x 3 fine neighbourhood of its fine position (2I, 2J)
 * with weights p(a) p(b), p(0) = 1, p(+-1) = 1/2.
 */
void orc_prolong_add(int n, const cplx *ec, cplx *e)
{
    static const double p[3] = {0.5, 1.0, 0.5};
    int nc = n / 2;
    for (int ic = 0; ic < nc; ic++)
        for (int jc = 0; jc < nc; jc++) {
            cplx v = ec[(size_t)ic * nc + jc];
            for (int a = -1; a <= 1; a++)
                for (int b = -1; b <= 1; b++) {
                    int i = 2 * ic + a, j = 2 * jc + b;
                    if (i >= 0 && j >= 0 && i < n && j < n)
                        e[(size_t)i * n + j] += p[a + 1] * p[b + 1] * v;
                }
        }
}

/* Coefficient field on the next coarser grid by injection: c(I,J) = f(2I,2J). */
void orc_inject(int n, const double *f, double *c)
{
    int nc = n / 2;
    for (int ic = 0; ic < nc; ic++)
        for (int jc = 0; jc < nc; jc++)
            c[(size_t)ic * nc + jc] = f[(size_t)(2 * ic) * n + 2 * jc];
}

/* ------------------------------------------------------------------------
 * Banded LU with partial pivoting (the coarsest-grid direct solve).
 * Storage is the LAPACK general-band layout: entry (i, j) of the N x N matrix
 * lives at ab[(kl + ku + i - j) + j * ldab], ldab = 2*kl + ku + 1; the top kl
 * rows hold the fill-in that row interchanges create.
 * ---------------------------------------------------------------------- */
typedef struct {
    int N, kl, ku, ldab;
    cplx *ab;
    int *ipiv;
} band_lu;

#define BAND(L, i, j) ((L)->ab[(size_t)((L)->kl + (L)->ku + (i) - (j)) + (size_t)(j) * (L)->ldab])

static int imin(int a, int b) { return a < b ? a : b; }

/* In-place LU: P A = L U, L unit lower with kl sub-diagonals, U with kl+ku. */
static int band_factor(band_lu *L)
{
    int N = L->N, kl = L->kl, ku = L->ku;
    for (int j = 0; j < N; j++) {
        int last = imin(N - 1, j + kl);
        int p = j;
        double best = cabs(BAND(L, j, j));
        for (int i = j + 1; i <= last; i++)
            if (cabs(BAND(L, i, j)) > best) {
                best = cabs(BAND(L, i, j));
                p = i;
            }
        L->ipiv[j] = p;
        if (best == 0.0)
            return -1;
        int cend = imin(N - 1, j + kl + ku);
        if (p != j)
            for (int c = j; c <= cend; c++) {
                cplx t = BAND(L, j, c);
                BAND(L, j, c) = BAND(L, p, c);
                BAND(L, p, c) = t;
            }
        for (int i = j + 1; i <= last; i++)
            BAND(L, i, j) /= BAND(L, j, j);
        for (int i = j + 1; i <= last; i++)
            for (int c = j + 1; c <= cend; c++)
                BAND(L, i, c) -= BAND(L, i, j) * BAND(L, j, c);
    }
    return 0;
}

/* Solve A x = b in place using the factor. */
static void band_solve(const band_lu *L, cplx *b)
{
    int N = L->N, kl = L->kl, ku = L->ku;
    for (int j = 0; j < N; j++) {
        int p = L->ipiv[j];
        if (p != j) {
            cplx t = b[j];
            b[j] = b[p];
            b[p] = t;
        }
        for (int i = j + 1; i <= imin(N - 1, j + kl); i++)
            b[i] -= BAND(L, i, j) * b[j];
    }
    for (int i = N - 1; i >= 0; i--) {
        cplx s = b[i];
        for (int c = i + 1; c <= imin(N - 1, i + kl + ku); c++)
            s -= BAND(L, i, c) * b[c];
        b[i] = s / BAND(L, i, i);
    }
}

/* Assemble the operator of one level (shift included) into band storage. */
static band_lu *band_assemble(int n, double h, double omega, const double *kappa,
                              const double *gamma, double shift)
{
    band_lu *L = calloc(1, sizeof(band_lu));
    L->N = n * n;
    L->kl = n;
    L->ku = n;
    L->ldab = 2 * n + n + 1;
    L->ab = calloc((size_t)L->ldab * L->N, sizeof(cplx));
    L->ipiv = calloc(L->N, sizeof(int));
    double ih2 = 1.0 / (h * h);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            int q = i * n + j;
            BAND(L, q, q) = 4.0 * ih2 - mass_coef(omega, kappa[q], gamma[q], shift);
            if (i > 0) BAND(L, q, q - n) = -ih2;
            if (i < n - 1) BAND(L, q, q + n) = -ih2;
            if (j > 0) BAND(L, q, q - 1) = -ih2;
            if (j < n - 1) BAND(L, q, q + 1) = -ih2;
        }
    return L;
}

static void band_free(band_lu *L)
{
    if (!L) return;
    free(L->ab);
    free(L->ipiv);
    free(L);
}

/* Exposed for tests: solve Op x = b on one grid by banded LU (x overwrites b). */
int orc_band_solve(int n, double h, double omega, const double *kappa,
                   const double *gamma, double shift, cplx *b)
{
    band_lu *L = band_assemble(n, h, omega, kappa, gamma, shift);
    int rc = band_factor(L);
    if (rc == 0)
        band_solve(L, b);
    band_free(L);
    return rc;
}

/* ------------------------------------------------------------------------
 * SL multigrid hierarchy and V-cycle (section 2.2, Algorithm 1).
 * Level l has n_l = n / 2^l points per side and mesh width h_l = 2^l h; its
 * operator is re-discretised with kappa and gamma injected from level l-1.
 * ---------------------------------------------------------------------- */
typedef struct {
    int levels;
    double omega, beta, weight;
    int n[16];
    double h[16];
    double *kappa[16], *gamma[16];
    band_lu *coarse;
    int coarse_gmres;  /* 0: exact coarsest solve; k > 0: GMRES(k) + Jacobi */
} orc_hier;

orc_hier *orc_hier_create(int n, int levels, double omega, const double *kappa,
                          const double *gamma, double beta, double weight)
{
    if (levels < 1 || levels > 16 || (n % (1 << (levels - 1))) != 0)
        return NULL;
    orc_hier *H = calloc(1, sizeof(orc_hier));
    H->levels = levels;
    H->omega = omega;
    H->beta = beta;
    H->weight = weight;
    size_t N = (size_t)n * n;
    for (int l = 0; l < levels; l++) {
        H->n[l] = n >> l;
        H->h[l] = (double)(1 << l) / n;
        size_t Nl = (size_t)H->n[l] * H->n[l];
        H->kappa[l] = malloc(Nl * sizeof(double));
        H->gamma[l] = malloc(Nl * sizeof(double));
        if (l == 0) {
            memcpy(H->kappa[0], kappa, N * sizeof(double));
            memcpy(H->gamma[0], gamma, N * sizeof(double));
        } else {
            orc_inject(H->n[l - 1], H->kappa[l - 1], H->kappa[l]);
            orc_inject(H->n[l - 1], H->gamma[l - 1], H->gamma[l]);
        }
    }
    int L = levels - 1;
    H->coarse = band_assemble(H->n[L], H->h[L], omega, H->kappa[L], H->gamma[L], beta);
    if (band_factor(H->coarse) != 0) {
        band_free(H->coarse);
        H->coarse = NULL;
    }
    return H;
}

void orc_hier_free(orc_hier *H)
{
    if (!H) return;
    for (int l = 0; l < H->levels; l++) {
        free(H->kappa[l]);
        free(H->gamma[l]);
    }
    band_free(H->coarse);
    free(H);
}

int orc_hier_level_n(const orc_hier *H, int l) { return H->n[l]; }
const double *orc_hier_level_kappa(const orc_hier *H, int l) { return H->kappa[l]; }
const double *orc_hier_level_gamma(const orc_hier *H, int l) { return H->gamma[l]; }

/* Plain inner products for the coarse GMRES (defined again below for FGMRES). */
static double cg_norm(const cplx *v, size_t N)
{
    double s = 0.0;
    for (size_t p = 0; p < N; p++)
        s += creal(v[p]) * creal(v[p]) + cimag(v[p]) * cimag(v[p]);
    return sqrt(s);
}

static cplx cg_dot(const cplx *u, const cplx *v, size_t N)
{
    cplx s = 0.0;
    for (size_t p = 0; p < N; p++)
        s += conj(u[p]) * v[p];
    return s;
}

/*
 * Coarsest-level solve of section 4's setting: k steps of GMRES on
 * M_L x = f with the diagonal (Jacobi) right preconditioner D^-1,
 * D = diag(M_L), from x = 0, one cycle (no restart).  Plain definition:
 * x = D^-1 V y with V an orthonormal basis (modified Gram-Schmidt) of the
 * Krylov space K_k(M_L D^-1, f) and y minimising ||f - M_L D^-1 V y||,
 * found from the Hessenberg matrix by a dense least-squares solve (normal
 * equations are avoided: the (k+1) x k system is solved by Householder QR
 * written out below).  The iteration stops early on an exact breakdown.
 */
static void coarse_gmres(const orc_hier *H, int l, int k, const cplx *f, cplx *x)
{
    int n = H->n[l];
    size_t N = (size_t)n * n;
    double h = H->h[l], om = H->omega, sh = H->beta;
    cplx *V = calloc((size_t)(k + 1) * N, sizeof(cplx));
    cplx *z = malloc(N * sizeof(cplx)), *w = malloc(N * sizeof(cplx));
    cplx *Dinv = malloc(N * sizeof(cplx));
    cplx *Hm = calloc((size_t)(k + 1) * k, sizeof(cplx)); /* Hm[i*k + j] */
    for (size_t p = 0; p < N; p++)
        Dinv[p] = 1.0 / (4.0 / (h * h) - mass_coef(om, H->kappa[l][p], H->gamma[l][p], sh));
    memset(x, 0, N * sizeof(cplx));
    double beta = cg_norm(f, N);
    if (beta == 0.0)
        goto out;
    for (size_t p = 0; p < N; p++)
        V[p] = f[p] / beta;
    int kk = 0;
    for (int j = 0; j < k; j++) {
        cplx *vj = V + (size_t)j * N;
        for (size_t p = 0; p < N; p++)
            z[p] = Dinv[p] * vj[p];
        orc_apply(n, h, om, H->kappa[l], H->gamma[l], sh, z, w);
        for (int i = 0; i <= j; i++) {
            cplx *vi = V + (size_t)i * N;
            cplx hij = cg_dot(vi, w, N);
            Hm[i * k + j] = hij;
            for (size_t p = 0; p < N; p++)
                w[p] -= hij * vi[p];
        }
        double hn = cg_norm(w, N);
        Hm[(j + 1) * k + j] = hn;
        kk = j + 1;
        if (hn == 0.0)
            break;
        for (size_t p = 0; p < N; p++)
            V[(size_t)(j + 1) * N + p] = w[p] / hn;
    }
    {
        /* least squares min || beta e_1 - Hm y || over y in C^kk by
         * Householder QR of the (kk+1) x kk matrix */
        int m = kk + 1;
        cplx *A = malloc((size_t)m * kk * sizeof(cplx)), *rhs = calloc(m, sizeof(cplx));
        cplx *y = calloc(kk > 0 ? kk : 1, sizeof(cplx));
        for (int i = 0; i < m; i++)
            for (int j = 0; j < kk; j++)
                A[i * kk + j] = Hm[i * k + j];
        rhs[0] = beta;
        for (int c = 0; c < kk; c++) {
            double nrm = 0.0;
            for (int i = c; i < m; i++)
                nrm += creal(A[i * kk + c] * conj(A[i * kk + c]));
            nrm = sqrt(nrm);
            if (nrm == 0.0)
                continue;
            cplx a0 = A[c * kk + c];
            cplx ph = cabs(a0) > 0.0 ? a0 / cabs(a0) : 1.0;
            cplx *u = calloc(m, sizeof(cplx));
            for (int i = c; i < m; i++)
                u[i] = A[i * kk + c];
            u[c] += ph * nrm;
            double un = 0.0;
            for (int i = c; i < m; i++)
                un += creal(u[i] * conj(u[i]));
            for (int j = c; j < kk; j++) {
                cplx t = 0.0;
                for (int i = c; i < m; i++)
                    t += conj(u[i]) * A[i * kk + j];
                for (int i = c; i < m; i++)
                    A[i * kk + j] -= 2.0 * u[i] * t / un;
            }
            cplx t = 0.0;
            for (int i = c; i < m; i++)
                t += conj(u[i]) * rhs[i];
            for (int i = c; i < m; i++)
                rhs[i] -= 2.0 * u[i] * t / un;
            free(u);
        }
        for (int i = kk - 1; i >= 0; i--) {
            cplx t = rhs[i];
            for (int j = i + 1; j < kk; j++)
                t -= A[i * kk + j] * y[j];
            y[i] = t / A[i * kk + i];
        }
        for (int j = 0; j < kk; j++)
            for (size_t p = 0; p < N; p++)
                x[p] += Dinv[p] * y[j] * V[(size_t)j * N + p];
        free(A);
        free(rhs);
        free(y);
    }
out:
    free(V);
    free(z);
    free(w);
    free(Dinv);
    free(Hm);
}

/* Coarsest solver: 0 = exact (banded LU), k > 0 = GMRES(k) with Jacobi. */
int orc_hier_set_coarse_gmres(orc_hier *H, int k)
{
    if (!H || k < 0)
        return -1;
    H->coarse_gmres = k;
    return 0;
}

/*
 * v = V-cycle(0, f) on the shifted operator M of level l (Algorithm 1 with
 * one pre- and one post-relaxation).  On the coarsest level the system is
 * solved directly; the relaxations Algorithm 1 places around that solve act
 * on an exact solution and are omitted.
 */
static void vcycle_level(const orc_hier *H, int l, const cplx *f, cplx *v)
{
    int n = H->n[l];
    size_t N = (size_t)n * n;
    double h = H->h[l], om = H->omega, sh = H->beta;
    if (l == H->levels - 1) {
        if (H->coarse_gmres > 0) {
            /* Algorithm 1 at the deepest level: the pre-relaxation is
             * overwritten by the solve (GMRES from zero); the
             * post-relaxation follows the inexact solve */
            coarse_gmres(H, l, H->coarse_gmres, f, v);
            orc_jacobi(n, h, om, H->kappa[l], H->gamma[l], sh, H->weight, f, v);
            return;
        }
        memcpy(v, f, N * sizeof(cplx));
        band_solve(H->coarse, v);
        return;
    }
    memset(v, 0, N * sizeof(cplx));
    orc_jacobi(n, h, om, H->kappa[l], H->gamma[l], sh, H->weight, f, v);
    cplx *r = malloc(N * sizeof(cplx));
    orc_residual(n, h, om, H->kappa[l], H->gamma[l], sh, f, v, r);
    size_t Nc = N / 4;
    cplx *fc = malloc(Nc * sizeof(cplx));
    cplx *vc = malloc(Nc * sizeof(cplx));
    orc_restrict(n, r, fc);
    vcycle_level(H, l + 1, fc, vc);
    orc_prolong_add(n, vc, v);
    orc_jacobi(n, h, om, H->kappa[l], H->gamma[l], sh, H->weight, f, v);
    free(r);
    free(fc);
    free(vc);
}

int orc_vcycle(const orc_hier *H, const cplx *f, cplx *v)
{
    if (!H || !H->coarse)
        return -1;
    vcycle_level(H, 0, f, v);
    return 0;
}

/* ------------------------------------------------------------------------
 * Restarted flexible GMRES (FGMRES(m), Saad 1993, cited in section 3) with
 * right preconditioning as in eq. 2.5, modified Gram-Schmidt Arnoldi and
 * complex Givens rotations.  x starts at zero; each cycle restarts from the
 * true residual b - A x.  The iteration stops when the true relative
 * residual ||b - A x|| / ||b|| <= tol; the implicit Givens estimate only
 * decides when a cycle ends early.
 * ---------------------------------------------------------------------- */
typedef void (*orc_prec_fn)(void *ctx, const cplx *in, cplx *out);

typedef struct {
    int iterations;      /* preconditioner applications / Arnoldi steps */
    int restarts;        /* completed cycles */
    int converged;       /* 1 when the true relative residual <= tol */
    double true_relres;  /* final ||b - A x|| / ||b|| */
} orc_fgmres_stats;

static double vnorm(const cplx *v, size_t N)
{
    double s = 0.0;
    for (size_t p = 0; p < N; p++)
        s += creal(v[p]) * creal(v[p]) + cimag(v[p]) * cimag(v[p]);
    return sqrt(s);
}

/* Hermitian inner product <u, v> = sum conj(u) v */
static cplx vdot(const cplx *u, const cplx *v, size_t N)
{
    cplx s = 0.0;
    for (size_t p = 0; p < N; p++)
        s += conj(u[p]) * v[p];
    return s;
}

/*
 * A is the level-0 Helmholtz operator of the hierarchy (shift 0).
 * prec == NULL selects the SL V-cycle of the hierarchy (M_V).
 * hist (optional, length maxit + 1): hist[k] = implicit residual estimate
 * ||r_k|| / ||b|| after k iterations (hist[0] = initial).
 */
int orc_fgmres(const orc_hier *H, orc_prec_fn prec, void *ctx, int m, double tol,
               int maxit, const cplx *b, cplx *x, double *hist,
               orc_fgmres_stats *st)
{
    int n = H->n[0];
    size_t N = (size_t)n * n;
    double h = H->h[0], om = H->omega;
    const double *kap = H->kappa[0], *gam = H->gamma[0];
    cplx *V = malloc((size_t)(m + 1) * N * sizeof(cplx));
    cplx *Z = malloc((size_t)m * N * sizeof(cplx));
    cplx *w = malloc(N * sizeof(cplx));
    cplx *Hm = calloc((size_t)(m + 1) * m, sizeof(cplx)); /* Hm[i*m + j] */
    cplx *cs = malloc(m * sizeof(cplx)), *sn = malloc(m * sizeof(cplx));
    cplx *g = malloc((m + 1) * sizeof(cplx)), *y = malloc(m * sizeof(cplx));
    double bnorm = vnorm(b, N);
    int its = 0, restarts = 0, conv = 0;
    double relres = 1.0;
    memset(x, 0, N * sizeof(cplx));
    if (hist) hist[0] = 1.0;
    if (bnorm == 0.0) {
        conv = 1;
        relres = 0.0;
        goto done;
    }
    for (;;) {
        /* true residual r = b - A x, start vector v_0 = r / ||r|| */
        orc_residual(n, h, om, kap, gam, 0.0, b, x, V);
        double beta = vnorm(V, N);
        relres = beta / bnorm;
        if (relres <= tol) {
            conv = 1;
            break;
        }
        if (its >= maxit)
            break;
        for (size_t p = 0; p < N; p++)
            V[p] /= beta;
        memset(g, 0, (m + 1) * sizeof(cplx));
        memset(Hm, 0, (size_t)(m + 1) * m * sizeof(cplx));
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && its < maxit; j++) {
            cplx *vj = V + (size_t)j * N, *zj = Z + (size_t)j * N;
            if (prec)
                prec(ctx, vj, zj);
            else
                orc_vcycle(H, vj, zj);
            orc_apply(n, h, om, kap, gam, 0.0, zj, w);
            for (int i = 0; i <= j; i++) {
                cplx *vi = V + (size_t)i * N;
                cplx hij = vdot(vi, w, N);
                Hm[i * m + j] = hij;
                for (size_t p = 0; p < N; p++)
                    w[p] -= hij * vi[p];
            }
            double hn = vnorm(w, N);
            Hm[(j + 1) * m + j] = hn;
            /* previous rotations, then the new one that zeroes H[j+1][j] */
            for (int i = 0; i < j; i++) {
                cplx a = Hm[i * m + j], c2 = Hm[(i + 1) * m + j];
                Hm[i * m + j] = cs[i] * a + sn[i] * c2;
                Hm[(i + 1) * m + j] = -conj(sn[i]) * a + cs[i] * c2;
            }
            cplx a = Hm[j * m + j], c2 = Hm[(j + 1) * m + j];
            double t = sqrt(cabs(a) * cabs(a) + cabs(c2) * cabs(c2));
            if (cabs(a) == 0.0) {
                cs[j] = 0.0;
                sn[j] = 1.0;
                Hm[j * m + j] = c2;
            } else {
                cplx ph = a / cabs(a);
                cs[j] = cabs(a) / t;
                sn[j] = ph * conj(c2) / t;
                Hm[j * m + j] = ph * t;
            }
            Hm[(j + 1) * m + j] = 0.0;
            g[j + 1] = -conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            its++;
            k = j + 1;
            if (hist) hist[its] = cabs(g[j + 1]) / bnorm;
            if (hn == 0.0 || cabs(g[j + 1]) / bnorm <= tol)
                break;
            for (size_t p = 0; p < N; p++)
                V[(size_t)(j + 1) * N + p] = w[p] / hn;
        }
        /* y = H_k^{-1} g_k (upper triangular), x += Z y */
        for (int i = k - 1; i >= 0; i--) {
            cplx s = g[i];
            for (int c = i + 1; c < k; c++)
                s -= Hm[i * m + c] * y[c];
            y[i] = s / Hm[i * m + i];
        }
        for (int i = 0; i < k; i++)
            for (size_t p = 0; p < N; p++)
                x[p] += y[i] * Z[(size_t)i * N + p];
        restarts++;
    }
done:
    if (st) {
        st->iterations = its;
        st->restarts = restarts;
        st->converged = conv;
        st->true_relres = relres;
    }
    free(V);
    free(Z);
    free(w);
    free(Hm);
    free(cs);
    free(sn);
    free(g);
    free(y);
    return conv ? 0 : 1;
}

/* Level-0 Helmholtz residual in the hierarchy (used by the Python wrappers). */
void orc_hier_residual_A(const orc_hier *H, const cplx *f, const cplx *x, cplx *r)
{
    orc_residual(H->n[0], H->h[0], H->omega, H->kappa[0], H->gamma[0], 0.0, f, x, r);
}
