/*
 * helm.h -- C ABI of the MI355X (gfx950) library for the discrete
 * heterogeneous 2D Helmholtz equation, solved by flexible GMRES with a
 * shifted-Laplacian (SL) multigrid preconditioner, optionally augmented by a
 * U-Net (Azulay & Treister, "Multigrid-augmented deep learning
 * preconditioners for the Helmholtz equation").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grids: an n x n array of unknowns u[i*n + j] (row-major, j fastest) on
 *    the unit square, h = 1/n, zero values outside the array (Dirichlet, the
 *    zero padding of section 2.4).  n must be even and divisible by
 *    2^(levels-1).
 *  - complex64 fields are interleaved float pairs (re, im), complex128 fields
 *    interleaved double pairs.  A batch of nrhs fields is contiguous:
 *    [nrhs][n][n][2].
 *  - Every array argument is a DEVICE pointer owned by the caller, unless a
 *    comment says "host".  The library never frees caller memory.  Handles
 *    own their internal device workspaces and release them in *_destroy.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued on it; entry points do not synchronise the device
 *    unless their comment says so.
 *  - A batch of zero fields (nrhs = 0) is a no-op that returns 0; its array
 *    pointers may then be NULL.
 *  - Return value: 0 = success, > 0 = completed with a warning
 *    (HELM_NOT_CONVERGED), < 0 = error; helm_last_error() then holds a
 *    message for the calling thread.  On error no output is guaranteed.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HELM_OK 0
#define HELM_NOT_CONVERGED 1
#define HELM_E_INVALID (-1) /* bad argument: null pointer, size, option */
#define HELM_E_NOMEM (-2)   /* device or host allocation failed        */
#define HELM_E_HIP (-3)     /* a HIP runtime call failed               */
#define HELM_E_SHAPE (-4)   /* grid size incompatible with the levels  */

#define HELM_OP_A 0 /* Helmholtz operator, eq. 2.1-2.2            */
#define HELM_OP_M 1 /* shifted-Laplacian operator, eq. 2.4        */

typedef struct helm_handle helm_handle;

/* Setup options; a NULL pointer selects every default. */
typedef struct {
    double beta;          /* SL shift beta of eq. 2.4 (alpha = 1); default 0.5   */
    double jacobi_weight; /* damped-Jacobi weight (section 4); default 0.8       */
    int levels;           /* V-cycle levels; 0 = coarsest level 64^2, or n^2 if
                             n <= 64 (default)                                   */
    int coarse_gmres;     /* coarsest-level solver: 0 = exact (dense inverse,
                             default); k in [1, 30] = k GMRES steps with the
                             Jacobi (diagonal) right preconditioner from zero,
                             then one damped Jacobi post-relaxation (the
                             setting of section 4; needs levels >= 2)          */
} helm_opts;

/*
 * helm_setup -- per-medium set-up of the multigrid hierarchy.
 * Operator (eq. 2.1-2.2, section 2.2):
 *   (A u)(i,j) = (4u(i,j) - u(i+-1,j) - u(i,j+-1)) / h^2
 *                - omega^2 kappa(i,j)^2 (1 - i gamma(i,j)) u(i,j)
 * and the SL operator M replaces gamma by gamma + beta (eq. 2.4 with
 * alpha = 1).  Level l has n/2^l points per side, mesh width 2^l h, and its
 * coefficients injected from the fine grid (re-discretisation, section 2.2).
 * The coarsest level's operator is inverted once here, in double precision
 * on the host, and stored as a dense complex64 matrix.
 *   slowness, gamma : device float [n][n]; read during the call only.
 *   omega           : angular frequency, > 0.
 *   out             : receives the handle (host pointer to a pointer).
 * This call synchronises `stream` (the coarsest coefficients are copied to
 * the host).  Errors: HELM_E_INVALID, HELM_E_SHAPE, HELM_E_NOMEM, HELM_E_HIP.
 */
int helm_setup(const float *slowness, double omega, const float *gamma, int n,
               const helm_opts *opts, void *stream, helm_handle **out);

/* Release a handle and its device memory (NULL is ignored). */
void helm_destroy(helm_handle *h);

/* Grid size of level l of the hierarchy, or -1 if l is out of range. */
int helm_level_size(const helm_handle *h, int l);

/* Number of levels of the hierarchy. */
int helm_num_levels(const helm_handle *h);

/*
 * helm_apply -- y = Op x on the fine grid for a batch (eq. 2.2, the stencil
 * applied as a 3x3 convolution plus a pointwise mass product, section 2.4).
 *   op : HELM_OP_A or HELM_OP_M.
 *   x, y : complex64 [nrhs][n][n]; must not overlap.
 */
int helm_apply(helm_handle *h, int op, const float *x, float *y, int nrhs,
               void *stream);

/*
 * helm_sl_vcycle -- v = V-cycle(0, f) on M (Algorithm 1): one damped Jacobi
 * pre- and post-relaxation per level, full-weighting restriction and
 * bilinear prolongation (eq. 2.9), the direct solve on the coarsest level.
 * This is the SL preconditioner M_V.
 *   f, v : complex64 [nrhs][n][n]; must not overlap.
 */
int helm_sl_vcycle(helm_handle *h, const float *f, float *v, int nrhs, void *stream);

/*
 * helm_sl_vcycle_noalloc -- helm_sl_vcycle for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same result as helm_sl_vcycle (same
 * kernels in the same order), but the cycle's workspace (restricted
 * right-hand sides and corrections of every level below the finest, partial
 * sums of the coarsest-level solve) is carved from a fixed 64 MiB device
 * array of the library instead of the handle's allocations.  The call itself
 * allocates nothing; the array of each device exists from library load to
 * process end, and its address is looked up the first time the call runs on
 * that device.  The caller still owns f and v.
 *   f, v : complex64 [nrhs][n][n]; must not overlap.
 * Limit: helm_sl_vcycle_noalloc_bytes(h, nrhs) <= 64 MiB (about 11
 * right-hand sides at 1024^2, 45 at 512^2); larger batches return
 * HELM_E_INVALID without launching anything.  Calls on one device share the
 * array: calls that overlap in time on one device (other streams or
 * threads) race, so serialise them.  Launches of this call are not timed by
 * the profiling hook.
 */
int helm_sl_vcycle_noalloc(helm_handle *h, const float *f, float *v, int nrhs, void *stream);
/* Workspace bytes helm_sl_vcycle_noalloc needs for nrhs fields of medium h,
 * and the fixed maximum. */
size_t helm_sl_vcycle_noalloc_bytes(const helm_handle *h, int nrhs);
size_t helm_sl_vcycle_noalloc_max_bytes(void);

/* Preconditioners for helm_fgmres_solve. */
#define HELM_PREC_SL 0        /* M_V: one SL V-cycle                           */
#define HELM_PREC_UNET_CGC 1  /* M_CU: Jacobi, U-Net coarse correction, Jacobi */
#define HELM_PREC_UNET_DEFL 2 /* M_VU: U-Net, then an SL V-cycle (eq. 3.4)     */

typedef struct {
    int m;               /* Krylov subspace size per cycle; default 20           */
    double tol;          /* target true relative residual; default 1e-7          */
    int maxit;           /* maximum preconditioner applications; default 20000   */
    int prec;            /* HELM_PREC_*; default HELM_PREC_SL                    */
    void *net;           /* unet_net* for the U-Net preconditioners, else NULL   */
    double stall_ratio;  /* fall back to M_V when |g_{j+1}|/|g_j| exceeds this on
                            3 consecutive steps (0 = never); default 0           */
    int graph;           /* 1: capture each restart cycle (m Arnoldi steps with
                            their preconditioner applications, the update of x
                            and the true residual) into a HIP graph once and
                            replay it; default 0.  Ignored while the profiling
                            hook is active.                                      */
    void *encoder;       /* unet_net* encoder of an encoder-solver `net`, or
                            NULL.  Given, each problem's medium is encoded
                            (unet_pair_encode_medium) right before its solve,
                            so one call takes any number of media; without it
                            the solver must hold the one problem's context.  */
} helm_fgmres_opts;

typedef struct {
    int iterations;      /* preconditioner applications                          */
    int restarts;        /* completed FGMRES cycles                              */
    int converged;       /* 1 if the true relative residual reached tol          */
    int fallback;        /* nonzero if the solve switched to the plain SL
                            V-cycle: 1 after a stalled residual reduction, 2
                            after a non-finite preconditioned direction (that
                            step is dropped and its cycle ends)                  */
    double true_relres;  /* final ||b - A x|| / ||b|| recomputed in FP64         */
    /* Convergence factor of eq. 4.1, rho = (||r_T|| / ||r_0||)^(1/T), with T
       the first iteration whose implicit residual is reduced 1e6 (1e7) times
       from ||b||; if that never happens, T = iterations and ||r_T|| is the
       final true residual. */
    int its_1e6, its_1e7;
    double rho_1e6, rho_1e7;
} helm_fgmres_stats;

/*
 * helm_fgmres_solve -- restarted flexible GMRES (section 3, FGMRES(m) with
 * right preconditioning, eq. 2.5) for a batch of independent right-hand
 * sides on one or more media.
 *   probs[p]         : handle of medium p, p < nprob.
 *   rhs_per_prob[p]  : host int, number of right-hand sides of medium p.
 *   b[p]             : complex64 [rhs_per_prob[p]][n_p][n_p], device.
 *   x[p]             : complex128 [rhs_per_prob[p]][n_p][n_p], device;
 *                      output (overwritten; the iteration starts from 0).
 *   stats            : host array with one entry per right-hand side, in
 *                      problem order; may be NULL.
 * The Krylov vectors are complex64 with FP64-accumulated inner products;
 * the Hessenberg least-squares problem, the solution and the true residual
 * b - A x that starts each cycle are FP64.  The iteration stops when that
 * true relative residual is <= tol.  The host synchronises once per cycle.
 * Problems with distinct handles run concurrently on internal streams (one
 * host thread each, up to 8), which fills the GPU when the batch holds many
 * small or uneven grids; the call waits on `stream` first and `stream` waits
 * on all of them before the call returns.  Problems are solved one after
 * another when a network preconditioner is used (the network's workspace is
 * shared) or while the profiling hook is active.
 * Returns HELM_NOT_CONVERGED if some right-hand side reached maxit first.
 */
int helm_fgmres_solve(helm_handle *const *probs, int nprob, const int *rhs_per_prob,
                      const float *const *b, double *const *x,
                      const helm_fgmres_opts *opts, helm_fgmres_stats *stats,
                      void *stream);

/*
 * helm_block_fgmres_solve -- block restarted flexible GMRES(m) (the solver
 * of the paper's experiments, section 4: Calandra et al., block size 10,
 * m = 10) on one medium: the nrhs right-hand sides are taken in blocks of
 * `block` consecutive fields (the last block may be smaller), and the
 * fields of a block share one block Krylov space.  Per block and cycle:
 * R = B - A X in FP64 (stored complex64) = V_0 beta by Cholesky QR applied
 * twice; each step applies the preconditioner to the block (M_V, M_CU or
 * M_VU as in helm_fgmres_solve), W = A Z_j, two classical block
 * Gram-Schmidt passes and Cholesky QR twice; the block Hessenberg
 * least-squares problem is solved in FP64 by Householder QR; X (complex128)
 * += Z Y at the cycle's end or when every column's estimate is below tol.
 * Gram entries accumulate in FP64 in a fixed order.
 *   b : complex64 [nrhs][n][n];  x : complex128 [nrhs][n][n] (output).
 *   opts : m, tol, maxit (block steps), prec, net as for helm_fgmres_solve
 *          (stall_ratio, graph and encoder are ignored); NULL = m 10,
 *          tol 1e-7, maxit 20000, M_V.  (m + 1) block^2 <= 4096, block <= 16.
 *   stats : host array [nrhs]; iterations = block steps of that field's
 *          block; rho per column from the block least-squares residual.
 * Synchronises `stream` once per block step and once per cycle start.
 * A block whose residual block is rank-deficient at a cycle start (a zero
 * right-hand side, or fields with linearly dependent residuals) cannot be
 * factored by Cholesky QR: its fields are then solved again from zero one
 * at a time (block size 1; their stats count only that solve).  Returns
 * HELM_NOT_CONVERGED if a field misses tol within maxit steps.
 */
int helm_block_fgmres_solve(helm_handle *h, int nrhs, const float *b, double *x, int block,
                            const helm_fgmres_opts *opts, helm_fgmres_stats *stats, void *stream);

/*
 * helm_training_triples -- supervised training data (section 3.4, eq.
 * 3.8-3.9 with a single flexible-GMRES step): for given x,
 *   b = A x,  z = M_V(b) (one SL V-cycle),  alpha = (Az)^H b / |Az|^2,
 *   r = b - alpha A z  (the residual of x~ = alpha z),  e = x - alpha z,
 * so that A e = r up to rounding.  The random x is an input.
 *   x, r, e : complex64 [nrhs][n][n]; r and e are outputs; no overlap.
 */
int helm_training_triples(helm_handle *h, const float *x, float *r, float *e, int nrhs,
                          void *stream);

/*
 * helm_training_triples_seeded -- training triples with the random x
 * drawn on the device from (seed, sample index), so that a training run is
 * reproducible from its seed and the index of its next sample (section 3.4
 * draws x at random; eq. 3.8), and a chosen number of smoothing steps.
 * Sample b of the call has index index0 + b.
 * Its point p takes the Philox4x32-10 block (Salmon et al., SC 2011) of
 * counter (p, index_lo, index_hi, 0) under key (seed_lo, seed_hi); the
 * first two 32-bit words a, c give u1 = (a + 1) 2^-32 and u2 = c 2^-32, and
 * the Box-Muller transform in double precision gives
 *   Re x = sqrt(-2 ln u1) cos(2 pi u2),  Im x = sqrt(-2 ln u1) sin(2 pi u2),
 * each rounded once to float: iid N(0, 1) real and imaginary parts.
 *   ksteps : k, the number of FGMRES steps of eq. 3.8 (the paper draws k from
 *          1..10 per sample; here one k per call), in [1, 30].  k = 1 is the
 *          closed form of helm_training_triples.  k > 1: FGMRES(max(k, 10))
 *          with M_V from zero on b = A x, stopped after k steps (no restart
 *          for k <= 10), the iterate x~ in FP64; r = b - A x~ evaluated in
 *          FP64, e = x - x~, both rounded once.  This uses the handle's FGMRES
 *          workspace (a later solve with another restart length reallocates
 *          it) and synchronises `stream` once.
 *   x    : complex64 [nrhs][n][n] receiving the drawn x, or NULL (kept in the
 *          handle's workspace only).
 *   r, e : as for helm_training_triples.
 * The handle keeps a workspace of 4 nrhs complex64 fields for these calls
 * (grown on demand, released by helm_destroy); calls on one handle must not
 * overlap.
 */
int helm_training_triples_seeded(helm_handle *h, unsigned long long seed, unsigned long long index0,
                                 int ksteps, float *x, float *r, float *e, int nrhs, void *stream);

/*
 * helm_training_triples_batch -- a batch of seeded training triples, each
 * sample with its own index and its own number of FGMRES steps (section 3.4
 * draws k from 1..10 per sample; eq. 3.8).  Sample b draws x from (seed,
 * index[b]) exactly as helm_training_triples_seeded draws sample index[b],
 * and takes ksteps[b] steps of one FGMRES(max(max_b ksteps[b], 10)) with M_V
 * from zero on b = A x that advances all samples together (sample b leaves
 * after its k steps); x~, r = b - A x~ and e = x - x~ as there (k = 1 too
 * goes through FGMRES here, not through the closed form).
 *   index  : host array of nrhs sample indices;
 *   ksteps : host array of nrhs step counts, each in [1, 30];
 *   x, r, e: as for helm_training_triples_seeded.
 * Uses the handle's triple and FGMRES workspaces, synchronises `stream`;
 * calls on one handle must not overlap.
 */
int helm_training_triples_batch(helm_handle *h, unsigned long long seed, const unsigned long long *index,
                                const int *ksteps, float *x, float *r, float *e, int nrhs, void *stream);

/*
 * helm_triples_mix -- augmentation by linear combinations of triples
 * (section 3.4): for nin triples (r_j, e_j) of ONE medium (A e_j = r_j),
 *   r'_b = sum_j c[b][j] r_j,   e'_b = sum_j c[b][j] e_j,   b < nout,
 * which again satisfy A e'_b = r'_b.  FP32 arithmetic, sums in j order.
 *   r, e         : complex64 [nin][npts] inputs;
 *   coef         : device float [nout][nin] real coefficients;
 *   r_out, e_out : complex64 [nout][npts]; must not overlap the inputs.
 * nin, nout <= 32.
 */
int helm_triples_mix(const float *r, const float *e, int nin, long long npts, const float *coef, int nout,
                     float *r_out, float *e_out, void *stream);

/* Slowness injected at the coarse points (2I, 2J): float [n/2][n/2] (the
 * network's kappa input channel). */
int helm_coarse_slowness(helm_handle *h, float *kc, void *stream);

/*
 * Kernel timing hook (measurement support, not part of the method).  While
 * active, the library records a HIP event pair on the launch stream around
 * every launch of the kernel families in the mask (bit 1 << family), and sums
 * the algorithmic work of each launch: the bytes the operation must move
 * once (sweeps, Gram-Schmidt, coarse solve) or its FLOPs counted as 2 per
 * multiply-add over the real (unpadded) channels (convolutions).  Work of
 * kernels that skip converged right-hand sides counts the right-hand sides
 * active at the start of the current restart cycle.
 * helm_profile_read synchronises on a family's events and returns its summed
 * device time, launch count and work; the records stay until the next
 * helm_profile_start.  helm_profile_stop ends recording.  The hook is
 * process-wide; concurrent solves on several threads share it.
 * helm_profile_sample(k), k >= 1 (default 1): only about one launch in k
 * of each family is timed, chosen by a fixed hash of the launch's index
 * since helm_profile_start (so that the subset does not alias with a
 * repeated sequence of launches), and the launch count and work cover those
 * launches only (each event costs a few microseconds of queue time between
 * kernels).  The events carry no system-scope fence:
 * they serve timing only.
 */
#define HELM_PROF_NONE 0
#define HELM_PROF_COARSE 1 /* dense coarsest-level solve (bytes)              */
#define HELM_PROF_DOWN 2   /* fused pre-smooth + residual + restriction (bytes) */
#define HELM_PROF_UP 3     /* fused prolongation + post-smooth (bytes)        */
#define HELM_PROF_CGS 4    /* the Gram-Schmidt passes of an Arnoldi step (bytes) */
#define HELM_PROF_APPLY 5  /* stencil apply (bytes)                           */
#define HELM_PROF_CONV 6   /* 3x3 convolutions, forward and data gradient (FLOPs) */
#define HELM_PROF_WGRAD 7  /* 3x3 convolution weight gradients (FLOPs)        */
int helm_profile_start(unsigned family_mask);
int helm_profile_read(int family, double *total_ms, long long *launches, double *work);
int helm_profile_stop(void);
int helm_profile_sample(int every);

/*
 * Launch-shape autotuner of the network convolutions.  With enable = 1, the
 * first convolution of each new shape (batch, height, width, input and output
 * channels, epilogue) times the candidate tile heights and workgroup counts
 * with HIP events on its stream and keeps the fastest for later calls of that
 * shape (calls under graph capture use the table or the built-in heuristic).
 * 0 returns to the heuristic, keeping the table; -1 also clears it.
 * Returns the previous setting.  helm_autotune_entries: shapes tuned so far.
 */
int helm_autotune(int enable);
int helm_autotune_entries(void);
/*
 * Test hook: force one candidate launch shape of the tuner on every
 * convolution (forward and data gradient) until called with kind < 0.
 *   kind   : 0 = the 256-thread register-staged kernel, 1 = the 512-thread
 *            direct-to-LDS kernel (a convolution whose first source is read
 *            through the x2 upsampling always runs on kind 1);
 *   mf     : 2 or 4 (tile heights 8 / 16 rows for kind 0, 16 / 32 for kind 1);
 *   per_cu : workgroups per compute unit, 1..64 (the tuner tries 1, 2, 4, 8).
 * Every candidate computes the same result in the same summation order; the
 * hook lets tests check each against the oracle.  Returns HELM_E_INVALID for
 * a shape outside these ranges.  Process-wide.
 */
int helm_autotune_force(int kind, int mf, int per_cu);

/*
 * Allocator hook.  Every device workspace the library owns (handles, FGMRES
 * solves, networks, the training-triple generator) is obtained from
 *   alloc(bytes, ctx)            -> device pointer, NULL on failure
 * and returned through
 *   release(ptr, bytes, ctx)
 * (for example a caching allocator of the host framework), instead of
 * hipMalloc / hipFree.  Both functions, or neither (NULL, NULL: back to
 * hipMalloc / hipFree), must be given; ctx is passed through.  A block goes
 * back to the allocator it came from even after the registration changes.
 * The library synchronises the device before handing a block to `release`
 * (its kernels may still read it on internal streams).  The functions may be
 * called from the library's internal host threads (concurrent problems of
 * helm_fgmres_solve), one at a time per call site.  Process-wide; register
 * before creating handles or networks.  The fixed array of
 * helm_sl_vcycle_noalloc is not covered (it is never allocated).
 */
typedef void *(*helm_alloc_fn)(size_t bytes, void *ctx);
typedef void (*helm_free_fn)(void *ptr, size_t bytes, void *ctx);
int helm_set_allocator(helm_alloc_fn alloc, helm_free_fn release, void *ctx);
/* Bytes of device memory the library currently holds (all allocators). */
size_t helm_allocated_bytes(void);

/* Thread-local text describing the last error of this thread ("" if none). */
const char *helm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H */
