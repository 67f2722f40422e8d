// Internal declarations shared by the translation units of libhelm.
// Not part of the public ABI (include/helm.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/helm.h"

namespace helm {

void set_error(const std::string &msg);
// Device memory of the library's workspaces (alloc.hip): through the
// allocator registered with helm_set_allocator, else hipMalloc / hipFree.
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t dev_free(void *p);
template <typename T>
inline hipError_t dev_malloc(T **p, size_t bytes)
{
    return dev_malloc(reinterpret_cast<void **>(p), bytes);
}
// Timing hook (prof.hip): event on stream s at the start/end of a family's launch.
// work_per_rhs x nb (or x the active right-hand sides when masked) is added
// to the family's algorithmic work when the stop mark is recorded
void prof_mark(int family, hipStream_t s, bool start, double work_per_rhs = 0.0, int nb = 1,
               bool masked = false);
void prof_set_active(int nact);
bool prof_enabled();
// suspend (true) / resume (false) timing of this thread's launches
void prof_suspend(bool on);

#define HELM_HIP_CHECK(call)                                                        \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            ::helm::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
            return HELM_E_HIP;                                                      \
        }                                                                           \
    } while (0)

// ---------------------------------------------------------------- sweeps
// All grid kernels take a batch of fields: field b starts at ptr + b*stride
// (stride in complex elements).  `active` (may be null) masks batch entries.

struct Level {
    int n;          // points per side
    float ih2;      // 1 / h_l^2
    float2 *mass;   // omega^2 kappa^2 (1 - i gamma), complex64 [n][n]
};

// y = Op x with Op = A (shift 0) or the shifted operator (shift beta).
void launch_apply(const Level &L, float shift, const float2 *x, size_t xs, float2 *y,
                  size_t ys, int nb, const int *active, hipStream_t s);

// Fused pre-relaxation from zero + residual + full-weighting restriction:
//   v = w D^-1 f,  fc = R (f - Op v)
// With `scale` (per batch entry, may be null) the input is read as scale[b] * f.
void launch_down(const Level &L, float shift, float w, const float2 *f, size_t fs,
                 float2 *fc, size_t fcs, int nb, const int *active, hipStream_t s,
                 const double *scale = nullptr);

// Fused prolongation + correction + post-relaxation:
//   v' = w D^-1 f + P vc,  v = v' + w D^-1 (f - Op v')
// `scale` as for launch_down; with `accumulate` the result is added to v.
void launch_up(const Level &L, float shift, float w, const float2 *f, size_t fs,
               const float2 *vc, size_t vcs, float2 *v, size_t vs, int nb,
               const int *active, hipStream_t s, const double *scale = nullptr,
               int accumulate = 0);

// v = X f with the dense coarsest-level inverse X (N x N complex64, row-major).
// `scale` as for launch_down; with `accumulate` the result is added to v.
// `scratch` (coarse_scratch(N, nb) complex, may be null): with four or more
// right-hand sides the product runs as a tiled GEMM reading X once.
size_t coarse_scratch(int N, int nb);
void launch_coarse_solve(const float2 *X, int N, const float2 *f, size_t fs, float2 *v,
                         size_t vs, int nb, const int *active, hipStream_t s,
                         const double *scale = nullptr, int accumulate = 0, float2 *scratch = nullptr);

// Coarsest solve by k GMRES steps with the Jacobi right preconditioner from
// zero, then one damped Jacobi sweep (weight w) on the shifted operator;
// one workgroup per field; `work` holds coarse_gmres_elems(N, k, nb)
// complex values.  HELM_E_INVALID when k or the grid is out of range.
size_t coarse_gmres_elems(int Nc, int k, int nb);
int launch_coarse_gmres(const Level &L, float shift, float w, int k, const float2 *f, size_t fs, float2 *v,
                        size_t vs, int nb, const int *active, hipStream_t s, float2 *work);

// mode 0: y = f - Op x;  mode 1: y = x + w D^-1 (f - Op x);  mode 2: y = w D^-1 f.
// With fscale, field b of f is read as fscale[b] f_b.
void launch_resjac(const Level &L, float shift, float w, int mode, const float2 *x, size_t xs,
                   const float2 *f, size_t fs, float2 *y, size_t ys, int nb, const int *active,
                   hipStream_t s, const double *fscale = nullptr);

// Level-l coefficients by injection from the fine fields, computed in double
// and rounded once: mass = omega^2 kappa^2 (1 - i gamma) at (2^l I, 2^l J).
void launch_level_mass(const float *kappa, const float *gamma, int n, int stride_pow,
                       double omega, float2 *mass, int nl, hipStream_t s);

// FP64 true residual r = b - A x (x complex128), stored complex64 unscaled,
// with per-block partial sums of |r|^2 in FP64.
void launch_true_residual(const float *kappa, const float *gamma, int n, double omega,
                          const float2 *b, size_t bs, const double2 *x, size_t xs,
                          float2 *r, size_t rs, double *partial, int nblk, int nb,
                          const int *active, hipStream_t s);

// ---------------------------------------------------------------- krylov
constexpr int MAXM = 30;              // largest Krylov subspace per cycle
constexpr int MAXV = 32;              // per-right-hand-side coefficient storage
constexpr int MAXP = 2 * MAXM + 4;    // partial sums per block of an Arnoldi pass

// Per-right-hand-side FGMRES state in device memory (struct of arrays).
struct FgState {
    int m, nb;
    int *active, *incycle, *k, *its;
    int *fallback, *stall;     // sticky switch to the plain SL V-cycle (1: stalled,
                               // 2: non-finite preconditioned direction), stall counter
    int *mask_net, *mask_sl;   // per-step masks: network path / SL path
    int *t6, *t7;              // first iteration whose implicit residual is <= 1e-6 / 1e-7 of ||b||
    double stall_ratio;        // 0 = never fall back
    double *bnorm, *beta, *relres, *scale, *nu;
    double *rel6, *rel7;       // implicit relative residual at t6 / t7
    double2 *H;   // [nb][(m+1)*m], H[i*m + j]
    double2 *g;   // [nb][m+1]
    double *cs;   // [nb][m]
    double2 *sn;  // [nb][m]
    double2 *hc;  // [nb][MAXV] projection coefficients of the current step
    double2 *ac;  // [nb][MAXV] delayed re-orthogonalisation coefficients
    double2 *y;   // [nb][MAXV]
    double tol;
    int maxit;
    const int *maxit_rhs;  // per right-hand side iteration limits (device), or null: maxit for all
};

// Workgroups per right-hand side of the Krylov reductions for nb
// right-hand sides of N points (never more than for nb = 1).
int krylov_nblk(size_t N, int nb);

// One Arnoldi step j (delayed CGS2): pass A (inner products), reduction with
// the Givens update of Hessenberg column j and the stop test, pass B (final
// v_j and the next candidate).  V[b] holds m+1 vectors of N points; slot j
// holds the candidate, slot j+1 holds w = A z_j.
void launch_arnoldi_step(const FgState &S, float2 *V, size_t vsb, size_t N, int j,
                         double2 *partial, int nblk, hipStream_t s);
// mask_net = active && !fallback, mask_sl = active && (fallback || !use_net)
void launch_masks(const FgState &S, int use_net, hipStream_t s);
void launch_xupdate(double2 *x, size_t xs, const float2 *Z, size_t zstride_b, size_t N,
                    const double2 *y, int ystride, const int *kcount, int nb,
                    const int *active, hipStream_t s);

}  // namespace helm
