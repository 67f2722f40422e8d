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
void launch_down(const Level &L, float shift, float w, const float2 *f, size_t fs,
                 float2 *fc, size_t fcs, int nb, const int *active, hipStream_t s);

// Fused prolongation + correction + post-relaxation:
//   v' = w D^-1 f + P vc,  v = v' + w D^-1 (f - Op v')
void launch_up(const Level &L, float shift, float w, const float2 *f, size_t fs,
               const float2 *vc, size_t vcs, float2 *v, size_t vs, int nb,
               const int *active, hipStream_t s);

// v = X f with the dense coarsest-level inverse X (N x N complex64, row-major).
void launch_coarse_solve(const float2 *X, int N, const float2 *f, size_t fs, float2 *v,
                         size_t vs, int nb, const int *active, hipStream_t s);

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
int krylov_nblk(size_t N);

// partial[b][blk][i] = sum over the block's points of conj(V_i) w, i < nv.
void launch_dots(const float2 *V, size_t vstride_b, size_t N, const float2 *w,
                 size_t ws, int nv, double2 *partial, int nblk, int nb, const int *active,
                 hipStream_t s);
// w -= sum_i h_i V_i (h from hcoef[b][i]); then partial dots conj(V_i) w (mode 0)
// or partial |w|^2 (mode 1).
void launch_update(const float2 *V, size_t vstride_b, size_t N, float2 *w, size_t ws,
                   int nv, const double2 *hcoef, int hstride, int mode, double2 *partial,
                   int nblk, int nb, const int *active, hipStream_t s);
void launch_scale(float2 *w, size_t ws, size_t N, const double *scale, int nb,
                  const int *active, hipStream_t s);
void launch_xupdate(double2 *x, size_t xs, const float2 *Z, size_t zstride_b, size_t N,
                    const double2 *y, int ystride, const int *kcount, int nb,
                    const int *active, hipStream_t s);

}  // namespace helm
