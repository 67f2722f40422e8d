// Per-medium handle of libhelm (internal).
#pragma once

#include <vector>

#include "helm_internal.h"

struct unet_net;

struct helm_handle {
    int n = 0;
    int levels = 0;
    double omega = 0.0;
    double beta = 0.5;
    double jacobi_w = 0.8;
    int coarse_gmres = 0;      // 0: dense inverse Xc; k > 0: GMRES(k) + Jacobi (coarse_gmres.hip)
    float *kappa0 = nullptr;   // fine slowness copy (float [n][n])
    float *gamma0 = nullptr;   // fine attenuation copy (float [n][n])
    std::vector<helm::Level> lv;
    float2 *Xc = nullptr;      // dense inverse of the coarsest shifted operator
    int Nc = 0;                // coarsest unknowns
    // V-cycle workspace: per level l >= 1, f_l and v_l for `ws_nb` fields
    int ws_nb = 0;
    int ws_gen = 0;  // bumped on every reallocation (captured graphs hold the pointers)
    std::vector<float2 *> wf, wv;
    float2 *cpart = nullptr;   // partial sums of the coarsest-level GEMM
    // FGMRES workspace (see fgmres.hip)
    void *fg = nullptr;
    // training-triple workspace (train_data.hip): A z and the x drawn by the
    // seeded generator for `tw_nb` fields, FP64 partial sums
    int tw_nb = 0;
    float2 *tw = nullptr, *tx = nullptr;
    double *tpart = nullptr;
    double2 *txt = nullptr;  // the k-step FGMRES iterate x~ (complex128)
    float *kcoarse = nullptr;  // slowness at the coarse points, [n/2][n/2] (encoder input)
};

namespace helm {
// Workspace of one V-cycle over nb fields: per level l >= 1 the restricted
// right-hand side f_l and the correction v_l ([nb][n_l][n_l] each), and the
// workspace of the coarsest solve (coarse_ws(h, nb)).
struct VcycleWs {
    static constexpr int MAXL = 12;
    float2 *wf[MAXL] = {}, *wv[MAXL] = {};
    float2 *cpart = nullptr;
};
// complex elements of a VcycleWs carved from one buffer, and the carving
size_t vcycle_ws_elems(const helm_handle *h, int nb);
// complex elements of the coarsest solve's workspace (GEMM partial sums, or
// the GMRES vectors of a GMRES coarsest solver) for nb fields
size_t coarse_ws(const helm_handle *h, int nb);
void vcycle_carve(const helm_handle *h, int nb, float2 *base, VcycleWs &ws);
// the V-cycle on a given workspace: kernel launches only (no allocation)
void vcycle_with(helm_handle *h, const VcycleWs &ws, const float2 *f, size_t fs, float2 *v, size_t vs,
                 int nb, const int *active, hipStream_t s, const double *scale = nullptr,
                 int accumulate = 0);
int ensure_vcycle_ws(helm_handle *h, int nb);
// v = V-cycle(0, f) on M, batch of nb fields (strides in complex elements);
// with `scale` the input is read as scale[b] * f (the cycle is linear).
int vcycle(helm_handle *h, const float2 *f, size_t fs, float2 *v, size_t vs, int nb,
           const int *active, hipStream_t s, const double *scale = nullptr, int accumulate = 0);
void fgmres_free(helm_handle *h);
// FGMRES(m) of one problem with nb right-hand sides (fgmres.hip); x is
// complex128 [nb][n][n] and starts from zero.  maxit_rhs (host, nb ints, or
// null): an iteration limit per right-hand side in place of maxit.
int fgmres_one(helm_handle *h, int nb, const float2 *b, double2 *x, int m, double tol, int maxit, int prec,
               unet_net *net, double stall_ratio, helm_fgmres_stats *stats, hipStream_t s, bool use_graph,
               const int *maxit_rhs = nullptr);
}  // namespace helm
