// Restarted flexible GMRES driver (FGMRES(m), Saad 1993, as used in section
// 3 and section 4 with right preconditioning, eq. 2.5) over a batch of
// independent right-hand sides.
//
// Per cycle and right-hand side b:
//   r = b - A x (FP64, x complex128), beta = ||r||, v_0 = r / beta
//   for j < m:  z_j = Prec(v_j); w = A z_j;
//               orthogonalise w against v_0..v_j (delayed CGS2, krylov.hip),
//               Hessenberg column j, complex Givens rotation on it (FP64),
//               g_{j+1} = implicit residual
//   x += Z y with y = H_k^-1 g_k (FP64)
// The iteration stops once the FP64 true relative residual ||b - A x||/||b||
// is <= tol; the implicit estimate |g_{j+1}| only ends a cycle early.
// Right-hand sides that have stopped are masked out of every kernel.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "handle.h"
#include "unet_net.h"

namespace helm {

namespace {

struct FgWork {
    int nb = 0, m = 0;
    size_t N = 0;
    float2 *V = nullptr, *Z = nullptr;
    double2 *partial = nullptr;
    double *rpartial = nullptr;
    void *state = nullptr;
    size_t state_bytes = 0;
    int *h_i = nullptr;       // pinned: active flags
    double *h_d = nullptr;    // pinned: relres
    int *h_its = nullptr;     // pinned: iteration counts
    int *h_fb = nullptr;      // pinned: fallback flags
    int *h_a = nullptr;       // pinned: active flags read inside a restart cycle
    int *h_net = nullptr;     // pinned: network batch [idx | pos]
    int *h_mx = nullptr;      // pinned: per right-hand side iteration limits
    int *d_mx = nullptr;      // device copy of h_mx (in the state block)
    int *d_net = nullptr;     // device copy of h_net
    float2 *t1 = nullptr, *t2 = nullptr;  // network-preconditioner scratch
    FgState S{};
    // captured restart cycles, replayed while the key matches
    struct Graph {
        const void *b = nullptr, *x = nullptr, *net = nullptr;
        int nb = 0, nnet = 0, prec = 0, hgen = 0, ngen = 0;
        double tol = 0.0, stall = 0.0;
        int maxit = 0;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    hipStream_t cap = nullptr;  // capture stream (capture needs a non-null stream)
};

__device__ __forceinline__ double2 dmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// y = R^-1 g on the rotated (upper triangular) Hessenberg matrix: one
// wavefront per right-hand side, lane t owns row t; column-oriented back
// substitution with the pivot value broadcast from its lane.
__global__ __launch_bounds__(64) void k_solve_y(FgState S)
{
    const int b = blockIdx.x;
    if (!S.incycle[b]) return;
    const int m = S.m, k = S.k[b], t = threadIdx.x;
    const double2 *H = S.H + (size_t)b * (m + 1) * m;
    double2 hrow[MAXV];
    double2 s = make_double2(0.0, 0.0);
    if (t < k) s = S.g[(size_t)b * (m + 1) + t];
#pragma unroll
    for (int c = 0; c < MAXV; ++c)
        hrow[c] = (t < k && c < k) ? H[t * m + c] : make_double2(0.0, 0.0);
    double2 yv = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = MAXV - 1; i >= 0; --i) {
        if (i < k) {
            double2 mine = make_double2(0.0, 0.0);
            if (t == i) {
                double2 d = hrow[i];
                double den = d.x * d.x + d.y * d.y;
                mine = make_double2((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den);
                yv = mine;
            }
            double2 yi = make_double2(__shfl(mine.x, i, 64), __shfl(mine.y, i, 64));
            if (t < i) {
                double2 q = dmul(hrow[i], yi);
                s.x -= q.x;
                s.y -= q.y;
            }
        }
    }
    if (t < k) S.y[(size_t)b * MAXV + t] = yv;
}

// beta = ||r|| from the true-residual partial sums; first call sets ||b||.
__global__ void k_restart(FgState S, const double *__restrict__ rpartial, int nblk, int first)
{
    const int b = blockIdx.x;
    if (!first && !S.incycle[b]) return;
    __shared__ double red[4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double s = 0.0;
    for (int q = threadIdx.x; q < nblk; q += 256) s += rpartial[(size_t)b * nblk + q];
    s = wave_sum(s);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double beta = sqrt((red[0] + red[1]) + (red[2] + red[3]));
    if (first) {
        S.bnorm[b] = beta;
        S.its[b] = 0;
    }
    S.beta[b] = beta;
    S.relres[b] = S.bnorm[b] > 0.0 ? beta / S.bnorm[b] : 0.0;
    S.g[(size_t)b * (S.m + 1)] = make_double2(beta, 0.0);
    S.scale[b] = beta > 0.0 ? 1.0 / beta : 0.0;
    S.k[b] = 0;
}

template <typename T>
int dalloc(T **p, size_t count)
{
    if (dev_malloc((void **)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        set_error("helm_fgmres_solve: device allocation failed");
        return HELM_E_NOMEM;
    }
    return HELM_OK;
}

void work_free(FgWork *w)
{
    if (!w) return;
    dev_free(w->V);
    dev_free(w->Z);
    dev_free(w->partial);
    dev_free(w->rpartial);
    dev_free(w->state);
    dev_free(w->t1);
    dev_free(w->t2);
    dev_free(w->d_net);
    for (auto &g : w->graphs) hipGraphExecDestroy(g.exec);
    if (w->cap) hipStreamDestroy(w->cap);
    if (w->h_net) hipHostFree(w->h_net);
    if (w->h_mx) hipHostFree(w->h_mx);
    if (w->h_fb) hipHostFree(w->h_fb);
    if (w->h_a) hipHostFree(w->h_a);
    if (w->h_i) hipHostFree(w->h_i);
    if (w->h_d) hipHostFree(w->h_d);
    if (w->h_its) hipHostFree(w->h_its);
    delete w;
}

int work_ensure(helm_handle *h, int nb, int m, bool scratch, FgWork **out)
{
    FgWork *w = (FgWork *)h->fg;
    size_t N = (size_t)h->n * h->n;
    if (w && w->nb >= nb && w->m == m && w->N == N && (!scratch || w->t1)) {
        *out = w;
        return HELM_OK;
    }
    if (w && w->t1) scratch = true;
    work_free(w);
    h->fg = nullptr;
    w = new FgWork();
    w->nb = nb;
    w->m = m;
    w->N = N;
    int nblk = krylov_nblk(N, 1);  // the most any batch uses
    int rc;
    if ((rc = dalloc(&w->V, (size_t)nb * (m + 1) * N)) || (rc = dalloc(&w->Z, (size_t)nb * m * N)) ||
        (rc = dalloc(&w->partial, (size_t)nb * nblk * MAXP)) ||
        (rc = dalloc(&w->rpartial, (size_t)nb * nblk))) {
        work_free(w);
        return rc;
    }
    // state: ints, then doubles, then double2s, each section 256-byte aligned
    auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t ni = 11 * (size_t)nb, nd = 7 * (size_t)nb + (size_t)nb * m;
    size_t nz = (size_t)nb * ((m + 1) * m + (m + 1) + m + 3 * MAXV);
    size_t off_d = align(ni * sizeof(int)), off_z = align(off_d + nd * sizeof(double));
    size_t bytes = off_z + nz * sizeof(double2);
    if (dev_malloc(&w->state, bytes) != hipSuccess) {
        work_free(w);
        set_error("helm_fgmres_solve: device allocation failed");
        return HELM_E_NOMEM;
    }
    w->state_bytes = bytes;
    char *p = (char *)w->state;
    FgState &S = w->S;
    S.m = m;
    S.nb = nb;
    S.active = (int *)p;
    S.incycle = S.active + nb;
    S.k = S.incycle + nb;
    S.its = S.k + nb;
    S.fallback = S.its + nb;
    S.stall = S.fallback + nb;
    S.mask_net = S.stall + nb;
    S.mask_sl = S.mask_net + nb;
    S.t6 = S.mask_sl + nb;
    S.t7 = S.t6 + nb;
    w->d_mx = S.t7 + nb;
    S.maxit_rhs = nullptr;
    S.bnorm = (double *)(p + off_d);
    S.beta = S.bnorm + nb;
    S.relres = S.beta + nb;
    S.scale = S.relres + nb;
    S.nu = S.scale + nb;
    S.rel6 = S.nu + nb;
    S.rel7 = S.rel6 + nb;
    S.cs = S.rel7 + nb;
    S.H = (double2 *)(p + off_z);
    S.g = S.H + (size_t)nb * (m + 1) * m;
    S.sn = S.g + (size_t)nb * (m + 1);
    S.hc = S.sn + (size_t)nb * m;
    S.ac = S.hc + (size_t)nb * MAXV;
    S.y = S.ac + (size_t)nb * MAXV;
    if ((char *)(S.y + (size_t)nb * MAXV) > (char *)w->state + bytes) {
        work_free(w);
        set_error("helm_fgmres_solve: internal workspace layout error");
        return HELM_E_INVALID;
    }
    if (hipMemset(w->state, 0, bytes) != hipSuccess) {
        work_free(w);
        set_error("helm_fgmres_solve: clearing the solver state failed");
        return HELM_E_HIP;
    }
    if (scratch && (dalloc(&w->t1, (size_t)nb * N) || dalloc(&w->t2, (size_t)nb * N) ||
                    dev_malloc(&w->d_net, 2 * nb * sizeof(int)) != hipSuccess)) {
        work_free(w);
        set_error("helm_fgmres_solve: device allocation failed");
        return HELM_E_NOMEM;
    }
    if (hipHostMalloc((void **)&w->h_net, 2 * nb * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&w->h_mx, nb * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&w->h_fb, nb * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&w->h_a, nb * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&w->h_i, nb * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&w->h_d, nb * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&w->h_its, nb * sizeof(int)) != hipSuccess) {
        work_free(w);
        set_error("helm_fgmres_solve: pinned host allocation failed");
        return HELM_E_NOMEM;
    }
    h->fg = w;
    *out = w;
    return HELM_OK;
}

// z = Prec(v) for the network preconditioners (section 3.2).  Slot j holds
// the candidate unnormalised, as for M_V: every kernel that reads it as the
// preconditioner's input multiplies by S.scale (1 / its norm) on load.
// Right-hand sides in fallback use M_V.
//   M_CU (Algorithm 2 with the network coarse correction):
//       e1 = w D_A^-1 v,  e2 = e1 + Net(v - A e1),  z = e2 + w D_A^-1 (v - A e2)
//   M_VU (eq. 3.4):  e0 = Net(v),  z = e0 + V(0, v - A e0)
int apply_net_prec(helm_handle *h, unet_net *net, int prec, FgWork *w, const FgState &S,
                   float2 *v, size_t vs, float2 *z, size_t zs, int nb, int nnet, hipStream_t s)
{
    // the network runs on the nnet right-hand sides that used it at the start
    // of the restart cycle (w->d_net: their indices, then the inverse map)
    const int *idx = w->d_net, *pos = w->d_net + nb;
    const size_t N = w->N;
    const Level &L0 = h->lv[0];
    const float jw = (float)h->jacobi_w;
    const double *sc = S.scale;
    launch_masks(S, 1, s);
    int rc;
    if (prec == HELM_PREC_UNET_DEFL) {
        if ((rc = net->wrap_apply(h, v, vs, z, zs, nb, 0, s, S.mask_net, nnet, idx, pos, sc))) return rc;
        launch_resjac(L0, 0.f, jw, 0, z, zs, v, vs, w->t2, N, nb, S.active, s, sc);
        return vcycle(h, w->t2, N, z, zs, nb, S.active, s, nullptr, 1);
    }
    // coarse-grid-correction form
    launch_resjac(L0, 0.f, jw, 2, v, vs, v, vs, w->t1, N, nb, S.mask_net, s, sc);
    launch_resjac(L0, 0.f, jw, 0, w->t1, N, v, vs, w->t2, N, nb, S.mask_net, s, sc);
    if ((rc = net->wrap_apply(h, w->t2, N, w->t1, N, nb, 1, s, S.mask_net, nnet, idx, pos))) return rc;
    launch_resjac(L0, 0.f, jw, 1, w->t1, N, v, vs, z, zs, nb, S.mask_net, s, sc);
    return vcycle(h, v, vs, z, zs, nb, S.mask_sl, s, sc);
}

// Replays the captured restart cycle for this key, capturing it first.  The
// workspaces the cycle touches are allocated before capture.
// Capture and instantiation run one at a time across threads (replays run
// concurrently): a capture must not overlap calls that are unsafe during
// capture, such as allocations, on other threads.
std::mutex g_capture_mu;

template <class F>
int replay_cycle(FgWork *w, const FgState &S, int nnet, const float2 *b, const double2 *x, int prec,
                 unet_net *net, int hgen, hipStream_t s, F &&cycle)
{
    const int ngen = net ? net->gen : 0;
    FgWork::Graph *g = nullptr;
    for (auto &e : w->graphs)
        if (e.b == b && e.x == x && e.net == net && e.nb == S.nb && e.nnet == nnet && e.prec == prec &&
            e.tol == S.tol && e.stall == S.stall_ratio && e.maxit == S.maxit && e.hgen == hgen &&
            e.ngen == ngen)
            g = &e;
    if (!g) {
        if (!w->cap && hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking) != hipSuccess) {
            set_error("helm_fgmres_solve: creating the capture stream failed");
            return HELM_E_HIP;
        }
        if (w->graphs.size() >= 8) {  // bounded cache
            hipGraphExecDestroy(w->graphs.front().exec);
            w->graphs.erase(w->graphs.begin());
        }
        std::lock_guard<std::mutex> lk(g_capture_mu);
        hipGraph_t graph = nullptr;
        HELM_HIP_CHECK(hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal));
        int rc = cycle(w->cap);
        hipError_t e = hipStreamEndCapture(w->cap, &graph);
        if (rc) {
            if (graph) hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) {
            set_error(std::string("helm_fgmres_solve: graph capture failed: ") + hipGetErrorString(e));
            return HELM_E_HIP;
        }
        FgWork::Graph ng;
        ng.b = b;
        ng.x = x;
        ng.net = net;
        ng.nb = S.nb;
        ng.nnet = nnet;
        ng.prec = prec;
        ng.tol = S.tol;
        ng.stall = S.stall_ratio;
        ng.maxit = S.maxit;
        ng.hgen = hgen;
        ng.ngen = ngen;
        e = hipGraphInstantiate(&ng.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            set_error(std::string("helm_fgmres_solve: graph instantiation failed: ") + hipGetErrorString(e));
            return HELM_E_HIP;
        }
        w->graphs.push_back(ng);
        g = &w->graphs.back();
    }
    HELM_HIP_CHECK(hipGraphLaunch(g->exec, s));
    return HELM_OK;
}

// Arnoldi steps between refreshes of the network batch in an eager solve
constexpr int NET_SEG = 2;

// One problem (medium) with nb right-hand sides.
int solve_problem(helm_handle *h, int nb, const float2 *b, double2 *x, int m, double tol,
                  int maxit, int prec, unet_net *net, double stall_ratio,
                  helm_fgmres_stats *stats, hipStream_t s, bool use_graph, const int *maxit_rhs = nullptr)
{
    FgWork *w = nullptr;
    const bool use_net = prec != HELM_PREC_SL;
    int rc = work_ensure(h, nb, m, use_net, &w);
    if (rc) return rc;
    FgState S = w->S;
    S.tol = tol;
    S.maxit = maxit;
    S.stall_ratio = use_net ? stall_ratio : 0.0;
    if (maxit_rhs) {  // per right-hand side limits (never captured: the graph key holds maxit only)
        use_graph = false;
        for (int i = 0; i < nb; ++i) w->h_mx[i] = maxit_rhs[i];
        HELM_HIP_CHECK(hipMemcpyAsync(w->d_mx, w->h_mx, nb * sizeof(int), hipMemcpyHostToDevice, s));
        S.maxit_rhs = w->d_mx;
    }
    const size_t N = w->N;
    const int nblk = krylov_nblk(N, nb);
    const size_t vsb = (size_t)(m + 1) * N, zsb = (size_t)m * N;
    const Level &L0 = h->lv[0];
    std::vector<int> restarts(nb, 0);
    std::vector<char> done(nb, 0);

    HELM_HIP_CHECK(hipMemsetAsync(x, 0, (size_t)nb * N * sizeof(double2), s));
    HELM_HIP_CHECK(hipMemsetAsync(S.fallback, 0, 2 * (size_t)nb * sizeof(int), s));
    HELM_HIP_CHECK(hipMemsetAsync(S.t6, 0, 2 * (size_t)nb * sizeof(int), s));
    for (int i = 0; i < nb; ++i) w->h_i[i] = 1;
    HELM_HIP_CHECK(hipMemcpyAsync(S.active, w->h_i, nb * sizeof(int), hipMemcpyHostToDevice, s));
    HELM_HIP_CHECK(hipMemcpyAsync(S.incycle, w->h_i, nb * sizeof(int), hipMemcpyHostToDevice, s));
    launch_true_residual(h->kappa0, h->gamma0, h->n, h->omega, b, N, x, N, w->V, vsb, w->rpartial,
                         nblk, nb, nullptr, s);
    hipLaunchKernelGGL(k_restart, dim3(nb), dim3(256), 0, s, S, w->rpartial, nblk, 1);
    int nnet = 0;
    // Arnoldi steps j0 .. j1 - 1 of a restart cycle, then (last) the
    // least-squares update of x and the true residual that starts the next
    // cycle; kernels only (capturable)
    auto cycle = [&](hipStream_t cs, int j0, int j1, bool last) -> int {
        int rc2;
        for (int j = j0; j < j1; ++j) {
            float2 *vj = w->V + (size_t)j * N, *zj = w->Z + (size_t)j * N;
            float2 *wj = w->V + (size_t)(j + 1) * N;
            if (!use_net) {
                // slot j holds the candidate direction, unnormalised; the V-cycle
                // reads it scaled by 1 / (its norm)
                rc2 = vcycle(h, vj, vsb, zj, zsb, nb, S.active, cs, S.scale);
            } else {
                rc2 = apply_net_prec(h, net, prec, w, S, vj, vsb, zj, zsb, nb, nnet, cs);
            }
            if (rc2) return rc2;
            launch_apply(L0, 0.f, zj, zsb, wj, vsb, nb, S.active, cs);
            launch_arnoldi_step(S, w->V, vsb, N, j, w->partial, nblk, cs);
        }
        if (!last) return HELM_OK;
        hipLaunchKernelGGL(k_solve_y, dim3(nb), dim3(64), 0, cs, S);
        launch_xupdate(x, N, w->Z, zsb, N, S.y, MAXV, S.k, nb, S.incycle, cs);
        launch_true_residual(h->kappa0, h->gamma0, h->n, h->omega, b, N, x, N, w->V, vsb,
                             w->rpartial, nblk, nb, S.incycle, cs);
        hipLaunchKernelGGL(k_restart, dim3(nb), dim3(256), 0, cs, S, w->rpartial, nblk, 0);
        return HELM_OK;
    };
    // the network batch: right-hand sides that are active and not in
    // fallback (flags in act and fb), written to d_net; returns its size
    auto set_net_batch = [&](const int *act, const int *fb) -> int {
        int cnt = 0;
        for (int i = 0; i < nb; ++i) w->h_net[nb + i] = -1;
        for (int i = 0; i < nb; ++i)
            if (act[i] && !fb[i]) {
                w->h_net[cnt] = i;
                w->h_net[nb + i] = cnt++;
            }
        return cnt;
    };
    for (;;) {
        HELM_HIP_CHECK(hipMemcpyAsync(w->h_d, S.relres, nb * sizeof(double), hipMemcpyDeviceToHost, s));
        HELM_HIP_CHECK(hipMemcpyAsync(w->h_its, S.its, nb * sizeof(int), hipMemcpyDeviceToHost, s));
        if (use_net)
            HELM_HIP_CHECK(hipMemcpyAsync(w->h_fb, S.fallback, nb * sizeof(int), hipMemcpyDeviceToHost, s));
        HELM_HIP_CHECK(hipStreamSynchronize(s));
        int nact = 0;
        for (int i = 0; i < nb; ++i) {
            if (!done[i] && (w->h_d[i] <= tol || w->h_its[i] >= (maxit_rhs ? maxit_rhs[i] : maxit))) done[i] = 1;
            w->h_i[i] = done[i] ? 0 : 1;
            nact += w->h_i[i];
        }
        if (nact == 0) break;
        prof_set_active(nact);
        nnet = 0;
        if (use_net) {
            // gather the right-hand sides still using the network
            nnet = set_net_batch(w->h_i, w->h_fb);
            HELM_HIP_CHECK(hipMemcpyAsync(w->d_net, w->h_net, 2 * nb * sizeof(int), hipMemcpyHostToDevice, s));
        }
        HELM_HIP_CHECK(hipMemcpyAsync(S.active, w->h_i, nb * sizeof(int), hipMemcpyHostToDevice, s));
        HELM_HIP_CHECK(hipMemcpyAsync(S.incycle, w->h_i, nb * sizeof(int), hipMemcpyHostToDevice, s));
        if (use_graph) {
            // everything the cycle touches is allocated before capture
            if ((rc = ensure_vcycle_ws(h, nb))) return rc;
            if (use_net && nnet > 0 && (rc = net->ensure_ws(nnet, h->n / 2, h->n / 2, false))) return rc;
            rc = replay_cycle(w, S, nnet, b, x, prec, net, h->ws_gen, s,
                              [&](hipStream_t cs) { return cycle(cs, 0, m, true); });
        } else if (!use_net) {
            rc = cycle(s, 0, m, true);
        } else {
            // Right-hand sides that converge (or fall back) inside the cycle
            // leave the network batch at the next segment boundary instead of
            // at the cycle's end: the network is most of an M_VU step, and a
            // host round trip every NET_SEG steps costs little next to it.
            for (int j0 = 0; j0 < m && !rc; j0 += NET_SEG) {
                const int j1 = std::min(m, j0 + NET_SEG);
                rc = cycle(s, j0, j1, j1 == m);
                if (rc || j1 == m || nnet == 0) continue;
                HELM_HIP_CHECK(hipMemcpyAsync(w->h_a, S.active, nb * sizeof(int), hipMemcpyDeviceToHost, s));
                HELM_HIP_CHECK(hipMemcpyAsync(w->h_fb, S.fallback, nb * sizeof(int), hipMemcpyDeviceToHost, s));
                HELM_HIP_CHECK(hipStreamSynchronize(s));
                int cnt = 0;
                for (int i = 0; i < nb; ++i) cnt += w->h_a[i] && !w->h_fb[i];
                if (cnt == nnet) continue;  // nobody left the batch
                nnet = set_net_batch(w->h_a, w->h_fb);
                HELM_HIP_CHECK(hipMemcpyAsync(w->d_net, w->h_net, 2 * nb * sizeof(int), hipMemcpyHostToDevice, s));
            }
        }
        if (rc) return rc;
        for (int i = 0; i < nb; ++i)
            if (w->h_i[i]) restarts[i]++;
        HELM_HIP_CHECK(hipGetLastError());
    }
    prof_set_active(-1);
    HELM_HIP_CHECK(hipMemcpyAsync(w->h_fb, S.fallback, nb * sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<int> t67(2 * (size_t)nb);
    std::vector<double> r67(2 * (size_t)nb);
    HELM_HIP_CHECK(hipMemcpyAsync(t67.data(), S.t6, 2 * nb * sizeof(int), hipMemcpyDeviceToHost, s));
    HELM_HIP_CHECK(hipMemcpyAsync(r67.data(), S.rel6, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
    HELM_HIP_CHECK(hipStreamSynchronize(s));
    int nconv = 0;
    for (int i = 0; i < nb; ++i) {
        bool conv = w->h_d[i] <= tol;
        nconv += conv;
        if (stats) {
            stats[i].iterations = w->h_its[i];
            stats[i].restarts = restarts[i];
            stats[i].converged = conv ? 1 : 0;
            stats[i].fallback = w->h_fb[i];
            stats[i].true_relres = w->h_d[i];
            // eq. 4.1: rho = (||r_T|| / ||r_0||)^(1/T), T the first iteration
            // reaching the reduction, else the last one with the final residual
            for (int q = 0; q < 2; ++q) {
                int T = t67[(size_t)q * nb + i];
                double rel = r67[(size_t)q * nb + i];
                if (T == 0) {
                    T = w->h_its[i];
                    rel = w->h_d[i];
                }
                const double rho = T > 0 ? std::pow(rel, 1.0 / T) : 0.0;
                if (q == 0) {
                    stats[i].its_1e6 = T;
                    stats[i].rho_1e6 = rho;
                } else {
                    stats[i].its_1e7 = T;
                    stats[i].rho_1e7 = rho;
                }
            }
        }
    }
    return nconv == nb ? HELM_OK : HELM_NOT_CONVERGED;
}

}  // namespace

int fgmres_one(helm_handle *h, int nb, const float2 *b, double2 *x, int m, double tol, int maxit, int prec,
               unet_net *net, double stall_ratio, helm_fgmres_stats *stats, hipStream_t s, bool use_graph,
               const int *maxit_rhs)
{
    return solve_problem(h, nb, b, x, m, tol, maxit, prec, net, stall_ratio, stats, s, use_graph, maxit_rhs);
}

void fgmres_free(helm_handle *h)
{
    if (h && h->fg) {
        work_free((FgWork *)h->fg);
        h->fg = nullptr;
    }
}

}  // namespace helm

using namespace helm;

extern "C" int helm_fgmres_solve(helm_handle *const *probs, int nprob, const int *rhs_per_prob,
                                 const float *const *b, double *const *x,
                                 const helm_fgmres_opts *opts, helm_fgmres_stats *stats,
                                 void *stream)
{
    if (!probs || nprob < 0 || (nprob > 0 && (!rhs_per_prob || !b || !x))) {
        set_error("helm_fgmres_solve: invalid argument");
        return HELM_E_INVALID;
    }
    int m = 20, maxit = 20000, prec = HELM_PREC_SL, graph = 0;
    double tol = 1e-7, stall = 0.0;
    unet_net *net = nullptr, *enc = nullptr;
    if (opts) {
        enc = (unet_net *)opts->encoder;
        graph = opts->graph;
        m = opts->m;
        tol = opts->tol;
        maxit = opts->maxit;
        prec = opts->prec;
        net = (unet_net *)opts->net;
        stall = opts->stall_ratio;
    }
    if (m < 1 || m > MAXM || !(tol > 0.0) || maxit < 0) {
        set_error("helm_fgmres_solve: m must be in [1, 30], tol > 0, maxit >= 0");
        return HELM_E_INVALID;
    }
    if (prec != HELM_PREC_SL && prec != HELM_PREC_UNET_CGC && prec != HELM_PREC_UNET_DEFL) {
        set_error("helm_fgmres_solve: unknown preconditioner");
        return HELM_E_INVALID;
    }
    if (prec != HELM_PREC_SL && !net) {
        set_error("helm_fgmres_solve: the network preconditioners need opts->net");
        return HELM_E_INVALID;
    }
    if (enc && (!net || !net->cfg.context || prec == HELM_PREC_SL)) {
        set_error("helm_fgmres_solve: opts->encoder goes with an encoder-solver's solver as opts->net");
        return HELM_E_INVALID;
    }
    if (net && (!net->cfg.head ||
                (net->cfg.context && !enc && (nprob != 1 || !net->ctx_valid || !net->ctx_shared)))) {
        // a solver's context belongs to one medium: encode it first, or pass
        // the encoder so that every problem's medium is encoded in turn
        set_error("helm_fgmres_solve: a network with a head is needed; an encoder-solver's solver takes "
                  "one problem whose medium was encoded with unet_pair_encode (nb = 1), or any number of "
                  "problems with opts->encoder");
        return HELM_E_INVALID;
    }
    std::vector<int> offs(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        if (!probs[p] || rhs_per_prob[p] < 0 || (rhs_per_prob[p] > 0 && (!b[p] || !x[p]))) {
            set_error("helm_fgmres_solve: invalid problem entry");
            return HELM_E_INVALID;
        }
        if (rhs_per_prob[p] > 0 && net &&
            (probs[p]->n % (1 << net->cfg.levels) ||
             (net->cfg.context && !enc && net->ctx_H != probs[p]->n / 2))) {
            set_error("helm_fgmres_solve: grid size not divisible by 2^levels of the network");
            return HELM_E_SHAPE;
        }
        offs[p + 1] = offs[p] + rhs_per_prob[p];
    }
    hipStream_t s = (hipStream_t)stream;
    const bool use_graph = graph && !prof_enabled();
    std::vector<int> rcs(nprob, HELM_OK);
    std::vector<std::string> errs(nprob);
    auto run = [&](int p, hipStream_t st) {
        if (rhs_per_prob[p] == 0) return;
        rcs[p] = solve_problem(probs[p], rhs_per_prob[p], (const float2 *)b[p], (double2 *)x[p], m, tol,
                               maxit, prec, net, stall, stats ? stats + offs[p] : nullptr, st, use_graph);
        if (rcs[p] < 0) errs[p] = helm_last_error();
    };
    // group problems by handle: one handle's workspaces serve one solve at a time
    std::vector<std::vector<int>> groups;
    for (int p = 0; p < nprob; ++p) {
        bool placed = false;
        for (auto &g : groups)
            if (probs[g[0]] == probs[p]) {
                g.push_back(p);
                placed = true;
                break;
            }
        if (!placed) groups.push_back({p});
    }
    const int T = (int)std::min<size_t>(8, groups.size());
    if (T <= 1 || net || prof_enabled()) {
        // one after another (the network's workspace is shared); with an
        // encoder, in order of grid size, so the network's workspaces and
        // context buffers are resized once per size
        std::vector<int> order(nprob);
        for (int p = 0; p < nprob; ++p) order[p] = p;
        if (enc)
            std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return probs[a]->n < probs[c]->n; });
        for (int p : order) {
            if (enc && rhs_per_prob[p] > 0) {
                int rce = unet_pair_encode_medium(enc, net, probs[p], s);
                if (rce) return rce;
            }
            run(p, s);
            if (rcs[p] < 0) return rcs[p];
        }
    } else {
        std::vector<hipStream_t> st(T, nullptr);
        std::vector<hipEvent_t> ev(T + 1, nullptr);
        int rc = HELM_OK;
        for (int t = 0; t < T && !rc; ++t)
            if (hipStreamCreateWithFlags(&st[t], hipStreamNonBlocking) != hipSuccess) rc = HELM_E_HIP;
        for (int t = 0; t <= T && !rc; ++t)
            if (hipEventCreateWithFlags(&ev[t], hipEventDisableTiming) != hipSuccess) rc = HELM_E_HIP;
        // every workspace (and capture stream) exists before the workers
        // start, so no allocation overlaps a capture on another thread
        for (int p = 0; p < nprob && !rc; ++p) {
            if (rhs_per_prob[p] == 0) continue;
            FgWork *w = nullptr;
            if ((rc = work_ensure(probs[p], rhs_per_prob[p], m, false, &w))) break;
            if ((rc = ensure_vcycle_ws(probs[p], rhs_per_prob[p]))) break;
            if (use_graph && !w->cap && hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking) != hipSuccess)
                rc = HELM_E_HIP;
        }
        if (!rc && hipEventRecord(ev[T], s) != hipSuccess) rc = HELM_E_HIP;
        for (int t = 0; t < T && !rc; ++t)
            if (hipStreamWaitEvent(st[t], ev[T], 0) != hipSuccess) rc = HELM_E_HIP;
        if (!rc) {
            std::vector<std::thread> th;
            for (int t = 0; t < T; ++t)
                th.emplace_back([&, t]() {
                    for (size_t g = t; g < groups.size(); g += T)
                        for (int p : groups[g]) {
                            run(p, st[t]);
                            if (rcs[p] < 0) return;
                        }
                });
            for (auto &t : th) t.join();
            for (int t = 0; t < T; ++t)
                if (hipEventRecord(ev[t], st[t]) != hipSuccess || hipStreamWaitEvent(s, ev[t], 0) != hipSuccess)
                    rc = HELM_E_HIP;
        }
        for (auto e : ev)
            if (e) hipEventDestroy(e);
        for (auto q : st)
            if (q) hipStreamDestroy(q);
        if (rc) {
            set_error("helm_fgmres_solve: internal stream set-up failed");
            return rc;
        }
        for (int p = 0; p < nprob; ++p)
            if (rcs[p] < 0) {
                set_error(errs[p]);
                return rcs[p];
            }
    }
    int status = HELM_OK;
    for (int p = 0; p < nprob; ++p)
        if (rcs[p] == HELM_NOT_CONVERGED) status = HELM_NOT_CONVERGED;
    return status;
}
