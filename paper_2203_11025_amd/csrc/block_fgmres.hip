// Block flexible GMRES (the solver of the paper's experiments, section 4:
// block restarted FGMRES(m) of Calandra, Gratton, Langou, Pinel and Vasseur
// with s right-hand sides sharing one block Krylov space).
//
// One cycle from X (complex128):
//   R = B - A X (FP64 residual, stored complex64), R = V_0 beta
//   step j:  Z_j = Prec(V_j) (s fields at once), W = A Z_j,
//            two classical block Gram-Schmidt passes C = [V_0..V_j]^H W,
//            W -= [V_0..V_j] C, and W = V_{j+1} H_{j+1,j} by Cholesky QR
//            applied twice (G = W^H W = R^H R, W <- W R^-1).
//   X += [Z_0..Z_j] Y with Y = argmin ||E_1 beta - Hbar Y||_F.
// Vectors are complex64; every Gram entry accumulates in FP64 and is reduced
// in a fixed order; the block Hessenberg matrix, its least-squares problem
// (Householder QR), the Cholesky factors and X are FP64.  The Gram
// matrices, the Cholesky factors and the updates stay on the device; a
// block step synchronises once, to bring the new Hessenberg block column and
// the factor to the host, which reduces the least-squares problem (s <= 16,
// (m + 1) s^2 <= 4096).
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "block_lsq.h"
#include "handle.h"
#include "unet_net.h"

namespace helm {

namespace {

constexpr int BF_T = 256, BF_TI = 2, BF_SMAX = 16;

__device__ __forceinline__ double bf_wsum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// part[chunk][i][k] = sum over the chunk's points of conj(A_i) B_k for basis
// vectors i in [i0, i0 + BF_TI) (blockIdx.x tile) and columns k < s (SM >=
// s slots).  A_i = A + i * N, B_k = B + k * N.  grid (ceil(na / BF_TI),
// nchunk): the i-tiles of one chunk run together, so B's chunk is read from
// HBM once and from the L2 by the other tiles.
template <int SM>
__global__ __launch_bounds__(BF_T) void k_block_gram(const float2 *__restrict__ A, int na,
                                                     const float2 *__restrict__ Bv, int s, size_t N, int chunk,
                                                     double2 *__restrict__ part)
{
    const int i0 = blockIdx.x * BF_TI, c = blockIdx.y;
    const size_t p0 = (size_t)c * chunk, p1 = std::min(N, p0 + (size_t)chunk);
    double ar[BF_TI][SM], ai[BF_TI][SM];
#pragma unroll
    for (int i = 0; i < BF_TI; ++i)
#pragma unroll
        for (int k = 0; k < SM; ++k) ar[i][k] = ai[i][k] = 0.0;
    for (size_t p = p0 + threadIdx.x; p < p1; p += BF_T) {
        float2 a[BF_TI];
#pragma unroll
        for (int i = 0; i < BF_TI; ++i) a[i] = i0 + i < na ? A[(size_t)(i0 + i) * N + p] : make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < SM; ++k) {
            if (k < s) {
                const float2 b = Bv[(size_t)k * N + p];
#pragma unroll
                for (int i = 0; i < BF_TI; ++i) {
                    ar[i][k] += (double)a[i].x * b.x + (double)a[i].y * b.y;
                    ai[i][k] += (double)a[i].x * b.y - (double)a[i].y * b.x;
                }
            }
        }
    }
    __shared__ double sr[BF_T / 64][BF_TI * SM], si[BF_T / 64][BF_TI * SM];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < BF_TI; ++i)
#pragma unroll
        for (int k = 0; k < SM; ++k) {
            const double x = bf_wsum(ar[i][k]), y = bf_wsum(ai[i][k]);
            if (lane == 0) {
                sr[wv][i * SM + k] = x;
                si[wv][i * SM + k] = y;
            }
        }
    __syncthreads();
    for (int q = threadIdx.x; q < BF_TI * SM; q += BF_T) {
        const int i = q / SM, k = q - i * SM;
        if (i0 + i < na && k < s) {
            double x = 0.0, y = 0.0;
            for (int w = 0; w < BF_T / 64; ++w) {
                x += sr[w][q];
                y += si[w][q];
            }
            part[((size_t)c * na + i0 + i) * s + k] = make_double2(x, y);
        }
    }
}

// out[i][k] = sum over chunks (in order) of part[chunk][i][k]
// out = the Gram matrix; hc_mode 1 also stores it to hc, 2 adds it to hc
// (the two Gram-Schmidt passes' coefficients of one Hessenberg block column).
// One wavefront per entry: lane l sums chunks l, l + 64, ..., then the
// lanes' sums are added in a fixed butterfly order.
__global__ __launch_bounds__(256) void k_block_gram_sum(const double2 *__restrict__ part, int nchunk, int nik,
                                                        double2 *__restrict__ out, double2 *__restrict__ hc,
                                                        int hc_mode)
{
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (q >= nik) return;  // whole wavefronts leave together
    double x = 0.0, y = 0.0;
    for (int c = lane; c < nchunk; c += 64) {
        const double2 v = part[(size_t)c * nik + q];
        x += v.x;
        y += v.y;
    }
    x = bf_wsum(x);
    y = bf_wsum(y);
    if (lane != 0) return;
    out[q] = make_double2(x, y);
    if (hc_mode == 1) hc[q] = make_double2(x, y);
    else if (hc_mode == 2) hc[q] = make_double2(hc[q].x + x, hc[q].y + y);
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zcmul(double2 a, double2 b)  // conj(a) b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// One Cholesky QR pass on the device (one workgroup, s <= 16): the Gram
// matrix G = W^H W = R^H R (R upper, real diagonal), Rinv = R^-1 for the
// update W <- W R^-1, and the accumulated factor Ra <- R Ra (Ra <- R on the
// first pass).  *fail records a pivot that is not positive (then Rinv is
// the identity and W is left as it is).
__global__ __launch_bounds__(256) void k_block_chol(const double2 *__restrict__ G, int s, double2 *__restrict__ Rinv,
                                                    double2 *__restrict__ Ra, int pass, int *__restrict__ fail)
{
    __shared__ double2 R[BF_SMAX][BF_SMAX], X[BF_SMAX][BF_SMAX], A[BF_SMAX][BF_SMAX];
    __shared__ int bad;
    const int t = threadIdx.x, i = t / BF_SMAX, k = t % BF_SMAX;
    if (t == 0) bad = 0;
    R[i][k] = X[i][k] = make_double2(0.0, 0.0);
    A[i][k] = (pass > 0 && i < s && k < s) ? Ra[i * s + k] : make_double2(0.0, 0.0);
    __syncthreads();
    for (int j = 0; j < s; ++j) {
        if (t == 0) {
            double d = G[j * s + j].x;
            for (int q = 0; q < j; ++q) d -= R[q][j].x * R[q][j].x + R[q][j].y * R[q][j].y;
            if (!(d > 0.0)) {
                bad = 1;
                d = 1.0;
            }
            R[j][j] = make_double2(sqrt(d), 0.0);
        }
        __syncthreads();
        if (t > j && t < s) {
            double2 v = G[j * s + t];
            for (int q = 0; q < j; ++q) {
                const double2 p = zcmul(R[q][j], R[q][t]);
                v.x -= p.x;
                v.y -= p.y;
            }
            R[j][t] = make_double2(v.x / R[j][j].x, v.y / R[j][j].x);
        }
        __syncthreads();
    }
    if (t < s) {  // column t of R^-1 by back substitution
        const int c = t;
        X[c][c] = make_double2(1.0 / R[c][c].x, 0.0);
        for (int r = c - 1; r >= 0; --r) {
            double2 v = make_double2(0.0, 0.0);
            for (int q = r + 1; q <= c; ++q) {
                const double2 p = zmul(R[r][q], X[q][c]);
                v.x += p.x;
                v.y += p.y;
            }
            X[r][c] = make_double2(-v.x / R[r][r].x, -v.y / R[r][r].x);
        }
    }
    __syncthreads();
    if (i < s && k < s) {
        Rinv[i * s + k] = bad ? make_double2(i == k ? 1.0 : 0.0, 0.0) : X[i][k];
        double2 v = R[i][k];
        if (pass > 0) {
            v = make_double2(0.0, 0.0);
            for (int q = 0; q < s; ++q) {
                const double2 p = zmul(R[i][q], A[q][k]);
                v.x += p.x;
                v.y += p.y;
            }
        }
        Ra[i * s + k] = v;
    }
    if (t == 0 && (pass == 0 || bad)) *fail = bad;
}

// Per point p, with P = sum_{i < na} A_i[p] C[i][k] (C double2 [na][s]):
//   MODE 0: Out_k[p] -= P      (complex64; the Gram-Schmidt update)
//   MODE 1: Out_k[p]  = P      (complex64, Out may be A: every A_i[p] is
//                               read before any Out_k[p] is written)
//   MODE 2: X_k[p]   += P      (complex128; the solution update, FP64)
// Sums in i order; FP32 products for MODE 0 and 1, FP64 for MODE 2.
template <int SM, int MODE>
__global__ __launch_bounds__(BF_T) void k_block_combine(const float2 *A, int na, const double2 *__restrict__ C,
                                                        int s, size_t N, float2 *Out, double2 *__restrict__ X)
{
    extern __shared__ double2 cs[];  // [na][s]
    for (int q = threadIdx.x; q < na * s; q += BF_T) cs[q] = C[q];
    __syncthreads();
    for (size_t p = (size_t)blockIdx.x * BF_T + threadIdx.x; p < N; p += (size_t)gridDim.x * BF_T) {
        if constexpr (MODE == 2) {
            double xr[SM], xi[SM];
#pragma unroll
            for (int k = 0; k < SM; ++k) xr[k] = xi[k] = 0.0;
            for (int i = 0; i < na; ++i) {
                const float2 a = A[(size_t)i * N + p];
#pragma unroll
                for (int k = 0; k < SM; ++k)
                    if (k < s) {
                        const double2 c = cs[i * s + k];
                        xr[k] += a.x * c.x - a.y * c.y;
                        xi[k] += a.x * c.y + a.y * c.x;
                    }
            }
#pragma unroll
            for (int k = 0; k < SM; ++k)
                if (k < s) {
                    double2 &x = X[(size_t)k * N + p];
                    x = make_double2(x.x + xr[k], x.y + xi[k]);
                }
        } else {
            float xr[SM], xi[SM];
#pragma unroll
            for (int k = 0; k < SM; ++k) xr[k] = xi[k] = 0.f;
            for (int i = 0; i < na; ++i) {
                const float2 a = A[(size_t)i * N + p];
#pragma unroll
                for (int k = 0; k < SM; ++k)
                    if (k < s) {
                        const double2 c = cs[i * s + k];
                        const float cr = (float)c.x, ci = (float)c.y;
                        xr[k] = fmaf(a.x, cr, fmaf(-a.y, ci, xr[k]));
                        xi[k] = fmaf(a.x, ci, fmaf(a.y, cr, xi[k]));
                    }
            }
#pragma unroll
            for (int k = 0; k < SM; ++k)
                if (k < s) {
                    float2 &o = Out[(size_t)k * N + p];
                    if (MODE == 0)
                        o = make_float2(o.x - xr[k], o.y - xi[k]);
                    else
                        o = make_float2(xr[k], xi[k]);
                }
        }
    }
}

struct BlockWork {
    size_t N = 0;
    int s = 0, m = 0, nchunk = 0;  // nchunk: most Gram point chunks (part's size)
    float2 *V = nullptr, *Z = nullptr, *t1 = nullptr, *t2 = nullptr;
    double2 *part = nullptr, *G = nullptr, *C = nullptr;
    double2 *Hc = nullptr, *Ra = nullptr;  // Hessenberg block column, accumulated Cholesky factor
    int *fail = nullptr;
    double *rpart = nullptr;
    ~BlockWork()
    {
        dev_free(Hc);
        dev_free(Ra);
        dev_free(fail);
        dev_free(V);
        dev_free(Z);
        dev_free(t1);
        dev_free(t2);
        dev_free(part);
        dev_free(G);
        dev_free(C);
        dev_free(rpart);
    }
};

int sm_of(int s) { return s <= 4 ? 4 : s <= 8 ? 8 : 16; }

// w.G (device, na x s, row-major) = A^H B over N points; hc_mode as
// k_block_gram_sum (w.Hc)
void gram(BlockWork &w, const float2 *A, int na, const float2 *B, int s, int hc_mode, hipStream_t st)
{
    // enough point chunks for about 256 workgroups over the row tiles (a
    // small grid or a thin block would otherwise leave most of the GPU idle),
    // within the workspace's chunk count (chunks of at least 256 points; of
    // 8192 points or fewer on large grids)
    const int ntiles = (na + BF_TI - 1) / BF_TI;
    const int nck = (int)std::min<size_t>(
        w.nchunk, std::max<size_t>((w.N + 8191) / 8192, (size_t)(256 + ntiles - 1) / ntiles));
    const int chunk = (int)((w.N + nck - 1) / nck);
    const dim3 grid(ntiles, nck);
#define BF_G(S) hipLaunchKernelGGL(k_block_gram<S>, grid, dim3(BF_T), 0, st, A, na, B, s, w.N, chunk, w.part)
    switch (sm_of(s)) {
    case 4: BF_G(4); break;
    case 8: BF_G(8); break;
    default: BF_G(16); break;
    }
#undef BF_G
    const int nik = na * s;
    hipLaunchKernelGGL(k_block_gram_sum, dim3((nik + 3) / 4), dim3(256), 0, st, w.part, nck, nik, w.G, w.Hc, hc_mode);
}

// the combination of k_block_combine with device coefficients C [na][s]
template <int MODE>
void combine(BlockWork &w, const float2 *A, int na, const double2 *C, int s, float2 *Out, double2 *X, hipStream_t st)
{
    const int gx = (int)std::min<size_t>(2048, (w.N + BF_T - 1) / BF_T);
    const size_t lds = (size_t)na * s * sizeof(double2);
#define BF_C(S) hipLaunchKernelGGL((k_block_combine<S, MODE>), dim3(gx), dim3(BF_T), lds, st, A, na, C, s, w.N, Out, X)
    switch (sm_of(s)) {
    case 4: BF_C(4); break;
    case 8: BF_C(8); break;
    default: BF_C(16); break;
    }
#undef BF_C
}

// W (s fields) = Q R by Cholesky QR applied twice, on the device: W is
// overwritten by Q, R (s x s upper, row-major) left in w.Ra, *w.fail set on a
// rank-deficient block.  No host synchronisation.
void chol_qr2(BlockWork &w, float2 *W, int s, hipStream_t st)
{
    for (int pass = 0; pass < 2; ++pass) {
        gram(w, W, s, W, s, 0, st);
        hipLaunchKernelGGL(k_block_chol, dim3(1), dim3(BF_SMAX * BF_SMAX), 0, st, w.G, s, w.C, w.Ra, pass, w.fail);
        combine<1>(w, W, s, w.C, s, W, nullptr, st);
    }
}

// the accumulated Cholesky factor and failure flag of chol_qr2 (synchronises)
int chol_result(BlockWork &w, int s, std::vector<cd> &R, bool &ok, hipStream_t st)
{
    std::vector<double2> h((size_t)s * s);
    int f = 0;
    HELM_HIP_CHECK(hipMemcpyAsync(h.data(), w.Ra, h.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipMemcpyAsync(&f, w.fail, sizeof(int), hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    R.resize(h.size());
    for (size_t q = 0; q < h.size(); ++q) R[q] = cd(h[q].x, h[q].y);
    ok = f == 0;
    return HELM_OK;
}

// z = Prec(v) for s fields
int block_prec(helm_handle *h, BlockWork &w, int prec, unet_net *net, const float2 *v, float2 *z, int s,
               hipStream_t st)
{
    const size_t N = w.N;
    const Level &L0 = h->lv[0];
    const float jw = (float)h->jacobi_w;
    if (prec == HELM_PREC_SL) return vcycle(h, v, N, z, N, s, nullptr, st);
    int rc;
    if (prec == HELM_PREC_UNET_DEFL) {  // e0 = Net(v), z = e0 + V(0, v - A e0)
        if ((rc = net->wrap_apply(h, v, N, z, N, s, 0, st))) return rc;
        launch_resjac(L0, 0.f, jw, 0, z, N, v, N, w.t2, N, s, nullptr, st);
        return vcycle(h, w.t2, N, z, N, s, nullptr, st, nullptr, 1);
    }
    // Algorithm 2: e1 = w D^-1 v, e2 = e1 + Net(v - A e1), z = e2 + w D^-1 (v - A e2)
    launch_resjac(L0, 0.f, jw, 2, v, N, v, N, w.t1, N, s, nullptr, st);
    launch_resjac(L0, 0.f, jw, 0, w.t1, N, v, N, w.t2, N, s, nullptr, st);
    if ((rc = net->wrap_apply(h, w.t2, N, w.t1, N, s, 1, st))) return rc;
    launch_resjac(L0, 0.f, jw, 1, w.t1, N, v, N, z, N, s, nullptr, st);
    return HELM_OK;
}

// one block of s right-hand sides
// (*rank_deficient is set when a cycle starts from a residual block that
// Cholesky QR cannot factor; the block then stops with its current x)
int block_solve(helm_handle *h, BlockWork &w, int s, const float2 *b, double2 *x, int m, double tol, int maxit,
                int prec, unet_net *net, helm_fgmres_stats *stats, hipStream_t st, bool *rank_deficient)
{
    const size_t N = w.N;
    const int nblk = 256;
    HELM_HIP_CHECK(hipMemsetAsync(x, 0, (size_t)s * N * sizeof(double2), st));
    std::vector<double> bn(s), rel(s, 1.0), rp((size_t)s * nblk);
    std::vector<int> t6(s, -1), t7(s, -1);
    std::vector<double> e6(s, 0.0), e7(s, 0.0);
    int its = 0, cycles = 0;
    bool first = true;
    BlockLsq lsq;
    for (;;) {
        // R = B - A X in FP64, stored complex64 in slot 0, with its norms
        launch_true_residual(h->kappa0, h->gamma0, h->n, h->omega, b, N, x, N, w.V, N, w.rpart, nblk, s, nullptr,
                             st);
        HELM_HIP_CHECK(hipMemcpyAsync(rp.data(), w.rpart, rp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HELM_HIP_CHECK(hipStreamSynchronize(st));
        bool all = true;
        for (int k = 0; k < s; ++k) {
            double r2 = 0.0;
            for (int q = 0; q < nblk; ++q) r2 += rp[(size_t)k * nblk + q];
            if (first) bn[k] = std::sqrt(r2);
            rel[k] = bn[k] > 0.0 ? std::sqrt(r2) / bn[k] : 0.0;
            all = all && rel[k] <= tol;
        }
        first = false;
        if (all || its >= maxit) break;
        std::vector<cd> beta;
        bool ok;
        chol_qr2(w, w.V, s, st);
        int rc = chol_result(w, s, beta, ok, st);
        if (rc) return rc;
        if (!ok) {  // rank-deficient residual block
            if (rank_deficient) *rank_deficient = true;
            break;
        }
        lsq.reset(s, m, beta);
        std::vector<cd> Y;
        std::vector<double> est;
        int kk = 0;
        for (int j = 0; j < m; ++j) {
            float2 *Vj = w.V + (size_t)j * s * N, *Zj = w.Z + (size_t)j * s * N, *W = w.V + (size_t)(j + 1) * s * N;
            if ((rc = block_prec(h, w, prec, net, Vj, Zj, s, st))) return rc;
            launch_apply(h->lv[0], 0.f, Zj, N, W, N, s, nullptr, st);
            const int na = (j + 1) * s;
            // two Gram-Schmidt passes (their coefficients summed into w.Hc)
            // and the Cholesky QR, all on the device; one round trip brings
            // the Hessenberg block column and the factor back
            for (int pass = 0; pass < 2; ++pass) {
                gram(w, w.V, na, W, s, pass == 0 ? 1 : 2, st);
                combine<0>(w, w.V, na, w.G, s, W, nullptr, st);
            }
            chol_qr2(w, W, s, st);
            std::vector<double2> hc((size_t)na * s);
            HELM_HIP_CHECK(hipMemcpyAsync(hc.data(), w.Hc, hc.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
            std::vector<cd> Rn;
            if ((rc = chol_result(w, s, Rn, ok, st))) return rc;
            for (int i = 0; i < na; ++i)
                for (int k = 0; k < s; ++k) lsq.h(i, j * s + k) = cd(hc[(size_t)i * s + k].x, hc[(size_t)i * s + k].y);
            for (int i = 0; i < s; ++i)
                for (int k = 0; k < s; ++k) lsq.h(na + i, j * s + k) = ok ? Rn[i * s + k] : cd(0.0);
            ++its;
            kk = j + 1;
            // least squares over the first (j + 2) s rows and (j + 1) s columns
            lsq.add_column(j, est);
            bool done = true;
            for (int k = 0; k < s; ++k) {
                const double e = bn[k] > 0.0 ? est[k] / bn[k] : 0.0;
                if (t6[k] < 0 && e <= 1e-6) t6[k] = its, e6[k] = e;
                if (t7[k] < 0 && e <= 1e-7) t7[k] = its, e7[k] = e;
                done = done && e <= tol;
            }
            if (!ok || done || its >= maxit) break;
        }
        lsq.solve(kk, Y);
        if (kk > 0) {
            std::vector<double2> yh(Y.size());
            for (size_t q = 0; q < Y.size(); ++q) yh[q] = make_double2(Y[q].real(), Y[q].imag());
            HELM_HIP_CHECK(hipMemcpyAsync(w.C, yh.data(), yh.size() * sizeof(double2), hipMemcpyHostToDevice, st));
            combine<2>(w, w.Z, kk * s, w.C, s, nullptr, x, st);
            // the host copy of Y must outlive the transfer
            HELM_HIP_CHECK(hipStreamSynchronize(st));
        }
        ++cycles;
    }
    for (int k = 0; k < s && stats; ++k) {
        helm_fgmres_stats &o = stats[k];
        o.iterations = its;
        o.restarts = cycles;
        o.converged = rel[k] <= tol;
        o.fallback = 0;
        o.true_relres = rel[k];
        o.its_1e6 = t6[k] >= 0 ? t6[k] : its;
        o.its_1e7 = t7[k] >= 0 ? t7[k] : its;
        o.rho_1e6 = t6[k] > 0 ? std::pow(e6[k], 1.0 / t6[k]) : 0.0;
        o.rho_1e7 = t7[k] > 0 ? std::pow(e7[k], 1.0 / t7[k]) : 0.0;
    }
    bool conv = true;
    for (int k = 0; k < s; ++k) conv = conv && rel[k] <= tol;
    return conv ? HELM_OK : HELM_NOT_CONVERGED;
}

}  // namespace

}  // namespace helm

using namespace helm;

extern "C" int helm_block_fgmres_solve(helm_handle *h, int nrhs, const float *b, double *x, int block,
                                       const helm_fgmres_opts *opts, helm_fgmres_stats *stats, void *stream)
{
    if (!h || nrhs < 0 || (nrhs > 0 && (!b || !x)) || block < 1 || block > BF_SMAX) {
        set_error("helm_block_fgmres_solve: invalid argument (block size in [1, 16])");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    int m = 10, maxit = 20000, prec = HELM_PREC_SL;
    double tol = 1e-7;
    unet_net *net = nullptr;
    if (opts) {
        m = opts->m;
        tol = opts->tol;
        maxit = opts->maxit;
        prec = opts->prec;
        net = (unet_net *)opts->net;
    }
    const int sb0 = std::min(block, nrhs);
    if (m < 1 || (size_t)(m + 1) * sb0 * sb0 > 4096 || !(tol > 0.0) || maxit < 0) {
        // the coefficients of one update, (m + 1) s x s complex doubles, sit in 64 KB of LDS
        set_error("helm_block_fgmres_solve: m >= 1 with (m + 1) * block^2 <= 4096, tol > 0, maxit >= 0");
        return HELM_E_INVALID;
    }
    if (prec != HELM_PREC_SL && prec != HELM_PREC_UNET_CGC && prec != HELM_PREC_UNET_DEFL) {
        set_error("helm_block_fgmres_solve: unknown preconditioner");
        return HELM_E_INVALID;
    }
    if (prec != HELM_PREC_SL &&
        (!net || !net->cfg.head || h->n % (1 << net->cfg.levels) ||
         (net->cfg.context && (!net->ctx_valid || !net->ctx_shared || net->ctx_H != h->n / 2)))) {
        set_error("helm_block_fgmres_solve: the network preconditioners need opts->net with a head (an "
                  "encoder-solver's solver holding this medium's context)");
        return HELM_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    const int s = std::min(block, nrhs);
    BlockWork w;
    w.N = (size_t)h->n * h->n;
    w.s = s;
    w.m = m;
    // Gram partial sums: up to nchunk point chunks per launch (see gram())
    w.nchunk = (int)std::max((w.N + 8191) / 8192, std::min<size_t>((w.N + 255) / 256, 256));
    const size_t nab = (size_t)(m + 1) * s;
    if (dev_malloc(&w.V, nab * w.N * sizeof(float2)) != hipSuccess ||
        dev_malloc(&w.Z, (size_t)m * s * w.N * sizeof(float2)) != hipSuccess ||
        dev_malloc(&w.t1, (size_t)s * w.N * sizeof(float2)) != hipSuccess ||
        dev_malloc(&w.t2, (size_t)s * w.N * sizeof(float2)) != hipSuccess ||
        dev_malloc(&w.part, (size_t)w.nchunk * nab * s * sizeof(double2)) != hipSuccess ||
        dev_malloc(&w.G, nab * s * sizeof(double2)) != hipSuccess ||
        dev_malloc(&w.C, nab * s * sizeof(double2)) != hipSuccess ||
        dev_malloc(&w.Hc, nab * s * sizeof(double2)) != hipSuccess ||
        dev_malloc(&w.Ra, (size_t)BF_SMAX * BF_SMAX * sizeof(double2)) != hipSuccess ||
        dev_malloc(&w.fail, sizeof(int)) != hipSuccess ||
        dev_malloc(&w.rpart, (size_t)s * 256 * sizeof(double)) != hipSuccess) {
        set_error("helm_block_fgmres_solve: device allocation failed");
        return HELM_E_NOMEM;
    }
    int status = HELM_OK;
    const size_t N = w.N;
    for (int b0 = 0; b0 < nrhs; b0 += s) {
        const int sb = std::min(s, nrhs - b0);
        bool rank_deficient = false;
        int rc = block_solve(h, w, sb, (const float2 *)b + (size_t)b0 * N, (double2 *)x + (size_t)b0 * N, m, tol,
                             maxit, prec, net, stats ? stats + b0 : nullptr, st, &rank_deficient);
        if (rc < 0) return rc;
        if (rank_deficient && sb > 1) {
            // a zero right-hand side or linearly dependent residuals: the
            // block's fields are solved one at a time instead (block size
            // 1, where only a zero residual, which has converged, is
            // rank-deficient)
            rc = HELM_OK;
            for (int k = 0; k < sb; ++k) {
                const size_t o = (size_t)(b0 + k) * N;
                int rk = block_solve(h, w, 1, (const float2 *)b + o, (double2 *)x + o, m, tol, maxit, prec, net,
                                     stats ? stats + b0 + k : nullptr, st, nullptr);
                if (rk < 0) return rk;
                if (rk == HELM_NOT_CONVERGED) rc = HELM_NOT_CONVERGED;
            }
        }
        if (rc == HELM_NOT_CONVERGED) status = HELM_NOT_CONVERGED;
    }
    HELM_HIP_CHECK(hipGetLastError());
    return status;
}
