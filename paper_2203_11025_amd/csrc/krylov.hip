// Arnoldi (classical Gram-Schmidt with one re-orthogonalisation, CGS2)
// kernels of the flexible GMRES driver.  Vectors are complex64; every inner
// product accumulates in FP64 (each complex64 product is exact in FP64), and
// the reductions are two-stage with a fixed order, so results are
// bit-reproducible run to run.  The FGMRES iteration itself follows Saad's
// flexible GMRES with right preconditioning (section 3, eq. 2.5).
#include "helm_internal.h"

namespace helm {

namespace {

constexpr int MAXV = 32;  // largest Krylov subspace per cycle

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-level (256 threads) sum of NV complex accumulators, thread i < NV
// writes partial i.
template <int NV>
__device__ __forceinline__ void block_store(double (&ar)[NV], double (&ai)[NV], double2 *out)
{
    __shared__ double sr[4][NV], si[4][NV];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double a = wave_sum(ar[i]), c = wave_sum(ai[i]);
        if (lane == 0) {
            sr[wv][i] = a;
            si[wv][i] = c;
        }
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        int i = threadIdx.x;
        out[i] = make_double2((sr[0][i] + sr[1][i]) + (sr[2][i] + sr[3][i]),
                              (si[0][i] + si[1][i]) + (si[2][i] + si[3][i]));
    }
}

// partial[b][blk][i] = sum_p conj(V_i[p]) w[p]
template <int NV>
__global__ __launch_bounds__(256) void k_dots(const float2 *__restrict__ V, size_t vsb,
                                              size_t N, const float2 *__restrict__ w,
                                              size_t ws, double2 *__restrict__ partial,
                                              int nblk, const int *__restrict__ active)
{
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    V += (size_t)b * vsb;
    w += (size_t)b * ws;
    double ar[NV], ai[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) ar[i] = ai[i] = 0.0;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)nblk * 256) {
        float2 c = w[p];
        double cx = c.x, cy = c.y;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            float2 v = V[(size_t)i * N + p];
            ar[i] += (double)v.x * cx + (double)v.y * cy;
            ai[i] += (double)v.x * cy - (double)v.y * cx;
        }
    }
    block_store<NV>(ar, ai, partial + ((size_t)b * nblk + blockIdx.x) * MAXV);
}

// w -= sum_i h_i V_i in FP64, stored complex64; then mode 0: partial
// conj(V_i) w of the stored w, mode 1: partial |w|^2 (in component 0).
template <int NV>
__global__ __launch_bounds__(256) void k_update(const float2 *__restrict__ V, size_t vsb,
                                                size_t N, float2 *__restrict__ w, size_t ws,
                                                const double2 *__restrict__ hcoef, int hstride,
                                                int mode, double2 *__restrict__ partial,
                                                int nblk, const int *__restrict__ active)
{
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    V += (size_t)b * vsb;
    w += (size_t)b * ws;
    hcoef += (size_t)b * hstride;
    double hr[NV], hi[NV], ar[NV], ai[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double2 h = hcoef[i];
        hr[i] = h.x;
        hi[i] = h.y;
        ar[i] = ai[i] = 0.0;
    }
    double nrm = 0.0;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)nblk * 256) {
        float2 c = w[p];
        double cx = c.x, cy = c.y;
        float2 v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            v[i] = V[(size_t)i * N + p];
            cx -= hr[i] * v[i].x - hi[i] * v[i].y;
            cy -= hr[i] * v[i].y + hi[i] * v[i].x;
        }
        float2 o = make_float2((float)cx, (float)cy);
        w[p] = o;
        double ox = o.x, oy = o.y;
        if (mode == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                ar[i] += (double)v[i].x * ox + (double)v[i].y * oy;
                ai[i] += (double)v[i].x * oy - (double)v[i].y * ox;
            }
        } else {
            nrm += ox * ox + oy * oy;
        }
    }
    double2 *out = partial + ((size_t)b * nblk + blockIdx.x) * MAXV;
    if (mode == 0) {
        block_store<NV>(ar, ai, out);
    } else {
        double z[1] = {nrm}, zi[1] = {0.0};
        block_store<1>(z, zi, out);
    }
}

__global__ __launch_bounds__(256) void k_scale(float2 *__restrict__ w, size_t ws, size_t N,
                                               const double *__restrict__ scale,
                                               const int *__restrict__ active)
{
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    w += (size_t)b * ws;
    const float s = (float)scale[b];
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        float2 c = w[p];
        w[p] = make_float2(c.x * s, c.y * s);
    }
}

// x += sum_{i < k_b} y_i Z_i in FP64 (x complex128)
__global__ __launch_bounds__(256) void k_xupdate(double2 *__restrict__ x, size_t xs,
                                                 const float2 *__restrict__ Z, size_t zsb,
                                                 size_t N, const double2 *__restrict__ y,
                                                 int ystride, const int *__restrict__ kcount,
                                                 const int *__restrict__ active)
{
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int k = kcount[b];
    if (k == 0) return;
    __shared__ double2 sy[MAXV];
    if (threadIdx.x < k) sy[threadIdx.x] = y[(size_t)b * ystride + threadIdx.x];
    __syncthreads();
    x += (size_t)b * xs;
    Z += (size_t)b * zsb;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        double2 a = x[p];
        for (int i = 0; i < k; ++i) {
            float2 z = Z[(size_t)i * N + p];
            double2 c = sy[i];
            a.x += c.x * z.x - c.y * z.y;
            a.y += c.x * z.y + c.y * z.x;
        }
        x[p] = a;
    }
}

template <int NV>
void dots_dispatch(const float2 *V, size_t vsb, size_t N, const float2 *w, size_t ws,
                   double2 *partial, int nblk, int nb, const int *active, hipStream_t s)
{
    hipLaunchKernelGGL(k_dots<NV>, dim3(nblk, nb), dim3(256), 0, s, V, vsb, N, w, ws, partial,
                       nblk, active);
}

template <int NV>
void update_dispatch(const float2 *V, size_t vsb, size_t N, float2 *w, size_t ws,
                     const double2 *h, int hstride, int mode, double2 *partial, int nblk, int nb,
                     const int *active, hipStream_t s)
{
    hipLaunchKernelGGL(k_update<NV>, dim3(nblk, nb), dim3(256), 0, s, V, vsb, N, w, ws, h,
                       hstride, mode, partial, nblk, active);
}

using dots_fn = void (*)(const float2 *, size_t, size_t, const float2 *, size_t, double2 *, int,
                         int, const int *, hipStream_t);
using update_fn = void (*)(const float2 *, size_t, size_t, float2 *, size_t, const double2 *,
                           int, int, double2 *, int, int, const int *, hipStream_t);

template <int... I>
constexpr auto make_dots_table(std::integer_sequence<int, I...>)
{
    return std::array<dots_fn, sizeof...(I)>{&dots_dispatch<I + 1>...};
}
template <int... I>
constexpr auto make_update_table(std::integer_sequence<int, I...>)
{
    return std::array<update_fn, sizeof...(I)>{&update_dispatch<I + 1>...};
}

const auto kDots = make_dots_table(std::make_integer_sequence<int, MAXV>{});
const auto kUpdate = make_update_table(std::make_integer_sequence<int, MAXV>{});

}  // namespace

int krylov_nblk(size_t N)
{
    size_t b = (N + 1023) / 1024;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

void launch_dots(const float2 *V, size_t vsb, size_t N, const float2 *w, size_t ws, int nv,
                 double2 *partial, int nblk, int nb, const int *active, hipStream_t s)
{
    kDots[nv - 1](V, vsb, N, w, ws, partial, nblk, nb, active, s);
}

void launch_update(const float2 *V, size_t vsb, size_t N, float2 *w, size_t ws, int nv,
                   const double2 *hcoef, int hstride, int mode, double2 *partial, int nblk, int nb,
                   const int *active, hipStream_t s)
{
    kUpdate[nv - 1](V, vsb, N, w, ws, hcoef, hstride, mode, partial, nblk, nb, active, s);
}

void launch_scale(float2 *w, size_t ws, size_t N, const double *scale, int nb, const int *active,
                  hipStream_t s)
{
    int g = (int)std::min<size_t>(1024, (N + 1023) / 1024);
    hipLaunchKernelGGL(k_scale, dim3(g, nb), dim3(256), 0, s, w, ws, N, scale, active);
}

void launch_xupdate(double2 *x, size_t xs, const float2 *Z, size_t zsb, size_t N,
                    const double2 *y, int ystride, const int *kcount, int nb, const int *active,
                    hipStream_t s)
{
    int g = (int)std::min<size_t>(1024, (N + 1023) / 1024);
    hipLaunchKernelGGL(k_xupdate, dim3(g, nb), dim3(256), 0, s, x, xs, Z, zsb, N, y, ystride,
                       kcount, active);
}

}  // namespace helm
