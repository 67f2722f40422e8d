// Training data of section 3.4 (eq. 3.8-3.9) on the device: for a random
// x, b = A x, one flexible-GMRES step from zero with the SL V-cycle as
// preconditioner gives x~ = alpha z, z = M_V(b), alpha minimising
// ||b - alpha A z||; the triple is (r = b - A x~, e = x - x~, kappa_c).
#include <vector>

#include "handle.h"

namespace helm {

namespace {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// partial sums of w^H b (re, im) and w^H w per block and right-hand side
__global__ __launch_bounds__(256) void k_dot_wb(const float2 *__restrict__ w,
                                                const float2 *__restrict__ b, size_t N,
                                                double *__restrict__ part, int nblk)
{
    const int rb = blockIdx.y;
    w += (size_t)rb * N;
    b += (size_t)rb * N;
    double sr = 0.0, si = 0.0, ww = 0.0;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)nblk * 256) {
        float2 a = w[p], c = b[p];
        sr += (double)a.x * c.x + (double)a.y * c.y;
        si += (double)a.x * c.y - (double)a.y * c.x;
        ww += (double)a.x * a.x + (double)a.y * a.y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    ww = wave_sum(ww);
    __shared__ double red[4][3];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wv][0] = sr;
        red[wv][1] = si;
        red[wv][2] = ww;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int q = threadIdx.x;
        part[((size_t)rb * nblk + blockIdx.x) * 3 + q] =
            (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
}

// alpha = (w^H b) / (w^H w); r = b - alpha w (in place over b), e = x - alpha z
__global__ __launch_bounds__(256) void k_triple_finish(const double *__restrict__ part, int nblk,
                                                       size_t N, const float2 *__restrict__ x,
                                                       const float2 *__restrict__ z,
                                                       const float2 *__restrict__ w,
                                                       float2 *__restrict__ r,
                                                       float2 *__restrict__ e)
{
    const int rb = blockIdx.y;
    __shared__ double al[2];
    if (threadIdx.x == 0) {
        double sr = 0.0, si = 0.0, ww = 0.0;
        for (int k = 0; k < nblk; ++k) {
            sr += part[((size_t)rb * nblk + k) * 3];
            si += part[((size_t)rb * nblk + k) * 3 + 1];
            ww += part[((size_t)rb * nblk + k) * 3 + 2];
        }
        al[0] = ww > 0.0 ? sr / ww : 0.0;
        al[1] = ww > 0.0 ? si / ww : 0.0;
    }
    __syncthreads();
    const float ar = (float)al[0], ai = (float)al[1];
    const size_t o = (size_t)rb * N;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        float2 wv = w[o + p], zv = z[o + p], bv = r[o + p], xv = x[o + p];
        r[o + p] = make_float2(bv.x - (ar * wv.x - ai * wv.y), bv.y - (ar * wv.y + ai * wv.x));
        e[o + p] = make_float2(xv.x - (ar * zv.x - ai * zv.y), xv.y - (ar * zv.y + ai * zv.x));
    }
}

__global__ void k_coarse_kappa(const float *__restrict__ k, int n, float *__restrict__ kc)
{
    const int nc = n / 2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc * nc; i += gridDim.x * blockDim.x) {
        int I = i / nc, J = i - I * nc;
        kc[i] = k[(size_t)(2 * I) * n + 2 * J];
    }
}

}  // namespace

}  // namespace helm

using namespace helm;

extern "C" int helm_training_triples(helm_handle *h, const float *x, float *r, float *e, int nrhs,
                                     void *stream)
{
    if (!h || nrhs < 0 || (nrhs > 0 && (!x || !r || !e))) {
        set_error("helm_training_triples: invalid argument");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)h->n * h->n;
    const float2 *xx = (const float2 *)x;
    float2 *rr = (float2 *)r, *ee = (float2 *)e;
    float2 *w = nullptr;
    double *part = nullptr;
    const int nblk = (int)std::min<size_t>(256, (N + 1023) / 1024);
    if (hipMallocAsync((void **)&w, (size_t)nrhs * N * sizeof(float2), s) != hipSuccess ||
        hipMallocAsync((void **)&part, (size_t)nrhs * nblk * 3 * sizeof(double), s) != hipSuccess) {
        set_error("helm_training_triples: device allocation failed");
        return HELM_E_NOMEM;
    }
    // b = A x (into r), z = M_V b (into e), w = A z
    launch_apply(h->lv[0], 0.f, xx, N, rr, N, nrhs, nullptr, s);
    int rc = vcycle(h, rr, N, ee, N, nrhs, nullptr, s);
    if (rc) return rc;
    launch_apply(h->lv[0], 0.f, ee, N, w, N, nrhs, nullptr, s);
    hipLaunchKernelGGL(k_dot_wb, dim3(nblk, nrhs), dim3(256), 0, s, w, rr, N, part, nblk);
    hipLaunchKernelGGL(k_triple_finish, dim3(nblk, nrhs), dim3(256), 0, s, part, nblk, N, xx, ee, w,
                       rr, ee);
    hipFreeAsync(w, s);
    hipFreeAsync(part, s);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

extern "C" int helm_coarse_slowness(helm_handle *h, float *kc, void *stream)
{
    if (!h || !kc) {
        set_error("helm_coarse_slowness: invalid argument");
        return HELM_E_INVALID;
    }
    hipLaunchKernelGGL(k_coarse_kappa, dim3(256), dim3(256), 0, (hipStream_t)stream, h->kappa0, h->n,
                       kc);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}
