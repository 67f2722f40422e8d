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

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC 2011): ten rounds, each two 32 x 32 -> 64-bit
// products of counter words 0 and 2 with the published multipliers, the high
// halves mixed with words 1 and 3 and the key; the key is bumped by the
// published Weyl increments between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                       (uint32_t)p0);
    }
    return c;
}

// x[b][p] for sample index s = index0 + b: the Philox block of counter
// (p, s_lo, s_hi, 0) under key (seed_lo, seed_hi) gives words (a, c, -, -);
// u1 = (a + 1) 2^-32 in (0, 1], u2 = c 2^-32 in [0, 1); Box-Muller in double:
// Re x = sqrt(-2 ln u1) cos(2 pi u2), Im x = sqrt(-2 ln u1) sin(2 pi u2),
// each rounded once to float.
__global__ __launch_bounds__(256) void k_philox_normals(uint64_t seed, uint64_t index0, size_t N,
                                                         float2 *__restrict__ x)
{
    const uint64_t s = index0 + blockIdx.y;
    x += (size_t)blockIdx.y * N;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        const uint4 o = philox4x32_10(make_uint4((uint32_t)p, (uint32_t)s, (uint32_t)(s >> 32), 0u),
                                      (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u1 = ((double)o.x + 1.0) * 0x1.0p-32, u2 = (double)o.y * 0x1.0p-32;
        const double rad = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        x[p] = make_float2((float)(rad * cs), (float)(rad * sn));
    }
}

// e = x - x~ with x~ complex128 (computed in double, rounded once)
__global__ __launch_bounds__(256) void k_err_from_iterate(const float2 *__restrict__ x,
                                                          const double2 *__restrict__ xt, size_t n,
                                                          float2 *__restrict__ e)
{
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (size_t)gridDim.x * 256) {
        const float2 a = x[p];
        const double2 t = xt[p];
        e[p] = make_float2((float)((double)a.x - t.x), (float)((double)a.y - t.y));
    }
}

// out_b[p] = sum_j c[b][j] in_j[p] for r and e together; the coefficients
// sit in LDS (nout x nin <= 32 x 32)
__global__ __launch_bounds__(256) void k_mix(const float2 *__restrict__ r, const float2 *__restrict__ e, int nin,
                                             size_t npts, const float *__restrict__ coef, int nout,
                                             float2 *__restrict__ ro, float2 *__restrict__ eo)
{
    __shared__ float c[32 * 32];
    for (int i = threadIdx.x; i < nout * nin; i += 256) c[i] = coef[i];
    __syncthreads();
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < npts; p += (size_t)gridDim.x * 256) {
        for (int b = 0; b < nout; ++b) {
            float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
            for (int j = 0; j < nin; ++j) {
                const float w = c[b * nin + j];
                const float2 x = r[(size_t)j * npts + p], y = e[(size_t)j * npts + p];
                ar = fmaf(w, x.x, ar);
                ai = fmaf(w, x.y, ai);
                br = fmaf(w, y.x, br);
                bi = fmaf(w, y.y, bi);
            }
            ro[(size_t)b * npts + p] = make_float2(ar, ai);
            eo[(size_t)b * npts + p] = make_float2(br, bi);
        }
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

namespace {

// the handle's triple workspace for nrhs fields (grown, never shrunk)
int ensure_triple_ws(helm_handle *h, int nrhs, int nblk)
{
    if (nrhs <= h->tw_nb) return HELM_OK;
    const size_t N = (size_t)h->n * h->n;
    dev_free(h->tw);
    dev_free(h->tx);
    dev_free(h->tpart);
    dev_free(h->txt);
    h->tw = h->tx = nullptr;
    h->tpart = nullptr;
    h->txt = nullptr;
    h->tw_nb = 0;
    if (dev_malloc(&h->tw, (size_t)nrhs * N * sizeof(float2)) != hipSuccess ||
        dev_malloc(&h->tx, (size_t)nrhs * N * sizeof(float2)) != hipSuccess ||
        dev_malloc(&h->txt, (size_t)nrhs * N * sizeof(double2)) != hipSuccess ||
        dev_malloc(&h->tpart, (size_t)nrhs * std::max(nblk * 3, 256) * sizeof(double)) != hipSuccess) {
        set_error("helm_training_triples: device allocation failed");
        return HELM_E_NOMEM;
    }
    h->tw_nb = nrhs;
    return HELM_OK;
}

int triples(helm_handle *h, const float2 *xx, float2 *rr, float2 *ee, int nrhs, hipStream_t s)
{
    const size_t N = (size_t)h->n * h->n;
    const int nblk = (int)std::min<size_t>(256, (N + 1023) / 1024);
    float2 *w = h->tw;
    double *part = h->tpart;
    // b = A x (into r), z = M_V b (into e), w = A z
    launch_apply(h->lv[0], 0.f, xx, N, rr, N, nrhs, nullptr, s);
    int rc = vcycle(h, rr, N, ee, N, nrhs, nullptr, s);
    if (rc) return rc;
    launch_apply(h->lv[0], 0.f, ee, N, w, N, nrhs, nullptr, s);
    hipLaunchKernelGGL(k_dot_wb, dim3(nblk, nrhs), dim3(256), 0, s, w, rr, N, part, nblk);
    hipLaunchKernelGGL(k_triple_finish, dim3(nblk, nrhs), dim3(256), 0, s, part, nblk, N, xx, ee, w,
                       rr, ee);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

// x~ = k steps of FGMRES(max(k, 10)) with the SL V-cycle from zero on
// b = A x, then r = b - A x~ (FP64 residual of the FP64 iterate) and
// e = x - x~.  The restart length never restarts within k <= 10 steps and is
// fixed for every k up to 10, so the solver's workspace is reused.
int triples_k(helm_handle *h, const float2 *xx, float2 *rr, float2 *ee, int nrhs, int k, hipStream_t s)
{
    const size_t N = (size_t)h->n * h->n;
    launch_apply(h->lv[0], 0.f, xx, N, h->tw, N, nrhs, nullptr, s);  // b into the workspace
    int rc = fgmres_one(h, nrhs, h->tw, h->txt, std::max(k, 10), 1e-300, k, HELM_PREC_SL, nullptr, 0.0,
                        nullptr, s, false);
    if (rc < 0) return rc;
    const int nblk = 256;
    launch_true_residual(h->kappa0, h->gamma0, h->n, h->omega, h->tw, N, h->txt, N, rr, N, h->tpart, nblk,
                         nrhs, nullptr, s);
    const int gx = (int)std::min<size_t>(4096, ((size_t)nrhs * N + 255) / 256);
    hipLaunchKernelGGL(k_err_from_iterate, dim3(gx), dim3(256), 0, s, xx, h->txt, (size_t)nrhs * N, ee);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

// triples_k with one k per sample: one batched FGMRES(max(k, 10)) whose
// right-hand side b stops after its own k_b steps (no restart for k <= 10).
int triples_ks(helm_handle *h, const float2 *xx, float2 *rr, float2 *ee, int nrhs, const int *ks, hipStream_t s)
{
    const size_t N = (size_t)h->n * h->n;
    int kmax = 1;
    for (int b = 0; b < nrhs; ++b) kmax = std::max(kmax, ks[b]);
    launch_apply(h->lv[0], 0.f, xx, N, h->tw, N, nrhs, nullptr, s);  // b into the workspace
    int rc = fgmres_one(h, nrhs, h->tw, h->txt, std::max(kmax, 10), 1e-300, kmax, HELM_PREC_SL, nullptr, 0.0,
                        nullptr, s, false, ks);
    if (rc < 0) return rc;
    const int nblk = 256;
    launch_true_residual(h->kappa0, h->gamma0, h->n, h->omega, h->tw, N, h->txt, N, rr, N, h->tpart, nblk,
                         nrhs, nullptr, s);
    const int gx = (int)std::min<size_t>(4096, ((size_t)nrhs * N + 255) / 256);
    hipLaunchKernelGGL(k_err_from_iterate, dim3(gx), dim3(256), 0, s, xx, h->txt, (size_t)nrhs * N, ee);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

int triple_nblk(const helm_handle *h)
{
    const size_t N = (size_t)h->n * h->n;
    return (int)std::min<size_t>(256, (N + 1023) / 1024);
}

}  // namespace

extern "C" int helm_training_triples(helm_handle *h, const float *x, float *r, float *e, int nrhs,
                                     void *stream)
{
    if (!h || nrhs < 0 || (nrhs > 0 && (!x || !r || !e))) {
        set_error("helm_training_triples: invalid argument");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    int rc = ensure_triple_ws(h, nrhs, triple_nblk(h));
    if (rc) return rc;
    return triples(h, (const float2 *)x, (float2 *)r, (float2 *)e, nrhs, (hipStream_t)stream);
}

extern "C" int helm_training_triples_seeded(helm_handle *h, unsigned long long seed,
                                            unsigned long long index0, int ksteps, float *x, float *r,
                                            float *e, int nrhs, void *stream)
{
    if (!h || nrhs < 0 || (nrhs > 0 && (!r || !e)) || ksteps < 1 || ksteps > MAXM) {
        set_error("helm_training_triples_seeded: invalid argument (ksteps in [1, 30])");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    int rc = ensure_triple_ws(h, nrhs, triple_nblk(h));
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)h->n * h->n;
    float2 *xx = x ? (float2 *)x : h->tx;
    const int gx = (int)std::min<size_t>(1024, (N + 255) / 256);
    hipLaunchKernelGGL(k_philox_normals, dim3(gx, nrhs), dim3(256), 0, s, (uint64_t)seed, (uint64_t)index0, N,
                       xx);
    if (ksteps == 1) return triples(h, xx, (float2 *)r, (float2 *)e, nrhs, s);
    return triples_k(h, xx, (float2 *)r, (float2 *)e, nrhs, ksteps, s);
}

extern "C" int helm_training_triples_batch(helm_handle *h, unsigned long long seed,
                                           const unsigned long long *index, const int *ksteps, float *x, float *r,
                                           float *e, int nrhs, void *stream)
{
    bool ok = h && nrhs >= 0 && (nrhs == 0 || (index && ksteps && r && e));
    for (int b = 0; ok && b < nrhs; ++b) ok = ksteps[b] >= 1 && ksteps[b] <= MAXM;
    if (!ok) {
        set_error("helm_training_triples_batch: invalid argument (index and ksteps arrays, each k in [1, 30])");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    int rc = ensure_triple_ws(h, nrhs, triple_nblk(h));
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)h->n * h->n;
    float2 *xx = x ? (float2 *)x : h->tx;
    const int gx = (int)std::min<size_t>(1024, (N + 255) / 256);
    for (int b = 0; b < nrhs; ++b)
        hipLaunchKernelGGL(k_philox_normals, dim3(gx, 1), dim3(256), 0, s, (uint64_t)seed, (uint64_t)index[b], N,
                           xx + (size_t)b * N);
    return triples_ks(h, xx, (float2 *)r, (float2 *)e, nrhs, ksteps, s);
}

extern "C" int helm_triples_mix(const float *r, const float *e, int nin, long long npts, const float *coef,
                                int nout, float *r_out, float *e_out, void *stream)
{
    if (nin < 0 || nout < 0 || nin > 32 || nout > 32 || npts < 0 ||
        (nin > 0 && nout > 0 && npts > 0 && (!r || !e || !coef || !r_out || !e_out))) {
        set_error("helm_triples_mix: invalid argument (at most 32 inputs and outputs)");
        return HELM_E_INVALID;
    }
    if (nin == 0 || nout == 0 || npts == 0) return HELM_OK;
    const float2 *ri = (const float2 *)r, *ei = (const float2 *)e;
    float2 *ro = (float2 *)r_out, *eo = (float2 *)e_out;
    const size_t bytes = (size_t)npts * sizeof(float2);
    auto overlap = [&](const float2 *a, size_t na, const float2 *b, size_t nb_) {
        return (const char *)a < (const char *)b + nb_ * bytes && (const char *)b < (const char *)a + na * bytes;
    };
    if (overlap(ri, nin, ro, nout) || overlap(ri, nin, eo, nout) || overlap(ei, nin, ro, nout) ||
        overlap(ei, nin, eo, nout)) {
        set_error("helm_triples_mix: outputs overlap the inputs");
        return HELM_E_INVALID;
    }
    const int gx = (int)std::min<long long>(2048, (npts + 255) / 256);
    hipLaunchKernelGGL(k_mix, dim3(gx), dim3(256), 0, (hipStream_t)stream, ri, ei, nin, (size_t)npts, coef, nout,
                       ro, eo);
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
