// Coarsest-level solve of the SL V-cycle by k GMRES steps with the diagonal
// (Jacobi) right preconditioner, from zero, followed by Algorithm 1's
// post-relaxation: the coarsest solver of the paper's experiments (section
// 4), an alternative to the exact dense inverse.
//
// One 1024-thread workgroup per right-hand side; the coarsest grid has at
// most 16384 points (PPT <= 16 points per thread, p = tid + 1024 q).  The
// Krylov vectors V_0..V_k and the preconditioned vectors Z_j = D^-1 V_j live
// in a workspace of (2k + 1) N complex values per right-hand side.  Arnoldi
// step j: w = M Z_j, two classical Gram-Schmidt passes against V_0..V_j
// (each one block reduction of all j + 1 products: every wavefront sums its
// lanes, one LDS slot per (product, wavefront), one barrier), the norm, and
// V_{j+1} = w / |w|.  Products and norms accumulate in FP64; the
// (k + 1) x k Hessenberg least-squares problem is solved by one thread with
// complex Givens rotations in FP64.  x = sum_j y_j Z_j, then one damped
// Jacobi sweep on M x = f.
#include "helm_internal.h"

namespace helm {

namespace {

constexpr int CG_T = 1024, CG_NW = CG_T / 64, CG_KMAX = 30;

__device__ __forceinline__ double cg_wsum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// shifted mass and the reciprocal of the diagonal 4/h^2 - mass at point p
__device__ __forceinline__ void cg_diag(const float2 *mass, size_t p, float ih2, float shift, float2 &mM,
                                        float2 &dinv)
{
    const float2 m = mass[p];
    mM = make_float2(m.x, m.y - shift * m.x);
    const float dr = 4.f * ih2 - mM.x, di = -mM.y, dd = dr * dr + di * di;
    dinv = make_float2(dr / dd, -di / dd);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// (M z)(p) with zero values outside the n x n grid
__device__ __forceinline__ float2 cg_apply(const float2 *z, int n, size_t p, float ih2, float2 mM)
{
    const int i = (int)(p / n), j = (int)(p - (size_t)i * n);
    const float2 c = z[p];
    float2 s = make_float2(4.f * c.x, 4.f * c.y);
    if (i > 0) s.x -= z[p - n].x, s.y -= z[p - n].y;
    if (i < n - 1) s.x -= z[p + n].x, s.y -= z[p + n].y;
    if (j > 0) s.x -= z[p - 1].x, s.y -= z[p - 1].y;
    if (j < n - 1) s.x -= z[p + 1].x, s.y -= z[p + 1].y;
    const float2 mz = cmul(mM, c);
    return make_float2(ih2 * s.x - mz.x, ih2 * s.y - mz.y);
}

template <int PPT>
__global__ __launch_bounds__(CG_T) void k_coarse_gmres(const float2 *__restrict__ mass, int n, float ih2,
                                                       float shift, float wj, int k, const float2 *__restrict__ f,
                                                       size_t fs, float2 *__restrict__ v, size_t vs,
                                                       const int *__restrict__ active, float2 *__restrict__ work)
{
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const size_t N = (size_t)n * n;
    f += (size_t)b * fs;
    v += (size_t)b * vs;
    float2 *V = work + (size_t)b * (2 * k + 1) * N;
    float2 *Z = V + (size_t)(k + 1) * N;
    __shared__ double red[2 * (CG_KMAX + 1)][CG_NW];
    __shared__ double hsum[2 * (CG_KMAX + 1)];
    __shared__ double2 Hs[(CG_KMAX + 1) * CG_KMAX];
    __shared__ double2 ys[CG_KMAX], gs[CG_KMAX + 1];
    __shared__ int skk;

    float2 mM[PPT], dinv[PPT], w[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const size_t p = tid + (size_t)CG_T * q;
        if (p < N) cg_diag(mass, p, ih2, shift, mM[q], dinv[q]);
    }
    // block sums: every wavefront puts its lane sum of value c into red[c],
    // then block_finish(nv) adds the wavefronts' sums of values 0..nv-1
    // (fixed order) into hsum
    auto wave_put = [&](int c, double val) {
        const double t = cg_wsum(val);
        if (lane == 0) red[c][wv] = t;
    };
    auto block_finish = [&](int nv) {
        __syncthreads();
        if (tid < nv) {
            double s = 0.0;
            for (int u = 0; u < CG_NW; ++u) s += red[tid][u];
            hsum[tid] = s;
        }
        __syncthreads();
    };

    // beta = ||f||, V_0 = f / beta, Z_0 = D^-1 V_0
    {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const size_t p = tid + (size_t)CG_T * q;
            if (p < N) {
                w[q] = f[p];
                s += (double)w[q].x * w[q].x + (double)w[q].y * w[q].y;
            }
        }
        wave_put(0, s);
        block_finish(1);
    }
    const double beta = sqrt(hsum[0]);
    if (beta == 0.0) {
        // M x = 0 from zero: x = 0 and the post-relaxation keeps it
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const size_t p = tid + (size_t)CG_T * q;
            if (p < N) v[p] = make_float2(0.f, 0.f);
        }
        return;
    }
    {
        const float ib = (float)(1.0 / beta);
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const size_t p = tid + (size_t)CG_T * q;
            if (p < N) {
                const float2 x = make_float2(w[q].x * ib, w[q].y * ib);
                V[p] = x;
                Z[p] = cmul(dinv[q], x);
            }
        }
    }
    if (tid == 0) skk = k;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        const float2 *zj = Z + (size_t)j * N;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const size_t p = tid + (size_t)CG_T * q;
            if (p < N) w[q] = cg_apply(zj, n, p, ih2, mM[q]);
        }
        if (tid == 0)
            for (int i = 0; i <= j; ++i) Hs[i * CG_KMAX + j] = make_double2(0.0, 0.0);
        for (int pass = 0; pass < 2; ++pass) {
            // products <V_i, w> for i <= j
            for (int i = 0; i <= j; ++i) {
                const float2 *vi = V + (size_t)i * N;
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    const size_t p = tid + (size_t)CG_T * q;
                    if (p < N) {
                        const float2 a = vi[p];
                        sr += (double)a.x * w[q].x + (double)a.y * w[q].y;
                        si += (double)a.x * w[q].y - (double)a.y * w[q].x;
                    }
                }
                wave_put(2 * i, sr);
                wave_put(2 * i + 1, si);
            }
            block_finish(2 * (j + 1));
            for (int i = 0; i <= j; ++i) {
                const double2 c = make_double2(hsum[2 * i], hsum[2 * i + 1]);
                if (tid == 0) {
                    Hs[i * CG_KMAX + j].x += c.x;
                    Hs[i * CG_KMAX + j].y += c.y;
                }
                const float2 cf = make_float2((float)c.x, (float)c.y);
                const float2 *vi = V + (size_t)i * N;
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    const size_t p = tid + (size_t)CG_T * q;
                    if (p < N) {
                        const float2 t = cmul(cf, vi[p]);
                        w[q].x -= t.x;
                        w[q].y -= t.y;
                    }
                }
            }
            __syncthreads();  // hsum is reused below
        }
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const size_t p = tid + (size_t)CG_T * q;
            if (p < N) s += (double)w[q].x * w[q].x + (double)w[q].y * w[q].y;
        }
        wave_put(0, s);
        block_finish(1);
        const double hn = sqrt(hsum[0]);
        if (tid == 0) Hs[(j + 1) * CG_KMAX + j] = make_double2(hn, 0.0);
        if (!(hn > 1e-300 * beta)) {  // exact breakdown: the space is invariant
            if (tid == 0) skk = j + 1;
            __syncthreads();
            break;
        }
        const float ih = (float)(1.0 / hn);
        float2 *vn = V + (size_t)(j + 1) * N, *zn = Z + (size_t)(j + 1) * N;
        if (j + 1 < k) {
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const size_t p = tid + (size_t)CG_T * q;
                if (p < N) {
                    const float2 x = make_float2(w[q].x * ih, w[q].y * ih);
                    vn[p] = x;
                    zn[p] = cmul(dinv[q], x);
                }
            }
        }
        __syncthreads();
    }
    // least squares min || beta e_1 - H y || by complex Givens rotations
    if (tid == 0) {
        const int kk = skk;
        double2 *g = gs;
        for (int i = 0; i <= kk; ++i) g[i] = make_double2(0.0, 0.0);
        g[0] = make_double2(beta, 0.0);
        for (int j = 0; j < kk; ++j) {
            const double2 a = Hs[j * CG_KMAX + j], c2 = Hs[(j + 1) * CG_KMAX + j];
            const double na = sqrt(a.x * a.x + a.y * a.y), nc = sqrt(c2.x * c2.x + c2.y * c2.y);
            const double t = sqrt(na * na + nc * nc);
            double cs;
            double2 sn, ph;
            if (na == 0.0) {
                cs = 0.0;
                sn = make_double2(1.0, 0.0);
                ph = make_double2(1.0, 0.0);
            } else {
                ph = make_double2(a.x / na, a.y / na);
                cs = na / t;
                // sn = ph conj(c2) / t
                sn = make_double2((ph.x * c2.x + ph.y * c2.y) / t, (ph.y * c2.x - ph.x * c2.y) / t);
            }
            // rotate columns j .. kk-1 of rows j, j+1 and g
            for (int c = j; c < kk; ++c) {
                const double2 u = Hs[j * CG_KMAX + c], l = Hs[(j + 1) * CG_KMAX + c];
                // u' = cs u + sn l;  l' = -conj(sn) u + cs l
                const double2 un = make_double2(cs * u.x + sn.x * l.x - sn.y * l.y,
                                                cs * u.y + sn.x * l.y + sn.y * l.x);
                const double2 ln = make_double2(-(sn.x * u.x + sn.y * u.y) + cs * l.x,
                                                -(sn.x * u.y - sn.y * u.x) + cs * l.y);
                Hs[j * CG_KMAX + c] = un;
                Hs[(j + 1) * CG_KMAX + c] = ln;
            }
            const double2 gj = g[j];
            g[j] = make_double2(cs * gj.x, cs * gj.y);
            g[j + 1] = make_double2(-(sn.x * gj.x + sn.y * gj.y), -(sn.x * gj.y - sn.y * gj.x));
        }
        for (int i = kk - 1; i >= 0; --i) {
            double2 s = g[i];
            for (int c = i + 1; c < kk; ++c) {
                const double2 hc = Hs[i * CG_KMAX + c], yc = ys[c];
                s.x -= hc.x * yc.x - hc.y * yc.y;
                s.y -= hc.x * yc.y + hc.y * yc.x;
            }
            const double2 d = Hs[i * CG_KMAX + i];
            const double dd = d.x * d.x + d.y * d.y;
            ys[i] = make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd);
        }
    }
    __syncthreads();
    // x = sum_j y_j Z_j into v, then x + w D^-1 (f - M x)
    const int kk = skk;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const size_t p = tid + (size_t)CG_T * q;
        if (p < N) {
            double xr = 0.0, xi = 0.0;
            for (int j = 0; j < kk; ++j) {
                const float2 zz = Z[(size_t)j * N + p];
                const double2 y = ys[j];
                xr += y.x * zz.x - y.y * zz.y;
                xi += y.x * zz.y + y.y * zz.x;
            }
            v[p] = make_float2((float)xr, (float)xi);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const size_t p = tid + (size_t)CG_T * q;
        if (p < N) {
            const float2 ax = cg_apply(v, n, p, ih2, mM[q]), ff = f[p];
            const float2 rr = make_float2(ff.x - ax.x, ff.y - ax.y), d = cmul(dinv[q], rr);
            w[q] = make_float2(v[p].x + wj * d.x, v[p].y + wj * d.y);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const size_t p = tid + (size_t)CG_T * q;
        if (p < N) v[p] = w[q];
    }
}

}  // namespace

size_t coarse_gmres_elems(int Nc, int k, int nb) { return (size_t)nb * (2 * k + 1) * Nc; }

int launch_coarse_gmres(const Level &L, float shift, float w, int k, const float2 *f, size_t fs, float2 *v,
                        size_t vs, int nb, const int *active, hipStream_t s, float2 *work)
{
    const size_t N = (size_t)L.n * L.n;
    if (k < 1 || k > CG_KMAX || N > (size_t)16 * CG_T) return HELM_E_INVALID;
    const int ppt = (int)((N + CG_T - 1) / CG_T);
#define CG_LAUNCH(P)                                                                                         \
    hipLaunchKernelGGL(k_coarse_gmres<P>, dim3(nb), dim3(CG_T), 0, s, L.mass, L.n, L.ih2, shift, w, k, f, fs, \
                       v, vs, active, work)
    if (ppt <= 1)
        CG_LAUNCH(1);
    else if (ppt <= 2)
        CG_LAUNCH(2);
    else if (ppt <= 4)
        CG_LAUNCH(4);
    else if (ppt <= 8)
        CG_LAUNCH(8);
    else
        CG_LAUNCH(16);
#undef CG_LAUNCH
    return HELM_OK;
}

}  // namespace helm
