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

// The same solve for a coarsest grid of at most CG_T points and k <= KR,
// with 256 threads of PPTR points each: the Krylov vectors V_0..V_k sit in
// LDS (Z_j = D^-1 V_j is formed where it is needed, with the same rounding
// as the stored Z_j of k_coarse_gmres), and the 2 (j + 1) products of a
// Gram-Schmidt pass go through one batched reduction over four wavefronts
// instead of sixteen: the lane butterflies, not the arithmetic, bound the
// 1024-thread form on a grid this small.  Products and norms accumulate in
// FP64 as there; the sums are taken in another order.
constexpr int CGR_T = 256, CGR_NW = CGR_T / 64, PPTR = CG_T / CGR_T;
template <int KR>
__global__ __launch_bounds__(CGR_T) void k_coarse_gmres_r(const float2 *__restrict__ mass, int n, float ih2,
                                                          float shift, float wj, int k,
                                                          const float2 *__restrict__ f, size_t fs,
                                                          float2 *__restrict__ v, size_t vs,
                                                          const int *__restrict__ active)
{
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int N = n * n;
    f += (size_t)b * fs;
    v += (size_t)b * vs;
    __shared__ float2 Vs[(KR + 1) * CG_T];  // V_i at point p: Vs[i * CG_T + p]
    __shared__ float2 dv[CG_T];             // D^-1 per point
    __shared__ float2 xb[CG_T];             // x for the post-relaxation
    __shared__ double red[2 * (KR + 1)][CGR_NW];
    __shared__ double hsum[2 * (KR + 1)];
    __shared__ double2 Hs[(KR + 1) * KR];
    __shared__ double2 ys[KR], gs[KR + 1];
    __shared__ int skk;

    // this thread's points p = tid + CGR_T q
    float2 mM[PPTR], dinv[PPTR], w[PPTR];
    int pi[PPTR], pj[PPTR];
    bool in[PPTR];
#pragma unroll
    for (int q = 0; q < PPTR; ++q) {
        const int p = tid + CGR_T * q;
        in[q] = p < N;
        mM[q] = dinv[q] = make_float2(0.f, 0.f);
        if (in[q]) cg_diag(mass, p, ih2, shift, mM[q], dinv[q]);
        dv[p] = dinv[q];
        pi[q] = in[q] ? p / n : 0;
        pj[q] = in[q] ? p - pi[q] * n : 0;
    }
    // (M Z_j)(p) with Z_j = D^-1 V_j, zero outside the grid
    auto apply_z = [&](const float2 *Vj, int q) __attribute__((always_inline)) {
        const int p = tid + CGR_T * q;
        auto zq = [&](int r) { return cmul(dv[r], Vj[r]); };
        const float2 c = zq(p);
        float2 t = make_float2(4.f * c.x, 4.f * c.y);
        if (pi[q] > 0) {
            const float2 u = zq(p - n);
            t.x -= u.x, t.y -= u.y;
        }
        if (pi[q] < n - 1) {
            const float2 u = zq(p + n);
            t.x -= u.x, t.y -= u.y;
        }
        if (pj[q] > 0) {
            const float2 u = zq(p - 1);
            t.x -= u.x, t.y -= u.y;
        }
        if (pj[q] < n - 1) {
            const float2 u = zq(p + 1);
            t.x -= u.x, t.y -= u.y;
        }
        const float2 mz = cmul(mM[q], c);
        return make_float2(ih2 * t.x - mz.x, ih2 * t.y - mz.y);
    };
    // sums of the nv values val[0..nv-1] over the workgroup into hsum
    double val[2 * (KR + 1)];
    auto block_sums = [&](int nv) __attribute__((always_inline)) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int c = 0; c < 2 * (KR + 1); ++c)
                if (c < nv) val[c] += __shfl_xor(val[c], o, 64);
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < 2 * (KR + 1); ++c)
                if (c < nv) red[c][wv] = val[c];
        __syncthreads();
        if (tid < nv) {
            double t = 0.0;
            for (int u = 0; u < CGR_NW; ++u) t += red[tid][u];
            hsum[tid] = t;
        }
        __syncthreads();
    };
    auto norm2 = [&]() __attribute__((always_inline)) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < PPTR; ++q) t += (double)w[q].x * w[q].x + (double)w[q].y * w[q].y;
        return t;
    };

#pragma unroll
    for (int q = 0; q < PPTR; ++q) w[q] = in[q] ? f[tid + CGR_T * q] : make_float2(0.f, 0.f);
    val[0] = norm2();
    block_sums(1);
    const double beta = sqrt(hsum[0]);
    if (beta == 0.0) {
#pragma unroll
        for (int q = 0; q < PPTR; ++q)
            if (in[q]) v[tid + CGR_T * q] = make_float2(0.f, 0.f);
        return;
    }
    {
        const float ib = (float)(1.0 / beta);
#pragma unroll
        for (int q = 0; q < PPTR; ++q) Vs[tid + CGR_T * q] = make_float2(w[q].x * ib, w[q].y * ib);
    }
    if (tid == 0) skk = k;
    __syncthreads();  // V_0 and D^-1 complete; hsum is reused below
    for (int j = 0; j < k; ++j) {
        const float2 *Vj = Vs + j * CG_T;
#pragma unroll
        for (int q = 0; q < PPTR; ++q) w[q] = in[q] ? apply_z(Vj, q) : make_float2(0.f, 0.f);
        if (tid == 0)
            for (int i = 0; i <= j; ++i) Hs[i * KR + j] = make_double2(0.0, 0.0);
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int i = 0; i < KR; ++i)
                if (i <= j) {
                    double sr = 0.0, si = 0.0;
#pragma unroll
                    for (int q = 0; q < PPTR; ++q) {
                        const float2 a = Vs[i * CG_T + tid + CGR_T * q];
                        sr += (double)a.x * w[q].x + (double)a.y * w[q].y;
                        si += (double)a.x * w[q].y - (double)a.y * w[q].x;
                    }
                    val[2 * i] = sr;
                    val[2 * i + 1] = si;
                }
            block_sums(2 * (j + 1));
            for (int i = 0; i <= j; ++i) {
                const double2 c = make_double2(hsum[2 * i], hsum[2 * i + 1]);
                if (tid == 0) {
                    Hs[i * KR + j].x += c.x;
                    Hs[i * KR + j].y += c.y;
                }
                const float2 cf = make_float2((float)c.x, (float)c.y);
#pragma unroll
                for (int q = 0; q < PPTR; ++q) {
                    const float2 t = cmul(cf, Vs[i * CG_T + tid + CGR_T * q]);
                    w[q].x -= t.x;
                    w[q].y -= t.y;
                }
            }
            __syncthreads();  // hsum is reused below
        }
        val[0] = norm2();
        block_sums(1);
        const double hn = sqrt(hsum[0]);
        if (tid == 0) Hs[(j + 1) * KR + j] = make_double2(hn, 0.0);
        if (!(hn > 1e-300 * beta)) {  // exact breakdown: the space is invariant
            if (tid == 0) skk = j + 1;
            __syncthreads();
            break;
        }
        if (j + 1 < k) {
            const float ih = (float)(1.0 / hn);
#pragma unroll
            for (int q = 0; q < PPTR; ++q)
                Vs[(j + 1) * CG_T + tid + CGR_T * q] = make_float2(w[q].x * ih, w[q].y * ih);
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
            const double2 a = Hs[j * KR + j], c2 = Hs[(j + 1) * KR + j];
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
                sn = make_double2((ph.x * c2.x + ph.y * c2.y) / t, (ph.y * c2.x - ph.x * c2.y) / t);
            }
            for (int c = j; c < kk; ++c) {
                const double2 u = Hs[j * KR + c], l = Hs[(j + 1) * KR + c];
                const double2 un = make_double2(cs * u.x + sn.x * l.x - sn.y * l.y,
                                                cs * u.y + sn.x * l.y + sn.y * l.x);
                const double2 ln = make_double2(-(sn.x * u.x + sn.y * u.y) + cs * l.x,
                                                -(sn.x * u.y - sn.y * u.x) + cs * l.y);
                Hs[j * KR + c] = un;
                Hs[(j + 1) * KR + c] = ln;
            }
            const double2 gj = g[j];
            g[j] = make_double2(cs * gj.x, cs * gj.y);
            g[j + 1] = make_double2(-(sn.x * gj.x + sn.y * gj.y), -(sn.x * gj.y - sn.y * gj.x));
        }
        for (int i = kk - 1; i >= 0; --i) {
            double2 t = g[i];
            for (int c = i + 1; c < kk; ++c) {
                const double2 hc = Hs[i * KR + c], yc = ys[c];
                t.x -= hc.x * yc.x - hc.y * yc.y;
                t.y -= hc.x * yc.y + hc.y * yc.x;
            }
            const double2 d = Hs[i * KR + i];
            const double dd = d.x * d.x + d.y * d.y;
            ys[i] = make_double2((t.x * d.x + t.y * d.y) / dd, (t.y * d.x - t.x * d.y) / dd);
        }
    }
    __syncthreads();
    // x = sum_j y_j Z_j, then x + w D^-1 (f - M x)
    const int kk = skk;
    float2 x[PPTR];
#pragma unroll
    for (int q = 0; q < PPTR; ++q) {
        double xr = 0.0, xi = 0.0;
        for (int j = 0; j < kk; ++j) {
            const float2 zz = cmul(dinv[q], Vs[j * CG_T + tid + CGR_T * q]);
            const double2 y = ys[j];
            xr += y.x * zz.x - y.y * zz.y;
            xi += y.x * zz.y + y.y * zz.x;
        }
        x[q] = in[q] ? make_float2((float)xr, (float)xi) : make_float2(0.f, 0.f);
        xb[tid + CGR_T * q] = x[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPTR; ++q) {
        if (!in[q]) continue;
        const int p = tid + CGR_T * q;
        float2 t = make_float2(4.f * x[q].x, 4.f * x[q].y);
        if (pi[q] > 0) t.x -= xb[p - n].x, t.y -= xb[p - n].y;
        if (pi[q] < n - 1) t.x -= xb[p + n].x, t.y -= xb[p + n].y;
        if (pj[q] > 0) t.x -= xb[p - 1].x, t.y -= xb[p - 1].y;
        if (pj[q] < n - 1) t.x -= xb[p + 1].x, t.y -= xb[p + 1].y;
        const float2 mx = cmul(mM[q], x[q]);
        const float2 ax = make_float2(ih2 * t.x - mx.x, ih2 * t.y - mx.y), ff = f[p];
        const float2 rr = make_float2(ff.x - ax.x, ff.y - ax.y), d = cmul(dinv[q], rr);
        v[p] = make_float2(x[q].x + wj * d.x, x[q].y + wj * d.y);
    }
}

}  // namespace

size_t coarse_gmres_elems(int Nc, int k, int nb) { return (size_t)nb * (2 * k + 1) * Nc; }

int launch_coarse_gmres(const Level &L, float shift, float w, int k, const float2 *f, size_t fs, float2 *v,
                        size_t vs, int nb, const int *active, hipStream_t s, float2 *work)
{
    const size_t N = (size_t)L.n * L.n;
    if (k < 1 || k > CG_KMAX || N > (size_t)16 * CG_T) return HELM_E_INVALID;
    if (N <= (size_t)CG_T && k <= 10) {
        hipLaunchKernelGGL(k_coarse_gmres_r<10>, dim3(nb), dim3(CGR_T), 0, s, L.mass, L.n, L.ih2, shift, w, k, f,
                           fs, v, vs, active);
        return HELM_OK;
    }
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
