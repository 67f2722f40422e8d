// Arnoldi kernels of the flexible GMRES driver.
//
// Orthogonalisation is classical Gram-Schmidt with one re-orthogonalisation
// whose second pass is delayed by one step and merged with the projection of
// the next vector (the "delayed CGS2" low-synchronisation scheme of
// Swirydowicz, Langou, Ananthan, Yang and Thomas, 2020).  Step j keeps
// V_0..V_{j-1} final and slot j holding the candidate u (orthogonalised once,
// norm nu).  With w = A z_j:
//   pass A (one read of V_0..V_{j-1}, u, w), one fixed-order reduction:
//       a = V^H u,  c = V^H w,  alpha = u^H u,  beta = u^H w,  gw = w^H w
//   reduction (one block per right-hand side):
//       nu'^2 = alpha - |a|^2,  v_j = (u - V a) / nu'
//       h_i = c_i (i < j),  h_j = (beta - a^H c) / nu',
//       h_{j+1,j}^2 = gw - |c|^2 - |h_j|^2,  then the Givens update of column j
//   pass B (one read of V_0..V_{j-1}, u, w): writes v_j to slot j and the new
//       candidate u' = w - sum_{i<=j} h_i v_i to slot j+1.
// The preconditioner is applied to u / nu, which differs from the final v_j
// only by the delayed re-orthogonalisation; flexible GMRES allows any
// preconditioned direction z_j.
// Column j is rotated at step j with H(j+1,j) = ||u'|| (the once-orthogonal
// candidate).  The next step finds u' = V a' + nu' v_{j+1}; the exact column
// would be h + a' with H(j+1,j) = nu'.  a' is the loss of orthogonality of
// one classical pass over complex64 vectors, |a'| ~ 1e-7 ||u'||, and it is
// not folded back, so A Z = V H holds to that order.  It affects only the
// implicit residual that decides when a cycle ends: every stop is decided by
// the FP64 true residual recomputed from x at the cycle's end, and x itself
// is updated in FP64 from the stored directions Z.
//
// Vectors are complex64; every inner product accumulates in FP64 (each
// complex64 product is exact in FP64) and is reduced in a fixed order, so
// results are bit-reproducible.  Hessenberg column, Givens rotations and the
// implicit residual are FP64 (section 3: FGMRES with right preconditioning,
// eq. 2.5).
#include <algorithm>

#include "helm_internal.h"

namespace helm {

namespace {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double2 dmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 dconj(double2 a) { return make_double2(a.x, -a.y); }
// conj(a) * b
__device__ __forceinline__ double2 cdot(double2 a, double2 b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Block-level (256 threads) sum of NP complex accumulators; entry i is
// written by thread i.
template <int NP>
__device__ __forceinline__ void block_store(double (&ar)[NP], double (&ai)[NP], double2 *out)
{
    __shared__ double sr[4][NP], si[4][NP];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double a = wave_sum(ar[i]), c = wave_sum(ai[i]);
        if (lane == 0) {
            sr[wv][i] = a;
            si[wv][i] = c;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NP; i += 256)
        out[i] = make_double2((sr[0][i] + sr[1][i]) + (sr[2][i] + sr[3][i]),
                              (si[0][i] + si[1][i]) + (si[2][i] + si[3][i]));
}

// Pass A of step J: partial sums of a_i = <v_i, u>, c_i = <v_i, w> (i < J),
// alpha = <u, u>, beta = <u, w>, gw = <w, w>, stored as
// [a_0..a_{J-1}, c_0..c_{J-1}, alpha, beta, gw].
template <int J>
__global__ __launch_bounds__(256) void k_arnoldi_a(FgState S, const float2 *__restrict__ V,
                                                   size_t vsb, size_t N,
                                                   double2 *__restrict__ partial, int nblk)
{
    constexpr int NP = 2 * J + 3;
    constexpr int JV = J > 0 ? J : 1;
    const int b = blockIdx.y;
    if (!S.active[b]) return;
    // two consecutive points per lane (16-byte loads; N is even)
    const float4 *Vb = reinterpret_cast<const float4 *>(V + (size_t)b * vsb);
    const size_t N2 = N / 2;
    const float4 *u = Vb + (size_t)J * N2;
    const float4 *w = Vb + (size_t)(J + 1) * N2;
    constexpr int U = 1;  // point pairs per thread per step (two measured slower at every j)
    double ar[NP], ai[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) ar[i] = ai[i] = 0.0;
    for (size_t p0 = (size_t)blockIdx.x * 256 * U + threadIdx.x; p0 < N2;
         p0 += (size_t)nblk * 256 * U) {
        float4 uu[U], ww[U], v[U][JV];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            size_t p = p0 + 256 * q;
            bool ok = p < N2;
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            uu[q] = ok ? u[p] : z;
            ww[q] = ok ? w[p] : z;
#pragma unroll
            for (int i = 0; i < J; ++i) v[q][i] = ok ? Vb[(size_t)i * N2 + p] : z;
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double ux = h ? uu[q].z : uu[q].x, uy = h ? uu[q].w : uu[q].y;
                const double wx = h ? ww[q].z : ww[q].x, wy = h ? ww[q].w : ww[q].y;
#pragma unroll
                for (int i = 0; i < J; ++i) {
                    const double vx = h ? v[q][i].z : v[q][i].x, vy = h ? v[q][i].w : v[q][i].y;
                    ar[i] += vx * ux + vy * uy;
                    ai[i] += vx * uy - vy * ux;
                    ar[J + i] += vx * wx + vy * wy;
                    ai[J + i] += vx * wy - vy * wx;
                }
                ar[2 * J] += ux * ux + uy * uy;
                ar[2 * J + 1] += ux * wx + uy * wy;
                ai[2 * J + 1] += ux * wy - uy * wx;
                ar[2 * J + 2] += wx * wx + wy * wy;
            }
    }
    block_store<NP>(ar, ai, partial + ((size_t)b * nblk + blockIdx.x) * MAXP);
}

// Reduction of pass A and the Givens update of column j (one block per
// right-hand side).  Sets S.hc = [h_0..h_j], S.ac = [a_0..a_{j-1}], S.nu =
// nu', the Hessenberg column, rotations, g and the next candidate's scale;
// clears the active flag when the cycle stops at this step.
__global__ __launch_bounds__(1024) void k_arnoldi_reduce(FgState S,
                                                         const double2 *__restrict__ partial,
                                                         int nblk, int j)
{
    const int b = blockIdx.x;
    if (!S.active[b]) return;
    const int m = S.m;
    const int np = 2 * j + 3;
    __shared__ double2 part[16][MAXP];
    __shared__ double2 red[MAXP];
    __shared__ double2 col[MAXV + 1], sn_s[MAXV];
    __shared__ double cs_s[MAXV];
    __shared__ double sums[3][2];
    __shared__ int drop;
    const int t = threadIdx.x;
    if (t == 0) drop = 0;
    {
        // fixed-order sums over blocks: 64 entries x 16 row groups
        const double2 *pb = partial + (size_t)b * nblk * MAXP;
        const int r0 = t >> 6, i = t & 63;
        double sr = 0.0, si = 0.0;
        if (i < np) {
#pragma unroll 8
            for (int q = r0; q < nblk; q += 16) {
                double2 v = pb[(size_t)q * MAXP + i];
                sr += v.x;
                si += v.y;
            }
        }
        part[r0][i] = make_double2(sr, si);
    }
    double *cs = S.cs + (size_t)b * m;
    double2 *sn = S.sn + (size_t)b * m;
    double2 *H = S.H + (size_t)b * (m + 1) * m;
    double2 *g = S.g + (size_t)b * (m + 1);
    if (t < j) {
        cs_s[t] = cs[t];
        sn_s[t] = sn[t];
    }
    __syncthreads();
    if (t < np) {
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            tr += part[r][t].x;
            ti += part[r][t].y;
        }
        red[t] = make_double2(tr, ti);
    }
    __syncthreads();
    // |a|^2, |c|^2 and a^H c over i < j, one lane per i (wave 0)
    if (t < 64) {
        double aa = 0.0, cc = 0.0, acr = 0.0, aci = 0.0;
        if (t < j) {
            double2 a = red[t], c = red[j + t];
            aa = a.x * a.x + a.y * a.y;
            cc = c.x * c.x + c.y * c.y;
            double2 q = cdot(a, c);
            acr = q.x;
            aci = q.y;
        }
        aa = wave_sum(aa);
        cc = wave_sum(cc);
        acr = wave_sum(acr);
        aci = wave_sum(aci);
        if (t == 0) {
            sums[0][0] = aa;
            sums[1][0] = cc;
            sums[2][0] = acr;
            sums[2][1] = aci;
        }
    }
    if (t < j) {
        S.hc[(size_t)b * MAXV + t] = red[j + t];
        S.ac[(size_t)b * MAXV + t] = red[t];
        col[t] = red[j + t];
    }
    __syncthreads();
    if (t == 0) {
        double alpha = red[2 * j].x, gw = red[2 * j + 2].x;
        double2 beta = red[2 * j + 1];
        double aa = sums[0][0], cc = sums[1][0];
        double2 ac = make_double2(sums[2][0], sums[2][1]);
        // A non-finite preconditioned direction (a network output of NaN or
        // Inf) poisons w = A z_j and every sum that involves it; the
        // candidate and the basis are finite (they passed the previous
        // step).  Step j is dropped: the cycle ends on its first j columns,
        // so x is updated by finite coefficients only, and this right-hand
        // side switches to the plain SL V-cycle for the rest of its solve.
        if (!(isfinite(alpha) && isfinite(gw) && isfinite(beta.x) && isfinite(beta.y) &&
              isfinite(aa) && isfinite(cc) && isfinite(ac.x) && isfinite(ac.y))) {
            S.fallback[b] = 2;
            ++S.its[b];
            S.active[b] = 0;
            drop = 1;
        }
    }
    __syncthreads();
    if (drop) return;
    if (t == 0) {
        double alpha = red[2 * j].x, gw = red[2 * j + 2].x;
        double2 beta = red[2 * j + 1];
        double aa = sums[0][0], cc = sums[1][0];
        double2 ac = make_double2(sums[2][0], sums[2][1]);
        double nu2 = alpha - aa;
        double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
        double2 hj = nu > 0.0 ? make_double2((beta.x - ac.x) / nu, (beta.y - ac.y) / nu)
                              : make_double2(0.0, 0.0);
        double hn2 = gw - cc - (hj.x * hj.x + hj.y * hj.y);
        double hn = hn2 > 0.0 ? sqrt(hn2) : 0.0;
        S.hc[(size_t)b * MAXV + j] = hj;
        S.nu[b] = nu;
        col[j] = hj;
        // previous rotations in order; `a` carries the running second component
        double2 a = col[0];
        for (int i = 0; i < j; ++i) {
            double2 c = col[i + 1];
            double2 t1 = dmul(sn_s[i], c);
            col[i] = make_double2(cs_s[i] * a.x + t1.x, cs_s[i] * a.y + t1.y);
            double2 t2 = dmul(dconj(sn_s[i]), a);
            a = make_double2(cs_s[i] * c.x - t2.x, cs_s[i] * c.y - t2.y);
        }
        // new rotation [c s; -conj(s) c] zeroing hn under a
        double am = hypot(a.x, a.y);
        double tt = hypot(am, hn);
        double cj;
        double2 sj;
        if (am == 0.0) {
            cj = 0.0;
            sj = make_double2(1.0, 0.0);
            col[j] = make_double2(hn, 0.0);
        } else {
            double2 ph = make_double2(a.x / am, a.y / am);
            cj = am / tt;
            sj = make_double2(ph.x * hn / tt, ph.y * hn / tt);
            col[j] = make_double2(ph.x * tt, ph.y * tt);
        }
        col[j + 1] = make_double2(0.0, 0.0);
        cs[j] = cj;
        sn[j] = sj;
        double2 gj = g[j];
        double2 t3 = dmul(dconj(sj), gj);
        g[j + 1] = make_double2(-t3.x, -t3.y);
        g[j] = make_double2(cj * gj.x, cj * gj.y);
        S.k[b] = j + 1;
        int its = ++S.its[b];
        double res = hypot(t3.x, t3.y);
        // first iterations reaching a 1e6 / 1e7 reduction of the implicit
        // residual (convergence factor of eq. 4.1)
        const double rr = S.bnorm[b] > 0.0 ? res / S.bnorm[b] : 0.0;
        if (S.t6[b] == 0 && rr <= 1e-6) {
            S.t6[b] = its;
            S.rel6[b] = rr;
        }
        if (S.t7[b] == 0 && rr <= 1e-7) {
            S.t7[b] = its;
            S.rel7[b] = rr;
        }
        // stall detection: residual reduction |g_{j+1}| / |g_j| above the
        // ratio on 3 consecutive steps (not the first of a cycle) switches
        // this right-hand side to the plain SL V-cycle for good
        if (S.stall_ratio > 0.0 && j > 0) {
            double prev = hypot(gj.x, gj.y);
            if (prev > 0.0 && res > S.stall_ratio * prev) {
                if (++S.stall[b] >= 3) S.fallback[b] = 1;
            } else {
                S.stall[b] = 0;
            }
        }
        S.scale[b] = hn > 0.0 ? 1.0 / hn : 0.0;
        const int lim = S.maxit_rhs ? S.maxit_rhs[b] : S.maxit;
        if (nu == 0.0 || hn == 0.0 || res <= S.tol * S.bnorm[b] || its >= lim || j + 1 >= m)
            S.active[b] = 0;
    }
    __syncthreads();
    if (t <= j + 1) H[t * m + j] = col[t];
}

// Pass B of step J: v_J = (u - sum a_i v_i) / nu' into slot J and the next
// candidate u' = w - sum_{i<=J} h_i v_i into slot J+1.  Right-hand sides
// whose cycle stopped at this step are inactive and skip it.
template <int J>
__global__ __launch_bounds__(256) void k_arnoldi_b(FgState S, float2 *__restrict__ V, size_t vsb,
                                                   size_t N)
{
    constexpr int JV = J > 0 ? J : 1;
    const int b = blockIdx.y;
    if (!S.active[b]) return;
    // two consecutive points per lane (16-byte loads and stores; N is even)
    float4 *Vb = reinterpret_cast<float4 *>(V + (size_t)b * vsb);
    const size_t N2 = N / 2;
    float4 *u = Vb + (size_t)J * N2;
    float4 *w = Vb + (size_t)(J + 1) * N2;
    double hr[J + 1], hi[J + 1], cr[JV], ci[JV];
#pragma unroll
    for (int i = 0; i <= J; ++i) {
        double2 h = S.hc[(size_t)b * MAXV + i];
        hr[i] = h.x;
        hi[i] = h.y;
    }
#pragma unroll
    for (int i = 0; i < J; ++i) {
        double2 a = S.ac[(size_t)b * MAXV + i];
        cr[i] = a.x;
        ci[i] = a.y;
    }
    const double inu = 1.0 / S.nu[b];
    constexpr int U = J <= 8 ? 2 : 1;  // point pairs per thread per step (register budget)
    for (size_t p0 = (size_t)blockIdx.x * 256 * U + threadIdx.x; p0 < N2;
         p0 += (size_t)gridDim.x * 256 * U) {
        float4 uu[U], ww[U], v[U][JV];
        bool ok[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            size_t p = p0 + 256 * q;
            ok[q] = p < N2;
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            uu[q] = ok[q] ? u[p] : z;
            ww[q] = ok[q] ? w[p] : z;
#pragma unroll
            for (int i = 0; i < J; ++i) v[q][i] = ok[q] ? Vb[(size_t)i * N2 + p] : z;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            float ov[4], ow[4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double ux = h ? uu[q].z : uu[q].x, uy = h ? uu[q].w : uu[q].y;
                double wx = h ? ww[q].z : ww[q].x, wy = h ? ww[q].w : ww[q].y;
#pragma unroll
                for (int i = 0; i < J; ++i) {
                    const double vx = h ? v[q][i].z : v[q][i].x, vy = h ? v[q][i].w : v[q][i].y;
                    ux -= cr[i] * vx - ci[i] * vy;
                    uy -= cr[i] * vy + ci[i] * vx;
                    wx -= hr[i] * vx - hi[i] * vy;
                    wy -= hr[i] * vy + hi[i] * vx;
                }
                const float vjx = (float)(ux * inu), vjy = (float)(uy * inu);
                const double vx = vjx, vy = vjy;
                wx -= hr[J] * vx - hi[J] * vy;
                wy -= hr[J] * vy + hi[J] * vx;
                ov[2 * h] = vjx;
                ov[2 * h + 1] = vjy;
                ow[2 * h] = (float)wx;
                ow[2 * h + 1] = (float)wy;
            }
            if (ok[q]) {
                u[p0 + 256 * q] = make_float4(ov[0], ov[1], ov[2], ov[3]);
                w[p0 + 256 * q] = make_float4(ow[0], ow[1], ow[2], ow[3]);
            }
        }
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

__global__ void k_masks(FgState S, int use_net)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= S.nb) return;
    const int a = S.active[b], fb = S.fallback[b];
    S.mask_net[b] = (a && use_net && !fb) ? 1 : 0;
    S.mask_sl[b] = (a && (!use_net || fb)) ? 1 : 0;
}

using pa_fn = void (*)(const FgState &, const float2 *, size_t, size_t, double2 *, int, hipStream_t);
using pb_fn = void (*)(const FgState &, float2 *, size_t, size_t, int, hipStream_t);

template <int J>
void pa_dispatch(const FgState &S, const float2 *V, size_t vsb, size_t N, double2 *partial, int nblk,
                 hipStream_t s)
{
    hipLaunchKernelGGL(k_arnoldi_a<J>, dim3(nblk, S.nb), dim3(256), 0, s, S, V, vsb, N, partial,
                       nblk);
}
template <int J>
void pb_dispatch(const FgState &S, float2 *V, size_t vsb, size_t N, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(k_arnoldi_b<J>, dim3(nblk, S.nb), dim3(256), 0, s, S, V, vsb, N);
}

template <int... I>
constexpr std::array<pa_fn, sizeof...(I)> make_pa(std::integer_sequence<int, I...>)
{
    return {&pa_dispatch<I>...};
}
template <int... I>
constexpr std::array<pb_fn, sizeof...(I)> make_pb(std::integer_sequence<int, I...>)
{
    return {&pb_dispatch<I>...};
}

const auto kPassA = make_pa(std::make_integer_sequence<int, MAXM>{});
const auto kPassB = make_pb(std::make_integer_sequence<int, MAXM>{});

}  // namespace

int krylov_nblk(size_t N, int nb)
{
    // at least two point pairs per thread; about 2048 workgroups over the
    // batch, at least 64 per right-hand side (fewer, longer blocks amortise
    // the FP64 block reductions: on MI355X, 1024^2 x 32, the passes stream
    // 2% faster than with 8192 workgroups and 5% faster than with 16384)
    size_t b = (N + 511) / 512;
    const size_t cap = std::min<size_t>(1024, std::max<size_t>(64, 2048 / (size_t)std::max(1, nb)));
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

void launch_arnoldi_step(const FgState &S, float2 *V, size_t vsb, size_t N, int j,
                         double2 *partial, int nblk, hipStream_t s)
{
    prof_mark(HELM_PROF_CGS, s, true);
    kPassA[j](S, V, vsb, N, partial, nblk, s);
    hipLaunchKernelGGL(k_arnoldi_reduce, dim3(S.nb), dim3(1024), 0, s, S, partial, nblk, j);
    kPassB[j](S, V, vsb, N, nblk, s);
    // both passes read v_0..v_{j-1}, the candidate and w; the second writes
    // v_j and the next candidate: 16 (j + 2) + 16 B per point
    prof_mark(HELM_PROF_CGS, s, false, (16.0 * (j + 2) + 16.0) * N, S.nb, true);
}

void launch_masks(const FgState &S, int use_net, hipStream_t s)
{
    hipLaunchKernelGGL(k_masks, dim3((S.nb + 63) / 64), dim3(64), 0, s, S, use_net);
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
