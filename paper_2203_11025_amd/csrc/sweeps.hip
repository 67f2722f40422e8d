// Grid sweeps of the Helmholtz / shifted-Laplacian multigrid on gfx950.
//
// Every kernel here is HBM-bound: complex64 fields, FP32 arithmetic.  The
// operator is the 5-point stencil of eq. 2.2 with the attenuated mass term
// of eq. 2.1; the shifted operator of eq. 2.4 (alpha = 1) adds `shift` to
// the attenuation.  Zero values outside the n x n array give the Dirichlet
// condition of the zero-padded convolution form (section 2.4).
//
// Layout: row-major [n][n] float2 per field, a batch of fields at a fixed
// element stride.  Mass coefficient per level: float2 m = omega^2 kappa^2 (1,
// -gamma); the operator's mass is (m.x, m.y - shift * m.x).
#include "helm_internal.h"

namespace helm {

namespace {

__device__ __forceinline__ float2 f2(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ float2 operator+(float2 a, float2 b) { return f2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 operator-(float2 a, float2 b) { return f2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 operator*(float s, float2 a) { return f2(s * a.x, s * a.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return f2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// 1 / b through the hardware reciprocal (1 ulp): the sweeps are partly
// bound by arithmetic, and IEEE divisions cost about ten instructions each
__device__ __forceinline__ float2 cinv(float2 b)
{
    const float r = __builtin_amdgcn_rcpf(b.x * b.x + b.y * b.y);
    return f2(b.x * r, -b.y * r);
}
__device__ __forceinline__ float2 op_mass(float2 m, float shift) { return f2(m.x, m.y - shift * m.x); }

__device__ __forceinline__ float2 shfl_up1(float2 v)
{
    return f2(__shfl_up(v.x, 1, 64), __shfl_up(v.y, 1, 64));
}
__device__ __forceinline__ float2 shfl_down1(float2 v)
{
    return f2(__shfl_down(v.x, 1, 64), __shfl_down(v.y, 1, 64));
}

// ------------------------------------------------------------------ apply
// One wavefront owns a strip of 64 columns and R consecutive rows; it walks
// down the rows keeping the up / centre / down values in registers, so every
// element is read from memory once per strip; left and right neighbours come
// from adjacent lanes (the strip's edge lanes load their outer neighbour).
__global__ __launch_bounds__(256) void k_apply(const float2 *__restrict__ x, size_t xs,
                                               float2 *__restrict__ y, size_t ys,
                                               const float2 *__restrict__ mass, int n,
                                               float ih2, float shift, int R,
                                               const int *__restrict__ active)
{
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const int lane = threadIdx.x;
    const int j = blockIdx.x * 64 + lane;
    const int i0 = (blockIdx.y * 4 + threadIdx.y) * R;
    if (i0 >= n) return;
    x += (size_t)b * xs;
    y += (size_t)b * ys;
    auto ld = [&](int i, int jj) {
        return (i >= 0 && i < n && jj >= 0 && jj < n) ? x[(size_t)i * n + jj] : f2(0.f, 0.f);
    };
    float2 up = ld(i0 - 1, j), cur = ld(i0, j);
    const int iend = min(i0 + R, n);
    for (int i = i0; i < iend; ++i) {
        float2 dn = ld(i + 1, j);
        float2 lf = shfl_up1(cur), rt = shfl_down1(cur);
        if (lane == 0) lf = ld(i, j - 1);
        if (lane == 63) rt = ld(i, j + 1);
        if (j < n) {
            size_t p = (size_t)i * n + j;
            float2 m = op_mass(mass[p], shift);
            float2 lap = ih2 * (4.f * cur - up - dn - lf - rt);
            y[p] = lap - cmul(m, cur);
        }
        up = cur;
        cur = dn;
    }
}

// ------------------------------------------------------------------ residual / Jacobi
// mode 0: y = f - Op x;  mode 1: y = x + w D^-1 (f - Op x);  mode 2: y = w D^-1 f
// (Jacobi from a zero guess).  f is read as fscale[b] f when fscale is given.
// Same register-window walk as k_apply.
__global__ __launch_bounds__(256) void k_resjac(const float2 *__restrict__ x, size_t xs,
                                                const float2 *__restrict__ f, size_t fs,
                                                float2 *__restrict__ y, size_t ys,
                                                const float2 *__restrict__ mass, int n, float ih2,
                                                float shift, float w, int mode, int R,
                                                const int *__restrict__ active,
                                                const double *__restrict__ fscale)
{
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const float fsc = fscale ? (float)fscale[b] : 1.f;
    const int lane = threadIdx.x;
    const int j = blockIdx.x * 64 + lane;
    const int i0 = (blockIdx.y * 4 + threadIdx.y) * R;
    if (i0 >= n) return;
    x += (size_t)b * xs;
    f += (size_t)b * fs;
    y += (size_t)b * ys;
    if (mode == 2) {
        if (j >= n) return;
        const int iend = min(i0 + R, n);
        for (int i = i0; i < iend; ++i) {
            size_t p = (size_t)i * n + j;
            float2 m = op_mass(mass[p], shift);
            y[p] = w * cmul(fsc * f[p], cinv(f2(4.f * ih2 - m.x, -m.y)));
        }
        return;
    }
    auto ld = [&](int i, int jj) {
        return (i >= 0 && i < n && jj >= 0 && jj < n) ? x[(size_t)i * n + jj] : f2(0.f, 0.f);
    };
    float2 up = ld(i0 - 1, j), cur = ld(i0, j);
    const int iend = min(i0 + R, n);
    for (int i = i0; i < iend; ++i) {
        float2 dn = ld(i + 1, j);
        float2 lf = shfl_up1(cur), rt = shfl_down1(cur);
        if (lane == 0) lf = ld(i, j - 1);
        if (lane == 63) rt = ld(i, j + 1);
        if (j < n) {
            size_t p = (size_t)i * n + j;
            float2 m = op_mass(mass[p], shift);
            float2 opx = ih2 * (4.f * cur - up - dn - lf - rt) - cmul(m, cur);
            float2 res = fsc * f[p] - opx;
            y[p] = mode == 0 ? res : cur + w * cmul(res, cinv(f2(4.f * ih2 - m.x, -m.y)));
        }
        up = cur;
        cur = dn;
    }
}

// ------------------------------------------------------------------ down
// Fused: v = w D^-1 f (Jacobi from a zero guess), r = f - Op v, fc = R r.
// Since D v = w f, (Op v)(p) = w f(p) - ih2 * sum of the 4 neighbours of v,
// so r = (1 - w) f + ih2 * (v_N + v_S + v_W + v_E).
// Tile: 32 x 8 coarse outputs; fine region of v with a 2-point halo in LDS.
constexpr int DN_CW = 32, DN_CH = 8;
constexpr int DN_VW = 2 * DN_CW + 3, DN_VH = 2 * DN_CH + 3;

__global__ __launch_bounds__(256) void k_down(const float2 *__restrict__ f, size_t fs,
                                              float2 *__restrict__ fc, size_t fcs,
                                              const float2 *__restrict__ mass, int n,
                                              float ih2, float shift, float w,
                                              const double *__restrict__ scale,
                                              const int *__restrict__ active)
{
    __shared__ float2 sv[DN_VH][DN_VW + 1];
    __shared__ float2 sf[DN_VH][DN_VW + 1];
    constexpr int NLD = (DN_VH * DN_VW + 255) / 256;
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    f += (size_t)b * fs;
    fc += (size_t)b * fcs;
    const float sc = scale ? (float)scale[b] : 1.f;
    const int nc = n / 2;
    const int I0 = blockIdx.y * DN_CH, J0 = blockIdx.x * DN_CW;
    const int fi0 = 2 * I0 - 2, fj0 = 2 * J0 - 2;
    const int tid = threadIdx.x;
    float2 fl[NLD], ml[NLD];
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        int idx = tid + 256 * q;
        int r = idx / DN_VW, c = idx - r * DN_VW;
        int i = fi0 + r, j = fj0 + c;
        fl[q] = ml[q] = f2(0.f, 0.f);
        if (idx < DN_VH * DN_VW && i >= 0 && i < n && j >= 0 && j < n) {
            size_t p = (size_t)i * n + j;
            fl[q] = f[p];
            ml[q] = mass[p];
        }
    }
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        int idx = tid + 256 * q;
        if (idx < DN_VH * DN_VW) {
            int r = idx / DN_VW, c = idx - r * DN_VW;
            int i = fi0 + r, j = fj0 + c;
            float2 fv = sc * fl[q];
            float2 m = op_mass(ml[q], shift);
            float2 vv = (i >= 0 && i < n && j >= 0 && j < n) ? w * cmul(fv, cinv(f2(4.f * ih2 - m.x, -m.y)))
                                                             : f2(0.f, 0.f);
            sf[r][c] = fv;
            sv[r][c] = vv;
        }
    }
    __syncthreads();
    // residual on rows/cols 1..size-2 of the region; zero outside the grid
    for (int idx = tid; idx < (DN_VH - 2) * (DN_VW - 2); idx += 256) {
        int r = 1 + idx / (DN_VW - 2), c = 1 + idx % (DN_VW - 2);
        int i = fi0 + r, j = fj0 + c;
        float2 res = f2(0.f, 0.f);
        if (i >= 0 && i < n && j >= 0 && j < n)
            res = (1.f - w) * sf[r][c] + ih2 * (sv[r - 1][c] + sv[r + 1][c] + sv[r][c - 1] + sv[r][c + 1]);
        sf[r][c] = res;  // each residual point reads only its own f entry
    }
    __syncthreads();
    const int tx = tid & 31, ty = tid >> 5;
    const int I = I0 + ty, J = J0 + tx;
    if (I < nc && J < nc) {
        const int r = 2 * ty + 2, c = 2 * tx + 2;
        float2 s = 0.25f * sf[r][c] +
                   0.125f * (sf[r - 1][c] + sf[r + 1][c] + sf[r][c - 1] + sf[r][c + 1]) +
                   0.0625f * (sf[r - 1][c - 1] + sf[r - 1][c + 1] + sf[r + 1][c - 1] + sf[r + 1][c + 1]);
        fc[(size_t)I * nc + J] = s;
    }
}

// ------------------------------------------------------------------ up
// Fused: v' = w D^-1 f + P vc (correction added to the pre-relaxed value),
// then one Jacobi sweep v = v' + w D^-1 (f - Op v').  Tile: 64 x 16 fine
// outputs; v' on a 1-point halo and the needed coarse values in LDS.
constexpr int UP_W = 64, UP_H = 16;
constexpr int UP_CW = UP_W / 2 + 2, UP_CH = UP_H / 2 + 2;

__global__ __launch_bounds__(256) void k_up(const float2 *__restrict__ f, size_t fs,
                                            const float2 *__restrict__ vc, size_t vcs,
                                            float2 *__restrict__ v, size_t vs,
                                            const float2 *__restrict__ mass, int n, float ih2,
                                            float shift, float w, const double *__restrict__ scale,
                                            int accumulate, const int *__restrict__ active)
{
    __shared__ float2 svc[UP_CH][UP_CW + 1];
    __shared__ float2 sv[UP_H + 2][UP_W + 3];
    __shared__ float2 sf[UP_H][UP_W];
    __shared__ float2 sd[UP_H][UP_W];
    constexpr int RW = UP_W + 2, RH = UP_H + 2;
    constexpr int NLC = (UP_CH * UP_CW + 255) / 256, NLD = (RH * RW + 255) / 256;
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    f += (size_t)b * fs;
    vc += (size_t)b * vcs;
    v += (size_t)b * vs;
    const float sc = scale ? (float)scale[b] : 1.f;
    const int nc = n / 2;
    const int i0 = blockIdx.y * UP_H, j0 = blockIdx.x * UP_W;
    const int I0 = i0 / 2 - 1, J0 = j0 / 2 - 1;
    const int tid = threadIdx.x;
    float2 cl[NLC], fl[NLD], ml[NLD];
#pragma unroll
    for (int q = 0; q < NLC; ++q) {
        int idx = tid + 256 * q;
        int r = idx / UP_CW, c = idx - r * UP_CW;
        int I = I0 + r, J = J0 + c;
        cl[q] = (idx < UP_CH * UP_CW && I >= 0 && I < nc && J >= 0 && J < nc) ? vc[(size_t)I * nc + J]
                                                                              : f2(0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        int idx = tid + 256 * q;
        int r = idx / RW, c = idx - r * RW;
        int i = i0 - 1 + r, j = j0 - 1 + c;
        fl[q] = ml[q] = f2(0.f, 0.f);
        if (idx < RH * RW && i >= 0 && i < n && j >= 0 && j < n) {
            size_t p = (size_t)i * n + j;
            fl[q] = f[p];
            ml[q] = mass[p];
        }
    }
#pragma unroll
    for (int q = 0; q < NLC; ++q) {
        int idx = tid + 256 * q;
        if (idx < UP_CH * UP_CW) {
            int r = idx / UP_CW, c = idx - r * UP_CW;
            svc[r][c] = cl[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        int idx = tid + 256 * q;
        if (idx >= RH * RW) continue;
        int r = idx / RW, c = idx - r * RW;
        int i = i0 - 1 + r, j = j0 - 1 + c;
        float2 vp = f2(0.f, 0.f);
        if (i >= 0 && i < n && j >= 0 && j < n) {
            float2 fv = sc * fl[q];
            float2 m = op_mass(ml[q], shift);
            float2 d = f2(4.f * ih2 - m.x, -m.y);
            // bilinear prolongation: even index -> one coarse point (weight 1),
            // odd index -> the two neighbours (weight 1/2 each)
            int ra = (i >> 1) - I0, rb = ((i + 1) >> 1) - I0;
            int ca = (j >> 1) - J0, cb = ((j + 1) >> 1) - J0;
            float wr = (i & 1) ? 0.5f : 1.f, wc = (j & 1) ? 0.5f : 1.f;
            float2 pv = svc[ra][ca];
            if (j & 1) pv = pv + svc[ra][cb];
            if (i & 1) {
                pv = pv + svc[rb][ca];
                if (j & 1) pv = pv + svc[rb][cb];
            }
            vp = w * cmul(fv, cinv(d)) + (wr * wc) * pv;
            if (r >= 1 && r <= UP_H && c >= 1 && c <= UP_W) {
                sf[r - 1][c - 1] = fv;
                sd[r - 1][c - 1] = d;
            }
        }
        sv[r][c] = vp;
    }
    __syncthreads();
    for (int idx = tid; idx < UP_H * UP_W; idx += 256) {
        int r = idx / UP_W, c = idx - r * UP_W;
        int i = i0 + r, j = j0 + c;
        if (i < n && j < n) {
            float2 vp = sv[r + 1][c + 1];
            float2 d = sd[r][c];
            float2 nb4 = sv[r][c + 1] + sv[r + 2][c + 1] + sv[r + 1][c] + sv[r + 1][c + 2];
            float2 res = sf[r][c] - (cmul(d, vp) - ih2 * nb4);
            float2 z = vp + w * cmul(res, cinv(d));
            if (accumulate) z = z + v[(size_t)i * n + j];
            v[(size_t)i * n + j] = z;
        }
    }
}

// ------------------------------------------------------------------ coarse
// v = X f for NB right-hand sides at once; one wavefront per row of X, each
// lane streaming two complex entries (16 bytes) per load.
template <int NB>
__global__ __launch_bounds__(256) void k_coarse(const float2 *__restrict__ X, int N,
                                                const float2 *__restrict__ f, size_t fs,
                                                float2 *__restrict__ v, size_t vs, int b0,
                                                const double *__restrict__ scale, int accumulate,
                                                const int *__restrict__ active)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= N) return;
    float ar[NB], ai[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) ar[q] = ai[q] = 0.f;
    const float2 *xr = X + (size_t)row * N;
    const int nvec = (N / 128) * 128;
    // X rows start 8-byte aligned; the 16-byte path needs an even row offset
    const bool al = (((size_t)row * N) & 1) == 0;
    int k0 = 0;
    if (al) {
#pragma unroll 4
        for (int k = 2 * lane; k < nvec; k += 128) {
            float4 a = *reinterpret_cast<const float4 *>(xr + k);
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                float4 c = *reinterpret_cast<const float4 *>(f + (size_t)(b0 + q) * fs + k);
                ar[q] += a.x * c.x - a.y * c.y + a.z * c.z - a.w * c.w;
                ai[q] += a.x * c.y + a.y * c.x + a.z * c.w + a.w * c.z;
            }
        }
        k0 = nvec;
    }
    for (int k = k0 + lane; k < N; k += 64) {
        float2 a = xr[k];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            float2 c = f[(size_t)(b0 + q) * fs + k];
            ar[q] += a.x * c.x - a.y * c.y;
            ai[q] += a.x * c.y + a.y * c.x;
        }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
        for (int off = 32; off > 0; off >>= 1) {
            ar[q] += __shfl_xor(ar[q], off, 64);
            ai[q] += __shfl_xor(ai[q], off, 64);
        }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (!active || active[b0 + q]) {
                float sc = scale ? (float)scale[b0 + q] : 1.f;
                float2 z = f2(sc * ar[q], sc * ai[q]);
                if (accumulate) z = z + v[(size_t)(b0 + q) * vs + row];
                v[(size_t)(b0 + q) * vs + row] = z;
            }
    }
}

// Many right-hand sides: V = X F as a tiled complex GEMM, so X is read once
// for up to 32 right-hand sides; k_coarse_finish adds the split ranges in
// order and applies scale / accumulate / the active mask.
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Complex GEMM on FP32 MFMA (16x16x4), computed transposed so that each
// lane's four accumulator rows are four right-hand sides:
//   X^T[c][row] = sum_k F^T[c][k] M^-1^T[k][row],
// complex as four real products per step (re += Fr Mr - Fi Mi, im += Fr Mi
// + Fi Mr).  MFMA operand layout (64 lanes): A (16 x 4) lane l holds row
// l % 16, k = l / 16; B (4 x 16) lane l holds k = l / 16, column l % 16;
// D (16 x 16) lane l holds rows 4 (l / 16) .. + 3 of column l % 16.  A
// workgroup (4 wavefronts) owns CG_ROWS rows of M^-1 (16 per wavefront), up
// to 32 right-hand sides (two 16-wide tiles) and one of CG_SPLIT ranges of
// the sum.  CG_BK-deep slices of M^-1 and F are staged in LDS with k
// contiguous (coalesced global reads, contiguous LDS writes) in rows padded
// to CG_KP entries: a fragment read (16 rows x 4 k) then touches 64
// distinct banks.  k_coarse_finish adds the ranges in order and applies the
// scale.
constexpr int CG_ROWS = 64, CG_BK = 64, CG_SPLIT = 8, CG_KP = CG_BK + 2;
__global__ __launch_bounds__(256) void k_coarse_gemm(const float2 *__restrict__ X, int N,
                                                     const float2 *__restrict__ f, size_t fs, int nb,
                                                     float2 *__restrict__ part)
{
    __shared__ float2 xs[CG_ROWS][CG_KP];
    __shared__ float2 fsh[32][CG_KP];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r0 = blockIdx.x * CG_ROWS, sp = blockIdx.y, c0 = blockIdx.z * 32;
    const int kper = ((N + CG_SPLIT - 1) / CG_SPLIT + CG_BK - 1) / CG_BK * CG_BK;
    const int kb = sp * kper, ke = min(N, kb + kper);
    f32x4_t accr[2], acci[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) accr[t] = acci[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int lr = lane & 15, lk = lane >> 4;
    constexpr int NXL = CG_ROWS * CG_BK / 256, NFL = 32 * CG_BK / 256;  // loads per thread
    for (int k0 = kb; k0 < ke; k0 += CG_BK) {
        // M^-1 slice (rows r0 .. + 63, k k0 .. + 63, coalesced along k) and
        // F slice (right-hand sides c0 .. + 31): all loads issued before the
        // LDS stores
        float2 xv[NXL], fv[NFL];
#pragma unroll
        for (int q = 0; q < NXL; ++q) {
            const int i = tid + 256 * q, r = i / CG_BK, kk = i - r * CG_BK;
            const int row = r0 + r, k = k0 + kk;
            xv[q] = (row < N && k < ke) ? X[(size_t)row * N + k] : f2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < NFL; ++q) {
            const int i = tid + 256 * q, c = i / CG_BK, kk = i - c * CG_BK;
            const int k = k0 + kk;
            fv[q] = (c0 + c < nb && k < ke) ? f[(size_t)(c0 + c) * fs + k] : f2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < NXL; ++q) {
            const int i = tid + 256 * q;
            xs[i / CG_BK][i % CG_BK] = xv[q];
        }
#pragma unroll
        for (int q = 0; q < NFL; ++q) {
            const int i = tid + 256 * q;
            fsh[i / CG_BK][i % CG_BK] = fv[q];
        }
        __syncthreads();
#pragma unroll 4
        for (int kq = 0; kq < CG_BK; kq += 4) {
            const float2 b = xs[wv * 16 + lr][kq + lk];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const float2 a = fsh[t * 16 + lr][kq + lk];
                accr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, accr[t], 0, 0, 0);
                accr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, accr[t], 0, 0, 0);
                acci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, acci[t], 0, 0, 0);
                acci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, acci[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const int row = r0 + wv * 16 + lr;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = c0 + t * 16 + 4 * lk + q;
            if (row < N && c < nb) part[((size_t)sp * nb + c) * N + row] = f2(accr[t][q], acci[t][q]);
        }
}

__global__ void k_coarse_finish(const float2 *__restrict__ part, int N, int nb, float2 *__restrict__ v,
                                size_t vs, const double *__restrict__ scale, int accumulate,
                                const int *__restrict__ active)
{
    const size_t total = (size_t)nb * N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / N), row = (int)(i % N);
        if (active && !active[c]) continue;
        float2 z = part[(size_t)c * N + row];
#pragma unroll
        for (int sp = 1; sp < CG_SPLIT; ++sp) z = z + part[((size_t)sp * nb + c) * N + row];
        const float sc = scale ? (float)scale[c] : 1.f;
        z = f2(sc * z.x, sc * z.y);
        if (accumulate) z = z + v[(size_t)c * vs + row];
        v[(size_t)c * vs + row] = z;
    }
}

// ------------------------------------------------------------------ setup
__global__ void k_level_mass(const float *__restrict__ kappa, const float *__restrict__ gamma,
                             int n, int sp, double omega, float2 *__restrict__ mass, int nl)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nl * nl) return;
    int I = idx / nl, J = idx - I * nl;
    size_t p = (size_t)(I << sp) * n + (J << sp);
    double k = kappa[p], g = gamma[p];
    double w2k2 = omega * omega * k * k;
    mass[idx] = make_float2((float)w2k2, (float)(-w2k2 * g));
}

// ------------------------------------------------------------------ FP64 residual
__global__ __launch_bounds__(256) void k_true_residual(
    const float *__restrict__ kappa, const float *__restrict__ gamma, int n, double omega,
    const float2 *__restrict__ b, size_t bs, const double2 *__restrict__ x, size_t xs,
    float2 *__restrict__ r, size_t rs, double *__restrict__ partial, int nblk,
    const int *__restrict__ active)
{
    const int bi = blockIdx.y;
    if (active && !active[bi]) return;
    b += (size_t)bi * bs;
    x += (size_t)bi * xs;
    r += (size_t)bi * rs;
    const size_t N = (size_t)n * n;
    const double ih2 = (double)n * (double)n;
    double acc = 0.0;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)nblk * 256) {
        int i = (int)(p / n), j = (int)(p - (size_t)i * n);
        double2 c = x[p];
        double sr = 4.0 * c.x, si = 4.0 * c.y;
        if (i > 0) { sr -= x[p - n].x; si -= x[p - n].y; }
        if (i < n - 1) { sr -= x[p + n].x; si -= x[p + n].y; }
        if (j > 0) { sr -= x[p - 1].x; si -= x[p - 1].y; }
        if (j < n - 1) { sr -= x[p + 1].x; si -= x[p + 1].y; }
        double k = kappa[p], g = gamma[p];
        double mr = omega * omega * k * k, mi = -mr * g;
        double ar = sr * ih2 - (mr * c.x - mi * c.y);
        double ai = si * ih2 - (mr * c.y + mi * c.x);
        float2 bv = b[p];
        double rr = (double)bv.x - ar, ri = (double)bv.y - ai;
        r[p] = make_float2((float)rr, (float)ri);
        acc += rr * rr + ri * ri;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[(size_t)bi * nblk + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace

// ================================================================== launchers

void launch_apply(const Level &L, float shift, const float2 *x, size_t xs, float2 *y, size_t ys,
                  int nb, const int *active, hipStream_t s)
{
    const int n = L.n;
    const int strips = (n + 63) / 64;
    // rows per wavefront: enough waves to fill the chip, runs of up to 16
    // rows otherwise (on MI355X at 1024^2 x 32: 5.8 TB/s, against 5.6 with
    // runs of 32 and 5.76 with runs of 4)
    long long waves_at_1 = (long long)strips * n * nb;
    int R = (int)std::min<long long>(16, std::max<long long>(2, waves_at_1 / 8192));
    dim3 grid(strips, (n + 4 * R - 1) / (4 * R), nb), block(64, 4);
    prof_mark(HELM_PROF_APPLY, s, true);
    hipLaunchKernelGGL(k_apply, grid, block, 0, s, x, xs, y, ys, L.mass, n, L.ih2, shift, R,
                       active);
    // x read, y written, medium read: 24 B per point
    prof_mark(HELM_PROF_APPLY, s, false, 24.0 * n * n, nb, active != nullptr);
}

void launch_resjac(const Level &L, float shift, float w, int mode, const float2 *x, size_t xs,
                   const float2 *f, size_t fs, float2 *y, size_t ys, int nb, const int *active,
                   hipStream_t s, const double *fscale)
{
    const int n = L.n;
    const int strips = (n + 63) / 64;
    long long waves_at_1 = (long long)strips * n * nb;
    int R = (int)std::min<long long>(16, std::max<long long>(2, waves_at_1 / 8192));
    dim3 grid(strips, (n + 4 * R - 1) / (4 * R), nb), block(64, 4);
    hipLaunchKernelGGL(k_resjac, grid, block, 0, s, x, xs, f, fs, y, ys, L.mass, n, L.ih2, shift, w,
                       mode, R, active, fscale);
}

void launch_down(const Level &L, float shift, float w, const float2 *f, size_t fs, float2 *fc,
                 size_t fcs, int nb, const int *active, hipStream_t s, const double *scale)
{
    const int nc = L.n / 2;
    dim3 grid((nc + DN_CW - 1) / DN_CW, (nc + DN_CH - 1) / DN_CH, nb);
    prof_mark(HELM_PROF_DOWN, s, true);
    hipLaunchKernelGGL(k_down, grid, dim3(256), 0, s, f, fs, fc, fcs, L.mass,
                       L.n, L.ih2, shift, w, scale, active);
    // f and the medium read, the coarse residual written (the pre-smoothed
    // iterate is recomputed by the prolongation sweep, never stored): 18 B
    // per fine point
    prof_mark(HELM_PROF_DOWN, s, false, 18.0 * L.n * L.n, nb, active != nullptr);
}

void launch_up(const Level &L, float shift, float w, const float2 *f, size_t fs,
               const float2 *vc, size_t vcs, float2 *v, size_t vs, int nb, const int *active,
               hipStream_t s, const double *scale, int accumulate)
{
    const int n = L.n;
    dim3 grid((n + UP_W - 1) / UP_W, (n + UP_H - 1) / UP_H, nb);
    prof_mark(HELM_PROF_UP, s, true);
    hipLaunchKernelGGL(k_up, grid, dim3(256), 0, s, f, fs, vc, vcs, v, vs, L.mass, n, L.ih2,
                       shift, w, scale, accumulate, active);
    // f, the medium and the coarse correction read, v written (and read when
    // accumulating): 26 (34) B per fine point
    prof_mark(HELM_PROF_UP, s, false, (accumulate ? 34.0 : 26.0) * n * n, nb, active != nullptr);
}

size_t coarse_scratch(int N, int nb) { return (size_t)CG_SPLIT * nb * N; }

void launch_coarse_solve(const float2 *X, int N, const float2 *f, size_t fs, float2 *v,
                         size_t vs, int nb, const int *active, hipStream_t s, const double *scale,
                         int accumulate, float2 *scratch)
{
    dim3 grid((N + 3) / 4), block(256);
    prof_mark(HELM_PROF_COARSE, s, true);
    if (nb >= 4 && scratch) {
        // X read once for all right-hand sides
        dim3 g((N + CG_ROWS - 1) / CG_ROWS, CG_SPLIT, (nb + 31) / 32);
        hipLaunchKernelGGL(k_coarse_gemm, g, dim3(256), 0, s, X, N, f, fs, nb, scratch);
        size_t tot = (size_t)nb * N;
        hipLaunchKernelGGL(k_coarse_finish, dim3((unsigned)std::min<size_t>(8192, (tot + 255) / 256)),
                           dim3(256), 0, s, scratch, N, nb, v, vs, scale, accumulate, active);
    } else {
        int b0 = 0;
        while (b0 < nb) {
            int left = nb - b0;
            if (left >= 2) {
                hipLaunchKernelGGL(k_coarse<2>, grid, block, 0, s, X, N, f, fs, v, vs, b0, scale, accumulate,
                                   active);
                b0 += 2;
            } else {
                hipLaunchKernelGGL(k_coarse<1>, grid, block, 0, s, X, N, f, fs, v, vs, b0, scale, accumulate,
                                   active);
                b0 += 1;
            }
        }
    }
    prof_mark(HELM_PROF_COARSE, s, false, 8.0 * N * N + (accumulate ? 24.0 : 16.0) * N * nb, 1, false);
}

void launch_level_mass(const float *kappa, const float *gamma, int n, int stride_pow,
                       double omega, float2 *mass, int nl, hipStream_t s)
{
    int tot = nl * nl;
    hipLaunchKernelGGL(k_level_mass, dim3((tot + 255) / 256), dim3(256), 0, s, kappa, gamma, n,
                       stride_pow, omega, mass, nl);
}

void launch_true_residual(const float *kappa, const float *gamma, int n, double omega,
                          const float2 *b, size_t bs, const double2 *x, size_t xs, float2 *r,
                          size_t rs, double *partial, int nblk, int nb, const int *active,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_true_residual, dim3(nblk, nb), dim3(256), 0, s, kappa, gamma, n, omega,
                       b, bs, x, xs, r, rs, partial, nblk, active);
}

}  // namespace helm
