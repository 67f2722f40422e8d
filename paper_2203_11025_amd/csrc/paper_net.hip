// The paper's own network (section 3.1, eq. 3.1-3.3), FP32 on the device:
// learned 5x5 stride-2 transfers (a convolution down, a transposed
// convolution up), ResNet blocks with ELU (one per level, three at the
// coarsest), BN after every convolution but the last, and 4 input channels
// (Re r^, Im r^, kappa^2, gamma) on the fine grid; the output is the error on
// the fine grid.  Used through the unet_* entry points with cfg.arch = 1.
//
// Layout: NCHW float, batch-major.  Every convolution is one of three
// gathers between a "fine" grid (n_f) and a "coarse" grid (n_c) related by
// fine = s * coarse + a - pad for tap a (s = 2, K = 5, pad = 2 for the
// transfers; s = 1, K = 3, pad = 1 for the ResNet convolutions, where the two
// grids coincide), with weights W[c_coarse][c_fine][K][K]:
//   gather to coarse: coarse(I) = sum W fine(s I + a - pad)   (convolution;
//                     data gradient of a transposed convolution)
//   gather to fine:   fine(i) = sum W coarse((i + pad - a) / s) (transposed
//                     convolution; data gradient of a convolution)
//   weight gradient:  dW[a] = sum coarse(I) fine(s I + a - pad)
// The two gathers run as implicit GEMMs on FP32 MFMA; the weight gradient,
// BN statistics and every reduction accumulate in FP64 in a fixed order.
#include <cmath>
#include <string>
#include <vector>

#include "handle.h"
#include "paper_net.h"
#include "unet_internal.h"

namespace helm {

namespace {

constexpr int PN_T = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double pn_wsum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum of one double per thread over the 256-thread block; valid in thread 0
__device__ __forceinline__ double pn_bsum(double v, double *sh)
{
    v = pn_wsum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return t;
}

// ------------------------------------------------------------ MFMA gathers
// The two gathers as implicit GEMMs on FP32 MFMA (v_mfma_f32_16x16x4_f32:
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16], and rows
// 4 (l / 16) .. + 3 of column l % 16 of D).  The output points form
// lattices on which every tap is a plain offset: a gather to coarse has one
// lattice, the coarse grid, with input point s (Y, X) + (a - pad, c - pad);
// a gather to fine with s = 2 splits the fine grid into the four classes
// (py, px) = (i % 2, j % 2), each the lattice (Y, X) -> (2 Y + py, 2 X + px),
// reached by the taps a = py + pad (mod 2) with input point (Y, X) +
// ((py + pad - a) / 2, (px + pad - c) / 2); with s = 1 the offsets are
// (pad - a, pad - c).  Per class the GEMM is
//   D[out channel][point] = sum over (in channel, tap) of Wp[in][tap][out] X[in][point + offset(tap)],
// Wp the weights repacked so that output channels are contiguous.  A
// workgroup (NWV = 1, 2 or 4 wavefronts, as many as the output channels
// fill; wavefront w owns output channels 16 w .. + 15 of the block) owns an
// 8 x 16 tile of one lattice (8 pixel fragments, one
// per lattice row) and walks the input channels four at a time (one MFMA K
// step per tap): the input patch under the tile and the chunk's weights go
// to LDS, the next chunk's loads are in flight in registers during the
// current chunk's MFMAs (two LDS buffers, one barrier per chunk), and each
// tap costs a wavefront one A read, 8 B reads and 8 MFMAs.
constexpr int PM_TY = 8, PM_TX = 16, PM_CI = 4;

struct PmArgs {
    const float *in;
    int inC, inOff, Cin, Hin, Win;
    const float *Wp;  // [Cin][K * K][Cout]
    float *out;
    int outC, outOff, Cout, Hout, Wout;
    int mode, s, K, pad, acc;  // mode 0: gather to coarse, 1: gather to fine
    int tiles_x, tiles_per_class;
};

// Wp[i][t][o] = W[o * wco + i * wci + t] for t < K * K
__global__ void k_pn_wpack(const float *__restrict__ W, int Cout, int Cin, int KK, int wco, int wci,
                           float *__restrict__ Wp)
{
    const size_t n = (size_t)Cin * KK * Cout;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int o = (int)(e % Cout);
        const size_t r = e / Cout;
        const int t = (int)(r % KK), i = (int)(r / KK);
        Wp[e] = W[(size_t)o * wco + (size_t)i * wci + t];
    }
}

// IS: input step of the lattice (s for a gather to coarse, else 1); MAXT:
// taps of a class at most; PHM x PWM: the largest input patch of a tile
template <int IS, int MAXT, int PHM, int PWM, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_pn_mm(PmArgs g)
{
    constexpr int NT = 64 * NWV, CO = 16 * NWV;            // threads; output channels per workgroup
    constexpr int PS = PHM * PWM;                          // patch floats per channel
    constexpr int NP = (PM_CI * PS + NT - 1) / NT;         // patch loads per thread
    constexpr int NW = (MAXT * PM_CI * CO + NT - 1) / NT;   // weight loads per thread
    __shared__ float sP[2][PM_CI * PS];
    __shared__ float sW[2][MAXT * PM_CI * CO];
    __shared__ int sT[MAXT];    // per tap: (dy + 64) | (dx + 64) << 8 | (a K + c) << 16
    __shared__ int sI[3];       // taps, dymin, dxmin
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int cls = blockIdx.x / g.tiles_per_class, tile = blockIdx.x - cls * g.tiles_per_class;
    const int ty = tile / g.tiles_x, tx = tile - ty * g.tiles_x;
    const int co0 = blockIdx.y * CO, b = blockIdx.z;
    const int os = g.mode == 0 ? 1 : g.s;
    const int py = cls / os, px = cls - py * os;
    const int LY = (g.Hout - py + os - 1) / os, LX = (g.Wout - px + os - 1) / os;
    const int Y0 = ty * PM_TY, X0 = tx * PM_TX;
    if (tid == 0) {
        int nt = 0, dymin = 1 << 20, dxmin = 1 << 20;
        for (int a = 0; a < g.K; ++a) {
            int dy;
            if (g.mode == 0) {
                dy = a - g.pad;
            } else {
                const int q = py + g.pad - a;
                if (((q % g.s) + g.s) % g.s) continue;
                dy = q / g.s;
            }
            for (int c = 0; c < g.K; ++c) {
                int dx;
                if (g.mode == 0) {
                    dx = c - g.pad;
                } else {
                    const int q = px + g.pad - c;
                    if (((q % g.s) + g.s) % g.s) continue;
                    dx = q / g.s;
                }
                if (nt < MAXT) sT[nt++] = (dy + 64) | ((dx + 64) << 8) | ((a * g.K + c) << 16);
                dymin = min(dymin, dy);
                dxmin = min(dxmin, dx);
            }
        }
        sI[0] = nt;
        sI[1] = dymin;
        sI[2] = dxmin;
    }
    __syncthreads();
    const int nt = sI[0], dymin = sI[1], dxmin = sI[2];
    const int row0 = IS * Y0 + dymin, col0 = IS * X0 + dxmin;
    const float *inb = g.in + ((size_t)b * g.inC + g.inOff) * g.Hin * g.Win;
    float pp[NP], pw[NW];
    // global loads of chunk ic0 into registers (zero outside the image, the
    // input channels or the output channels)
    auto load = [&](int ic0) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int e = tid + NT * q;
            float v = 0.f;
            if (e < PM_CI * PS) {
                const int ch = e / PS, rem = e - ch * PS, r = rem / PWM, c = rem - r * PWM;
                const int ic = ic0 + ch, y = row0 + r, x = col0 + c;
                if (ic < g.Cin && y >= 0 && y < g.Hin && x >= 0 && x < g.Win)
                    v = inb[((size_t)ic * g.Hin + y) * g.Win + x];
            }
            pp[q] = v;
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int e = tid + NT * q;
            float v = 0.f;
            if (e < MAXT * PM_CI * CO) {
                const int o = e % CO, ic = (e / CO) % PM_CI, t = e / (CO * PM_CI);
                if (t < nt && ic0 + ic < g.Cin && co0 + o < g.Cout)
                    v = g.Wp[((size_t)(ic0 + ic) * g.K * g.K + (sT[t] >> 16)) * g.Cout + co0 + o];
            }
            pw[q] = v;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int e = tid + NT * q;
            if (e < PM_CI * PS) sP[buf][e] = pp[q];
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int e = tid + NT * q;
            if (e < MAXT * PM_CI * CO) sW[buf][e] = pw[q];
        }
    };
    f32x4 acc[PM_TY];
#pragma unroll
    for (int f = 0; f < PM_TY; ++f) acc[f] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nch = (g.Cin + PM_CI - 1) / PM_CI;
    load(0);
    store(0);
    __syncthreads();
    const int k = lane >> 4, j = lane & 15;
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nch;
        if (more) load((ch + 1) * PM_CI);
        const float *P = &sP[buf][k * PS + IS * j];
        const float *Wb = &sW[buf][k * CO + wv * 16 + j];
        for (int t = 0; t < nt; ++t) {
            const int tv = sT[t];
            const int dy = (tv & 255) - 64 - dymin, dx = ((tv >> 8) & 255) - 64 - dxmin;
            const float a = Wb[t * PM_CI * CO];
            const float *Pt = P + dy * PWM + dx;
#pragma unroll
            for (int f = 0; f < PM_TY; ++f)
                acc[f] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Pt[IS * f * PWM], acc[f], 0, 0, 0);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
    }
    // lane holds output channels co0 + 16 wv + 4 k .. + 3 at lattice point (Y0 + f, X0 + j)
    const int X = X0 + j;
    if (X >= LX) return;
#pragma unroll
    for (int f = 0; f < PM_TY; ++f) {
        const int Y = Y0 + f;
        if (Y >= LY) continue;
        const int oy = os * Y + py, ox = os * X + px;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int oc = co0 + wv * 16 + 4 * k + r;
            if (oc >= g.Cout) continue;
            float *o = g.out + (((size_t)b * g.outC + g.outOff + oc) * g.Hout + oy) * g.Wout + ox;
            *o = g.acc ? *o + acc[f][r] : acc[f][r];
        }
    }
}

// ------------------------------------------------------- MFMA weight gradient
// dW[cc][fc][a][c] = sum over samples and coarse points (I, J) of
// co[cc](I, J) fi[fc](s I + a - pad, s J + c - pad), per tap a GEMM over the
// points: D[cc][fc] += sum_p co[cc][p] fi_tap[fc][p] on FP32 MFMA (K step: 4
// consecutive points of a tile row).  A workgroup (4 wavefronts; wavefront w
// owns coarse channels 16 w .. + 15 of a block of 64, all K * K taps) owns 16
// fine channels and a range of 8 x 16 point tiles (split over the points);
// per tile the coarse values and the fine patch under the tile go to LDS,
// the next tile's loads in flight in registers during the MFMAs.  Partial
// sums per split, reduced in a fixed order by k_pn_wsum.  With K = 5 the 25
// taps' accumulators leave no registers for the prefetch, and a tile's
// staging waits for its loads after the barrier (the tile's 800 MFMAs per
// wavefront cover that).
constexpr int PW_TY = 8, PW_TX = 16, PW_CC = 64, PW_FC = 16, PW_SC = PW_TY * PW_TX + 4;

template <int S, int K>
__global__ __launch_bounds__(256, 2) void k_pn_mmw(const float *__restrict__ co, int coC, int coOff, int Cc, int Hc,
                                                   const float *__restrict__ fi, int fiC, int fiOff, int Cf, int Hf,
                                                   int pad, int tiles_x, int tiles_per_sample, int ntiles,
                                                   int per_split, float *__restrict__ part)
{
    constexpr int KK = K * K;
    constexpr int PH = S * (PW_TY - 1) + K, PWD = S * (PW_TX - 1) + K;  // fine patch under a tile
    constexpr int PSF = PH * PWD;
    constexpr bool PF = K <= 3;                         // prefetch the next tile in registers
    constexpr int NC = PF ? PW_CC * PW_TY * PW_TX / 256 : 1;  // coarse loads per thread
    constexpr int NF = PF ? (PW_FC * PSF + 255) / 256 : 1;    // fine loads per thread
    __shared__ float sC[PW_CC * PW_SC];
    __shared__ float sF[PW_FC * PSF];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ncb = (Cc + PW_CC - 1) / PW_CC;
    const int cc0 = (blockIdx.y % ncb) * PW_CC, fc0 = (blockIdx.y / ncb) * PW_FC;
    const int t_begin = blockIdx.x * per_split, t_end = min(ntiles, t_begin + per_split);
    f32x4 acc[KK];
#pragma unroll
    for (int t = 0; t < KK; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float pc[NC], pf[NF];
    // the tile's values straight into LDS (no prefetch)
    auto stage = [&](int tl) {
        const int b = tl / tiles_per_sample, r = tl - b * tiles_per_sample;
        const int Y0 = (r / tiles_x) * PW_TY, X0 = (r - (r / tiles_x) * tiles_x) * PW_TX;
        const float *cb = co + ((size_t)b * coC + coOff) * Hc * Hc;
        const float *fb = fi + ((size_t)b * fiC + fiOff) * Hf * Hf;
        for (int e = tid; e < PW_CC * PW_TY * PW_TX; e += 256) {
            const int c = e / (PW_TY * PW_TX), p = e - c * (PW_TY * PW_TX);
            const int Y = Y0 + p / PW_TX, X = X0 + p % PW_TX;
            float v = 0.f;
            if (cc0 + c < Cc && Y < Hc && X < Hc) v = cb[((size_t)(cc0 + c) * Hc + Y) * Hc + X];
            sC[c * PW_SC + p] = v;
        }
        const int y0 = S * Y0 - pad, x0 = S * X0 - pad;
        for (int e = tid; e < PW_FC * PSF; e += 256) {
            const int c = e / PSF, rem = e - c * PSF, rr = rem / PWD, cl = rem - rr * PWD;
            const int y = y0 + rr, x = x0 + cl;
            float v = 0.f;
            if (fc0 + c < Cf && y >= 0 && y < Hf && x >= 0 && x < Hf) v = fb[((size_t)(fc0 + c) * Hf + y) * Hf + x];
            sF[e] = v;
        }
    };
    auto load = [&](int tl) {
        const int b = tl / tiles_per_sample, r = tl - b * tiles_per_sample;
        const int Y0 = (r / tiles_x) * PW_TY, X0 = (r - (r / tiles_x) * tiles_x) * PW_TX;
        const float *cb = co + ((size_t)b * coC + coOff) * Hc * Hc;
        const float *fb = fi + ((size_t)b * fiC + fiOff) * Hf * Hf;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int e = tid + 256 * q;
            const int c = e / (PW_TY * PW_TX), p = e - c * (PW_TY * PW_TX);
            const int Y = Y0 + p / PW_TX, X = X0 + p % PW_TX;
            float v = 0.f;
            if (cc0 + c < Cc && Y < Hc && X < Hc) v = cb[((size_t)(cc0 + c) * Hc + Y) * Hc + X];
            pc[q] = v;
        }
        const int y0 = S * Y0 - pad, x0 = S * X0 - pad;
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const int e = tid + 256 * q;
            float v = 0.f;
            if (e < PW_FC * PSF) {
                const int c = e / PSF, rem = e - c * PSF, rr = rem / PWD, cl = rem - rr * PWD;
                const int y = y0 + rr, x = x0 + cl;
                if (fc0 + c < Cf && y >= 0 && y < Hf && x >= 0 && x < Hf)
                    v = fb[((size_t)(fc0 + c) * Hf + y) * Hf + x];
            }
            pf[q] = v;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int e = tid + 256 * q;
            const int c = e / (PW_TY * PW_TX), p = e - c * (PW_TY * PW_TX);
            sC[c * PW_SC + p] = pc[q];
        }
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const int e = tid + 256 * q;
            if (e < PW_FC * PSF) sF[e] = pf[q];
        }
    };
    const int k = lane >> 4, j = lane & 15;
    if (t_begin < t_end) {
        if constexpr (PF) {
            load(t_begin);
            store();
        } else {
            stage(t_begin);
        }
    }
    __syncthreads();
    for (int tl = t_begin; tl < t_end; ++tl) {
        const bool more = tl + 1 < t_end;
        if constexpr (PF)
            if (more) load(tl + 1);
        // points p = 4 q + k of the tile: row p / 16, column p % 16
        const float *Cw = &sC[(wv * 16 + j) * PW_SC + k];
        const float *Fj = &sF[j * PSF];
#pragma unroll 2
        for (int q = 0; q < PW_TY * PW_TX / 4; ++q) {
            const int p = 4 * q + k, py = p / PW_TX, px = p % PW_TX;
            const float a = Cw[4 * q];
            const float *Fp = Fj + S * py * PWD + S * px;
#pragma unroll
            for (int ta = 0; ta < K; ++ta)
#pragma unroll
                for (int tc = 0; tc < K; ++tc)
                    acc[ta * K + tc] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(a, Fp[ta * PWD + tc], acc[ta * K + tc], 0, 0, 0);
        }
        if (more) {
            __syncthreads();  // every wavefront is done with this tile
            if constexpr (PF)
                store();
            else
                stage(tl + 1);
            __syncthreads();
        }
    }
    // D[cc][fc]: lane holds fine channel fc0 + j and coarse channels cc0 + 16 wv + 4 k .. + 3
    const size_t per = (size_t)Cc * Cf * KK;
#pragma unroll
    for (int t = 0; t < KK; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int cc = cc0 + wv * 16 + 4 * k + r, fc = fc0 + j;
            if (cc < Cc && fc < Cf) part[blockIdx.x * per + ((size_t)cc * Cf + fc) * KK + t] = acc[t][r];
        }
}

// dW[e] += sum over splits of part[split][e] (FP64, split order)
__global__ void k_pn_wsum(const float *__restrict__ part, int nsplit, size_t n, float *__restrict__ dW)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < nsplit; ++q) s += part[(size_t)q * n + e];
        dW[e] += (float)s;
    }
}

// BN statistics of channel c (blockIdx.x) over B x HW: mean, var (biased),
// and the scale / shift of the batch normalisation with weight g, bias bb
// The per-channel reductions over B x HW values run in nsplit contiguous
// ranges per channel (grid (nsplit, C)), each block writing its FP64 pair
// to part[(c nsplit + split) 2 + k]; k_pn_psum adds a channel's pairs in
// split order.
__device__ __forceinline__ void pn_range(int B, int HW, int nsplit, size_t &q0, size_t &q1)
{
    const size_t N = (size_t)B * HW, per = (N + nsplit - 1) / nsplit;
    q0 = (size_t)blockIdx.x * per;
    q1 = q0 + per < N ? q0 + per : N;
}

__device__ __forceinline__ void pn_put(double s1, double s2, int nsplit, double *part)
{
    __shared__ double sh[4];
    s1 = pn_bsum(s1, sh);
    s2 = pn_bsum(s2, sh);
    if (threadIdx.x == 0) {
        const size_t o = ((size_t)blockIdx.y * nsplit + blockIdx.x) * 2;
        part[o] = s1;
        part[o + 1] = s2;
    }
}

// sums[2 c + k] = sum over splits of part (thread per channel)
__global__ void k_pn_psum(const double *__restrict__ part, int nsplit, int C, double *__restrict__ sums)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s1 = 0.0, s2 = 0.0;
    for (int q = 0; q < nsplit; ++q) {
        s1 += part[((size_t)c * nsplit + q) * 2];
        s2 += part[((size_t)c * nsplit + q) * 2 + 1];
    }
    sums[2 * c] = s1;
    sums[2 * c + 1] = s2;
}

// partial sums of y and y^2 of channel blockIdx.y
__global__ __launch_bounds__(PN_T) void k_pn_bn_stats(const float *__restrict__ y, int yC, int yOff, int B, int HW,
                                                      int nsplit, double *__restrict__ part)
{
    const int c = blockIdx.y;
    size_t q0, q1;
    pn_range(B, HW, nsplit, q0, q1);
    double s1 = 0.0, s2 = 0.0;
    for (size_t q = q0 + threadIdx.x; q < q1; q += PN_T) {
        const size_t b = q / HW, p = q - b * HW;
        const double v = y[((b * yC) + yOff + c) * HW + p];
        s1 += v;
        s2 += v * v;
    }
    pn_put(s1, s2, nsplit, part);
}

// mean, var (biased), rstd and the BN scale / shift from the sums (thread per channel)
__global__ void k_pn_bn_stats_fin(const double *__restrict__ sums, int C, double N, const float *__restrict__ g,
                                  const float *__restrict__ bb, float eps, float *__restrict__ mean,
                                  float *__restrict__ var, float *__restrict__ rstd, float *__restrict__ sc,
                                  float *__restrict__ sf)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const double s1 = sums[2 * c], s2 = sums[2 * c + 1];
    {
        const double m = s1 / N, vv = std::max(s2 / N - m * m, 0.0);
        const double r = 1.0 / std::sqrt(vv + (double)eps);
        mean[c] = (float)m;
        var[c] = (float)vv;
        rstd[c] = (float)r;
        sc[c] = (float)(g[c] * r);
        sf[c] = (float)(bb[c] - m * g[c] * r);
    }
}

// out = sc * in + sf per channel, then ELU when act; grid (tiles, B*C)
__global__ __launch_bounds__(PN_T) void k_pn_bn_apply(const float *__restrict__ in, int inC, int inOff,
                                                      float *__restrict__ out, int outC, int outOff, int C, int HW,
                                                      const float *__restrict__ sc, const float *__restrict__ sf,
                                                      int act)
{
    const int b = blockIdx.y / C, c = blockIdx.y - b * C;
    const int p = blockIdx.x * PN_T + threadIdx.x;
    if (p >= HW) return;
    float z = in[((size_t)b * inC + inOff + c) * HW + p] * sc[c] + sf[c];
    if (act) z = z > 0.f ? z : expm1f(z);
    out[((size_t)b * outC + outOff + c) * HW + p] = z;
}

// per-channel sums of dz and dz * yhat for the BN backward, dz = d_out
// (times elu'(z) from the stored output a when act: 1 for a > 0, a + 1
// otherwise); yhat = (y - mean) rstd.  red[c] = (sum dz, sum dz yhat).
__global__ __launch_bounds__(PN_T) void k_pn_bn_bsum(const float *__restrict__ dout, int dC, int dOff,
                                                     const float *__restrict__ a, int aC, int aOff,
                                                     const float *__restrict__ y, int yC, int yOff, int B, int HW,
                                                     const float *__restrict__ mean, const float *__restrict__ rstd,
                                                     int act, int nsplit, double *__restrict__ part)
{
    const int c = blockIdx.y;
    size_t q0, q1;
    pn_range(B, HW, nsplit, q0, q1);
    double s1 = 0.0, s2 = 0.0;
    const float m = mean[c], r = rstd[c];
    for (size_t q = q0 + threadIdx.x; q < q1; q += PN_T) {
        const size_t b = q / HW, p = q - b * HW;
        float dz = dout[((b * dC) + dOff + c) * HW + p];
        if (act) {
            const float av = a[((b * aC) + aOff + c) * HW + p];
            dz *= av > 0.f ? 1.f : av + 1.f;
        }
        const float yh = (y[((b * yC) + yOff + c) * HW + p] - m) * r;
        s1 += dz;
        s2 += (double)dz * yh;
    }
    pn_put(s1, s2, nsplit, part);
}

// dy += g rstd (dz - sum dz / N - yhat sum dz yhat / N); grid (tiles, B*C)
__global__ __launch_bounds__(PN_T) void k_pn_bn_bapply(const float *__restrict__ dout, int dC, int dOff,
                                                       const float *__restrict__ a, int aC, int aOff,
                                                       const float *__restrict__ y, int yC, int yOff,
                                                       float *__restrict__ dy, int dyC, int dyOff, int B, int C,
                                                       int HW, const float *__restrict__ mean,
                                                       const float *__restrict__ rstd, const float *__restrict__ g,
                                                       int act, const double *__restrict__ red)
{
    const int b = blockIdx.y / C, c = blockIdx.y - b * C;
    const int p = blockIdx.x * PN_T + threadIdx.x;
    if (p >= HW) return;
    const double N = (double)B * HW;
    float dz = dout[((size_t)b * dC + dOff + c) * HW + p];
    if (act) {
        const float av = a[((size_t)b * aC + aOff + c) * HW + p];
        dz *= av > 0.f ? 1.f : av + 1.f;
    }
    const float r = rstd[c], yh = (y[((size_t)b * yC + yOff + c) * HW + p] - mean[c]) * r;
    const float v = g[c] * r * (dz - (float)(red[2 * c] / N) - yh * (float)(red[2 * c + 1] / N));
    dy[((size_t)b * dyC + dyOff + c) * HW + p] += v;
}

// dg += sum dz yhat, db += sum dz (one thread per channel)
__global__ void k_pn_bn_pgrad(const double *__restrict__ red, int C, float *__restrict__ dg, float *__restrict__ db)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    dg[c] += (float)red[2 * c + 1];
    db[c] += (float)red[2 * c];
}

// out = elu(in) over whole tensors (n elements)
__global__ void k_pn_elu(const float *__restrict__ in, float *__restrict__ out, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * PN_T + threadIdx.x; i < n; i += (size_t)gridDim.x * PN_T) {
        const float z = in[i];
        out[i] = z > 0.f ? z : expm1f(z);
    }
}

// din += dout * elu'(in) from the output a = elu(in)
__global__ void k_pn_elu_b(const float *__restrict__ dout, const float *__restrict__ a, float *__restrict__ din,
                           size_t n)
{
    for (size_t i = (size_t)blockIdx.x * PN_T + threadIdx.x; i < n; i += (size_t)gridDim.x * PN_T) {
        const float av = a[i];
        din[i] += dout[i] * (av > 0.f ? 1.f : av + 1.f);
    }
}

// out = x + y (tensors of one shape), or x += y with out == x
__global__ void k_pn_add(const float *x, const float *__restrict__ y, float *out, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * PN_T + threadIdx.x; i < n; i += (size_t)gridDim.x * PN_T) out[i] = x[i] + y[i];
}

// out[b][c] += bias[c] over HW; grid (tiles, B*C)
__global__ void k_pn_bias(float *__restrict__ out, int C, int HW, const float *__restrict__ bias)
{
    const int c = blockIdx.y % C;
    const int p = blockIdx.x * PN_T + threadIdx.x;
    if (p < HW) out[(size_t)blockIdx.y * HW + p] += bias[c];
}

// partial sums over samples and points of dout of channel blockIdx.y (the bias gradient)
__global__ __launch_bounds__(PN_T) void k_pn_bias_g(const float *__restrict__ dout, int B, int C, int HW, int nsplit,
                                                    double *__restrict__ part)
{
    const int c = blockIdx.y;
    size_t q0, q1;
    pn_range(B, HW, nsplit, q0, q1);
    double s = 0.0;
    for (size_t q = q0 + threadIdx.x; q < q1; q += PN_T) {
        const size_t b = q / HW, p = q - b * HW;
        s += dout[(b * C + c) * HW + p];
    }
    pn_put(s, 0.0, nsplit, part);
}

// db[c] += sums[2 c] (thread per channel)
__global__ void k_pn_bias_fin(const double *__restrict__ sums, int C, float *__restrict__ db)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C) db[c] += (float)sums[2 * c];
}

// network input: sample q reads field b = idx ? idx[q] : q, scaled by
// fscale[b] when given: u = h^2 fscale r_b; s_q = RMS |u|; x0[q] =
// (Re u / s_q, Im u / s_q, kappa^2, gamma) (zero when s_q = 0).  kappa and
// gamma: [n][n] shared by the batch (kstride 0) or per sample.  grid (nq)
__global__ __launch_bounds__(PN_T) void k_pn_input(const float2 *__restrict__ r, size_t rs, int n,
                                                   const float *__restrict__ kap, const float *__restrict__ gam,
                                                   size_t kstride, const int *__restrict__ idx,
                                                   const double *__restrict__ fscale, double *__restrict__ sq,
                                                   float *__restrict__ x0)
{
    const int q = blockIdx.x;
    const int b = idx ? idx[q] : q;
    const size_t N = (size_t)n * n;
    const float2 *rb = r + (size_t)b * rs;
    const double h2 = 1.0 / ((double)n * n), f = fscale ? fscale[b] : 1.0;
    double s2 = 0.0;
    for (size_t p = threadIdx.x; p < N; p += PN_T) {
        const float2 v = rb[p];
        s2 += (double)v.x * v.x + (double)v.y * v.y;
    }
    __shared__ double sh[4];
    __shared__ double ssh;
    s2 = pn_bsum(s2, sh);
    if (threadIdx.x == 0) {
        const double s = std::fabs(f) * h2 * std::sqrt(s2 / (double)N);
        ssh = s;
        sq[q] = s;
    }
    __syncthreads();
    const double s = ssh;
    const float k = s > 0.0 ? (float)(f * h2 / s) : 0.f;
    const float *kb = kap + (size_t)q * kstride, *gb = gam + (size_t)q * kstride;
    float *x = x0 + (size_t)q * 4 * N;
    for (size_t p = threadIdx.x; p < N; p += PN_T) {
        const float2 v = rb[p];
        const float kk = kb[p];
        x[p] = k * v.x;
        x[N + p] = k * v.y;
        x[2 * N + p] = kk * kk;
        x[3 * N + p] = gb[p];
    }
}

// e_b (+)= s_q (out0 + i out1), q = pos ? pos[b] : b; q < 0 or mask[b] == 0:
// e_b = 0 (untouched when accumulating).  grid (tiles of N, nb)
__global__ void k_pn_output(const float *__restrict__ out, const double *__restrict__ sq, int n, float2 *e, size_t es,
                            int accumulate, const int *__restrict__ mask, const int *__restrict__ pos)
{
    const int b = blockIdx.y;
    const size_t N = (size_t)n * n;
    const size_t p = (size_t)blockIdx.x * PN_T + threadIdx.x;
    if (p >= N) return;
    const int q = pos ? pos[b] : b;
    float2 *eb = e + (size_t)b * es;
    if (q < 0 || (mask && !mask[b])) {
        if (!accumulate) eb[p] = make_float2(0.f, 0.f);
        return;
    }
    const float s = (float)sq[q];
    const float *o = out + (size_t)q * 2 * N;
    float2 v = make_float2(s * o[p], s * o[N + p]);
    if (accumulate) v = make_float2(eb[p].x + v.x, eb[p].y + v.y);
    eb[p] = v;
}

// loss parts and gradient: d = out_b - e_b / s_b, part[b] = sum |d|^2,
// dout = 2 d / (B n^2).  grid (B)
__global__ __launch_bounds__(PN_T) void k_pn_loss(const float *__restrict__ out, const double *__restrict__ sq, int n,
                                                  int B, const float2 *__restrict__ e, float *__restrict__ dout,
                                                  double *__restrict__ part)
{
    const int b = blockIdx.x;
    const size_t N = (size_t)n * n;
    const double s = sq[b];
    const float is = s > 0.0 ? (float)(1.0 / s) : 0.f, k = (float)(2.0 / ((double)B * N));
    double acc = 0.0;
    for (size_t p = threadIdx.x; p < N; p += PN_T) {
        const float2 t = e[(size_t)b * N + p];
        const float d0 = out[(size_t)b * 2 * N + p] - t.x * is, d1 = out[(size_t)b * 2 * N + N + p] - t.y * is;
        acc += (double)d0 * d0 + (double)d1 * d1;
        dout[(size_t)b * 2 * N + p] = k * d0;
        dout[(size_t)b * 2 * N + N + p] = k * d1;
    }
    __shared__ double sh[4];
    acc = pn_bsum(acc, sh);
    if (threadIdx.x == 0) part[b] = acc;
}

int tiles(size_t n) { return (int)((n + PN_T - 1) / PN_T); }

// ranges per channel of a reduction over n values: about 1024 blocks in all,
// at most 64 per channel (so C nsplit <= 1024 for C <= 512), 1024 values each at least
int pn_nsplit(int C, size_t n)
{
    return (int)std::max<size_t>(1, std::min<size_t>({(size_t)64, (size_t)(1024 / C), n / 1024}));
}

}  // namespace

// ------------------------------------------------------------------ PaperNet

void PaperNet::build(const int *widths, int levels, int in_ch, int out_ch, int coarsest_blocks)
{
    L = levels;
    cin = in_ch;
    cout = out_ch;
    w.assign(widths, widths + levels);
    layers.clear();
    size_t off = 0, boff = 0;
    auto add = [&](int kind, int ci, int co, int K) {
        PLayer l;
        l.kind = kind;
        l.ci = ci;
        l.co = co;
        l.K = K;
        l.w_off = off;
        off += (size_t)ci * co * K * K;
        if (kind == PL_OUT) {
            l.b_off = off;
            off += co;
        } else {
            l.g_off = off;
            l.b_off = off + co;
            off += 2 * (size_t)co;
            l.rm_off = boff;
            l.rv_off = boff + co;
            boff += 2 * (size_t)co;
            l.bn = nbn++;
        }
        layers.push_back(l);
        return (int)layers.size() - 1;
    };
    nbn = 0;
    int c_in = in_ch;
    for (int l = 1; l <= L; ++l) {
        const int c = w[l - 1];
        add(PL_DOWN, c_in, c, 5);
        const int nb = l == L ? coarsest_blocks : 1;
        for (int r = 0; r < nb; ++r) {
            add(PL_RES1, c, c, 3);
            add(PL_RES2, c, c, 3);
        }
        c_in = c;
    }
    int ch = w[L - 1];
    for (int l = L - 1; l >= 1; --l) {
        add(PL_UP, ch, w[l - 1], 5);
        ch = 2 * w[l - 1];
    }
    add(PL_OUT, ch, out_ch, 5);
    nparams = off;
    nbuf = boff;
    cblocks = coarsest_blocks;
}

PaperNet::~PaperNet() { free_all(); }

// one gather (mode 0: to coarse, 1: to fine; see above) through the MFMA
// kernel: the weights W[c_coarse][c_fine][K][K] are repacked output-channel
// contiguous into wpk first
void PaperNet::gather(int mode, const float *in, int inC, int inOff, int Cin, int Hin, const float *W, float *out,
                      int outC, int outOff, int Cout, int Hout, int s, int K, int pad, int acc, int B, hipStream_t st)
{
    const int KK = K * K;
    const int wco = mode == 0 ? Cin * KK : KK, wci = mode == 0 ? KK : Cout * KK;
    const size_t nw = (size_t)Cin * KK * Cout;
    hipLaunchKernelGGL(k_pn_wpack, dim3((unsigned)std::min<size_t>(1024, (nw + 255) / 256)), dim3(256), 0, st, W,
                       Cout, Cin, KK, wco, wci, wpk);
    PmArgs g{in, inC, inOff, Cin, Hin, Hin, wpk, out, outC, outOff, Cout, Hout, Hout, mode, s, K, pad, acc, 0, 0};
    const int os = mode == 0 ? 1 : s;
    const int L = (Hout + os - 1) / os;  // lattice side of class (0, 0), the largest
    g.tiles_x = (L + PM_TX - 1) / PM_TX;
    g.tiles_per_class = g.tiles_x * ((L + PM_TY - 1) / PM_TY);
    // wavefronts per workgroup: as many 16-channel fragments as Cout fills, at most 4
    const int nwv = Cout <= 16 ? 1 : Cout <= 32 ? 2 : 4;
    const dim3 grid(g.tiles_per_class * os * os, (Cout + 16 * nwv - 1) / (16 * nwv), B);
    const bool big = mode == 0 && s == 2 && K == 5;  // else mode 0 with s = 1, K = 3, or mode 1 (checked at build)
#define PN_MM(NWV)                                                                        \
    do {                                                                                  \
        if (big)                                                                          \
            hipLaunchKernelGGL((k_pn_mm<2, 25, 19, 35, NWV>), grid, dim3(64 * NWV), 0, st, g); \
        else                                                                              \
            hipLaunchKernelGGL((k_pn_mm<1, 9, 10, 18, NWV>), grid, dim3(64 * NWV), 0, st, g);  \
    } while (0)
    if (nwv == 1)
        PN_MM(1);
    else if (nwv == 2)
        PN_MM(2);
    else
        PN_MM(4);
#undef PN_MM
}

// dW (+)= the weight gradient of one transfer or ResNet convolution (coarse
// tensor co, fine tensor fi; see k_pn_mmw), split over the points so that
// about 512 workgroups run
void PaperNet::wgrad(const float *co, int coC, int coOff, int Cc, int Hc, const float *fi, int fiC, int fiOff, int Cf,
                     int Hf, int s, int K, int pad, int B, float *dW, hipStream_t st)
{
    const int tiles_x = (Hc + PW_TX - 1) / PW_TX, tps = tiles_x * ((Hc + PW_TY - 1) / PW_TY);
    const int ntiles = B * tps;
    const int blocks = ((Cc + PW_CC - 1) / PW_CC) * ((Cf + PW_FC - 1) / PW_FC);
    int nsplit = std::max(1, std::min(512 / blocks, ntiles));
    const int per = (ntiles + nsplit - 1) / nsplit;
    nsplit = (ntiles + per - 1) / per;
    const size_t n = (size_t)Cc * Cf * K * K;
    const dim3 grid(nsplit, blocks);
    if (s == 2 && K == 5)
        hipLaunchKernelGGL((k_pn_mmw<2, 5>), grid, dim3(256), 0, st, co, coC, coOff, Cc, Hc, fi, fiC, fiOff, Cf, Hf,
                           pad, tiles_x, tps, ntiles, per, wgp);
    else  // s = 1, K = 3 (checked at build)
        hipLaunchKernelGGL((k_pn_mmw<1, 3>), grid, dim3(256), 0, st, co, coC, coOff, Cc, Hc, fi, fiC, fiOff, Cf, Hf,
                           pad, tiles_x, tps, ntiles, per, wgp);
    hipLaunchKernelGGL(k_pn_wsum, dim3((unsigned)std::min<size_t>(2048, (n + 255) / 256)), dim3(256), 0, st, wgp,
                       nsplit, n, dW);
}

void PaperNet::free_ws()
{
    for (auto &t : T) {
        (void)dev_free(t.v);
        (void)dev_free(t.g);
    }
    T.clear();
    ops.clear();
    (void)dev_free(sq);
    (void)dev_free(part);
    (void)dev_free(red);
    (void)dev_free(rpart);
    sq = nullptr;
    part = nullptr;
    red = nullptr;
    rpart = nullptr;
    wsB = wsN = 0;
    wsTrain = false;
}

void PaperNet::free_all()
{
    free_ws();
    (void)dev_free(bnf);
    (void)dev_free(dlast_buf);
    (void)dev_free(wpk);
    (void)dev_free(wgp);
    bnf = dlast_buf = wpk = wgp = nullptr;
}

// the BN scratch arrays; the parameters, their gradient, the Adam moments
// and the buffers belong to the owning unet_net
int PaperNet::alloc_params()
{
    size_t nw = 1;
    for (const auto &l : layers) nw = std::max(nw, (size_t)l.ci * l.co * l.K * l.K);
    // weight-gradient partials: at most 512 / blocks splits of Cc Cf K^2, so
    // 512 x 64 x 16 x 25 floats, or one layer's weights when a layer has
    // more than 512 blocks
    const size_t np = std::max(nw, (size_t)512 * PW_CC * PW_FC * 25);
    if (dev_malloc(&bnf, std::max<size_t>(7 * (nbuf / 2), 1) * 4) != hipSuccess ||
        dev_malloc(&wpk, nw * sizeof(float)) != hipSuccess || dev_malloc(&wgp, np * sizeof(float)) != hipSuccess) {
        set_error("unet (paper network): device allocation failed");
        return HELM_E_NOMEM;
    }
    return HELM_OK;
}

// per BN layer, 7 float arrays of its channels: mean, var, rstd, scale,
// shift (training), scale, shift (inference)
float *PaperNet::bnarr(int bn, int which) const
{
    size_t off = 0;
    for (const auto &l : layers)
        if (l.kind != PL_OUT && l.bn < bn) off += 7 * (size_t)l.co;
    int co = 0;
    for (const auto &l : layers)
        if (l.kind != PL_OUT && l.bn == bn) co = l.co;
    return bnf + off + (size_t)which * co;
}

int PaperNet::tensor(int C, int n, bool train)
{
    PTensor t;
    t.C = C;
    t.n = n;
    const size_t bytes = (size_t)wsB * C * n * n * sizeof(float);
    if (dev_malloc(&t.v, bytes) != hipSuccess || (train && dev_malloc(&t.g, bytes) != hipSuccess)) return -1;
    T.push_back(t);
    return (int)T.size() - 1;
}

int PaperNet::ensure_ws(int B, int n, bool train)
{
    if (B <= wsB && n == wsN && (!train || wsTrain)) return HELM_OK;
    const int nB = std::max(B, wsB);
    const bool tr = train || wsTrain;
    free_ws();
    wsB = nB;
    wsN = n;
    wsTrain = tr;
    auto fail = [&]() {
        free_ws();
        set_error("unet (paper network): out of device memory for the workspace");
        return HELM_E_NOMEM;
    };
    // tensors and the op list of eq. 3.1-3.3
    x0t = tensor(cin, n, tr);
    if (x0t < 0) return fail();
    int li = 0;
    std::vector<int> cat(L + 1, -1);
    // concatenation buffers of the up path: level l (1 <= l < L) holds
    // [BN(P elu(y^(l+1))), x^(l)] with 2 w_l channels
    for (int l = 1; l < L; ++l)
        if ((cat[l] = tensor(2 * w[l - 1], n >> l, tr)) < 0) return fail();
    PView cur{x0t, 0, cin};
    for (int l = 1; l <= L; ++l) {
        const int c = w[l - 1], nl = n >> l;
        // down: y = R cur; a = elu(BN(y))
        const int yd = tensor(c, nl, tr), ad = tensor(c, nl, tr);
        if (yd < 0 || ad < 0) return fail();
        ops.push_back(POp{PO_CONV, cur, {}, {yd, 0, c}, li, 2, 2});
        ops.push_back(POp{PO_BN, {yd, 0, c}, {}, {ad, 0, c}, li, 0, 0, true});
        ++li;
        PView h{ad, 0, c};
        const int nb = l == L ? cblocks : 1;
        for (int r = 0; r < nb; ++r) {
            const bool last = r == nb - 1;
            const int y1 = tensor(c, nl, tr), t1 = tensor(c, nl, tr), y2 = tensor(c, nl, tr),
                      s2 = tensor(c, nl, tr);
            if (y1 < 0 || t1 < 0 || y2 < 0 || s2 < 0) return fail();
            PView outv;
            if (last && l < L) {
                outv = PView{cat[l], c, c};  // the skip half of the level's concatenation
            } else {
                const int a2 = tensor(c, nl, tr);
                if (a2 < 0) return fail();
                outv = PView{a2, 0, c};
            }
            ops.push_back(POp{PO_CONV, h, {}, {y1, 0, c}, li, 1, 1});
            ops.push_back(POp{PO_BN, {y1, 0, c}, {}, {t1, 0, c}, li, 0, 0, true});
            ++li;
            ops.push_back(POp{PO_CONV, {t1, 0, c}, {}, {y2, 0, c}, li, 1, 1});
            ops.push_back(POp{PO_ADD, {y2, 0, c}, h, {s2, 0, c}, -1});
            ops.push_back(POp{PO_BN, {s2, 0, c}, {}, outv, li, 0, 0, true});
            ++li;
            h = outv;
        }
        cur = h;
    }
    // up: v = elu(y^(l+1)); u = BN(P v) into cat[l][0, w_l)
    PView y = cur;
    for (int l = L - 1; l >= 1; --l) {
        const int c = w[l - 1], nl = n >> l;
        const int v = tensor(y.C, n >> (l + 1), tr), yu = tensor(c, nl, tr);
        if (v < 0 || yu < 0) return fail();
        ops.push_back(POp{PO_ELU, y, {}, {v, 0, y.C}, -1});
        ops.push_back(POp{PO_CONVT, {v, 0, y.C}, {}, {yu, 0, c}, li, 2, 2});
        ops.push_back(POp{PO_BN, {yu, 0, c}, {}, {cat[l], 0, c}, li, 0, 0, false});
        ++li;
        y = PView{cat[l], 0, 2 * c};
    }
    const int vo = tensor(y.C, n >> 1, tr);
    outt = tensor(cout, n, tr);
    if (vo < 0 || outt < 0) return fail();
    ops.push_back(POp{PO_ELU, y, {}, {vo, 0, y.C}, -1});
    ops.push_back(POp{PO_CONVT, {vo, 0, y.C}, {}, {outt, 0, cout}, li, 2, 2});
    ops.push_back(POp{PO_BIAS, {outt, 0, cout}, {}, {outt, 0, cout}, li});
    if (dev_malloc(&sq, (size_t)wsB * sizeof(double)) != hipSuccess ||
        dev_malloc(&part, (size_t)wsB * sizeof(double)) != hipSuccess ||
        dev_malloc(&red, 2 * 512 * sizeof(double)) != hipSuccess ||
        dev_malloc(&rpart, 2 * 1024 * sizeof(double)) != hipSuccess)
        return fail();
    return HELM_OK;
}

void PaperNet::forward(int B, bool training, hipStream_t st)
{
    for (const POp &o : ops) {
        const PTensor &ti = T[o.in.t], &to = T[o.out.t];
        const int ni = ti.n, no = to.n;
        if (o.kind == PO_CONV || o.kind == PO_CONVT) {
            const PLayer &l = layers[o.layer];
            const float *Wt = P + l.w_off;
            gather(o.kind == PO_CONV ? 0 : 1, ti.v, ti.C, o.in.off, l.ci, ni, Wt, to.v, to.C, o.out.off, l.co, no,
                   o.s, l.K, o.pad, 0, B, st);
        } else if (o.kind == PO_BN) {
            const PLayer &l = layers[o.layer];
            float *sc, *sf;
            if (training) {
                const int ns = pn_nsplit(l.co, (size_t)B * ni * ni);
                hipLaunchKernelGGL(k_pn_bn_stats, dim3(ns, l.co), dim3(PN_T), 0, st, ti.v, ti.C, o.in.off, B, ni * ni,
                                   ns, rpart);
                hipLaunchKernelGGL(k_pn_psum, dim3((l.co + 63) / 64), dim3(64), 0, st, rpart, ns, l.co, red);
                hipLaunchKernelGGL(k_pn_bn_stats_fin, dim3((l.co + 63) / 64), dim3(64), 0, st, red, l.co,
                                   (double)B * ni * ni, P + l.g_off, P + l.b_off, 1e-5f, bnarr(l.bn, 0),
                                   bnarr(l.bn, 1), bnarr(l.bn, 2), bnarr(l.bn, 3), bnarr(l.bn, 4));
                sc = bnarr(l.bn, 3);
                sf = bnarr(l.bn, 4);
            } else {
                sc = bnarr(l.bn, 5);
                sf = bnarr(l.bn, 6);
            }
            hipLaunchKernelGGL(k_pn_bn_apply, dim3(tiles((size_t)ni * ni), B * l.co), dim3(PN_T), 0, st, ti.v, ti.C,
                               o.in.off, to.v, to.C, o.out.off, l.co, ni * ni, sc, sf, o.act ? 1 : 0);
        } else if (o.kind == PO_ELU) {
            // whole tensors only (the views of ELU ops cover their tensor)
            const size_t n = (size_t)B * ti.C * ni * ni;
            hipLaunchKernelGGL(k_pn_elu, dim3(std::min(tiles(n), 4096)), dim3(PN_T), 0, st, ti.v, to.v, n);
        } else if (o.kind == PO_ADD) {
            const size_t n = (size_t)B * ti.C * ni * ni;
            hipLaunchKernelGGL(k_pn_add, dim3(std::min(tiles(n), 4096)), dim3(PN_T), 0, st, ti.v, T[o.in2.t].v, to.v,
                               n);
        } else if (o.kind == PO_BIAS) {
            const PLayer &l = layers[o.layer];
            hipLaunchKernelGGL(k_pn_bias, dim3(tiles((size_t)no * no), B * l.co), dim3(PN_T), 0, st, to.v, l.co,
                               no * no, P + l.b_off);
        }
    }
}

void PaperNet::backward(int B, hipStream_t st)
{
    for (auto &t : T) (void)hipMemsetAsync(t.g, 0, (size_t)wsB * t.C * t.n * t.n * sizeof(float), st);
    (void)hipMemsetAsync(G, 0, nparams * sizeof(float), st);
    // the caller has written d out into T[outt].g (after the zeroing)
    (void)hipMemcpyAsync(T[outt].g, dlast, (size_t)B * cout * wsN * wsN * sizeof(float), hipMemcpyDeviceToDevice, st);
    for (int k = (int)ops.size() - 1; k >= 0; --k) {
        const POp &o = ops[k];
        const PTensor &ti = T[o.in.t], &to = T[o.out.t];
        const int ni = ti.n, no = to.n;
        if (o.kind == PO_CONV) {
            // out = gather_coarse(in): d in += gather_fine(d out), dW += wg(coarse = d out, fine = in)
            const PLayer &l = layers[o.layer];
            if (o.in.t != x0t)
                gather(1, to.g, to.C, o.out.off, l.co, no, P + l.w_off, ti.g, ti.C, o.in.off, l.ci, ni, o.s, l.K, o.pad,
                       1, B, st);
            wgrad(to.g, to.C, o.out.off, l.co, no, ti.v, ti.C, o.in.off, l.ci, ni, o.s, l.K, o.pad, B, G + l.w_off, st);
        } else if (o.kind == PO_CONVT) {
            // out = gather_fine(in): d in += gather_coarse(d out), dW += wg(coarse = in, fine = d out)
            const PLayer &l = layers[o.layer];
            gather(0, to.g, to.C, o.out.off, l.co, no, P + l.w_off, ti.g, ti.C, o.in.off, l.ci, ni, o.s, l.K, o.pad,
                   1, B, st);
            wgrad(ti.v, ti.C, o.in.off, l.ci, ni, to.g, to.C, o.out.off, l.co, no, o.s, l.K, o.pad, B, G + l.w_off, st);
        } else if (o.kind == PO_BN) {
            const PLayer &l = layers[o.layer];
            const int act = o.act ? 1 : 0;
            const int ns = pn_nsplit(l.co, (size_t)B * ni * ni);
            hipLaunchKernelGGL(k_pn_bn_bsum, dim3(ns, l.co), dim3(PN_T), 0, st, to.g, to.C, o.out.off, to.v, to.C,
                               o.out.off, ti.v, ti.C, o.in.off, B, ni * ni, bnarr(l.bn, 0), bnarr(l.bn, 2), act, ns,
                               rpart);
            hipLaunchKernelGGL(k_pn_psum, dim3((l.co + 63) / 64), dim3(64), 0, st, rpart, ns, l.co, red);
            hipLaunchKernelGGL(k_pn_bn_bapply, dim3(tiles((size_t)ni * ni), B * l.co), dim3(PN_T), 0, st, to.g, to.C,
                               o.out.off, to.v, to.C, o.out.off, ti.v, ti.C, o.in.off, ti.g, ti.C, o.in.off, B, l.co,
                               ni * ni, bnarr(l.bn, 0), bnarr(l.bn, 2), P + l.g_off, act, red);
            hipLaunchKernelGGL(k_pn_bn_pgrad, dim3((l.co + 63) / 64), dim3(64), 0, st, red, l.co, G + l.g_off,
                               G + l.b_off);
        } else if (o.kind == PO_ELU) {
            const size_t n = (size_t)B * ti.C * ni * ni;
            hipLaunchKernelGGL(k_pn_elu_b, dim3(std::min(tiles(n), 4096)), dim3(PN_T), 0, st, to.g, to.v, ti.g, n);
        } else if (o.kind == PO_ADD) {
            const size_t n = (size_t)B * ti.C * ni * ni;
            hipLaunchKernelGGL(k_pn_add, dim3(std::min(tiles(n), 4096)), dim3(PN_T), 0, st, ti.g, to.g, ti.g, n);
            hipLaunchKernelGGL(k_pn_add, dim3(std::min(tiles(n), 4096)), dim3(PN_T), 0, st, T[o.in2.t].g, to.g,
                               T[o.in2.t].g, n);
        } else if (o.kind == PO_BIAS) {
            const PLayer &l = layers[o.layer];
            const int ns = pn_nsplit(l.co, (size_t)B * no * no);
            hipLaunchKernelGGL(k_pn_bias_g, dim3(ns, l.co), dim3(PN_T), 0, st, to.g, B, l.co, no * no, ns, rpart);
            hipLaunchKernelGGL(k_pn_psum, dim3((l.co + 63) / 64), dim3(64), 0, st, rpart, ns, l.co, red);
            hipLaunchKernelGGL(k_pn_bias_fin, dim3((l.co + 63) / 64), dim3(64), 0, st, red, l.co, G + l.b_off);
        }
    }
}

void PaperNet::refold(hipStream_t st)
{
    for (const auto &l : layers)
        if (l.kind != PL_OUT)
            launch_fold_bn(P + l.g_off, P + l.b_off, BUF + l.rm_off, BUF + l.rv_off, l.co, 1e-5f, bnarr(l.bn, 5),
                           bnarr(l.bn, 6), st);
}

int PaperNet::input(const float2 *r, size_t rs, int nq, int n, const float *kap, const float *gam, size_t kstride,
                    const int *idx, const double *fscale, hipStream_t st)
{
    hipLaunchKernelGGL(k_pn_input, dim3(nq), dim3(PN_T), 0, st, r, rs, n, kap, gam, kstride, idx, fscale, sq,
                       T[x0t].v);
    return HELM_OK;
}

void PaperNet::output(int nb, int n, float2 *e, size_t es, int accumulate, const int *mask, const int *pos,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_pn_output, dim3(tiles((size_t)n * n), nb), dim3(PN_T), 0, st, T[outt].v, sq, n, e, es,
                       accumulate, mask, pos);
}

int PaperNet::loss_grad(const float2 *r, const float2 *e, const float *kap, const float *gam, size_t kstride, int B,
                        int n, double *loss, hipStream_t st)
{
    int rc = ensure_ws(B, n, true);
    if (rc) return rc;
    input(r, (size_t)n * n, B, n, kap, gam, kstride, nullptr, nullptr, st);
    forward(B, true, st);
    // d out into the gradient of the output tensor's spare: dlast
    if (!dlast_buf || dlast_n < (size_t)wsB * cout * n * n) {
        (void)dev_free(dlast_buf);
        dlast_n = (size_t)wsB * cout * n * n;
        if (dev_malloc(&dlast_buf, dlast_n * sizeof(float)) != hipSuccess) {
            dlast_buf = nullptr;
            set_error("unet (paper network): out of device memory");
            return HELM_E_NOMEM;
        }
    }
    dlast = dlast_buf;
    hipLaunchKernelGGL(k_pn_loss, dim3(B), dim3(PN_T), 0, st, T[outt].v, sq, n, B, e, dlast_buf, part);
    backward(B, st);
    std::vector<double> h(B);
    HELM_HIP_CHECK(hipMemcpyAsync(h.data(), part, B * sizeof(double), hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += h[b];
    *loss = s / ((double)B * n * n);
    return HELM_OK;
}

void PaperNet::update_running(int B, hipStream_t st)
{
    for (const auto &l : layers) {
        if (l.kind == PL_OUT) continue;
        // channels of the BN input: the layer's output grid
        int nl = wsN;
        const int li = (int)(&l - &layers[0]);
        for (const POp &o : ops)
            if (o.kind == PO_BN && o.layer == li) nl = T[o.in.t].n;
        launch_bn_running(BUF + l.rm_off, BUF + l.rv_off, bnarr(l.bn, 0), bnarr(l.bn, 1), l.co, 0.1f,
                          (double)B * nl * nl, st);
    }
}

}  // namespace helm
