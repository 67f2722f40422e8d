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
// A workgroup owns one (sample, output channel) pair, so its weight reads
// are uniform across the workgroup.  BN statistics and every reduction
// accumulate in FP64 in a fixed order.  These are plain VALU kernels: the
// network is small and runs on the 128^2 grid of the paper's experiments.
#include <cmath>
#include <string>
#include <vector>

#include "handle.h"
#include "paper_net.h"
#include "unet_internal.h"

namespace helm {

namespace {

constexpr int PN_T = 256;

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

// out (+)= gather to coarse; grid (tiles of Hc*Wc, B*Cc)
__global__ __launch_bounds__(PN_T) void k_pn_gc(const float *__restrict__ in, int inC, int inOff, int Cf, int Hf,
                                                int Wf, const float *__restrict__ W, float *__restrict__ out,
                                                int outC, int outOff, int Cc, int Hc, int Wc, int s, int K, int pad,
                                                int acc)
{
    const int b = blockIdx.y / Cc, oc = blockIdx.y - b * Cc;
    const int q = blockIdx.x * PN_T + threadIdx.x;
    if (q >= Hc * Wc) return;
    const int I = q / Wc, J = q - I * Wc;
    const float *w = W + (size_t)oc * Cf * K * K;
    const float *x = in + ((size_t)b * inC + inOff) * Hf * Wf;
    float sum = 0.f;
    for (int fc = 0; fc < Cf; ++fc) {
        const float *xf = x + (size_t)fc * Hf * Wf;
        const float *wf = w + (size_t)fc * K * K;
        for (int a = 0; a < K; ++a) {
            const int i = s * I + a - pad;
            if (i < 0 || i >= Hf) continue;
            for (int c = 0; c < K; ++c) {
                const int j = s * J + c - pad;
                if (j < 0 || j >= Wf) continue;
                sum = fmaf(wf[a * K + c], xf[(size_t)i * Wf + j], sum);
            }
        }
    }
    float *o = out + (((size_t)b * outC + outOff + oc) * Hc + I) * Wc + J;
    *o = acc ? *o + sum : sum;
}

// out (+)= gather to fine; grid (tiles of Hf*Wf, B*Cf)
__global__ __launch_bounds__(PN_T) void k_pn_gf(const float *__restrict__ in, int inC, int inOff, int Cc, int Hc,
                                                int Wc, const float *__restrict__ W, float *__restrict__ out,
                                                int outC, int outOff, int Cf, int Hf, int Wf, int s, int K, int pad,
                                                int acc)
{
    const int b = blockIdx.y / Cf, fc = blockIdx.y - b * Cf;
    const int q = blockIdx.x * PN_T + threadIdx.x;
    if (q >= Hf * Wf) return;
    const int i = q / Wf, j = q - i * Wf;
    const float *x = in + ((size_t)b * inC + inOff) * Hc * Wc;
    float sum = 0.f;
    for (int cc = 0; cc < Cc; ++cc) {
        const float *xc = x + (size_t)cc * Hc * Wc;
        const float *wc = W + ((size_t)cc * Cf + fc) * K * K;
        for (int a = 0; a < K; ++a) {
            const int ti = i + pad - a;
            if (ti < 0 || ti % s) continue;
            const int I = ti / s;
            if (I >= Hc) continue;
            for (int c = 0; c < K; ++c) {
                const int tj = j + pad - c;
                if (tj < 0 || tj % s) continue;
                const int J = tj / s;
                if (J >= Wc) continue;
                sum = fmaf(wc[a * K + c], xc[(size_t)I * Wc + J], sum);
            }
        }
    }
    float *o = out + (((size_t)b * outC + outOff + fc) * Hf + i) * Wf + j;
    *o = acc ? *o + sum : sum;
}

// dW[cc][fc][a][c] += sum over samples and coarse points of coarse * fine;
// one workgroup per (cc, fc), K*K FP64 accumulators per thread
template <int K>
__global__ __launch_bounds__(PN_T) void k_pn_wg(const float *__restrict__ co, int coC, int coOff, int Cc, int Hc,
                                                int Wc, const float *__restrict__ fi, int fiC, int fiOff, int Cf,
                                                int Hf, int Wf, int B, int s, int pad, float *__restrict__ dW)
{
    const int cc = blockIdx.x / Cf, fc = blockIdx.x - cc * Cf;
    double acc[K * K];
#pragma unroll
    for (int t = 0; t < K * K; ++t) acc[t] = 0.0;
    const size_t per = (size_t)Hc * Wc;
    for (size_t q = threadIdx.x; q < (size_t)B * per; q += PN_T) {
        const int b = (int)(q / per);
        const int r = (int)(q - (size_t)b * per), I = r / Wc, J = r - I * Wc;
        const float g = co[(((size_t)b * coC + coOff + cc) * Hc + I) * Wc + J];
        if (g == 0.f) continue;
        const float *xf = fi + ((size_t)b * fiC + fiOff + fc) * Hf * Wf;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int i = s * I + a - pad;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int j = s * J + c - pad;
                if (i >= 0 && i < Hf && j >= 0 && j < Wf) acc[a * K + c] += (double)g * xf[(size_t)i * Wf + j];
            }
        }
    }
    __shared__ double sh[4];
#pragma unroll
    for (int t = 0; t < K * K; ++t) {
        const double v = pn_bsum(acc[t], sh);
        if (threadIdx.x == 0) dW[((size_t)cc * Cf + fc) * K * K + t] += (float)v;
    }
}

// BN statistics of channel c (blockIdx.x) over B x HW: mean, var (biased),
// and the scale / shift of the batch normalisation with weight g, bias bb
__global__ __launch_bounds__(PN_T) void k_pn_bn_stats(const float *__restrict__ y, int yC, int yOff, int B, int HW,
                                                      const float *__restrict__ g, const float *__restrict__ bb,
                                                      float eps, float *__restrict__ mean, float *__restrict__ var,
                                                      float *__restrict__ rstd, float *__restrict__ sc,
                                                      float *__restrict__ sf)
{
    const int c = blockIdx.x;
    double s1 = 0.0, s2 = 0.0;
    for (size_t q = threadIdx.x; q < (size_t)B * HW; q += PN_T) {
        const size_t b = q / HW, p = q - b * HW;
        const double v = y[((b * yC) + yOff + c) * HW + p];
        s1 += v;
        s2 += v * v;
    }
    __shared__ double sh[4];
    s1 = pn_bsum(s1, sh);
    s2 = pn_bsum(s2, sh);
    if (threadIdx.x == 0) {
        const double N = (double)B * HW, m = s1 / N, vv = std::max(s2 / N - m * m, 0.0);
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
                                                     int act, double *__restrict__ red)
{
    const int c = blockIdx.x;
    double s1 = 0.0, s2 = 0.0;
    const float m = mean[c], r = rstd[c];
    for (size_t q = threadIdx.x; q < (size_t)B * HW; q += PN_T) {
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
    __shared__ double sh[4];
    s1 = pn_bsum(s1, sh);
    s2 = pn_bsum(s2, sh);
    if (threadIdx.x == 0) {
        red[2 * c] = s1;
        red[2 * c + 1] = s2;
    }
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

// dbias[c] += sum over samples and points of dout (one block per channel)
__global__ __launch_bounds__(PN_T) void k_pn_bias_g(const float *__restrict__ dout, int B, int C, int HW,
                                                    float *__restrict__ db)
{
    const int c = blockIdx.x;
    double s = 0.0;
    for (size_t q = threadIdx.x; q < (size_t)B * HW; q += PN_T) {
        const size_t b = q / HW, p = q - b * HW;
        s += dout[(b * C + c) * HW + p];
    }
    __shared__ double sh[4];
    s = pn_bsum(s, sh);
    if (threadIdx.x == 0) db[c] += (float)s;
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
    sq = nullptr;
    part = nullptr;
    red = nullptr;
    wsB = wsN = 0;
    wsTrain = false;
}

void PaperNet::free_all()
{
    free_ws();
    (void)dev_free(bnf);
    (void)dev_free(dlast_buf);
    bnf = dlast_buf = nullptr;
}

// the BN scratch arrays; the parameters, their gradient, the Adam moments
// and the buffers belong to the owning unet_net
int PaperNet::alloc_params()
{
    if (dev_malloc(&bnf, std::max<size_t>(7 * (nbuf / 2), 1) * 4) != hipSuccess) {
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
        dev_malloc(&red, 2 * 512 * sizeof(double)) != hipSuccess)
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
            if (o.kind == PO_CONV)
                hipLaunchKernelGGL(k_pn_gc, dim3(tiles((size_t)no * no), B * l.co), dim3(PN_T), 0, st, ti.v, ti.C,
                                   o.in.off, l.ci, ni, ni, Wt, to.v, to.C, o.out.off, l.co, no, no, o.s, l.K, o.pad, 0);
            else
                hipLaunchKernelGGL(k_pn_gf, dim3(tiles((size_t)no * no), B * l.co), dim3(PN_T), 0, st, ti.v, ti.C,
                                   o.in.off, l.ci, ni, ni, Wt, to.v, to.C, o.out.off, l.co, no, no, o.s, l.K, o.pad, 0);
        } else if (o.kind == PO_BN) {
            const PLayer &l = layers[o.layer];
            float *sc, *sf;
            if (training) {
                hipLaunchKernelGGL(k_pn_bn_stats, dim3(l.co), dim3(PN_T), 0, st, ti.v, ti.C, o.in.off, B, ni * ni,
                                   P + l.g_off, P + l.b_off, 1e-5f, bnarr(l.bn, 0), bnarr(l.bn, 1), bnarr(l.bn, 2),
                                   bnarr(l.bn, 3), bnarr(l.bn, 4));
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
                hipLaunchKernelGGL(k_pn_gf, dim3(tiles((size_t)ni * ni), B * l.ci), dim3(PN_T), 0, st, to.g, to.C,
                                   o.out.off, l.co, no, no, P + l.w_off, ti.g, ti.C, o.in.off, l.ci, ni, ni, o.s, l.K,
                                   o.pad, 1);
            if (l.K == 5)
                hipLaunchKernelGGL(k_pn_wg<5>, dim3(l.co * l.ci), dim3(PN_T), 0, st, to.g, to.C, o.out.off, l.co, no,
                                   no, ti.v, ti.C, o.in.off, l.ci, ni, ni, B, o.s, o.pad, G + l.w_off);
            else
                hipLaunchKernelGGL(k_pn_wg<3>, dim3(l.co * l.ci), dim3(PN_T), 0, st, to.g, to.C, o.out.off, l.co, no,
                                   no, ti.v, ti.C, o.in.off, l.ci, ni, ni, B, o.s, o.pad, G + l.w_off);
        } else if (o.kind == PO_CONVT) {
            // out = gather_fine(in): d in += gather_coarse(d out), dW += wg(coarse = in, fine = d out)
            const PLayer &l = layers[o.layer];
            hipLaunchKernelGGL(k_pn_gc, dim3(tiles((size_t)ni * ni), B * l.ci), dim3(PN_T), 0, st, to.g, to.C,
                               o.out.off, l.co, no, no, P + l.w_off, ti.g, ti.C, o.in.off, l.ci, ni, ni, o.s, l.K,
                               o.pad, 1);
            hipLaunchKernelGGL(k_pn_wg<5>, dim3(l.ci * l.co), dim3(PN_T), 0, st, ti.v, ti.C, o.in.off, l.ci, ni, ni,
                               to.g, to.C, o.out.off, l.co, no, no, B, o.s, o.pad, G + l.w_off);
        } else if (o.kind == PO_BN) {
            const PLayer &l = layers[o.layer];
            const int act = o.act ? 1 : 0;
            hipLaunchKernelGGL(k_pn_bn_bsum, dim3(l.co), dim3(PN_T), 0, st, to.g, to.C, o.out.off, to.v, to.C,
                               o.out.off, ti.v, ti.C, o.in.off, B, ni * ni, bnarr(l.bn, 0), bnarr(l.bn, 2), act, red);
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
            hipLaunchKernelGGL(k_pn_bias_g, dim3(l.co), dim3(PN_T), 0, st, to.g, B, l.co, no * no, G + l.b_off);
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
