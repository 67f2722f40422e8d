// Internal declarations of the U-Net part of libhelm (not the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "helm_internal.h"

namespace helm {

using bf16 = __bf16;

// One input source of a convolution: NHWC bf16 taking C channels (a
// multiple of 32) of the concatenated input; `shared` = 1 when every batch
// entry reads batch entry 0 (a context tensor computed once per medium).
// The tensor itself may hold fewer channels per pixel (`stride`, a multiple
// of 8; 0 means C): the channels from `stride` to C read as zero.
struct Src {
    const bf16 *p;
    int C;
    int shared;  // one tensor for the whole batch (read as sample 0)
    int stride = 0;
    // up = 1: the tensor is stored at half resolution (H/2 x W/2) and read
    // through the x2 bilinear upsampling (half-pixel centres, edges clamped),
    // each upsampled value rounded to bf16 as a stored upsampled tensor
    // would be.  Only the first source of an inference convolution with
    // H and W even, a second source and at most 32 output channels may set
    // it.
    int up = 0;
};
// Up to three sources concatenated along channels (by addressing only).
// The convolution weights of these Ctot channels start at channel woff of
// rows of wstride channels (0: Ctot, i.e. the weights cover exactly these
// sources); a subset of a layer's inputs is convolved with its weight slice.
struct Srcs {
    Src s[3];
    int n;
    int Ctot;
    int wstride = 0, woff = 0;
};

// ---------------------------------------------------------------- convolution
// 3x3 convolution, zero padding 1, implicit GEMM on bf16 MFMA with FP32
// accumulation.  Wt: bf16 [Cout][9][Ctot] (tap = ky*3 + kx).
//   mode 0: out32[p][co] = conv (raw, FP32)
//   mode 1: out16[p][co] = bf16(LeakyReLU(conv * scale[co] + shift[co]))
// Optional epilogue work of an inference (mode 1) convolution:
//   pool     : also write the 2x2 max-pooled activation [B][H/2][W/2][Cout]
//   head_out : apply the 1x1 head (head_w [2][Cout], head_b [2]) and write
//              [B][H][W][2] FP32 instead of the activation (needs Cout <= 64)
//   cmap     : FP16 [H][W][Cout] added to the raw convolution before the
//              folded BN, the same for every batch entry (the part of the
//              convolution over a context shared by the batch)
// and of a raw (mode 0) convolution:
//   raw16    : write the raw output as FP16 [B][H][W][Cout] here instead
//              of out32
//   nseg ... : route channel ranges of the FP32 raw output: range k is
//              [seg_hi[k-1], seg_hi[k]) (from 0; the last ends at Cout);
//              with seg_p[k] its channels are written to seg_p[k] (seg_C[k]
//              channels per pixel, at channel c - seg_hi[k-1]; stored, not
//              added), without it they go to out32 as usual.  Boundaries
//              are multiples of 16 (one range per 16-channel fragment),
//              seg_C a multiple of 4.
constexpr int CONV_MAX_SEG = 4;
struct ConvEpi {
    bf16 *pool = nullptr;
    const float *head_w = nullptr, *head_b = nullptr;
    float *head_out = nullptr;
    const _Float16 *cmap = nullptr;
    _Float16 *raw16 = nullptr;
    int nseg = 0;
    float *seg_p[CONV_MAX_SEG] = {};
    int seg_hi[CONV_MAX_SEG] = {};
    int seg_C[CONV_MAX_SEG] = {};
    // set by launch_conv3x3: the bf16 output exceeds the last-level cache,
    // so its stores stream past the caches (nontemporal)
    int nt = 0;
};
void launch_conv3x3(const Srcs &in, int B, int H, int W, const bf16 *Wt, int Cout, int mode,
                    float *out32, bf16 *out16, const float *scale, const float *shift,
                    float slope, hipStream_t s, const ConvEpi &epi = ConvEpi());
// Launch-shape autotuner of launch_conv3x3: enable = 1 tunes each new shape
// on first use, 0 uses the heuristic, -1 also forgets the table.  Returns
// the previous setting.
int conv_autotune(int enable);
int conv_autotune_entries();
// force one candidate launch shape on every convolution (kind < 0: off); -1 if invalid
int conv_force(int kind, int mf, int per_cu);
// Weight gradient: dW[co][tap][ci] = sum_p dy[p][co] * X[p + tap offset][ci],
// X the concatenated sources; written (not accumulated) as FP32 [Cout][9][Ctot].
// `part` is scratch of launch_wgrad_scratch(...) floats.
size_t wgrad_scratch(int B, int H, int W, int Cout, int Ctot);
void launch_wgrad(const Srcs &x, const bf16 *dy, int B, int H, int W, int Cout, float *dW,
                  float *part, hipStream_t s);

// ---------------------------------------------------------------- pointwise
// Per-channel mean and 1/sqrt(var + eps) (biased variance) of y [P][C] FP32.
void launch_bn_stats(const float *y, size_t P, int C, double *part, float *mean, float *rstd,
                     float *var_out, hipStream_t s);
// a = bf16(LeakyReLU(g (y - mean) rstd + b))
void launch_bn_act_fwd(const float *y, size_t P, int C, const float *mean, const float *rstd,
                       const float *g, const float *b, float slope, bf16 *a, hipStream_t s);
// Backward of bn_act: from da (FP32) computes dgamma, dbeta (FP32, added into
// dg, db) and dy (bf16) for the convolution backward.
void launch_bn_act_bwd(const float *da, const float *y, size_t P, int C, const float *mean,
                       const float *rstd, const float *g, const float *b, float slope,
                       double *part, float *dg, float *db, bf16 *dy, hipStream_t s);

void launch_maxpool_fwd(const bf16 *in, int B, int H, int W, int C, bf16 *out, uint8_t *arg,
                        hipStream_t s);
// din[argmax position] += dout (din FP32 [B][H][W][din_C], dout channels
// [coff_in, coff_in + C) of a [B][H/2][W/2][cstride_in] tensor)
void launch_maxpool_bwd(const float *dout, const uint8_t *arg, int B, int H, int W, int C,
                        int cstride_in, int coff_in, float *din, int din_C, hipStream_t s);
// bilinear x2 upsampling (half-pixel centres, edge clamped)
void launch_up2_fwd(const bf16 *in, int B, int h, int w, int C, bf16 *out, hipStream_t s);
// adjoint: din[B][h][w][C] (+)= up2^T (dout channels [coff, coff + C) of a
// tensor with cstride channels)
void launch_up2_bwd(const float *dout, int cstride, int coff, int B, int h, int w, int C,
                    float *din, int accumulate, hipStream_t s);
// dst[p][c] (+)= src[p][coff + c] for c < C
void launch_slice_add(const float *src, int cstride, int coff, size_t P, int C, float *dst,
                      int accumulate, hipStream_t s);
void launch_f32_to_bf16(const float *x, size_t n, bf16 *y, hipStream_t s);
// x [B][C][H][W] FP32 -> y [B][H][W][Cp] bf16 (channels >= C zero)
void launch_nchw_to_nhwc(const float *x, int B, int C, int H, int W, int Cp, bf16 *y, hipStream_t s);
// x [B][H][W][C] FP32 -> y [B][C][H][W] FP32
void launch_nhwc_to_nchw(const float *x, int B, int C, int H, int W, float *y, hipStream_t s);

// 1x1 head with bias: out[p][k] = sum_c Wh[k][c] a[p][c] + bh[k], k < 2
void launch_head_fwd(const bf16 *a, size_t P, int C, const float *Wh, const float *bh, float *out,
                     hipStream_t s);
// da = Wh^T dout; dWh, dbh summed over pixels (added into the FP32 grads)
void launch_head_bwd(const float *dout, const bf16 *a, size_t P, int C, const float *Wh,
                     float *da, double *part, float *dWh, float *dbh, hipStream_t s);

// ---------------------------------------------------------------- wrapper
// rc = R(h^2 r) per right-hand side (fine n -> coarse n/2), s_b = RMS |rc|,
// x0[b][I][J][0..7] = (Re rc / s, Im rc / s, kappa_c, 0, ...) (x0_stride
// channels per pixel, a multiple of 8; the others untouched), kappa_c either
// injected from the fine slowness (kappa_fine != null) or given on the coarse
// grid.  s[b] = 0 marks an all-zero residual.
// Sample b of the network batch reads right-hand side q = idx[b] (b if idx is
// null), multiplied by fscale[q] when fscale is given.
void launch_net_input(const float2 *r, size_t rstride, int nb, int n, const float *kappa_fine,
                      const float *kappa_c, float2 *rc, double *part, double *s, bf16 *x0,
                      int x0_stride, hipStream_t s_, const int *idx = nullptr,
                      const double *fscale = nullptr);
// e (+)= P (s_q (out0 + i out1)) on the fine grid for each of the nb
// right-hand sides, q = pos[b] its sample in the network batch (b if pos is
// null); q < 0 or mask[b] == 0: e_b = 0 (untouched when accumulating).
// out [batch][n/2][n/2][2] FP32.
void launch_net_output(const float *out, const double *s, int nb, int n, float2 *e,
                       size_t estride, int accumulate, hipStream_t st, const int *mask = nullptr,
                       const int *pos = nullptr);
// Loss of one batch: d = P out_b - e_b / s_b (fine), loss = mean_b |d|^2 / n^2,
// dout = (2 / (B n^2)) 4 R(d) split into (re, im).  loss_out: device double.
void launch_loss_grad(const float *out, const double *s, int nb, int n, const float2 *e,
                      float2 *dfine, double *part, float *dout, double *loss_out,
                      hipStream_t st);

// ---------------------------------------------------------------- parameters
// Packed bf16 convolution weights from the canonical FP32 master
// W[co][ci][3][3]: Wp[co][tap][cp] = W[co][map[cp]][tap] (0 where map < 0);
// transposed and flipped copy for the data gradient:
// Wd[cp][tap][co] = W[co][map[cp]][8 - tap].
void launch_pack_weights(const float *W, int Cout, int Cin, const int *map, int Cpad, bf16 *Wp,
                         bf16 *Wd, hipStream_t s);
// Canonical gradient from the packed one: gW[co][ci][tap] (+)= dW[co][tap][cp].
void launch_unpack_wgrad(const float *dW, int Cout, int Cin, const int *map, int Cpad,
                         float *gW, hipStream_t s);
// Adam with bias correction on FP32 masters.
void launch_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1,
                 float b2, float eps, int step, hipStream_t s);
void launch_bn_running(float *rm, float *rv, const float *mean, const float *var, int C,
                       float momentum, double count, hipStream_t s);
void launch_fold_bn(const float *g, const float *b, const float *rm, const float *rv, int C,
                    float eps, float *scale, float *shift, hipStream_t s);

}  // namespace helm
