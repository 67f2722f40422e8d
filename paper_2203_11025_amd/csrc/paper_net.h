// The paper's own network (section 3.1), internal to libhelm: see
// paper_net.hip.  Owned by a unet_net whose cfg.arch is 1.
#pragma once

#include <vector>

#include "helm_internal.h"

namespace helm {

enum { PL_DOWN, PL_RES1, PL_RES2, PL_UP, PL_OUT };
enum { PO_CONV, PO_CONVT, PO_BN, PO_ELU, PO_ADD, PO_BIAS };

// one convolution (and its BN, except the output layer) in the flat
// parameter order: weights [c_coarse][c_fine][K][K], then BN weight and bias
// (the output layer: its bias)
struct PLayer {
    int kind = 0, ci = 0, co = 0, K = 0, bn = -1;
    size_t w_off = 0, g_off = 0, b_off = 0, rm_off = 0, rv_off = 0;
};

// an activation tensor [B][C][n][n] of the workspace, with its gradient
struct PTensor {
    float *v = nullptr, *g = nullptr;
    int C = 0, n = 0;
};

// channels [off, off + C) of tensor t
struct PView {
    int t = -1, off = 0, C = 0;
};

// one step of the forward pass (the backward pass walks them in reverse)
struct POp {
    int kind = 0;
    PView in, in2, out;
    int layer = -1;  // parameter layer (convolutions, BN, bias)
    int s = 1, pad = 1;
    bool act = false;  // BN followed by ELU
};

struct PaperNet {
    int L = 0, cin = 4, cout = 2, cblocks = 3, nbn = 0;
    std::vector<int> w;
    std::vector<PLayer> layers;
    size_t nparams = 0, nbuf = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr, *BUF = nullptr;
    float *bnf = nullptr;  // per BN layer: mean, var, rstd, scale, shift (training), scale, shift (inference)
    int step = 0;
    // workspace
    int wsB = 0, wsN = 0;
    bool wsTrain = false;
    std::vector<PTensor> T;
    std::vector<POp> ops;
    int x0t = -1, outt = -1;
    double *sq = nullptr, *part = nullptr, *red = nullptr, *rpart = nullptr;
    float *dlast = nullptr, *dlast_buf = nullptr;
    size_t dlast_n = 0;
    float *wpk = nullptr;  // repacked weights of one gather
    float *wgp = nullptr;  // weight-gradient partials
    void wgrad(const float *co, int coC, int coOff, int Cc, int Hc, const float *fi, int fiC, int fiOff, int Cf, int Hf,
               int s, int K, int pad, int B, float *dW, hipStream_t st);
    void gather(int mode, const float *in, int inC, int inOff, int Cin, int Hin, const float *W, float *out,
                int outC, int outOff, int Cout, int Hout, int s, int K, int pad, int acc, int B, hipStream_t st);

    ~PaperNet();
    void build(const int *widths, int levels, int in_ch, int out_ch, int coarsest_blocks);
    int alloc_params();
    void free_ws();
    void free_all();
    float *bnarr(int bn, int which) const;
    int tensor(int C, int n, bool train);
    int ensure_ws(int B, int n, bool train);
    void forward(int B, bool training, hipStream_t st);
    void backward(int B, hipStream_t st);
    void refold(hipStream_t st);
    void update_running(int B, hipStream_t st);
    // x0 of nq samples (see k_pn_input); kappa / gamma fine [n][n], shared
    // (kstride 0) or per sample (kstride n^2)
    int input(const float2 *r, size_t rs, int nq, int n, const float *kap, const float *gam, size_t kstride,
              const int *idx, const double *fscale, hipStream_t st);
    void output(int nb, int n, float2 *e, size_t es, int accumulate, const int *mask, const int *pos,
                hipStream_t st);
    int loss_grad(const float2 *r, const float2 *e, const float *kap, const float *gam, size_t kstride, int B, int n,
                  double *loss, hipStream_t st);
};

}  // namespace helm
