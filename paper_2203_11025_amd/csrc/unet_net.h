// The U-Net object behind the unet_net handle of include/unet.h (internal).
#pragma once

#include <string>
#include <vector>

#include "../../include/unet.h"
#include "paper_net.h"
#include "unet_internal.h"

struct helm_handle;

struct unet_net {
    // one 3x3 convolution with its batch normalisation
    struct Layer {
        std::string name;
        int level = 0, cout = 0, nsrc = 0, cin_real = 0, cin_pad = 0;
        int src_real[3] = {0, 0, 0}, src_pad[3] = {0, 0, 0};
        size_t w_off = 0, g_off = 0, b_off = 0, rm_off = 0, rv_off = 0, sc_off = 0;
        helm::bf16 *Wp = nullptr, *Wd = nullptr;  // packed forward / data-gradient weights
        int *map = nullptr;                        // padded -> canonical input channel
        float *mean = nullptr, *rstd = nullptr, *var = nullptr;  // batch statistics
    };
    // per-layer activations of the current workspace
    struct Act {
        float *y32 = nullptr;   // raw convolution output (training)
        helm::bf16 *a = nullptr;  // activation
        float *g = nullptr;     // gradient w.r.t. the activation (training)
    };

    unet_cfg cfg{};
    std::vector<Layer> L;
    size_t nparams = 0, nbuf = 0, head_w = 0, head_b = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr, *BUF = nullptr;
    float *scale = nullptr, *shift = nullptr;  // folded inference BN
    int step = 0;
    // arch 1: the paper's network (owns its workspace; P, G, M, V and BUF
    // above are shared with it) and the loss of its last batch
    helm::PaperNet *pn = nullptr;
    double pn_loss = 0.0;
    int init_paper(const unet_cfg &c);
    // training-data cursor saved with the state: the seed of the sample
    // generator and the index of the next sample to draw
    uint64_t data_seed = 0, data_next = 0;

    int wsB = 0, wsH = 0, wsW = 0;
    bool wsTrain = false;
    std::vector<Act> act;
    std::vector<helm::bf16 *> pooled, up;
    std::vector<uint8_t *> arg;
    helm::bf16 *x0 = nullptr, *dy = nullptr;
    // channels per pixel of the network input x0: in_ch rounded up to 8
    int x0_stride() const { return (cfg.in_ch + 7) / 8 * 8; }
    float *out = nullptr, *gout = nullptr, *dX = nullptr, *dW = nullptr, *wpart = nullptr;
    float *xin = nullptr;
    double *red = nullptr, *s = nullptr, *dloss = nullptr;
    float2 *rcoarse = nullptr, *dfine = nullptr;
    // encoder-solver: context tensors per level (solver), their gradients
    // (solver-owned copies of the encoder outputs), their gradients
    std::vector<const helm::bf16 *> ctxp;
    std::vector<helm::bf16 *> ctxbuf;
    int ctx_shared = 0, ctx_B = 0, ctx_H = 0, ctx_valid = 0;
    // With a context shared by the batch, the part of each context-taking
    // convolution over the context is the same for every sample: cmap[i]
    // (FP16 [H_l][W_l][cout], layer i) holds it, computed when the context is
    // attached; inference adds it in the epilogue instead of convolving the
    // context again.  Invalid once the weights change.
    std::vector<_Float16 *> cmap;
    int cmap_valid = 0;
    bool use_cmap(bool training, int H) const
    {
        return !training && cfg.context && ctx_valid && ctx_shared && cmap_valid && H == ctx_H;
    }
    void compute_cmaps(hipStream_t st);
    int gen = 0;  // bumped when workspace or context storage moves (captured graphs hold pointers)
    std::vector<float *> gctx;
    int attach_context(const unet_net &enc, int nb, int H, int W, hipStream_t st);
    void clear_context();
    void adam_update(const unet_train_opts &o, double count, hipStream_t st);

    ~unet_net();
    int init(const unet_cfg &c);
    int ensure_ws(int B, int H, int W, bool training);
    void free_ws();
    int enc_index(int level, char ab) const;
    int dec_index(int level, char ab) const;
    // sources of layer i; without_ctx drops the context (weights sliced)
    helm::Srcs layer_srcs(int i, bool without_ctx = false) const;
    void run_layer(int i, const helm::Srcs &src, int B, int H, int W, bool training, hipStream_t st,
                   const helm::ConvEpi &epi = helm::ConvEpi());
    void forward_from_x0(int B, int H, int W, bool training, hipStream_t st);
    void backward(int B, int H, int W, hipStream_t st);  // zero, head, layers
    void layers_backward(int B, int H, int W, hipStream_t st, bool seeded);
    int output_layer(int level) const;  // layer whose activation is level's output
    void repack(hipStream_t st);
    void refold(hipStream_t st);
    int pack_nchw_input(const float *x, int B, int H, int W, hipStream_t st);
    int unpack_nchw_output(float *o, int B, int H, int W, hipStream_t st);
    // e (+)= P s Net(R(h^2 r)/s, kappa_c) for nb fields of medium h (mask,
    // may be null: entries b with mask[b] == 0 are left unchanged, or set to
    // zero when not accumulating).  With idx/pos the network runs on the nnet
    // right-hand sides idx[0..nnet) only (pos: the inverse map, -1 for the
    // others, which are treated as masked).  fscale (may be null): field b
    // is read as fscale[b] r_b.
    int wrap_apply(helm_handle *h, const float2 *r, size_t rs, float2 *e, size_t es, int nb,
                   int accumulate, hipStream_t st, const int *mask = nullptr, int nnet = -1,
                   const int *idx = nullptr, const int *pos = nullptr, const double *fscale = nullptr);
    int loss_grad(const unet_batch &bt, hipStream_t st);
};
