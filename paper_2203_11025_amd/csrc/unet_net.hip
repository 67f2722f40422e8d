// Host orchestration of the U-Net: parameters, forward (training and
// inference batch normalisation), backward, loss, Adam, and the residual ->
// error wrapper used by the preconditioners.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/unet.h"
#include "handle.h"
#include "unet_internal.h"
#include "unet_net.h"

namespace helm {

namespace {

constexpr float SLOPE = 0.2f;
constexpr float BN_EPS = 1e-5f;
constexpr float BN_MOM = 0.1f;

template <typename T>
int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    if (dev_malloc((void **)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        set_error("unet: device allocation failed");
        return HELM_E_NOMEM;
    }
    return HELM_OK;
}

int pad32(int c) { return (c + 31) / 32 * 32; }

}  // namespace
}  // namespace helm

using namespace helm;

void unet_net::free_ws()
{
    for (auto &a : act) {
        dev_free(a.y32);
        dev_free(a.a);
        dev_free(a.g);
    }
    act.clear();
    for (auto p : pooled) dev_free(p);
    for (auto p : arg) dev_free(p);
    for (auto p : up) dev_free(p);
    for (auto p : gctx) dev_free(p);
    gctx.clear();
    pooled.clear();
    arg.clear();
    up.clear();
    dev_free(x0);
    dev_free(out);
    dev_free(gout);
    dev_free(dX);
    dev_free(dy);
    dev_free(dW);
    dev_free(wpart);
    dev_free(red);
    dev_free(rcoarse);
    dev_free(s);
    dev_free(dfine);
    dev_free(dloss);
    dev_free(xin);
    x0 = nullptr;
    out = gout = dX = dW = wpart = nullptr;
    dy = nullptr;
    red = nullptr;
    rcoarse = dfine = nullptr;
    s = dloss = nullptr;
    xin = nullptr;
    wsB = wsH = wsW = 0;
    wsTrain = false;
}

unet_net::~unet_net()
{
    delete pn;
    free_ws();
    for (auto p : ctxbuf) dev_free(p);
    for (auto p : cmap) dev_free(p);
    for (auto &l : L) {
        dev_free(l.Wp);
        dev_free(l.Wd);
        dev_free(l.map);
        dev_free(l.mean);
        dev_free(l.rstd);
        dev_free(l.var);
    }
    dev_free(P);
    dev_free(G);
    dev_free(M);
    dev_free(V);
    dev_free(BUF);
    dev_free(scale);
    dev_free(shift);
}

int unet_net::init_paper(const unet_cfg &c)
{
    cfg = c;
    pn = new PaperNet();
    pn->build(c.widths, c.levels, c.in_ch, c.out_ch, 3);
    nparams = pn->nparams;
    nbuf = pn->nbuf;
    int rc;
    if ((rc = dalloc(&P, nparams)) || (rc = dalloc(&G, nparams)) || (rc = dalloc(&M, nparams)) ||
        (rc = dalloc(&V, nparams)) || (rc = dalloc(&BUF, nbuf)))
        return rc;
    pn->P = P;
    pn->G = G;
    pn->M = M;
    pn->V = V;
    pn->BUF = BUF;
    return pn->alloc_params();
}

int unet_net::init(const unet_cfg &c)
{
    cfg = c;
    const int Lv = cfg.levels;
    auto add = [&](const std::string &name, int level, std::vector<int> real, std::vector<int> padc,
                   int cout) {
        Layer l;
        l.name = name;
        l.level = level;
        l.cout = cout;
        l.nsrc = (int)real.size();
        l.cin_real = l.cin_pad = 0;
        for (int k = 0; k < l.nsrc; ++k) {
            l.src_real[k] = real[k];
            l.src_pad[k] = padc[k];
            l.cin_real += real[k];
            l.cin_pad += padc[k];
        }
        L.push_back(l);
    };
    const int *w = cfg.widths;
    // with an encoder context, level l's context (w_l channels) is the last
    // source of enc{l}a and dec{l}a (eq. 3.5)
    auto cx = [&](std::vector<int> v, int l) {
        if (cfg.context) v.push_back(w[l]);
        return v;
    };
    for (int l = 0; l < Lv; ++l) {
        if (l == 0)
            add("enc0a", 0, cx({cfg.in_ch}, 0), cx({pad32(cfg.in_ch)}, 0), w[0]);
        else
            add("enc" + std::to_string(l) + "a", l, cx({w[l - 1]}, l), cx({w[l - 1]}, l), w[l]);
        add("enc" + std::to_string(l) + "b", l, {w[l]}, {w[l]}, w[l]);
    }
    for (int l = Lv - 2; l >= 0; --l) {
        add("dec" + std::to_string(l) + "a", l, cx({w[l + 1], w[l]}, l), cx({w[l + 1], w[l]}, l), w[l]);
        add("dec" + std::to_string(l) + "b", l, {w[l]}, {w[l]}, w[l]);
    }
    ctxp.assign(Lv, nullptr);
    // flat offsets
    size_t off = 0, boff = 0;
    int rc;
    for (auto &l : L) {
        l.w_off = off;
        off += (size_t)l.cout * l.cin_real * 9;
        l.g_off = off;
        off += l.cout;
        l.b_off = off;
        off += l.cout;
        l.rm_off = boff;
        boff += l.cout;
        l.rv_off = boff;
        boff += l.cout;
        // padded channel -> canonical channel map
        std::vector<int> map(l.cin_pad, -1);
        int cr = 0, cp = 0;
        for (int k = 0; k < l.nsrc; ++k) {
            for (int q = 0; q < l.src_real[k]; ++q) map[cp + q] = cr + q;
            cr += l.src_real[k];
            cp += l.src_pad[k];
        }
        if ((rc = dalloc(&l.map, map.size())) || (rc = dalloc(&l.Wp, (size_t)l.cout * 9 * l.cin_pad)) ||
            (rc = dalloc(&l.Wd, (size_t)l.cout * 9 * l.cin_pad)) || (rc = dalloc(&l.mean, l.cout)) ||
            (rc = dalloc(&l.rstd, l.cout)) || (rc = dalloc(&l.var, l.cout)))
            return rc;
        if (hipMemcpy(l.map, map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
            set_error("unet_create: upload failed");
            return HELM_E_HIP;
        }
    }
    head_w = off;
    if (cfg.head) off += (size_t)cfg.out_ch * w[0];
    head_b = off;
    if (cfg.head) off += cfg.out_ch;
    nparams = off;
    nbuf = boff;
    size_t nsc = 0;
    for (auto &l : L) {
        l.sc_off = nsc;
        nsc += l.cout;
    }
    if ((rc = dalloc(&P, nparams)) || (rc = dalloc(&G, nparams)) || (rc = dalloc(&M, nparams)) ||
        (rc = dalloc(&V, nparams)) || (rc = dalloc(&BUF, nbuf)) || (rc = dalloc(&scale, nsc)) ||
        (rc = dalloc(&shift, nsc)))
        return rc;
    if (hipMemset(P, 0, nparams * 4) || hipMemset(M, 0, nparams * 4) || hipMemset(V, 0, nparams * 4)) {
        set_error("unet_create: clearing parameters failed");
        return HELM_E_HIP;
    }
    return HELM_OK;
}

int unet_net::ensure_ws(int B, int H, int W, bool training)
{
    if (B <= wsB && H == wsH && W == wsW && (!training || wsTrain)) return HELM_OK;
    int nB = std::max(B, wsB);
    bool tr = training || wsTrain;
    free_ws();
    ++gen;
    const int Lv = cfg.levels;
    int rc;
    act.resize(L.size());
    size_t maxdx = 0, maxdy = 0, maxdw = 0, maxpart = 0;
    for (size_t i = 0; i < L.size(); ++i) {
        const Layer &l = L[i];
        size_t Pl = (size_t)nB * (H >> l.level) * (W >> l.level);
        if ((rc = dalloc(&act[i].a, Pl * l.cout))) return rc;
        if (tr) {
            if ((rc = dalloc(&act[i].y32, Pl * l.cout)) || (rc = dalloc(&act[i].g, Pl * l.cout))) return rc;
        }
        maxdx = std::max(maxdx, Pl * l.cin_pad);
        maxdy = std::max(maxdy, Pl * l.cout);
        maxdw = std::max(maxdw, (size_t)l.cout * 9 * l.cin_pad);
        maxpart = std::max(maxpart, wgrad_scratch(nB, H >> l.level, W >> l.level, l.cout, l.cin_pad));
    }
    pooled.assign(Lv, nullptr);
    arg.assign(Lv, nullptr);
    up.assign(Lv, nullptr);
    for (int l = 1; l < Lv; ++l) {
        size_t Pl = (size_t)nB * (H >> l) * (W >> l);
        if ((rc = dalloc(&pooled[l], Pl * cfg.widths[l - 1])) || (rc = dalloc(&arg[l], Pl * cfg.widths[l - 1])))
            return rc;
    }
    for (int l = 0; l < Lv - 1; ++l) {
        size_t Pl = (size_t)nB * (H >> l) * (W >> l);
        if ((rc = dalloc(&up[l], Pl * cfg.widths[l + 1]))) return rc;
    }
    if (cfg.context && tr) {
        gctx.assign(Lv, nullptr);
        for (int l = 0; l < Lv; ++l)
            if ((rc = dalloc(&gctx[l], (size_t)nB * (H >> l) * (W >> l) * cfg.widths[l]))) return rc;
    }
    size_t P0 = (size_t)nB * H * W;
    if ((rc = dalloc(&x0, P0 * x0_stride())) || (rc = dalloc(&out, P0 * cfg.out_ch)) ||
        (rc = dalloc(&xin, P0 * cfg.out_ch)))
        return rc;
    if (hipMemset(x0, 0, P0 * x0_stride() * sizeof(bf16)) != hipSuccess) {
        set_error("unet: clearing the input workspace failed");
        return HELM_E_HIP;
    }
    if ((rc = dalloc(&red, 1 << 20))) return rc;  // reduction scratch (8 MB)
    if (tr) {
        if ((rc = dalloc(&gout, P0 * cfg.out_ch)) || (rc = dalloc(&dX, maxdx)) || (rc = dalloc(&dy, maxdy)) ||
            (rc = dalloc(&dW, maxdw)) || (rc = dalloc(&wpart, maxpart)))
            return rc;
    }
    // wrapper scratch: coarse residual, scales, fine residual of the loss
    if ((rc = dalloc(&rcoarse, P0)) || (rc = dalloc(&s, nB)) || (rc = dalloc(&dloss, 1)))
        return rc;
    if (tr && (rc = dalloc(&dfine, (size_t)nB * 4 * H * W))) return rc;
    wsB = nB;
    wsH = H;
    wsW = W;
    wsTrain = tr;
    return HELM_OK;
}

// One 3x3 convolution layer with BN and LeakyReLU.
void unet_net::run_layer(int i, const Srcs &src, int B, int H, int W, bool training, hipStream_t st,
                         const ConvEpi &epi)
{
    Layer &l = L[i];
    Act &a = act[i];
    const size_t Pl = (size_t)B * H * W;
    // 2 FLOPs per multiply-add over the real input channels (without the
    // context when its part comes from the context map)
    const int cin = epi.cmap ? l.cin_real - l.src_real[l.nsrc - 1] : l.cin_real;
    const double flops = 18.0 * cin * l.cout * (double)Pl;
    prof_mark(HELM_PROF_CONV, st, true);
    if (training) {
        launch_conv3x3(src, B, H, W, l.Wp, l.cout, 0, a.y32, nullptr, nullptr, nullptr, SLOPE, st);
        prof_mark(HELM_PROF_CONV, st, false, flops);
        launch_bn_stats(a.y32, Pl, l.cout, red, l.mean, l.rstd, l.var, st);
        launch_bn_act_fwd(a.y32, Pl, l.cout, l.mean, l.rstd, P + l.g_off, P + l.b_off, SLOPE, a.a, st);
    } else {
        launch_conv3x3(src, B, H, W, l.Wp, l.cout, 1, nullptr, a.a, scale + l.sc_off, shift + l.sc_off,
                       SLOPE, st, epi);
        prof_mark(HELM_PROF_CONV, st, false, flops);
    }
}

Srcs unet_net::layer_srcs(int i, bool without_ctx) const
{
    const Layer &l = L[i];
    Srcs s{};
    s.n = l.nsrc;
    s.Ctot = l.cin_pad;
    s.wstride = l.cin_pad;
    const std::string &nm = l.name;
    int lev = l.level;
    if (nm == "enc0a") {
        s.s[0] = {x0, l.src_pad[0], 0, x0_stride()};
    } else if (nm[0] == 'e' && nm.back() == 'a') {
        s.s[0] = {pooled[lev], l.src_pad[0], 0};
    } else if (nm.back() == 'b') {
        s.s[0] = {act[i - 1].a, l.src_pad[0], 0};
    } else {  // decoder 'a': [upsampled, skip]
        s.s[0] = {up[lev], l.src_pad[0], 0};
        s.s[1] = {act[enc_index(lev, 'b')].a, l.src_pad[1], 0};
    }
    if (cfg.context && nm.back() == 'a') {
        if (without_ctx) {  // the context is the last source and the last weight columns
            s.n = l.nsrc - 1;
            s.Ctot = l.cin_pad - l.src_pad[l.nsrc - 1];
        } else {
            s.s[l.nsrc - 1] = {ctxp[lev], l.src_pad[l.nsrc - 1], ctx_shared};
        }
    }
    return s;
}

// cmap[i] = the convolution of layer i over the context alone (raw, rounded
// to FP16, one sample): the context columns of the packed weights applied
// to it.
void unet_net::compute_cmaps(hipStream_t st)
{
    for (size_t i = 0; i < L.size(); ++i) {
        const Layer &l = L[i];
        if (!cmap[i]) continue;
        const int lev = l.level, cc = l.src_pad[l.nsrc - 1];
        Srcs s{};
        s.n = 1;
        s.Ctot = cc;
        s.wstride = l.cin_pad;
        s.woff = l.cin_pad - cc;
        s.s[0] = {ctxp[lev], cc, 1};
        ConvEpi e;
        e.raw16 = cmap[i];
        launch_conv3x3(s, 1, ctx_H >> lev, ctx_H >> lev, l.Wp, l.cout, 0, nullptr, nullptr, nullptr, nullptr,
                       SLOPE, st, e);
    }
    if (!cmap_valid) ++gen;  // captured graphs that convolve the context are stale
    cmap_valid = 1;
}

int unet_net::enc_index(int level, char ab) const { return 2 * level + (ab == 'b' ? 1 : 0); }

int unet_net::output_layer(int level) const
{
    return level == cfg.levels - 1 ? enc_index(level, 'b') : dec_index(level, 'b');
}

int unet_net::dec_index(int level, char ab) const
{
    // decoders follow the 2L encoder layers, level L-2 first
    return 2 * cfg.levels + 2 * (cfg.levels - 2 - level) + (ab == 'b' ? 1 : 0);
}

// Training keeps every intermediate tensor the backward pass reads (pooling
// arguments, the last activation) and runs pooling and the head on their own.
// In inference the second convolution of a 32-channel encoder level also
// writes the pooled tensor, and a 32-channel last convolution applies the head.
void unet_net::forward_from_x0(int B, int H, int W, bool training, hipStream_t st)
{
    const int Lv = cfg.levels;
    const int last = Lv >= 2 ? dec_index(0, 'b') : enc_index(0, 'b');
    const bool fuse_head = !training && cfg.head && cfg.widths[0] == 32;
    const bool maps = use_cmap(training, H);
    // a context-taking layer: its sources, and the context map when used;
    // up (inference decoders): the first source is the coarse activation,
    // upsampled inside the convolution
    auto run_a = [&](int i, int Hl, int Wl, const bf16 *up = nullptr) {
        ConvEpi e;
        if (maps) e.cmap = cmap[i];
        Srcs src = layer_srcs(i, maps);
        if (up) {
            src.s[0].p = up;
            src.s[0].up = 1;
        }
        run_layer(i, src, B, Hl, Wl, training, st, e);
    };
    for (int l = 0; l < Lv; ++l) {
        int Hl = H >> l, Wl = W >> l;
        if (l > 0 && (training || cfg.widths[l - 1] != 32))
            launch_maxpool_fwd(act[enc_index(l - 1, 'b')].a, B, H >> (l - 1), W >> (l - 1),
                               cfg.widths[l - 1], pooled[l], training ? arg[l] : nullptr, st);
        run_a(enc_index(l, 'a'), Hl, Wl);
        ConvEpi epi;
        // pooling in the epilogue pays for 32-channel layers only (wider
        // channel blocks run out of registers)
        if (!training && l < Lv - 1 && cfg.widths[l] == 32) epi.pool = pooled[l + 1];
        if (fuse_head && enc_index(l, 'b') == last) {
            epi.head_w = P + head_w;
            epi.head_b = P + head_b;
            epi.head_out = out;
        }
        run_layer(enc_index(l, 'b'), layer_srcs(enc_index(l, 'b')), B, Hl, Wl, training, st, epi);
    }
    for (int l = Lv - 2; l >= 0; --l) {
        int Hl = H >> l, Wl = W >> l;
        const bf16 *prev = (l == Lv - 2) ? act[enc_index(Lv - 1, 'b')].a : act[dec_index(l + 1, 'b')].a;
        // Upsampling inside the convolution saves writing and re-reading
        // the upsampled tensor, but its in-LDS expansion is VALU work that
        // the workgroup's barriers serialise with the MFMAs: it pays for
        // 32-channel outputs only (on MI355X: 0.86 ms against 0.99 ms for
        // upsampling plus convolution at 512^2 x 32 samples, while 64- and
        // 128-channel outputs lose 12-25%).  Training keeps the upsampled
        // tensor for the backward pass.
        if (!training && cfg.widths[l] == 32) {
            run_a(dec_index(l, 'a'), Hl, Wl, prev);
        } else {
            launch_up2_fwd(prev, B, Hl / 2, Wl / 2, cfg.widths[l + 1], up[l], st);
            run_a(dec_index(l, 'a'), Hl, Wl);
        }
        ConvEpi epi;
        if (fuse_head && dec_index(l, 'b') == last) {
            epi.head_w = P + head_w;
            epi.head_b = P + head_b;
            epi.head_out = out;
        }
        run_layer(dec_index(l, 'b'), layer_srcs(dec_index(l, 'b')), B, Hl, Wl, training, st, epi);
    }
    if (!cfg.head || fuse_head) return;
    launch_head_fwd(act[last].a, (size_t)B * H * W, cfg.widths[0], P + head_w, P + head_b, out, st);
}

// Every activation gradient and context gradient is first stored, then
// added to, so none is cleared: the head stores the last layer's; a 'b'
// layer's data gradient stores its 'a' layer's; a decoder 'a' layer's stores
// its skip input's and its level's context gradient (the encoder layer below
// adds the pooling share, the encoder 'a' layer of the level adds its context
// share); the bottom encoder 'a' layer stores its context gradient; the
// upsampling adjoint stores the gradient of the tensor it reads (its only
// consumer), or adds to it when the caller seeded that gradient (`seeded`:
// an encoder whose outputs carry the solver's context gradients).
void unet_net::backward(int B, int H, int W, hipStream_t st)
{
    const int Lv = cfg.levels;
    int last = Lv >= 2 ? dec_index(0, 'b') : enc_index(0, 'b');
    launch_head_bwd(gout, act[last].a, (size_t)B * H * W, cfg.widths[0], P + head_w, act[last].g, red,
                    G + head_w, G + head_b, st);
    layers_backward(B, H, W, st, false);
}

void unet_net::layers_backward(int B, int H, int W, hipStream_t st, bool seeded)
{
    const int Lv = cfg.levels;
    for (int i = (int)L.size() - 1; i >= 0; --i) {
        Layer &l = L[i];
        Act &a = act[i];
        const int Hl = H >> l.level, Wl = W >> l.level;
        const size_t Pl = (size_t)B * Hl * Wl;
        launch_bn_act_bwd(a.g, a.y32, Pl, l.cout, l.mean, l.rstd, P + l.g_off, P + l.b_off, SLOPE, red,
                          G + l.g_off, G + l.b_off, dy, st);
        Srcs src = layer_srcs(i);
        const double flops = 18.0 * l.cin_real * l.cout * (double)Pl;
        prof_mark(HELM_PROF_WGRAD, st, true);
        launch_wgrad(src, dy, B, Hl, Wl, l.cout, dW, wpart, st);
        prof_mark(HELM_PROF_WGRAD, st, false, flops);
        launch_unpack_wgrad(dW, l.cout, l.cin_real, l.map, l.cin_pad, G + l.w_off, st);
        const bool has_ctx = cfg.context && l.name.back() == 'a';
        if (i == 0 && !has_ctx) continue;  // no gradient w.r.t. the network input
        // data gradient: a 3x3 convolution of dy with the flipped, transposed
        // weights.  Its channel ranges that are the first contribution to
        // another tensor's gradient are stored straight into it by the
        // convolution's epilogue: the previous activation of a 'b' layer
        // (its only consumer), the skip input of a decoder 'a' layer (the
        // pooling's share comes later, from the encoder layer below), and the
        // context of a decoder 'a' layer or of the bottom encoder layer (the
        // encoder 'a' layer of the same level adds its share later).  The
        // ranges read through the pooling or the upsampling adjoint stay in
        // dX, and so does the context share that is added second.
        const std::string &nm = l.name;
        const int lev = l.level;
        ConvEpi de;
        int hi = 0;
        // at most a gap, the skip input, a gap and the context: 4 ranges
        auto route = [&](int lo, int C, float *p) {
            if (lo > hi) {  // a gap stays in dX
                de.seg_p[de.nseg] = nullptr;
                de.seg_hi[de.nseg] = lo;
                de.seg_C[de.nseg++] = 0;
            }
            de.seg_p[de.nseg] = p;
            de.seg_hi[de.nseg] = lo + C;
            de.seg_C[de.nseg++] = C;
            hi = lo + C;
        };
        if (i > 0 && nm.back() == 'b') {
            route(0, l.cout, act[i - 1].g);
        } else if (i > 0 && nm[0] == 'd') {
            // dec{lev}a: [upsampled, skip (, context)]
            route(cfg.widths[lev + 1], cfg.widths[lev], act[enc_index(lev, 'b')].g);
        }
        // the context is the last source; a decoder layer of its level (dec
        // layers run first here) has written gctx[lev] already unless this
        // is the bottom level
        const bool ctx_first = has_ctx && (nm[0] == 'd' || lev == Lv - 1);
        if (ctx_first) route(l.cin_pad - cfg.widths[lev], cfg.widths[lev], gctx[lev]);
        if (de.nseg == 0) {
            // nothing routed: the plain epilogue
        } else if (hi < l.cin_pad) {
            de.seg_p[de.nseg] = nullptr;
            de.seg_hi[de.nseg] = l.cin_pad;
            de.seg_C[de.nseg++] = 0;
        }
        // one range covering every channel: the plain epilogue into it
        float *out = dX;
        if (de.nseg == 1 && de.seg_p[0] && de.seg_C[0] == l.cin_pad) {
            out = de.seg_p[0];
            de.nseg = 0;
        }
        Srcs ds{};
        ds.n = 1;
        ds.Ctot = l.cout;
        ds.s[0] = {dy, l.cout, 0};
        prof_mark(HELM_PROF_CONV, st, true);
        launch_conv3x3(ds, B, Hl, Wl, l.Wd, l.cin_pad, 0, out, nullptr, nullptr, nullptr, SLOPE, st, de);
        prof_mark(HELM_PROF_CONV, st, false, flops);
        if (has_ctx && !ctx_first)
            launch_slice_add(dX, l.cin_pad, l.cin_pad - cfg.widths[lev], Pl, cfg.widths[lev], gctx[lev], 1, st);
        if (i == 0) continue;
        if (nm.back() == 'b') {
            // routed above
        } else if (nm[0] == 'e') {
            // enc{lev}a, lev >= 1: through the max pooling into enc{lev-1}b
            int src_layer = enc_index(lev - 1, 'b');
            launch_maxpool_bwd(dX, arg[lev], B, Hl * 2, Wl * 2, cfg.widths[lev - 1], l.cin_pad, 0,
                               act[src_layer].g, cfg.widths[lev - 1], st);
        } else {
            // dec{lev}a: [upsampled, skip (, context)]
            int prev = (lev == Lv - 2) ? enc_index(Lv - 1, 'b') : dec_index(lev + 1, 'b');
            launch_up2_bwd(dX, l.cin_pad, 0, B, Hl / 2, Wl / 2, cfg.widths[lev + 1], act[prev].g, seeded ? 1 : 0,
                           st);
        }
    }
}

// Copies the encoder's per-level outputs f^(l) (eq. 3.5) into storage the
// solver owns, so the encoder may be run again or destroyed afterwards.
int unet_net::attach_context(const unet_net &enc, int nb, int H, int W, hipStream_t st)
{
    const int Lv = cfg.levels;
    if (ctxbuf.empty() || ctx_B != nb || ctx_H != H) {
        ++gen;
        cmap_valid = 0;
        for (auto p : ctxbuf) dev_free(p);
        for (auto p : cmap) dev_free(p);
        ctxbuf.assign(Lv, nullptr);
        cmap.assign(L.size(), nullptr);
        ctx_valid = 0;
        for (size_t i = 0; i < L.size() && nb == 1 && H == W; ++i)
            if (L[i].name.back() == 'a' &&
                dev_malloc(&cmap[i], (size_t)(H >> L[i].level) * (W >> L[i].level) * L[i].cout * sizeof(_Float16)) !=
                    hipSuccess) {
                set_error("unet_pair_encode: out of device memory for the context maps");
                return HELM_E_NOMEM;
            }
        for (int l = 0; l < Lv; ++l)
            if (dev_malloc(&ctxbuf[l], (size_t)nb * (H >> l) * (W >> l) * cfg.widths[l] * sizeof(bf16)) !=
                hipSuccess) {
                set_error("unet_pair_encode: out of device memory for the context");
                return HELM_E_NOMEM;
            }
    }
    for (int l = 0; l < Lv; ++l) {
        size_t bytes = (size_t)nb * (H >> l) * (W >> l) * cfg.widths[l] * sizeof(bf16);
        if (hipMemcpyAsync(ctxbuf[l], enc.act[enc.output_layer(l)].a, bytes, hipMemcpyDeviceToDevice, st) !=
            hipSuccess) {
            set_error("unet_pair_encode: context copy failed");
            return HELM_E_HIP;
        }
        ctxp[l] = ctxbuf[l];
    }
    ctx_B = nb;
    ctx_H = H;
    ctx_shared = nb == 1;
    ctx_valid = 1;
    if (ctx_shared && H == W) {
        compute_cmaps(st);
    } else if (cmap_valid) {
        cmap_valid = 0;
        ++gen;
    }
    return HELM_OK;
}

void unet_net::clear_context()
{
    ctx_valid = 0;
    if (cmap_valid) ++gen;
    cmap_valid = 0;
    for (auto &p : ctxp) p = nullptr;
}

// Adam on the FP32 masters, BN running statistics, bf16 repack; count is the
// number of level-0 pixels in the batch.
void unet_net::adam_update(const unet_train_opts &o, double count, hipStream_t st)
{
    step += 1;
    launch_adam(P, G, M, V, nparams, o.lr, o.beta1, o.beta2, o.eps, step, st);
    for (auto &l : L) {
        // statistics of each layer at its own resolution
        double cnt = count / (double)(1u << (2 * l.level));
        launch_bn_running(BUF + l.rm_off, BUF + l.rv_off, l.mean, l.var, l.cout, BN_MOM, cnt, st);
    }
    repack(st);
}

void unet_net::repack(hipStream_t st)
{
    if (pn) {  // FP32 weights are used as they are; fold the inference BN
        pn->refold(st);
        return;
    }
    if (cmap_valid) {  // the context maps hold the previous weights
        cmap_valid = 0;
        ++gen;  // captured graphs that add the maps are stale
    }
    for (auto &l : L)
        launch_pack_weights(P + l.w_off, l.cout, l.cin_real, l.map, l.cin_pad, l.Wp, l.Wd, st);
    refold(st);
}

void unet_net::refold(hipStream_t st)
{
    for (auto &l : L)
        launch_fold_bn(P + l.g_off, P + l.b_off, BUF + l.rm_off, BUF + l.rv_off, l.cout, BN_EPS,
                       scale + l.sc_off, shift + l.sc_off, st);
}

int unet_net::wrap_apply(helm_handle *h, const float2 *r, size_t rs, float2 *e, size_t es, int nb,
                         int accumulate, hipStream_t st, const int *mask, int nnet, const int *idx,
                         const int *pos, const double *fscale)
{
    const int n = h->n, nc = n / 2;
    if (nnet < 0) {
        nnet = nb;
        idx = pos = nullptr;
    }
    if (pn) {  // the paper's network on the fine grid
        if (nnet > 0) {
            int rc = pn->ensure_ws(nnet, n, false);
            if (rc) return rc;
            pn->input(r, rs, nnet, n, h->kappa0, h->gamma0, 0, idx, fscale, st);
            pn->forward(nnet, false, st);
        }
        pn->output(nb, n, e, es, accumulate, mask, pos, st);
        return HELM_OK;
    }
    if (nnet > 0) {
        int rc = ensure_ws(nnet, nc, nc, false);
        if (rc) return rc;
        launch_net_input(r, rs, nnet, n, h->kappa0, nullptr, rcoarse, red, s, x0, x0_stride(), st, idx,
                         fscale);
        forward_from_x0(nnet, nc, nc, false, st);
    }
    launch_net_output(out, s, nb, n, e, es, accumulate, st, mask, pos);
    return HELM_OK;
}

int unet_net::loss_grad(const unet_batch &bt, hipStream_t st)
{
    const int n = bt.n, nc = n / 2, nb = bt.nb;
    int rc = ensure_ws(nb, nc, nc, true);
    if (rc) return rc;
    launch_net_input((const float2 *)bt.r, (size_t)n * n, nb, n, nullptr, bt.kappa_c, rcoarse, red, s,
                     x0, x0_stride(), st);
    forward_from_x0(nb, nc, nc, true, st);
    launch_loss_grad(out, s, nb, n, (const float2 *)bt.e, dfine, red, gout, dloss, st);
    hipMemsetAsync(G, 0, nparams * sizeof(float), st);
    backward(nb, nc, nc, st);
    return HELM_OK;
}

int unet_net::pack_nchw_input(const float *x, int B, int H, int W, hipStream_t st)
{
    launch_nchw_to_nhwc(x, B, cfg.in_ch, H, W, x0_stride(), x0, st);
    return HELM_OK;
}

int unet_net::unpack_nchw_output(float *o, int B, int H, int W, hipStream_t st)
{
    launch_nhwc_to_nchw(out, B, cfg.out_ch, H, W, o, st);
    return HELM_OK;
}

extern "C" {

int helm_autotune(int enable) { return helm::conv_autotune(enable); }

int helm_autotune_force(int kind, int mf, int per_cu)
{
    if (helm::conv_force(kind, mf, per_cu)) {
        helm::set_error("helm_autotune_force: kind must be 0 or 1, mf 2 or 4, per_cu in [1, 64]");
        return HELM_E_INVALID;
    }
    return HELM_OK;
}

int helm_autotune_entries(void) { return helm::conv_autotune_entries(); }

int unet_create(const unet_cfg *cfg, unet_net **out)
{
    if (!cfg || !out) {
        set_error("unet_create: null argument");
        return HELM_E_INVALID;
    }
    *out = nullptr;
    if (cfg->arch == 1) {
        bool ok = cfg->levels >= 1 && cfg->levels <= 6 && cfg->in_ch == 4 && cfg->out_ch == 2 && cfg->head == 1 &&
                  cfg->context == 0;
        for (int l = 0; ok && l < cfg->levels; ++l) ok = cfg->widths[l] >= 1 && cfg->widths[l] <= 512;
        if (!ok) {
            set_error("unet_create: the paper's network (arch 1) takes levels 1..6, widths in [1, 512], in_ch 4, "
                      "out_ch 2, head 1, context 0");
            return HELM_E_INVALID;
        }
        auto *net = new unet_net();
        int rc = net->init_paper(*cfg);
        if (rc) {
            delete net;
            return rc;
        }
        *out = net;
        return HELM_OK;
    }
    if (cfg->arch != 0) {
        set_error("unet_create: arch must be 0 or 1");
        return HELM_E_INVALID;
    }
    if (cfg->levels < 1 || cfg->levels > 6 || cfg->in_ch < 1 || cfg->in_ch > 32 ||
        (cfg->head && cfg->out_ch != 2) || (!cfg->head && cfg->context)) {
        set_error("unet_create: unsupported configuration (levels 1..6, in_ch 1..32, out_ch 2 with a "
                  "head; an encoder (head 0) takes no context)");
        return HELM_E_INVALID;
    }
    for (int l = 0; l < cfg->levels; ++l)
        if (cfg->widths[l] < 32 || cfg->widths[l] % 32 != 0 || cfg->widths[l] > 256) {
            set_error("unet_create: widths must be multiples of 32 in [32, 256]");
            return HELM_E_INVALID;
        }
    auto *net = new unet_net();
    int rc = net->init(*cfg);
    if (rc) {
        delete net;
        return rc;
    }
    *out = net;
    return HELM_OK;
}

void unet_destroy(unet_net *net) { delete net; }

long long unet_num_params(const unet_net *net) { return net ? (long long)net->nparams : -1; }
long long unet_num_buffers(const unet_net *net) { return net ? (long long)net->nbuf : -1; }

int unet_set_params(unet_net *net, const float *params, const float *buffers, void *stream)
{
    if (!net || !params) {
        set_error("unet_set_params: null argument");
        return HELM_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    HELM_HIP_CHECK(hipMemcpyAsync(net->P, params, net->nparams * 4, hipMemcpyDeviceToDevice, st));
    if (buffers) {
        HELM_HIP_CHECK(hipMemcpyAsync(net->BUF, buffers, net->nbuf * 4, hipMemcpyDeviceToDevice, st));
    } else {
        std::vector<float> b(net->nbuf);
        for (auto &l : net->L) {
            std::fill(b.begin() + l.rm_off, b.begin() + l.rm_off + l.cout, 0.f);
            std::fill(b.begin() + l.rv_off, b.begin() + l.rv_off + l.cout, 1.f);
        }
        if (net->pn)
            for (const auto &l : net->pn->layers)
                if (l.kind != PL_OUT) {
                    std::fill(b.begin() + l.rm_off, b.begin() + l.rm_off + l.co, 0.f);
                    std::fill(b.begin() + l.rv_off, b.begin() + l.rv_off + l.co, 1.f);
                }
        HELM_HIP_CHECK(hipMemcpyAsync(net->BUF, b.data(), net->nbuf * 4, hipMemcpyHostToDevice, st));
        HELM_HIP_CHECK(hipStreamSynchronize(st));
    }
    HELM_HIP_CHECK(hipMemsetAsync(net->M, 0, net->nparams * 4, st));
    HELM_HIP_CHECK(hipMemsetAsync(net->V, 0, net->nparams * 4, st));
    net->step = 0;
    net->repack(st);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

// ---------------------------------------------------------------- state files
// Layout (little-endian): the 8-byte tag "HELMUNT1", then int32 in_ch,
// out_ch, levels, widths[6], context, head, arch; int64 nparams, nbuf; int32 Adam
// step; uint64 data seed, next sample index; then FP32 arrays: parameters
// [nparams], BN buffers [nbuf], Adam first moments [nparams], second moments
// [nparams].
static const char STATE_TAG[8] = {'H', 'E', 'L', 'M', 'U', 'N', 'T', '1'};

struct StateHead {
    int32_t cfg[12];
    int64_t np, nb;
    int32_t step;
    uint64_t seed, next;
};

static void state_head(const unet_net *net, StateHead &h)
{
    const unet_cfg &c = net->cfg;
    int32_t v[12] = {c.in_ch, c.out_ch, c.levels, 0, 0, 0, 0, 0, 0, c.context, c.head, c.arch};
    for (int l = 0; l < 6; ++l) v[3 + l] = l < c.levels ? c.widths[l] : 0;
    std::copy(v, v + 12, h.cfg);
    h.np = (int64_t)net->nparams;
    h.nb = (int64_t)net->nbuf;
    h.step = net->step;
    h.seed = net->data_seed;
    h.next = net->data_next;
}

static bool write_all(FILE *f, const void *p, size_t bytes) { return fwrite(p, 1, bytes, f) == bytes; }
static bool read_all(FILE *f, void *p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }

int unet_save(unet_net *net, const char *path, void *stream)
{
    if (!net || !path) {
        set_error("unet_save: null argument");
        return HELM_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    std::vector<float> buf(3 * net->nparams + net->nbuf);
    float *p = buf.data(), *b = p + net->nparams, *m = b + net->nbuf, *v = m + net->nparams;
    HELM_HIP_CHECK(hipMemcpyAsync(p, net->P, net->nparams * 4, hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipMemcpyAsync(b, net->BUF, net->nbuf * 4, hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipMemcpyAsync(m, net->M, net->nparams * 4, hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipMemcpyAsync(v, net->V, net->nparams * 4, hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    StateHead h;
    state_head(net, h);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) {
        set_error(std::string("unet_save: cannot open ") + tmp);
        return HELM_E_INVALID;
    }
    bool ok = write_all(f, STATE_TAG, 8) && write_all(f, h.cfg, sizeof h.cfg) && write_all(f, &h.np, 8) &&
              write_all(f, &h.nb, 8) && write_all(f, &h.step, 4) && write_all(f, &h.seed, 8) &&
              write_all(f, &h.next, 8) && write_all(f, buf.data(), buf.size() * 4);
    ok = (fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        set_error(std::string("unet_save: writing ") + path + " failed");
        return HELM_E_INVALID;
    }
    return HELM_OK;
}

int unet_load(unet_net *net, const char *path, void *stream)
{
    if (!net || !path) {
        set_error("unet_load: null argument");
        return HELM_E_INVALID;
    }
    FILE *f = fopen(path, "rb");
    if (!f) {
        set_error(std::string("unet_load: cannot open ") + path);
        return HELM_E_INVALID;
    }
    char tag[8];
    StateHead h, mine;
    state_head(net, mine);
    bool ok = read_all(f, tag, 8) && std::equal(tag, tag + 8, STATE_TAG) && read_all(f, h.cfg, sizeof h.cfg) &&
              read_all(f, &h.np, 8) && read_all(f, &h.nb, 8) && read_all(f, &h.step, 4) &&
              read_all(f, &h.seed, 8) && read_all(f, &h.next, 8);
    if (!ok || !std::equal(h.cfg, h.cfg + 12, mine.cfg) || h.np != mine.np || h.nb != mine.nb || h.step < 0) {
        fclose(f);
        set_error(std::string("unet_load: ") + path + " is not a state file of a network of this configuration");
        return HELM_E_INVALID;
    }
    std::vector<float> buf(3 * net->nparams + net->nbuf);
    ok = read_all(f, buf.data(), buf.size() * 4);
    fclose(f);
    if (!ok) {
        set_error(std::string("unet_load: ") + path + " is truncated");
        return HELM_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    float *p = buf.data(), *b = p + net->nparams, *m = b + net->nbuf, *v = m + net->nparams;
    HELM_HIP_CHECK(hipMemcpyAsync(net->P, p, net->nparams * 4, hipMemcpyHostToDevice, st));
    HELM_HIP_CHECK(hipMemcpyAsync(net->BUF, b, net->nbuf * 4, hipMemcpyHostToDevice, st));
    HELM_HIP_CHECK(hipMemcpyAsync(net->M, m, net->nparams * 4, hipMemcpyHostToDevice, st));
    HELM_HIP_CHECK(hipMemcpyAsync(net->V, v, net->nparams * 4, hipMemcpyHostToDevice, st));
    net->repack(st);
    HELM_HIP_CHECK(hipStreamSynchronize(st));  // the host copy is released on return
    net->step = h.step;
    net->data_seed = h.seed;
    net->data_next = h.next;
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

int unet_set_cursor(unet_net *net, unsigned long long seed, unsigned long long next)
{
    if (!net) {
        set_error("unet_set_cursor: null network");
        return HELM_E_INVALID;
    }
    net->data_seed = seed;
    net->data_next = next;
    return HELM_OK;
}

int unet_get_cursor(const unet_net *net, unsigned long long *seed, unsigned long long *next)
{
    if (!net || !seed || !next) {
        set_error("unet_get_cursor: null argument");
        return HELM_E_INVALID;
    }
    *seed = net->data_seed;
    *next = net->data_next;
    return HELM_OK;
}

// splitmix64 (Steele, Lea and Flood 2014) for the initial weights
static uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// standard normal by the Box-Muller transform of two uniforms in (0, 1]
static double normal01(uint64_t &state)
{
    double u1 = ((splitmix64(state) >> 11) + 1.0) * 0x1.0p-53;
    double u2 = ((splitmix64(state) >> 11) + 1.0) * 0x1.0p-53;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

int unet_init(unet_net *net, unsigned long long seed, void *stream)
{
    if (!net) {
        set_error("unet_init: null network");
        return HELM_E_INVALID;
    }
    std::vector<float> p(net->nparams, 0.f);
    uint64_t st = seed * 0x2545F4914F6CDD1Dull + 1;
    const double gain2 = 2.0 / (1.0 + SLOPE * SLOPE);  // LeakyReLU(0.2) gain squared
    if (net->pn) {
        // the paper's network: normal weights with std sqrt(2 / fan-in) (fan-in
        // cin K^2, a quarter of it for the stride-2 transposed convolutions),
        // BN weight 1, biases 0
        for (const auto &l : net->pn->layers) {
            const bool tr = l.kind == PL_UP || l.kind == PL_OUT;
            const double fan = (double)l.ci * l.K * l.K / (tr ? 4.0 : 1.0);
            const double sd = std::sqrt(2.0 / fan);
            for (size_t i = 0; i < (size_t)l.ci * l.co * l.K * l.K; ++i) p[l.w_off + i] = (float)(sd * normal01(st));
            if (l.kind != PL_OUT)
                for (int c = 0; c < l.co; ++c) p[l.g_off + c] = 1.f;
        }
    }
    for (auto &l : net->L) {
        const double sd = std::sqrt(gain2 / (9.0 * l.cin_real));
        for (size_t i = 0; i < (size_t)l.cout * l.cin_real * 9; ++i) p[l.w_off + i] = (float)(sd * normal01(st));
        for (int c = 0; c < l.cout; ++c) p[l.g_off + c] = 1.f;
    }
    if (net->cfg.head && !net->pn) {
        const double sd = std::sqrt(1.0 / net->cfg.widths[0]);
        for (size_t i = 0; i < (size_t)net->cfg.out_ch * net->cfg.widths[0]; ++i)
            p[net->head_w + i] = (float)(sd * normal01(st));
    }
    float *dp = nullptr;
    if (dev_malloc(&dp, net->nparams * sizeof(float)) != hipSuccess) {
        set_error("unet_init: out of device memory");
        return HELM_E_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    int rc = HELM_OK;
    if (hipMemcpyAsync(dp, p.data(), net->nparams * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("unet_init: copy failed");
        rc = HELM_E_HIP;
    }
    if (!rc) rc = unet_set_params(net, dp, nullptr, stream);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) {
        set_error("unet_init: synchronisation failed");
        rc = HELM_E_HIP;
    }
    dev_free(dp);
    return rc;
}

int unet_get_params(unet_net *net, float *params, float *buffers, void *stream)
{
    if (!net) {
        set_error("unet_get_params: null argument");
        return HELM_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    if (params) HELM_HIP_CHECK(hipMemcpyAsync(params, net->P, net->nparams * 4, hipMemcpyDeviceToDevice, st));
    if (buffers) HELM_HIP_CHECK(hipMemcpyAsync(buffers, net->BUF, net->nbuf * 4, hipMemcpyDeviceToDevice, st));
    return HELM_OK;
}

int unet_forward(unet_net *net, const float *x, int B, int H, int W, float *out, int training,
                 void *stream)
{
    if (!net || !x || !out || B < 1 || H < 1 || W < 1) {
        set_error("unet_forward: invalid argument");
        return HELM_E_INVALID;
    }
    const int div = 1 << (net->cfg.levels - 1);
    if (H % div || W % div) {
        set_error("unet_forward: H and W must be divisible by 2^(levels-1)");
        return HELM_E_SHAPE;
    }
    hipStream_t st = (hipStream_t)stream;
    if (net->pn) {
        if (H != W || H % (1 << net->cfg.levels)) {
            set_error("unet_forward: the paper's network needs H = W divisible by 2^levels");
            return HELM_E_SHAPE;
        }
        int rc = net->pn->ensure_ws(B, H, training != 0);
        if (rc) return rc;
        const size_t N = (size_t)H * W;
        HELM_HIP_CHECK(hipMemcpyAsync(net->pn->T[net->pn->x0t].v, x, (size_t)B * 4 * N * sizeof(float),
                                      hipMemcpyDeviceToDevice, st));
        net->pn->forward(B, training != 0, st);
        HELM_HIP_CHECK(hipMemcpyAsync(out, net->pn->T[net->pn->outt].v, (size_t)B * 2 * N * sizeof(float),
                                      hipMemcpyDeviceToDevice, st));
        HELM_HIP_CHECK(hipGetLastError());
        return HELM_OK;
    }
    if (!net->cfg.head) {
        set_error("unet_forward: an encoder has no head output (use unet_pair_encode)");
        return HELM_E_INVALID;
    }
    if (net->cfg.context && (!net->ctx_valid || net->ctx_H != H || (!net->ctx_shared && net->ctx_B != B))) {
        set_error("unet_forward: attach a matching encoder context first (unet_pair_encode)");
        return HELM_E_INVALID;
    }
    int rc = net->ensure_ws(B, H, W, training != 0);
    if (rc) return rc;
    rc = net->pack_nchw_input(x, B, H, W, st);
    if (rc) return rc;
    net->forward_from_x0(B, H, W, training != 0, st);
    rc = net->unpack_nchw_output(out, B, H, W, st);
    if (rc) return rc;
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

int unet_infer(unet_net *net, helm_handle *h, const float *r, float *e, int nrhs, void *stream)
{
    if (!net || !h || nrhs < 0 || (nrhs > 0 && (!r || !e))) {
        set_error("unet_infer: invalid argument");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    const int div = 1 << net->cfg.levels;  // the network runs on n/2
    if (h->n % div) {
        set_error("unet_infer: n must be divisible by 2^levels");
        return HELM_E_SHAPE;
    }
    if (!net->cfg.head || (net->cfg.context && (!net->ctx_valid || !net->ctx_shared || net->ctx_H != h->n / 2))) {
        set_error("unet_infer: needs a network with a head and, for a solver, the medium's context "
                  "(unet_pair_encode with nb = 1)");
        return HELM_E_INVALID;
    }
    size_t N = (size_t)h->n * h->n;
    int rc = net->wrap_apply(h, (const float2 *)r, N, (float2 *)e, N, nrhs, 0, (hipStream_t)stream);
    if (rc) return rc;
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

int unet_loss_grad(unet_net *net, const unet_batch *batch, double *loss_out, float *grads,
                   void *stream)
{
    if (net && net->pn) {
        if (!batch || !batch->r || !batch->e || !batch->kappa_f || !batch->gamma_f || batch->nb < 1 ||
            batch->n % (1 << net->cfg.levels)) {
            set_error("unet_loss_grad: the paper's network needs r, e, kappa_f, gamma_f and n divisible by "
                      "2^levels");
            return HELM_E_INVALID;
        }
        hipStream_t st = (hipStream_t)stream;
        const size_t N = (size_t)batch->n * batch->n;
        int rc = net->pn->loss_grad((const float2 *)batch->r, (const float2 *)batch->e, batch->kappa_f,
                                    batch->gamma_f, batch->fine_shared ? 0 : N, batch->nb, batch->n, &net->pn_loss,
                                    st);
        if (rc) return rc;
        if (grads) HELM_HIP_CHECK(hipMemcpyAsync(grads, net->G, net->nparams * 4, hipMemcpyDeviceToDevice, st));
        if (loss_out) *loss_out = net->pn_loss;
        HELM_HIP_CHECK(hipGetLastError());
        return HELM_OK;
    }
    if (!net || !batch || !batch->r || !batch->e || !batch->kappa_c || batch->nb < 1) {
        set_error("unet_loss_grad: invalid argument");
        return HELM_E_INVALID;
    }
    if (!net->cfg.head || net->cfg.context) {
        set_error("unet_loss_grad: encoder-solver pairs train through unet_pair_loss_grad");
        return HELM_E_INVALID;
    }
    const int div = 1 << net->cfg.levels;
    if (batch->n % div) {
        set_error("unet_loss_grad: n must be divisible by 2^levels");
        return HELM_E_SHAPE;
    }
    hipStream_t st = (hipStream_t)stream;
    int rc = net->loss_grad(*batch, st);
    if (rc) return rc;
    if (grads) HELM_HIP_CHECK(hipMemcpyAsync(grads, net->G, net->nparams * 4, hipMemcpyDeviceToDevice, st));
    if (loss_out) {
        HELM_HIP_CHECK(hipMemcpyAsync(loss_out, net->dloss, sizeof(double), hipMemcpyDeviceToHost, st));
        HELM_HIP_CHECK(hipStreamSynchronize(st));
    }
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

int unet_train_step(unet_net *net, const unet_batch *batch, const unet_train_opts *opts,
                    double *loss_out, void *stream)
{
    unet_train_opts o{1e-3f, 0.9f, 0.999f, 1e-8f};
    if (opts) o = *opts;
    hipStream_t st = (hipStream_t)stream;
    int rc = unet_loss_grad(net, batch, nullptr, nullptr, stream);
    if (rc) return rc;
    if (net->pn) {
        net->pn->update_running(batch->nb, st);  // the statistics of this batch, before the refold
        net->adam_update(o, 0.0, st);
        if (loss_out) *loss_out = net->pn_loss;
        HELM_HIP_CHECK(hipGetLastError());
        return HELM_OK;
    }
    net->adam_update(o, (double)batch->nb * (batch->n / 2) * (batch->n / 2), st);
    if (loss_out) {
        HELM_HIP_CHECK(hipMemcpyAsync(loss_out, net->dloss, sizeof(double), hipMemcpyDeviceToHost, st));
        HELM_HIP_CHECK(hipStreamSynchronize(st));
    }
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

static int check_pair(const unet_net *enc, const unet_net *sol, const char *who)
{
    if (!enc || !sol || enc->pn || sol->pn || enc->cfg.head || enc->cfg.in_ch != 1 || !sol->cfg.context ||
        !sol->cfg.head || enc->cfg.levels != sol->cfg.levels) {
        set_error(std::string(who) + ": needs an encoder (head 0, in_ch 1) and a solver (context 1) "
                                     "with the same levels");
        return HELM_E_INVALID;
    }
    for (int l = 0; l < enc->cfg.levels; ++l)
        if (enc->cfg.widths[l] != sol->cfg.widths[l]) {
            set_error(std::string(who) + ": encoder and solver widths differ");
            return HELM_E_INVALID;
        }
    return HELM_OK;
}

int unet_pair_encode(unet_net *enc, unet_net *sol, const float *kappa_c, int nb, int nc, void *stream)
{
    int rc = check_pair(enc, sol, "unet_pair_encode");
    if (rc) return rc;
    if (!kappa_c || nb < 1 || nc < 1 || nc % (1 << (enc->cfg.levels - 1))) {
        set_error("unet_pair_encode: invalid kappa_c, nb or nc (nc divisible by 2^(levels-1))");
        return HELM_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    if ((rc = enc->ensure_ws(nb, nc, nc, false))) return rc;
    enc->pack_nchw_input(kappa_c, nb, nc, nc, st);
    enc->forward_from_x0(nb, nc, nc, false, st);
    if ((rc = sol->attach_context(*enc, nb, nc, nc, st))) return rc;
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

int unet_pair_encode_medium(unet_net *enc, unet_net *sol, helm_handle *h, void *stream)
{
    int rc = check_pair(enc, sol, "unet_pair_encode_medium");
    if (rc) return rc;
    if (!h || h->n % (1 << enc->cfg.levels)) {
        set_error("unet_pair_encode_medium: invalid handle (n divisible by 2^levels)");
        return HELM_E_INVALID;
    }
    const int nc = h->n / 2;
    if (!h->kcoarse && dev_malloc(&h->kcoarse, (size_t)nc * nc * sizeof(float)) != hipSuccess) {
        set_error("unet_pair_encode_medium: out of device memory");
        return HELM_E_NOMEM;
    }
    if ((rc = helm_coarse_slowness(h, h->kcoarse, stream))) return rc;
    return unet_pair_encode(enc, sol, h->kcoarse, 1, nc, stream);
}

int unet_pair_loss_grad(unet_net *enc, unet_net *sol, const unet_batch *batch, double *loss_out,
                        float *enc_grads, float *sol_grads, void *stream)
{
    int rc = check_pair(enc, sol, "unet_pair_loss_grad");
    if (rc) return rc;
    if (!batch || !batch->r || !batch->e || !batch->kappa_c || batch->nb < 1 ||
        batch->n % (1 << sol->cfg.levels)) {
        set_error("unet_pair_loss_grad: invalid batch (n divisible by 2^levels)");
        return HELM_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    const int nb = batch->nb, nc = batch->n / 2;
    // encoder in training mode on each sample's medium; per-sample contexts
    if ((rc = enc->ensure_ws(nb, nc, nc, true))) return rc;
    enc->pack_nchw_input(batch->kappa_c, nb, nc, nc, st);
    enc->forward_from_x0(nb, nc, nc, true, st);
    if ((rc = sol->attach_context(*enc, nb, nc, nc, st))) return rc;
    sol->ctx_shared = 0;
    rc = sol->loss_grad(*batch, st);
    if (rc) return rc;
    // the gradient reaching each context flows back through the encoder
    HELM_HIP_CHECK(hipMemsetAsync(enc->G, 0, enc->nparams * sizeof(float), st));
    // seed the encoder's output gradients (stores; the encoder's backward
    // adds the upsampling shares to them)
    for (int l = 0; l < enc->cfg.levels; ++l)
        launch_slice_add(sol->gctx[l], enc->cfg.widths[l], 0, (size_t)nb * (nc >> l) * (nc >> l),
                         enc->cfg.widths[l], enc->act[enc->output_layer(l)].g, 0, st);
    enc->layers_backward(nb, nc, nc, st, true);
    // the training-mode context is not the medium's inference context
    sol->clear_context();
    if (enc_grads)
        HELM_HIP_CHECK(hipMemcpyAsync(enc_grads, enc->G, enc->nparams * 4, hipMemcpyDeviceToDevice, st));
    if (sol_grads)
        HELM_HIP_CHECK(hipMemcpyAsync(sol_grads, sol->G, sol->nparams * 4, hipMemcpyDeviceToDevice, st));
    if (loss_out) {
        HELM_HIP_CHECK(hipMemcpyAsync(loss_out, sol->dloss, sizeof(double), hipMemcpyDeviceToHost, st));
        HELM_HIP_CHECK(hipStreamSynchronize(st));
    }
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

int unet_pair_train_step(unet_net *enc, unet_net *sol, const unet_batch *batch,
                         const unet_train_opts *opts, double *loss_out, void *stream)
{
    unet_train_opts o{1e-3f, 0.9f, 0.999f, 1e-8f};
    if (opts) o = *opts;
    hipStream_t st = (hipStream_t)stream;
    int rc = unet_pair_loss_grad(enc, sol, batch, nullptr, nullptr, nullptr, stream);
    if (rc) return rc;
    const double count = (double)batch->nb * (batch->n / 2) * (batch->n / 2);
    sol->adam_update(o, count, st);
    enc->adam_update(o, count, st);
    if (loss_out) {
        HELM_HIP_CHECK(hipMemcpyAsync(loss_out, sol->dloss, sizeof(double), hipMemcpyDeviceToHost, st));
        HELM_HIP_CHECK(hipStreamSynchronize(st));
    }
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

}  // extern "C"
