"""CPU oracle of the U-Net preconditioner, its training loss and Adam.

TEST INFRASTRUCTURE ONLY: the plain reference the GPU network is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it.  It shares no code with the GPU library.

Written with plain PyTorch CPU operations (conv2d, batch_norm, leaky_relu,
max_pool2d, interpolate) in the precision of the tensors passed in (float32
for parity, float64 for finite-difference checks); gradients come from
torch.autograd over these operations.

Network (section 3.1 gives the U-Net idea; the layer recipe here is the
configured network's): L levels of widths w_0..w_{L-1}; level l applies twice
[3x3 convolution (zero padding 1, no bias) -> batch normalisation ->
LeakyReLU(0.2)]; 2x2 max pooling between levels; on the way up a bilinear x2
upsampling (half-pixel centres) concatenated as [upsampled, skip] and the
same double convolution; a 1x1 convolution with bias maps w_0 channels to
(Re e, Im e).  With an encoder context (section 3.3, eq. 3.5) the context
tensor f^(l) of level l is concatenated to the input of down-level l and
after [upsampled, skip] at up-level l.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch
import torch.nn.functional as F

from oracle import helm_oracle

SLOPE = 0.2
EPS = 1e-5
MOMENTUM = 0.1


@dataclass
class UNetCfg:
    in_ch: int = 3
    out_ch: int = 2
    widths: tuple = (32, 64, 128, 256)
    context: bool = False   # solver of an encoder-solver pair
    head: bool = True       # False for an encoder (its outputs are the contexts)

    @property
    def levels(self):
        return len(self.widths)


def layer_specs(cfg: UNetCfg):
    """[(name, cin, cout)] of the 3x3 convolutions, in forward order."""
    w = cfg.widths
    L = cfg.levels
    ctx = (lambda l: w[l]) if cfg.context else (lambda l: 0)
    specs = []
    for l in range(L):
        cin = (cfg.in_ch if l == 0 else w[l - 1]) + ctx(l)
        specs.append((f"enc{l}a", cin, w[l]))
        specs.append((f"enc{l}b", w[l], w[l]))
    for l in range(L - 2, -1, -1):
        cin = w[l + 1] + w[l] + ctx(l)
        specs.append((f"dec{l}a", cin, w[l]))
        specs.append((f"dec{l}b", w[l], w[l]))
    return specs


def param_shapes(cfg: UNetCfg):
    """Ordered {name: shape} of every parameter (the canonical flat order)."""
    shapes = {}
    for name, cin, cout in layer_specs(cfg):
        shapes[name + ".w"] = (cout, cin, 3, 3)
        shapes[name + ".g"] = (cout,)
        shapes[name + ".b"] = (cout,)
    if cfg.head:
        shapes["head.w"] = (cfg.out_ch, cfg.widths[0], 1, 1)
        shapes["head.b"] = (cfg.out_ch,)
    return shapes


def buffer_shapes(cfg: UNetCfg):
    """BN running statistics."""
    out = {}
    for name, _, cout in layer_specs(cfg):
        out[name + ".rm"] = (cout,)
        out[name + ".rv"] = (cout,)
    return out


def init_params(cfg: UNetCfg, seed: int, dtype=torch.float32):
    """Kaiming-normal (fan-in, LeakyReLU gain) convolution weights from a seeded
    numpy generator; BN weight 1, bias 0; head small normal, bias 0."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in param_shapes(cfg).items():
        if name.endswith(".w") and not name.startswith("head"):
            fan_in = shape[1] * 9
            std = math.sqrt(2.0 / ((1 + SLOPE ** 2) * fan_in))
            p[name] = torch.tensor(rng.standard_normal(shape) * std, dtype=dtype)
        elif name == "head.w":
            p[name] = torch.tensor(rng.standard_normal(shape) * math.sqrt(1.0 / shape[1]),
                                   dtype=dtype)
        elif name.endswith(".g"):
            p[name] = torch.ones(shape, dtype=dtype)
        else:
            p[name] = torch.zeros(shape, dtype=dtype)
    buf = {}
    for name, shape in buffer_shapes(cfg).items():
        buf[name] = torch.zeros(shape, dtype=dtype) if name.endswith(".rm") else torch.ones(shape, dtype=dtype)
    return p, buf


def flatten(cfg, p):
    return torch.cat([p[k].reshape(-1) for k in param_shapes(cfg)])


def unflatten(cfg, flat, dtype=torch.float32):
    out, off = {}, 0
    flat = torch.as_tensor(flat)
    for k, shape in param_shapes(cfg).items():
        n = int(np.prod(shape))
        out[k] = flat[off:off + n].reshape(shape).to(dtype).clone()
        off += n
    return out


def bf16_round(t):
    """Round to the nearest bfloat16 (ties to even), back in t's dtype."""
    return t.to(torch.bfloat16).to(t.dtype)


class _RoundGrad(torch.autograd.Function):
    """Identity forward; rounds the incoming gradient to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.view_as(x)

    @staticmethod
    def backward(ctx, g):
        return bf16_round(g)


def _ste_round(t):
    """bfloat16 rounding in the forward pass, identity in the backward pass."""
    return t + (bf16_round(t) - t).detach()


# When True the forward pass rounds weights, activations and the network
# input to bfloat16, and the backward pass rounds the gradient that reaches
# each convolution output, at the points where a bf16 device implementation
# does (FP32 accumulation everywhere else).  Off by default.
EMULATE_BF16 = False

# Spread measurement only (off by default, no effect on the arithmetic when
# None): a (torch.Generator, rel) pair.  With EMULATE_BF16 on, every
# convolution output is multiplied by (1 + rel * N(0, 1)) before its bf16
# rounding, which models another FP32 summation order inside every layer (a
# sum of K terms in FP32 carries a relative error of order sqrt(K) 2^-24).
JITTER = None


def _jitter(y):
    if JITTER is None:
        return y
    gen, rel_ = JITTER
    f = 1.0 + rel_ * torch.randn(y.shape, generator=gen, dtype=torch.float64).to(y.dtype)
    return y * f


def _block(x, p, buf, name, training, stats):
    """3x3 conv -> BN -> LeakyReLU."""
    if EMULATE_BF16:
        y = _RoundGrad.apply(_jitter(F.conv2d(x, _ste_round(p[name + ".w"]), padding=1)))
    else:
        y = F.conv2d(x, p[name + ".w"], padding=1)
    if training:
        mean = y.mean(dim=(0, 2, 3))
        var = y.var(dim=(0, 2, 3), unbiased=False)
        if stats is not None:
            stats[name] = (mean.detach(), var.detach())
        z = (y - mean[None, :, None, None]) / torch.sqrt(var[None, :, None, None] + EPS)
    else:
        z = (y - buf[name + ".rm"][None, :, None, None]) / torch.sqrt(
            buf[name + ".rv"][None, :, None, None] + EPS)
    z = z * p[name + ".g"][None, :, None, None] + p[name + ".b"][None, :, None, None]
    a = F.leaky_relu(z, SLOPE)
    return _ste_round(a) if EMULATE_BF16 else a


def up2(x):
    """Bilinear x2 upsampling with half-pixel centres, edge-clamped."""
    return F.interpolate(x, scale_factor=2, mode="bilinear", align_corners=False)


def forward(cfg: UNetCfg, p, buf, x, ctx=None, training=False, stats=None):
    """x: [B, in_ch, H, W].  Returns the head output [B, out_ch, H, W], or for
    an encoder (head=False) the list of per-level context tensors."""
    L = cfg.levels
    skips = []
    h = _ste_round(x) if EMULATE_BF16 else x
    for l in range(L):
        if l > 0:
            h = F.max_pool2d(h, 2)
        if cfg.context:
            h = torch.cat([h, ctx[l]], dim=1)
        h = _block(h, p, buf, f"enc{l}a", training, stats)
        h = _block(h, p, buf, f"enc{l}b", training, stats)
        skips.append(h)
    outs = [None] * L
    outs[L - 1] = h
    for l in range(L - 2, -1, -1):
        u = up2(h)
        if EMULATE_BF16:
            u = _ste_round(u)
        h = torch.cat([u, skips[l]], dim=1)
        if cfg.context:
            h = torch.cat([h, ctx[l]], dim=1)
        h = _block(h, p, buf, f"dec{l}a", training, stats)
        h = _block(h, p, buf, f"dec{l}b", training, stats)
        outs[l] = h
    if not cfg.head:
        return outs
    return F.conv2d(h, p["head.w"], p["head.b"])


def update_running_stats(buf, stats, count):
    """BN running statistics (momentum 0.1, unbiased running variance)."""
    for name, (mean, var) in stats.items():
        unb = var * count / max(count - 1, 1)
        buf[name + ".rm"].mul_(1 - MOMENTUM).add_(MOMENTUM * mean)
        buf[name + ".rv"].mul_(1 - MOMENTUM).add_(MOMENTUM * unb)


def encode(cfg_enc: UNetCfg, p, buf, kappa_c, training=False, stats=None, dtype=torch.float32):
    """Encoder of an encoder-solver pair (section 3.3, eq. 3.5): the headless
    network on the coarse slowness [B, n, n] (or [n, n]); returns the
    per-level contexts f^(l) (the up-path output at level l, the bottleneck
    output at the last level)."""
    k = torch.as_tensor(np.asarray(kappa_c), dtype=dtype)
    if k.dim() == 2:
        k = k[None]
    return forward(cfg_enc, p, buf, k[:, None], training=training, stats=stats)


# ----------------------------------------------------------------- wrapper

def _restrict_c(x):
    return helm_oracle.restrict(x)


def _prolong_c(xc):
    return helm_oracle.prolong(xc)


def net_input(r, kappa_c, n):
    """R(h^2 r) / s with s the RMS of |R(h^2 r)| on the coarse grid (input
    scaling of section 3.4; the RMS normalisation makes the map positively
    homogeneous).  Returns (input [3, n/2, n/2] float64, s)."""
    h2 = 1.0 / (n * n)
    rc = _restrict_c(h2 * np.asarray(r, dtype=np.complex128))
    s = float(np.sqrt(np.mean(np.abs(rc) ** 2)))
    if s == 0.0:
        return None, 0.0
    z = rc / s
    inp = np.stack([z.real, z.imag, np.asarray(kappa_c, dtype=np.float64)])
    return inp, s


def unet_apply(cfg, p, buf, r, kappa_c, ctx=None, dtype=torch.float32):
    """e = P s Net(R(h^2 r)/s, kappa_c): the network as an error predictor for
    residual r on the fine grid (network on the grid n/2)."""
    n = r.shape[-1]
    inp, s = net_input(r, kappa_c, n)
    if s == 0.0:
        return np.zeros((n, n), dtype=np.complex128)
    x = torch.tensor(inp[None], dtype=dtype)
    with torch.no_grad():
        out = forward(cfg, p, buf, x, ctx=ctx, training=False)[0].double().numpy()
    ec = s * (out[0] + 1j * out[1])
    return _prolong_c(ec)


def cgc_compose(hier, net_fn, r, weight=0.8):
    """Algorithm 2 with a coarse-grid correction given as a map net_fn from a
    fine residual to a fine error estimate: a damped Jacobi sweep on A from
    zero, the correction of the new residual, a damped Jacobi sweep on A.
        e1 = w D_A^-1 r,  e2 = e1 + net_fn(r - A e1),  e = e2 + w D_A^-1 (r - A e2)"""
    kap, gam, om = hier.kappa0, hier.gamma0, hier.omega
    e1 = helm_oracle.jacobi(kap, gam, om, r, np.zeros_like(r), shift=0.0, weight=weight)
    r1 = helm_oracle.residual(kap, gam, om, r, e1)
    e2 = e1 + net_fn(r1)
    return helm_oracle.jacobi(kap, gam, om, r, e2, shift=0.0, weight=weight)


def defl_compose(hier, net_fn, r):
    """Eq. 3.4 with the error estimate given as a map net_fn: e0 = net_fn(r),
    then an SL V-cycle from zero on the remaining residual,
        e = e0 + V(0, r - A e0)."""
    e0 = net_fn(r)
    r1 = hier.residual_A(r, e0)
    return e0 + hier.vcycle(r1)


def precond_cgc(hier, cfg, p, buf, r, kappa_c, weight=0.8, ctx=None):
    """M_CU: Jacobi on A, network coarse correction of the new residual,
    Jacobi on A (Algorithm 2 with the network's coarse-grid correction)."""
    return cgc_compose(hier, lambda v: unet_apply(cfg, p, buf, v, kappa_c, ctx=ctx), r, weight)


def precond_defl(hier, cfg, p, buf, r, kappa_c, ctx=None):
    """M_VU (eq. 3.4): e0 = network(r), then an SL V-cycle on the remaining
    residual: e = e0 + V(0, r - A e0)."""
    return defl_compose(hier, lambda v: unet_apply(cfg, p, buf, v, kappa_c, ctx=ctx), r)


# ----------------------------------------------------------------- training

def training_loss(cfg, p, buf, r_batch, e_batch, kappa_c_batch, ctx=None, stats=None,
                  dtype=torch.float32):
    """Mean over the batch of ||P Net(R(h^2 r)/s) - e/s||^2 / N_fine (the
    supervised error loss of eq. 3.7 with the input scaling of section 3.4).
    r_batch, e_batch: complex [B, n, n]; kappa_c_batch: [B, n/2, n/2]."""
    B, n = r_batch.shape[0], r_batch.shape[-1]
    xs, targets = [], []
    for b in range(B):
        inp, s = net_input(r_batch[b], kappa_c_batch[b], n)
        xs.append(inp)
        targets.append(np.asarray(e_batch[b]) / s)
    x = torch.tensor(np.stack(xs), dtype=dtype)
    out = forward(cfg, p, buf, x, ctx=ctx, training=True, stats=stats)
    loss = 0.0
    for b in range(B):
        ec = out[b, 0] + 1j * out[b, 1]
        e = prolong_torch(ec)
        t = torch.tensor(targets[b])
        d = e - t.to(e.dtype)
        loss = loss + (d.real ** 2 + d.imag ** 2).sum() / (n * n)
    return loss / B


def prolong_torch(ec):
    """Bilinear prolongation of eq. 2.9 as a transposed stride-2 convolution
    with (1/4)[1 2 1; 2 4 2; 1 2 1] (output padding 1), on a complex tensor."""
    k = torch.tensor([[1.0, 2.0, 1.0], [2.0, 4.0, 2.0], [1.0, 2.0, 1.0]],
                     dtype=ec.real.dtype) / 4.0
    parts = []
    for comp in (ec.real, ec.imag):
        y = F.conv_transpose2d(comp[None, None], k[None, None], stride=2, padding=1,
                               output_padding=1)
        parts.append(y[0, 0])
    return torch.complex(parts[0], parts[1])


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) with bias correction, no weight decay; updates the
    dicts in place.  step counts from 1."""
    for k in params:
        g = grads[k]
        m[k] = b1 * m[k] + (1 - b1) * g
        v[k] = b2 * v[k] + (1 - b2) * g * g
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        params[k] = params[k] - lr * mh / (torch.sqrt(vh) + eps)
    return params, m, v


def training_triple(hier, x):
    """Training data of section 3.4 (eq. 3.8-3.9) with one flexible-GMRES
    step from zero and the SL V-cycle as preconditioner: b = A x,
    z = V(b), alpha = argmin ||b - alpha A z||, r = b - alpha A z,
    e = x - alpha z."""
    kap, gam, om = hier.kappa0, hier.gamma0, hier.omega
    x = np.asarray(x, dtype=np.complex128)
    b = helm_oracle.apply(kap, gam, om, x)
    z = hier.vcycle(b)
    w = helm_oracle.apply(kap, gam, om, z)
    alpha = np.vdot(w, b) / np.vdot(w, w)
    return b - alpha * w, x - alpha * z


def training_triple_k(hier, x, k):
    """Training data of eq. 3.8-3.9 with k flexible-GMRES steps: b = A x,
    x~ = k steps of FGMRES(max(k, 10)) with the SL V-cycle from zero (fewer
    if the solve ends exactly earlier), r = b - A x~, e = x - x~."""
    kap, gam, om = hier.kappa0, hier.gamma0, hier.omega
    x = np.asarray(x, dtype=np.complex128)
    b = helm_oracle.apply(kap, gam, om, x)
    xt, st = hier.fgmres(b, m=max(k, 10), tol=1e-300, maxit=k)
    return b - helm_oracle.apply(kap, gam, om, xt), x - xt, st["iterations"]


def mix_triples(r, e, coef):
    """Augmentation by linear combinations (section 3.4): r'_b = sum_j
    coef[b, j] r_j and e'_b = sum_j coef[b, j] e_j for triples of one
    medium."""
    c = np.asarray(coef, dtype=np.float64)
    r = np.asarray(r, dtype=np.complex128)
    e = np.asarray(e, dtype=np.complex128)
    return np.tensordot(c, r, axes=(1, 0)), np.tensordot(c, e, axes=(1, 0))


def pair_training_loss(cfg_enc, pe, bufe, cfg_sol, ps, bufs, r_batch, e_batch, kappa_c_batch,
                       stats_e=None, stats_s=None, dtype=torch.float32):
    """Joint loss of an encoder-solver pair: the solver's training loss with
    each sample's contexts computed by the encoder from its own medium (both
    networks with training-mode BN; trained together as in section 4.3.2)."""
    ctx = encode(cfg_enc, pe, bufe, kappa_c_batch, training=True, stats=stats_e, dtype=dtype)
    return training_loss(cfg_sol, ps, bufs, r_batch, e_batch, kappa_c_batch, ctx=ctx, stats=stats_s,
                         dtype=dtype)
