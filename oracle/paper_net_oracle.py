"""CPU oracle of the paper's own network (section 3.1, eq. 3.1-3.3).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
library.  Plain PyTorch CPU operations (conv2d, conv_transpose2d,
batch_norm, elu) in the precision of the tensors passed in; gradients from
torch.autograd.

The network maps the fine grid to the fine grid; its transfers are learned:
  input   x^(0): 4 channels (Re r^, Im r^, kappa^2, gamma) on n x n, with
          r^ = h^2 r / s (section 3.4's h^2 scaling; s the RMS of |h^2 r|,
          which makes the map positively homogeneous);
  down    for l = 1..L:  x^(l) = elu(BN(R_l x^(l-1)))            (eq. 3.1)
          R_l a 5 x 5 convolution of stride 2 (zero padding 2) from c_{l-1}
          to c_l channels (c_0 = 4), then ResNet blocks at level l:
          x <- elu(BN(x + K2 elu(BN(K1 x))))                     (eq. 3.2)
          with 3 x 3 K1, K2 (c_l -> c_l): one block per level, three at the
          coarsest level L;
  up      y^(L) = x^(L); for l = L-1..1:
          y^(l) = cat(BN(P_{l+1} elu(y^(l+1))), x^(l))           (eq. 3.3)
          P a 5 x 5 transposed convolution of stride 2 (padding 2, output
          padding 1) to c_l channels;
  output  e = P_1 elu(y^(1)): the transposed convolution to 2 channels
          (Re e, Im e) on the fine grid, with a bias (no BN).
Convolutions before a BN carry no bias.  BN: eps 1e-5, momentum 0.1, batch
statistics (biased variance) in training, running statistics in inference.
elu(z) = z for z > 0, exp(z) - 1 otherwise.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch
import torch.nn.functional as F

EPS = 1e-5
MOMENTUM = 0.1


@dataclass
class PaperNetCfg:
    widths: tuple = (16, 32, 64)
    in_ch: int = 4
    out_ch: int = 2
    coarsest_blocks: int = 3

    @property
    def levels(self):
        return len(self.widths)


def layers(cfg: PaperNetCfg):
    """(name, kind, cin, cout, k) in forward order; kind: 'down' (5x5 stride 2
    + BN), 'res1'/'res2' (3x3 + BN, the two convolutions of a ResNet block),
    'up' (5x5 transposed + BN), 'out' (5x5 transposed with bias)."""
    out = []
    L = cfg.levels
    cin = cfg.in_ch
    for l in range(1, L + 1):
        c = cfg.widths[l - 1]
        out.append((f"down{l}", "down", cin, c, 5))
        for r in range(cfg.coarsest_blocks if l == L else 1):
            out.append((f"res{l}_{r}a", "res1", c, c, 3))
            out.append((f"res{l}_{r}b", "res2", c, c, 3))
        cin = c
    ch = cfg.widths[L - 1]
    for l in range(L - 1, 0, -1):
        c = cfg.widths[l - 1]
        out.append((f"up{l}", "up", ch, c, 5))
        ch = 2 * c
    out.append(("out", "out", ch, cfg.out_ch, 5))
    return out


def param_shapes(cfg: PaperNetCfg):
    """Flat parameter order: per layer its weight (conv: [cout][cin][k][k];
    transposed: [cin][cout][k][k]), then BN weight and bias [cout] (the
    output layer: its bias [out_ch] instead)."""
    shapes = {}
    for name, kind, cin, cout, k in layers(cfg):
        if kind in ("up", "out"):
            shapes[name + ".w"] = (cin, cout, k, k)
        else:
            shapes[name + ".w"] = (cout, cin, k, k)
        if kind == "out":
            shapes[name + ".bias"] = (cout,)
        else:
            shapes[name + ".g"] = (cout,)
            shapes[name + ".b"] = (cout,)
    return shapes


def buffer_shapes(cfg: PaperNetCfg):
    return {f"{name}.{s}": (cout,) for name, kind, cin, cout, k in layers(cfg) if kind != "out"
            for s in ("rm", "rv")}


def init_params(cfg: PaperNetCfg, seed: int, dtype=torch.float32):
    """Seeded test initialisation: normal weights with std sqrt(2 / fan-in)
    (fan-in = cin k^2 for convolutions; for transposed convolutions the
    inputs that reach one output, cin k^2 / 4), BN weight 1, bias 0; running
    mean 0, variance 1."""
    g = torch.Generator().manual_seed(seed)
    p = {}
    for name, kind, cin, cout, k in layers(cfg):
        fan = cin * k * k / (4.0 if kind in ("up", "out") else 1.0)
        shape = param_shapes(cfg)[name + ".w"]
        p[name + ".w"] = (torch.randn(shape, generator=g, dtype=torch.float64) * np.sqrt(2.0 / fan)).to(dtype)
        if kind == "out":
            p[name + ".bias"] = torch.zeros(cout, dtype=dtype)
        else:
            p[name + ".g"] = torch.ones(cout, dtype=dtype)
            p[name + ".b"] = torch.zeros(cout, dtype=dtype)
    buf = {k: (torch.zeros(s, dtype=dtype) if k.endswith(".rm") else torch.ones(s, dtype=dtype))
           for k, s in buffer_shapes(cfg).items()}
    return p, buf


def flatten(cfg, p):
    return torch.cat([p[k].reshape(-1) for k in param_shapes(cfg)])


def unflatten(cfg, flat, dtype=torch.float32):
    out, off = {}, 0
    for k, shape in param_shapes(cfg).items():
        n = int(np.prod(shape))
        out[k] = flat[off:off + n].reshape(shape).to(dtype).clone()
        off += n
    return out


def _bn(y, p, buf, name, training, stats):
    if training:
        mean = y.mean(dim=(0, 2, 3))
        var = y.var(dim=(0, 2, 3), unbiased=False)
        if stats is not None:
            stats[name] = (mean.detach(), var.detach())
    else:
        mean, var = buf[name + ".rm"], buf[name + ".rv"]
    z = (y - mean[None, :, None, None]) / torch.sqrt(var[None, :, None, None] + EPS)
    return z * p[name + ".g"][None, :, None, None] + p[name + ".b"][None, :, None, None]


def forward(cfg: PaperNetCfg, p, buf, x, training=False, stats=None):
    """x: [B, 4, n, n] -> e: [B, 2, n, n]."""
    L = cfg.levels
    h = x
    skips = []
    for l in range(1, L + 1):
        h = F.elu(_bn(F.conv2d(h, p[f"down{l}.w"], stride=2, padding=2), p, buf, f"down{l}", training, stats))
        for r in range(cfg.coarsest_blocks if l == L else 1):
            a, b = f"res{l}_{r}a", f"res{l}_{r}b"
            t = F.elu(_bn(F.conv2d(h, p[a + ".w"], padding=1), p, buf, a, training, stats))
            h = F.elu(_bn(h + F.conv2d(t, p[b + ".w"], padding=1), p, buf, b, training, stats))
        skips.append(h)
    y = skips[L - 1]
    for l in range(L - 1, 0, -1):
        u = _bn(F.conv_transpose2d(F.elu(y), p[f"up{l}.w"], stride=2, padding=2, output_padding=1), p, buf,
                f"up{l}", training, stats)
        y = torch.cat([u, skips[l - 1]], dim=1)
    return F.conv_transpose2d(F.elu(y), p["out.w"], p["out.bias"], stride=2, padding=2, output_padding=1)


def update_running_stats(buf, stats, counts):
    """BN running statistics (momentum 0.1, unbiased running variance);
    counts[name] = values per channel in the batch."""
    for name, (mean, var) in stats.items():
        c = counts[name]
        buf[name + ".rm"].mul_(1 - MOMENTUM).add_(MOMENTUM * mean)
        buf[name + ".rv"].mul_(1 - MOMENTUM).add_(MOMENTUM * var * c / max(c - 1, 1))


def net_input(r, kappa, gamma, n):
    """The 4 input channels and the scale s: r^ = h^2 r / s with s the RMS of
    |h^2 r| over the fine grid (s = 0 gives a zero input and zero output)."""
    h2 = 1.0 / (n * n)
    rr = np.asarray(r, dtype=np.complex128) * h2
    s = float(np.sqrt(np.mean(np.abs(rr) ** 2)))
    q = rr / s if s > 0 else np.zeros_like(rr)
    k = np.asarray(kappa, dtype=np.float64)
    return np.stack([q.real, q.imag, k * k, np.asarray(gamma, dtype=np.float64)]), s


def apply(cfg, p, buf, r, kappa, gamma, dtype=torch.float32):
    """e = s Net(r^, kappa^2, gamma) on the fine grid (inference BN)."""
    n = r.shape[-1]
    x, s = net_input(r, kappa, gamma, n)
    if s == 0:
        return np.zeros((n, n), dtype=np.complex128)
    pp = {k: v.to(dtype) for k, v in p.items()}
    bb = {k: v.to(dtype) for k, v in buf.items()}
    with torch.no_grad():
        o = forward(cfg, pp, bb, torch.tensor(x[None], dtype=dtype)).double().numpy()[0]
    return s * (o[0] + 1j * o[1])


def training_loss(cfg, p, buf, r_batch, e_batch, kappa, gamma, stats=None, dtype=torch.float32):
    """Mean over the batch of ||Net(r^_b) - e_b / s_b||^2 / n^2 (eq. 3.7 in
    the scaled form), training-mode BN; kappa, gamma: [n, n] or [B, n, n]."""
    B, n = r_batch.shape[0], r_batch.shape[-1]
    kap = np.broadcast_to(np.asarray(kappa), (B, n, n))
    gam = np.broadcast_to(np.asarray(gamma), (B, n, n))
    xs, ts = [], []
    for b in range(B):
        x, s = net_input(r_batch[b], kap[b], gam[b], n)
        xs.append(x)
        ts.append(np.asarray(e_batch[b]) / s)
    out = forward(cfg, p, buf, torch.tensor(np.stack(xs), dtype=dtype), training=True, stats=stats)
    t = torch.tensor(np.stack([np.stack([v.real, v.imag]) for v in ts]), dtype=out.dtype)
    return ((out - t) ** 2).sum() / (n * n) / B
