"""Gradient-parity bounds derived from the oracle's own rounding spread.

A bf16 network's gradients through several training-mode BN layers are
sensitive to where each bf16 rounding lands: a different FP32 summation
order flips some rounding decisions, and every BN backward on the way to a
tensor amplifies the difference.  How large that is depends on the network
and the batch, so it is measured here, on the CPU, for the exact network and
batch a test uses:
  g64  the FP64 oracle (reference gradient),
  gE   the oracle with bf16 rounding at the device's rounding points,
  gE'  the same with every convolution output multiplied by (1 + 1e-6 N(0,1))
       before its bf16 rounding (K draws, oracle hook JITTER): the size of
       the FP32 summation-order differences of a K-term sum, applied inside
       every layer the way another device's summation order applies them.
       Each draw flips rounding decisions without changing the mathematics.
       (Perturbing only the network input under-counts: a device's
       differences enter at every layer, and the bf16 rounding of the
       activations, not of the gradients, is what the training-mode BN
       layers amplify; measured on this oracle, forward rounding alone moves
       the deepest gradients by about 25% from FP64, gradient rounding alone
       by about 1%.)
spread_E(t) = max over draws of rel(gE', gE) (and rel(gE, g64) for the FP32
comparison).  A device gradient is one more such realisation, so it must lie
within twice the measured spread (plus a small floor) of the oracle.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import unet_oracle as U

FLOOR_REL = 2e-3
FLOOR_COS = 1e-5
MARGIN = 2.0


def rel(a, b):
    return float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300))


def cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def oracle_grads(loss_fn, params_list, dtype, emulate, r):
    """loss_fn(params_list (cast to dtype, requiring grad), r) -> loss.
    Returns (loss, [{name: flat float64 gradient}] per network)."""
    pgs = [{k: v.detach().clone().to(dtype).requires_grad_(True) for k, v in p.items()}
           for p in params_list]
    U.EMULATE_BF16 = emulate
    try:
        lo = loss_fn(pgs, r, dtype)
        lo.backward()
    finally:
        U.EMULATE_BF16 = False
    return lo.item(), [{k: pg[k].grad.double().reshape(-1).numpy() for k in pg} for pg in pgs]


JITTER_REL = 1e-6


def measure(loss_fn, params_list, r, draws=4, seed=12345):
    """Reference gradients and per-tensor spreads.  Returns a dict with
    'g64', 'g32', 'gE' (lists of per-network dicts) and 'spread32'/'spreadE'
    (lists of {name: (rel, 1 - cos)})."""
    _, g64 = oracle_grads(loss_fn, params_list, torch.float64, False, r)
    l32, g32 = oracle_grads(loss_fn, params_list, torch.float32, False, r)
    lE, gE = oracle_grads(loss_fn, params_list, torch.float32, True, r)
    pert = []
    for d in range(draws):
        U.JITTER = (torch.Generator().manual_seed(seed + d), JITTER_REL)
        try:
            pert.append(oracle_grads(loss_fn, params_list, torch.float32, True, r)[1])
        finally:
            U.JITTER = None
    spread32, spreadE = [], []
    for i in range(len(params_list)):
        s32, sE = {}, {}
        for k in g64[i]:
            re = max(rel(d[i][k], gE[i][k]) for d in pert)
            ce = max(1 - cos(d[i][k], gE[i][k]) for d in pert)
            sE[k] = (re, ce)
            s32[k] = (max(re, rel(gE[i][k], g64[i][k])), max(ce, 1 - cos(gE[i][k], g64[i][k])))
        spread32.append(s32)
        spreadE.append(sE)
    return dict(g64=g64, g32=g32, gE=gE, loss32=l32, lossE=lE, spread32=spread32, spreadE=spreadE)


def check(device_flat, cfg, ref, spread, label):
    """Compare a device gradient (flat, canonical order of cfg) with the
    reference per tensor; returns the list of tensors outside the bound and
    prints the table."""
    bad, off = [], 0
    for k, shape in U.param_shapes(cfg).items():
        cnt = int(np.prod(shape))
        g = np.asarray(device_flat[off:off + cnt], dtype=np.float64)
        off += cnt
        r_, c_ = rel(g, ref[k]), cos(g, ref[k])
        s_rel, s_cos = spread[k]
        tol, ctol = MARGIN * s_rel + FLOOR_REL, MARGIN ** 2 * s_cos + FLOOR_COS
        print(f"{label} {k:10s} rel={r_:.3e} (bound {tol:.3e})  1-cos={1 - c_:.2e} (bound {ctol:.2e})")
        if r_ > tol or 1 - c_ > ctol:
            bad.append((label, k, r_, c_, tol, ctol))
    return bad
