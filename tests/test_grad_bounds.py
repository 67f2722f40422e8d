"""The gradient bounds of tests/grad_bounds.py separate rounding from
mistakes: gradients computed with a backward term dropped (planted in the
oracle, on the CPU) fall outside the bounds the device tests use, while an
independent rounding realisation stays inside them."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet_oracle as U
from tests import grad_bounds as GB

WIDTHS = (32, 64, 128)


def _setup():
    cfg = U.UNetCfg(widths=WIDTHS)
    p, buf = U.init_params(cfg, 21)
    rng = np.random.default_rng(4)
    n, nb = 64, 3
    r = (rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))).astype(np.complex64)
    e = (rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))).astype(np.complex64) * 1e-4
    kc = rng.uniform(0.25, 1.0, (nb, n // 2, n // 2)).astype(np.float32)

    def loss_fn(pgs, rr, dtype):
        bb = {k: v.to(dtype) for k, v in buf.items()}
        return U.training_loss(cfg, pgs[0], bb, rr, e, kc, dtype=dtype)

    return cfg, p, r, loss_fn


def _block_mutant(kind):
    def blk(x, p, buf, name, training, stats):
        y = F.conv2d(x, U._ste_round(p[name + ".w"]), padding=1)
        mean = y.mean(dim=(0, 2, 3))
        var = y.var(dim=(0, 2, 3), unbiased=False)
        if kind == "bn_mean":
            mean = mean.detach()
        if kind == "bn_var":
            var = var.detach()
        z = (y - mean[None, :, None, None]) / torch.sqrt(var[None, :, None, None] + U.EPS)
        z = z * p[name + ".g"][None, :, None, None] + p[name + ".b"][None, :, None, None]
        return U._ste_round(F.leaky_relu(z, U.SLOPE))
    return blk


@pytest.fixture(scope="module")
def measured():
    torch.manual_seed(0)
    cfg, p, r, loss_fn = _setup()
    return cfg, p, r, loss_fn, GB.measure(loss_fn, [p], r)


def test_another_rounding_realisation_passes(measured):
    cfg, p, r, loss_fn, M = measured
    rng = np.random.default_rng(777)
    rp = (r * (1 + 1e-6 * rng.standard_normal(r.shape))).astype(r.dtype)
    _, g = GB.oracle_grads(loss_fn, [p], torch.float32, True, rp)
    flat = np.concatenate([g[0][k] for k in U.param_shapes(cfg)])
    assert not GB.check(flat, cfg, M["g32"][0], M["spread32"][0], "fp32")
    assert not GB.check(flat, cfg, M["gE"][0], M["spreadE"][0], "bf16e")


@pytest.mark.parametrize("kind", ["bn_mean", "bn_var"])
def test_a_dropped_bn_backward_term_fails(measured, monkeypatch, kind):
    cfg, p, r, loss_fn, M = measured
    monkeypatch.setattr(U, "_block", _block_mutant(kind))
    _, g = GB.oracle_grads(loss_fn, [p], torch.float32, True, r)
    flat = np.concatenate([g[0][k] for k in U.param_shapes(cfg)])
    assert GB.check(flat, cfg, M["g32"][0], M["spread32"][0], "fp32")


def test_a_dropped_skip_gradient_fails(measured, monkeypatch):
    """The concat split of the decoder losing the skip half of dx."""
    cfg, p, r, loss_fn, M = measured
    real_cat = torch.cat

    def cat(ts, dim=0):
        # the plain network concatenates only [upsampled, skip] along channels
        if dim == 1 and len(ts) == 2:
            ts = [ts[0], ts[1].detach()]
        return real_cat(ts, dim=dim)

    monkeypatch.setattr(U.torch, "cat", cat)
    _, g = GB.oracle_grads(loss_fn, [p], torch.float32, True, r)
    flat = np.concatenate([g[0][k] for k in U.param_shapes(cfg)])
    assert GB.check(flat, cfg, M["g32"][0], M["spread32"][0], "fp32")
