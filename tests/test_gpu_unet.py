"""GPU parity of the U-Net (bf16 MFMA convolutions, FP32 accumulation)
against the FP32 CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import helm_oracle, unet_oracle as U
from paper_2203_11025_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    from paper_2203_11025_amd import unet

    assert torch.cuda.is_available()
    unet.lib()
    return unet


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def make(N, widths, seed, random_stats=True):
    cfg = U.UNetCfg(widths=tuple(widths))
    p, buf = U.init_params(cfg, seed)
    rng = np.random.default_rng(seed + 1)
    # perturb BN affine parameters and running statistics so every term is exercised
    for k in p:
        if k.endswith(".g"):
            p[k] = torch.tensor(rng.uniform(0.5, 1.5, p[k].shape), dtype=torch.float32)
        elif k.endswith(".b") and not k.startswith("head"):
            p[k] = torch.tensor(rng.normal(0, 0.1, p[k].shape), dtype=torch.float32)
        elif k == "head.b":
            p[k] = torch.tensor(rng.normal(0, 0.1, p[k].shape), dtype=torch.float32)
    if random_stats:
        for k in buf:
            buf[k] = torch.tensor(rng.uniform(-0.2, 0.2, buf[k].shape) if k.endswith(".rm")
                                  else rng.uniform(0.5, 2.0, buf[k].shape), dtype=torch.float32)
    net = N.UNet(widths=widths)
    flat = U.flatten(cfg, p)
    bflat = torch.cat([buf[k].reshape(-1) for k in U.buffer_shapes(cfg)])
    net.set_params(flat, bflat)
    return cfg, p, buf, net


# 144: 32-row tiles (images of 128 and more) with a ragged last tile at
# every level
@pytest.mark.parametrize("widths,B,H", [((32, 64), 2, 16), ((32, 64, 128), 1, 40),
                                         ((32, 64, 128, 256), 2, 64), ((32, 64, 128, 256), 2, 144)])
@pytest.mark.parametrize("training", [False, True])
def test_forward_parity(N, widths, B, H, training):
    cfg, p, buf, net = make(N, widths, 3)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((B, 3, H, H)).astype(np.float32)
    x[:, 2] = rng.uniform(0.25, 1.0, (B, H, H))
    out = net.forward(torch.from_numpy(x), training=training).cpu().numpy()
    ref = U.forward(cfg, p, buf, torch.from_numpy(x), training=training).numpy()
    assert rel(out, ref) <= 2e-2, rel(out, ref)
    # the image frame alone (clamped upsampling and zero padding meet
    # there), and the rows and columns at every 16-pixel tile seam
    frame = np.zeros((H, H), bool)
    frame[[0, -1], :] = frame[:, [0, -1]] = True
    seams = np.zeros((H, H), bool)
    seams[15::16, :] = seams[16::16, :] = seams[:, 15::16] = seams[:, 16::16] = True
    for sel in (frame, seams):
        assert rel(out[..., sel], ref[..., sel]) <= 2e-2, rel(out[..., sel], ref[..., sel])


def test_params_roundtrip(N):
    cfg, p, buf, net = make(N, (32, 64), 7)
    pp, bb = net.get_params()
    np.testing.assert_array_equal(pp.cpu().numpy(), U.flatten(cfg, p).numpy())


def test_infer_wrapper_parity(N):
    """e = P s Net(R(h^2 r)/s, kappa_c) on the fine grid of a medium."""
    from paper_2203_11025_amd import helm

    n = 64
    kap = inputs.smooth_medium(n, 4.0, seed=1)
    gam = inputs.sponge_gamma(n, width=8)
    om = inputs.omega_for_ppw(n)
    h = helm.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), om, levels=2)
    cfg, p, buf, net = make(N, (32, 64, 128), 11)
    rng = np.random.default_rng(2)
    r = (rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))).astype(np.complex64)
    r[2] = 0
    e = net.infer(h, torch.from_numpy(r).cuda()).cpu().numpy()
    kc = kap.astype(np.float64)[::2, ::2]
    for b in range(2):
        ref = U.unet_apply(cfg, p, buf, r[b], kc)
        assert rel(e[b], ref) <= 2e-2, rel(e[b], ref)
    assert np.all(e[2] == 0)
    # positive homogeneity (RMS scaling): Net(c r) = c Net(r)
    e2 = net.infer(h, torch.from_numpy(4.0 * r[:1]).cuda()).cpu().numpy()
    assert rel(e2[0], 4.0 * e[0]) <= 1e-5


def _batch(n, nb, seed):
    rng = np.random.default_rng(seed)
    r = (rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))).astype(np.complex64)
    e = (rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))).astype(np.complex64) * 1e-4
    kc = rng.uniform(0.25, 1.0, (nb, n // 2, n // 2)).astype(np.float32)
    return r, e, kc


def _grad_table(cfg, p, g, pg):
    off, rows = 0, []
    for k, shape in U.param_shapes(cfg).items():
        cnt = int(np.prod(shape))
        gg = g[off:off + cnt]
        ref = pg[k].grad.reshape(-1).numpy()
        off += cnt
        cos = float(np.dot(gg, ref) / (np.linalg.norm(gg) * np.linalg.norm(ref) + 1e-30))
        rows.append((k, float(rel(gg, ref)), cos))
    print("\n".join(f"{k:12s} rel={r:.3e} cos={c:.6f}" for k, r, c in rows))
    return rows


@pytest.mark.parametrize("emulate", [True, False])
def test_loss_and_gradient_parity(N, emulate):
    """Loss and every parameter gradient against the oracle's autograd.
    With bf16 emulation in the oracle (same rounding points as the device)
    the agreement is tight; against the plain FP32 oracle the bf16 rounding
    noise grows with the number of BN layers between a tensor and the output,
    so the bound scales with that depth."""
    widths = (32, 64, 128)
    cfg, p, buf, net = make(N, widths, 21, random_stats=False)
    n, nb = 64, 3
    r, e, kc = _batch(n, nb, 4)
    loss, g = net.loss_grad(torch.from_numpy(r).cuda(), torch.from_numpy(e).cuda(),
                            torch.from_numpy(kc).cuda())
    g = g.cpu().numpy()
    pg = {k: v.clone().requires_grad_(True) for k, v in p.items()}
    U.EMULATE_BF16 = emulate
    try:
        lo = U.training_loss(cfg, pg, buf, r, e, kc)
        lo.backward()
    finally:
        U.EMULATE_BF16 = False
    assert abs(loss - lo.item()) <= (2e-3 if emulate else 2e-2) * abs(lo.item()), (loss, lo.item())
    rows = _grad_table(cfg, p, g, pg)
    names = [nm for nm, _, _ in U.layer_specs(cfg)]
    bad = []
    for k, r_, c in rows:
        layer = k.split(".")[0]
        depth = 0 if layer == "head" else len(names) - names.index(layer)
        # emulated: what remains is bf16 rounding decisions that flip under a
        # different FP32 accumulation order, amplified by BN backward; BN bias
        # gradients (batch sums of dy) cancel most, hence the floor
        tol = 0.12 if emulate else 0.03 + 0.025 * (1 + depth)
        ctol = 5e-3 if emulate else 2.5e-3 * (1 + depth)
        if r_ > tol or c < 1 - ctol:
            bad.append((k, r_, c))
    assert not bad, bad


def test_adam_step_closed_form(N):
    """First Adam step from fresh moments: dtheta = -lr g / (|g| + eps) with
    the gradient the library computes for the same batch."""
    widths = (32, 64)
    cfg, p, buf, net = make(N, widths, 31, random_stats=False)
    n, nb = 32, 2
    r, e, kc = _batch(n, nb, 8)
    args = (torch.from_numpy(r).cuda(), torch.from_numpy(e).cuda(), torch.from_numpy(kc).cuda())
    _, g = net.loss_grad(*args)
    p0, _ = net.get_params()
    net.train_step(*args, lr=1e-3)
    p1, b1 = net.get_params()
    g = g.double()
    expect = p0.double() - 1e-3 * g / (g.abs() + 1e-8)
    assert torch.allclose(p1.double(), expect, rtol=0, atol=2e-6)


def test_training_reduces_loss(N):
    """A few Adam steps on a fixed batch lower the loss (sanity of the full
    training step, BN running statistics included)."""
    widths = (32, 64)
    cfg, p, buf, net = make(N, widths, 41, random_stats=False)
    n, nb = 32, 4
    r, e, kc = _batch(n, nb, 9)
    args = (torch.from_numpy(r).cuda(), torch.from_numpy(e).cuda(), torch.from_numpy(kc).cuda())
    losses = [net.train_step(*args, lr=1e-3) for _ in range(30)]
    assert losses[-1] < 0.8 * losses[0], losses[::5]
