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


def test_loss_and_gradient_parity(N):
    """Loss and every parameter gradient of the training loss (eq. 3.7)
    against the oracle's autograd, both the plain FP32 oracle and the oracle
    with bf16 rounding at the device's rounding points.  The per-tensor
    bounds come from the rounding spread the oracle itself shows on this
    network and batch (tests/grad_bounds.py): bf16 rounding decisions flip
    under another summation order and every BN backward amplifies them, so
    the device must lie within twice that measured spread."""
    from tests import grad_bounds as GB

    widths = (32, 64, 128)
    cfg, p, buf, net = make(N, widths, 21, random_stats=False)
    n, nb = 64, 3
    r, e, kc = _batch(n, nb, 4)
    loss, g = net.loss_grad(torch.from_numpy(r).cuda(), torch.from_numpy(e).cuda(),
                            torch.from_numpy(kc).cuda())
    g = g.cpu().numpy()

    def loss_fn(pgs, rr, dtype):
        bb = {k: v.to(dtype) for k, v in buf.items()}
        return U.training_loss(cfg, pgs[0], bb, rr, e, kc, dtype=dtype)

    M = GB.measure(loss_fn, [p], r)
    assert abs(loss - M["lossE"]) <= 2e-3 * abs(M["lossE"]), (loss, M["lossE"])
    assert abs(loss - M["loss32"]) <= 2e-2 * abs(M["loss32"]), (loss, M["loss32"])
    bad = GB.check(g, cfg, M["g32"][0], M["spread32"][0], "fp32")
    bad += GB.check(g, cfg, M["gE"][0], M["spreadE"][0], "bf16e")
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


CANDIDATES = [(kind, mf, per_cu) for kind in (0, 1) for mf in (2, 4) for per_cu in (1, 8)]


@pytest.mark.parametrize("training", [False, True])
def test_every_tuner_candidate_matches_oracle(N, training):
    """Each launch shape the autotuner can pick (both kernels, both tile
    heights, the fewest and the most workgroups) forced on every
    convolution of the configured 4-level network on a ragged 144^2 image;
    each against the FP32 oracle at the network bar."""
    from paper_2203_11025_amd import helm

    cfg, p, buf, net = make(N, (32, 64, 128, 256), 5)
    rng = np.random.default_rng(6)
    H, B = 144, 2
    x = rng.standard_normal((B, 3, H, H)).astype(np.float32)
    x[:, 2] = rng.uniform(0.25, 1.0, (B, H, H))
    ref = U.forward(cfg, p, buf, torch.from_numpy(x), training=training).numpy()
    outs = {}
    try:
        for cand in CANDIDATES:
            helm.autotune_force(*cand)
            outs[cand] = net.forward(torch.from_numpy(x), training=training).cpu().numpy()
    finally:
        helm.autotune_force(-1)
    for cand, out in outs.items():
        assert rel(out, ref) <= 2e-2, (cand, rel(out, ref))
    # the workgroup count only changes which workgroup walks which tiles:
    # the outputs of one kernel and tile height are identical
    for kind in (0, 1):
        for mf in (2, 4):
            assert np.array_equal(outs[(kind, mf, 1)], outs[(kind, mf, 8)]), (kind, mf)
    spread = max(float(np.abs(o - outs[CANDIDATES[0]]).max()) for o in outs.values())
    print(f"largest difference between candidates: {spread:.3e}")
