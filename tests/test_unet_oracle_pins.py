"""Pins of the U-Net oracle: explicit loops for the layer primitives, closed
forms for bilinear upsampling and the first Adam step, FP64 central finite
differences for the gradients, and the homogeneity the RMS scaling implies."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import helm_oracle, unet_oracle as U

TINY = U.UNetCfg(in_ch=3, out_ch=2, widths=(4, 8))


def test_config_network_parameter_count():
    """4 levels 32/64/128/256, input (Re r, Im r, kappa): 1,945,506 parameters
    (convolutions + BN affine + 1x1 head)."""
    cfg = U.UNetCfg()
    conv = sum(int(np.prod(s)) for k, s in U.param_shapes(cfg).items() if k.endswith(".w"))
    head_b = 2
    assert conv + head_b == 1_945_506
    ctxcfg = U.UNetCfg(context=True)
    assert [s[1] for s in U.layer_specs(ctxcfg)][:2] == [35, 32]


def test_conv_matches_explicit_loop():
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.standard_normal((1, 2, 5, 6)))
    w = torch.tensor(rng.standard_normal((3, 2, 3, 3)))
    y = F.conv2d(x, w, padding=1).numpy()
    xp = np.pad(x.numpy(), ((0, 0), (0, 0), (1, 1), (1, 1)))
    ref = np.zeros((1, 3, 5, 6))
    for co in range(3):
        for i in range(5):
            for j in range(6):
                ref[0, co, i, j] = np.sum(xp[0, :, i:i + 3, j:j + 3] * w.numpy()[co])
    np.testing.assert_allclose(y, ref, atol=1e-12)


def test_bilinear_up_closed_form():
    """Half-pixel centres: [a, b] -> [a, 3a/4 + b/4, a/4 + 3b/4, b]."""
    x = torch.tensor([[[[1.0, 5.0]]]], dtype=torch.float64).repeat(1, 1, 2, 1)
    y = U.up2(x)[0, 0, 0].numpy()
    np.testing.assert_allclose(y, [1.0, 2.0, 4.0, 5.0], atol=1e-14)


def test_batchnorm_training_statistics():
    torch.manual_seed(1)
    p, buf = U.init_params(TINY, 3, dtype=torch.float64)
    x = torch.randn(4, 3, 8, 8, dtype=torch.float64)
    stats = {}
    y = F.conv2d(x, p["enc0a.w"], padding=1)
    U._block(x, p, buf, "enc0a", True, stats)
    mean, var = stats["enc0a"]
    np.testing.assert_allclose(mean.numpy(), y.numpy().mean(axis=(0, 2, 3)), atol=1e-12)
    np.testing.assert_allclose(var.numpy(), y.numpy().var(axis=(0, 2, 3)), atol=1e-12)
    z = (y - mean[None, :, None, None]) / torch.sqrt(var[None, :, None, None] + U.EPS)
    np.testing.assert_allclose(z.mean(dim=(0, 2, 3)).numpy(), 0.0, atol=1e-12)
    np.testing.assert_allclose(z.var(dim=(0, 2, 3), unbiased=False).numpy(), 1.0, atol=1e-4)


def test_gradients_match_central_differences():
    """Training-mode loss gradients (autograd) against FP64 central
    differences on a tiny network, every parameter tensor sampled."""
    p, buf = U.init_params(TINY, 5, dtype=torch.float64)
    rng = np.random.default_rng(7)
    x = torch.tensor(rng.standard_normal((2, 3, 8, 8)))
    probe = torch.tensor(rng.standard_normal((2, 2, 8, 8)))

    def loss_of(pp):
        return (U.forward(TINY, pp, buf, x, training=True) * probe).sum()

    pg = {k: v.clone().requires_grad_(True) for k, v in p.items()}
    loss_of(pg).backward()
    h = 1e-6
    for k, v in p.items():
        flat = v.reshape(-1)
        for idx in rng.choice(flat.numel(), size=min(3, flat.numel()), replace=False):
            pp = {kk: vv.clone() for kk, vv in p.items()}
            pm = {kk: vv.clone() for kk, vv in p.items()}
            pp[k].reshape(-1)[idx] += h
            pm[k].reshape(-1)[idx] -= h
            fd = (loss_of(pp) - loss_of(pm)).item() / (2 * h)
            ad = pg[k].grad.reshape(-1)[idx].item()
            assert abs(fd - ad) <= 1e-5 * max(1.0, abs(fd)), (k, idx, fd, ad)


def test_adam_first_step_closed_form():
    p = {"a": torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64)}
    g = {"a": torch.tensor([0.3, -1e-3, 0.0], dtype=torch.float64)}
    m = {"a": torch.zeros(3, dtype=torch.float64)}
    v = {"a": torch.zeros(3, dtype=torch.float64)}
    new, _, _ = U.adam_step(dict(p), g, m, v, 1, lr=1e-3)
    expect = p["a"] - 1e-3 * g["a"] / (g["a"].abs() + 1e-8)
    np.testing.assert_allclose(new["a"].numpy(), expect.numpy(), atol=1e-15)


def test_prolong_torch_matches_oracle_prolongation():
    rng = np.random.default_rng(3)
    ec = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    a = U.prolong_torch(torch.tensor(ec)).numpy()
    np.testing.assert_allclose(a, helm_oracle.prolong(ec), atol=1e-14)


def test_wrapper_positively_homogeneous_and_zero():
    cfg = U.UNetCfg(widths=(4, 8, 16))
    p, buf = U.init_params(cfg, 11, dtype=torch.float64)
    n = 32
    rng = np.random.default_rng(4)
    r = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    kc = rng.uniform(0.25, 1.0, (n // 2, n // 2))
    e1 = U.unet_apply(cfg, p, buf, r, kc, dtype=torch.float64)
    e2 = U.unet_apply(cfg, p, buf, 7.5 * r, kc, dtype=torch.float64)
    np.testing.assert_allclose(e2, 7.5 * e1, rtol=1e-10, atol=1e-12 * np.abs(e2).max())
    assert np.all(U.unet_apply(cfg, p, buf, 0 * r, kc) == 0)


def test_maxpool_first_maximum_gradient():
    """Ties route the gradient to the first maximum in (0,0),(0,1),(1,0),(1,1) order."""
    x = torch.tensor([[[[1.0, 3.0], [3.0, 2.0]]]], requires_grad=True)
    F.max_pool2d(x, 2).sum().backward()
    np.testing.assert_array_equal(x.grad.numpy()[0, 0], [[0.0, 1.0], [0.0, 0.0]])


def test_training_triple_residual_and_one_step_minimiser(oracle):
    """A e = r, and x~ = x - e is the one-step FGMRES(SL) iterate from zero."""
    n = 32
    kap = np.full((n, n), 0.8)
    kap[10:20, 5:25] = 0.5
    from paper_2203_11025_amd import inputs
    gam = inputs.sponge_gamma(n, width=4).astype(np.float64)
    om = inputs.omega_for_ppw(n)
    H = oracle.Hierarchy(kap, gam, om, 2)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    r, e = U.training_triple(H, x)
    np.testing.assert_allclose(oracle.apply(kap, gam, om, e), r, atol=1e-9 * np.abs(r).max())
    b = oracle.apply(kap, gam, om, x)
    x1, st = H.fgmres(b, m=5, tol=1e-14, maxit=1)
    np.testing.assert_allclose(x - e, x1, atol=1e-10 * np.abs(x1).max())


TINY_ENC = U.UNetCfg(in_ch=1, widths=(4, 8), head=False)
TINY_SOL = U.UNetCfg(in_ch=3, widths=(4, 8), context=True)


def test_pair_context_shapes_and_zero_context_weights():
    """The encoder yields one context per level (w_l channels at the level's
    resolution); a solver whose context weight columns are zero computes the
    plain network with the remaining columns (the context is the last input
    of enc{l}a and dec{l}a)."""
    pe, be = U.init_params(TINY_ENC, 1, dtype=torch.float64)
    ps, bs = U.init_params(TINY_SOL, 2, dtype=torch.float64)
    rng = np.random.default_rng(3)
    kc = rng.uniform(0.25, 1.0, (2, 8, 8))
    ctx = U.encode(TINY_ENC, pe, be, kc, dtype=torch.float64)
    assert [tuple(c.shape) for c in ctx] == [(2, 4, 8, 8), (2, 8, 4, 4)]
    plain = U.UNetCfg(in_ch=3, widths=(4, 8))
    pp = {}
    for k, v in ps.items():
        pp[k] = v.clone()
    for name, cin, cout in U.layer_specs(TINY_SOL):
        if name.endswith("a"):
            lev = int(name[3])
            wctx = TINY_SOL.widths[lev]
            ps[name + ".w"][:, cin - wctx:] = 0
            pp[name + ".w"] = ps[name + ".w"][:, :cin - wctx].clone()
    x = torch.tensor(rng.standard_normal((2, 3, 8, 8)))
    y_pair = U.forward(TINY_SOL, ps, bs, x, ctx=ctx)
    y_plain = U.forward(plain, pp, bs, x)
    np.testing.assert_allclose(y_pair.numpy(), y_plain.numpy(), atol=1e-12)


def test_pair_gradients_match_central_differences():
    """Joint encoder-solver gradients (autograd through the contexts) against
    FP64 central differences, sampled in every parameter tensor of both."""
    pe, be = U.init_params(TINY_ENC, 4, dtype=torch.float64)
    ps, bs = U.init_params(TINY_SOL, 5, dtype=torch.float64)
    rng = np.random.default_rng(8)
    kc = rng.uniform(0.25, 1.0, (2, 8, 8))
    x = torch.tensor(rng.standard_normal((2, 3, 8, 8)))
    probe = torch.tensor(rng.standard_normal((2, 2, 8, 8)))

    def loss_of(a, b):
        ctx = U.encode(TINY_ENC, a, be, kc, training=True, dtype=torch.float64)
        return (U.forward(TINY_SOL, b, bs, x, ctx=ctx, training=True) * probe).sum()

    ga = {k: v.clone().requires_grad_(True) for k, v in pe.items()}
    gb = {k: v.clone().requires_grad_(True) for k, v in ps.items()}
    loss_of(ga, gb).backward()
    h = 1e-6
    for which, base, grads in (("enc", pe, ga), ("sol", ps, gb)):
        for k, v in base.items():
            flat = v.reshape(-1)
            for idx in rng.choice(flat.numel(), size=min(2, flat.numel()), replace=False):
                plus = {kk: vv.clone() for kk, vv in base.items()}
                minus = {kk: vv.clone() for kk, vv in base.items()}
                plus[k].reshape(-1)[idx] += h
                minus[k].reshape(-1)[idx] -= h
                if which == "enc":
                    fd = (loss_of(plus, ps) - loss_of(minus, ps)).item() / (2 * h)
                else:
                    fd = (loss_of(pe, plus) - loss_of(pe, minus)).item() / (2 * h)
                ad = grads[k].grad.reshape(-1)[idx].item()
                assert abs(fd - ad) <= 1e-5 * max(1.0, abs(fd)), (which, k, idx, fd, ad)
