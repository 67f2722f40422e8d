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


# ------------------------------------------------------------------ the
# compositions of Algorithm 2 and eq. 3.4, the input scaling, the loss of
# eq. 3.7, inference BN and running statistics, Adam beyond step 1, and the
# encoder's outputs (eq. 3.5)

def _const_hier(oracle, n, kappa, gamma, levels=2):
    from paper_2203_11025_amd import inputs
    kap = np.full((n, n), kappa)
    gam = np.full((n, n), gamma)
    om = inputs.omega_for_ppw(n)
    return kap, gam, om, oracle.Hierarchy(kap, gam, om, levels)


def _spsolve_fn(kap, gam, om):
    import scipy.sparse.linalg as spl
    from tests import pins
    A = pins.helmholtz_matrix(kap, gam, om)
    n = kap.shape[0]
    return lambda v: spl.spsolve(A, np.asarray(v, complex).ravel()).reshape(n, n)


def test_defl_keeps_an_exact_e0(oracle):
    """Eq. 3.4 is a deflation: an exact error estimate e0 = A^-1 r leaves a
    zero residual, and the V-cycle adds nothing."""
    n = 32
    from paper_2203_11025_amd import inputs
    kap = inputs.smooth_medium(n, 3.0, seed=5).astype(np.float64)
    gam = inputs.sponge_gamma(n, width=4).astype(np.float64)
    om = inputs.omega_for_ppw(n)
    H = oracle.Hierarchy(kap, gam, om, 2)
    rng = np.random.default_rng(1)
    r = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    exact = _spsolve_fn(kap, gam, om)
    z = U.defl_compose(H, exact, r)
    np.testing.assert_allclose(z, exact(r), rtol=0, atol=1e-9 * np.abs(exact(r)).max())
    # a zero estimate leaves the plain V-cycle
    np.testing.assert_allclose(U.defl_compose(H, lambda v: 0 * v, r), H.vcycle(r), atol=1e-14)
    # an estimate that is off by d is corrected by V(0, -A d), not by V(0, r)
    d = 1e-3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    z2 = U.defl_compose(H, lambda v: exact(v) + d, r)
    np.testing.assert_allclose(z2, exact(r) + d - H.vcycle(oracle.apply(kap, gam, om, d)),
                               atol=1e-9 * np.abs(exact(r)).max())


@pytest.mark.parametrize("k,l", [(1, 1), (3, 5), (20, 9)])
def test_cgc_zero_network_is_two_jacobi_sweeps_on_an_eigenmode(oracle, k, l):
    """Algorithm 2 with a zero correction is two damped Jacobi sweeps on A
    from zero.  For a constant medium and constant attenuation the diagonal
    d = 4/h^2 - omega^2 kappa^2 (1 - i gamma) is constant and a DST-I mode phi
    with eigenvalue lambda maps to (w/d)(2 - w lambda/d) phi."""
    from tests import pins
    n, kappa, gamma, w = 24, 0.7, 0.05, 0.8
    kap, gam, om, H = _const_hier(oracle, n, kappa, gamma)
    phi = pins.dst_mode(n, k, l).astype(complex)
    lam = pins.dst_eigenvalue(n, k, l, kappa, gamma, om)
    d = 4.0 * n * n - om ** 2 * kappa ** 2 * (1 - 1j * gamma)
    z = U.cgc_compose(H, lambda v: 0 * v, phi, weight=w)
    np.testing.assert_allclose(z, (w / d) * (2 - w * lam / d) * phi, atol=1e-12 * np.abs(z).max())


def test_cgc_exact_correction_is_an_exact_solve(oracle):
    """With the exact coarse correction net_fn = A^-1, the middle step of
    Algorithm 2 lands on A^-1 r (it corrects the residual left by the first
    sweep), and the last sweep keeps it."""
    n = 32
    from paper_2203_11025_amd import inputs
    kap = inputs.smooth_medium(n, 3.0, seed=6).astype(np.float64)
    gam = inputs.sponge_gamma(n, width=4).astype(np.float64)
    om = inputs.omega_for_ppw(n)
    H = oracle.Hierarchy(kap, gam, om, 2)
    rng = np.random.default_rng(2)
    r = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    exact = _spsolve_fn(kap, gam, om)
    z = U.cgc_compose(H, exact, r)
    np.testing.assert_allclose(z, exact(r), atol=1e-9 * np.abs(exact(r)).max())


def test_net_input_scale_is_the_rms_of_the_restricted_residual():
    """A residual that lives on the even-even points only restricts to a
    quarter of those values (full weighting puts 1/2 x 1/2 on the centre), so
    s = (h^2 / 4) sqrt(mean |r(2I, 2J)|^2) over the n/2 x n/2 coarse grid."""
    n = 16
    rng = np.random.default_rng(3)
    vals = rng.standard_normal((n // 2, n // 2)) + 1j * rng.standard_normal((n // 2, n // 2))
    vals[0, 0] = 9.0  # far from the mean of |.|: a mean-abs scale would differ
    r = np.zeros((n, n), complex)
    r[::2, ::2] = vals
    kc = rng.uniform(0.25, 1.0, (n // 2, n // 2))
    inp, s = U.net_input(r, kc, n)
    s_expect = (1.0 / n ** 2) / 4.0 * np.sqrt(np.mean(np.abs(vals) ** 2))
    assert abs(s - s_expect) <= 1e-14 * s_expect
    np.testing.assert_allclose(inp[0] + 1j * inp[1], (vals / n ** 2 / 4.0) / s_expect, rtol=1e-12)
    np.testing.assert_array_equal(inp[2], kc)


def test_training_loss_closed_form_for_a_constant_network():
    """All convolution weights and BN biases zero: every activation is zero,
    so the network returns its head bias c everywhere on the coarse grid.
    Bilinear prolongation of a constant is c inside and c/2 on the last fine
    row and column (their far neighbour is the zero ghost), c/4 in that
    corner.  With residuals on the even-even points s_b is known (previous
    test), and the loss is mean_b sum_ij |c q_i q_j - e_b(i,j)/s_b|^2 / n^2."""
    cfg = U.UNetCfg(widths=(4, 8))
    p, buf = U.init_params(cfg, 1, dtype=torch.float64)
    for k in p:
        if k != "head.b" and not k.endswith(".g"):
            p[k] = torch.zeros_like(p[k])
    c = np.array([0.3, -1.7])
    p["head.b"] = torch.tensor(c)
    n, B = 16, 3
    rng = np.random.default_rng(4)
    r = np.zeros((B, n, n), complex)
    svals = []
    for b in range(B):
        vals = (b + 1) * (rng.standard_normal((n // 2, n // 2)) + 1j * rng.standard_normal((n // 2, n // 2)))
        r[b, ::2, ::2] = vals
        svals.append(np.sqrt(np.mean(np.abs(vals) ** 2)) / (4.0 * n * n))
    e = rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))
    kc = rng.uniform(0.25, 1.0, (B, n // 2, n // 2))
    q = np.ones(n)
    q[-1] = 0.5
    pc = (c[0] + 1j * c[1]) * np.outer(q, q)
    expect = np.mean([np.sum(np.abs(pc - e[b] / svals[b]) ** 2) / n ** 2 for b in range(B)])
    got = U.training_loss(cfg, p, buf, r, e, kc, dtype=torch.float64).item()
    assert abs(got - expect) <= 1e-12 * expect, (got, expect)


def test_inference_bn_and_running_statistics_match_torch_batchnorm():
    """BN of a block in inference mode and the running-statistics update
    (momentum 0.1, unbiased running variance) against torch.nn.BatchNorm2d,
    over several updates from the initial statistics."""
    torch.manual_seed(0)
    cfg = U.UNetCfg(widths=(4, 8))
    p, buf = U.init_params(cfg, 2, dtype=torch.float64)
    p["enc0a.g"] = torch.tensor([0.5, 1.5, 1.0, 2.0], dtype=torch.float64)
    p["enc0a.b"] = torch.tensor([0.1, -0.2, 0.0, 0.3], dtype=torch.float64)
    bn = torch.nn.BatchNorm2d(4, eps=U.EPS, momentum=U.MOMENTUM).double()
    with torch.no_grad():
        bn.weight.copy_(p["enc0a.g"])
        bn.bias.copy_(p["enc0a.b"])
    for step in range(4):
        x = torch.randn(3, 3, 6, 6, dtype=torch.float64) * (step + 1)
        y = F.conv2d(x, p["enc0a.w"], padding=1)
        stats = {}
        a_train = U._block(x, p, buf, "enc0a", True, stats)
        U.update_running_stats(buf, {"enc0a": stats["enc0a"]}, y.shape[0] * y.shape[2] * y.shape[3])
        bn.train()
        ref_train = F.leaky_relu(bn(y), U.SLOPE)
        np.testing.assert_allclose(a_train.detach().numpy(), ref_train.detach().numpy(), atol=1e-12)
        np.testing.assert_allclose(buf["enc0a.rm"].numpy(), bn.running_mean.numpy(), atol=1e-14)
        np.testing.assert_allclose(buf["enc0a.rv"].numpy(), bn.running_var.numpy(), rtol=1e-13)
        bn.eval()
        x2 = torch.randn(2, 3, 6, 6, dtype=torch.float64)
        a_inf = U._block(x2, p, buf, "enc0a", False, None)
        ref_inf = F.leaky_relu(bn(F.conv2d(x2, p["enc0a.w"], padding=1)), U.SLOPE)
        np.testing.assert_allclose(a_inf.detach().numpy(), ref_inf.detach().numpy(), atol=1e-12)


def test_adam_matches_torch_adam_over_several_steps():
    """Bias-corrected Adam without weight decay against torch.optim.Adam for
    five steps with changing gradients (steps beyond the first exercise the
    moment recursions and the bias corrections)."""
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(7)
    ours = {"a": torch.tensor(p0)}
    m = {"a": torch.zeros(7, dtype=torch.float64)}
    v = {"a": torch.zeros(7, dtype=torch.float64)}
    ref = torch.nn.Parameter(torch.tensor(p0))
    opt = torch.optim.Adam([ref], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = torch.tensor(rng.standard_normal(7) * 10.0 ** rng.integers(-4, 2, 7))
        ours, m, v = U.adam_step(ours, {"a": g}, m, v, step, lr=1e-3)
        ref.grad = g.clone()
        opt.step()
        np.testing.assert_allclose(ours["a"].numpy(), ref.detach().numpy(), rtol=0, atol=1e-15)


def test_encoder_contexts_are_the_up_path_outputs():
    """Eq. 3.5: f^(l) is the encoder's output on its way up at level l.  So
    the level-0 context depends on the deeper levels' weights (it would not
    if it were the level-0 down-path output), and the deepest context is the
    bottleneck, which the up-path weights do not touch."""
    ce = U.UNetCfg(in_ch=1, widths=(4, 8, 16), head=False)
    p, buf = U.init_params(ce, 3, dtype=torch.float64)
    kc = np.random.default_rng(6).uniform(0.25, 1.0, (1, 16, 16))
    base = U.encode(ce, p, buf, kc, dtype=torch.float64)
    deep = {k: (v * 1.3 if k == "enc2b.w" else v) for k, v in p.items()}
    c_deep = U.encode(ce, deep, buf, kc, dtype=torch.float64)
    assert not np.allclose(c_deep[0].numpy(), base[0].numpy())
    up = {k: (v * 1.3 if k == "dec0b.w" else v) for k, v in p.items()}
    c_up = U.encode(ce, up, buf, kc, dtype=torch.float64)
    np.testing.assert_array_equal(c_up[2].numpy(), base[2].numpy())
    np.testing.assert_array_equal(c_up[1].numpy(), base[1].numpy())
    assert not np.allclose(c_up[0].numpy(), base[0].numpy())
    # the level-0 context is the output of dec0b (not of enc0b)
    stats = {}
    outs = U.forward(ce, p, buf, torch.tensor(kc)[:, None], training=False)
    np.testing.assert_array_equal(outs[0].numpy(), base[0].numpy())


def test_training_loss_gradients_match_central_differences():
    """The full training loss (input scaling, network, prolongation, the
    /n^2 and batch mean of eq. 3.7) differentiated by autograd against FP64
    central differences, a few weights in every tensor of a network with the
    widths the device gradient tests use."""
    cfg = U.UNetCfg(widths=(32, 64, 128))
    p, buf = U.init_params(cfg, 8, dtype=torch.float64)
    n, B = 32, 2
    rng = np.random.default_rng(9)
    r = rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))
    e = 1e-4 * (rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n)))
    kc = rng.uniform(0.25, 1.0, (B, n // 2, n // 2))
    pg = {k: v.clone().requires_grad_(True) for k, v in p.items()}
    U.training_loss(cfg, pg, buf, r, e, kc, dtype=torch.float64).backward()
    h = 1e-5
    torch.set_grad_enabled(False)
    try:
        for k, v in p.items():
            flat = v.reshape(-1)
            for idx in rng.choice(flat.numel(), size=min(2, flat.numel()), replace=False):
                old = flat[idx].item()
                flat[idx] = old + h
                lp = U.training_loss(cfg, p, buf, r, e, kc, dtype=torch.float64).item()
                flat[idx] = old - h
                lm = U.training_loss(cfg, p, buf, r, e, kc, dtype=torch.float64).item()
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                ad = pg[k].grad.reshape(-1)[idx].item()
                scale = max(abs(fd), 1e-3 * pg[k].grad.abs().max().item())
                assert abs(fd - ad) <= 1e-5 * scale, (k, idx, fd, ad)
    finally:
        torch.set_grad_enabled(True)
