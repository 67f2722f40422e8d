"""GPU parity of the encoder-solver pair (section 3.3, eq. 3.5) against the
CPU oracle, through the C ABI: contexts, solver output, joint gradients, the
pair inside FGMRES, and the error paths of a pair used the wrong way."""
import numpy as np
import pytest
import torch

from oracle import unet_oracle as U
from paper_2203_11025_amd import inputs

pytestmark = pytest.mark.gpu

WIDTHS = (32, 64, 128)


@pytest.fixture(scope="module")
def N():
    from paper_2203_11025_amd import unet

    assert torch.cuda.is_available()
    unet.lib()
    return unet


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def make_pair(N, seed, widths=WIDTHS, perturb=True):
    ce = U.UNetCfg(in_ch=1, widths=widths, head=False)
    cs = U.UNetCfg(in_ch=3, widths=widths, context=True)
    pe, be = U.init_params(ce, seed)
    ps, bs = U.init_params(cs, seed + 1)
    rng = np.random.default_rng(seed + 2)
    if perturb:
        for p, b in ((pe, be), (ps, bs)):
            for k in p:
                if k.endswith(".g"):
                    p[k] = torch.tensor(rng.uniform(0.5, 1.5, p[k].shape), dtype=torch.float32)
                elif k.endswith(".b"):
                    p[k] = torch.tensor(rng.normal(0, 0.1, p[k].shape), dtype=torch.float32)
            for k in b:
                b[k] = torch.tensor(rng.uniform(-0.2, 0.2, b[k].shape) if k.endswith(".rm")
                                    else rng.uniform(0.5, 2.0, b[k].shape), dtype=torch.float32)
    enc = N.UNet(widths=widths, head=False)
    sol = N.UNet(widths=widths, context=True)
    for net, cfg, p, b in ((enc, ce, pe, be), (sol, cs, ps, bs)):
        net.set_params(U.flatten(cfg, p), torch.cat([b[k].reshape(-1) for k in U.buffer_shapes(cfg)]))
    return ce, pe, be, cs, ps, bs, enc, sol


@pytest.mark.parametrize("nb,B,H", [(2, 2, 32), (1, 3, 40)])
def test_pair_forward_parity(N, nb, B, H):
    """Per-sample contexts (nb = B) and one shared medium (nb = 1)."""
    ce, pe, be, cs, ps, bs, enc, sol = make_pair(N, 3)
    rng = np.random.default_rng(7)
    kc = rng.uniform(0.25, 1.0, (nb, H, H)).astype(np.float32)
    x = rng.standard_normal((B, 3, H, H)).astype(np.float32)
    N.pair_encode(enc, sol, torch.from_numpy(kc))
    out = sol.forward(torch.from_numpy(x)).cpu().numpy()
    ctx = U.encode(ce, pe, be, kc)
    if nb == 1:
        ctx = [c.expand(B, -1, -1, -1) for c in ctx]
    ref = U.forward(cs, ps, bs, torch.from_numpy(x), ctx=ctx).numpy()
    assert rel(out, ref) <= 2e-2, rel(out, ref)


@pytest.mark.parametrize("H", [64, 144])
def test_shared_context_maps(N, H):
    """With one medium for the whole batch, inference adds each layer's
    convolution over the context from a map computed at encode time.  The
    map path, the path that convolves the context again (taken once the
    weights change without a new encode), and the oracle agree; a new encode
    brings the maps back with the new weights."""
    widths = (32, 64, 128, 256)
    ce, pe, be, cs, ps, bs, enc, sol = make_pair(N, 13, widths=widths)
    rng = np.random.default_rng(17)
    B = 3
    kc = rng.uniform(0.25, 1.0, (1, H, H)).astype(np.float32)
    x = torch.from_numpy(rng.standard_normal((B, 3, H, H)).astype(np.float32))
    N.pair_encode(enc, sol, torch.from_numpy(kc))
    out_map = sol.forward(x).cpu().numpy()
    ctx = [c.expand(B, -1, -1, -1) for c in U.encode(ce, pe, be, kc)]
    ref = U.forward(cs, ps, bs, x, ctx=ctx).numpy()
    assert rel(out_map, ref) <= 2e-2, rel(out_map, ref)
    # same weights set again: the maps are dropped, the context is convolved
    sol.set_params(U.flatten(cs, ps), torch.cat([bs[k].reshape(-1) for k in U.buffer_shapes(cs)]))
    out_cat = sol.forward(x).cpu().numpy()
    assert rel(out_map, out_cat) <= 5e-3, rel(out_map, out_cat)
    # new solver weights, old context: no stale maps
    ps2 = {k: v * 1.1 if k.endswith(".w") else v for k, v in ps.items()}
    sol.set_params(U.flatten(cs, ps2), torch.cat([bs[k].reshape(-1) for k in U.buffer_shapes(cs)]))
    ref2 = U.forward(cs, ps2, bs, x, ctx=ctx).numpy()
    out2 = sol.forward(x).cpu().numpy()
    assert rel(out2, ref2) <= 2e-2, rel(out2, ref2)
    N.pair_encode(enc, sol, torch.from_numpy(kc))
    out3 = sol.forward(x).cpu().numpy()
    assert rel(out3, ref2) <= 2e-2, rel(out3, ref2)
    assert rel(out3, out2) <= 5e-3, rel(out3, out2)


def test_pair_loss_and_gradient_parity(N):
    """Joint loss and both networks' gradients against the oracle's autograd,
    the plain FP32 oracle and the bf16-emulating one, within twice the
    rounding spread the oracle shows on this pair and batch
    (tests/grad_bounds.py).  Encoder gradients come through the whole solver
    first, so their spread is the largest."""
    from tests import grad_bounds as GB

    ce, pe, be, cs, ps, bs, enc, sol = make_pair(N, 11, perturb=False)
    n, nb = 64, 3
    rng = np.random.default_rng(4)
    r = (rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))).astype(np.complex64)
    e = (rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))).astype(np.complex64) * 1e-4
    kc = rng.uniform(0.25, 1.0, (nb, n // 2, n // 2)).astype(np.float32)
    loss, ge, gs = N.pair_loss_grad(enc, sol, torch.from_numpy(r).cuda(), torch.from_numpy(e).cuda(),
                                    torch.from_numpy(kc).cuda())

    def loss_fn(pgs, rr, dtype):
        bbe = {k: v.to(dtype) for k, v in be.items()}
        bbs = {k: v.to(dtype) for k, v in bs.items()}
        return U.pair_training_loss(ce, pgs[0], bbe, cs, pgs[1], bbs, rr, e, kc, dtype=dtype)

    M = GB.measure(loss_fn, [pe, ps], r)
    assert abs(loss - M["lossE"]) <= 2e-3 * abs(M["lossE"]), (loss, M["lossE"])
    assert abs(loss - M["loss32"]) <= 2e-2 * abs(M["loss32"]), (loss, M["loss32"])
    bad = []
    for i, (cfg, g) in enumerate(((ce, ge.cpu().numpy()), (cs, gs.cpu().numpy()))):
        tag = "enc" if i == 0 else "sol"
        bad += GB.check(g, cfg, M["g32"][i], M["spread32"][i], tag + "-fp32")
        bad += GB.check(g, cfg, M["gE"][i], M["spreadE"][i], tag + "-bf16e")
    assert not bad, bad


def test_pair_in_fgmres_matches_oracle_and_converges(N, oracle):
    """M_VU with an encoder-solver: the first preconditioned step against the
    oracle's preconditioner, then a full solve to the FP64 tolerance."""
    from paper_2203_11025_amd import helm

    n = 64
    kap = inputs.smooth_medium(n, 4.0, seed=5)
    gam = inputs.sponge_gamma(n, width=8)
    om = inputs.omega_for_ppw(n)
    h = helm.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), om, levels=2)
    ce, pe, be, cs, ps, bs, enc, sol = make_pair(N, 21)
    kc = kap[::2, ::2].copy()
    N.pair_encode(enc, sol, torch.from_numpy(kc))
    b = inputs.point_sources(n, 1, seed=2, margin=8)
    xs, st, rc = helm.fgmres_solve([h], [torch.from_numpy(b).cuda()], m=5, tol=1e-12, maxit=1,
                                   prec="unet_defl", net=sol)
    H = oracle.Hierarchy(kap, gam, om, 2)
    ctx = U.encode(ce, pe, be, kc)
    f = lambda v: U.precond_defl(H, cs, ps, bs, v, kc.astype(np.float64), ctx=ctx)
    xo, sto = H.fgmres(b[0], m=5, tol=1e-12, maxit=1, prec=f)
    assert rel(xs[0].cpu().numpy()[0], xo) <= 2e-2
    xs, st, rc = helm.fgmres_solve([h], [torch.from_numpy(b).cuda()], m=10, tol=1e-7,
                                   prec="unet_defl", net=sol)
    assert rc == 0 and st[0]["converged"]
    r = b[0].astype(complex) - oracle.apply(kap, gam, om, xs[0].cpu().numpy()[0])
    assert np.linalg.norm(r) / np.linalg.norm(b[0]) <= 1e-7


def test_pair_training_reduces_loss(N):
    ce, pe, be, cs, ps, bs, enc, sol = make_pair(N, 31, widths=(32, 64), perturb=False)
    n, nb = 32, 4
    rng = np.random.default_rng(9)
    r = (rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))).astype(np.complex64)
    e = (rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))).astype(np.complex64) * 1e-4
    kc = rng.uniform(0.25, 1.0, (nb, n // 2, n // 2)).astype(np.float32)
    args = (torch.from_numpy(r).cuda(), torch.from_numpy(e).cuda(), torch.from_numpy(kc).cuda())
    p0e, _ = enc.get_params()
    losses = [N.pair_train_step(enc, sol, *args, lr=1e-3) for _ in range(30)]
    p1e, _ = enc.get_params()
    assert losses[-1] < 0.8 * losses[0], losses[::5]
    assert not torch.equal(p0e, p1e)  # the encoder is trained too


def test_pair_misuse_is_rejected(N):
    """A solver without a context, an encoder used as a network, and a stale
    context after training are errors, not silent results."""
    from paper_2203_11025_amd import helm

    n = 32
    kap = inputs.constant_medium(n, 1.0)
    gam = inputs.sponge_gamma(n, width=4)
    h = helm.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(),
                    inputs.omega_for_ppw(n), levels=2)
    _, _, _, _, _, _, enc, sol = make_pair(N, 41, widths=(32, 64), perturb=False)
    b = torch.from_numpy(inputs.point_sources(n, 1, seed=1, margin=4)).cuda()
    with pytest.raises(helm.HelmError):
        helm.fgmres_solve([h], [b], m=5, tol=1e-7, prec="unet_defl", net=sol)
    with pytest.raises(helm.HelmError):
        enc.forward(torch.zeros(1, 1, 16, 16))
    with pytest.raises(helm.HelmError):
        helm.fgmres_solve([h], [b], m=5, tol=1e-7, prec="unet_defl", net=enc)
    kc = torch.from_numpy(kap[::2, ::2].copy())
    N.pair_encode(enc, sol, kc)
    xs, st, rc = helm.fgmres_solve([h], [b], m=5, tol=1e-7, prec="unet_defl", net=sol)
    assert rc == 0
    rr = torch.zeros(1, n, n, dtype=torch.complex64, device="cuda")
    N.pair_train_step(enc, sol, rr + 1, rr + 1e-4, kc[None].cuda())
    with pytest.raises(helm.HelmError):
        helm.fgmres_solve([h], [b], m=5, tol=1e-7, prec="unet_defl", net=sol)


def test_every_tuner_candidate_at_the_1024_workload_network_grid(N):
    """The network of the 1024^2 workload runs on the 512^2 coarse grid with
    one shared medium (context maps, the fused x2 upsampling of the first
    decoder convolution).  Every launch shape the autotuner can pick is
    forced on every convolution and checked against the FP32 oracle."""
    from paper_2203_11025_amd import helm

    widths = (32, 64, 128, 256)
    ce, pe, be, cs, ps, bs, enc, sol = make_pair(N, 51, widths=widths)
    rng = np.random.default_rng(52)
    nc, B = 512, 2
    kc = rng.uniform(0.25, 1.0, (1, nc, nc)).astype(np.float32)
    x = rng.standard_normal((B, 3, nc, nc)).astype(np.float32)
    x[:, 2] = kc[0]
    ctx = [c.expand(B, -1, -1, -1) for c in U.encode(ce, pe, be, kc)]
    ref = U.forward(cs, ps, bs, torch.from_numpy(x), ctx=ctx).numpy()
    outs = {}
    try:
        for kind in (0, 1):
            for mf in (2, 4):
                for per_cu in (1, 2, 4, 8):
                    helm.autotune_force(kind, mf, per_cu)
                    N.pair_encode(enc, sol, torch.from_numpy(kc))
                    outs[(kind, mf, per_cu)] = sol.forward(torch.from_numpy(x)).cpu().numpy()
    finally:
        helm.autotune_force(-1)
    for cand, out in outs.items():
        r_ = rel(out, ref)
        print(f"candidate {cand}: rel {r_:.3e}")
        assert r_ <= 2e-2, (cand, r_)
