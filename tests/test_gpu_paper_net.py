"""The paper's own network (section 3.1, eq. 3.1-3.3; cfg.arch = 1) on the
GPU against its CPU oracle, through the C ABI: forward in both BN modes, the
fine-grid wrapper, loss and every parameter gradient (FP32 on both sides, so
the bounds are tight), training, the state files, and the network inside
FGMRES and block FGMRES."""
import numpy as np
import pytest
import torch

from oracle import paper_net_oracle as PN
from paper_2203_11025_amd import inputs

pytestmark = pytest.mark.gpu

WIDTHS = (8, 16, 32)


@pytest.fixture(scope="module")
def mods():
    from paper_2203_11025_amd import helm, train, unet

    assert torch.cuda.is_available()
    unet.lib()
    return helm, unet, train


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(unet, seed, widths=WIDTHS, perturb=True):
    cfg = PN.PaperNetCfg(widths=widths)
    p, buf = PN.init_params(cfg, seed)
    if perturb:
        rng = np.random.default_rng(seed)
        for k in p:
            if k.endswith(".g"):
                p[k] = torch.tensor(rng.uniform(0.5, 1.5, p[k].shape), dtype=torch.float32)
            elif k.endswith(".b") or k.endswith(".bias"):
                p[k] = torch.tensor(rng.normal(0, 0.1, p[k].shape), dtype=torch.float32)
        for k in buf:
            buf[k] = torch.tensor(rng.uniform(-0.2, 0.2, buf[k].shape) if k.endswith(".rm")
                                  else rng.uniform(0.5, 2.0, buf[k].shape), dtype=torch.float32)
    net = unet.UNet(widths=widths, arch=1)
    net.set_params(PN.flatten(cfg, p), torch.cat([buf[k].reshape(-1) for k in PN.buffer_shapes(cfg)]))
    return cfg, p, buf, net


@pytest.mark.parametrize("training", [False, True])
def test_forward_parity(mods, training):
    helm, unet, _ = mods
    cfg, p, buf, net = make(unet, 3)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 32, 32)).astype(np.float32)
    out = net.forward(torch.from_numpy(x), training=training).cpu().numpy()
    ref = PN.forward(cfg, p, buf, torch.from_numpy(x), training=training).detach().numpy()
    assert out.shape == (2, 2, 32, 32)
    assert rel(out, ref) <= 1e-4, rel(out, ref)


def test_fine_grid_wrapper_parity(mods, oracle):
    helm, unet, _ = mods
    cfg, p, buf, net = make(unet, 5)
    n = 64
    kap = inputs.smooth_medium(n, 4.0, seed=2)
    gam = inputs.sponge_gamma(n, width=8)
    h = helm.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), inputs.omega_for_ppw(n), levels=2)
    rng = np.random.default_rng(3)
    r = (rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))).astype(np.complex64)
    e = net.infer(h, torch.from_numpy(r).cuda()).cpu().numpy()
    for b in range(2):
        ref = PN.apply(cfg, p, buf, r[b], kap, gam)
        assert rel(e[b], ref) <= 1e-4, rel(e[b], ref)
    z = net.infer(h, torch.zeros((1, n, n), dtype=torch.complex64, device="cuda")).cpu().numpy()
    assert np.count_nonzero(z) == 0


def test_loss_and_gradient_parity(mods):
    helm, unet, _ = mods
    cfg, p, buf, net = make(unet, 7, perturb=False)
    n, B = 32, 3
    rng = np.random.default_rng(4)
    r = (rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))).astype(np.complex64)
    e = ((rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))) * 1e-4).astype(np.complex64)
    kap = rng.uniform(0.5, 1.0, (n, n)).astype(np.float32)
    gam = rng.uniform(0.0, 0.3, (n, n)).astype(np.float32)
    loss, g = net.loss_grad(torch.from_numpy(r).cuda(), torch.from_numpy(e).cuda(), None,
                            kappa_f=torch.from_numpy(kap).cuda(), gamma_f=torch.from_numpy(gam).cuda())
    pg = {k: v.clone().requires_grad_(True) for k, v in p.items()}
    lo = PN.training_loss(cfg, pg, buf, r, e, kap, gam)
    lo.backward()
    assert abs(loss - lo.item()) <= 1e-4 * abs(lo.item()), (loss, lo.item())
    g = g.cpu().numpy()
    off, worst = 0, 0.0
    for k, shape in PN.param_shapes(cfg).items():
        cnt = int(np.prod(shape))
        a, b = g[off:off + cnt], pg[k].grad.reshape(-1).numpy()
        off += cnt
        rr = rel(a, b)
        cs = float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        worst = max(worst, rr)
        assert rr <= 2e-3 and cs >= 0.99999, (k, rr, cs)
    print(f"worst per-tensor gradient relative error {worst:.2e}")


def test_training_lowers_the_loss_and_state_roundtrip(mods, tmp_path):
    helm, unet, train = mods
    n = 64
    kap = inputs.smooth_medium(n, 4.0, seed=8)
    gam = inputs.sponge_gamma(n, width=8, interior=0.0)
    h = helm.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), inputs.omega_for_ppw(n), levels=2)
    net = unet.UNet(widths=WIDTHS, arch=1)
    net.init(9)
    losses = train.train(net, [h], steps=60, batch=8, lr=1e-3, seed=2, ksteps="random")
    assert all(np.isfinite(losses))
    assert np.mean(losses[-10:]) < 0.9 * np.mean(losses[:10]), (losses[:3], losses[-3:])
    net.save_state(tmp_path / "pn.state")
    other = unet.UNet(widths=WIDTHS, arch=1)
    other.load_state(tmp_path / "pn.state")
    for a, b in zip(net.get_params(), other.get_params()):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    plain = unet.UNet(widths=(32, 64))
    with pytest.raises(helm.HelmError, match="not a state file"):
        plain.load_state(tmp_path / "pn.state")


def test_paper_network_in_fgmres_and_block_fgmres(mods, oracle):
    """M_VU and M_CU with the paper's network (trained briefly) in FGMRES,
    and M_VU in block FGMRES, reach the FP64 tolerance and the exact
    solution.  A briefly trained network is no reliable preconditioner (its
    e0 can be larger than the error), so both forms run with the stall
    safeguard, which may switch a right-hand side to the plain V-cycle.  A
    network whose output layer is zero gives e0 = 0, so M_VU reduces to M_V
    exactly (eq. 3.4): FGMRES and block FGMRES with it must take the plain-SL
    iterations and reach the same solution."""
    helm, unet, train = mods
    n = 64
    kap = inputs.smooth_medium(n, 4.0, seed=10)
    gam = inputs.sponge_gamma(n, width=8, interior=0.0)
    om = inputs.omega_for_ppw(n)
    h = helm.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), om, levels=2)
    net = unet.UNet(widths=WIDTHS, arch=1)
    net.init(11)
    train.train(net, [h], steps=60, batch=8, lr=1e-3, seed=3, ksteps="random")
    b = inputs.point_sources(n, 3, seed=4, margin=8)
    solve = oracle.direct_solver(kap, gam, om)
    for prec in ("unet_defl", "unet_cgc"):
        xs, st, rc = helm.fgmres_solve([h], [torch.from_numpy(b).cuda()], m=10, tol=1e-7, prec=prec, net=net,
                                       maxit=3000, stall_ratio=0.95)
        print(prec, "FGMRES iterations", [s["iterations"] for s in st], "fallbacks", [s["fallback"] for s in st])
        assert rc == 0 and all(s["true_relres"] <= 1e-7 for s in st), prec
        for k in range(3):
            assert rel(xs[0].cpu().numpy()[k], solve(b[k])) <= 1e-5
    cfg = PN.PaperNetCfg(widths=WIDTHS)
    p, buf = PN.init_params(cfg, 5)
    p["out.w"].zero_()
    p["out.bias"].zero_()
    zero = unet.UNet(widths=WIDTHS, arch=1)
    zero.set_params(PN.flatten(cfg, p), torch.cat([buf[k].reshape(-1) for k in PN.buffer_shapes(cfg)]))
    bt = torch.from_numpy(b).cuda()
    xf, sf, rcf = helm.fgmres_solve([h], [bt], m=10, tol=1e-7, prec="sl", maxit=500)
    xz, sz, rcz = helm.fgmres_solve([h], [bt], m=10, tol=1e-7, prec="unet_defl", net=zero, maxit=500)
    assert rcf == 0 and rcz == 0
    assert [s["iterations"] for s in sz] == [s["iterations"] for s in sf]
    assert rel(xz[0].cpu().numpy(), xf[0].cpu().numpy()) <= 1e-6
    xv, sv, rcv = helm.block_fgmres_solve(h, bt, block=3, m=10, tol=1e-7, prec="sl", maxit=500)
    xb, sb, rcb = helm.block_fgmres_solve(h, bt, block=3, m=10, tol=1e-7, prec="unet_defl", net=zero, maxit=500)
    print("block FGMRES iterations", [s["iterations"] for s in sb], "M_V", [s["iterations"] for s in sv])
    assert rcv == 0 and rcb == 0
    assert [s["iterations"] for s in sb] == [s["iterations"] for s in sv]
    for k in range(3):
        assert rel(xb.cpu().numpy()[k], solve(b[k])) <= 1e-5
        assert rel(xb.cpu().numpy()[k], xv.cpu().numpy()[k]) <= 1e-6
