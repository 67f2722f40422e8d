"""Batching machinery on the GPU: restart cycles captured into HIP graphs
(replayed several times, eager work between the replays, every result
checked against the eager solve) and uneven multi-problem batches solved
concurrently in one call, checked against one-by-one solves and the FP64
oracle residual."""
import numpy as np
import pytest
import torch

from oracle import unet_oracle as U
from paper_2203_11025_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2203_11025_amd import helm

    assert torch.cuda.is_available()
    helm.lib()
    return helm


def handle(H, kap, gam, n, levels=0):
    return H.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), inputs.omega_for_ppw(n),
                    levels=levels)


def true_relres(oracle, kap, gam, n, b, x):
    r = b.astype(complex) - oracle.apply(kap, gam, inputs.omega_for_ppw(n), x)
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_graph_replays_match_eager_sl(H, oracle):
    n = 128
    kap = inputs.smooth_medium(n, 8.0, seed=5)
    gam = inputs.sponge_gamma(n, width=16)
    h = handle(H, kap, gam, n, levels=3)
    b = torch.from_numpy(inputs.point_sources(n, 3, seed=9)).cuda()
    x_e, st_e, rc = H.fgmres_solve([h], [b], m=10, tol=1e-7)
    assert rc == 0
    ref = x_e[0].cpu().numpy()
    xg = torch.empty(b.shape, dtype=torch.complex128, device="cuda")  # same buffers: cached graph
    for rep in range(3):
        xs, st, rc = H.fgmres_solve([h], [b], m=10, tol=1e-7, graph=True, xs=[xg])
        torch.cuda.synchronize()
        assert rc == 0
        got = xs[0].cpu().numpy()
        assert [s["iterations"] for s in st] == [s["iterations"] for s in st_e]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        # eager work between the replays
        x2, _, _ = H.fgmres_solve([h], [b[:1]], m=10, tol=1e-7)
        torch.cuda.synchronize()
    for k in range(3):
        assert true_relres(oracle, kap, gam, n, b[k].cpu().numpy(), got[k]) <= 1e-7


def test_graph_replays_match_eager_network(H, oracle):
    """M_VU with the network: the graph holds the network's kernels too, and
    is captured again when the number of right-hand sides using it changes."""
    from paper_2203_11025_amd import unet

    n = 64
    kap = inputs.smooth_medium(n, 4.0, seed=6)
    gam = inputs.sponge_gamma(n, width=8)
    h = handle(H, kap, gam, n, levels=2)
    cfg = U.UNetCfg(widths=(32, 64, 128))
    p, buf = U.init_params(cfg, 3)
    net = unet.UNet(widths=(32, 64, 128))
    net.set_params(U.flatten(cfg, p), torch.cat([buf[k].reshape(-1) for k in U.buffer_shapes(cfg)]))
    b = torch.from_numpy(inputs.point_sources(n, 2, seed=4, margin=8)).cuda()
    xe, ste, rc = H.fgmres_solve([h], [b], m=8, tol=1e-7, prec="unet_defl", net=net)
    assert rc == 0
    ref = xe[0].cpu().numpy()
    for rep in range(2):
        xs, st, rc = H.fgmres_solve([h], [b], m=8, tol=1e-7, prec="unet_defl", net=net, graph=True)
        torch.cuda.synchronize()
        assert rc == 0
        assert [s["iterations"] for s in st] == [s["iterations"] for s in ste]
        np.testing.assert_allclose(xs[0].cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        net.forward(torch.zeros(1, 3, 32, 32))  # eager network work in between
        torch.cuda.synchronize()


def test_uneven_batch_concurrent_matches_one_by_one(H, oracle):
    """Six layered media of three grid sizes in one call (concurrent streams,
    graphs on), against solving each problem alone."""
    sizes = [64, 128, 256, 64, 128, 256]
    probs, rhs, meta = [], [], []
    for k, n in enumerate(sizes):
        kap = inputs.layered_medium(n, seed=100 + k)
        gam = inputs.sponge_gamma(n, width=min(16, n // 8))
        probs.append(handle(H, kap, gam, n))
        rhs.append(torch.from_numpy(inputs.point_sources(n, 2, seed=200 + k, margin=min(16, n // 8))).cuda())
        meta.append((kap, gam, n))
    xs, st, rc = H.fgmres_solve(probs, rhs, m=20, tol=1e-7, graph=True)
    torch.cuda.synchronize()
    assert rc == 0 and len(st) == 12
    for k in range(len(sizes)):
        x1, st1, rc1 = H.fgmres_solve([probs[k]], [rhs[k]], m=20, tol=1e-7)
        assert rc1 == 0
        assert [s["iterations"] for s in st1] == [s["iterations"] for s in st[2 * k:2 * k + 2]]
        ref = x1[0].cpu().numpy()
        np.testing.assert_allclose(xs[k].cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        kap, gam, n = meta[k]
        for j in range(2):
            assert true_relres(oracle, kap, gam, n, rhs[k][j].cpu().numpy(), ref[j]) <= 1e-7


def test_same_handle_twice_in_one_call(H):
    n = 64
    kap = inputs.smooth_medium(n, 4.0, seed=8)
    gam = inputs.sponge_gamma(n, width=8)
    h = handle(H, kap, gam, n, levels=2)
    h2 = handle(H, kap, gam, n, levels=2)
    b = torch.from_numpy(inputs.point_sources(n, 2, seed=3, margin=8)).cuda()
    xs, st, rc = H.fgmres_solve([h, h2, h], [b, b, b[:1]], m=10, tol=1e-7)
    assert rc == 0 and len(st) == 5
    a, c, d = (t.cpu().numpy() for t in xs)
    np.testing.assert_allclose(a, c, rtol=0, atol=1e-12 * np.abs(a).max())
    # a batch of one may sum the coarse GEMV in another order: solution bar
    assert np.linalg.norm(d[0] - a[0]) <= 1e-5 * np.linalg.norm(a[0])


def test_autotuned_convolutions_match_oracle(H):
    """With the launch-shape autotuner on, each new convolution shape is tuned
    on first use; the network output still matches the oracle, and a second
    call reuses the table."""
    from paper_2203_11025_amd import unet

    cfg = U.UNetCfg(widths=(32, 64, 128))
    p, buf = U.init_params(cfg, 17)
    net = unet.UNet(widths=(32, 64, 128))
    net.set_params(U.flatten(cfg, p), torch.cat([buf[k].reshape(-1) for k in U.buffer_shapes(cfg)]))
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 64, 64)).astype(np.float32)
    prev = H.autotune(1)
    try:
        out1 = net.forward(torch.from_numpy(x)).cpu().numpy()
        n1 = H.autotune_entries()
        out2 = net.forward(torch.from_numpy(x)).cpu().numpy()
        assert n1 > 0 and H.autotune_entries() == n1
    finally:
        H.autotune(-1)
        H.autotune(prev)
    ref = U.forward(cfg, p, buf, torch.from_numpy(x)).numpy()
    assert np.linalg.norm(out1 - ref) / np.linalg.norm(ref) <= 2e-2
    np.testing.assert_array_equal(out1, out2)
