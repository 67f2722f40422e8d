"""GPU parity of the SL path (helm_apply, helm_sl_vcycle, helm_fgmres_solve)
against the FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2203_11025_amd import inputs

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(2024)


def crandn(*shape):
    return (RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)).astype(np.complex64)


@pytest.fixture(scope="module")
def H():
    from paper_2203_11025_amd import helm

    assert torch.cuda.is_available()
    helm.lib()
    return helm


def medium(n, seed, sponge=16):
    kap = inputs.smooth_medium(n, max(2.0, n / 16), seed=seed)
    gam = inputs.sponge_gamma(n, width=min(sponge, n // 4))
    return kap, gam, inputs.omega_for_ppw(n)


def handle(H, kap, gam, om, levels=0):
    return H.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), om, levels=levels)


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [40, 96, 128, 512])
@pytest.mark.parametrize("op", ["A", "M"])
def test_apply_parity(H, oracle, n, op):
    kap, gam, om = medium(n, n)
    h = handle(H, kap, gam, om, levels=1 if n <= 64 else 0)
    x = crandn(3, n, n)
    y = h.apply(torch.from_numpy(x).cuda(), op=op).cpu().numpy()
    shift = 0.0 if op == "A" else 0.5
    for k in range(3):
        ref = oracle.apply(kap, gam, om, x[k], shift=shift)
        assert relerr(y[k], ref) <= 1e-6
        assert np.abs(y[k] - ref).max() <= 5e-6 * np.abs(ref).max()


@pytest.mark.parametrize("n,levels", [(32, 1), (64, 2), (96, 2), (128, 3), (256, 3), (512, 4)])
def test_vcycle_parity(H, oracle, n, levels):
    kap, gam, om = medium(n, 100 + n)
    h = handle(H, kap, gam, om, levels=levels)
    ho = oracle.Hierarchy(kap, gam, om, levels)
    f = crandn(2, n, n)
    v = h.vcycle(torch.from_numpy(f).cuda()).cpu().numpy()
    for k in range(2):
        ref = ho.vcycle(f[k])
        assert relerr(v[k], ref) <= 1e-5, (n, levels, k, relerr(v[k], ref))


@pytest.mark.parametrize("nb", [5, 37])
def test_vcycle_many_rhs_parity(H, oracle, nb):
    """Four or more right-hand sides take the tiled GEMM for the coarsest
    solve (37: two right-hand-side tiles, the second partial); every one is
    compared with the oracle, with a zero field in the batch."""
    n, levels = 64, 2
    kap, gam, om = medium(n, 300 + nb)
    h = handle(H, kap, gam, om, levels=levels)
    ho = oracle.Hierarchy(kap, gam, om, levels)
    f = crandn(nb, n, n)
    f[3] = 0
    v = h.vcycle(torch.from_numpy(f).cuda()).cpu().numpy()
    assert np.all(v[3] == 0)
    for k in range(nb):
        if k != 3:
            ref = ho.vcycle(f[k])
            assert relerr(v[k], ref) <= 1e-5, (nb, k, relerr(v[k], ref))


def test_vcycle_point_source_and_zero(H, oracle):
    n = 128
    kap, gam, om = medium(n, 7)
    h = handle(H, kap, gam, om, levels=3)
    ho = oracle.Hierarchy(kap, gam, om, 3)
    f = np.stack([inputs.point_source(n), np.zeros((n, n), np.complex64)])
    v = h.vcycle(torch.from_numpy(f).cuda()).cpu().numpy()
    assert relerr(v[0], ho.vcycle(f[0])) <= 1e-5
    assert np.all(v[1] == 0)


def _true_relres(oracle, kap, gam, om, b, x):
    r = b.astype(np.complex128) - oracle.apply(kap, gam, om, x)
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_fgmres_plain128_matches_oracle(H, oracle):
    """The 128^2 constant-medium point-source workload, FGMRES(10), 3 levels."""
    P = inputs.config_problem("plain128")
    n = P["n"]
    h = handle(H, P["kappa"], P["gamma"], P["omega"], levels=P["levels"])
    b = P["b"]
    xs, st, rc = H.fgmres_solve([h], [torch.from_numpy(b).cuda()], m=P["m"], tol=1e-7)
    assert rc == 0 and st[0]["converged"]
    x = xs[0].cpu().numpy()[0]
    assert _true_relres(oracle, P["kappa"], P["gamma"], P["omega"], b[0], x) <= 1e-7
    assert st[0]["true_relres"] <= 1e-7
    ho = oracle.Hierarchy(P["kappa"], P["gamma"], P["omega"], P["levels"])
    xo, sto = ho.fgmres(b[0], m=P["m"], tol=1e-10)
    assert relerr(x, xo) <= 1e-5
    # iteration counts agree within the band rounding allows
    xo7, sto7, hist = ho.fgmres(b[0], m=P["m"], tol=1e-7, history=True)
    assert abs(st[0]["iterations"] - sto7["iterations"]) <= max(3, 0.1 * sto7["iterations"])
    # convergence factor of eq. 4.1 at a 1e6 reduction, from the GPU's
    # implicit residuals, against the oracle's residual history
    rho_o, T_o = oracle.convergence_factor(hist, 1e6)
    assert abs(st[0]["its_1e6"] - T_o) <= max(3, 0.1 * T_o), (st[0]["its_1e6"], T_o)
    assert abs(st[0]["rho_1e6"] - rho_o) <= 0.02, (st[0]["rho_1e6"], rho_o)
    assert 0 < st[0]["its_1e6"] <= st[0]["its_1e7"] <= st[0]["iterations"]
    assert 0 < st[0]["rho_1e6"] < 1 and 0 < st[0]["rho_1e7"] < 1


def test_fgmres_batch_heterogeneous(H, oracle):
    """Several right-hand sides in one launch, including a zero one."""
    n = 128
    kap, gam, om = medium(n, 21)
    h = handle(H, kap, gam, om, levels=3)
    b = inputs.point_sources(n, 3, seed=5)
    b = np.concatenate([b, crandn(1, n, n), np.zeros((1, n, n), np.complex64)])
    xs, st, rc = H.fgmres_solve([h], [torch.from_numpy(b).cuda()], m=10, tol=1e-7)
    assert rc == 0
    x = xs[0].cpu().numpy()
    ho = oracle.Hierarchy(kap, gam, om, 3)
    for k in range(4):
        assert st[k]["converged"] and st[k]["true_relres"] <= 1e-7
        assert _true_relres(oracle, kap, gam, om, b[k], x[k]) <= 1e-7
        xo, _ = ho.fgmres(b[k], m=10, tol=1e-10)
        assert relerr(x[k], xo) <= 1e-5
    assert st[4]["iterations"] == 0 and np.all(x[4] == 0)


def test_fgmres_two_problems(H, oracle):
    n1, n2 = 64, 128
    k1, g1, o1 = medium(n1, 31)
    k2, g2, o2 = medium(n2, 32)
    h1, h2 = handle(H, k1, g1, o1, levels=2), handle(H, k2, g2, o2, levels=3)
    b1, b2 = inputs.point_sources(n1, 2, seed=1, margin=8), inputs.point_sources(n2, 1, seed=2)
    xs, st, rc = H.fgmres_solve([h1, h2], [torch.from_numpy(b1).cuda(), torch.from_numpy(b2).cuda()],
                                m=20, tol=1e-7)
    assert rc == 0 and len(st) == 3
    x1, x2 = xs[0].cpu().numpy(), xs[1].cpu().numpy()
    for k in range(2):
        assert _true_relres(oracle, k1, g1, o1, b1[k], x1[k]) <= 1e-7
    assert _true_relres(oracle, k2, g2, o2, b2[0], x2[0]) <= 1e-7


def test_fgmres_maxit_not_converged(H):
    n = 64
    kap, gam, om = medium(n, 41)
    h = handle(H, kap, gam, om, levels=2)
    b = torch.from_numpy(inputs.point_source(n)[None]).cuda()
    xs, st, rc = H.fgmres_solve([h], [b], m=10, tol=1e-12, maxit=5)
    assert rc == H.HELM_NOT_CONVERGED
    assert st[0]["iterations"] == 5 and not st[0]["converged"]


def test_fgmres_plain512_full_size(H, oracle):
    """The 512^2 smooth-medium workload (4 levels, FGMRES(20)): the FP64
    oracle residual of the result, and the solution against the oracle's own
    FGMRES driven to 1e-10 (so the reference is not the error source)."""
    P = inputs.config_problem("plain512")
    h = handle(H, P["kappa"], P["gamma"], P["omega"], levels=P["levels"])
    xs, st, rc = H.fgmres_solve([h], [torch.from_numpy(P["b"]).cuda()], m=P["m"], tol=1e-7)
    assert rc == 0 and st[0]["converged"]
    x = xs[0].cpu().numpy()[0]
    assert _true_relres(oracle, P["kappa"], P["gamma"], P["omega"], P["b"][0], x) <= 1e-7
    ho = oracle.Hierarchy(P["kappa"], P["gamma"], P["omega"], P["levels"])
    xo, sto = ho.fgmres(P["b"][0], m=P["m"], tol=1e-10)
    err = relerr(x, xo)
    print(f"512^2 plain SL: relerr vs oracle {err:.3e}, its {st[0]['iterations']} vs {sto['iterations']}")
    assert err <= 1e-5, err


def test_setup_rejects_bad_shapes(H):
    kap, gam, om = medium(64, 1)
    with pytest.raises(H.HelmError):
        handle(H, kap, gam, om, levels=8)
    with pytest.raises(H.HelmError):
        H.Handle(torch.from_numpy(kap[:63, :63].copy()).cuda(),
                 torch.from_numpy(gam[:63, :63].copy()).cuda(), om)
    with pytest.raises(H.HelmError):
        handle(H, kap, gam, -1.0)


def test_empty_batches(H):
    """Zero right-hand sides are no-ops in every batched entry point, also
    next to a problem that has right-hand sides."""
    from paper_2203_11025_amd import unet

    n = 64
    kap, gam, om = medium(n, 51)
    h = handle(H, kap, gam, om, levels=2)
    empty = torch.zeros((0, n, n), dtype=torch.complex64, device="cuda")
    assert h.apply(empty).shape == (0, n, n)
    assert h.vcycle(empty).shape == (0, n, n)
    b = torch.from_numpy(inputs.point_sources(n, 1, seed=3, margin=8)).cuda()
    xs, st, rc = H.fgmres_solve([h, h], [empty, b], m=10, tol=1e-7)
    assert rc == 0 and len(st) == 1 and st[0]["converged"]
    xs, st, rc = H.fgmres_solve([], [], m=10, tol=1e-7)
    assert rc == 0 and st == []
    net = unet.UNet(widths=(32, 64))
    net.init(1)
    assert net.infer(h, empty).shape == (0, n, n)


def test_fgmres_2048_largest_grid(H, oracle):
    """The largest grid of the uneven-batch workload: 2048^2 layered medium,
    6 levels (64^2 coarsest), plain SL; the FP64 oracle residual of the
    result meets the tolerance."""
    n = 2048
    kap = inputs.layered_medium(n, seed=77)
    gam = inputs.sponge_gamma(n)
    om = inputs.omega_for_ppw(n)
    h = handle(H, kap, gam, om, levels=6)
    b = inputs.point_sources(n, 2, seed=78)
    xs, st, rc = H.fgmres_solve([h], [torch.from_numpy(b).cuda()], m=20, tol=1e-7)
    assert rc == 0 and all(s["converged"] for s in st)
    x = xs[0].cpu().numpy()
    for k in range(2):
        assert _true_relres(oracle, kap, gam, om, b[k], x[k]) <= 1e-7


def test_profile_sampling(H):
    """Live kernel timing: every launch, then about one in four (a fixed
    hashed subset: 11 of the first 40), with the same work per launch."""
    n = 64
    kap, gam, om = medium(n, 61)
    h = handle(H, kap, gam, om, levels=2)
    x = torch.from_numpy(crandn(2, n, n)).cuda()
    counts = {}
    for every in (1, 4):
        H.profile_start("apply", every=every)
        for _ in range(40):
            h.apply(x)
        torch.cuda.synchronize()
        ms, launches, work = H.profile_read("apply")
        assert ms > 0.0
        counts[every] = (launches, work / launches)
    H.profile_stop()
    assert counts[1][0] == 40 and counts[4][0] == 11
    assert counts[4][1] == counts[1][1] == 24.0 * n * n * 2
