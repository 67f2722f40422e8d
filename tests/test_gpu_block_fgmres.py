"""Block FGMRES (section 4: block restarted FGMRES(10), block size 10) on the
GPU against the oracle's block FGMRES and the exact solution, through the C
ABI."""
import numpy as np
import pytest
import torch

from oracle import block_fgmres as BF
from paper_2203_11025_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2203_11025_amd import helm, unet

    assert torch.cuda.is_available()
    unet.lib()
    return helm, unet


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _problem(helm, n, seed, levels):
    kap = inputs.smooth_medium(n, max(2.0, n / 16), seed=seed)
    gam = inputs.sponge_gamma(n, width=min(16, n // 8))
    om = inputs.omega_for_ppw(n)
    h = helm.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), om, levels=levels)
    return kap, gam, om, h


@pytest.mark.parametrize("n,levels,nrhs,block,m", [(128, 3, 7, 3, 10), (64, 2, 10, 10, 10), (96, 2, 4, 4, 6),
                                                    (48, 2, 16, 16, 5)])
def test_block_fgmres_matches_the_exact_solution_and_the_oracle(H, oracle, n, levels, nrhs, block, m):
    """Blocks of 3 + 3 + 1, one block of 10, a 96^2 grid and the largest
    block (16, with the device-side Cholesky QR at its full size): every field
    reaches the FP64 tolerance, the solution matches the exact solution of
    the discrete system to 1e-5, and the block iteration counts are the
    oracle's within 10% (R23)."""
    helm, _ = H
    kap, gam, om, h = _problem(helm, n, n + nrhs, levels)
    b = inputs.point_sources(n, nrhs, seed=5, margin=min(16, n // 8)).astype(np.complex64)
    x, st, rc = helm.block_fgmres_solve(h, torch.from_numpy(b).cuda(), block=block, m=m, tol=1e-7)
    assert rc == 0 and all(s["converged"] and s["true_relres"] <= 1e-7 for s in st)
    x = x.cpu().numpy()
    solve = oracle.direct_solver(kap, gam, om)
    ho = oracle.Hierarchy(kap, gam, om, levels)
    for b0 in range(0, nrhs, block):
        blk = b[b0:b0 + block]
        xo, so = BF.block_fgmres(ho, blk.astype(complex), m=m, tol=1e-7)
        its = st[b0]["iterations"]
        assert abs(its - so["iterations"]) <= max(2, 0.1 * so["iterations"]), (b0, its, so["iterations"])
        for k in range(blk.shape[0]):
            ref = solve(blk[k])
            assert rel(x[b0 + k], ref) <= 1e-5, (b0 + k, rel(x[b0 + k], ref))


def test_rank_deficient_block_is_solved_field_by_field(H, oracle):
    """A block holding a zero right-hand side and two equal ones has a
    residual block Cholesky QR cannot factor: its fields are solved one at a
    time instead.  Every field converges, the zero field stays zero, the two
    equal fields get equal solutions and all match the exact solution; a
    second, full-rank block in the same call is solved as a block."""
    helm, _ = H
    n = 64
    kap, gam, om, h = _problem(helm, n, 21, 2)
    src = inputs.point_sources(n, 5, seed=8, margin=8).astype(np.complex64)
    b = np.stack([src[0], np.zeros_like(src[0]), src[1], src[0], src[2], src[3], src[4]])
    x, st, rc = helm.block_fgmres_solve(h, torch.from_numpy(b).cuda(), block=4, m=10, tol=1e-7)
    x = x.cpu().numpy()
    assert rc == 0 and all(s["converged"] and s["true_relres"] <= 1e-7 for s in st), st
    assert np.all(x[1] == 0.0)
    assert np.array_equal(x[0], x[3])
    solve = oracle.direct_solver(kap, gam, om)
    for k in (0, 2, 4, 5, 6):
        assert rel(x[k], solve(b[k])) <= 1e-5, (k, rel(x[k], solve(b[k])))
    # the second block (fields 4-6) kept one block iteration count
    assert st[4]["iterations"] == st[5]["iterations"] == st[6]["iterations"]


def test_block_of_one_is_fgmres(H):
    """Block size 1 runs the same method as helm_fgmres_solve (another
    orthogonalisation and stop bookkeeping): same iterations within 10%,
    same solution to 1e-5."""
    helm, _ = H
    n = 128
    kap, gam, om, h = _problem(helm, n, 9, 3)
    b = torch.from_numpy(inputs.point_sources(n, 2, seed=6)).cuda()
    xb, sb, rcb = helm.block_fgmres_solve(h, b, block=1, m=10, tol=1e-7)
    xs, ss, rcs = helm.fgmres_solve([h], [b], m=10, tol=1e-7)
    assert rcb == 0 and rcs == 0
    for k in range(2):
        assert abs(sb[k]["iterations"] - ss[k]["iterations"]) <= max(2, 0.1 * ss[k]["iterations"])
        assert rel(xb.cpu().numpy()[k], xs[0].cpu().numpy()[k]) <= 1e-5


def test_block_fgmres_with_network_preconditioners(H, oracle):
    """M_VU inside block FGMRES with a seeded (untrained) network converges to
    the FP64 tolerance and to the exact solution (the V-cycle cleans up the
    network's error).  M_CU with an untrained network is not a convergent
    preconditioner (Jacobi sweeps around a random map); its block solve must
    still report the FP64 true residual of the x it returns."""
    helm, unet = H
    n = 64
    kap, gam, om, h = _problem(helm, n, 12, 2)
    net = unet.UNet(widths=(32, 64))
    net.init(4)
    b = inputs.point_sources(n, 4, seed=8, margin=8).astype(np.complex64)
    solve = oracle.direct_solver(kap, gam, om)
    x, st, rc = helm.block_fgmres_solve(h, torch.from_numpy(b).cuda(), block=4, m=10, tol=1e-7, prec="unet_defl",
                                        net=net, maxit=500)
    assert rc == 0 and all(s["true_relres"] <= 1e-7 for s in st)
    x = x.cpu().numpy()
    for k in range(4):
        assert rel(x[k], solve(b[k])) <= 1e-5, k
    x, st, rc = helm.block_fgmres_solve(h, torch.from_numpy(b).cuda(), block=4, m=10, tol=1e-7, prec="unet_cgc",
                                        net=net, maxit=30)
    x = x.cpu().numpy()
    for k in range(4):
        r = b[k].astype(complex) - oracle.apply(kap, gam, om, x[k])
        assert abs(np.linalg.norm(r) / np.linalg.norm(b[k]) - st[k]["true_relres"]) <= 1e-6 * st[k]["true_relres"]


def test_block_fgmres_argument_checks(H):
    helm, _ = H
    kap, gam, om, h = _problem(helm, 64, 3, 2)
    b = torch.zeros((2, 64, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(helm.HelmError, match="block size"):
        helm.block_fgmres_solve(h, b, block=17)
    with pytest.raises(helm.HelmError, match="4096"):
        helm.block_fgmres_solve(h, b, block=2, m=1100)
    x, st, rc = helm.block_fgmres_solve(h, b, block=2)
    assert rc == 0 and np.count_nonzero(x.cpu().numpy()) == 0
