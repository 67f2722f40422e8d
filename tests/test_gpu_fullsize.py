"""Parity at the full size of the 1024^2 workload, in the launch
configuration the benchmark times: all 32 right-hand sides in one batched
solve, FGMRES(20), 5 SL levels, the convolution autotuner on, the
encoder-solver pair with its shared context for M_VU.  Sampled solutions are
compared with the exact solution of the discrete system (the oracle's sparse
LU, factored once)."""
import os

import numpy as np
import pytest
import torch

from paper_2203_11025_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2203_11025_amd", "weights", "pair_base.safetensors")
SAMPLES = (0, 19)


@pytest.fixture(scope="module")
def setup():
    from oracle import helm_oracle
    from paper_2203_11025_amd import helm, unet

    assert torch.cuda.is_available()
    P = inputs.config_problem("multi1024")
    solve = helm_oracle.direct_solver(P["kappa"], P["gamma"], P["omega"])
    ref = {k: solve(P["b"][k]) for k in SAMPLES}
    h = helm.Handle(torch.from_numpy(P["kappa"]).cuda(), torch.from_numpy(P["gamma"]).cuda(),
                    P["omega"], levels=P["levels"])
    return helm, unet, P, h, ref


def _check(P, xs, st, ref, label):
    x = xs[0]
    assert all(s["converged"] and s["true_relres"] <= 1e-7 for s in st), label
    for k in SAMPLES:
        err = float(np.linalg.norm(x[k].cpu().numpy() - ref[k]) / np.linalg.norm(ref[k]))
        print(f"{label} rhs {k}: relerr vs exact {err:.3e}, its {st[k]['iterations']}, "
              f"relres {st[k]['true_relres']:.2e}, rho_1e6 {st[k]['rho_1e6']:.3f}")
        assert err <= 1e-5, (label, k, err)


def test_plain_sl_1024_batch_matches_exact_solution(setup):
    helm, unet, P, h, ref = setup
    b = torch.from_numpy(P["b"]).cuda()
    xs, st, rc = helm.fgmres_solve([h], [b], m=P["m"], tol=P["tol"])
    assert rc == 0
    _check(P, xs, st, ref, "M_V")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="pretrained weights absent")
def test_mvu_1024_batch_matches_exact_solution(setup):
    helm, unet, P, h, ref = setup
    enc = unet.UNet(head=False)
    sol = unet.UNet(context=True)
    unet.load(WEIGHTS, encoder=enc, solver=sol)
    prev = helm.autotune(1)
    try:
        unet.pair_encode(enc, sol, h.coarse_slowness())
        b = torch.from_numpy(P["b"]).cuda()
        xs, st, rc = helm.fgmres_solve([h], [b], m=P["m"], tol=P["tol"], prec="unet_defl", net=sol)
    finally:
        helm.autotune(prev)
    assert rc == 0
    assert all(s["fallback"] == 0 for s in st)
    _check(P, xs, st, ref, "M_VU")
