"""The uneven batch (many media of uneven grid sizes in one solve call): the
encoder-solver M_VU (eq. 3.4, section 3.3) with each medium encoded in turn
and the plain-SL fallback at a residual ratio of 0.95, through the C ABI."""
import os

import numpy as np
import pytest
import torch

from paper_2203_11025_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2203_11025_amd", "weights", "pair_base.safetensors")


@pytest.fixture(scope="module")
def setup():
    from paper_2203_11025_amd import helm, unet

    assert torch.cuda.is_available()
    P = inputs.config_problems("uneven6")
    hs = [helm.Handle(torch.from_numpy(p["kappa"]).cuda(), torch.from_numpy(p["gamma"]).cuda(), p["omega"],
                      levels=p["levels"]) for p in P]
    bs = [torch.from_numpy(p["b"]).cuda() for p in P]
    enc, sol = unet.UNet(head=False), unet.UNet(context=True)
    if os.path.exists(WEIGHTS):
        unet.load(WEIGHTS, encoder=enc, solver=sol)
    else:
        enc.init(1)
        sol.init(2)
    return helm, unet, P, hs, bs, enc, sol


def test_uneven_media_in_one_call_match_one_by_one_and_the_oracle_residual(setup, oracle):
    """Six layered media of 256^2 to 2048^2 with 8 sources each: one call
    with the encoder equals per-medium calls (encode, then solve) bit for
    bit, and every solution meets the FP64 true residual, rechecked by the
    oracle's operator for one right-hand side per medium."""
    helm, unet, P, hs, bs, enc, sol = setup
    prev = helm.autotune(0)
    try:
        xs, st, rc = helm.fgmres_solve(hs, bs, m=20, tol=1e-7, prec="unet_defl", net=sol, encoder=enc,
                                       stall_ratio=0.95)
        assert rc == 0
        assert all(s["converged"] and s["true_relres"] <= 1e-7 for s in st)
        off = 0
        for p, (h, b) in enumerate(zip(hs, bs)):
            unet.pair_encode_medium(enc, sol, h)
            x1, st1, rc1 = helm.fgmres_solve([h], [b], m=20, tol=1e-7, prec="unet_defl", net=sol,
                                             stall_ratio=0.95)
            assert rc1 == 0
            assert np.array_equal(x1[0].cpu().numpy(), xs[p].cpu().numpy()), p
            assert [s["iterations"] for s in st1] == [s["iterations"] for s in st[off:off + len(st1)]]
            k = p % b.shape[0]
            x = xs[p][k].cpu().numpy()
            r = P[p]["b"][k].astype(complex) - oracle.apply(P[p]["kappa"], P[p]["gamma"], P[p]["omega"], x)
            relres = np.linalg.norm(r) / np.linalg.norm(P[p]["b"][k])
            print(f"medium {p} n={h.n}: its mean {np.mean([s['iterations'] for s in st1]):.1f} "
                  f"fallbacks {sum(s['fallback'] for s in st1)} oracle relres {relres:.2e}")
            assert relres <= 1.05e-7
            off += len(st1)
    finally:
        helm.autotune(prev)


def test_encoder_option_misuse_is_rejected(setup):
    helm, unet, P, hs, bs, enc, sol = setup
    with pytest.raises(helm.HelmError, match="encoder"):
        helm.fgmres_solve(hs[:1], bs[:1], prec="sl", encoder=enc)
    plain = unet.UNet()
    plain.init(3)
    with pytest.raises(helm.HelmError, match="encoder"):
        helm.fgmres_solve(hs[:1], bs[:1], prec="unet_defl", net=plain, encoder=enc)
