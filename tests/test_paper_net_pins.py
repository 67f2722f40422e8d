"""Pins of the oracle of the paper's own network (section 3.1, eq. 3.1-3.3):
the strided and transposed 5x5 convolutions against explicit loops, the
ResNet block in closed form, the wrapper's homogeneity, and the gradients
against FP64 central differences."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import paper_net_oracle as PN


def test_layer_list_and_shapes():
    cfg = PN.PaperNetCfg(widths=(8, 16, 32))
    names = [l[0] for l in PN.layers(cfg)]
    assert names == ["down1", "res1_0a", "res1_0b", "down2", "res2_0a", "res2_0b", "down3", "res3_0a", "res3_0b",
                     "res3_1a", "res3_1b", "res3_2a", "res3_2b", "up2", "up1", "out"]
    p, buf = PN.init_params(cfg, 1)
    x = torch.randn(2, 4, 32, 32)
    assert PN.forward(cfg, p, buf, x).shape == (2, 2, 32, 32)
    # up2: 32 -> 16 channels, concat 16 -> 32; up1: 32 -> 8, concat 8 -> 16; out: 16 -> 2
    assert p["up2.w"].shape == (32, 16, 5, 5) and p["up1.w"].shape == (32, 8, 5, 5)
    assert p["out.w"].shape == (16, 2, 5, 5)


def test_strided_convolution_against_an_explicit_loop():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 6, 6))
    w = rng.standard_normal((2, 3, 5, 5))
    ref = np.zeros((2, 3, 3))
    for co in range(2):
        for I in range(3):
            for J in range(3):
                for ci in range(3):
                    for a in range(5):
                        for b in range(5):
                            i, j = 2 * I + a - 2, 2 * J + b - 2
                            if 0 <= i < 6 and 0 <= j < 6:
                                ref[co, I, J] += w[co, ci, a, b] * x[ci, i, j]
    got = F.conv2d(torch.tensor(x[None]), torch.tensor(w), stride=2, padding=2)[0].numpy()
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_transposed_convolution_against_an_explicit_loop_and_as_the_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 3, 3))
    w = rng.standard_normal((3, 2, 5, 5))
    ref = np.zeros((2, 6, 6))
    for ci in range(3):
        for I in range(3):
            for J in range(3):
                for a in range(5):
                    for b in range(5):
                        i, j = 2 * I + a - 2, 2 * J + b - 2
                        if 0 <= i < 6 and 0 <= j < 6:
                            ref[:, i, j] += w[ci, :, a, b] * x[ci, I, J]
    got = F.conv_transpose2d(torch.tensor(x[None]), torch.tensor(w), stride=2, padding=2,
                             output_padding=1)[0].numpy()
    np.testing.assert_allclose(got, ref, atol=1e-12)
    # <R u, v> = <u, P v> with the same weights: P is the adjoint of R
    u = rng.standard_normal((2, 6, 6))
    Ru = F.conv2d(torch.tensor(u[None]), torch.tensor(w).transpose(0, 1).contiguous().transpose(0, 1),
                  stride=2, padding=2)
    wt = torch.tensor(w)  # [3 (coarse), 2 (fine), 5, 5]
    Ru = F.conv2d(torch.tensor(u[None]), wt, stride=2, padding=2)[0].numpy()
    Pv = F.conv_transpose2d(torch.tensor(x[None]), wt, stride=2, padding=2, output_padding=1)[0].numpy()
    assert abs(np.sum(Ru * x) - np.sum(u * Pv)) <= 1e-10 * abs(np.sum(Ru * x))


def test_resnet_block_with_a_zero_second_convolution_is_elu_of_bn():
    """eq. 3.2 with K2 = 0: x' = elu(BN(x)); in inference with running mean
    m and variance v: elu(g (x - m) / sqrt(v + eps) + b)."""
    cfg = PN.PaperNetCfg(widths=(4,), coarsest_blocks=1)
    p, buf = PN.init_params(cfg, 2, dtype=torch.float64)
    p["res1_0b.w"].zero_()
    buf["res1_0b.rm"] = torch.tensor([0.1, -0.2, 0.3, 0.0], dtype=torch.float64)
    buf["res1_0b.rv"] = torch.tensor([2.0, 0.5, 1.0, 3.0], dtype=torch.float64)
    p["res1_0b.g"] = torch.tensor([1.5, 0.5, 1.0, 2.0], dtype=torch.float64)
    p["res1_0b.b"] = torch.tensor([0.1, 0.0, -0.3, 0.2], dtype=torch.float64)
    x = torch.randn(1, 4, 8, 8, dtype=torch.float64)
    h = F.elu(PN._bn(F.conv2d(x, p["down1.w"], stride=2, padding=2), p, buf, "down1", False, None))
    m, v = buf["res1_0b.rm"], buf["res1_0b.rv"]
    ref = F.elu(p["res1_0b.g"][None, :, None, None] * (h - m[None, :, None, None])
                / torch.sqrt(v[None, :, None, None] + 1e-5) + p["res1_0b.b"][None, :, None, None])
    t = F.elu(PN._bn(F.conv2d(h, p["res1_0a.w"], padding=1), p, buf, "res1_0a", False, None))
    got = F.elu(PN._bn(h + F.conv2d(t, p["res1_0b.w"], padding=1), p, buf, "res1_0b", False, None))
    assert torch.allclose(got, ref, atol=1e-12)


def test_wrapper_is_positively_homogeneous_and_zero_preserving():
    cfg = PN.PaperNetCfg(widths=(4, 8))
    p, buf = PN.init_params(cfg, 3)
    rng = np.random.default_rng(2)
    n = 16
    r = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    kap = rng.uniform(0.5, 1.0, (n, n))
    gam = np.zeros((n, n))
    e1 = PN.apply(cfg, p, buf, r, kap, gam, dtype=torch.float64)
    e2 = PN.apply(cfg, p, buf, 7.5 * r, kap, gam, dtype=torch.float64)
    assert np.linalg.norm(e2 - 7.5 * e1) <= 1e-12 * np.linalg.norm(e2)
    assert np.count_nonzero(PN.apply(cfg, p, buf, 0 * r, kap, gam)) == 0


def test_gradients_match_central_differences():
    cfg = PN.PaperNetCfg(widths=(4, 8))
    p, buf = PN.init_params(cfg, 4, dtype=torch.float64)
    rng = np.random.default_rng(3)
    n, B = 16, 2
    r = rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))
    e = rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))
    kap = rng.uniform(0.5, 1.0, (n, n))
    gam = rng.uniform(0.0, 0.3, (n, n))
    pg = {k: v.clone().requires_grad_(True) for k, v in p.items()}
    loss = PN.training_loss(cfg, pg, buf, r * 1e-4, e * 1e-8, kap, gam, dtype=torch.float64)
    loss.backward()
    picks = ["down1.w", "res1_0a.w", "res2_2b.g", "up1.w", "up1.b", "out.w", "out.bias", "res2_0b.w"]
    for k in picks:
        g = pg[k].grad.reshape(-1)
        for idx in (0, g.numel() // 2, g.numel() - 1):
            def f(delta):
                q = {kk: v.clone() for kk, v in p.items()}
                q[k].reshape(-1)[idx] += delta
                return PN.training_loss(cfg, q, buf, r * 1e-4, e * 1e-8, kap, gam, dtype=torch.float64).item()
            d = 1e-6
            fd = (f(d) - f(-d)) / (2 * d)
            assert abs(fd - g[idx].item()) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, g[idx].item())
