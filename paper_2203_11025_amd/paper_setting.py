"""The paper's own test setting (section 4) and its homogeneous-medium
experiment (section 4.1), run with this library.

Setting: the unit square on a 128 x 128 grid, omega = 20 pi (about 12.5
points per wavelength), an absorbing layer of width 10 (attenuation zero in
the interior, quadratic ramp to 1 at the edge), SL V-cycles with beta = 0.5,
3 levels, one damped Jacobi pre- and post-relaxation (weight 0.8) and the
coarsest level solved by GMRES(10) with the Jacobi preconditioner.  The
network (the configured U-Net, a plain network for one known medium) is
trained on triples from that medium with k in 1..10 FGMRES steps per sample
(eq. 3.8), linear-combination augmentation and the section-4 schedule of the
learning rate and batch size.  The preconditioners M_V, M_JU (Algorithm 2)
and M_VU (eq. 3.4) are compared by the convergence factor of eq. 4.1
(residual reduction 1e6) of FGMRES(10) on random right-hand sides, and the
network by its relative error ||e_net - e|| / ||e|| on held-out triples.

    python -m paper_2203_11025_amd.paper_setting [--medium homogeneous|smooth]
        [--epochs 100] [--dataset 1000] [--rhs 10] [--arch 0|1] [--block 10]
        [--sweep] [--out results.json]

The paper reports, for the homogeneous medium, a final relative training
error of 0.18 and rho_VU = 0.231, rho_JU = 0.313 against 0.88 for M_V; those
come from its own network (5x5 strided transfers, ResNet blocks) and block
FGMRES(10), so they are sanity ranges here, not targets.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from functools import partial

import numpy as np

N = 128
OMEGA = 20 * np.pi
LAYER = 10


def medium(kind="homogeneous", n=N, seed=0):
    """Slowness and attenuation of the section-4 setting: kappa = 1
    (homogeneous, section 4.1) or a smooth medium with kappa^2 in [0.25, 1]."""
    from . import inputs

    if kind == "homogeneous":
        kap = np.ones((n, n), dtype=np.float32)
    else:
        k2 = inputs.smooth_medium(n, n / 16, seed=seed, lo=0.25, hi=1.0)
        kap = np.sqrt(k2).astype(np.float32)
    gam = inputs.sponge_gamma(n, width=LAYER, interior=0.0, edge=1.0)
    return kap, gam


def relative_error(net, h, seed, count, ksteps="random"):
    """Mean of ||e_net - e|| / ||e|| over held-out triples (indices from
    2^40 on), e_net from the network wrapper (inference BN)."""
    import torch

    from . import train

    n = h.n
    data = train.Batches([h], 1, ksteps=ksteps)
    errs = []
    for i in range(count):
        r, e, _ = data.fill(seed, (1 << 40) + i)
        en = net.infer(h, r)
        a, b = en.cpu().numpy(), e.cpu().numpy()
        errs.append(np.linalg.norm(a - b) / np.linalg.norm(b))
    torch.cuda.synchronize()
    return float(np.mean(errs))


def solve_all(h, net, rhs, m=10, tol=1e-7, maxit=2000, block=0):
    """FGMRES(m) with M_V, M_JU and M_VU on the same right-hand sides (block
    FGMRES(m) with blocks of `block` right-hand sides when block > 0, as in
    section 4); per preconditioner the mean iterations to a 1e6 reduction and
    the mean convergence factor of eq. 4.1 at that reduction."""
    import torch

    from . import helm

    out = {}
    for name, prec in (("V", "sl"), ("JU", "unet_cgc"), ("VU", "unet_defl")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pnet = None if prec == "sl" else net
        if block > 0:
            _, st, rc = helm.block_fgmres_solve(h, rhs, block=block, m=m, tol=tol, maxit=maxit, prec=prec, net=pnet)
        else:
            _, st, rc = helm.fgmres_solve([h], [rhs], m=m, tol=tol, maxit=maxit, prec=prec, net=pnet)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = dict(rho=float(np.mean([s["rho_1e6"] for s in st])),
                         its_1e6=float(np.mean([s["its_1e6"] for s in st])),
                         its=float(np.mean([s["iterations"] for s in st])),
                         relres_max=float(max(s["true_relres"] for s in st)),
                         fallbacks=int(sum(s["fallback"] for s in st)), status=rc, seconds=dt)
    return out


def sweep(h, net, rhs):
    """The influence of the block size and of the subspace size (section
    4.3.4): block FGMRES(10) with blocks of 1, 2, 5 and 10 right-hand sides,
    and block FGMRES(m) with blocks of 10 for m = 5, 10, 20; per setting and
    preconditioner the mean rho of eq. 4.1 and the mean iterations to 1e-7."""
    out = []
    for block, m in ((1, 10), (2, 10), (5, 10), (10, 10), (10, 5), (10, 20)):
        r = solve_all(h, net, rhs, m=m, block=block)
        out.append({"block": block, "m": m, **{k: {"rho": v["rho"], "its": v["its"]} for k, v in r.items()}})
    return out


def run(kind="homogeneous", epochs=100, dataset=1000, lr0=1e-3, batch0=20, t0=48, rhs=10, seed=1,
        widths=None, log=True, arch=0, block=0, do_sweep=False):
    """arch 0: the configured U-Net between fixed transfers (widths 32..256);
    arch 1: the paper's network of section 3.1 (widths 16..128, learned 5x5
    strided transfers, ELU ResNet blocks, 4 input channels)."""
    import torch

    from . import helm, train, unet

    kap, gam = medium(kind)
    h = helm.Handle(torch.from_numpy(kap).cuda(), torch.from_numpy(gam).cuda(), OMEGA, levels=3, coarse_gmres=10)
    if widths is None:
        widths = (16, 32, 64, 128) if arch == 1 else (32, 64, 128, 256)
    net = unet.UNet(widths=widths, arch=arch)
    net.init(seed)
    rng = np.random.default_rng(seed + 1000)
    b = (rng.standard_normal((rhs, N, N)) + 1j * rng.standard_normal((rhs, N, N))).astype(np.complex64)
    b = torch.from_numpy(b).cuda()
    before = solve_all(h, net, b, block=block)
    err0 = relative_error(net, h, seed + 7, 16)
    t = time.perf_counter()
    sched = partial(train.paper_schedule, lr0=lr0, batch0=batch0, t0=t0)
    losses = train.train(net, [h], steps=epochs, seed=seed, dataset=dataset, ksteps="random", augment=True,
                         schedule=sched, log=1 if log else None)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t
    err1 = relative_error(net, h, seed + 7, 16)
    after = solve_all(h, net, b, block=block)
    swept = sweep(h, net, b) if do_sweep else None
    return dict(medium=kind, n=N, omega=OMEGA, layer=LAYER, levels=3, coarse="GMRES(10)+Jacobi", arch=arch,
                widths=list(widths), nparams=net.nparams, krylov=f"block FGMRES(10), block {block}" if block else
                "FGMRES(10)", epochs=epochs,
                dataset=dataset, lr0=lr0, batch0=batch0, t0=t0, steps=len(losses), train_seconds=t_train,
                loss_first=losses[0] if losses else None, loss_last=losses[-1] if losses else None,
                rel_error_untrained=err0, rel_error_trained=err1, untrained=before, trained=after, sweep=swept)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--medium", default="homogeneous", choices=["homogeneous", "smooth"])
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--dataset", type=int, default=1000)
    ap.add_argument("--lr0", type=float, default=1e-3)
    ap.add_argument("--batch0", type=int, default=20)
    ap.add_argument("--t0", type=int, default=48)
    ap.add_argument("--rhs", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--arch", type=int, default=0, choices=[0, 1])
    ap.add_argument("--block", type=int, default=0, help="block size of block FGMRES (0: FGMRES per RHS)")
    ap.add_argument("--sweep", action="store_true", help="after training, sweep the block and subspace sizes")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.medium, a.epochs, a.dataset, a.lr0, a.batch0, a.t0, a.rhs, a.seed, arch=a.arch, block=a.block,
              do_sweep=a.sweep)
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
