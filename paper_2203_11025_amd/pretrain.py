"""Pretraining of the encoder-solver pair (section 3.4 with the encoder of
section 3.3) on triples the method generates (eq. 3.8-3.9) from many smooth
random media, all in the library's kernels.

    python -m paper_2203_11025_amd.pretrain --minutes 15 --out PATH
    python -m paper_2203_11025_amd.pretrain --plain --media 200 --ksteps random --minutes 13 --out PATH

Media: n^2 grids (default 512, network on 256^2), slowness from seeded white
noise smoothed by a Gaussian of sigma n/32 cells mapped to [0.25, 1], seeds
10000 + i; 10 points per wavelength; the quadratic sponge.  Each Adam step
(lr 1e-3 by default, optionally decayed linearly in time, batch 16) takes
`per_medium` samples from consecutive media.  `--resume` continues from
saved weights (e.g. fine-tuning at a larger grid).  The
weights are saved every `--save-every` seconds and at the end; a short
evaluation compares FGMRES iterations of M_VU and plain SL on a held-out
medium.

--plain trains one plain U-Net (no encoder; the network of M_CU in
Algorithm 2) instead, and evaluates it on 8 held-out media (seeds 90000 +
k) with the centre point source: FGMRES(20) iterations to 1e-7 with M_CU,
with M_VU and with plain SL.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

from . import helm, inputs, train, unet

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                           "pair_base.safetensors")


def make_medium(n, seed, dev):
    kap = inputs.smooth_medium(n, n / 32.0, seed=seed)
    gam = inputs.sponge_gamma(n)
    levels = max(2, int(np.log2(n // 64)) + 1)  # coarsest 64^2
    return helm.Handle(torch.from_numpy(kap).to(dev), torch.from_numpy(gam).to(dev),
                       inputs.omega_for_ppw(n), levels=levels)


def evaluate(enc, sol, n, seed, nrhs, dev):
    """Mean FGMRES(20) iterations to 1e-7: M_VU with the pair, plain SL."""
    h = make_medium(n, seed, dev)
    b = torch.from_numpy(inputs.point_sources(n, nrhs, seed=seed + 1)).to(dev)
    unet.pair_encode(enc, sol, h.coarse_slowness())
    _, st_net, _ = helm.fgmres_solve([h], [b], m=20, tol=1e-7, prec="unet_defl", net=sol)
    _, st_sl, _ = helm.fgmres_solve([h], [b], m=20, tol=1e-7)
    return (float(np.mean([s["iterations"] for s in st_net])),
            float(np.mean([s["iterations"] for s in st_sl])))


def evaluate_plain(net, n, dev, media=8):
    """Per held-out medium (seeds 90000 + k, centre source): iterations of
    FGMRES(20) to 1e-7 with M_CU, M_VU (the plain network, maxit 2000, no
    fallback) and plain SL."""
    out = []
    for k in range(media):
        h = make_medium(n, 90000 + k, dev)
        b = torch.from_numpy(inputs.point_source(n)[None]).to(dev)
        row = {"seed": 90000 + k}
        for name, prec in (("M_CU", "unet_cgc"), ("M_VU", "unet_defl"), ("M_V", "sl")):
            _, st, rc = helm.fgmres_solve([h], [b], m=20, tol=1e-7, maxit=2000, prec=prec,
                                          net=None if prec == "sl" else net)
            row[name] = st[0]["iterations"] if rc == 0 else None
        out.append(row)
        print(f"[pretrain] held-out medium {90000 + k}: " +
              ", ".join(f"{k2} {v}" for k2, v in row.items() if k2 != "seed"), flush=True)
    return out


def main_plain(a, dev):
    t_start = time.perf_counter()
    handles = [make_medium(a.n, 10000 + i, dev) for i in range(a.media)]
    torch.cuda.synchronize()
    print(f"[pretrain] {a.media} media of {a.n}^2 ready ({time.perf_counter() - t_start:.1f} s)", flush=True)
    net = unet.UNet()
    if a.resume:
        net.load_state(a.resume)
    else:
        net.init(a.seed)
    ks = a.ksteps if a.ksteps == "random" else int(a.ksteps)
    budget = a.minutes * 60.0
    t0 = time.perf_counter()
    step, chunk, hist = 0, 500, []
    while step < a.max_steps and time.perf_counter() - t0 < budget:
        k = min(chunk, a.max_steps - step)
        # consecutive chunks continue the same run: the data cursor lives in the network
        losses = train.train(net, handles, steps=k, batch=a.batch, lr=a.lr, seed=a.seed, per_medium=a.per_medium,
                             ksteps=ks, resume=step > 0 or bool(a.resume))
        step += len(losses)
        hist.extend(losses)
        print(f"[pretrain] step {step} loss {np.mean(hist[-chunk:]):.4e} ({time.perf_counter() - t0:.0f} s)",
              flush=True)
    net.save_state(a.out)
    torch.cuda.synchronize()
    print(f"[pretrain] {step} steps in {time.perf_counter() - t0:.0f} s; saved {a.out}", flush=True)
    rows = evaluate_plain(net, a.n, dev)
    for name in ("M_CU", "M_VU", "M_V"):
        v = [r[name] for r in rows]
        ok = [x for x in v if x is not None]
        print(f"[pretrain] {name}: mean {np.mean(ok) if ok else float('nan'):.1f} iterations over {len(ok)} of "
              f"{len(v)} media converged", flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--media", type=int, default=32)
    ap.add_argument("--minutes", type=float, default=15.0)
    ap.add_argument("--max-steps", type=int, default=10 ** 9)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--per-medium", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=None,
                    help="decay the learning rate linearly (in time) to this value; default constant")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--save-every", type=float, default=120.0)
    ap.add_argument("--log-every", type=int, default=500)
    ap.add_argument("--plain", action="store_true", help="train one plain U-Net (M_CU's network)")
    ap.add_argument("--ksteps", default="1", help="FGMRES steps k of eq. 3.8: an int or 'random' (1..10)")
    a = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    if a.plain:
        return main_plain(a, dev)
    t_start = time.perf_counter()
    handles = [make_medium(a.n, 10000 + i, dev) for i in range(a.media)]
    torch.cuda.synchronize()
    print(f"[pretrain] {a.media} media of {a.n}^2 ready ({time.perf_counter() - t_start:.1f} s)", flush=True)
    enc = unet.UNet(head=False)
    sol = unet.UNet(context=True)
    if a.resume:
        unet.load(a.resume, encoder=enc, solver=sol)
    else:
        enc.init(a.seed)
        sol.init(a.seed + 1)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)

    def save():
        tmp = a.out + ".tmp"
        unet.save(tmp, encoder=enc, solver=sol)
        os.replace(tmp, a.out)

    ks = a.ksteps if a.ksteps == "random" else int(a.ksteps)
    budget = a.minutes * 60.0
    t0 = time.perf_counter()
    last_save = t0
    step, chunk, hist = 0, 200, []
    while step < a.max_steps and time.perf_counter() - t0 < budget:
        k = min(chunk, a.max_steps - step)
        lr = a.lr
        if a.lr_final is not None:
            f = min(1.0, (time.perf_counter() - t0) / budget)
            lr = a.lr + (a.lr_final - a.lr) * f
        losses = train.train_pair(enc, sol, handles, steps=k, batch=a.batch, lr=lr,
                                  seed=a.seed * 100003 + step, per_medium=a.per_medium, ksteps=ks)
        # rotate the starting medium so consecutive chunks see every medium
        handles = handles[k * a.batch // a.per_medium % len(handles):] + \
            handles[:k * a.batch // a.per_medium % len(handles)]
        step += len(losses)
        hist.extend(losses)
        if step % a.log_every < chunk:
            print(f"[pretrain] step {step} loss {np.mean(hist[-chunk:]):.4e} "
                  f"({time.perf_counter() - t0:.0f} s)", flush=True)
        if time.perf_counter() - last_save > a.save_every:
            save()
            last_save = time.perf_counter()
    save()
    torch.cuda.synchronize()
    print(f"[pretrain] {step} steps in {time.perf_counter() - t0:.0f} s; saved {a.out}", flush=True)
    it_net, it_sl = evaluate(enc, sol, a.n, 90000, 4, dev)
    print(f"[pretrain] held-out {a.n}^2 medium: M_VU {it_net:.1f} iterations, SL {it_sl:.1f}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
