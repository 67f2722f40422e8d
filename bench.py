#!/usr/bin/env python3
"""Benchmark: FGMRES wall seconds per right-hand side to a true (FP64)
relative residual of 1e-7 on one MI355X, U-Net + SL against plain SL.

Default workload (multi1024): 1024^2 smooth random medium (sigma 32 cells,
slowness in [0.25, 1]), 10 points per wavelength, quadratic 16-cell sponge,
32 point sources at seeded positions solved in one batched launch, FGMRES(20),
SL V(1,1) with 5 levels (coarsest 64^2 solved exactly).  The learned
preconditioner is the encoder-solver pair used as deflation beside the SL
V-cycle (M_VU, eq. 3.4 with the context of eq. 3.5), starting from the
pretrained weights when they are present (else seeded initial weights), after
200 mini-retraining Adam steps on triples of this medium (batch 16, k of
eq. 3.8 drawn from 1..10 FGMRES steps per sample, lr 1e-3).

One timed step = the encoder pass on the medium plus the complete batched
solve of all right-hand sides, inputs resident in HBM.  The plain-SL solve of
the same right-hand sides is timed the same way.  `value` is the U-Net + SL
seconds per right-hand side; the mini-retraining is timed separately and also
reported amortised over the batch.  Both solves also report the mean
convergence factor of eq. 4.1 at a 1e6 and a 1e7 residual reduction.

Prints one JSON line.  Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
DEFAULT_WEIGHTS = os.path.join(ROOT, "paper_2203_11025_amd", "weights", "pair_base.safetensors")
PROFILE_EVERY = 4  # timed launches of the dominant family: one in four

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "conv_multi1024_traffic.md")
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
FAMILIES = ("conv", "cgs", "down", "up", "apply", "coarse")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="multi1024")
    ap.add_argument("--prec", default="unet_defl", choices=["unet_defl", "unet_cgc"])
    ap.add_argument("--retrain", type=int, default=200, help="mini-retraining Adam steps")
    ap.add_argument("--retrain-lr", type=float, default=1e-3,
                    help="mini-retraining learning rate")
    ap.add_argument("--retrain-k", default="random",
                    help="FGMRES steps k of the retraining triples (eq. 3.8): an int, or 'random' for "
                         "k drawn from 1..10 per sample")
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--stall-ratio", type=float, default=0.0,
                    help="fall back to M_V on stalls (0 = never; the uneven-batch setting uses 0.95)")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured restart cycles (the timed region then cannot time the "
                         "dominant kernel family with events, so the roofline object is omitted)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the built-in convolution launch shapes instead of tuning them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of this many MiB (a reference "
                         "kernel of known traffic for hardware-counter runs)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget of the CPU oracle sample")
    return ap.parse_args()


def measured_traffic(kernel):
    """HBM bytes per launch of the convolutions from the committed counter
    runs, or None when the kernel source changed since they were taken."""
    import hashlib
    import re

    if kernel != "conv" or not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m1 = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+)", text)
    m2 = re.search(r"kernel_source_sha256: ([0-9a-f]+)", text)
    src = os.path.join(ROOT, "paper_2203_11025_amd", "csrc", "unet_kernels.hip")
    if not (m1 and m2 and os.path.exists(src)):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m2.group(1):
        return None
    return float(m1.group(1))


def rho_means(stats):
    """Mean convergence factor of eq. 4.1 over the right-hand sides at a
    1e6 and a 1e7 residual reduction (helm_fgmres_stats rho_1e6 / rho_1e7)."""
    import numpy as np

    return {"rho_1e6_mean": float(np.mean([s["rho_1e6"] for s in stats])),
            "rho_1e7_mean": float(np.mean([s["rho_1e7"] for s in stats]))}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(P, enc, sol, prec, gpu_iterations, budget_s):
    """The oracle on this host: the first K iterations of the same U-Net + SL
    FGMRES solve of the first right-hand side (FP64 C sweeps and Krylov
    method, FP32 PyTorch CPU network with the GPU's current weights), scaled
    to seconds per right-hand side by the GPU solve's iteration count."""
    import numpy as np
    import torch

    from oracle import helm_oracle
    from oracle import unet_oracle as U

    ce = U.UNetCfg(in_ch=1, widths=enc.widths, head=False)
    cs = U.UNetCfg(in_ch=3, widths=sol.widths, context=True)
    pe, be = enc.get_params()
    ps, bs = sol.get_params()
    pe, ps = U.unflatten(ce, pe.cpu()), U.unflatten(cs, ps.cpu())
    def bufs(cfg, flat):
        out, off = {}, 0
        for k, shape in U.buffer_shapes(cfg).items():
            cnt = int(np.prod(shape))
            out[k] = flat[off:off + cnt].reshape(shape).clone()
            off += cnt
        return out
    be, bs = bufs(ce, be.cpu()), bufs(cs, bs.cpu())
    t_all = time.perf_counter()
    H = helm_oracle.Hierarchy(P["kappa"], P["gamma"], P["omega"], P["levels"])
    kc = P["kappa"].astype(np.float64)[::2, ::2]
    ctx = U.encode(ce, pe, be, kc)
    if prec == "unet_defl":
        f = lambda v: U.precond_defl(H, cs, ps, bs, v, kc, ctx=ctx)
    else:
        f = lambda v: U.precond_cgc(H, cs, ps, bs, v, kc, ctx=ctx)
    b = P["b"][0]
    t0 = time.perf_counter()
    H.fgmres(b, m=P["m"], tol=1e-30, maxit=1, prec=f)
    t1 = time.perf_counter() - t0
    k = int(max(1, min(gpu_iterations, (budget_s - (time.perf_counter() - t_all)) / max(t1, 1e-6))))
    t0 = time.perf_counter()
    H.fgmres(b, m=P["m"], tol=1e-30, maxit=k, prec=f)
    dt = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": dt / k * gpu_iterations,
        "unit": "s/RHS",
        "cores": torch.get_num_threads(),
        "cpu_model": model,
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": f"first {k} FGMRES({P['m']}) iterations of the same {P['n']}^2 {prec} solve of one "
                  f"right-hand side ({dt:.1f} s; FP64 C sweeps on one core, FP32 PyTorch CPU network "
                  f"on {torch.get_num_threads()} threads), scaled by the GPU solve's "
                  f"{gpu_iterations} iterations",
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are "
                          "not implemented (the path shards by medium and right-hand side "
                          "with no exchange)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2203_11025_amd import helm, inputs, train, unet

    def sync():
        torch.cuda.synchronize()

    P = inputs.config_problem(a.workload)
    dev = torch.device("cuda:0")
    if a.copy_probe:
        src = torch.ones(a.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        sync()
        del src, dst
    t_setup = time.perf_counter()
    kap = torch.from_numpy(P["kappa"]).to(dev)
    gam = torch.from_numpy(P["gamma"]).to(dev)
    b = torch.from_numpy(P["b"]).to(dev)
    nrhs = b.shape[0]
    h = helm.Handle(kap, gam, P["omega"], levels=P["levels"])
    sync()
    t_setup = time.perf_counter() - t_setup
    log(f"setup n={P['n']} levels={h.levels} nrhs={nrhs} ({t_setup:.2f} s)")

    if not a.no_autotune:
        helm.autotune(1)
    enc = unet.UNet(head=False)
    sol = unet.UNet(context=True)
    pretrained = os.path.exists(a.weights)
    if pretrained:
        unet.load(a.weights, encoder=enc, solver=sol)
    else:
        enc.init(1)
        sol.init(2)
    log(f"network: {'pretrained ' + os.path.basename(a.weights) if pretrained else 'seeded init'}")

    # mini-retraining on the medium (section 3.4), timed on its own
    sync()
    t0 = time.perf_counter()
    rk = a.retrain_k if a.retrain_k == "random" else int(a.retrain_k)
    losses = train.train_pair(enc, sol, [h], steps=a.retrain, batch=16, lr=a.retrain_lr, seed=11, ksteps=rk)
    sync()
    t_retrain = time.perf_counter() - t0
    if losses:
        log(f"retrain {a.retrain} steps {t_retrain:.1f} s loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    kc = h.coarse_slowness()
    x = torch.empty(b.shape, dtype=torch.complex128, device=dev)

    graph = a.graph

    def solve_net():
        unet.pair_encode(enc, sol, kc)
        return helm.fgmres_solve([h], [b], m=P["m"], tol=P["tol"], prec=a.prec, net=sol,
                                 stall_ratio=a.stall_ratio, xs=[x], graph=graph)

    def solve_sl():
        return helm.fgmres_solve([h], [b], m=P["m"], tol=P["tol"], xs=[x], graph=graph)

    # warmup; the first U-Net + SL pass also profiles every kernel family to
    # find the dominant one
    for i in range(a.warmup):
        if i == 0:
            helm.profile_start(*FAMILIES)
        _, st, _ = solve_net()
        if i == 0:
            fam = {f: helm.profile_read(f) for f in FAMILIES}
            helm.profile_stop()
        log(f"warmup {i} U-Net+SL its mean {np.mean([s['iterations'] for s in st]):.1f}")
        _, st, _ = solve_sl()
        log(f"warmup {i} SL its mean {np.mean([s['iterations'] for s in st]):.1f}")
    sync()
    if a.warmup == 0:
        fam = {"conv": (1.0, 1, 0.0)}
    dominant = max(fam, key=lambda f: fam[f][0])

    # timed: U-Net + SL, the dominant kernel family timed live with HIP events
    # on every PROFILE_EVERY-th launch (each event pair costs a few
    # microseconds of queue time; not with graph replay: the events cannot be
    # re-recorded inside a graph)
    if not graph:
        helm.profile_start(dominant, every=PROFILE_EVERY)
    sync()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        _, st_net, rc_net = solve_net()
    sync()
    dt_net = time.perf_counter() - t0
    d_ms, d_launches, d_work = helm.profile_read(dominant) if not graph else (0.0, 0, 0.0)
    helm.profile_stop()
    its_net = [s["iterations"] for s in st_net]
    relres_net = max(s["true_relres"] for s in st_net)
    log(f"timed U-Net+SL: {dt_net / a.steps * 1e3:.1f} ms/step its mean {np.mean(its_net):.1f} "
        f"relres {relres_net:.2e}")

    # timed: plain SL on the same right-hand sides
    sync()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        _, st_sl, rc_sl = solve_sl()
    sync()
    dt_sl = time.perf_counter() - t0
    its_sl = [s["iterations"] for s in st_sl]
    relres_sl = max(s["true_relres"] for s in st_sl)
    log(f"timed SL: {dt_sl / a.steps * 1e3:.1f} ms/step its mean {np.mean(its_sl):.1f} "
        f"relres {relres_sl:.2e}")

    # the SL sweep families, profiled over one extra plain-SL solve
    helm.profile_start(*FAMILIES[1:])
    solve_sl()
    sweeps = {}
    for f in FAMILIES[1:]:
        ms, n_l, work = helm.profile_read(f)
        if n_l:
            gbs = work / (ms / 1e3) / 1e9
            sweeps[f] = {"achieved_GBs": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 3),
                         "avg_launch_us": round(ms * 1e3 / n_l, 2), "launches": n_l}
    helm.profile_stop()

    ms_per_step = dt_net * 1000.0 / a.steps
    value = ms_per_step / 1000.0 / nrhs
    sl_value = dt_sl / a.steps / nrhs
    unit_is_flops = dominant in ("conv", "wgrad")
    avg_s = max(d_ms / 1e3 / max(d_launches, 1), 1e-12)
    if unit_is_flops:
        achieved = d_work / max(d_launches, 1) / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_BF16_TFLOPS}
    else:
        achieved = d_work / max(d_launches, 1) / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    roof.update({"traffic": measured_traffic(dominant), "kernel": dominant, "avg_launch_us": avg_s * 1e6,
                 "launches": d_launches, "sampled_every": PROFILE_EVERY, "work_per_launch": d_work / max(d_launches, 1),
                 "time_share_warmup": round(fam[dominant][0] / sum(v[0] for v in fam.values()), 3)})
    out = {
        "metric": "FGMRES secs to rel-res 1e-7 per RHS: U-Net+SL vs plain SL",
        "value": value,
        "unit": "s/RHS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+bf16",
        "data": "synthetic",
        "config": {
            "workload": f"{P['n']}^2 smooth medium (sigma {P.get('sigma', '-')}), {nrhs} point sources "
                        f"in one batch, FGMRES({P['m']}) to true relres {P['tol']:g}; U-Net+SL = "
                        f"{a.prec} with the encoder-solver pair; SL = V(1,1) {h.levels} levels",
            "n": P["n"], "nrhs": nrhs, "prec": a.prec,
            "network": "pretrained" if pretrained else "seeded init",
            "retrain_steps": a.retrain, "retrain_lr": a.retrain_lr, "retrain_k": a.retrain_k, "graph": graph, "autotune": not a.no_autotune,
        },
        "unet_sl": {"s_per_rhs": value, "iterations_mean": float(np.mean(its_net)),
                    "iterations_max": int(max(its_net)), "true_relres_max": relres_net,
                    **rho_means(st_net),
                    "fallbacks": int(sum(s["fallback"] for s in st_net)), "status": rc_net},
        "plain_sl": {"s_per_rhs": sl_value, "iterations_mean": float(np.mean(its_sl)),
                     "iterations_max": int(max(its_sl)), "true_relres_max": relres_sl,
                     **rho_means(st_sl), "status": rc_sl},
        "speedup_vs_plain_sl": sl_value / value,
        "retrain": {"steps": a.retrain, "seconds": t_retrain,
                    "loss_first": losses[0] if losses else None,
                    "loss_last": losses[-1] if losses else None},
        "value_amortized": value + (t_retrain + t_setup) / nrhs,
        "setup_s": t_setup,
        "roofline": roof if d_launches else None,
        "sweeps": sweeps,
    }
    if not a.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(P, enc, sol, a.prec, its_net[0], a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
