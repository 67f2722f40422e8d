"""Timing of one part of the solve in isolation, for profiling under
rocprofv3 (kernel trace or counters):

    python -m paper_2203_11025_amd.netbench [--mode net|sl|uneven|retrain|papernet] [--workload multi1024]
        [--nrhs 32] [--reps 10] [--autotune] [--graph] [--copy-probe MIB]

--mode net: one application is unet_infer on nrhs residuals (restriction,
scaling, the encoder-solver's solver network with the encoder's shared
context maps, prolongation), the network application of M_VU (eq. 3.4).
--mode sl: one application is one FGMRES(20) cycle (maxit 20) with the SL
V-cycle on nrhs point sources: 20 V-cycles, 20 operator applications and 20
Arnoldi steps, the x update and the true residual.
--mode retrain: reps mini-retraining steps of the encoder-solver pair on
the medium (batch 16, k of eq. 3.8 drawn from 1..10 per sample, lr 1e-3:
the benchmark's retraining), after one untimed step; prints the split of a
step between the triples and the Adam step, and the rates of the weight-
gradient and the other convolutions from the library's timing hook.
--mode papernet: the paper's network (section 3.1; widths 16..128, 4
levels) on an n x n grid (--n, default 128) for a batch of --nrhs samples:
milliseconds per inference forward pass and per training step (forward,
loss, backward, Adam), with the convolutions' FLOPs counted as 2 per
multiply-add.
--mode uneven: the uneven batch (--workload uneven24 or uneven6: many
layered media of 256^2..2048^2, 8 point sources each) solved in one
helm_fgmres_solve call, first with the encoder-solver M_VU (each medium
encoded in turn, plain-SL fallback at a residual ratio of 0.95, --graph for
replayed restart cycles), then with plain SL (problems run concurrently);
reps timed solves of each.
The inputs are seeded.  --copy-probe first copies a buffer of that many MiB
once (a plain copy kernel of known size, to scale HBM counters by).  Prints
one JSON line: milliseconds per application (and, for the network, the
convolutions' rate from the library's live timing hook).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "pair_base.safetensors")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="multi1024")
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--mode", default="net", choices=["net", "sl", "uneven", "retrain", "papernet"])
    ap.add_argument("--graph", action="store_true")
    ap.add_argument("--n", type=int, default=128, help="--mode papernet: fine grid")
    ap.add_argument("--uneven-prec", default="both", choices=["both", "unet", "sl"],
                    help="--mode uneven: which solves to time")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import helm, inputs, unet

    if a.copy_probe:
        src = torch.ones(a.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.mode == "uneven":
        return uneven(a)
    if a.mode == "retrain":
        return retrain(a)
    if a.mode == "papernet":
        return papernet(a)
    P = inputs.config_problem(a.workload)
    h = helm.Handle(torch.from_numpy(P["kappa"]).cuda(), torch.from_numpy(P["gamma"]).cuda(), P["omega"],
                    levels=P["levels"])
    helm.autotune(1 if a.autotune else 0)
    if a.mode == "sl":
        b = torch.from_numpy(inputs.point_sources(P["n"], a.nrhs, seed=3)).cuda()
        x = torch.empty(b.shape, dtype=torch.complex128, device="cuda")
        helm.fgmres_solve([h], [b], m=20, tol=P["tol"], maxit=20, xs=[x])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(a.reps):
            helm.fgmres_solve([h], [b], m=20, tol=P["tol"], maxit=20, xs=[x])
            print(f"[netbench] cycle {i}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.reps
        print(json.dumps({"mode": "sl", "workload": a.workload, "nrhs": a.nrhs, "reps": a.reps,
                          "ms_per_cycle": dt * 1e3, "ms_per_iteration": dt * 1e3 / 20}))
        return 0
    enc, sol = unet.UNet(head=False), unet.UNet(context=True)
    if os.path.exists(a.weights):
        unet.load(a.weights, encoder=enc, solver=sol)
    else:
        enc.init(1)
        sol.init(2)
    unet.pair_encode(enc, sol, h.coarse_slowness())
    n = P["n"]
    rng = np.random.default_rng(5)
    r = torch.from_numpy((rng.standard_normal((a.nrhs, n, n), dtype=np.float32)
                          + 1j * rng.standard_normal((a.nrhs, n, n), dtype=np.float32)).astype(np.complex64)).cuda()
    sol.infer(h, r)  # warm-up (and tuning, with --autotune)
    torch.cuda.synchronize()
    helm.profile_start("conv")
    t0 = time.perf_counter()
    for i in range(a.reps):
        sol.infer(h, r)
        print(f"[netbench] application {i}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.reps
    ms, launches, work = helm.profile_read("conv")
    helm.profile_stop()
    print(json.dumps({"mode": "net", "workload": a.workload, "nrhs": a.nrhs, "net_grid": n // 2, "reps": a.reps,
                      "ms_per_application": dt * 1e3, "conv_ms_per_application": ms / a.reps,
                      "conv_launches": launches, "conv_tflops": work / (ms * 1e-3) / 1e12 if ms else None,
                      "autotune": a.autotune}))
    return 0


def retrain(a):
    import torch

    from . import helm, inputs, train, unet

    P = inputs.config_problem(a.workload)
    h = helm.Handle(torch.from_numpy(P["kappa"]).cuda(), torch.from_numpy(P["gamma"]).cuda(), P["omega"],
                    levels=P["levels"])
    helm.autotune(1 if a.autotune else 0)
    enc, sol = unet.UNet(head=False), unet.UNet(context=True)
    if os.path.exists(a.weights):
        unet.load(a.weights, encoder=enc, solver=sol)
    else:
        enc.init(1)
        sol.init(2)
    data = train.Batches([h], 16, ksteps="random")
    r, e, kc = data.fill(11, 0)
    unet.pair_train_step(enc, sol, r, e, kc, lr=1e-3)
    torch.cuda.synchronize()
    helm.profile_start("wgrad", "conv")
    t_data = t_step = 0.0
    for i in range(a.reps):
        t0 = time.perf_counter()
        r, e, kc = data.fill(11, 16 * (i + 1))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = unet.pair_train_step(enc, sol, r, e, kc, lr=1e-3)
        torch.cuda.synchronize()
        t_data += t1 - t0
        t_step += time.perf_counter() - t1
        print(f"[netbench] retrain step {i} loss {loss:.3e}", file=sys.stderr, flush=True)
    wms, wn, ww = helm.profile_read("wgrad")
    cms, cn, cw = helm.profile_read("conv")
    helm.profile_stop()
    print(json.dumps({"mode": "retrain", "workload": a.workload, "batch": 16, "reps": a.reps,
                      "ms_per_step": (t_data + t_step) * 1e3 / a.reps, "ms_triples": t_data * 1e3 / a.reps,
                      "ms_adam_step": t_step * 1e3 / a.reps, "autotune": a.autotune,
                      "wgrad_ms_per_step": wms / a.reps, "wgrad_tflops": ww / (wms * 1e-3) / 1e12 if wms else None,
                      "conv_ms_per_step": cms / a.reps, "conv_tflops": cw / (cms * 1e-3) / 1e12 if cms else None}))
    return 0


def papernet_flops(n, widths=(16, 32, 64, 128), cin=4, cout=2, coarsest_blocks=3):
    """FLOPs of one forward pass of the paper's network for one sample."""
    L = len(widths)
    f, c = 0.0, cin
    for l in range(1, L + 1):
        m = (n >> l) ** 2
        f += 2 * 25 * c * widths[l - 1] * m  # 5x5 stride-2 convolution
        f += (coarsest_blocks if l == L else 1) * 2 * (2 * 9 * widths[l - 1] ** 2 * m)  # ResNet blocks
        c = widths[l - 1]
    ch = widths[L - 1]
    for l in range(L - 1, 0, -1):  # transposed 5x5: every input point scatters to K^2 outputs
        f += 2 * 25 * ch * widths[l - 1] * (n >> (l + 1)) ** 2
        ch = 2 * widths[l - 1]
    f += 2 * 25 * ch * cout * (n >> 1) ** 2
    return f


def papernet(a):
    import numpy as np
    import torch

    from . import helm, inputs, unet

    n, B = a.n, a.nrhs
    widths = (16, 32, 64, 128)
    net = unet.UNet(widths=widths, arch=1)
    net.init(1)
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.standard_normal((B, 4, n, n), dtype=np.float32)).cuda()
    net.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.reps):
        net.forward(x)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / a.reps
    kap = torch.from_numpy(inputs.smooth_medium(n, max(2.0, n / 16), seed=1)).cuda()
    gam = torch.from_numpy(inputs.sponge_gamma(n, width=min(16, n // 8))).cuda()
    r = torch.from_numpy((rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))).astype(np.complex64)).cuda()
    e = torch.from_numpy((rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))).astype(np.complex64)).cuda()
    net.train_step(r, e, None, lr=1e-4, kappa_f=kap, gamma_f=gam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.reps):
        net.train_step(r, e, None, lr=1e-4, kappa_f=kap, gamma_f=gam)
        print(f"[netbench] papernet train step {i}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / a.reps
    f = papernet_flops(n, widths) * B
    print(json.dumps({"mode": "papernet", "n": n, "batch": B, "reps": a.reps, "gflop_forward": f / 1e9,
                      "ms_forward": t_fwd * 1e3, "tflops_forward": f / t_fwd / 1e12,
                      "ms_train_step": t_train * 1e3, "tflops_train_step": 3 * f / t_train / 1e12}))
    return 0


def uneven(a):
    import numpy as np
    import torch

    from . import helm, inputs, unet

    P = inputs.config_problems(a.workload)
    hs = [helm.Handle(torch.from_numpy(p["kappa"]).cuda(), torch.from_numpy(p["gamma"]).cuda(), p["omega"],
                      levels=p["levels"]) for p in P]
    bs = [torch.from_numpy(p["b"]).cuda() for p in P]
    xs = [torch.empty(b.shape, dtype=torch.complex128, device="cuda") for b in bs]
    enc, sol = unet.UNet(head=False), unet.UNet(context=True)
    if os.path.exists(a.weights):
        unet.load(a.weights, encoder=enc, solver=sol)
    else:
        enc.init(1)
        sol.init(2)
    helm.autotune(1 if a.autotune else 0)
    nrhs = sum(b.shape[0] for b in bs)
    out = {"mode": "uneven", "workload": a.workload, "media": len(P), "sizes": [p["n"] for p in P], "nrhs": nrhs,
           "reps": a.reps, "graph": a.graph, "autotune": a.autotune}
    runs = (("unet_sl", dict(prec="unet_defl", net=sol, encoder=enc, stall_ratio=0.95, graph=a.graph)),
            ("plain_sl", dict(prec="sl", graph=a.graph)))
    for name, kw in runs:
        if (a.uneven_prec == "unet" and name != "unet_sl") or (a.uneven_prec == "sl" and name != "plain_sl"):
            continue
        _, st, rc = helm.fgmres_solve(hs, bs, m=20, tol=1e-7, xs=xs, **kw)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(a.reps):
            _, st, rc = helm.fgmres_solve(hs, bs, m=20, tol=1e-7, xs=xs, **kw)
            torch.cuda.synchronize()
            print(f"[netbench] {name} solve {i} rc {rc}", file=sys.stderr, flush=True)
        dt = (time.perf_counter() - t0) / a.reps
        its, off, per = [s["iterations"] for s in st], 0, []
        for p, b in zip(P, bs):
            k = b.shape[0]
            per.append({"n": p["n"], "its_mean": float(np.mean(its[off:off + k])),
                        "fallbacks": int(sum(s["fallback"] for s in st[off:off + k]))})
            off += k
        out[name] = {"s_per_solve": dt, "s_per_rhs": dt / nrhs, "status": rc,
                     "iterations_mean": float(np.mean(its)),
                     "true_relres_max": float(max(s["true_relres"] for s in st)),
                     "fallbacks": int(sum(s["fallback"] for s in st)), "per_medium": per}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
