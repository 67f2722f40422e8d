"""Timing of one part of the solve in isolation, for profiling under
rocprofv3 (kernel trace or counters):

    python -m paper_2203_11025_amd.netbench [--mode net|sl] [--workload multi1024]
        [--nrhs 32] [--reps 10] [--autotune] [--copy-probe MIB]

--mode net: one application is unet_infer on nrhs residuals (restriction,
scaling, the encoder-solver's solver network with the encoder's shared
context maps, prolongation), the network application of M_VU (eq. 3.4).
--mode sl: one application is one FGMRES(20) cycle (maxit 20) with the SL
V-cycle on nrhs point sources: 20 V-cycles, 20 operator applications and 20
Arnoldi steps, the x update and the true residual.
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
    ap.add_argument("--mode", default="net", choices=["net", "sl"])
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


if __name__ == "__main__":
    sys.exit(main())
