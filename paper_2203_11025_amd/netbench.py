"""Timing of the network application of the M_VU preconditioner alone (the
encoder-solver pair of section 3.3 at the network grid of a workload), for
profiling the convolutions under rocprofv3 (kernel trace or counters).

    python -m paper_2203_11025_amd.netbench [--workload multi1024] [--nrhs 32]
        [--reps 10] [--autotune]

One application is unet_infer on nrhs residuals (restriction, scaling, the
solver network with the encoder's shared context maps, prolongation); the
residuals are seeded complex normals.  Prints one JSON line: milliseconds per
application and the convolutions' rate from the library's live timing hook.
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
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import helm, inputs, unet

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
    print(json.dumps({"workload": a.workload, "nrhs": a.nrhs, "net_grid": n // 2, "reps": a.reps,
                      "ms_per_application": dt * 1e3, "conv_ms_per_application": ms / a.reps,
                      "conv_launches": launches, "conv_tflops": work / (ms * 1e-3) / 1e12 if ms else None,
                      "autotune": a.autotune}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
