"""Training loop of the U-Net preconditioner (section 3.4): triples made on
the device by one SL-FGMRES step (eq. 3.8-3.9), the scaled error loss
(eq. 3.7) and Adam, all in the library's kernels.  The random vectors x are
drawn with torch's seeded device generator and passed in."""
from __future__ import annotations

import time

import torch


def random_x(batch, n, gen):
    """complex64 [batch, n, n] with iid N(0, 1) real and imaginary parts."""
    re = torch.randn((batch, n, n), device="cuda", generator=gen)
    im = torch.randn((batch, n, n), device="cuda", generator=gen)
    return torch.complex(re, im).contiguous()


def train(net, handles, steps, batch=16, lr=1e-3, seed=0, log=None, time_budget=None):
    """Adam steps on fresh triples from the given media (cycled).  Returns the
    list of losses.  Stops early when `time_budget` seconds have elapsed."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    kcs = [h.coarse_slowness() for h in handles]
    losses = []
    t0 = time.perf_counter()
    for step in range(steps):
        k = step % len(handles)
        h = handles[k]
        x = random_x(batch, h.n, gen)
        r, e = h.training_triples(x)
        kc = kcs[k].unsqueeze(0).expand(batch, -1, -1).contiguous()
        losses.append(net.train_step(r, e, kc, lr=lr))
        if log and (step % log == 0 or step == steps - 1):
            print(f"[train] step {step} loss {losses[-1]:.4e} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
    return losses
