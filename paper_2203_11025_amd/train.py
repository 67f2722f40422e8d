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


def _pair_batch(handles, kcs, k0, batch, per_medium, gen):
    """Triples from batch / per_medium consecutive media (cycled from k0),
    with each sample's coarse slowness."""
    rs, es, ks = [], [], []
    k = k0
    while sum(r.shape[0] for r in rs) < batch:
        h = handles[k % len(handles)]
        cnt = min(per_medium, batch - sum(r.shape[0] for r in rs))
        r, e = h.training_triples(random_x(cnt, h.n, gen))
        rs.append(r)
        es.append(e)
        ks.append(kcs[k % len(handles)].unsqueeze(0).expand(cnt, -1, -1))
        k += 1
    return torch.cat(rs), torch.cat(es), torch.cat(ks).contiguous(), k


def train_pair(encoder, solver, handles, steps, batch=16, lr=1e-3, seed=0, per_medium=None, log=None,
               time_budget=None):
    """Joint Adam steps of an encoder-solver pair on fresh triples (eq.
    3.8-3.9) from the given media of one grid size; each batch takes
    `per_medium` samples from consecutive media (all from one medium by
    default, the mini-retraining setting).  Returns the list of losses."""
    from .unet import pair_train_step

    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    kcs = [h.coarse_slowness() for h in handles]
    per_medium = per_medium or batch
    losses = []
    t0 = time.perf_counter()
    k = 0
    for step in range(steps):
        r, e, kc, k = _pair_batch(handles, kcs, k, batch, per_medium, gen)
        losses.append(pair_train_step(encoder, solver, r, e, kc, lr=lr))
        if log and (step % log == 0 or step == steps - 1):
            print(f"[train] step {step} loss {losses[-1]:.4e} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
    return losses


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
