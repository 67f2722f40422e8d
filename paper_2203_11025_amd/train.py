"""Training loop of the U-Net preconditioner (section 3.4): triples made on
the device by k SL-FGMRES steps (eq. 3.8-3.9) from x drawn by the library's
counter-based generator, optional augmentation by linear combinations, the
scaled error loss (eq. 3.7) and Adam, all in the library's kernels.

A run is reproducible from the network's training-data cursor (seed,
position): the sample at position p of the run is drawn from (seed, index
i(p)) and comes from medium (i // per_medium) mod (number of media).  With a
fixed data set of S samples (`dataset`), i(p) follows a seeded permutation of
0..S-1 per epoch; without one, i(p) = p (fresh samples).  unet_save /
unet_load keep the cursor with the weights and the Adam state, so a resumed
run continues bit for bit.  The batch tensors are allocated once and filled
in place by the library (no framework compute on the path); host code only
picks indices, k and mixing coefficients.
"""
from __future__ import annotations

import time

import numpy as np
import torch


def paper_schedule(epoch, lr0=1e-4, batch0=20, t0=48):
    """Learning rate and mini-batch size at an epoch (section 4): after t0
    epochs the rate is divided by 10 and the batch doubled, and again after
    each further t0 / 2^i epochs (changes at 48, 72, 84, 90, 93, ...), while
    the interval is at least one epoch."""
    changes, t, edge = 0, float(t0), float(t0)
    while epoch >= edge and t >= 1.0:
        changes += 1
        t /= 2.0
        edge += t
    return lr0 / 10.0 ** changes, batch0 * 2 ** changes


def _mix64(a, b):
    """splitmix64 of two words (host-side choices: k, permutations, mixing)."""
    z = (a * 0x9E3779B97F4A7C15 + b + 0x632BE59BD9B4E019) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


class Batches:
    """Fills preallocated (r, e, kappa_c) batch tensors from a list of media
    of one grid size."""

    def __init__(self, handles, batch, per_medium=None, ksteps=1, dataset=None, augment=False):
        n = handles[0].n
        if any(h.n != n for h in handles):
            raise ValueError("all media of a training run must have one grid size")
        if not (ksteps == "random" or 1 <= int(ksteps) <= 30):
            raise ValueError("ksteps: an int in [1, 30] or 'random' (1..10 per sample)")
        self.handles = handles
        self.n = n
        self.per_medium = per_medium or batch
        self.ksteps = ksteps
        self.dataset = dataset
        self.augment = augment
        self.alloc(batch)

    def alloc(self, batch):
        n = self.n
        self.batch = batch
        self.r = torch.empty((batch, n, n), dtype=torch.complex64, device="cuda")
        self.e = torch.empty_like(self.r)
        self.kc = torch.empty((batch, n // 2, n // 2), dtype=torch.float32, device="cuda")
        if self.augment:
            self.r2 = torch.empty_like(self.r)
            self.e2 = torch.empty_like(self.r)

    def index(self, seed, pos):
        if self.dataset is None:
            return pos
        S = self.dataset
        ep, j = divmod(pos, S)
        perm = np.random.default_rng(_mix64(seed, 0x5EED0000 + ep)).permutation(S)
        return int(perm[j])

    def k_of(self, seed, i):
        if self.ksteps == "random":
            return 1 + _mix64(seed ^ 0x4B4B4B4B, i) % 10
        return int(self.ksteps)

    def fill(self, seed, pos0):
        """The batch of positions pos0 .. pos0 + batch - 1 of the run."""
        idx = [self.index(seed, pos0 + b) for b in range(self.batch)]
        med = [(i // self.per_medium) % len(self.handles) for i in idx]
        order = sorted(range(self.batch), key=lambda b: med[b])  # medium groups contiguous
        idx = [idx[b] for b in order]
        med = [med[b] for b in order]
        b = 0
        while b < self.batch:
            h = self.handles[med[b]]
            if self.ksteps == "random":
                # every sample of one medium in one call, each with its own k
                c = 1
                while b + c < self.batch and med[b + c] == med[b]:
                    c += 1
                h.training_triples_batch(seed, idx[b:b + c], [self.k_of(seed, i) for i in idx[b:b + c]],
                                         self.r[b:b + c], self.e[b:b + c])
            else:
                # a run of consecutive indices from one medium per call
                c = 1
                while b + c < self.batch and med[b + c] == med[b] and idx[b + c] == idx[b] + c:
                    c += 1
                h.training_triples_seeded(seed, idx[b], self.r[b:b + c], self.e[b:b + c],
                                          ksteps=self.k_of(seed, idx[b]))
            for j in range(b, b + c):
                h.coarse_slowness(out=self.kc[j])
            b += c
        if self.augment:
            self._mix(seed, pos0, med)
        # the batch's one medium (None when it mixes media)
        self.medium = med[0] if all(m == med[0] for m in med) else None
        return self.r, self.e, self.kc

    def _mix(self, seed, pos0, med):
        """Replace each medium group of the batch by a random orthogonal
        combination of its triples (section 3.4's augmentation), written by
        the library into the second buffer pair, which then becomes the
        batch."""
        from .helm import triples_mix

        b = 0
        while b < self.batch:
            g = 1  # a group of at most 32 samples of one medium
            while b + g < self.batch and med[b + g] == med[b] and g < 32:
                g += 1
            q = np.ones((1, 1))
            if g > 1:
                rng = np.random.default_rng(_mix64(seed ^ 0xA06A06, pos0 + b))
                q, t = np.linalg.qr(rng.standard_normal((g, g)))
                q = q * np.sign(np.diag(t))[None, :]  # Haar-distributed orthogonal
            coef = torch.from_numpy(q.astype(np.float32)).cuda()
            triples_mix(self.r[b:b + g], self.e[b:b + g], coef, self.r2[b:b + g], self.e2[b:b + g])
            b += g
        self.r, self.r2 = self.r2, self.r
        self.e, self.e2 = self.e2, self.e


def _run(step_fn, net, handles, steps, batch, lr, seed, per_medium, log, time_budget, resume,
         ksteps=1, dataset=None, augment=False, schedule=None):
    """Common loop.  With `schedule` (a function epoch -> (lr, batch), e.g.
    paper_schedule) and a `dataset` size, `steps` counts epochs instead of
    Adam steps, and each epoch sweeps the data set once."""
    if not resume:
        net.set_cursor(seed, 0)
    seed, pos = net.cursor()
    data = Batches(handles, batch, per_medium, ksteps, dataset, augment)
    losses = []
    t0 = time.perf_counter()

    def one(lr_):
        nonlocal pos
        r, e, kc = data.fill(seed, pos)
        pos += data.batch
        net.set_cursor(seed, pos)
        losses.append(step_fn(r, e, kc, lr_, data))

    if schedule is None:
        for step in range(steps):
            one(lr)
            if log and (step % log == 0 or step == steps - 1):
                print(f"[train] step {step} loss {losses[-1]:.4e} ({time.perf_counter() - t0:.1f} s)",
                      flush=True)
            if time_budget is not None and time.perf_counter() - t0 > time_budget:
                break
        return losses
    if dataset is None:
        raise ValueError("a schedule needs a data-set size (epochs sweep it)")
    for _ in range(steps):
        epoch = pos // dataset
        lr_e, batch_e = schedule(epoch)
        if batch_e != data.batch:
            data.alloc(batch_e)
        end = (epoch + 1) * dataset
        while pos + data.batch <= end:
            one(lr_e)
        pos = end  # a last partial batch is dropped
        net.set_cursor(seed, pos)
        if log:
            print(f"[train] epoch {epoch} lr {lr_e:.1e} batch {batch_e} loss {np.mean(losses[-3:]):.4e} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
    return losses


def train_pair(encoder, solver, handles, steps, batch=16, lr=1e-3, seed=0, per_medium=None, log=None,
               time_budget=None, resume=False, ksteps=1, dataset=None, augment=False, schedule=None):
    """Joint Adam steps of an encoder-solver pair on triples (eq. 3.8-3.9)
    from the given media of one grid size; each batch takes `per_medium`
    consecutive samples from one medium (all from one medium by default, the
    mini-retraining setting).  The data cursor lives in the solver;
    resume=True continues from it, else the run starts at (seed, 0).
    Returns the list of losses."""
    from .unet import pair_train_step

    def step_fn(r, e, kc, lr_, data):
        return pair_train_step(encoder, solver, r, e, kc, lr=lr_)

    return _run(step_fn, solver, handles, steps, batch, lr, seed, per_medium, log, time_budget, resume,
                ksteps, dataset, augment, schedule)


def train(net, handles, steps, batch=16, lr=1e-3, seed=0, per_medium=None, log=None, time_budget=None,
          resume=False, ksteps=1, dataset=None, augment=False, schedule=None):
    """Adam steps of one network on triples from the given media (one grid
    size).  Returns the list of losses; stops early when `time_budget`
    seconds have elapsed."""

    def step_fn(r, e, kc, lr_, data):
        if getattr(net, "arch", 0) == 1:
            # the paper's network reads the fine medium: one medium per batch
            if data.medium is None:
                raise ValueError("the paper's network trains on batches of one medium (per_medium >= batch)")
            h = handles[data.medium]
            return net.train_step(r, e, kc, lr=lr_, kappa_f=h._keep[0], gamma_f=h._keep[1])
        return net.train_step(r, e, kc, lr=lr_)

    return _run(step_fn, net, handles, steps, batch, lr, seed, per_medium, log, time_budget, resume,
                ksteps, dataset, augment, schedule)
