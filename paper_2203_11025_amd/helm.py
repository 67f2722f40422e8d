"""ctypes binding of libhelm (include/helm.h).  Argument marshalling only:
every step of the solver runs in the library's HIP kernels.  PyTorch supplies
device memory and the current stream.

The library must have been built (python -m paper_2203_11025_amd.build);
loading fails loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelm.so")

HELM_OK = 0
HELM_NOT_CONVERGED = 1
HELM_OP_A = 0
HELM_OP_M = 1
PREC = {"sl": 0, "unet_cgc": 1, "unet_defl": 2}

EXPORTS = [
    "helm_setup", "helm_destroy", "helm_level_size", "helm_num_levels", "helm_apply",
    "helm_sl_vcycle", "helm_fgmres_solve", "helm_last_error", "helm_profile_start",
    "helm_profile_read", "helm_profile_stop", "helm_profile_sample", "helm_autotune", "helm_autotune_entries", "helm_autotune_force", "helm_training_triples", "helm_coarse_slowness",
    "helm_sl_vcycle_noalloc", "helm_sl_vcycle_noalloc_bytes", "helm_sl_vcycle_noalloc_max_bytes",
    "helm_training_triples_seeded", "helm_set_allocator", "helm_allocated_bytes", "helm_triples_mix",
    "helm_block_fgmres_solve", "helm_training_triples_batch",
]
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)
PROF = {"none": 0, "coarse": 1, "down": 2, "up": 3, "cgs": 4, "apply": 5, "conv": 6, "wgrad": 7}


class HelmError(RuntimeError):
    pass


class _Opts(C.Structure):
    _fields_ = [("beta", C.c_double), ("jacobi_weight", C.c_double), ("levels", C.c_int),
                ("coarse_gmres", C.c_int)]


class FgmresOpts(C.Structure):
    _fields_ = [("m", C.c_int), ("tol", C.c_double), ("maxit", C.c_int), ("prec", C.c_int),
                ("net", C.c_void_p), ("stall_ratio", C.c_double), ("graph", C.c_int),
                ("encoder", C.c_void_p)]


class FgmresStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("fallback", C.c_int), ("true_relres", C.c_double), ("its_1e6", C.c_int),
                ("its_1e7", C.c_int), ("rho_1e6", C.c_double), ("rho_1e7", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HelmError(f"{LIB_PATH} is missing: build it with "
                            "`python -m paper_2203_11025_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.c_int, C.c_double
        L.helm_setup.argtypes = [vp, dp, vp, ip, C.POINTER(_Opts), vp, C.POINTER(vp)]
        L.helm_setup.restype = ip
        L.helm_destroy.argtypes = [vp]
        L.helm_destroy.restype = None
        L.helm_level_size.argtypes = [vp, ip]
        L.helm_level_size.restype = ip
        L.helm_num_levels.argtypes = [vp]
        L.helm_num_levels.restype = ip
        L.helm_apply.argtypes = [vp, ip, vp, vp, ip, vp]
        L.helm_apply.restype = ip
        L.helm_sl_vcycle.argtypes = [vp, vp, vp, ip, vp]
        L.helm_sl_vcycle.restype = ip
        L.helm_sl_vcycle_noalloc.argtypes = [vp, vp, vp, ip, vp]
        L.helm_sl_vcycle_noalloc.restype = ip
        L.helm_sl_vcycle_noalloc_bytes.argtypes = [vp, ip]
        L.helm_sl_vcycle_noalloc_bytes.restype = C.c_size_t
        L.helm_sl_vcycle_noalloc_max_bytes.argtypes = []
        L.helm_sl_vcycle_noalloc_max_bytes.restype = C.c_size_t
        L.helm_fgmres_solve.argtypes = [C.POINTER(vp), ip, C.POINTER(ip), C.POINTER(vp),
                                        C.POINTER(vp), C.POINTER(FgmresOpts),
                                        C.POINTER(FgmresStats), vp]
        L.helm_fgmres_solve.restype = ip
        L.helm_block_fgmres_solve.argtypes = [vp, ip, vp, vp, ip, C.POINTER(FgmresOpts), C.POINTER(FgmresStats),
                                              vp]
        L.helm_block_fgmres_solve.restype = ip
        L.helm_last_error.argtypes = []
        L.helm_last_error.restype = C.c_char_p
        L.helm_training_triples.argtypes = [vp, vp, vp, vp, ip, vp]
        L.helm_training_triples.restype = ip
        L.helm_training_triples_seeded.argtypes = [vp, C.c_ulonglong, C.c_ulonglong, ip, vp, vp, vp, ip, vp]
        L.helm_triples_mix.argtypes = [vp, vp, ip, C.c_longlong, vp, ip, vp, vp, vp]
        L.helm_triples_mix.restype = ip
        L.helm_training_triples_seeded.restype = ip
        L.helm_training_triples_batch.argtypes = [vp, C.c_ulonglong, vp, vp, vp, vp, vp, ip, vp]
        L.helm_training_triples_batch.restype = ip
        L.helm_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
        L.helm_set_allocator.restype = ip
        L.helm_allocated_bytes.argtypes = []
        L.helm_allocated_bytes.restype = C.c_size_t
        L.helm_coarse_slowness.argtypes = [vp, vp, vp]
        L.helm_coarse_slowness.restype = ip
        L.helm_profile_start.argtypes = [C.c_uint]
        L.helm_profile_start.restype = ip
        L.helm_profile_read.argtypes = [ip, C.POINTER(dp), C.POINTER(C.c_longlong), C.POINTER(dp)]
        L.helm_profile_read.restype = ip
        L.helm_profile_stop.argtypes = []
        L.helm_profile_stop.restype = ip
        L.helm_profile_sample.argtypes = [ip]
        L.helm_profile_sample.restype = ip
        L.helm_autotune.argtypes = [ip]
        L.helm_autotune.restype = ip
        L.helm_autotune_entries.argtypes = []
        L.helm_autotune_entries.restype = ip
        L.helm_autotune_force.argtypes = [ip, ip, ip]
        L.helm_autotune_force.restype = ip
        _lib = L
    return _lib


def _check(rc, what):
    if rc < 0:
        msg = lib().helm_last_error().decode()
        raise HelmError(f"{what} failed ({rc}): {msg}")
    return rc


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HelmError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise HelmError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise HelmError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


class Handle:
    """One medium: the multigrid hierarchy of helm_setup."""

    def __init__(self, slowness, gamma, omega, levels=0, beta=0.5, jacobi_weight=0.8,
                 stream=None, coarse_gmres=0):
        n = slowness.shape[-1]
        if tuple(slowness.shape) != (n, n) or tuple(gamma.shape) != (n, n):
            raise HelmError("slowness and gamma must be [n, n]")
        self._keep = (slowness, gamma)
        opts = _Opts(beta, jacobi_weight, levels, int(coarse_gmres))
        h = C.c_void_p()
        _check(lib().helm_setup(_dev(slowness, torch.float32, "slowness"), float(omega),
                                _dev(gamma, torch.float32, "gamma"), n, C.byref(opts),
                                _stream(stream), C.byref(h)), "helm_setup")
        self._h = h
        self.n = n
        self.omega = float(omega)
        self.levels = lib().helm_num_levels(h)

    @property
    def ptr(self):
        return self._h

    def level_size(self, l):
        return lib().helm_level_size(self._h, l)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().helm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _batch(self, x, name):
        if x.dim() == 2:
            x = x.unsqueeze(0)
        if tuple(x.shape[1:]) != (self.n, self.n):
            raise HelmError(f"{name} must be [nrhs, {self.n}, {self.n}]")
        return x

    def apply(self, x, op="A", out=None, stream=None):
        x = self._batch(x, "x")
        y = torch.empty_like(x) if out is None else out
        opc = HELM_OP_A if op == "A" else HELM_OP_M
        _check(lib().helm_apply(self._h, opc, _dev(x, torch.complex64, "x"),
                                _dev(y, torch.complex64, "y"), x.shape[0], _stream(stream)),
               "helm_apply")
        return y

    def training_triples(self, x, stream=None):
        """(r, e) with one SL-FGMRES step from zero on b = A x (eq. 3.8-3.9)."""
        x = self._batch(x, "x")
        r = torch.empty_like(x)
        e = torch.empty_like(x)
        _check(lib().helm_training_triples(self._h, _dev(x, torch.complex64, "x"),
                                           _dev(r, torch.complex64, "r"),
                                           _dev(e, torch.complex64, "e"), x.shape[0],
                                           _stream(stream)), "helm_training_triples")
        return r, e

    def training_triples_seeded(self, seed, index0, r, e, x=None, ksteps=1, stream=None):
        """Triples of samples index0 .. index0 + len(r) - 1 with x drawn on
        the device from (seed, index) and k = ksteps FGMRES(M_V) steps
        (helm_training_triples_seeded), written into the given complex64
        [nrhs, n, n] views r and e (and x if given)."""
        r = self._batch(r, "r")
        e = self._batch(e, "e")
        xp = C.c_void_p(0) if x is None else _dev(self._batch(x, "x"), torch.complex64, "x")
        _check(lib().helm_training_triples_seeded(self._h, int(seed), int(index0), int(ksteps), xp,
                                                  _dev(r, torch.complex64, "r"),
                                                  _dev(e, torch.complex64, "e"), r.shape[0],
                                                  _stream(stream)), "helm_training_triples_seeded")
        return r, e

    def training_triples_batch(self, seed, index, ksteps, r, e, x=None, stream=None):
        """Triples of the samples with the given indices, sample b with
        ksteps[b] FGMRES(M_V) steps, all advanced together
        (helm_training_triples_batch), written into the given complex64
        [nrhs, n, n] views r and e (and x if given)."""
        r = self._batch(r, "r")
        e = self._batch(e, "e")
        nb = r.shape[0]
        if len(index) != nb or len(ksteps) != nb:
            raise HelmError("one index and one k per sample are required")
        idx = (C.c_ulonglong * max(nb, 1))(*[int(i) for i in index])
        ks = (C.c_int * max(nb, 1))(*[int(k) for k in ksteps])
        xp = C.c_void_p(0) if x is None else _dev(self._batch(x, "x"), torch.complex64, "x")
        _check(lib().helm_training_triples_batch(self._h, int(seed), idx, ks, xp, _dev(r, torch.complex64, "r"),
                                                 _dev(e, torch.complex64, "e"), nb, _stream(stream)),
               "helm_training_triples_batch")
        return r, e

    def coarse_slowness(self, out=None, stream=None):
        """Slowness at the coarse points, float [n/2, n/2] (into `out`, a
        contiguous view, if given)."""
        if out is not None:
            _check(lib().helm_coarse_slowness(self._h, _dev(out, torch.float32, "kc"), _stream(stream)),
                   "helm_coarse_slowness")
            return out
        kc = torch.empty((self.n // 2, self.n // 2), dtype=torch.float32, device="cuda")
        _check(lib().helm_coarse_slowness(self._h, _dev(kc, torch.float32, "kc"), _stream(stream)),
               "helm_coarse_slowness")
        return kc

    def vcycle(self, f, out=None, stream=None):
        f = self._batch(f, "f")
        v = torch.empty_like(f) if out is None else out
        _check(lib().helm_sl_vcycle(self._h, _dev(f, torch.complex64, "f"),
                                    _dev(v, torch.complex64, "v"), f.shape[0], _stream(stream)),
               "helm_sl_vcycle")
        return v

    def vcycle_noalloc(self, f, out, stream=None):
        """helm_sl_vcycle on the library's fixed device workspace (no
        allocation in the call); `out` is the caller's output buffer."""
        f = self._batch(f, "f")
        _check(lib().helm_sl_vcycle_noalloc(self._h, _dev(f, torch.complex64, "f"),
                                            _dev(out, torch.complex64, "out"), f.shape[0],
                                            _stream(stream)), "helm_sl_vcycle_noalloc")
        return out

    def vcycle_noalloc_bytes(self, nrhs):
        return lib().helm_sl_vcycle_noalloc_bytes(self._h, int(nrhs))


def fgmres_solve(problems, rhs, m=20, tol=1e-7, maxit=20000, prec="sl", net=None,
                 stall_ratio=0.0, xs=None, stream=None, graph=False, encoder=None):
    """Solve A x = b for every right-hand side of every problem.

    problems: list of Handle; rhs: list of complex64 tensors [nrhs_p, n_p, n_p].
    encoder: with an encoder-solver `net`, the encoder that encodes every
    problem's medium before its solve (any number of media per call).
    Returns (list of complex128 solutions, list of per-RHS stat dicts, status).
    """
    nprob = len(problems)
    if len(rhs) != nprob:
        raise HelmError("one right-hand-side batch per problem is required")
    rhs = [p._batch(b, "b") for p, b in zip(problems, rhs)]
    if xs is None:
        xs = [torch.empty(b.shape, dtype=torch.complex128, device=b.device) for b in rhs]
    probs = (C.c_void_p * nprob)(*[p.ptr.value for p in problems])
    counts = (C.c_int * nprob)(*[b.shape[0] for b in rhs])
    bp = (C.c_void_p * nprob)(*[_dev(b, torch.complex64, "b").value for b in rhs])
    xp = (C.c_void_p * nprob)(*[_dev(x, torch.complex128, "x").value for x in xs])
    total = sum(b.shape[0] for b in rhs)
    stats = (FgmresStats * max(total, 1))()
    opts = FgmresOpts(m, tol, maxit, PREC[prec] if isinstance(prec, str) else int(prec),
                      C.c_void_p(net.ptr.value if net is not None else 0), stall_ratio, int(graph),
                      C.c_void_p(encoder.ptr.value if encoder is not None else 0))
    rc = _check(lib().helm_fgmres_solve(probs, nprob, counts, bp, xp, C.byref(opts), stats,
                                        _stream(stream)), "helm_fgmres_solve")
    return xs, [stats[i].as_dict() for i in range(total)], rc


def block_fgmres_solve(problem, b, block=10, m=10, tol=1e-7, maxit=20000, prec="sl", net=None, x=None,
                       stream=None):
    """Block FGMRES(m) on one problem, blocks of `block` right-hand sides
    (helm_block_fgmres_solve).  Returns (complex128 solution, stats, status)."""
    b = problem._batch(b, "b")
    x = torch.empty(b.shape, dtype=torch.complex128, device=b.device) if x is None else x
    nrhs = b.shape[0]
    stats = (FgmresStats * max(nrhs, 1))()
    opts = FgmresOpts(m, tol, maxit, PREC[prec] if isinstance(prec, str) else int(prec),
                      C.c_void_p(net.ptr.value if net is not None else 0), 0.0, 0, C.c_void_p(0))
    rc = _check(lib().helm_block_fgmres_solve(problem.ptr, nrhs, _dev(b, torch.complex64, "b"),
                                              _dev(x, torch.complex128, "x"), int(block), C.byref(opts), stats,
                                              _stream(stream)), "helm_block_fgmres_solve")
    return x, [stats[i].as_dict() for i in range(nrhs)], rc


def profile_start(*families, every=1):
    """Start timing the launches of the given kernel families with HIP events
    on their launch streams (every `every`-th launch of each family), summing
    the timed launches' algorithmic work."""
    mask = 0
    for f in families:
        mask |= 1 << PROF[f]
    _check(lib().helm_profile_sample(int(every)), "helm_profile_sample")
    _check(lib().helm_profile_start(mask), "helm_profile_start")


def profile_read(family):
    """(summed device milliseconds, launches, algorithmic work) of one family
    since profile_start (bytes for sweeps, FLOPs for convolutions)."""
    ms = C.c_double()
    n = C.c_longlong()
    w = C.c_double()
    _check(lib().helm_profile_read(PROF[family], C.byref(ms), C.byref(n), C.byref(w)),
           "helm_profile_read")
    return ms.value, n.value, w.value


def profile_stop():
    _check(lib().helm_profile_stop(), "helm_profile_stop")


def autotune(enable=1):
    """Switch the convolution launch-shape autotuner (1 on, 0 off, -1 off and
    forget); returns the previous setting."""
    return lib().helm_autotune(int(enable))


def autotune_entries():
    return lib().helm_autotune_entries()



def autotune_force(kind=-1, mf=2, per_cu=1):
    """Force one tuner candidate launch shape on every convolution (test
    hook); kind < 0 switches it off."""
    _check(lib().helm_autotune_force(int(kind), int(mf), int(per_cu)), "helm_autotune_force")


_alloc_keep = None


def set_allocator(alloc=None, release=None):
    """Register Python callables alloc(bytes) -> device address and
    release(address, bytes) for the library's workspaces (helm_set_allocator);
    no arguments restore hipMalloc / hipFree."""
    global _alloc_keep
    if alloc is None:
        _check(lib().helm_set_allocator(ALLOC_FN(), FREE_FN(), None), "helm_set_allocator")
        _alloc_keep = None
        return
    a = ALLOC_FN(lambda nbytes, ctx: alloc(int(nbytes)) or None)
    f = FREE_FN(lambda ptr, nbytes, ctx: release(int(ptr), int(nbytes)))
    _check(lib().helm_set_allocator(a, f, None), "helm_set_allocator")
    _alloc_keep = (a, f, alloc, release)


def use_torch_allocator(device=None):
    """Back the library's workspaces by torch's caching allocator (blocks on
    the given device, default the current one)."""
    dev = torch.cuda.current_device() if device is None else int(device)

    def alloc(nbytes):
        return torch.cuda.caching_allocator_alloc(nbytes, device=dev)

    def release(ptr, nbytes):
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(alloc, release)


def triples_mix(r, e, coef, r_out, e_out, stream=None):
    """r_out[b] = sum_j coef[b, j] r[j] (and e) for triples of one medium
    (helm_triples_mix); coef: device float [nout, nin]."""
    nin, nout = r.shape[0], coef.shape[0]
    if tuple(coef.shape) != (nout, nin) or e.shape != r.shape or r_out.shape[0] != nout or e_out.shape != r_out.shape:
        raise HelmError("triples_mix: shapes do not match")
    npts = r[0].numel()
    _check(lib().helm_triples_mix(_dev(r, torch.complex64, "r"), _dev(e, torch.complex64, "e"), nin, npts,
                                  _dev(coef, torch.float32, "coef"), nout, _dev(r_out, torch.complex64, "r_out"),
                                  _dev(e_out, torch.complex64, "e_out"), _stream(stream)), "helm_triples_mix")
    return r_out, e_out


def allocated_bytes():
    """Device bytes the library currently holds."""
    return lib().helm_allocated_bytes()
