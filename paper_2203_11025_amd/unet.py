"""ctypes binding of the U-Net entry points (include/unet.h).  Argument
marshalling only; every step runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C

import torch

from .helm import HelmError, _check, _dev, _stream, lib as _helm_lib

EXPORTS = ["unet_create", "unet_destroy", "unet_num_params", "unet_num_buffers", "unet_init",
           "unet_set_params", "unet_get_params", "unet_forward", "unet_infer",
           "unet_loss_grad", "unet_train_step", "unet_pair_encode", "unet_pair_loss_grad",
           "unet_pair_train_step", "unet_save", "unet_load", "unet_set_cursor", "unet_get_cursor",
           "unet_pair_encode_medium"]


class Cfg(C.Structure):
    _fields_ = [("in_ch", C.c_int), ("out_ch", C.c_int), ("levels", C.c_int),
                ("widths", C.c_int * 6), ("context", C.c_int), ("head", C.c_int), ("arch", C.c_int)]


class Batch(C.Structure):
    _fields_ = [("nb", C.c_int), ("n", C.c_int), ("r", C.c_void_p), ("e", C.c_void_p),
                ("kappa_c", C.c_void_p), ("kappa_f", C.c_void_p), ("gamma_f", C.c_void_p),
                ("fine_shared", C.c_int)]


class TrainOpts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


_done = False


def lib():
    global _done
    L = _helm_lib()
    if not _done:
        vp, ip = C.c_void_p, C.c_int
        L.unet_create.argtypes = [C.POINTER(Cfg), C.POINTER(vp)]
        L.unet_create.restype = ip
        L.unet_destroy.argtypes = [vp]
        L.unet_destroy.restype = None
        L.unet_num_params.argtypes = [vp]
        L.unet_num_params.restype = C.c_longlong
        L.unet_num_buffers.argtypes = [vp]
        L.unet_num_buffers.restype = C.c_longlong
        L.unet_init.argtypes = [vp, C.c_ulonglong, vp]
        L.unet_init.restype = ip
        L.unet_set_params.argtypes = [vp, vp, vp, vp]
        L.unet_set_params.restype = ip
        L.unet_get_params.argtypes = [vp, vp, vp, vp]
        L.unet_get_params.restype = ip
        L.unet_forward.argtypes = [vp, vp, ip, ip, ip, vp, ip, vp]
        L.unet_forward.restype = ip
        L.unet_infer.argtypes = [vp, vp, vp, vp, ip, vp]
        L.unet_infer.restype = ip
        L.unet_loss_grad.argtypes = [vp, C.POINTER(Batch), C.POINTER(C.c_double), vp, vp]
        L.unet_loss_grad.restype = ip
        L.unet_train_step.argtypes = [vp, C.POINTER(Batch), C.POINTER(TrainOpts),
                                      C.POINTER(C.c_double), vp]
        L.unet_train_step.restype = ip
        L.unet_pair_encode.argtypes = [vp, vp, vp, ip, ip, vp]
        L.unet_pair_encode.restype = ip
        L.unet_pair_loss_grad.argtypes = [vp, vp, C.POINTER(Batch), C.POINTER(C.c_double), vp, vp, vp]
        L.unet_pair_loss_grad.restype = ip
        L.unet_pair_train_step.argtypes = [vp, vp, C.POINTER(Batch), C.POINTER(TrainOpts),
                                           C.POINTER(C.c_double), vp]
        L.unet_pair_train_step.restype = ip
        L.unet_pair_encode_medium.argtypes = [vp, vp, vp, vp]
        L.unet_pair_encode_medium.restype = ip
        L.unet_save.argtypes = [vp, C.c_char_p, vp]
        L.unet_save.restype = ip
        L.unet_load.argtypes = [vp, C.c_char_p, vp]
        L.unet_load.restype = ip
        L.unet_set_cursor.argtypes = [vp, C.c_ulonglong, C.c_ulonglong]
        L.unet_set_cursor.restype = ip
        L.unet_get_cursor.argtypes = [vp, C.POINTER(C.c_ulonglong), C.POINTER(C.c_ulonglong)]
        L.unet_get_cursor.restype = ip
        _done = True
    return L


class UNet:
    """context=True: the solver of an encoder-solver pair; head=False: an
    encoder (in_ch 1), whose per-level outputs are the solver's contexts."""

    def __init__(self, widths=(32, 64, 128, 256), in_ch=3, out_ch=2, context=False, head=True, arch=0):
        """arch=1: the paper's own network (section 3.1) on the fine grid,
        widths c_1..c_L of its levels below the fine grid."""
        if not head:
            in_ch = 1
        if arch == 1:
            in_ch = 4
        cfg = Cfg(in_ch, out_ch, len(widths), (C.c_int * 6)(*list(widths) + [0] * (6 - len(widths))),
                  int(context), int(head), int(arch))
        self.arch = int(arch)
        h = C.c_void_p()
        _check(lib().unet_create(C.byref(cfg), C.byref(h)), "unet_create")
        self._h = h
        self.widths = tuple(widths)
        self.in_ch, self.out_ch = in_ch, out_ch
        self.context, self.head = bool(context), bool(head)
        self.nparams = lib().unet_num_params(h)
        self.nbuf = lib().unet_num_buffers(h)

    @property
    def ptr(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().unet_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def save_state(self, path, stream=None):
        """Parameters, BN statistics, Adam state and data cursor (unet_save)."""
        _check(lib().unet_save(self._h, str(path).encode(), _stream(stream)), "unet_save")

    def load_state(self, path, stream=None):
        _check(lib().unet_load(self._h, str(path).encode(), _stream(stream)), "unet_load")

    def set_cursor(self, seed, next_index):
        _check(lib().unet_set_cursor(self._h, int(seed), int(next_index)), "unet_set_cursor")

    def cursor(self):
        """(seed, next sample index) of the training data."""
        a, b = C.c_ulonglong(), C.c_ulonglong()
        _check(lib().unet_get_cursor(self._h, C.byref(a), C.byref(b)), "unet_get_cursor")
        return a.value, b.value

    def init(self, seed, stream=None):
        """Seeded Kaiming-normal initial parameters (in the library)."""
        _check(lib().unet_init(self._h, seed, _stream(stream)), "unet_init")

    def set_params(self, params, buffers=None, stream=None):
        if params.numel() != self.nparams:
            raise HelmError(f"expected {self.nparams} parameters, got {params.numel()}")
        p = params.to(device="cuda", dtype=torch.float32).contiguous()
        b = None
        if buffers is not None:
            if buffers.numel() != self.nbuf:
                raise HelmError(f"expected {self.nbuf} buffer entries, got {buffers.numel()}")
            b = buffers.to(device="cuda", dtype=torch.float32).contiguous()
        _check(lib().unet_set_params(self._h, _dev(p, torch.float32, "params"),
                                     _dev(b, torch.float32, "buffers") if b is not None else None,
                                     _stream(stream)), "unet_set_params")
        torch.cuda.synchronize()

    def get_params(self, stream=None):
        p = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        b = torch.empty(self.nbuf, dtype=torch.float32, device="cuda")
        _check(lib().unet_get_params(self._h, _dev(p, torch.float32, "p"), _dev(b, torch.float32, "b"),
                                     _stream(stream)), "unet_get_params")
        torch.cuda.synchronize()
        return p, b

    def forward(self, x, training=False, stream=None):
        B, Cin, H, W = x.shape
        x = x.to(device="cuda", dtype=torch.float32).contiguous()
        out = torch.empty((B, self.out_ch, H, W), dtype=torch.float32, device="cuda")
        _check(lib().unet_forward(self._h, _dev(x, torch.float32, "x"), B, H, W,
                                  _dev(out, torch.float32, "out"), int(training), _stream(stream)),
               "unet_forward")
        return out

    def infer(self, handle, r, stream=None):
        r = handle._batch(r, "r")
        e = torch.empty_like(r)
        _check(lib().unet_infer(self._h, handle.ptr, _dev(r, torch.complex64, "r"),
                                _dev(e, torch.complex64, "e"), r.shape[0], _stream(stream)),
               "unet_infer")
        return e

    @staticmethod
    def _batch(r, e, kappa_c, kappa_f=None, gamma_f=None):
        """kappa_f / gamma_f: the fine medium for the paper's network, [n, n]
        (shared by the batch) or [nb, n, n]."""
        nb, n = r.shape[0], r.shape[-1]
        kc = C.c_void_p(0) if kappa_c is None else _dev(kappa_c, torch.float32, "kappa_c")
        kf = C.c_void_p(0) if kappa_f is None else _dev(kappa_f, torch.float32, "kappa_f")
        gf = C.c_void_p(0) if gamma_f is None else _dev(gamma_f, torch.float32, "gamma_f")
        shared = int(kappa_f is not None and kappa_f.dim() == 2)
        return Batch(nb, n, _dev(r, torch.complex64, "r"), _dev(e, torch.complex64, "e"), kc, kf, gf, shared)

    def loss_grad(self, r, e, kappa_c, stream=None, kappa_f=None, gamma_f=None):
        bt = self._batch(r, e, kappa_c, kappa_f, gamma_f)
        g = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        loss = C.c_double()
        _check(lib().unet_loss_grad(self._h, C.byref(bt), C.byref(loss), _dev(g, torch.float32, "g"),
                                    _stream(stream)), "unet_loss_grad")
        return loss.value, g

    def train_step(self, r, e, kappa_c, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None, kappa_f=None,
                   gamma_f=None):
        bt = self._batch(r, e, kappa_c, kappa_f, gamma_f)
        o = TrainOpts(lr, beta1, beta2, eps)
        loss = C.c_double()
        _check(lib().unet_train_step(self._h, C.byref(bt), C.byref(o), C.byref(loss),
                                     _stream(stream)), "unet_train_step")
        return loss.value


def pair_encode(encoder, solver, kappa_c, stream=None):
    """Run the encoder on kappa_c ([nc, nc] for one medium, or [nb, nc, nc])
    and store the per-level contexts in the solver."""
    k = kappa_c.to(device="cuda", dtype=torch.float32).contiguous()
    if k.dim() == 2:
        k = k[None]
    _check(lib().unet_pair_encode(encoder.ptr, solver.ptr, _dev(k, torch.float32, "kappa_c"),
                                  k.shape[0], k.shape[-1], _stream(stream)), "unet_pair_encode")


def pair_encode_medium(encoder, solver, handle, stream=None):
    """Encode the medium of a helm Handle (its coarse slowness) into the solver."""
    _check(lib().unet_pair_encode_medium(encoder.ptr, solver.ptr, handle.ptr, _stream(stream)),
           "unet_pair_encode_medium")


def pair_loss_grad(encoder, solver, r, e, kappa_c, stream=None):
    bt = UNet._batch(r, e, kappa_c)
    ge = torch.empty(encoder.nparams, dtype=torch.float32, device="cuda")
    gs = torch.empty(solver.nparams, dtype=torch.float32, device="cuda")
    loss = C.c_double()
    _check(lib().unet_pair_loss_grad(encoder.ptr, solver.ptr, C.byref(bt), C.byref(loss),
                                     _dev(ge, torch.float32, "ge"), _dev(gs, torch.float32, "gs"),
                                     _stream(stream)), "unet_pair_loss_grad")
    return loss.value, ge, gs


def pair_train_step(encoder, solver, r, e, kappa_c, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                    stream=None):
    bt = UNet._batch(r, e, kappa_c)
    o = TrainOpts(lr, beta1, beta2, eps)
    loss = C.c_double()
    _check(lib().unet_pair_train_step(encoder.ptr, solver.ptr, C.byref(bt), C.byref(o), C.byref(loss),
                                      _stream(stream)), "unet_pair_train_step")
    return loss.value


def save(path, **nets):
    """Write the FP32 parameters and BN buffers of named networks to a
    safetensors file (keys <name>.params, <name>.buffers, <name>.widths)."""
    from safetensors.torch import save_file

    out = {}
    for name, net in nets.items():
        p, b = net.get_params()
        out[f"{name}.params"] = p.cpu()
        out[f"{name}.buffers"] = b.cpu()
        out[f"{name}.widths"] = torch.tensor(net.widths, dtype=torch.int32)
    save_file(out, path)


def load(path, **nets):
    """Read parameters written by save() into networks of the same shape."""
    from safetensors.torch import load_file

    d = load_file(path)
    for name, net in nets.items():
        if tuple(d[f"{name}.widths"].tolist()) != net.widths:
            raise HelmError(f"{path}: widths of {name} differ")
        net.set_params(d[f"{name}.params"], d[f"{name}.buffers"])
