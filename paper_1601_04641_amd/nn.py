"""Thin ctypes binding of include/gpnn.h (the warm-start network, in libgpsscn.so).

Argument marshalling only: every layer, loss, gradient and Adam update runs in the
library's HIP kernels.  torch provides device memory and streams.  Functions carry the
C names; :class:`Net` bundles them around one model.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import gp

GPNN_OK, GPNN_ERR_INVALID, GPNN_ERR_HIP, GPNN_ERR_OOM, GPNN_ERR_STATE = 0, -1, -2, -3, -4

EXPORTS = ("gpnn_create", "gpnn_destroy", "gpnn_param_count", "gpnn_set_params", "gpnn_get_params",
           "gpnn_get_grads", "gpnn_forward", "gpnn_loss_backward", "gpnn_backward", "gpnn_adam_step", "gpnn_conv",
           "gpnn_conv_wgrad", "gpnn_last_error")

# standardisation of (nu_x, nu_y, nu_z, ln g) for nu ~ U[0.5, 4], ln g ~ U[0, ln 1000]
IN_MEAN = (2.25, 2.25, 2.25, 0.5 * math.log(1000.0))
IN_STD = (3.5 / math.sqrt(12),) * 3 + (math.log(1000.0) / math.sqrt(12),)


class gpnn_arch(ctypes.Structure):
    _fields_ = [("base", ctypes.c_int32), ("hidden", ctypes.c_int32), ("nstage", ctypes.c_int32),
                ("ch", ctypes.c_int32 * 7), ("max_batch", ctypes.c_int32), ("dx", ctypes.c_double),
                ("in_mean", ctypes.c_double * 4), ("in_std", ctypes.c_double * 4)]


class NNError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        super().__init__(f"{where}: code {code}" + (f": {detail}" if detail else ""))


_sig_done = False


def load():
    global _sig_done
    L = gp.load()
    if _sig_done:
        return L
    vp, i32, i64, f32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "gpnn_create": [P(gpnn_arch), vp, P(vp)],
        "gpnn_destroy": [vp],
        "gpnn_param_count": [vp, P(i64)],
        "gpnn_set_params": [vp, vp, i64],
        "gpnn_get_params": [vp, vp, i64],
        "gpnn_get_grads": [vp, vp, i64],
        "gpnn_forward": [vp, vp, i32, vp, i32],
        "gpnn_loss_backward": [vp, vp, P(d)],
        "gpnn_backward": [vp, vp],
        "gpnn_adam_step": [vp, f32, f32, f32, f32, i64],
        "gpnn_conv": [i32, i32, i32, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp],
        "gpnn_conv_wgrad": [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.gpnn_last_error.argtypes = [vp]
    L.gpnn_last_error.restype = ctypes.c_char_p
    _sig_done = True
    return L


def make_arch(base=4, hidden=384, ch=(64, 64, 64, 32, 16), dx=0.25, max_batch=16,
              in_mean=IN_MEAN, in_std=IN_STD) -> gpnn_arch:
    a = gpnn_arch()
    a.base, a.hidden, a.nstage = int(base), int(hidden), len(ch) - 1
    for i, c in enumerate(ch):
        a.ch[i] = int(c)
    a.max_batch, a.dx = int(max_batch), float(dx)
    for i in range(4):
        a.in_mean[i], a.in_std[i] = float(in_mean[i]), float(in_std[i])
    return a


def param_shapes(base, hidden, ch):
    """(name, shape) of the parameter vector in the order include/gpnn.h documents."""
    f2 = base ** 3 * ch[0]
    out = [("W1", (hidden, 4)), ("b1", (hidden,)), ("W2", (f2, hidden)), ("b2", (f2,))]
    for s in range(1, len(ch)):
        out += [(f"C{s}", (27, ch[s], ch[s - 1])), (f"c{s}", (ch[s],))]
    return out + [("wh", (ch[-1],)), ("bh", ())]


def flatten(w: dict, shapes) -> np.ndarray:
    return np.concatenate([np.asarray(w[k], dtype=np.float32).reshape(-1) for k, _ in shapes])


def unflatten(v: np.ndarray, shapes) -> dict:
    out, o = {}, 0
    for k, s in shapes:
        n = int(np.prod(s))
        out[k] = v[o:o + n].reshape(s)
        o += n
    return out


class Net:
    """One gpnn model on the current device and stream."""

    def __init__(self, base=4, hidden=384, ch=(64, 64, 64, 32, 16), dx=0.25, max_batch=16, stream=None):
        import torch
        self.cfg = dict(base=base, hidden=hidden, ch=tuple(ch), dx=dx, max_batch=max_batch)
        self.shapes = param_shapes(base, hidden, ch)
        self.N = base * 2 ** (len(ch) - 1)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._L = load()
        self._arch = make_arch(base, hidden, ch, dx, max_batch)
        h = ctypes.c_void_p()
        rc = self._L.gpnn_create(ctypes.byref(self._arch), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != GPNN_OK:
            raise NNError(rc, "gpnn_create")
        self._h = h
        n = ctypes.c_int64()
        self._chk(self._L.gpnn_param_count(self._h, ctypes.byref(n)), "gpnn_param_count")
        self.n_params = n.value
        assert self.n_params == sum(int(np.prod(s)) for _, s in self.shapes)

    def _chk(self, rc, name):
        if rc != GPNN_OK:
            raise NNError(rc, name, self._L.gpnn_last_error(self._h).decode(errors="replace"))

    def set_params(self, w):
        v = flatten(w, self.shapes) if isinstance(w, dict) else np.ascontiguousarray(w, dtype=np.float32)
        self._chk(self._L.gpnn_set_params(self._h, v.ctypes.data, v.size), "gpnn_set_params")

    def get_params(self) -> np.ndarray:
        v = np.empty(self.n_params, dtype=np.float32)
        self._chk(self._L.gpnn_get_params(self._h, v.ctypes.data, v.size), "gpnn_get_params")
        return v

    def get_grads(self) -> np.ndarray:
        v = np.empty(self.n_params, dtype=np.float32)
        self._chk(self._L.gpnn_get_grads(self._h, v.ctypes.data, v.size), "gpnn_get_grads")
        return v

    def forward(self, prm, out, complex_out=False):
        """prm: float32 [n, 4] device tensor; out: [n, N, N, N] float32, or complex64 /
        complex128 (complex_out=True; the kind follows out's dtype)."""
        import torch
        n = prm.shape[0]
        kind = 0
        if complex_out:
            kind = 2 if out.dtype == torch.complex128 else 1
        if out.numel() < n * self.N ** 3 or not out.is_contiguous():
            raise ValueError(f"out must hold {n} x {self.N}^3 contiguous values")
        self._chk(self._L.gpnn_forward(self._h, prm.data_ptr(), n, out.data_ptr(), kind), "gpnn_forward")
        self._last_points = n * self.N ** 3

    def loss_backward(self, target, want_loss=True):
        lp = getattr(self, "_last_points", None)
        if (lp is not None and target.numel() != lp) or not target.is_contiguous():
            raise ValueError("target must have one value per point of the last forward pass's output")
        v = ctypes.c_double()
        self._chk(self._L.gpnn_loss_backward(self._h, target.data_ptr(), ctypes.byref(v) if want_loss else None),
                  "gpnn_loss_backward")
        return v.value if want_loss else None

    def backward(self, grad_psi):
        """Parameter gradients of the last FP32 forward pass for an upstream dL/dpsi
        (FP32 device tensor shaped like that pass's output); overwrites the gradients."""
        import torch
        if not grad_psi.is_cuda or not grad_psi.is_contiguous() or grad_psi.dtype != torch.float32:
            raise ValueError("grad_psi must be a contiguous float32 device tensor")
        lp = getattr(self, "_last_points", None)
        if lp is not None and grad_psi.numel() != lp:   # (no forward pass yet: the library's state error)
            raise ValueError("grad_psi must have one value per point of the last forward pass's output")
        self._chk(self._L.gpnn_backward(self._h, grad_psi.data_ptr()), "gpnn_backward")

    def adam_step(self, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
        self._chk(self._L.gpnn_adam_step(self._h, lr, beta1, beta2, eps, int(t)), "gpnn_adam_step")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.gpnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gpnn_conv(ks, n, d, cin, cout, x, w, bias=None, act=0, gate=None, y=None, pre=None, stream=None):
    """Kernel-level convolution on BF16 tensors (torch.bfloat16, device)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    rc = load().gpnn_conv(ks, n, d, cin, cout, ptr(x), ptr(w), ptr(bias), act, ptr(gate), ptr(y), ptr(pre),
                          st.cuda_stream)
    if rc != GPNN_OK:
        raise NNError(rc, "gpnn_conv")


def gpnn_conv_wgrad(ks, n, d, cin, cout, dy, x, dw, db=None, stream=None):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = load().gpnn_conv_wgrad(ks, n, d, cin, cout, dy.data_ptr(), x.data_ptr(), dw.data_ptr(),
                                None if db is None else db.data_ptr(), st.cuda_stream)
    if rc != GPNN_OK:
        raise NNError(rc, "gpnn_conv_wgrad")
