"""Thin ctypes binding of the C-ABI in include/gp.h (libgpsscn.so).

Argument marshalling only: every step of the solver runs in the HIP kernels of the
library.  torch is used for device memory (``psi`` tensors) and streams, nothing else.
Functions carry the C names; :class:`Solver` bundles them around one context.
``load()`` raises if the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpsscn.so")

GP_OK, GP_ERR_INVALID, GP_ERR_HIP, GP_ERR_OOM = 0, -1, -2, -3
GP_ERR_NONFINITE, GP_ERR_ZERO_NORM, GP_ERR_UNSUPPORTED = -4, -5, -6
GP_C64, GP_C128 = 0, 1
GP_SPLIT_LIE, GP_SPLIT_STRANG = 0, 1
GP_FLAG_NONFINITE, GP_FLAG_ZERO_NORM = 1, 2

# names declared in include/gp.h (checked against the built library by the tests)
EXPORTS = ("gp_init", "gp_destroy", "gp_step_imag", "gp_step_real", "gp_norm", "gp_energy_mu",
           "gp_rms", "gp_raw_sums", "gp_set_g", "gp_set_psi", "gp_status", "gp_converge_imag",
           "gp_set_timing", "gp_get_timing", "gp_get_mapping", "gp_set_mapping", "gp_autotune",
           "gp_strerror", "gp_last_error",
           "gp_batch_init", "gp_batch_destroy", "gp_batch_step_imag", "gp_batch_step_real",
           "gp_batch_norm", "gp_batch_energy_mu", "gp_batch_rms", "gp_batch_raw_sums",
           "gp_batch_status", "gp_batch_residual", "gp_batch_converge_imag", "gp_batch_get_mapping",
           "gp_batch_set_mapping", "gp_batch_autotune", "gp_batch_set_yz_fusion", "gp_batch_get_yz_fusion", "gp_batch_set_timing",
           "gp_batch_get_timing", "gp_batch_last_error",
           "gp_set_alloc_cap", "gp_eval_sincos", "gp_stream_copy", "gp_raw_sums_noalloc",
           "gp_set_truncation", "gp_get_truncation", "gp_stop_rule_eval")


class GPError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        msg = f"{where}: {gp_strerror(code)} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class gp_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("nux", ctypes.c_double), ("nuy", ctypes.c_double), ("nuz", ctypes.c_double),
                ("g", ctypes.c_double), ("dt", ctypes.c_double),
                ("precision", ctypes.c_int32), ("split", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raise if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "gp_init": [P(gp_params), vp, vp, P(vp)],
        "gp_destroy": [vp],
        "gp_step_imag": [vp, i32],
        "gp_step_real": [vp, i32],
        "gp_norm": [vp, P(d)],
        "gp_energy_mu": [vp, P(d), P(d)],
        "gp_rms": [vp, P(d)],
        "gp_raw_sums": [vp, P(d)],
        "gp_set_g": [vp, d],
        "gp_set_psi": [vp, vp],
        "gp_status": [vp, P(i64), P(d), P(i32)],
        "gp_converge_imag": [vp, d, i32, i64, P(i64), P(d), P(i32)],
        "gp_set_timing": [vp, i32],
        "gp_get_timing": [vp, P(d), P(i64)],
        "gp_get_mapping": [vp, P(i32)],
        "gp_set_mapping": [vp, P(i32)],
        "gp_autotune": [vp, i32, i32, ctypes.c_char_p, P(i32)],
        "gp_batch_init": [P(gp_params), i32, vp, P(i64), vp, P(vp)],
        "gp_batch_destroy": [vp],
        "gp_batch_step_imag": [vp, i32, vp],
        "gp_batch_step_real": [vp, i32, vp],
        "gp_batch_norm": [vp, P(d)],
        "gp_batch_energy_mu": [vp, P(d), P(d)],
        "gp_batch_rms": [vp, P(d)],
        "gp_batch_raw_sums": [vp, P(d)],
        "gp_batch_status": [vp, P(i64), P(d), P(i32)],
        "gp_batch_residual": [vp, P(d), P(d)],
        "gp_batch_converge_imag": [vp, d, i32, i64, P(i64), P(d), P(i32)],
        "gp_batch_get_mapping": [vp, P(i32)],
        "gp_batch_set_mapping": [vp, P(i32)],
        "gp_batch_autotune": [vp, i32, i32, ctypes.c_char_p, P(i32)],
        "gp_set_alloc_cap": [i64],
        "gp_eval_sincos": [i32, vp, i64, vp, vp, vp],
        "gp_stream_copy": [vp, vp, i64, vp],
        "gp_raw_sums_noalloc": [P(gp_params), vp, vp, vp],
        "gp_set_truncation": [vp, i32],
        "gp_get_truncation": [vp, P(i32), P(i32)],
        "gp_stop_rule_eval": [P(d), i32, d, P(i32)],
        "gp_batch_set_yz_fusion": [vp, i32],
        "gp_batch_get_yz_fusion": [vp, P(i32), P(i32)],
        "gp_batch_set_timing": [vp, i32],
        "gp_batch_get_timing": [vp, P(d), P(i64)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.gp_strerror.argtypes = [ctypes.c_int]
    L.gp_strerror.restype = ctypes.c_char_p
    L.gp_last_error.argtypes = [vp]
    L.gp_last_error.restype = ctypes.c_char_p
    L.gp_batch_last_error.argtypes = [vp]
    L.gp_batch_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def gp_strerror(code: int) -> str:
    return load().gp_strerror(int(code)).decode()


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny, nz, dx, dy, dz, nux, nuy, nuz, g, dt, precision=GP_C128,
                split=GP_SPLIT_LIE) -> gp_params:
    return gp_params(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz), float(nux),
                     float(nuy), float(nuz), float(g), float(dt), int(precision), int(split))


def gp_init(params: gp_params, psi_ptr: int, stream_ptr: int):
    """Returns (code, handle)."""
    h = ctypes.c_void_p()
    rc = load().gp_init(ctypes.byref(params), ctypes.c_void_p(psi_ptr), ctypes.c_void_p(stream_ptr),
                        ctypes.byref(h))
    return rc, h


def set_alloc_cap(nbytes: int | None):
    """Make every later library allocation above nbytes fail with GP_ERR_OOM (None: no cap)."""
    load().gp_set_alloc_cap(-1 if nbytes is None else int(nbytes))


def stop_rule_eval(values, tol: float) -> int:
    """Index of the first check at which the convergence loops' stopping rule is met on
    the given sequence of checked values (-1: never).  Host only."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = ctypes.c_int32()
    rc = load().gp_stop_rule_eval(v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(v.size), float(tol),
                                  ctypes.byref(out))
    if rc:
        raise GPError(rc, "gp_stop_rule_eval")
    return out.value


def _stream_ptr(t, stream):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(t.device)
    return st.cuda_stream


def eval_sincos(x, stream=None):
    """(sin x, cos x) of the device phase-factor routine for a float32 or float64 device tensor."""
    import torch
    if not x.is_cuda or not x.is_contiguous() or x.dtype not in (torch.float32, torch.float64):
        raise ValueError("x must be a contiguous float32/float64 device tensor")
    sn, cs = torch.empty_like(x), torch.empty_like(x)
    prec = GP_C64 if x.dtype == torch.float32 else GP_C128
    rc = load().gp_eval_sincos(prec, ctypes.c_void_p(x.data_ptr()), x.numel(), ctypes.c_void_p(sn.data_ptr()),
                               ctypes.c_void_p(cs.data_ptr()), ctypes.c_void_p(_stream_ptr(x, stream)))
    if rc != GP_OK:
        raise GPError(rc, "gp_eval_sincos")
    return sn, cs


def stream_copy(src, dst, stream=None):
    """dst <- src (device tensors of equal byte size, a multiple of 16) by the library's copy kernel."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()) or \
            dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must be contiguous device tensors of the same byte size")
    rc = load().gp_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                               ctypes.c_void_p(_stream_ptr(src, stream)))
    if rc != GP_OK:
        raise GPError(rc, "gp_stream_copy")


def _check_like(psi, shape, dtype, device):
    """psi must match the context's shape, dtype and device and be contiguous device memory."""
    if tuple(psi.shape) != tuple(shape) or psi.dtype != dtype or psi.device != device:
        raise ValueError(f"psi must be {tuple(shape)} {dtype} on {device}, got {tuple(psi.shape)} "
                         f"{psi.dtype} on {psi.device}")
    if not psi.is_cuda or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous device tensor")


class Solver:
    """One gp_ctx bound to a caller-owned complex torch tensor psi of shape (nx, ny, nz)."""

    def __init__(self, psi, dx, dy, dz, nux, nuy, nuz, g, dt, split=GP_SPLIT_LIE, stream=None):
        import torch
        if not psi.is_cuda or not psi.is_contiguous() or psi.dim() != 3:
            raise ValueError("psi must be a contiguous 3D device tensor")
        if psi.dtype == torch.complex128:
            prec = GP_C128
        elif psi.dtype == torch.complex64:
            prec = GP_C64
        else:
            raise ValueError("psi must be complex64 or complex128")
        self.psi = psi
        self.stream = stream if stream is not None else torch.cuda.current_stream(psi.device)
        nx, ny, nz = psi.shape
        self.params = make_params(nx, ny, nz, dx, dy, dz, nux, nuy, nuz, g, dt, prec, split)
        with torch.cuda.device(psi.device):
            rc, h = gp_init(self.params, psi.data_ptr(), self.stream.cuda_stream)
        if rc != GP_OK:
            raise GPError(rc, "gp_init")
        self._h = h
        self._L = load()

    @classmethod
    def from_workload(cls, psi, w: dict, split=GP_SPLIT_LIE, stream=None):
        return cls(psi, w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"], w["g"], w["dt"],
                   split=split, stream=stream)

    def _chk(self, rc, name):
        if rc != GP_OK:
            raise GPError(rc, name, self._L.gp_last_error(self._h).decode(errors="replace"))

    def step_imag(self, n: int):
        self._chk(self._L.gp_step_imag(self._h, int(n)), "gp_step_imag")

    def step_real(self, n: int):
        self._chk(self._L.gp_step_real(self._h, int(n)), "gp_step_real")

    def norm(self) -> float:
        v = ctypes.c_double()
        self._chk(self._L.gp_norm(self._h, ctypes.byref(v)), "gp_norm")
        return v.value

    def energy_mu(self):
        e, m = ctypes.c_double(), ctypes.c_double()
        self._chk(self._L.gp_energy_mu(self._h, ctypes.byref(e), ctypes.byref(m)), "gp_energy_mu")
        return e.value, m.value

    def rms(self) -> np.ndarray:
        out = np.zeros(4)
        self._chk(self._L.gp_rms(self._h, _dp(out)), "gp_rms")
        return out

    def raw_sums(self) -> np.ndarray:
        out = np.zeros(9)
        self._chk(self._L.gp_raw_sums(self._h, _dp(out)), "gp_raw_sums")
        return out

    def set_g(self, g: float):
        self._chk(self._L.gp_set_g(self._h, float(g)), "gp_set_g")

    def set_psi(self, psi):
        """Continue on another buffer of the same shape, dtype and device (resume/checkpoint)."""
        _check_like(psi, self.psi.shape, self.psi.dtype, self.psi.device)
        self._chk(self._L.gp_set_psi(self._h, ctypes.c_void_p(psi.data_ptr())), "gp_set_psi")
        self.psi = psi

    def status(self):
        s, m, f = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int32()
        self._chk(self._L.gp_status(self._h, ctypes.byref(s), ctypes.byref(m), ctypes.byref(f)), "gp_status")
        return s.value, m.value, f.value

    def converge_imag(self, tol=1e-7, check_every=0, max_steps=10 ** 7):
        s, m, c = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int32()
        self._chk(self._L.gp_converge_imag(self._h, float(tol), int(check_every), int(max_steps),
                                           ctypes.byref(s), ctypes.byref(m), ctypes.byref(c)),
                  "gp_converge_imag")
        return s.value, m.value, bool(c.value)

    def set_timing(self, on: bool):
        self._chk(self._L.gp_set_timing(self._h, int(bool(on))), "gp_set_timing")

    def get_timing(self):
        ms = np.zeros(5)
        n = np.zeros(5, dtype=np.int64)
        self._chk(self._L.gp_get_timing(self._h, _dp(ms), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
                  "gp_get_timing")
        return ms, n

    def get_mapping(self):
        """[m_x, sw_x, m_y, sw_y, segments_z, m_z]"""
        out = (ctypes.c_int32 * 6)()
        self._chk(self._L.gp_get_mapping(self._h, out), "gp_get_mapping")
        return list(out)

    def set_mapping(self, mx=0, swx=0, my=0, swy=0, segz=0, mz=0):
        arr = (ctypes.c_int32 * 6)(int(mx), int(swx), int(my), int(swy), int(segz), int(mz))
        self._chk(self._L.gp_set_mapping(self._h, arr), "gp_set_mapping")

    def set_truncation(self, mode: int):
        """0: exact sweeps; 1: streaming x and y sweeps with the halo-truncated inverse;
        2: exact x sweep into a work array, then one fused pass of the truncated y sweep
        and the z sweep (see gp_set_truncation)."""
        self._chk(self._L.gp_set_truncation(self._h, int(mode)), "gp_set_truncation")

    def get_truncation(self):
        """(mode, H as [[x, y, z] imaginary, [x, y, z] real])"""
        m = ctypes.c_int32()
        h = (ctypes.c_int32 * 6)()
        self._chk(self._L.gp_get_truncation(self._h, ctypes.byref(m), h), "gp_get_truncation")
        return m.value, [list(h[0:3]), list(h[3:6])]

    def autotune(self, mode="real", steps=5, cache_path=None):
        """Time every line mapping on this grid and keep the fastest (see gp_autotune)."""
        out = (ctypes.c_int32 * 6)()
        cp = cache_path.encode() if cache_path else None
        self._chk(self._L.gp_autotune(self._h, 0 if mode == "imag" else 1, int(steps), cp, out), "gp_autotune")
        return list(out)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.gp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """One gp_batch over a caller-owned 1D complex torch tensor holding every instance's
    grid back to back (instance i: elements offsets[i] .. offsets[i] + nx*ny*nz)."""

    def __init__(self, psi, params, offsets, split=GP_SPLIT_LIE, stream=None):
        import torch
        if not psi.is_contiguous() or psi.dim() != 1:
            raise ValueError("psi must be a contiguous 1D device tensor")
        prec = GP_C128 if psi.dtype == torch.complex128 else GP_C64 if psi.dtype == torch.complex64 else None
        if prec is None:
            raise ValueError("psi must be complex64 or complex128")
        self.n = len(params)
        offsets = np.asarray(offsets, dtype=np.int64).reshape(-1)
        if self.n < 1 or len(offsets) != self.n:
            raise ValueError(f"{self.n} parameter sets but {len(offsets)} offsets")
        sizes = np.array([int(w["nx"]) * int(w["ny"]) * int(w["nz"]) for w in params], dtype=np.int64)
        if np.any(offsets < 0) or np.any(offsets + sizes > psi.numel()):
            raise ValueError("every instance [offset, offset + nx*ny*nz) must lie inside psi")
        order = np.argsort(offsets, kind="stable")
        if np.any(offsets[order][1:] < (offsets + sizes)[order][:-1]):
            raise ValueError("instance regions overlap")
        if not psi.is_cuda:
            raise ValueError("psi must be a contiguous 1D device tensor")
        arr = (gp_params * self.n)()
        for i, w in enumerate(params):
            arr[i] = make_params(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"],
                                 w["nuz"], w["g"], w["dt"], prec, split)
        self._params = arr
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.psi = psi
        self.stream = stream if stream is not None else torch.cuda.current_stream(psi.device)
        self._L = load()
        h = ctypes.c_void_p()
        with torch.cuda.device(psi.device):
            rc = self._L.gp_batch_init(arr, self.n, ctypes.c_void_p(psi.data_ptr()),
                                       self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != GP_OK:
            raise GPError(rc, "gp_batch_init")
        self._h = h

    def _chk(self, rc, name):
        if rc != GP_OK:
            raise GPError(rc, name, self._L.gp_batch_last_error(self._h).decode(errors="replace"))

    def _act(self, active):
        if active is None:
            return None
        a = np.ascontiguousarray(active, dtype=np.uint8)
        self._active_keep = a
        return a.ctypes.data_as(ctypes.c_void_p)

    def step_imag(self, n, active=None):
        self._chk(self._L.gp_batch_step_imag(self._h, int(n), self._act(active)), "gp_batch_step_imag")

    def step_real(self, n, active=None):
        self._chk(self._L.gp_batch_step_real(self._h, int(n), self._act(active)), "gp_batch_step_real")

    def norm(self):
        out = np.zeros(self.n)
        self._chk(self._L.gp_batch_norm(self._h, _dp(out)), "gp_batch_norm")
        return out

    def energy_mu(self):
        e, m = np.zeros(self.n), np.zeros(self.n)
        self._chk(self._L.gp_batch_energy_mu(self._h, _dp(e), _dp(m)), "gp_batch_energy_mu")
        return e, m

    def rms(self):
        out = np.zeros(4 * self.n)
        self._chk(self._L.gp_batch_rms(self._h, _dp(out)), "gp_batch_rms")
        return out.reshape(self.n, 4)

    def residual(self, allow_nonfinite=False):
        """(res, mu) per instance: || H[phi] phi - mu phi || and mu of phi = psi / sqrt(N).
        allow_nonfinite: return NaN/Inf entries (or a zero-norm instance's values) instead
        of raising, for callers that judge each instance themselves."""
        r, m = np.zeros(self.n), np.zeros(self.n)
        rc = self._L.gp_batch_residual(self._h, _dp(r), _dp(m))
        if allow_nonfinite and rc in (GP_ERR_NONFINITE, GP_ERR_ZERO_NORM):
            rc = GP_OK
        self._chk(rc, "gp_batch_residual")
        return r, m

    def raw_sums(self):
        out = np.zeros(9 * self.n)
        self._chk(self._L.gp_batch_raw_sums(self._h, _dp(out)), "gp_batch_raw_sums")
        return out.reshape(self.n, 9)

    def status(self):
        s = np.zeros(self.n, dtype=np.int64)
        m = np.zeros(self.n)
        f = np.zeros(self.n, dtype=np.int32)
        self._chk(self._L.gp_batch_status(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(m),
                                          f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "gp_batch_status")
        return s, m, f

    def converge_imag(self, tol=1e-7, check_every=0, max_steps=10 ** 6):
        s = np.zeros(self.n, dtype=np.int64)
        m = np.zeros(self.n)
        c = np.zeros(self.n, dtype=np.int32)
        self._chk(self._L.gp_batch_converge_imag(self._h, float(tol), int(check_every), int(max_steps),
                                                 s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(m),
                                                 c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
                  "gp_batch_converge_imag")
        return s, m, c.astype(bool)

    def get_mapping(self):
        out = (ctypes.c_int32 * 5)()
        self._chk(self._L.gp_batch_get_mapping(self._h, out), "gp_batch_get_mapping")
        return list(out)

    def set_mapping(self, mx=0, swx=0, my=0, swy=0, mz=0):
        arr = (ctypes.c_int32 * 5)(int(mx), int(swx), int(my), int(swy), int(mz))
        self._chk(self._L.gp_batch_set_mapping(self._h, arr), "gp_batch_set_mapping")

    def autotune(self, mode="imag", steps=4, cache_path=None):
        out = (ctypes.c_int32 * 5)()
        cp = cache_path.encode() if cache_path else None
        self._chk(self._L.gp_batch_autotune(self._h, 0 if mode == "imag" else 1, int(steps), cp, out),
                  "gp_batch_autotune")
        return list(out)

    def set_yz_fusion(self, on: bool):
        self._chk(self._L.gp_batch_set_yz_fusion(self._h, int(bool(on))), "gp_batch_set_yz_fusion")

    def get_yz_fusion(self):
        """(enabled, number of instances on the fused y+z path)"""
        e, f = ctypes.c_int32(), ctypes.c_int32()
        self._chk(self._L.gp_batch_get_yz_fusion(self._h, ctypes.byref(e), ctypes.byref(f)), "gp_batch_get_yz_fusion")
        return bool(e.value), f.value

    def set_timing(self, on):
        self._chk(self._L.gp_batch_set_timing(self._h, int(bool(on))), "gp_batch_set_timing")

    def get_timing(self):
        ms = np.zeros(5)
        n = np.zeros(5, dtype=np.int64)
        self._chk(self._L.gp_batch_get_timing(self._h, _dp(ms), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
                  "gp_batch_get_timing")
        return ms, n

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.gp_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
