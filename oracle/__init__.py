"""CPU FP64 oracle for the split-step Crank-Nicolson Gross-Pitaevskii solver.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
``cpu_baseline`` leg are the only code allowed to import this package; the product path
(``paper_1601_04641_amd``) never does, and this package imports nothing from it.

The arithmetic lives in ``gpref.cpp`` (plain C++, ``std::complex<double>``, OpenMP over
independent lines only).  This module builds it with g++ and wraps it with ctypes; the
wrapper does argument marshalling only.

Every function follows the paper's description of the method (program summary,
"Solution method"; the sub-step functions calcnu, calclux, calcluy, calcluz, calcrms,
calcmuen named under "Summary of revisions"); the readings taken where the paper prints
no formula are listed at the top of ``gpref.cpp``.  The pins that tie it to mathematics
independent of itself are in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgpref.so")
_SRC = os.path.join(_HERE, "gpref.cpp")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no fast-math) into oracle/libgpref.so."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp"
    cmd = ["g++", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("nux", ctypes.c_double), ("nuy", ctypes.c_double), ("nuz", ctypes.c_double),
                ("g", ctypes.c_double), ("dt", ctypes.c_double), ("split", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        vp, dp, i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32
        L.gpref_init.argtypes = [ctypes.POINTER(_Params), dp, ctypes.POINTER(vp)]
        for name, extra in [("gpref_destroy", []), ("gpref_set_g", [ctypes.c_double]),
                            ("gpref_step_imag", [i32]), ("gpref_step_real", [i32]),
                            ("gpref_last_npre", [dp]), ("gpref_norm", [dp]),
                            ("gpref_raw_sums", [dp]), ("gpref_energy_mu", [dp, dp]),
                            ("gpref_rms", [dp]),
                            ("gpref_substep", [i32, i32, ctypes.c_double])]:
            f = getattr(L, name)
            f.argtypes = [vp] + extra
            f.restype = ctypes.c_int
        L.gpref_init.restype = ctypes.c_int
        L.gpref_set_threads.argtypes = [i32]
        L.gpref_cn_line.argtypes = [i32, ctypes.c_double, ctypes.c_double, dp]
        L.gpref_cn_line.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> None:
    lib().gpref_set_threads(int(n))


def cn_line(psi_line: np.ndarray, c: complex) -> np.ndarray:
    """One Crank-Nicolson solve of a single line (copy returned)."""
    a = np.ascontiguousarray(psi_line, dtype=np.complex128).copy()
    rc = lib().gpref_cn_line(a.size, float(np.real(c)), float(np.imag(c)), _dptr(a.view(np.float64)))
    if rc != 0:
        raise ValueError("gpref_cn_line: invalid input")
    return a


class Oracle:
    """Owns a complex128 copy of psi ([nx][ny][nz], z fastest) and steps it in place."""

    def __init__(self, nx, ny, nz, dx, dy, dz, nux, nuy, nuz, g, dt, psi0, split=0):
        self.shape = (int(nx), int(ny), int(nz))
        self.psi = np.ascontiguousarray(psi0, dtype=np.complex128).reshape(self.shape).copy()
        self._p = _Params(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
                          float(nux), float(nuy), float(nuz), float(g), float(dt), int(split))
        h = ctypes.c_void_p()
        rc = lib().gpref_init(ctypes.byref(self._p), _dptr(self.psi.view(np.float64)), ctypes.byref(h))
        if rc != 0:
            raise ValueError("gpref_init: invalid parameters")
        self._h = h

    @classmethod
    def from_params(cls, prm: dict, psi0, split=0):
        return cls(prm["nx"], prm["ny"], prm["nz"], prm["dx"], prm["dy"], prm["dz"],
                   prm["nux"], prm["nuy"], prm["nuz"], prm["g"], prm["dt"], psi0,
                   split=prm.get("split", split))

    def _chk(self, rc, name):
        if rc != 0:
            raise ValueError(f"{name} failed ({rc})")

    def step_imag(self, n: int):
        self._chk(lib().gpref_step_imag(self._h, int(n)), "gpref_step_imag")

    def step_real(self, n: int):
        self._chk(lib().gpref_step_real(self._h, int(n)), "gpref_step_real")

    def substep(self, which: int, imag: bool, tau: float):
        self._chk(lib().gpref_substep(self._h, int(which), int(bool(imag)), float(tau)), "gpref_substep")

    def set_g(self, g: float):
        self._chk(lib().gpref_set_g(self._h, float(g)), "gpref_set_g")

    def last_npre(self) -> float:
        v = ctypes.c_double()
        self._chk(lib().gpref_last_npre(self._h, ctypes.byref(v)), "gpref_last_npre")
        return v.value

    def norm(self) -> float:
        v = ctypes.c_double()
        self._chk(lib().gpref_norm(self._h, ctypes.byref(v)), "gpref_norm")
        return v.value

    def raw_sums(self) -> np.ndarray:
        out = np.zeros(9)
        self._chk(lib().gpref_raw_sums(self._h, _dptr(out)), "gpref_raw_sums")
        return out

    def energy_mu(self):
        e, m = ctypes.c_double(), ctypes.c_double()
        self._chk(lib().gpref_energy_mu(self._h, ctypes.byref(e), ctypes.byref(m)), "gpref_energy_mu")
        return e.value, m.value

    def rms(self) -> np.ndarray:
        out = np.zeros(4)
        self._chk(lib().gpref_rms(self._h, _dptr(out)), "gpref_rms")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gpref_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
