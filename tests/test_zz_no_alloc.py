"""GPU: gp_raw_sums_noalloc, the observable sums without a context (file-scope device
scratch, no allocation), against gp_raw_sums of a context on the same state: bitwise,
on two calls in a row whose second state is smaller, in both precisions."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1601_04641_amd import gp, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gp.load()
    yield


def case(shape, prec, seed):
    nx, ny, nz = shape
    w = dict(nx=nx, ny=ny, nz=nz, dx=0.21, dy=0.17, dz=0.25, nux=1.1, nuy=1.6, nuz=0.9, g=30.0, dt=0.004)
    psi0 = inputs.perturbed_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], 1.0, 1.3, 0.8, seed=seed, amp=0.4) * 1.3
    dt = torch.complex128 if prec == gp.GP_C128 else torch.complex64
    return w, torch.from_numpy(psi0).to(device="cuda", dtype=dt)


def noalloc(w, psi, prec, out):
    p = gp.make_params(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"],
                       w["g"], w["dt"], prec)
    stream = torch.cuda.current_stream().cuda_stream
    return gp.load().gp_raw_sums_noalloc(ctypes.byref(p), ctypes.c_void_p(psi.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream))


@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
def test_noalloc_raw_sums_match_context(prec):
    out = torch.full((9,), float("nan"), dtype=torch.float64, device="cuda")
    # a grid large enough for the full 2048-block reduction, then a smaller one
    for shape, seed in (((160, 130, 96), 3), ((33, 47, 29), 4)):
        w, psi = case(shape, prec, seed)
        rc = noalloc(w, psi, prec, out)
        assert rc == gp.GP_OK
        torch.cuda.synchronize()
        got = out.cpu().numpy().copy()
        with gp.Solver.from_workload(psi, w) as s:
            want = s.raw_sums()
        say(f"case: noalloc raw sums {shape} prec {prec}: max rel diff "
            f"{np.max(np.abs(got - want) / np.abs(want)):.1e}")
        assert np.array_equal(got, want)


def test_noalloc_rejects_bad_arguments():
    out = torch.zeros(9, dtype=torch.float64, device="cuda")
    w, psi = case((8, 8, 8), gp.GP_C128, 1)
    assert noalloc(dict(w, nx=2), psi, gp.GP_C128, out) == gp.GP_ERR_INVALID
    assert noalloc(dict(w, nz=4096), psi, gp.GP_C128, out) == gp.GP_ERR_UNSUPPORTED
    p = gp.make_params(8, 8, 8, 0.1, 0.1, 0.1, 1, 1, 1, 1, 0.01, gp.GP_C128)
    L = gp.load()
    assert L.gp_raw_sums_noalloc(ctypes.byref(p), None, ctypes.c_void_p(out.data_ptr()), None) == gp.GP_ERR_INVALID
    assert L.gp_raw_sums_noalloc(ctypes.byref(p), ctypes.c_void_p(psi.data_ptr()), None, None) == gp.GP_ERR_INVALID
