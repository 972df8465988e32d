"""GPU: the device sin/cos of the real-time phase factor against an extended-precision
host reference, and the plain streaming-copy kernel the bandwidths are compared with.

sin/cos: Cody and Waite's reduction modulo pi/2 and Taylor series (the routine the
real-time potential step calls), evaluated on dense samples; the reference is the host
C library in 80-bit long double (numpy longdouble, 64-bit significand), 11 bits beyond
FP64, so its own error is below 1e-3 of an FP64 ulp.  Error is measured in ulps of the
true value rounded to the routine's precision.
"""
import ctypes
import sys

import numpy as np
import pytest

from paper_1601_04641_amd import gp

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


def ulp_err(got, x, dtype):
    xl = x.astype(np.longdouble)
    worst = []
    for f, g in ((np.sin, got[0]), (np.cos, got[1])):
        ref = f(xl)
        ulp = np.spacing(np.abs(ref).astype(dtype)).astype(np.longdouble)
        tiny = np.spacing(np.finfo(dtype).tiny)
        ulp = np.maximum(ulp, tiny)
        worst.append(float(np.max(np.abs(g.astype(np.longdouble) - ref) / ulp)))
    return worst


def samples(dtype, big):
    rng = np.random.default_rng(7)
    parts = [np.linspace(-1e4, 1e4, 1 << 23),                       # the reduced range, dense
             np.linspace(-0.125, 0.125, 1 << 20),                   # the short-series range
             rng.uniform(1e4, big, 1 << 20) * rng.choice([-1, 1], 1 << 20)]  # the FP64-reduced range
    return np.concatenate(parts).astype(dtype)


@pytest.mark.parametrize("dtype,big,bound", [(np.float32, 6e4, 1.5), (np.float64, 6e9, 1.5)])
def test_device_sincos_error_bound(dtype, big, bound):
    x = samples(dtype, big)
    xd = torch.from_numpy(x).cuda()
    s, c = gp.eval_sincos(xd)
    got = (s.cpu().numpy(), c.cpu().numpy())
    es, ec = ulp_err(got, x, dtype)
    say(f"case: sincos {np.dtype(dtype).name} on {x.size} arguments up to {big:.0e}: "
        f"worst {es:.3f} ulp (sin), {ec:.3f} ulp (cos)")
    assert es <= bound and ec <= bound
    # identities the quadrant logic must keep: exact zeros, odd/even symmetry
    assert got[0][np.nonzero(x == 0)[0]].tolist() == [0.0] * int(np.sum(x == 0))
    sm, cm = gp.eval_sincos(torch.from_numpy(-x).cuda())
    assert np.array_equal(sm.cpu().numpy(), -got[0]) and np.array_equal(cm.cpu().numpy(), got[1])


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) + 48, 64 << 20])
def test_stream_copy_is_exact(nbytes):
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    gp.stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_stream_copy_rejects_bad_sizes():
    L = gp.load()
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    assert L.gp_stream_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), 24, None) == gp.GP_ERR_INVALID
    assert L.gp_stream_copy(ctypes.c_void_p(a.data_ptr() + 8), ctypes.c_void_p(b.data_ptr()), 32, None) == \
        gp.GP_ERR_INVALID
    assert L.gp_stream_copy(None, ctypes.c_void_p(b.data_ptr()), 32, None) == gp.GP_ERR_INVALID
