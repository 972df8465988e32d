"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every function
include/gp.h declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1601_04641_amd import gp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp[a-z_]*)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gp.LIB_PATH):
        from paper_1601_04641_amd import build
        build.build()
    return gp.load()


def test_header_declares_the_binding_names():
    assert set(declared("gp.h")) == set(gp.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared("gp.h"):
        assert hasattr(lib, name), name


def test_strerror_and_codes(lib):
    assert gp.gp_strerror(gp.GP_OK) == "ok"
    for code in (gp.GP_ERR_INVALID, gp.GP_ERR_HIP, gp.GP_ERR_OOM, gp.GP_ERR_NONFINITE,
                 gp.GP_ERR_ZERO_NORM, gp.GP_ERR_UNSUPPORTED):
        assert gp.gp_strerror(code) not in ("ok", "unknown error code")
    assert gp.gp_strerror(12345) == "unknown error code"


@pytest.mark.parametrize("field,value", [("nx", 2), ("ny", 0), ("dx", 0.0), ("dz", -1.0),
                                         ("dt", 0.0), ("nuy", -0.5), ("g", float("nan")),
                                         ("dt", float("inf")), ("precision", 2), ("split", 7)])
def test_init_rejects_bad_params_without_device(lib, field, value):
    p = gp.make_params(8, 8, 8, 0.1, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0, 0.001)
    setattr(p, field, value)
    rc, h = gp.gp_init(p, 0x1000, 0)
    assert rc == gp.GP_ERR_INVALID and not h.value


def test_init_rejects_oversized_grids_without_device(lib):
    # more than 2048 points on an axis
    for n, prec in [((2049, 8, 8), gp.GP_C64), ((8, 8, 4096), gp.GP_C64), ((8, 2049, 8), gp.GP_C128),
                    ((8, 8, 2049), gp.GP_C128)]:
        p = gp.make_params(*n, 0.1, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0, 0.001, prec)
        rc, _ = gp.gp_init(p, 0x1000, 0)
        assert rc == gp.GP_ERR_UNSUPPORTED, n
    # every grid up to 2048 points per axis has a mapping, in both precisions (the paper's
    # large grids, lines of 1025-2048 points, z blocks beyond 64 KiB of LDS, wavefronts
    # whose rows span 2 GiB or more): init goes on to the device (and fails there only for
    # want of one)
    for n in [(1920, 1600, 1280), (1600, 1280, 960), (2048, 3, 5), (4, 3, 2032), (1100, 8, 8), (8, 8, 1020),
              (8, 8, 2040), (8, 8, 2048), (2048, 2048, 2048)]:
        for prec in (gp.GP_C64, gp.GP_C128):
            p = gp.make_params(*n, 0.1, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0, 0.001, prec)
            rc, _ = gp.gp_init(p, 0x1000, 0)
            assert rc != gp.GP_ERR_UNSUPPORTED, (n, prec)


def test_null_arguments(lib):
    p = gp.make_params(8, 8, 8, 0.1, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0, 0.001)
    assert lib.gp_init(ctypes.byref(p), None, None, None) == gp.GP_ERR_INVALID
    assert lib.gp_step_imag(None, 1) == gp.GP_ERR_INVALID
    assert lib.gp_step_real(None, 1) == gp.GP_ERR_INVALID
    assert lib.gp_norm(None, None) == gp.GP_ERR_INVALID
    assert lib.gp_destroy(None) == gp.GP_ERR_INVALID
    assert lib.gp_last_error(None) == b"null context"


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        gp._lib_backup = gp._lib
        try:
            gp._lib = None
            gp.load(str(tmp_path / "nope.so"))
        finally:
            gp._lib = gp._lib_backup


# ---------------------------------------------------------------- warm-start network (gpnn.h)
def test_gpnn_header_declares_the_binding_names():
    from paper_1601_04641_amd import nn
    assert set(declared("gpnn.h")) == set(nn.EXPORTS)


def test_library_exports_every_gpnn_symbol(lib):
    for name in declared("gpnn.h"):
        assert hasattr(lib, name), name


@pytest.mark.parametrize("field,value", [("hidden", 24), ("base", 0), ("max_batch", 0), ("dx", 0.0),
                                         ("last_ch", 48), ("nstage", 0), ("nstage", 7), ("first_ch", 8),
                                         ("base", 512)])
def test_gpnn_create_rejects_bad_arch_without_device(lib, field, value):
    from paper_1601_04641_amd import nn
    nn.load()
    a = nn.make_arch(base=2, hidden=32, ch=(32, 32, 16), dx=0.5, max_batch=2)
    if field == "last_ch":
        a.ch[a.nstage] = value
    elif field == "first_ch":
        a.ch[0] = value
    else:
        setattr(a, field, value)
    h = ctypes.c_void_p()
    assert lib.gpnn_create(ctypes.byref(a), None, ctypes.byref(h)) == nn.GPNN_ERR_INVALID
    assert not h.value


@pytest.mark.parametrize("args", [(2, 1, 4, 32, 16), (3, 1, 4, 8, 16), (3, 1, 4, 32, 24), (3, 0, 4, 32, 16),
                                  (3, 1, 0, 32, 16)])
def test_gpnn_conv_rejects_bad_shapes_without_device(lib, args):
    from paper_1601_04641_amd import nn
    nn.load()
    ks, n, d, cin, cout = args
    assert lib.gpnn_conv(ks, n, d, cin, cout, 0x1000, 0x1000, None, 0, None, 0x1000, None, None) == \
        nn.GPNN_ERR_INVALID
    assert lib.gpnn_conv_wgrad(ks, n, d, cin, cout, 0x1000, 0x1000, 0x1000, None, None) == nn.GPNN_ERR_INVALID


def test_batch_rejects_bad_offsets_before_the_device():
    """Offsets are checked against psi's length on the host: the C-ABI has no buffer
    length, so a short or overlapping layout would otherwise reach the kernels."""
    import torch
    ws = [dict(nx=4, ny=5, nz=6, dx=0.2, dy=0.2, dz=0.2, nux=1, nuy=1, nuz=1, g=1, dt=0.004),
          dict(nx=3, ny=3, nz=3, dx=0.2, dy=0.2, dz=0.2, nux=1, nuy=1, nuz=1, g=1, dt=0.004)]
    psi = torch.zeros(120 + 27, dtype=torch.complex64)
    for offs in ([0], [0, 120, 5], [0, 121], [-1, 120], [0, 100], [27, 0]):
        with pytest.raises(ValueError):
            gp.Batch(psi, ws, offs)
    with pytest.raises(ValueError, match="device"):   # a valid layout reaches the device check
        gp.Batch(psi, ws, [27, 0])


def test_set_psi_checks_shape_dtype_and_device():
    import torch
    a = torch.zeros((4, 5, 6), dtype=torch.complex128)
    for bad in (torch.zeros((4, 5, 7), dtype=torch.complex128), torch.zeros((4, 5, 6), dtype=torch.complex64),
                torch.zeros(120, dtype=torch.complex128)):
        with pytest.raises(ValueError):
            gp._check_like(bad, a.shape, a.dtype, a.device)
    with pytest.raises(ValueError):   # right shape and dtype, but host memory
        gp._check_like(a.clone(), a.shape, a.dtype, a.device)
