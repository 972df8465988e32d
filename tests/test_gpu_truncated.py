"""GPU: the halo-truncated Crank-Nicolson inverse (gp_set_truncation modes 1 and 2: streaming
x and y sweeps; streaming x sweep and the fused y+z pass), against the CPU FP64 oracle's
exact Thomas solves.

The truncation length H is chosen so that the dropped tail of the back-substitution,
|a|^(H+1) / (1 - |a|) of the largest forward value, is 1/100 of the storage precision's
unit roundoff; the results must therefore meet the exact sweeps' tolerances (complex128
1e-13 relative to max|psi|, complex64 2e-6).  Shapes include lines shorter than H + 1,
ragged sizes, both step kinds and both splittings, and the quench grid at full size.
"""
import sys

import numpy as np
import pytest

import oracle
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


def run(prm, psi0, prec, imag, n, split=0, mode=1):
    dt = torch.complex64 if prec == gp.GP_C64 else torch.complex128
    psi = torch.from_numpy(np.ascontiguousarray(psi0)).to(device="cuda", dtype=dt)
    with gp.Solver.from_workload(psi, prm, split=split) as s:
        s.set_truncation(mode)
        got, h = s.get_truncation()
        assert got == mode
        (s.step_imag if imag else s.step_real)(n)
        torch.cuda.synchronize()
        return psi.cpu().numpy().astype(np.complex128), h


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


SHAPES = [(3, 3, 3), (5, 7, 3), (33, 47, 29), (65, 9, 70), (130, 17, 33), (300, 5, 4), (4, 257, 6)]


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
@pytest.mark.parametrize("imag,split", [(True, 0), (False, 0), (True, 1), (False, 1)])
def test_truncated_sweeps_match_oracle(shape, prec, imag, split, mode):
    nx, ny, nz = shape
    prm = dict(nx=nx, ny=ny, nz=nz, dx=0.21, dy=0.17, dz=0.25, nux=1.1, nuy=1.6, nuz=0.9, g=30.0, dt=0.004)
    psi0 = inputs.perturbed_psi(nx, ny, nz, prm["dx"], prm["dy"], prm["dz"], 1.0, 1.3, 0.8, seed=nx * 5 + ny, amp=0.2)
    if prec == gp.GP_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    out, h = run(prm, psi0, prec, imag, 4, split=split, mode=mode)
    o = oracle.Oracle.from_params(prm, psi0, split=split)
    (o.step_imag if imag else o.step_real)(4)
    err = rel_err(out, o.psi)
    tol = 1e-13 if prec == gp.GP_C128 else 2e-6
    say(f"case: truncated mode {mode} {shape} prec {prec} imag {imag} split {split} H {h}: rel err {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("prec,imag", [(gp.GP_C64, False), (gp.GP_C128, False), (gp.GP_C64, True),
                                       (gp.GP_C128, True)])
def test_truncated_quench_grid(prec, imag, mode):
    w = inputs.WORKLOADS["quench_512x480x448"]
    prm = dict(w)
    if imag:
        prm["dt"] = w["dt_imag"]
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    psi0 = inputs.perturbed_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], 2.0, 2.5, 3.0, seed=9, amp=0.1)
    if prec == gp.GP_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    out, h = run(prm, psi0, prec, imag, 2, mode=mode)
    o = oracle.Oracle.from_params(prm, psi0)
    (o.step_imag if imag else o.step_real)(2)
    err = rel_err(out, o.psi)
    o.close()
    tol = (1e-12 if imag else 1e-13) if prec == gp.GP_C128 else 2e-6
    say(f"case: truncated mode {mode} quench grid prec {prec} imag {imag} H {h}: rel err {err:.2e}")
    assert err <= tol


def test_truncation_lengths_and_limits():
    """H from the rule: imaginary dt = 0.1 dx^2 (|a| = 0.024) needs 5 (complex64) and 11
    (complex128) terms, real dt = 0.01 dx^2 (|a| = 0.0025) 3 and 6; a large dt/dx^2 (|a|
    near 1) needs more than the kernels hold and is refused, the exact sweeps staying on."""
    prm = dict(nx=16, ny=12, nz=10, dx=0.2, dy=0.2, dz=0.2, nux=1.0, nuy=1.0, nuz=1.0, g=1.0, dt=0.004)
    psi0 = inputs.gaussian_psi(16, 12, 10, 0.2, 0.2, 0.2, 1, 1, 1)
    for prec, want in ((gp.GP_C64, (5, 3)), (gp.GP_C128, (11, 6))):
        dt = torch.complex64 if prec == gp.GP_C64 else torch.complex128
        psi = torch.from_numpy(psi0).to(device="cuda", dtype=dt)
        with gp.Solver.from_workload(psi, dict(prm, dt=0.1 * 0.04)) as s:
            _, h = s.get_truncation()
            assert h[0][0] == want[0], h
        with gp.Solver.from_workload(psi, dict(prm, dt=0.01 * 0.04)) as s:
            _, h = s.get_truncation()
            assert h[1][0] == want[1], h
        with gp.Solver.from_workload(psi, dict(prm, dt=4.0)) as s:
            with pytest.raises(gp.GPError) as ei:
                s.set_truncation(1)
            assert ei.value.code == gp.GP_ERR_UNSUPPORTED
            assert s.get_truncation()[0] == 0


def test_fused_pass_limits_and_norm():
    """The fused pass holds z lines of at most 1024 points; in imaginary time its norm
    partials renormalise like the exact z sweep's (norm 1 on return, mu_est as exact)."""
    prm = dict(nx=6, ny=5, nz=1100, dx=0.03, dy=0.03, dz=0.03, nux=1.0, nuy=1.0, nuz=1.0, g=1.0, dt=4e-4)
    psi = torch.zeros((6, 5, 1100), dtype=torch.complex64, device="cuda")
    with gp.Solver.from_workload(psi, prm) as s:
        with pytest.raises(gp.GPError) as ei:
            s.set_truncation(2)
        assert ei.value.code == gp.GP_ERR_UNSUPPORTED
    w = dict(inputs.WORKLOADS["imag_48x40x32"])
    psi0 = inputs.gaussian_psi(48, 40, 32, w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"])
    ests = []
    for mode in (0, 2):
        psi = torch.from_numpy(psi0).to("cuda")
        with gp.Solver.from_workload(psi, w) as s:
            s.set_truncation(mode)
            s.step_imag(37)
            assert abs(s.norm() - 1.0) <= 1e-12
            ests.append(s.status()[1])
    assert abs(ests[0] - ests[1]) <= 1e-12 * abs(ests[0])


@pytest.mark.parametrize("imag", [True, False])
def test_fused_pass_large_lds(imag):
    """960-point z lines: one group of rows needs 130-147 KB of LDS in complex64 (the
    blocks opt in beyond 64 KiB) and matches the oracle; complex128 would need 261-392 KB
    and is refused, the exact sweeps staying on.  dt = 0.1 dx^2 (imaginary) and
    0.01 dx^2 (real), as the workloads use (H = 5 / 3 in complex64, 11 / 6 in complex128)."""
    nx, ny, nz = 3, 40, 960
    dx = 0.03
    prm = dict(nx=nx, ny=ny, nz=nz, dx=dx, dy=dx, dz=dx, nux=1.3, nuy=1.1, nuz=0.9, g=30.0,
               dt=(0.1 if imag else 0.01) * dx * dx)
    psi0 = inputs.perturbed_psi(nx, ny, nz, dx, dx, dx, 0.03, 0.04, 0.05, seed=960, amp=0.2)
    psi = torch.from_numpy(psi0).to("cuda")
    with gp.Solver.from_workload(psi, prm) as s:
        with pytest.raises(gp.GPError) as ei:
            s.set_truncation(2)
        assert ei.value.code == gp.GP_ERR_UNSUPPORTED
        assert s.get_truncation()[0] == 0
    psi0 = psi0.astype(np.complex64).astype(np.complex128)
    out, h = run(prm, psi0, gp.GP_C64, imag, 3, mode=2)
    o = oracle.Oracle.from_params(prm, psi0)
    (o.step_imag if imag else o.step_real)(3)
    err = rel_err(out, o.psi)
    say(f"case: fused pass 960-point z lines imag {imag} H {h}: rel err {err:.2e}")
    assert err <= 2e-6
