"""GPU parity: the HIP path (through the C-ABI) against the CPU FP64 oracle.

Tolerances follow from the arithmetic: complex128 agrees
with the oracle to a few units of FP64 rounding per step; complex64 carries FP32 storage
and sweeps (unit roundoff 6e-8) and FP64 reductions, so one step differs by ~1e-7 of
max|psi| and the long imaginary-time run is held to the stated precision-form bound
(1e-5 relative mu, 1e-4 max|dpsi|).
"""
import math
import sys
import time

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


def dev_psi(psi0, prec):
    dt = torch.complex128 if prec == gp.GP_C128 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(psi0)).to(device="cuda", dtype=dt)


def run_gpu(prm, psi0, prec, imag, n, split=0, mapping=None):
    psi = dev_psi(psi0, prec)
    with gp.Solver.from_workload(psi, prm, split=split) as s:
        if mapping:
            s.set_mapping(*mapping)
        (s.step_imag if imag else s.step_real)(n)
        torch.cuda.synchronize()
        return psi.cpu().numpy().astype(np.complex128), s


def run_ref(prm, psi0, imag, n, split=0):
    o = oracle.Oracle.from_params(prm, psi0, split=split)
    (o.step_imag if imag else o.step_real)(n)
    return o


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# ----------------------------------------------------------------------------------------
# the small anisotropic imaginary-time workload, 500 steps
# ----------------------------------------------------------------------------------------
def c1():
    w = dict(inputs.WORKLOADS["imag_48x40x32"])
    psi0 = inputs.gaussian_psi(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"])
    return w, psi0


@pytest.fixture(scope="module")
def c1_ref():
    w, psi0 = c1()
    o = run_ref(w, psi0, True, w["steps"])
    return w, psi0, o, o.energy_mu(), o.rms(), o.norm()


def test_c1_imag_c128_matches_oracle(c1_ref):
    w, psi0, o, (e_r, mu_r), rms_r, n_r = c1_ref
    say("case: imag 48x40x32 c128 500 steps")
    psi = dev_psi(psi0, gp.GP_C128)
    with gp.Solver.from_workload(psi, w) as s:
        s.step_imag(w["steps"])
        e, mu = s.energy_mu()
        rms = s.rms()
        nrm = s.norm()
        steps, mu_est, flags = s.status()
    out = psi.cpu().numpy()
    say(f"mu {mu!r} vs {mu_r!r}; E {e!r} vs {e_r!r}; max|dpsi| {np.max(np.abs(out - o.psi)):.3e}")
    assert abs(mu - mu_r) <= 1e-10 * abs(mu_r)
    assert abs(e - e_r) <= 1e-10 * abs(e_r)
    assert np.max(np.abs(rms - rms_r) / rms_r) <= 1e-10
    assert abs(nrm - 1.0) <= 1e-12 and abs(n_r - 1.0) <= 1e-12
    assert np.max(np.abs(out - o.psi)) <= 1e-10
    assert np.all(out.imag == 0.0)   # imaginary time keeps a real state real, bitwise
    assert steps == w["steps"] and flags == 0
    assert abs(mu_est - (-math.log(o.last_npre()) / (2 * w["dt"]))) <= 1e-8 * abs(mu_est)


def test_c1_imag_c64_within_precision_bound(c1_ref):
    w, psi0, o, (e_r, mu_r), rms_r, _ = c1_ref
    say("case: imag 48x40x32 c64 500 steps")
    psi = dev_psi(psi0, gp.GP_C64)
    with gp.Solver.from_workload(psi, w) as s:
        s.step_imag(w["steps"])
        e, mu = s.energy_mu()
        rms = s.rms()
    out = psi.cpu().numpy().astype(np.complex128)
    say(f"c64 rel mu {abs(mu - mu_r) / mu_r:.2e}, rel E {abs(e - e_r) / e_r:.2e}, "
        f"max|dpsi| {np.max(np.abs(out - o.psi)):.2e}")
    assert abs(mu - mu_r) <= 1e-5 * abs(mu_r)
    assert abs(e - e_r) <= 1e-5 * abs(e_r)
    assert np.max(np.abs(rms - rms_r) / rms_r) <= 1e-5
    assert np.max(np.abs(out - o.psi)) <= 1e-4


# ----------------------------------------------------------------------------------------
# ragged and odd shapes, both time kinds, both splittings, both precisions
# ----------------------------------------------------------------------------------------
SHAPES = [(3, 3, 3), (5, 7, 3), (33, 47, 29), (65, 9, 70), (17, 130, 33), (100, 3, 5), (24, 20, 64)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
@pytest.mark.parametrize("imag,split", [(True, 0), (False, 0), (True, 1), (False, 1)])
def test_ragged_shapes_match_oracle(shape, prec, imag, split):
    nx, ny, nz = shape
    prm = dict(nx=nx, ny=ny, nz=nz, dx=0.21, dy=0.17, dz=0.25, nux=1.1, nuy=1.6, nuz=0.9, g=30.0, dt=0.004)
    psi0 = inputs.perturbed_psi(nx, ny, nz, prm["dx"], prm["dy"], prm["dz"], 1.0, 1.3, 0.8, seed=nx * 7 + nz,
                                amp=0.2)
    say(f"case: shape {shape} prec {prec} imag {imag} split {split}")
    out, _ = run_gpu(prm, psi0, prec, imag, 3, split=split)
    ref = run_ref(prm, psi0, imag, 3, split=split).psi
    err = rel_err(out, ref)
    tol = 1e-13 if prec == gp.GP_C128 else 2e-6
    say(f"  rel err {err:.2e} (tol {tol:.0e})")
    assert err <= tol


@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
@pytest.mark.parametrize("imag", [True, False])
def test_large_dt_long_head_correction(prec, imag):
    """dt/dx^2 ~ 5-40: c'_inf close to 1, so the constant-pivot solve needs Sherman-Morrison
    corrections longer than one thread's segment (applied inside the x/y sweeps with 8 or
    16 points per thread, the default mappings here)."""
    nx, ny, nz = 70, 45, 33
    prm = dict(nx=nx, ny=ny, nz=nz, dx=0.1, dy=0.15, dz=0.05, nux=1.0, nuy=1.2, nuz=0.8, g=5.0, dt=0.1)
    psi0 = inputs.perturbed_psi(nx, ny, nz, 0.1, 0.15, 0.05, 1.0, 1.2, 0.8, seed=12, amp=0.2)
    say(f"case: large dt prec {prec} imag {imag}")
    out, _ = run_gpu(prm, psi0, prec, imag, 2)
    ref = run_ref(prm, psi0, imag, 2).psi
    err = rel_err(out, ref)
    say(f"  rel err {err:.2e}")
    assert err <= (1e-12 if prec == gp.GP_C128 else 5e-6)


@pytest.mark.parametrize("imag", [True, False])
def test_large_dt_head_correction_separate_pass(imag):
    """The same large-dt problem in complex64 with 12 and 10 points per thread along x and y:
    instances without the in-kernel long correction, so the separate correction pass runs."""
    nx, ny, nz = 70, 45, 33
    prm = dict(nx=nx, ny=ny, nz=nz, dx=0.1, dy=0.15, dz=0.05, nux=1.0, nuy=1.2, nuz=0.8, g=5.0, dt=0.1)
    psi0 = inputs.perturbed_psi(nx, ny, nz, 0.1, 0.15, 0.05, 1.0, 1.2, 0.8, seed=12, amp=0.2)
    say(f"case: large dt, separate correction pass, c64 mapping (12, 4 | 10, 2) imag {imag}")
    out, _ = run_gpu(prm, psi0, gp.GP_C64, imag, 2, mapping=(12, 4, 10, 2, 0, 0))
    ref = run_ref(prm, psi0, imag, 2).psi
    err = rel_err(out, ref)
    say(f"  rel err {err:.2e}")
    assert err <= 5e-6


MAPPINGS = [(8, 1, 8, 1, 4, 0), (16, 1, 16, 2, 8, 0), (32, 2, 8, 4, 16, 0), (0, 4, 0, 1, 32, 0),
            (16, 4, 32, 1, 64, 0), (8, 2, 16, 4, 0, 0), (12, 4, 10, 2, 0, 0), (10, 1, 12, 1, 0, 0)]


@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
@pytest.mark.parametrize("mapping", MAPPINGS)
def test_every_line_mapping_agrees(prec, mapping):
    nx, ny, nz = 96, 70, 45
    prm = dict(nx=nx, ny=ny, nz=nz, dx=0.2, dy=0.2, dz=0.2, nux=1.0, nuy=1.4142, nuz=1.7321, g=50.0, dt=0.004)
    psi0 = inputs.perturbed_psi(nx, ny, nz, 0.2, 0.2, 0.2, 1.0, 1.4, 1.7, seed=4, amp=0.1)
    if prec == gp.GP_C128:   # complex128 runs 8 or 16 points per thread
        mapping = tuple((16 if v == 32 else 8 if v in (10, 12) else v) if i in (0, 2) else v
                        for i, v in enumerate(mapping))
    say(f"case: mapping {mapping} prec {prec}")
    for imag in (True, False):
        out, s = run_gpu(prm, psi0, prec, imag, 2, mapping=mapping)
        ref = run_ref(prm, psi0, imag, 2).psi
        err = rel_err(out, ref)
        say(f"  imag {imag} rel err {err:.2e}")
        assert err <= (1e-13 if prec == gp.GP_C128 else 2e-6)


def test_invalid_mapping_rejected():
    prm = dict(nx=48, ny=40, nz=32, dx=0.2, dy=0.2, dz=0.2, nux=1.0, nuy=1.0, nuz=1.0, g=1.0, dt=0.004)
    psi = dev_psi(inputs.gaussian_psi(48, 40, 32, 0.2, 0.2, 0.2, 1, 1, 1), gp.GP_C128)
    with gp.Solver.from_workload(psi, prm) as s:
        before = s.get_mapping()
        for bad in [(1, 1, 0, 0, 0, 0), (0, 3, 0, 0, 0, 0), (0, 0, 0, 0, 3, 0), (0, 0, 0, 0, 4, 3),
                    (64, 0, 0, 0, 0, 0), (0, 0, 0, 0, 128, 0), (0, 0, 24, 8, 0, 0)]:
            with pytest.raises(gp.GPError):
                s.set_mapping(*bad)
        assert s.get_mapping() == before


@pytest.mark.parametrize("prec,g", [(gp.GP_C128, 1e10), (gp.GP_C128, 1e14), (gp.GP_C64, 1e7), (gp.GP_C64, 1e9)])
def test_large_real_time_phases(prec, g):
    """One real-time step whose nonlinear phase tau g |psi|^2 reaches ~6e5..6e9 (complex128)
    or ~6e2..6e4 rad (complex64): every argument reduction of the phase factor's sin/cos
    is exercised.  The phase is computed from the stored precision's |psi|^2, so the bound
    scales with the largest phase: 10 x theta x unit roundoff."""
    nx, ny, nz = 16, 12, 10
    prm = dict(nx=nx, ny=ny, nz=nz, dx=0.2, dy=0.2, dz=0.2, nux=0.0, nuy=0.0, nuz=0.0, g=g, dt=0.001)
    psi0 = inputs.perturbed_psi(nx, ny, nz, 0.2, 0.2, 0.2, 1.0, 1.0, 1.0, seed=31, amp=0.3)
    if prec == gp.GP_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    theta = prm["dt"] * g * float(np.max(np.abs(psi0) ** 2))
    say(f"case: large phase prec {prec} g {g:.0e}: theta max {theta:.2e}")
    out, _ = run_gpu(prm, psi0, prec, False, 1)
    ref = run_ref(prm, psi0, False, 1).psi
    err = rel_err(out, ref)
    eps = 2.0 ** -53 if prec == gp.GP_C128 else 2.0 ** -24
    say(f"  rel err {err:.2e} (bound {10 * theta * eps + 1e-12:.2e})")
    assert err <= 10 * theta * eps + 1e-12


# ----------------------------------------------------------------------------------------
# full 512x480x448 shape: closed forms (any size) and one step against the oracle
# ----------------------------------------------------------------------------------------
BIG = (512, 480, 448)


def sine_factor(n, k, c):
    s2 = math.sin(k * math.pi / (2 * (n + 1))) ** 2
    return (1 - 4 * c * s2) / (1 + 4 * c * s2)


@pytest.mark.parametrize("prec", [gp.GP_C64, gp.GP_C128])
def test_full_size_sine_modes_closed_form(prec):
    nx, ny, nz = BIG
    d, dt = 0.05, 0.01 * 0.05 ** 2
    modes = (3, 2, 5)
    prm = dict(nx=nx, ny=ny, nz=nz, dx=d, dy=d, dz=d, nux=0.0, nuy=0.0, nuz=0.0, g=0.0, dt=dt)
    say(f"case: full-size sine modes prec {prec}")
    psi0 = inputs.sine_mode_psi(nx, ny, nz, *modes, dtype=np.complex64 if prec == gp.GP_C64 else np.complex128)
    psi = dev_psi(psi0, prec)
    want = torch.from_numpy(np.ascontiguousarray(psi0)).to("cuda")
    f = 1.0
    for n, k in zip(BIG, modes):
        f *= sine_factor(n, k, 1j * dt / (4 * d * d))
    with gp.Solver.from_workload(psi, prm) as s:
        s.step_real(1)
        torch.cuda.synchronize()
        err = float((psi - want * f).abs().max())
    tol = 1e-13 if prec == gp.GP_C128 else 1e-6
    say(f"  max err {err:.2e}")
    assert err <= tol
    del psi, want
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,imag", [(gp.GP_C64, False), (gp.GP_C128, False), (gp.GP_C128, True)])
def test_full_size_step_matches_oracle(prec, imag):
    """Quench workload grid in the default line mapping, 2 steps from a seeded state,
    compared with the oracle at every point (the benchmark's autotuned mapping is covered
    by test_gpu_mappings.test_quench_grid_in_benchmark_mapping)."""
    w = inputs.WORKLOADS["quench_512x480x448"]
    prm = dict(w)
    if imag:
        prm["dt"] = w["dt_imag"]
    nx, ny, nz = BIG
    say(f"case: full-size {BIG} prec {prec} imag {imag}: building input")
    psi0 = inputs.perturbed_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], 2.0, 2.5, 3.0, seed=9, amp=0.1)
    t0 = time.time()
    out, _ = run_gpu(prm, psi0, prec, imag, 2)
    say(f"  gpu done ({time.time() - t0:.1f}s); running oracle")
    t0 = time.time()
    ref = run_ref(prm, psi0, imag, 2).psi
    say(f"  oracle done ({time.time() - t0:.1f}s)")
    err = rel_err(out, ref)
    say(f"  rel err {err:.2e}")
    # imaginary time renormalises by a sum of 1.1e8 terms; the oracle's sequential FP64
    # partial sums (~7e6 terms per thread) carry ~sqrt(7e6)*1.1e-16 = 3e-13 relative error
    tol = (1e-12 if imag else 1e-13) if prec == gp.GP_C128 else 2e-6
    assert err <= tol


# ----------------------------------------------------------------------------------------
# invariants, determinism, graphs, quench, status and error paths
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
def test_real_time_norm_conserved(prec):
    w, psi0 = c1()
    prm = dict(w, dt=0.001)
    psi0 = inputs.perturbed_psi(48, 40, 32, 0.2, 0.2, 0.2, 1.0, 1.4, 1.7, seed=2, amp=0.3)
    psi = dev_psi(psi0, prec)
    with gp.Solver.from_workload(psi, prm) as s:
        n0 = s.norm()
        s.step_real(1000)
        n1 = s.norm()
    drift = abs(n1 - n0) / n0
    say(f"case: norm drift prec {prec}: {drift:.2e}")
    # complex128: FP64 roundoff.  complex64: the near-unit-modulus CN coefficient is
    # carried as an FP32 hi+lo pair, which removes the ~1.7e-4 per-1000-step bias of a
    # single-float coefficient; what remains is the per-point FP32 rounding of the phase
    # factor and of the stored values, fixed per point from step to step, whose
    # |psi|^2-weighted mean over a few hundred effective points is ~1e-9 per step.
    assert drift <= (1e-12 if prec == gp.GP_C128 else 3e-5)


@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
def test_bitwise_deterministic_and_graph_equals_eager(prec):
    w, psi0 = c1()
    outs = []
    for timing in (False, False, True):   # graphs, graphs again, eager with events
        psi = dev_psi(psi0, prec)
        with gp.Solver.from_workload(psi, w) as s:
            s.set_timing(timing)
            s.step_imag(37)
            s.step_real(21)
            torch.cuda.synchronize()
            outs.append(psi.cpu().numpy())
            if timing:
                ms, n = s.get_timing()
                assert n[0] == 58 and n[1] == 58 and n[2] == 58 and n[3] == 37
                assert np.all(ms[:4] > 0)
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


def test_quench_set_g_matches_oracle():
    w, psi0 = c1()
    psi = dev_psi(psi0, gp.GP_C128)
    o = oracle.Oracle.from_params(w, psi0)
    with gp.Solver.from_workload(psi, w) as s:
        s.step_imag(50)
        o.step_imag(50)
        s.set_g(w["g"] / 2)
        o.set_g(w["g"] / 2)
        s.step_real(40)
        o.step_real(40)
        e, mu = s.energy_mu()
        rms = s.rms()
        torch.cuda.synchronize()
        out = psi.cpu().numpy()
    e_r, mu_r = o.energy_mu()
    assert np.max(np.abs(out - o.psi)) <= 1e-11
    assert abs(mu - mu_r) <= 1e-11 * abs(mu_r) and abs(e - e_r) <= 1e-11 * abs(e_r)
    assert np.max(np.abs(rms - o.rms())) <= 1e-11


def test_raw_sums_match_oracle_on_generic_state():
    prm = dict(nx=33, ny=47, nz=29, dx=0.21, dy=0.17, dz=0.25, nux=1.1, nuy=1.6, nuz=0.9, g=30.0, dt=0.004)
    psi0 = inputs.perturbed_psi(33, 47, 29, 0.21, 0.17, 0.25, 1.0, 1.3, 0.8, seed=5, amp=0.4) * 1.3
    for prec in (gp.GP_C128, gp.GP_C64):
        psi = dev_psi(psi0, prec)
        with gp.Solver.from_workload(psi, prm) as s:
            raw = s.raw_sums()
        want = oracle.Oracle.from_params(prm, psi0.astype(np.complex64).astype(np.complex128)
                                         if prec == gp.GP_C64 else psi0).raw_sums()
        assert np.max(np.abs(raw - want) / np.abs(want)) <= 1e-12


def test_error_paths_nonfinite_and_zero():
    prm = dict(nx=16, ny=12, nz=10, dx=0.3, dy=0.3, dz=0.3, nux=1.0, nuy=1.0, nuz=1.0, g=1.0, dt=0.01)
    psi0 = inputs.gaussian_psi(16, 12, 10, 0.3, 0.3, 0.3, 1, 1, 1)
    psi = dev_psi(psi0, gp.GP_C128)
    with gp.Solver.from_workload(psi, prm) as s:
        psi[3, 4, 5] = complex(float("nan"), 0.0)
        with pytest.raises(gp.GPError) as ei:
            s.norm()
        assert ei.value.code == gp.GP_ERR_NONFINITE
        s.step_imag(1)
        _, _, flags = s.status()
        assert flags & gp.GP_FLAG_NONFINITE
    psi = dev_psi(np.zeros((16, 12, 10)), gp.GP_C128)
    with gp.Solver.from_workload(psi, prm) as s:
        with pytest.raises(gp.GPError) as ei:
            s.energy_mu()
        assert ei.value.code == gp.GP_ERR_ZERO_NORM
        s.step_imag(2)
        _, _, flags = s.status()
        assert flags & gp.GP_FLAG_ZERO_NORM


def test_init_rejects_host_memory_and_dtype_mismatch():
    prm = gp.make_params(8, 8, 8, 0.1, 0.1, 0.1, 1, 1, 1, 1, 0.001, gp.GP_C128)
    host = np.zeros((8, 8, 8), dtype=np.complex128)
    rc, _ = gp.gp_init(prm, host.ctypes.data, 0)
    assert rc == gp.GP_ERR_INVALID


def test_converge_imag_reaches_tolerance():
    w, psi0 = c1()
    psi = dev_psi(psi0, gp.GP_C128)
    with gp.Solver.from_workload(psi, w) as s:
        steps, mu, conv = s.converge_imag(tol=1e-9, check_every=100, max_steps=20000)
    o = run_ref(w, psi0, True, steps)
    assert conv
    assert abs(mu - o.energy_mu()[1]) <= 1e-10 * abs(mu)


@pytest.mark.parametrize("prec", [gp.GP_C64, gp.GP_C128])
def test_autotune_restores_state_caches_and_stays_exact(prec, tmp_path):
    nx, ny, nz = 96, 80, 72
    prm = dict(nx=nx, ny=ny, nz=nz, dx=0.2, dy=0.2, dz=0.2, nux=1.0, nuy=1.4142, nuz=1.7321, g=40.0, dt=0.004)
    psi0 = inputs.perturbed_psi(nx, ny, nz, 0.2, 0.2, 0.2, 1.0, 1.4, 1.7, seed=8, amp=0.1)
    psi = dev_psi(psi0, prec)
    before = psi.cpu().numpy()
    cache = str(tmp_path / "tune.txt")
    with gp.Solver.from_workload(psi, prm) as s:
        m1 = s.autotune("real", steps=2, cache_path=cache)
        assert np.array_equal(psi.cpu().numpy(), before)
        assert s.status()[0] == 0
        m2 = s.autotune("real", steps=2, cache_path=cache)
        assert m1 == m2 == s.get_mapping()
        s.step_real(2)
        torch.cuda.synchronize()
        out = psi.cpu().numpy().astype(np.complex128)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and lines[0].startswith(f"gfx950 {nx} {ny} {nz} {prec} 1 :")
    ref = run_ref(prm, psi0.astype(np.complex64).astype(np.complex128) if prec == gp.GP_C64 else psi0, False, 2).psi
    assert rel_err(out, ref) <= (1e-13 if prec == gp.GP_C128 else 2e-6)
