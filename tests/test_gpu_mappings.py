"""GPU parity of every line mapping a timed path can run, against the CPU FP64 oracle.

The benchmark and the paper-scale runs use the autotuner's mappings (its committed cache,
results/autotune_gfx950.txt), and the autotuner itself may pick any mapping the kernels
cover.  So:

* every z mapping (threads per line x points per thread) the autotuner tries, on thin
  grids whose z lines have the lengths of the timed grids (448, 384, 960, 1280, 1600);
* every x and y mapping (points per thread x segments per wavefront) it tries, on thin
  grids whose x or y lines have those lengths (384 ... 1920);
* the quench grid (512x480x448) in exactly the cached mapping the benchmark times, both
  precisions, real and imaginary time, every point against the oracle;

each for both step kinds.  A mapping the kernels do not cover is rejected by
gp_set_mapping (the check the autotuner uses) and skipped here as it is there.
Tolerances as in the other parity tests: complex128 1e-13 relative to max|psi|
(imaginary time at 1.1e8 points 1e-12, the oracle's own sequential norm sums), complex64
2e-6.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1601_04641_amd import gp, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "results", "autotune_gfx950.txt")

# the autotuner's candidate lists (gp_autotune)
LINE_M = (8, 10, 12, 16, 30, 32)
LINE_SW = (1, 2, 4, 8)
Z_SEG = (2, 4, 8, 16, 32, 64)
Z_M = (2, 4, 6, 7, 8, 12, 14, 15, 16, 20, 24, 32)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gp.load()
    yield


def cached_mapping(grid, prec, mode):
    """The last cache entry for (grid, precision, step kind), as gp_autotune reads it."""
    found = None
    for line in open(CACHE):
        head, _, tail = line.partition(":")
        f = head.split()
        if len(f) == 6 and f[0] == "gfx950" and tuple(int(v) for v in f[1:4]) == tuple(grid) \
                and int(f[4]) == prec and int(f[5]) == mode:
            found = tuple(int(v) for v in tail.split())
    return found


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def thin_case(shape, seed):
    nx, ny, nz = shape
    prm = dict(nx=nx, ny=ny, nz=nz, dx=0.03, dy=0.031, dz=0.029, nux=1.2, nuy=1.4, nuz=1.1, g=30.0, dt=4e-4)
    psi0 = inputs.perturbed_psi(nx, ny, nz, prm["dx"], prm["dy"], prm["dz"], 0.02, 0.025, 0.015, seed=seed, amp=0.2)
    return prm, psi0


def run_mappings(prm, psi0, prec, candidates):
    """Every candidate mapping the library accepts, both step kinds, vs the oracle."""
    refs = {}
    for imag in (True, False):
        o = oracle.Oracle.from_params(prm, psi0.astype(np.complex64).astype(np.complex128)
                                      if prec == gp.GP_C64 else psi0)
        (o.step_imag if imag else o.step_real)(2)
        refs[imag] = o.psi.copy()
        o.close()
    dt = torch.complex64 if prec == gp.GP_C64 else torch.complex128
    tol = 2e-6 if prec == gp.GP_C64 else 1e-13
    ran = 0
    for cand in candidates:
        for imag in (True, False):
            psi = torch.from_numpy(np.ascontiguousarray(psi0)).to(device="cuda", dtype=dt)
            with gp.Solver.from_workload(psi, prm) as s:
                try:
                    s.set_mapping(*cand)
                except gp.GPError as e:
                    assert e.code == gp.GP_ERR_INVALID
                    break   # not covered: the autotuner skips it too
                (s.step_imag if imag else s.step_real)(2)
                torch.cuda.synchronize()
                got = s.get_mapping()
                out = psi.cpu().numpy().astype(np.complex128)
            err = rel_err(out, refs[imag])
            say(f"  mapping {got} imag {imag}: rel err {err:.2e}")
            assert err <= tol, (got, imag, err)
            ran += 1
    return ran


Z_LENGTHS = [448, 384, 960, 1280, 1600]


@pytest.mark.parametrize("nz", Z_LENGTHS)
@pytest.mark.parametrize("prec", [gp.GP_C64, gp.GP_C128])
def test_every_z_mapping(nz, prec):
    prm, psi0 = thin_case((4, 3, nz), seed=nz)
    # the default mapping, then the autotuner's candidates (it skips a mapping whose last
    # segment would be empty; for some lengths that leaves only the default)
    cands = [(0, 0, 0, 0, 0, 0)] + [(0, 0, 0, 0, seg, m) for seg in Z_SEG for m in Z_M
                                    if seg * m >= nz and seg * m - nz < m]
    say(f"case: z mappings nz {nz} prec {prec}: {len(cands)} candidates")
    try:
        ran = run_mappings(prm, psi0, prec, cands)
    except gp.GPError as e:   # the grid itself has no mapping (complex128 z lines this long)
        assert prec == gp.GP_C128 and e.code == gp.GP_ERR_UNSUPPORTED
        pytest.skip(f"complex128 z lines of {nz} points are not supported")
    say(f"  {ran} runs")
    assert ran > 0


LINE_LENGTHS = [384, 448, 480, 512, 960, 1280, 1600, 1920]


@pytest.mark.parametrize("n", LINE_LENGTHS)
@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("prec", [gp.GP_C64, gp.GP_C128])
def test_every_line_mapping(n, axis, prec):
    shape = (n, 3, 4) if axis == 0 else (4, n, 3)
    prm, psi0 = thin_case(shape, seed=n + axis)
    cands = [((m, sw, 0, 0) if axis == 0 else (0, 0, m, sw)) + (0, 0) for m in LINE_M for sw in LINE_SW]
    say(f"case: {'xy'[axis]} mappings n {n} prec {prec}")
    try:
        ran = run_mappings(prm, psi0, prec, cands)
    except gp.GPError as e:
        assert prec == gp.GP_C128 and e.code == gp.GP_ERR_UNSUPPORTED
        pytest.skip(f"complex128 lines of {n} points are not supported")
    say(f"  {ran} runs")
    assert ran > 0


BIG = (512, 480, 448)


@pytest.mark.parametrize("prec", [gp.GP_C64, gp.GP_C128])
@pytest.mark.parametrize("imag", [False, True])
def test_quench_grid_in_benchmark_mapping(prec, imag):
    """The benchmark's timed configuration: the quench grid in the cached real-time mapping
    (the one bench.py applies), 2 steps from a seeded state, every point vs the oracle."""
    mp = cached_mapping(BIG, prec, 1)
    assert mp is not None, "the benchmark's mapping is missing from the autotuner cache"
    w = inputs.WORKLOADS["quench_512x480x448"]
    prm = dict(w)
    if imag:
        prm["dt"] = w["dt_imag"]
    nx, ny, nz = BIG
    say(f"case: quench grid prec {prec} imag {imag} mapping {mp}")
    psi0 = inputs.perturbed_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], 2.0, 2.5, 3.0, seed=9, amp=0.1)
    if prec == gp.GP_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    dt = torch.complex64 if prec == gp.GP_C64 else torch.complex128
    psi = torch.from_numpy(psi0).to(device="cuda", dtype=dt)
    with gp.Solver.from_workload(psi, prm) as s:
        s.set_mapping(*mp)
        assert tuple(s.get_mapping()) == mp
        (s.step_imag if imag else s.step_real)(2)
        torch.cuda.synchronize()
        out = psi.cpu().numpy().astype(np.complex128)
    del psi
    torch.cuda.empty_cache()
    t0 = time.time()
    o = oracle.Oracle.from_params(prm, psi0)
    (o.step_imag if imag else o.step_real)(2)
    say(f"  oracle {time.time() - t0:.1f}s")
    err = rel_err(out, o.psi)
    o.close()
    tol = (1e-12 if imag else 1e-13) if prec == gp.GP_C128 else 2e-6
    say(f"  rel err {err:.2e} (tol {tol:.0e})")
    assert err <= tol
