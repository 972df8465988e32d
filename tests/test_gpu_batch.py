"""GPU tests of the batched form: uneven instances advanced by the same launches.

Each instance is checked against the CPU FP64 oracle and against a single-grid context
given the same line mapping (real time: bitwise identical; imaginary time differs only in
the grouping of the FP64 norm sums).
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


def instances():
    """Uneven grids, traps, g and dt (dims include non-multiples of 8)."""
    out = []
    shapes = [(32, 40, 48), (96, 80, 64), (45, 33, 70), (64, 64, 32), (17, 90, 21), (72, 48, 96)]
    rng = np.random.default_rng(3)
    for k, (nx, ny, nz) in enumerate(shapes):
        d = 0.2 if k % 2 == 0 else 0.17
        out.append(dict(nx=nx, ny=ny, nz=nz, dx=d, dy=d * 1.1, dz=d * 0.9, nux=float(rng.uniform(0.5, 4)),
                        nuy=float(rng.uniform(0.5, 4)), nuz=float(rng.uniform(0.5, 4)),
                        g=float(np.exp(rng.uniform(0, np.log(1000)))), dt=0.1 * d * d))
    return out


def pack(ws, prec, seed=0):
    """Seeded generic initial states packed back to back; returns (host states, offsets)."""
    states, offs, off = [], [], 0
    for i, w in enumerate(ws):
        s = inputs.perturbed_psi(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"],
                                 seed=seed + i, amp=0.2)
        if prec == gp.GP_C64:
            s = s.astype(np.complex64).astype(np.complex128)
        states.append(s)
        offs.append(off)
        off += s.size
    return states, np.array(offs, dtype=np.int64), off


def to_dev(states, total, prec):
    dt = torch.complex64 if prec == gp.GP_C64 else torch.complex128
    flat = np.concatenate([s.reshape(-1) for s in states])
    assert flat.size == total
    return torch.from_numpy(flat).to(device="cuda", dtype=dt)


def unpack(psi, ws, offs):
    h = psi.cpu().numpy().astype(np.complex128)
    return [h[o:o + w["nx"] * w["ny"] * w["nz"]].reshape(w["nx"], w["ny"], w["nz"]) for w, o in zip(ws, offs)]


def c64_tolerance(w, s0, ref, imag, steps=20):
    """complex64 tolerance from the problem's own conditioning: the oracle is rerun from
    the initial state perturbed by FP32-sized relative noise (u = 6e-8), which measures the
    amplification A of an error committed at the start (sens = A u).  The FP32 path commits
    an error of about 2u per step (the rounding of psi after each sweep, with the
    coefficient tables rounded once), each amplified by at most A over the remaining steps:
    20 steps x 2u x A = 40 sens bounds the total (floor 5e-6 for well-conditioned cases).
    Strongly nonlinear real-time cases (g ~ 10^3) amplify input noise ~70x in 20 steps."""
    rng = np.random.default_rng(12345)
    o = oracle.Oracle.from_params(w, s0 * (1 + 6e-8 * rng.standard_normal(s0.shape)))
    (o.step_imag if imag else o.step_real)(steps)
    sens = float(np.max(np.abs(o.psi - ref)) / np.max(np.abs(ref)))
    return max(5e-6, 40 * sens)


@pytest.mark.parametrize("prec", [gp.GP_C64, gp.GP_C128])
@pytest.mark.parametrize("imag", [True, False])
def test_batch_matches_oracle_per_instance(prec, imag):
    ws = instances()
    states, offs, total = pack(ws, prec)
    psi = to_dev(states, total, prec)
    say(f"case: batch of {len(ws)} prec {prec} imag {imag}")
    with gp.Batch(psi, ws, offs) as b:
        (b.step_imag if imag else b.step_real)(20)
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
        raw = b.raw_sums()
    for i, (w, s0, out) in enumerate(zip(ws, states, outs)):
        o = oracle.Oracle.from_params(w, s0)
        (o.step_imag if imag else o.step_real)(20)
        err = float(np.max(np.abs(out - o.psi)) / np.max(np.abs(o.psi)))
        tol = 1e-12 if prec == gp.GP_C128 else c64_tolerance(w, s0, o.psi, imag)
        say(f"  instance {i} {w['nx']}x{w['ny']}x{w['nz']} g {w['g']:.1f}: rel err {err:.2e} (tol {tol:.1e})")
        assert err <= tol
        want = oracle.Oracle.from_params(w, out).raw_sums()
        assert np.max(np.abs(raw[i] - want) / np.abs(want)) <= 1e-12


@pytest.mark.parametrize("imag", [True, False])
def test_batch_long_segments_with_idle_wavefronts(imag):
    """32 points per thread, one segment per wavefront, in complex64 (the line sweeps'
    early-load scheme): the blocks hold 3 wavefronts for the 96-point lines, so on the
    smaller instances (17-64 points along x, 33-64 along y) one or two wavefronts of each
    block lie past the line's end.  Every instance against the oracle."""
    ws = instances()
    prec = gp.GP_C64
    states, offs, total = pack(ws, prec, seed=40)
    psi = to_dev(states, total, prec)
    say(f"case: batch of {len(ws)} c64 mapping x (32, 1) y (32, 1) imag {imag}")
    with gp.Batch(psi, ws, offs) as b:
        mz = b.get_mapping()[4]
        b.set_mapping(32, 1, 32, 1, mz)
        assert b.get_mapping()[:4] == [32, 1, 32, 1]
        (b.step_imag if imag else b.step_real)(20)
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
    for i, (w, s0, out) in enumerate(zip(ws, states, outs)):
        o = oracle.Oracle.from_params(w, s0)
        (o.step_imag if imag else o.step_real)(20)
        err = float(np.max(np.abs(out - o.psi)) / np.max(np.abs(o.psi)))
        tol = c64_tolerance(w, s0, o.psi, imag)
        say(f"  instance {i} {w['nx']}x{w['ny']}x{w['nz']}: rel err {err:.2e} (tol {tol:.1e})")
        assert err <= tol


def test_batch_real_time_bitwise_equals_single_grid_with_same_mapping():
    ws = instances()
    prec = gp.GP_C64
    states, offs, total = pack(ws, prec, seed=10)
    psi = to_dev(states, total, prec)
    with gp.Batch(psi, ws, offs) as b:
        assert b.get_yz_fusion() == (False, 0)  # default: the separate (single-grid) sweeps
        mx, swx, my, swy, mz = b.get_mapping()
        b.step_real(7)
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
    for w, s0, out in zip(ws, states, outs):
        seg = 2
        while seg < 64 and seg * mz < w["nz"]:
            seg *= 2
        single = to_dev([s0], s0.size, prec).reshape(w["nx"], w["ny"], w["nz"])
        with gp.Solver.from_workload(single, w) as s:
            s.set_mapping(mx, swx, my, swy, seg, mz)
            s.step_real(7)
            torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy().astype(np.complex128), out)


def long_correction_instances():
    """Two instances with dt/dx^2 ~ 2-10 (c'_inf close to 1: Sherman-Morrison corrections
    of tens of points, longer than a segment of 8) and one with a small dt (correction
    inside segment 0), so one launch runs both branches of the in-kernel correction."""
    big = dict(dx=0.1, dy=0.15, dz=0.05, nux=1.0, nuy=1.2, nuz=0.8, g=5.0, dt=0.1)
    return [dict(big, nx=70, ny=45, nz=33), dict(big, nx=40, ny=66, nz=24, g=40.0),
            dict(nx=48, ny=40, nz=36, dx=0.2, dy=0.22, dz=0.18, nux=1.3, nuy=0.9, nuz=2.0, g=20.0, dt=0.0001)]


@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
@pytest.mark.parametrize("imag", [True, False])
def test_batch_long_head_correction_matches_oracle(prec, imag):
    """Batched x/y sweeps with 8 points per thread apply corrections longer than a segment
    in-kernel (u_0 passed through LDS): every instance against the oracle, and in real time
    bitwise against single-grid contexts with the same mapping (whose separate correction
    pass performs the same operations)."""
    ws = long_correction_instances()
    states, offs, total = pack(ws, prec, seed=60)
    psi = to_dev(states, total, prec)
    say(f"case: batch long head correction prec {prec} imag {imag}")
    with gp.Batch(psi, ws, offs) as b:
        mz = b.get_mapping()[4]
        b.set_mapping(8, 1, 8, 1, mz)
        (b.step_imag if imag else b.step_real)(2)
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
    for i, (w, s0, out) in enumerate(zip(ws, states, outs)):
        o = oracle.Oracle.from_params(w, s0)
        (o.step_imag if imag else o.step_real)(2)
        err = float(np.max(np.abs(out - o.psi)) / np.max(np.abs(o.psi)))
        say(f"  instance {i} {w['nx']}x{w['ny']}x{w['nz']} dt {w['dt']}: rel err {err:.2e}")
        assert err <= (1e-12 if prec == gp.GP_C128 else 5e-6)
        if not imag:
            seg = 2
            while seg < 64 and seg * mz < w["nz"]:
                seg *= 2
            single = to_dev([s0], s0.size, prec).reshape(w["nx"], w["ny"], w["nz"])
            with gp.Solver.from_workload(single, w) as s:
                s.set_mapping(8, 1, 8, 1, seg, mz)
                s.step_real(2)
                torch.cuda.synchronize()
            assert np.array_equal(single.cpu().numpy().astype(np.complex128), out)


def test_batch_masking_leaves_inactive_instances_untouched():
    ws = instances()
    prec = gp.GP_C64
    states, offs, total = pack(ws, prec, seed=20)
    psi = to_dev(states, total, prec)
    active = np.array([1, 0, 1, 0, 1, 1], dtype=np.uint8)
    with gp.Batch(psi, ws, offs) as b:
        b.step_imag(5, active=active)
        b.step_real(3)                      # stays masked: same instances untouched
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
        steps, _, flags = b.status()
    for i in range(len(ws)):
        if active[i]:
            assert not np.array_equal(outs[i], states[i])
            assert steps[i] == 8
        else:
            assert np.array_equal(outs[i], states[i])
            assert steps[i] == 0
    assert np.all(flags == 0)


def test_batch_converges_each_instance():
    ws = [dict(w, g=min(w["g"], 50.0)) for w in instances()[:4]]
    prec = gp.GP_C128
    states = [inputs.gaussian_psi(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"])
              for w in ws]
    offs = np.cumsum([0] + [s.size for s in states[:-1]]).astype(np.int64)
    psi = to_dev(states, sum(s.size for s in states), prec)
    with gp.Batch(psi, ws, offs) as b:
        steps, mu, conv = b.converge_imag(tol=1e-8, check_every=50, max_steps=20000)
    say(f"steps {steps}, mu {mu}")
    assert np.all(conv)
    for w, s0, n, m in zip(ws, states, steps, mu):
        o = oracle.Oracle.from_params(w, s0)
        o.step_imag(int(n))
        assert abs(o.energy_mu()[1] - m) <= 1e-10 * abs(m)


def test_batch_autotune_restores_state():
    ws = instances()
    prec = gp.GP_C64
    states, offs, total = pack(ws, prec, seed=30)
    psi = to_dev(states, total, prec)
    before = psi.cpu().numpy()
    with gp.Batch(psi, ws, offs) as b:
        m = b.autotune("imag", steps=2)
        assert m == b.get_mapping()
        assert np.array_equal(psi.cpu().numpy(), before)
        assert np.all(b.status()[0] == 0)
        b.step_imag(3)
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
    for w, s0, out in zip(ws, states, outs):
        o = oracle.Oracle.from_params(w, s0)
        o.step_imag(3)
        assert float(np.max(np.abs(out - o.psi)) / np.max(np.abs(o.psi))) <= 5e-6


def test_batch_rejects_bad_arguments():
    ws = instances()[:2]
    states, offs, total = pack(ws, gp.GP_C64)
    psi = to_dev(states, total, gp.GP_C64)
    bad = [dict(ws[0], nx=2), ws[1]]
    with pytest.raises(gp.GPError):
        gp.Batch(psi, bad, offs)
    with gp.Batch(psi, ws, offs) as b:
        with pytest.raises(gp.GPError):
            b.set_mapping(mx=5)
        with pytest.raises(gp.GPError):
            b.set_mapping(mz=7)


@pytest.mark.parametrize("prec", [gp.GP_C128, gp.GP_C64])
def test_batch_residual_matches_oracle(prec):
    from oracle.residual import residual
    ws = instances()[:4]
    states, offs, total = pack(ws, prec, seed=40)
    psi = to_dev(states, total, prec)
    with gp.Batch(psi, ws, offs) as b:
        r, mu = b.residual()
        _, mu_obs = b.energy_mu()
    tol = 1e-10 if prec == gp.GP_C128 else 1e-5
    for i, (w, s0) in enumerate(zip(ws, states)):
        rr, mm = residual(s0, w)
        say(f"  instance {i}: res {r[i]:.6e} vs {rr:.6e}, mu {mu[i]:.8f} vs {mm:.8f}")
        assert abs(r[i] - rr) <= tol * rr and abs(mu[i] - mm) <= tol * abs(mm)
        assert abs(mu[i] - mu_obs[i]) <= 1e-12 * abs(mu_obs[i]) + (0 if prec == gp.GP_C128 else 1e-7 * abs(mm))


def test_batch_residual_small_at_converged_ground_state():
    ws = [dict(w, g=min(w["g"], 50.0)) for w in instances()[:3]]
    states = [inputs.gaussian_psi(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"])
              for w in ws]
    offs = np.cumsum([0] + [s.size for s in states[:-1]]).astype(np.int64)
    psi = to_dev(states, sum(s.size for s in states), gp.GP_C128)
    with gp.Batch(psi, ws, offs) as b:
        r0, mu0 = b.residual()
        b.converge_imag(tol=1e-10, check_every=50, max_steps=40000)
        r1, mu1 = b.residual()
    say(f"residual / mu: start {r0 / mu0}, converged {r1 / mu1}")
    # the imaginary-time fixed point differs from the discrete ground state by O(dt)
    assert np.all(r1 < 0.05 * r0) and np.all(r1 / mu1 < 5e-3)


@pytest.mark.parametrize("prec", [gp.GP_C64, gp.GP_C128])
@pytest.mark.parametrize("imag", [True, False])
def test_fused_yz_sweeps_agree_with_separate_sweeps(prec, imag):
    """The fused y+z plane kernel computes the same solves in a different rounding order."""
    ws = instances()
    states, offs, total = pack(ws, prec, seed=50)
    outs = []
    for fuse in (True, False):
        psi = to_dev(states, total, prec)
        with gp.Batch(psi, ws, offs) as b:
            b.set_yz_fusion(fuse)
            on, nf = b.get_yz_fusion()
            assert on == fuse and nf == (len(ws) if fuse else 0)
            (b.step_imag if imag else b.step_real)(12)
            torch.cuda.synchronize()
            outs.append(unpack(psi, ws, offs))
    for i, (w, s0, a, c) in enumerate(zip(ws, states, *outs)):
        err = float(np.max(np.abs(a - c)) / np.max(np.abs(c)))
        if prec == gp.GP_C128:
            tol = 1e-13
        else:  # two FP32 rounding orders: bounded by the problem's conditioning, as against the oracle
            o = oracle.Oracle.from_params(w, s0)
            (o.step_imag if imag else o.step_real)(12)
            tol = c64_tolerance(w, s0, o.psi, imag, steps=12)
        say(f"  instance {i}: fused vs separate {err:.2e} (tol {tol:.1e})")
        assert err <= tol


def test_mixed_fused_and_separate_instances_match_oracle():
    """An instance whose x-plane does not fit in LDS (120 x 101 complex128 = 194 KB) takes the separate y and z
    sweeps while the others are fused, in the same launches; both kinds match the oracle,
    and the per-instance norms (renormalisation) come from the right partial sums."""
    ws = instances()[:3] + [dict(instances()[1], nx=12, ny=120, nz=100, g=30.0)]
    prec = gp.GP_C128
    states, offs, total = pack(ws, prec, seed=60)
    psi = to_dev(states, total, prec)
    with gp.Batch(psi, ws, offs) as b:
        b.set_yz_fusion(True)
        assert b.get_yz_fusion() == (True, 3)
        b.step_imag(6)
        b.step_real(4)
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
        norms = b.norm()
    for i, (w, s0, out) in enumerate(zip(ws, states, outs)):
        o = oracle.Oracle.from_params(w, s0)
        o.step_imag(6)
        o.step_real(4)
        err = float(np.max(np.abs(out - o.psi)) / np.max(np.abs(o.psi)))
        say(f"  instance {i} {w['ny']}x{w['nz']}: rel err {err:.2e}, norm {norms[i]:.15f}")
        assert err <= 1e-12
        assert abs(norms[i] - o.norm()) <= 1e-12


@pytest.mark.parametrize("imag", [True, False])
def test_strang_batch_matches_oracle(imag):
    ws = instances()[:3]
    prec = gp.GP_C128
    states, offs, total = pack(ws, prec, seed=70)
    psi = to_dev(states, total, prec)
    with gp.Batch(psi, ws, offs, split=gp.GP_SPLIT_STRANG) as b:
        b.set_yz_fusion(True)
        assert b.get_yz_fusion()[1] == 0  # the fused kernel has no trailing half step
        (b.step_imag if imag else b.step_real)(9)
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
    for w, s0, out in zip(ws, states, outs):
        o = oracle.Oracle.from_params(w, s0, split=1)
        (o.step_imag if imag else o.step_real)(9)
        assert float(np.max(np.abs(out - o.psi)) / np.max(np.abs(o.psi))) <= 1e-12


@pytest.mark.parametrize("fuse", [False, True])
@pytest.mark.parametrize("imag", [True, False])
def test_batch_odd_sized_complex64_instance_first(fuse, imag):
    """An odd-sized complex64 instance first puts the next instance at an odd element
    offset (8- but not 16-byte aligned): the 16-byte plane and line copies must fall back
    to 8-byte ones there."""
    ws = instances()
    ws = [dict(ws[4], nx=17, ny=33, nz=21), dict(ws[0], nx=24, ny=20, nz=30), dict(ws[2], nx=14, ny=11, nz=9),
          dict(ws[1], nx=32, ny=24, nz=40)]
    states, offs, total = pack(ws, gp.GP_C64, seed=50)
    assert offs[1] % 2 == 1 and offs[3] % 2 == 1
    psi = to_dev(states, total, gp.GP_C64)
    say(f"case: odd offsets {offs.tolist()} fuse {fuse} imag {imag}")
    with gp.Batch(psi, ws, offs) as b:
        b.set_yz_fusion(fuse)
        (b.step_imag if imag else b.step_real)(5)
        torch.cuda.synchronize()
        outs = unpack(psi, ws, offs)
    for i, (w, s0, out) in enumerate(zip(ws, states, outs)):
        o = oracle.Oracle.from_params(w, s0)
        (o.step_imag if imag else o.step_real)(5)
        err = float(np.max(np.abs(out - o.psi)) / np.max(np.abs(o.psi)))
        tol = c64_tolerance(w, s0, o.psi, imag, steps=5)
        say(f"  instance {i} offset {offs[i]}: rel err {err:.2e} (tol {tol:.1e})")
        assert err <= tol


def test_batch_autotune_cache(tmp_path):
    ws = instances()
    states, offs, total = pack(ws, gp.GP_C64, seed=40)
    psi = to_dev(states, total, gp.GP_C64)
    cache = str(tmp_path / "btune.txt")
    with gp.Batch(psi, ws, offs) as b:
        m1 = b.autotune("imag", steps=1, cache_path=cache)
        f1 = b.get_yz_fusion()
        b.set_mapping(8, 1, 8, 1, 4)
        b.set_yz_fusion(not f1[0])
        m2 = b.autotune("imag", steps=1, cache_path=cache)   # a hit: no timing, stored choice
        assert m1 == m2 == b.get_mapping() and b.get_yz_fusion() == f1
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and lines[0].startswith("gfx950-batch ")
    with gp.Batch(psi, ws[:-1], offs[:-1]) as b:   # another batch: a miss, a second line
        b.autotune("imag", steps=1, cache_path=cache)
    assert len(open(cache).read().strip().splitlines()) == 2
