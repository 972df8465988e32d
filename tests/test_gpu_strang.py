"""GPU: the Strang splitting as a studied variant of the method's step (half potential
steps around the three Crank-Nicolson sweeps), complex128 on the 48x40x32 grid.

* Time-step order in real time, from a smooth start: the state error at fixed time falls
  like dt (Lie) and dt^2 (Strang); each GPU run also matches the FP64 oracle at the same dt.
* Imaginary-time fixed points: with g = 0 the Strang step is N_h C N_h and the Lie step
  C N (N = exp(-dt V), N_h = exp(-dt V / 2), C the sweeps), so N_h maps the Lie fixed
  point onto the Strang one with the same eigenvalue: psi_S = N_h psi_L / |N_h psi_L| and
  equal renormalisation estimates mu_est, an exact identity of the discrete steps.
"""
import math
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


def c1():
    return dict(inputs.WORKLOADS["imag_48x40x32"])


@pytest.mark.parametrize("split,order", [(gp.GP_SPLIT_LIE, 1.0), (gp.GP_SPLIT_STRANG, 2.0)])
def test_real_time_dt_order(split, order):
    w = c1()
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    # a smooth start (the Gaussian of a tighter trap, which then breathes): the splitting
    # error dominates the difference under dt halving (a start with grid-scale noise is
    # dominated by the sweeps' own second-order error instead, for both splittings)
    psi0 = inputs.gaussian_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], 2.0, 2.6, 3.2)
    t = 0.4
    res = []
    for k, dt in enumerate((0.008, 0.004, 0.002)):
        prm = dict(w, dt=dt)
        psi = torch.from_numpy(psi0).to("cuda")
        with gp.Solver.from_workload(psi, prm, split=split) as s:
            s.step_real(int(round(t / dt)))
            torch.cuda.synchronize()
            out = psi.cpu().numpy()
        res.append(out)
        if k == 0:   # parity with the oracle at the coarsest step
            o = oracle.Oracle.from_params(prm, psi0, split=split)
            o.step_real(int(round(t / dt)))
            err = float(np.max(np.abs(out - o.psi)) / np.max(np.abs(o.psi)))
            say(f"case: dt order split {split}: vs oracle {err:.2e}")
            assert err <= 1e-12
    e1 = float(np.max(np.abs(res[0] - res[1])))
    e2 = float(np.max(np.abs(res[1] - res[2])))
    p = math.log2(e1 / e2)
    say(f"  successive differences {e1:.3e}, {e2:.3e}: observed order {p:.3f} (expected {order})")
    assert abs(p - order) < 0.2


def test_strang_fixed_point_is_the_half_potential_image_of_lie():
    w = dict(c1(), g=0.0)
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    dt = w["dt"]
    psi0 = inputs.gaussian_psi(nx, ny, nz, w["dx"], w["dy"], w["dz"], w["nux"], w["nuy"], w["nuz"])
    out, mus = {}, {}
    for split in (gp.GP_SPLIT_LIE, gp.GP_SPLIT_STRANG):
        psi = torch.from_numpy(psi0).to("cuda")
        with gp.Solver.from_workload(psi, w, split=split) as s:
            steps, mu, conv = s.converge_imag(tol=1e-13, check_every=100, max_steps=200000)
            assert conv
            s.step_imag(2000)   # well past the stopping point
            mus[split] = s.status()[1]
            torch.cuda.synchronize()
            out[split] = psi.cpu().numpy()
    vx, vy, vz = (0.5 * nu ** 2 * inputs.axis(n, d) ** 2
                  for nu, n, d in zip((w["nux"], w["nuy"], w["nuz"]), (nx, ny, nz), (w["dx"], w["dy"], w["dz"])))
    V = vx[:, None, None] + vy[None, :, None] + vz[None, None, :]
    want = np.exp(-0.5 * dt * V) * out[gp.GP_SPLIT_LIE]
    dV = w["dx"] * w["dy"] * w["dz"]
    want /= math.sqrt(float(np.sum(np.abs(want) ** 2)) * dV)
    err = float(np.max(np.abs(out[gp.GP_SPLIT_STRANG] - want)) / np.max(np.abs(want)))
    say(f"case: Strang vs half-potential image of the Lie fixed point: {err:.2e}; "
        f"mu_est {mus[gp.GP_SPLIT_LIE]!r} vs {mus[gp.GP_SPLIT_STRANG]!r}")
    assert err <= 1e-10
    assert abs(mus[gp.GP_SPLIT_LIE] - mus[gp.GP_SPLIT_STRANG]) <= 1e-11 * mus[gp.GP_SPLIT_LIE]
