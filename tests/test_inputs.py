"""CPU: the seeded input generators shared by the oracle and the HIP path.

They hold none of the method's arithmetic; these checks pin what each one promises
(normalisation on the grid, separability, the stated distributions, determinism), so
that a workload means the same thing in the tests, the smoke check and the benchmark.
"""
import math

import numpy as np
import pytest

from paper_1601_04641_amd import inputs


def grid_norm(psi, dx, dy, dz):
    return float(np.sum(np.abs(psi) ** 2)) * dx * dy * dz


def test_axis_is_centred():
    for n in (3, 4, 17, 512):
        a = inputs.axis(n, 0.3)
        assert a.size == n and abs(a[0] + a[-1]) < 1e-12
        assert np.allclose(np.diff(a), 0.3)


@pytest.mark.parametrize("shape,d,nu", [((11, 9, 7), (0.3, 0.25, 0.4), (1.0, 1.4142, 1.7321)),
                                        ((20, 6, 13), (0.2, 0.2, 0.2), (0.0, 2.0, 0.7))])
def test_gaussian_is_normalised_and_separable(shape, d, nu):
    psi = inputs.gaussian_psi(*shape, *d, *nu)
    assert abs(grid_norm(psi, *d) - 1.0) < 1e-13
    f = inputs.gaussian_factors(*shape, *d, *nu)
    for v, h in zip(f, d):
        assert abs(float(np.sum(v * v)) * h - 1.0) < 1e-13
    prod = f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    assert np.max(np.abs(prod - psi)) <= 1e-13 * np.max(np.abs(psi))


def test_gaussian_cube_batch_rows_equal_gaussian_psi():
    prm = np.array([[1.0, 2.0, 0.5, 10.0], [3.0, 0.7, 1.1, 500.0]])
    out = inputs.gaussian_cube_batch(prm, 12, 0.25, dtype=np.complex128)
    for r in range(2):
        want = inputs.gaussian_psi(12, 12, 12, 0.25, 0.25, 0.25, *prm[r, :3])
        assert np.max(np.abs(out[r] - want)) <= 1e-13 * np.max(np.abs(want))


def test_perturbed_psi_is_normalised_seeded_and_complex():
    a = inputs.perturbed_psi(9, 8, 7, 0.2, 0.3, 0.25, 1.0, 1.3, 0.8, seed=4, amp=0.2)
    b = inputs.perturbed_psi(9, 8, 7, 0.2, 0.3, 0.25, 1.0, 1.3, 0.8, seed=4, amp=0.2)
    c = inputs.perturbed_psi(9, 8, 7, 0.2, 0.3, 0.25, 1.0, 1.3, 0.8, seed=5, amp=0.2)
    assert abs(grid_norm(a, 0.2, 0.3, 0.25) - 1.0) < 1e-13
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.max(np.abs(a.imag)) > 0.01 * np.max(np.abs(a))


def test_batch_draws_follow_their_laws():
    b = inputs.draw_batch(0, 400)
    assert b == inputs.draw_batch(0, 400)
    dims = set(range(32, 97, 8))
    for w in b:
        assert {w["nx"], w["ny"], w["nz"]} <= dims
        assert all(0.5 <= w[k] <= 4.0 for k in ("nux", "nuy", "nuz"))
        assert 1.0 <= w["g"] <= 1000.0
        assert abs(w["dt"] - 0.1 * w["dx"] ** 2) < 1e-15
    # log-uniform g: about half the draws below sqrt(1000)
    below = sum(w["g"] < math.sqrt(1000.0) for w in b) / len(b)
    assert 0.4 < below < 0.6
    p = inputs.draw_nn_params(2, 512)
    assert p.shape == (512, 4) and np.all((p[:, :3] >= 0.5) & (p[:, :3] <= 4.0))
    assert np.all((p[:, 3] >= 1.0) & (p[:, 3] <= 1000.0))
    assert not np.any(np.all(np.isin(p, inputs.draw_nn_params(1, 4096)), axis=1))


def test_paper_scale_workloads():
    for name, n in (("paper_imag_1920x1600x1280", (1920, 1600, 1280)), ("paper_real_1600x1280x960", (1600, 1280, 960))):
        w = inputs.WORKLOADS[name]
        assert (w["nx"], w["ny"], w["nz"]) == n and w["steps"] == 1000
        assert w["dx"] == w["dy"] == w["dz"]
    wi, wr = inputs.WORKLOADS["paper_imag_1920x1600x1280"], inputs.WORKLOADS["paper_real_1600x1280x960"]
    assert abs(wi["dt"] - 0.1 * wi["dx"] ** 2) < 1e-18 and abs(wr["dt"] - 0.01 * wr["dx"] ** 2) < 1e-18
    # the quench workload's box along x
    assert abs(wi["nx"] * wi["dx"] - 512 * 0.05) < 1e-9
