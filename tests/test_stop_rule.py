"""Host: the stopping rule of the imaginary-time convergence loops (gp_stop_rule_eval, the
same code gp_converge_imag and gp_batch_converge_imag run), on sequences whose limits are
known exactly: m_n = mu (1 + e_n) with e_n a sum of decaying modes, as mu(t) approaches
the ground state's value in imaginary time (each excited component decays like
exp(-(mu_k - mu_0) t), so its share of the checked value shrinks by a fixed ratio per check).
The rule must stop within tol of the limit, and not much later than needed."""
import ctypes

import numpy as np
import pytest

from paper_1601_04641_amd import gp

MU = 3.0
TOL = 1e-7


@pytest.fixture(scope="module", autouse=True)
def _lib():
    try:
        gp.load()
    except (RuntimeError, OSError) as e:
        pytest.skip(f"library not built: {e}")


def stop(e, tol=TOL):
    s = gp.stop_rule_eval(MU * (1.0 + np.asarray(e)), tol)
    return s


@pytest.mark.parametrize("q", [0.2, 0.5, 0.8, 0.9])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_single_mode(q, sign):
    k = np.arange(400)
    e = sign * 1e-3 * q ** k
    s = stop(e)
    assert s >= 0
    assert abs(e[s]) <= TOL
    # stops within two checks of the error first reaching tol / 2
    first = int(np.argmax(np.abs(e) <= 0.5 * TOL))
    assert s <= first + 2, (s, first)


def test_turning_point_is_not_a_limit():
    # a fast mode from above and a slower one from below: mu(t) overshoots the limit and
    # turns at about -1.35 tol, where successive changes are small; the earlier check
    # (geometric extrapolation from one pair of ratios) stopped right there
    k = np.arange(80)
    e = 1e-4 * 0.4 ** k - 2e-6 * 0.75 ** k
    s = stop(e)
    assert s >= 0
    assert abs(e[s]) <= TOL, (s, e[s])
    assert abs(e[s]) < 0.5 * np.max(np.abs(e[6:12]))


def test_two_mode_mixtures():
    """Seeded mixtures of a fast and a slower mode (either sign, slower amplitude 1e-4 to
    0.3 of the faster, ratios up to 0.85 per check)."""
    rng = np.random.default_rng(12345)
    k = np.arange(200)
    over, worst = 0, 0.0
    n = 3000
    for _ in range(n):
        a = 10 ** rng.uniform(-6, -2) * rng.choice([-1.0, 1.0])
        qa = rng.uniform(0.05, 0.8)
        b = abs(a) * 10 ** rng.uniform(-4, -0.5) * rng.choice([-1.0, 1.0])
        qb = rng.uniform(qa, 0.85)
        e = a * qa ** k + b * qb ** k
        s = stop(e)
        assert s >= 0
        worst = max(worst, abs(e[s]))
        over += abs(e[s]) > TOL
    assert worst <= 1.3 * TOL, worst
    assert over <= 0.01 * n, over


def test_rounding_floor():
    # geometric approach that ends in FP64 noise: the three-small-changes branch ends it
    rng = np.random.default_rng(7)
    k = np.arange(300)
    e = 1e-3 * 0.5 ** k + 2e-16 * rng.standard_normal(k.size)
    s = stop(e, tol=1e-13)
    assert s >= 0
    assert abs(e[s]) <= 1e-13


def test_alternating_approach():
    k = np.arange(200)
    e = 1e-3 * (-0.5) ** k
    s = stop(e)
    assert s >= 0 and abs(e[s]) <= TOL
    # three successive changes of at most tol/10: |d| = 1.5 |e_{n-1}| <= tol / 10
    first = int(np.argmax(1.5 * np.abs(e[:-1]) <= 0.1 * TOL)) + 1
    assert s == first + 2


def test_never_met():
    k = np.arange(100)
    assert stop(1e-3 * (1.0 + 0.01 * k)) == -1           # drifting
    assert stop(np.full(50, np.nan)) == -1
    assert gp.stop_rule_eval(np.array([]), TOL) == -1
    # a non-finite value restarts the rule: it needs fresh checks afterwards
    e = 1e-3 * 0.5 ** k
    e_bad = e.copy()
    s0 = stop(e)
    e_bad[s0 - 1] = np.nan
    assert stop(e_bad) > s0


def test_invalid_arguments():
    L = gp.load()
    out = ctypes.c_int32()
    assert L.gp_stop_rule_eval(None, -1, TOL, ctypes.byref(out)) == gp.GP_ERR_INVALID
    assert L.gp_stop_rule_eval(None, 3, TOL, ctypes.byref(out)) == gp.GP_ERR_INVALID
    assert L.gp_stop_rule_eval(None, 0, TOL, ctypes.byref(out)) == gp.GP_OK
