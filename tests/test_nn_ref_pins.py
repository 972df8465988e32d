"""Pins of the FP64 warm-start network reference against mathematics that does not use it:
brute-force and library convolutions, adjoint identities, a closed-form prior,
central finite differences of the whole network, and closed forms of Adam."""
import math

import numpy as np
import pytest
import scipy.ndimage

from oracle import gpnn_ref as R
from paper_1601_04641_amd import inputs


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv3d_matches_brute_force_loops():
    n, D, ci, co = 2, 3, 2, 3
    x, W, b = rnd((n, D, D, D, ci), 0), rnd((27, co, ci), 1), rnd((co,), 2)
    y = R.conv3d(x, W, b)
    for s in range(n):
        for i in range(D):
            for j in range(D):
                for k in range(D):
                    for o in range(co):
                        acc = b[o]
                        for a in range(3):
                            for bb in range(3):
                                for c in range(3):
                                    ii, jj, kk = i + a - 1, j + bb - 1, k + c - 1
                                    if 0 <= ii < D and 0 <= jj < D and 0 <= kk < D:
                                        acc += sum(W[(a * 3 + bb) * 3 + c, o, q] * x[s, ii, jj, kk, q]
                                                   for q in range(ci))
                        assert abs(y[s, i, j, k, o] - acc) <= 1e-12


def test_conv3d_single_channel_matches_scipy_correlate():
    x, W = rnd((1, 7, 6, 5, 1), 3), rnd((27, 1, 1), 4)
    want = scipy.ndimage.correlate(x[0, ..., 0], W[:, 0, 0].reshape(3, 3, 3), mode="constant", cval=0.0)
    assert np.max(np.abs(R.conv3d(x, W)[0, ..., 0] - want)) <= 1e-12


def test_conv3d_backward_passes_are_adjoints():
    x, W, dy = rnd((2, 4, 4, 4, 3), 5), rnd((27, 5, 3), 6), rnd((2, 4, 4, 4, 5), 7)
    lhs = float((R.conv3d(x, W) * dy).sum())
    assert abs(lhs - float((x * R.conv3d_bwd_data(dy, W)).sum())) <= 1e-10 * abs(lhs)
    assert abs(lhs - float((W * R.conv3d_bwd_weight(dy, x)).sum())) <= 1e-10 * abs(lhs)


def test_up2_and_pool2_sum_are_adjoints():
    a, b = rnd((2, 3, 3, 3, 4), 8), rnd((2, 6, 6, 6, 4), 9)
    assert abs(float((R.up2(a) * b).sum()) - float((a * R.pool2_sum(b)).sum())) <= 1e-11
    assert R.up2(a)[0, 5, 4, 3, 2] == a[0, 2, 2, 1, 2]


def test_log_prior_is_the_normalised_harmonic_ground_state():
    """exp(ln G) is the g = 0 ground state: unit norm, and H G = (sum nu / 2) G."""
    p = np.array([[0.7, 1.3, 2.1, 5.0]])
    n, dx = 96, 0.2
    G = np.exp(R.log_prior(p, n, dx))[0]
    assert abs((G ** 2).sum() * dx ** 3 - 1.0) <= 1e-10
    x = R.grid_axis(n, dx)
    i = n // 2 + 3
    # continuum H applied analytically at a point: -1/2 d2/dx2 exp(-nu x^2/2) + 1/2 nu^2 x^2 ...
    val = sum(0.5 * nu - 0.5 * nu ** 2 * x[i] ** 2 + 0.5 * nu ** 2 * x[i] ** 2 for nu in p[0, :3])
    assert abs(val - 0.5 * p[0, :3].sum()) <= 1e-12


def test_silu_grad_matches_finite_differences():
    x = np.linspace(-6, 6, 41)
    h = 1e-6
    fd = (R.silu(x + h) - R.silu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - R.silu_grad(x))) <= 1e-8


def tiny():
    return R.Arch(base=2, hidden=5, ch=(3, 2, 2), dx=0.5)


def test_whole_network_gradient_matches_central_differences():
    a = tiny()
    w = inputs.nn_init_weights(R.param_shapes(a), seed=11)
    rng = np.random.default_rng(12)
    for k in w:  # non-trivial head and biases so every path carries gradient
        w[k] = w[k] + 0.3 * rng.standard_normal(np.shape(w[k]))
    p = inputs.draw_nn_params(13, 3)
    psi0, _ = R.forward(w, p, a)
    target = psi0 * (1 + 0.3 * rng.standard_normal(psi0.shape)) + 0.01
    _, cache = R.forward(w, p, a)
    g = R.backward(w, cache, target, a)
    h = 1e-6
    for name, shp in R.param_shapes(a):
        flat = np.asarray(w[name]).reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            wp = {k: np.array(v, copy=True) for k, v in w.items()}
            wm = {k: np.array(v, copy=True) for k, v in w.items()}
            wp[name].reshape(-1)[idx] += h
            wm[name].reshape(-1)[idx] -= h
            fd = (R.loss(R.forward(wp, p, a)[0], target, a) - R.loss(R.forward(wm, p, a)[0], target, a)) / (2 * h)
            an = np.asarray(g[name]).reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_untrained_network_returns_the_prior():
    a = tiny()
    w = inputs.nn_init_weights(R.param_shapes(a), seed=1)
    p = inputs.draw_nn_params(2, 2)
    psi, _ = R.forward(w, p, a)
    assert np.max(np.abs(psi - np.exp(R.log_prior(p, a.n_out, a.dx)))) <= 1e-14


def test_loss_closed_form():
    a = tiny()
    t = rnd((2, 8, 8, 8), 3)
    assert R.loss(t, t, a) == 0.0
    assert abs(R.loss(1.1 * t, t, a) - 0.01 * (t ** 2).sum() * a.dx ** 3 / 2) <= 1e-12


def test_adam_constant_gradient_moves_by_lr_per_step():
    """With a constant gradient the bias-corrected moments are g and g^2, so each step
    moves every weight by exactly lr against the sign of its gradient (eps = 0)."""
    w0 = np.array([1.0, -2.0, 0.5])
    gv = np.array([3.0, -0.25, 1e-3])
    w, m, v = w0.copy(), np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        w, m, v = R.adam(w, gv, m, v, t, lr=0.01, eps=0.0)
        assert np.max(np.abs(w - (w0 - 0.01 * t * np.sign(gv)))) <= 1e-14


def test_adam_first_step_with_eps():
    w, _, _ = R.adam(np.array([0.0]), np.array([2e-8]), np.zeros(1), np.zeros(1), 1, lr=0.1, eps=1e-8)
    assert abs(w[0] + 0.1 * 2e-8 / (2e-8 + 1e-8)) <= 1e-16


def test_param_count_of_the_warm_start_network():
    n = sum(int(np.prod(s)) for _, s in R.param_shapes(R.Arch()))
    assert 1.5e6 <= n <= 2.5e6
