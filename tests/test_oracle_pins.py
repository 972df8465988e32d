"""Pins of the CPU FP64 oracle against mathematics that does not come from the oracle.

Each test checks the oracle against something the method or the physics fixes
independently of the oracle's own code: dense linear algebra (numpy), closed-form
eigenvalues of the Dirichlet second difference, Perron vectors of the one-step operator
at g = 0, the harmonic-oscillator ground state, exact conservation laws and symmetries,
and convergence orders.  The method is the split-step Crank-Nicolson scheme (paper:
program summary, "Solution method"; sub-step functions calcnu, calclux, calcluy, calcluz,
calcrms, calcmuen under "Summary of revisions").
"""
import math

import numpy as np
import pytest

import oracle
from paper_1601_04641_amd import inputs

NU = inputs.NU_PAPER


# ----------------------------------------------------------------------------------------
# independent dense building blocks (numpy only)
# ----------------------------------------------------------------------------------------
def kin1d(n, d):
    """-1/2 second difference / d^2 with homogeneous Dirichlet ghosts, dense."""
    D2 = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    return -0.5 * D2 / (d * d)


def cn1d(n, d, tau, imag):
    """Crank-Nicolson propagator of the kinetic part along one axis, from its definition:
    (I + z K/2) u = (I - z K/2) p with z = tau (imaginary time) or i tau (real time)."""
    K = kin1d(n, d)
    z = tau if imag else 1j * tau
    I = np.eye(n)
    return np.linalg.solve(I + 0.5 * z * K, I - 0.5 * z * K)


def pot3d(nx, ny, nz, dx, dy, dz, nux, nuy, nuz):
    x, y, z = inputs.axis(nx, dx), inputs.axis(ny, dy), inputs.axis(nz, dz)
    return 0.5 * (nux ** 2 * x[:, None, None] ** 2 + nuy ** 2 * y[None, :, None] ** 2
                  + nuz ** 2 * z[None, None, :] ** 2)


def dense_step(psi, prm, imag, split):
    """One full step built from Kronecker products of the dense 1D propagators."""
    nx, ny, nz = psi.shape
    dx, dy, dz, dt, g = prm["dx"], prm["dy"], prm["dz"], prm["dt"], prm["g"]
    V = pot3d(nx, ny, nz, dx, dy, dz, prm["nux"], prm["nuy"], prm["nuz"])

    def N(p, tau):
        w = V + g * np.abs(p) ** 2
        return p * (np.exp(-tau * w) if imag else np.exp(-1j * tau * w))

    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    Cx = np.kron(np.kron(cn1d(nx, dx, dt, imag), Iy), Iz)
    Cy = np.kron(np.kron(Ix, cn1d(ny, dy, dt, imag)), Iz)
    Cz = np.kron(np.kron(Ix, Iy), cn1d(nz, dz, dt, imag))
    p = N(psi, dt if split == 0 else 0.5 * dt).reshape(-1)
    p = Cz @ (Cy @ (Cx @ p))
    p = p.reshape(psi.shape)
    if split == 1:
        p = N(p, 0.5 * dt)
    if imag:
        p = p / math.sqrt(float(np.sum(np.abs(p) ** 2)) * dx * dy * dz)
    return p


def small_prm(**kw):
    prm = dict(nx=5, ny=4, nz=6, dx=0.3, dy=0.45, dz=0.25, nux=1.3, nuy=0.7, nuz=2.1,
               g=3.7, dt=0.05)
    prm.update(kw)
    return prm


# ----------------------------------------------------------------------------------------
# P1: one CN line solve equals the dense definition
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 17, 40])
@pytest.mark.parametrize("imag", [True, False])
def test_cn_line_matches_dense_solve(n, imag):
    rng = np.random.default_rng(n)
    d, tau = 0.37, 0.21
    p = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c = tau / (4 * d * d) * (1 if imag else 1j)
    got = oracle.cn_line(p, c)
    want = cn1d(n, d, tau, imag) @ p
    assert np.max(np.abs(got - want)) <= 1e-13 * max(1.0, np.max(np.abs(want)))


# ----------------------------------------------------------------------------------------
# P13: whole steps on tiny grids equal the dense Kronecker composition
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("split", [0, 1])
def test_full_step_matches_dense_kronecker(imag, split):
    prm = small_prm()
    psi0 = inputs.perturbed_psi(prm["nx"], prm["ny"], prm["nz"], prm["dx"], prm["dy"], prm["dz"],
                                prm["nux"], prm["nuy"], prm["nuz"], seed=3, amp=0.3)
    o = oracle.Oracle.from_params(prm, psi0, split=split)
    want = psi0.copy()
    for _ in range(3):
        want = dense_step(want, prm, imag, split)
    (o.step_imag if imag else o.step_real)(3)
    assert np.max(np.abs(o.psi - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("which,axis", [(1, 0), (2, 1), (3, 2)])
def test_single_sweep_acts_on_its_own_axis(which, axis):
    prm = small_prm()
    psi0 = inputs.perturbed_psi(prm["nx"], prm["ny"], prm["nz"], prm["dx"], prm["dy"], prm["dz"],
                                prm["nux"], prm["nuy"], prm["nuz"], seed=5, amp=0.3)
    o = oracle.Oracle.from_params(prm, psi0)
    o.substep(which, False, prm["dt"])
    n = psi0.shape[axis]
    d = (prm["dx"], prm["dy"], prm["dz"])[axis]
    C = cn1d(n, d, prm["dt"], False)
    want = np.moveaxis(np.tensordot(C, np.moveaxis(psi0, axis, 0), axes=(1, 0)), 0, axis)
    assert np.max(np.abs(o.psi - want)) <= 1e-13 * np.max(np.abs(want))


# ----------------------------------------------------------------------------------------
# P2: Dirichlet sine modes are eigenvectors; closed-form multiplier per sweep
# ----------------------------------------------------------------------------------------
def sine_multiplier(n, k, c):
    s2 = math.sin(k * math.pi / (2 * (n + 1))) ** 2
    return (1 - 4 * c * s2) / (1 + 4 * c * s2)


@pytest.mark.parametrize("modes", [(1, 1, 1), (1, 3, 2), (4, 1, 5)])
def test_sine_modes_closed_form(modes):
    nx, ny, nz, d, dt = 33, 20, 17, 0.15, 0.01
    prm = dict(nx=nx, ny=ny, nz=nz, dx=d, dy=1.3 * d, dz=0.8 * d, nux=0.0, nuy=0.0, nuz=0.0,
               g=0.0, dt=dt)
    psi0 = inputs.sine_mode_psi(nx, ny, nz, *modes)
    # real time: one step multiplies by a product of unit-modulus factors
    o = oracle.Oracle.from_params(prm, psi0)
    o.step_real(1)
    f = 1.0
    for n, k, dd in zip((nx, ny, nz), modes, (prm["dx"], prm["dy"], prm["dz"])):
        f *= sine_multiplier(n, k, 1j * dt / (4 * dd * dd))
    assert abs(abs(f) - 1) < 1e-15
    assert np.max(np.abs(o.psi - f * psi0)) <= 1e-13
    # imaginary time: shape kept, pre-renormalisation norm = f^2 * initial norm
    o2 = oracle.Oracle.from_params(prm, psi0)
    n0 = float(np.sum(np.abs(psi0) ** 2)) * prm["dx"] * prm["dy"] * prm["dz"]
    o2.step_imag(1)
    f2 = 1.0
    for n, k, dd in zip((nx, ny, nz), modes, (prm["dx"], prm["dy"], prm["dz"])):
        f2 *= sine_multiplier(n, k, dt / (4 * dd * dd))
    assert abs(o2.last_npre() / (f2 * f2 * n0) - 1) < 1e-13
    assert np.max(np.abs(o2.psi - psi0 / math.sqrt(n0))) <= 1e-13


# ----------------------------------------------------------------------------------------
# P4: g = 0 fixed point is the product of the 1D Perron vectors of C_a exp(-dt V_a)
# ----------------------------------------------------------------------------------------
def perron_1d(n, d, nu, dt):
    x = inputs.axis(n, d)
    e = np.exp(-dt * 0.5 * nu * nu * x * x)
    C = cn1d(n, d, dt, True)
    S = np.sqrt(e)[:, None] * C * np.sqrt(e)[None, :]   # similar to C diag(e), symmetric
    w, U = np.linalg.eigh(S)
    v = U[:, -1] / np.sqrt(e)
    v = v * np.sign(v[n // 2])
    H = kin1d(n, d) + np.diag(0.5 * nu * nu * x * x)
    return w[-1], v / np.linalg.norm(v), float(v @ H @ v / (v @ v))


def test_g0_fixed_point_is_perron_product():
    nx, ny, nz, d = 20, 16, 12, 0.4
    dt = 0.1 * d * d
    prm = dict(nx=nx, ny=ny, nz=nz, dx=d, dy=d, dz=d, nux=NU[0], nuy=NU[1], nuz=NU[2], g=0.0, dt=dt)
    psi0 = inputs.gaussian_psi(nx, ny, nz, d, d, d, *NU)
    o = oracle.Oracle.from_params(prm, psi0)
    prev = o.psi.copy()
    for _ in range(60):
        o.step_imag(100)
        if np.max(np.abs(o.psi - prev)) < 1e-14:
            break
        prev = o.psi.copy()
    (lx, vx, mx), (ly, vy, my), (lz, vz, mz) = (perron_1d(n, d, nu, dt)
                                                 for n, nu in zip((nx, ny, nz), NU))
    want = vx[:, None, None] * vy[None, :, None] * vz[None, None, :]
    want = want / math.sqrt(float(np.sum(want ** 2)) * d ** 3)
    assert np.max(np.abs(o.psi - want)) <= 1e-10
    assert abs(o.last_npre() / (lx * ly * lz) ** 2 - 1) <= 1e-12
    e, mu = o.energy_mu()
    assert abs(mu - (mx + my + mz)) <= 1e-11 * mu
    assert abs(e - mu) <= 1e-14 * mu          # g = 0: E = mu


# ----------------------------------------------------------------------------------------
# P5 / P11: harmonic-oscillator limit and second order in dx (g = 0)
# ----------------------------------------------------------------------------------------
def ground_mu_g0(d, steps_cap=4000):
    box = (4.8, 4.0, 3.2)
    nx, ny, nz = (int(round(2 * b / d)) for b in box)
    dt = 0.1 * d * d
    prm = dict(nx=nx, ny=ny, nz=nz, dx=d, dy=d, dz=d, nux=NU[0], nuy=NU[1], nuz=NU[2], g=0.0, dt=dt)
    o = oracle.Oracle.from_params(prm, inputs.gaussian_psi(nx, ny, nz, d, d, d, *NU))
    mu_prev = None
    done = 0
    while done < steps_cap:
        o.step_imag(100)
        done += 100
        mu = o.energy_mu()[1]
        if mu_prev is not None and abs(mu - mu_prev) < 1e-13:
            break
        mu_prev = mu
    return mu, o.rms()


@pytest.mark.slow
def test_harmonic_limit_and_dx_order():
    exact = 0.5 * sum(NU)
    mu_a, rms_a = ground_mu_g0(0.4)
    mu_b, rms_b = ground_mu_g0(0.2)
    # leading discrete error of the 3-point Laplacian: -d^2 sum(nu^2)/32
    for d, mu in ((0.4, mu_a), (0.2, mu_b)):
        lead = -d * d * sum(v * v for v in NU) / 32
        assert abs(mu - exact - lead) < 0.05 * abs(lead)
    ratio = (mu_a - exact) / (mu_b - exact)
    assert 3.8 < ratio < 4.2
    # <a^2> = 1/(2 nu_a) for the oscillator ground state, approached at second order in dx
    for a in range(3):
        ea, eb = rms_a[a] ** 2 * 2 * NU[a] - 1, rms_b[a] ** 2 * 2 * NU[a] - 1
        assert abs(eb) < 6e-3
        assert 3.6 < ea / eb < 4.5
    assert abs(rms_b[3] ** 2 - sum(r * r for r in rms_b[:3])) < 1e-14


# ----------------------------------------------------------------------------------------
# observables: kinetic link sum (ghost links included) = <psi, K psi>; dense energy
# ----------------------------------------------------------------------------------------
def test_observables_match_dense_quadratic_forms():
    prm = small_prm(nx=6, ny=5, nz=7)
    psi = inputs.perturbed_psi(prm["nx"], prm["ny"], prm["nz"], prm["dx"], prm["dy"], prm["dz"],
                               prm["nux"], prm["nuy"], prm["nuz"], seed=11, amp=0.5) * 1.7
    o = oracle.Oracle.from_params(prm, psi)
    raw = o.raw_sums()
    nx, ny, nz = psi.shape
    dV = prm["dx"] * prm["dy"] * prm["dz"]
    v = psi.reshape(-1)
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    Kx = np.kron(np.kron(kin1d(nx, prm["dx"]), Iy), Iz)
    Ky = np.kron(np.kron(Ix, kin1d(ny, prm["dy"])), Iz)
    Kz = np.kron(np.kron(Ix, Iy), kin1d(nz, prm["dz"]))
    V = pot3d(nx, ny, nz, prm["dx"], prm["dy"], prm["dz"], prm["nux"], prm["nuy"], prm["nuz"]).reshape(-1)
    n2 = np.abs(v) ** 2
    for q, K in ((1, Kx), (2, Ky), (3, Kz)):
        assert abs(raw[q] - dV * np.real(np.vdot(v, K @ v))) < 1e-12 * raw[q]
    assert abs(raw[0] - dV * n2.sum()) < 1e-13 * raw[0]
    assert abs(raw[4] - dV * (V * n2).sum()) < 1e-13 * raw[4]
    assert abs(raw[5] - dV * (n2 * n2).sum()) < 1e-13 * raw[5]
    # energy of the normalised state, from the dense Hamiltonian
    phi = v / math.sqrt(dV * n2.sum())
    H = Kx + Ky + Kz + np.diag(V)
    lin = dV * np.real(np.vdot(phi, H @ phi))
    quart = dV * np.sum(np.abs(phi) ** 4)
    e, mu = o.energy_mu()
    assert abs(e - (lin + 0.5 * prm["g"] * quart)) < 1e-12 * abs(e)
    assert abs(mu - (lin + prm["g"] * quart)) < 1e-12 * abs(mu)
    x, y, z = (inputs.axis(n, d) for n, d in ((nx, prm["dx"]), (ny, prm["dy"]), (nz, prm["dz"])))
    p3 = np.abs(phi.reshape(psi.shape)) ** 2 * dV
    rx = math.sqrt(np.sum(p3 * x[:, None, None] ** 2))
    rz = math.sqrt(np.sum(p3 * z[None, None, :] ** 2))
    rms = o.rms()
    assert abs(rms[0] - rx) < 1e-13 and abs(rms[2] - rz) < 1e-13


# ----------------------------------------------------------------------------------------
# P6, P8, P9: conservation and symmetries
# ----------------------------------------------------------------------------------------
def test_real_time_conserves_norm():
    prm = small_prm(nx=12, ny=10, nz=8, g=25.0, dt=0.01)
    psi0 = inputs.perturbed_psi(prm["nx"], prm["ny"], prm["nz"], prm["dx"], prm["dy"], prm["dz"],
                                prm["nux"], prm["nuy"], prm["nuz"], seed=7, amp=0.4)
    o = oracle.Oracle.from_params(prm, psi0)
    n0 = o.norm()
    o.step_real(400)
    assert abs(o.norm() - n0) < 400 * 4e-16 * n0
    assert np.max(np.abs(o.psi - psi0)) > 1e-2      # it did move


def test_imaginary_time_keeps_real_state_real():
    w = inputs.WORKLOADS["imag_48x40x32"]
    psi0 = inputs.gaussian_psi(w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                               w["nux"], w["nuy"], w["nuz"])
    o = oracle.Oracle.from_params(w, psi0)
    o.step_imag(50)
    assert np.all(o.psi.imag == 0.0)


@pytest.mark.parametrize("imag", [True, False])
def test_parity_symmetry(imag):
    prm = dict(nx=21, ny=16, nz=13, dx=0.3, dy=0.35, dz=0.4, nux=1.0, nuy=1.4142, nuz=1.7321,
               g=30.0, dt=0.01)
    psi0 = inputs.gaussian_psi(21, 16, 13, 0.3, 0.35, 0.4, 0.8, 1.1, 1.5)
    o = oracle.Oracle.from_params(prm, psi0)
    (o.step_imag if imag else o.step_real)(40)
    p = o.psi
    scale = np.max(np.abs(p))
    for ax in range(3):
        assert np.max(np.abs(p - np.flip(p, axis=ax))) < 1e-13 * scale


# ----------------------------------------------------------------------------------------
# P7, P10: the converged ground state is stationary in real time and satisfies the virial
# ----------------------------------------------------------------------------------------
def converged_ground_state(d=0.3, g=15.0, split=0):
    box = (4.8, 4.0, 3.3)
    nx, ny, nz = (int(round(2 * b / d)) for b in box)
    dt = 0.1 * d * d
    prm = dict(nx=nx, ny=ny, nz=nz, dx=d, dy=d, dz=d, nux=NU[0], nuy=NU[1], nuz=NU[2], g=g, dt=dt)
    o = oracle.Oracle.from_params(prm, inputs.gaussian_psi(nx, ny, nz, d, d, d, *NU), split=split)
    prev = None
    for _ in range(80):
        o.step_imag(100)
        mu = o.energy_mu()[1]
        if prev is not None and abs(mu - prev) < 1e-13 * abs(mu):
            break
        prev = mu
    return o, prm


@pytest.mark.slow
def test_ground_state_stationary_and_virial():
    o, prm = converged_ground_state()
    e, mu = o.energy_mu()
    raw = o.raw_sums()
    T, U, I = raw[1] + raw[2] + raw[3], raw[4], raw[5]
    # virial theorem for the harmonic trap with contact interaction: 2T - 2U + 3 (g/2) I = 0
    vir = (2 * T - 2 * U + 1.5 * prm["g"] * I) / (T + U)
    assert abs(vir) < 1e-3
    psi0 = o.psi.copy()
    t = 0.5
    n = int(round(t / prm["dt"]))
    o.step_real(n)
    drift = np.max(np.abs(np.abs(o.psi) - np.abs(psi0))) / np.max(np.abs(psi0))
    # the Lie imaginary-time fixed point is stationary up to the O(dt) splitting error
    assert drift < 5e-3
    dV = prm["dx"] * prm["dy"] * prm["dz"]
    phase = np.angle(np.vdot(psi0, o.psi) * dV)
    assert abs(phase + mu * n * prm["dt"]) < 1e-3 * mu * t


# ----------------------------------------------------------------------------------------
# P11: time-step order in real time (Lie 1, Strang 2)
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("split,order", [(0, 1.0), (1, 2.0)])
def test_real_time_dt_order(split, order):
    d = 0.4
    nx, ny, nz = 16, 14, 12
    base = dict(nx=nx, ny=ny, nz=nz, dx=d, dy=d, dz=d, nux=1.0, nuy=1.4142, nuz=1.7321, g=20.0)
    psi0 = inputs.perturbed_psi(nx, ny, nz, d, d, d, 1.3, 1.2, 1.9, seed=1, amp=0.1)
    t = 0.4
    res = []
    for dt in (0.02, 0.01, 0.005):
        prm = dict(base, dt=dt)
        o = oracle.Oracle.from_params(prm, psi0, split=split)
        o.step_real(int(round(t / dt)))
        res.append(o.psi.copy())
    r = np.max(np.abs(res[0] - res[1])) / np.max(np.abs(res[1] - res[2]))
    assert abs(math.log2(r) - order) < 0.2


# ---------------------------------------------------------------- stationary-equation residual
def _sine_mode(shape, modes):
    out = np.ones(shape)
    for a, (n, k) in enumerate(zip(shape, modes)):
        s = [1, 1, 1]
        s[a] = n
        out = out * np.sin(np.arange(1, n + 1) * k * np.pi / (n + 1)).reshape(s)
    return out


def _sine_eig(shape, modes, d):
    return sum(2.0 * np.sin(k * np.pi / (2 * (n + 1))) ** 2 / h ** 2 for n, k, h in zip(shape, modes, d))


def test_residual_zero_on_discrete_eigenmodes():
    """nu = 0, g = 0: products of Dirichlet sine modes are exact eigenvectors of -1/2 lap_h
    with eigenvalue sum 2 sin^2(k pi / (2(n+1))) / d^2."""
    from oracle.residual import residual
    shape, d = (9, 7, 6), (0.3, 0.25, 0.4)
    prm = dict(dx=d[0], dy=d[1], dz=d[2], nux=0.0, nuy=0.0, nuz=0.0, g=0.0)
    for modes in [(1, 1, 1), (2, 3, 1), (4, 1, 5)]:
        r, mu = residual(3.7 * _sine_mode(shape, modes), prm)
        assert r <= 1e-12 * mu
        assert abs(mu - _sine_eig(shape, modes, d)) <= 1e-12 * mu


def test_residual_of_a_two_mode_mixture_closed_form():
    """phi = a e1 + b e2 (orthonormal eigenvectors): mu = a^2 l1 + b^2 l2 and
    res = |a b| |l1 - l2|."""
    from oracle.residual import residual
    shape, d = (8, 6, 7), (0.2, 0.3, 0.25)
    prm = dict(dx=d[0], dy=d[1], dz=d[2], nux=0.0, nuy=0.0, nuz=0.0, g=0.0)
    dV = np.prod(d)
    e1, e2 = _sine_mode(shape, (1, 1, 1)), _sine_mode(shape, (3, 2, 1))
    e1 /= np.sqrt(dV * (e1 ** 2).sum())
    e2 /= np.sqrt(dV * (e2 ** 2).sum())
    a, b = 0.8, 0.6
    l1, l2 = _sine_eig(shape, (1, 1, 1), d), _sine_eig(shape, (3, 2, 1), d)
    r, mu = residual(a * e1 + b * e2, prm)
    assert abs(mu - (a * a * l1 + b * b * l2)) <= 1e-12 * mu
    assert abs(r - a * b * abs(l1 - l2)) <= 1e-11 * mu


def test_residual_matches_brute_force_on_a_tiny_grid():
    """Every term of H written out point by point with explicit loops (trap, nonlinearity,
    complex state)."""
    from oracle.residual import residual
    rng = np.random.default_rng(4)
    nx, ny, nz = 4, 3, 5
    prm = dict(dx=0.4, dy=0.5, dz=0.3, nux=1.3, nuy=0.7, nuz=2.1, g=17.0)
    psi = rng.standard_normal((nx, ny, nz)) + 1j * rng.standard_normal((nx, ny, nz))
    dV = prm["dx"] * prm["dy"] * prm["dz"]
    phi = psi / np.sqrt(dV * np.sum(np.abs(psi) ** 2))
    d = (prm["dx"], prm["dy"], prm["dz"])
    nu = (prm["nux"], prm["nuy"], prm["nuz"])
    dims = (nx, ny, nz)

    def at(i, j, k):
        return phi[i, j, k] if 0 <= i < nx and 0 <= j < ny and 0 <= k < nz else 0.0

    h = np.zeros_like(phi)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                idx = (i, j, k)
                v = 0.0
                lap = 0.0
                for a in range(3):
                    x = (idx[a] - (dims[a] - 1) / 2.0) * d[a]
                    v += 0.5 * nu[a] ** 2 * x * x
                    up = list(idx)
                    dn = list(idx)
                    up[a] += 1
                    dn[a] -= 1
                    lap += (at(*up) + at(*dn) - 2 * phi[idx]) / d[a] ** 2
                h[idx] = -0.5 * lap + v * phi[idx] + prm["g"] * abs(phi[idx]) ** 2 * phi[idx]
    mu = (dV * np.sum(np.conj(phi) * h)).real
    want = np.sqrt(dV * np.sum(np.abs(h - mu * phi) ** 2))
    r, m = residual(psi, prm)
    assert abs(m - mu) <= 1e-12 * abs(mu) and abs(r - want) <= 1e-12 * want


# ----------------------------------------------------------------------------------------
# P14: with g = 0 a Lie step maps a product state to the product of 1D results (the
# potential factor is a product of 1D factors, each sweep acts on its own axis); the 1D
# result of an axis is the potential step and sweep on a grid three points wide in the
# other axes, read on its centre row (zero potential there).  The large-grid GPU test
# builds its expected values this way.
# ----------------------------------------------------------------------------------------
def _centre_row_step(axis, f, prm, imag):
    shp = [3, 3, 3]
    shp[axis] = f.size
    psi0 = np.zeros(shp, dtype=np.complex128)
    idx = [1, 1, 1]
    idx[axis] = slice(None)
    psi0[tuple(idx)] = f
    o = oracle.Oracle.from_params(dict(prm, nx=shp[0], ny=shp[1], nz=shp[2], g=0.0), psi0)
    o.substep(0, imag, prm["dt"])
    o.substep(axis + 1, imag, prm["dt"])
    return o.psi[tuple(idx)].copy()


@pytest.mark.parametrize("imag", [False, True])
def test_lie_step_of_product_state_factorises(imag):
    nx, ny, nz, d = 23, 17, 12, 0.3
    prm = dict(nx=nx, ny=ny, nz=nz, dx=d, dy=d, dz=d, nux=1.0, nuy=1.4142, nuz=1.7321, g=0.0, dt=0.02)
    rng = np.random.default_rng(3)
    f = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in (nx, ny, nz)]
    o = oracle.Oracle.from_params(prm, np.einsum("i,j,k->ijk", *f))
    (o.step_imag if imag else o.step_real)(1)
    want = np.einsum("i,j,k->ijk", *(_centre_row_step(a, f[a], prm, imag) for a in range(3)))
    if imag:
        want /= math.sqrt(float(np.sum(np.abs(want) ** 2)) * d ** 3)
    assert np.max(np.abs(o.psi - want)) <= 1e-13 * np.max(np.abs(want))
