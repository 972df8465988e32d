"""Seeded synthetic inputs for the SSCN Gross-Pitaevskii workloads.

This module holds no arithmetic of the method itself: it only builds grids' initial
wavefunctions and draws trap parameters from seeds.  Both the GPU path and the CPU oracle
take its outputs as inputs; neither is imported here.

The paper's own input files are not available, so the workloads below are synthetic
stand-ins with the grid shapes of the paper's runs (x the longest axis, aspect ratios
like 6:5:4, paper: figure captions of the scalability study) and the sizes listed in
``WORKLOADS``.
"""
from __future__ import annotations

import math

import numpy as np

NU_PAPER = (1.0, 1.4142, 1.7321)

# Named workloads (grid, spacing, trap, nonlinearity, time step, step count).
WORKLOADS = {
    # small parity case: anisotropic trap, 500 imaginary steps
    "imag_48x40x32": dict(nx=48, ny=40, nz=32, dx=0.2, dy=0.2, dz=0.2, nux=1.0, nuy=1.4142,
                          nuz=1.7321, g=22.454, dt=0.1 * 0.2 ** 2, steps=500),
    # real-time quench at scale: 512x480x448, g 100 -> 50, dt = 0.01 dx^2
    "quench_512x480x448": dict(nx=512, ny=480, nz=448, dx=0.05, dy=0.05, dz=0.05, nux=1.0,
                               nuy=1.4142, nuz=1.7321, g=100.0, dt=0.01 * 0.05 ** 2,
                               dt_imag=0.1 * 0.05 ** 2, g_quench=50.0, steps=1000),
    # the paper's large run grids (1000 iterations each) with the quench workload's box and
    # trap: imaginary time on 1920x1600x1280, real time on 1600x1280x960 (complex64)
    "paper_imag_1920x1600x1280": dict(nx=1920, ny=1600, nz=1280, dx=0.05 * 512 / 1920, dy=0.05 * 512 / 1920,
                                      dz=0.05 * 512 / 1920, nux=1.0, nuy=1.4142, nuz=1.7321, g=100.0,
                                      dt=0.1 * (0.05 * 512 / 1920) ** 2, steps=1000),
    "paper_real_1600x1280x960": dict(nx=1600, ny=1280, nz=960, dx=0.016, dy=0.016, dz=0.016, nux=1.0,
                                     nuy=1.4142, nuz=1.7321, g=100.0, dt=0.01 * 0.016 ** 2, steps=1000),
    # precision form: 384^3, dx = 0.08, imaginary time (trap drawn per seed)
    "imag_384cube": dict(nx=384, ny=384, nz=384, dx=0.08, dy=0.08, dz=0.08, dt=0.1 * 0.08 ** 2,
                         steps=20000),
}


def axis(n: int, d: float) -> np.ndarray:
    """Cell-centred symmetric coordinates (i - (n-1)/2) d."""
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * d


def gaussian_psi(nx, ny, nz, dx, dy, dz, nux, nuy, nuz, dtype=np.complex128) -> np.ndarray:
    """Anisotropic Gaussian prod_a (nu_a/pi)^(1/4) exp(-nu_a a^2/2), normalised so that
    dx dy dz sum |psi|^2 = 1 on the grid.  nu_a = 0 uses width 1."""
    parts = []
    for n, d, nu in ((nx, dx, nux), (ny, dy, nuy), (nz, dz, nuz)):
        w = nu if nu > 0 else 1.0
        a = axis(n, d)
        parts.append((w / math.pi) ** 0.25 * np.exp(-0.5 * w * a * a))
    psi = parts[0][:, None, None] * parts[1][None, :, None] * parts[2][None, None, :]
    psi = psi / math.sqrt(float(np.sum(psi * psi)) * dx * dy * dz)
    return psi.astype(dtype)


def gaussian_factors(nx, ny, nz, dx, dy, dz, nux, nuy, nuz):
    """The three 1D factors whose outer product is gaussian_psi (each normalised on its
    own axis), for grids too large to build on the host."""
    out = []
    for n, d, nu in ((nx, dx, nux), (ny, dy, nuy), (nz, dz, nuz)):
        w = nu if nu > 0 else 1.0
        a = axis(n, d)
        f = np.exp(-0.5 * w * a * a)
        out.append(f / math.sqrt(float(np.sum(f * f)) * d))
    return out


def gaussian_cube_batch(prm, n: int, d: float, out: np.ndarray | None = None, dtype=np.complex64) -> np.ndarray:
    """gaussian_psi for many problems on one n^3 grid of spacing d: prm rows are
    (nu_x, nu_y, nu_z, g); returns [len(prm), n, n, n], each normalised on the grid."""
    prm = np.asarray(prm, dtype=np.float64)
    a = axis(n, d)
    if out is None:
        out = np.empty((len(prm), n, n, n), dtype=dtype)
    for i, (nux, nuy, nuz, _) in enumerate(prm):
        f = [np.exp(-0.5 * nu * a * a) for nu in (nux, nuy, nuz)]
        f = [v / math.sqrt(float(np.sum(v * v)) * d) for v in f]
        out[i] = (f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]).astype(dtype)
    return out


def perturbed_psi(nx, ny, nz, dx, dy, dz, nux, nuy, nuz, seed: int, amp=0.05,
                  dtype=np.complex128) -> np.ndarray:
    """Gaussian times a seeded complex perturbation (breaks every symmetry, including
    Im psi = 0), renormalised to unit grid norm.  Used where the test needs a generic state."""
    rng = np.random.default_rng(seed)
    base = gaussian_psi(nx, ny, nz, dx, dy, dz, nux, nuy, nuz, dtype=np.complex128)
    noise = rng.standard_normal((nx, ny, nz)) + 1j * rng.standard_normal((nx, ny, nz))
    psi = base * (1.0 + amp * noise)
    psi = psi / math.sqrt(float(np.sum(np.abs(psi) ** 2)) * dx * dy * dz)
    return psi.astype(dtype)


def sine_mode_psi(nx, ny, nz, kx, ky, kz, dtype=np.complex128) -> np.ndarray:
    """Product of discrete Dirichlet sine modes sin(i' k pi/(n+1)), i' = i+1 (1-based)."""
    parts = []
    for n, k in ((nx, kx), (ny, ky), (nz, kz)):
        i1 = np.arange(1, n + 1, dtype=np.float64)
        parts.append(np.sin(i1 * k * math.pi / (n + 1)))
    psi = parts[0][:, None, None] * parts[1][None, :, None] * parts[2][None, None, :]
    return psi.astype(dtype)


def draw_trap(seed: int):
    """nu ~ U[0.5, 4] per axis, g ~ U[0, 500] (precision-form workload)."""
    rng = np.random.default_rng(seed)
    nu = rng.uniform(0.5, 4.0, size=3)
    g = rng.uniform(0.0, 500.0)
    return tuple(float(v) for v in nu), float(g)


def draw_batch(seed: int, n: int, dims=tuple(range(32, 97, 8)), dx=0.2):
    """n instances: dims per axis uniform over `dims`, nu ~ U[0.5, 4]^3,
    g log-uniform on [1, 1000]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx, ny, nz = (int(v) for v in rng.choice(np.asarray(dims), size=3))
        nu = rng.uniform(0.5, 4.0, size=3)
        g = math.exp(rng.uniform(math.log(1.0), math.log(1000.0)))
        out.append(dict(nx=nx, ny=ny, nz=nz, dx=dx, dy=dx, dz=dx, nux=float(nu[0]),
                        nuy=float(nu[1]), nuz=float(nu[2]), g=float(g), dt=0.1 * dx * dx))
    return out


def nn_init_weights(shapes, seed: int):
    """Initial network weights for a list of (name, shape): uniform He-style for weight
    tensors (fan-in = last dim, x27 for 3D convolution kernels named 'C...'), zero for
    biases (names starting with 'b' or 'c') and for the head ('wh', 'bh'), so that an
    untrained network returns exactly its analytic prior."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, shp in shapes:
        if name in ("wh", "bh") or name[0] in "bc":
            out[name] = np.zeros(shp)
            continue
        fan_in = shp[-1] * (27 if name[0] == "C" else 1)
        lim = math.sqrt(6.0 / fan_in)
        out[name] = rng.uniform(-lim, lim, size=shp)
    return out


def draw_nn_params(seed: int, n: int):
    """n problems (nu_x, nu_y, nu_z, g) distributed as the batched workload:
    nu ~ U[0.5, 4]^3, g log-uniform on [1, 1000]."""
    rng = np.random.default_rng(seed)
    nu = rng.uniform(0.5, 4.0, size=(n, 3))
    g = np.exp(rng.uniform(0.0, math.log(1000.0), size=(n, 1)))
    return np.concatenate([nu, g], axis=1)

