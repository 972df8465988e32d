"""Residual of the stationary Gross-Pitaevskii equation on the grid, FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package header).  For a state psi on the grid
x_i = (i - (n-1)/2) dx with zero values outside (the Dirichlet ghosts of the solver), the
normalised state phi = psi / sqrt(N), N = dx dy dz sum |psi|^2, and the discrete operator
H[phi] = -1/2 lap_h + V + g |phi|^2 with the 3-point Laplacian along each axis,

    mu  = <phi, H[phi] phi>,      res = || H[phi] phi - mu phi ||,

inner products dx dy dz sum conj(a) b.  res is zero exactly when phi is a stationary
state of the discrete equation (the fixed point imaginary-time propagation approaches as
dt -> 0).  Written directly from the definition: apply H by shifted copies, then take
the inner products.
"""
from __future__ import annotations

import numpy as np


def apply_h(phi, prm):
    d = (prm["dx"], prm["dy"], prm["dz"])
    nu = (prm["nux"], prm["nuy"], prm["nuz"])
    out = np.zeros_like(phi)
    for a in range(3):
        n = phi.shape[a]
        x = (np.arange(n) - (n - 1) / 2.0) * d[a]
        shape = [1, 1, 1]
        shape[a] = n
        out += 0.5 * (nu[a] ** 2) * (x ** 2).reshape(shape) * phi
        pad = [(0, 0)] * 3
        pad[a] = (1, 1)
        pp = np.pad(phi, pad)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[a] = slice(0, n)
        hi[a] = slice(2, n + 2)
        out -= 0.5 * (pp[tuple(lo)] + pp[tuple(hi)] - 2.0 * phi) / d[a] ** 2
    return out + prm["g"] * np.abs(phi) ** 2 * phi


def residual(psi, prm):
    """(res, mu) of psi (any normalisation) for the parameters prm."""
    psi = np.asarray(psi, dtype=np.complex128)
    dV = prm["dx"] * prm["dy"] * prm["dz"]
    phi = psi / np.sqrt(dV * np.sum(np.abs(psi) ** 2))
    hphi = apply_h(phi, prm)
    mu = float(np.real(dV * np.sum(np.conj(phi) * hphi)))
    r = hphi - mu * phi
    return float(np.sqrt(dV * np.sum(np.abs(r) ** 2))), mu
