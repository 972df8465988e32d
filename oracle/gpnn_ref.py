"""FP64 CPU reference of the warm-start network: test infrastructure only.

Nothing in the product path imports this file; the tests compare the GPU kernels (BF16
operands, FP32 accumulation) with it.  It follows the definitions directly: each layer
is written from its mathematical definition with numpy (a matmul per tap for the
convolutions), the backward pass is the chain rule written out layer by layer, and Adam
is the published update (Kingma and Ba, Algorithm 1).

The network maps the trap and nonlinearity (nu_x, nu_y, nu_z, ln g) of one Gross-Pitaevskii
problem to a positive ground-state guess psi on the solver's grid (x_i = (i - (n-1)/2) dx):

    z0 = (p - mean) / std                                      4 inputs
    a1 = silu(W1 z0 + b1)                                      hidden
    a2 = silu(W2 a1 + b2), reshaped to [base]^3 x C0           channels last
    stage s = 1..S:  u = up2(a),  a = silu(conv3(u; Ws) + bs)  nearest x2, 3x3x3, zero pad
    f  = wh . a + bh + ln G(x; nu),  psi = exp(min(f, FMAX))
    ln G = 1/4 sum_a ln(nu_a / pi) - 1/2 sum_a nu_a x_a^2      (the trap's Gaussian ground
                                                                 state at g = 0)
Loss: L = (1/n) sum_samples dV sum_points (psi - target)^2.

Layouts: activations [n, D, D, D, C] (channels last); conv weights [27, Cout, Cin] with
tap t = (a*3 + b)*3 + c for the offset (a-1, b-1, c-1) along (x, y, z); dense weights
[Cout, Cin].  The convolution is a cross-correlation:
    y[p, o] = b[o] + sum_t sum_i W[t, o, i] x[p + off_t, i]   (x = 0 outside the grid)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FMAX = 10.0


@dataclass
class Arch:
    base: int = 4                     # edge of the first feature volume
    hidden: int = 384
    ch: tuple = (64, 64, 64, 32, 16)  # C0 (after the dense layers), then one per stage
    dx: float = 0.25
    in_mean: tuple = (2.25, 2.25, 2.25, 0.5 * math.log(1000.0))
    in_std: tuple = (3.5 / math.sqrt(12), 3.5 / math.sqrt(12), 3.5 / math.sqrt(12),
                     math.log(1000.0) / math.sqrt(12))

    @property
    def stages(self):
        return len(self.ch) - 1

    @property
    def n_out(self):
        return self.base * 2 ** self.stages


def param_shapes(a: Arch):
    """Ordered (name, shape) of every parameter."""
    out = [("W1", (a.hidden, 4)), ("b1", (a.hidden,)),
           ("W2", (a.base ** 3 * a.ch[0], a.hidden)), ("b2", (a.base ** 3 * a.ch[0],))]
    for s in range(1, a.stages + 1):
        out += [(f"C{s}", (27, a.ch[s], a.ch[s - 1])), (f"c{s}", (a.ch[s],))]
    out += [("wh", (a.ch[-1],)), ("bh", ())]
    return out


# ---------------------------------------------------------------- layers (definitions)
def silu(x):
    return x / (1.0 + np.exp(-x))


def silu_grad(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def _taps():
    return [(a - 1, b - 1, c - 1) for a in range(3) for b in range(3) for c in range(3)]


def _win(xp, off, dims):
    """Slice of a 1-padded volume: element p of the result is x[p + off]."""
    a, b, c = (o + 1 for o in off)
    return xp[:, a:a + dims[0], b:b + dims[1], c:c + dims[2], :]


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))


def conv3d(x, W, b=None):
    D = x.shape[1:4]
    xp = _pad(x)
    y = np.zeros(x.shape[:4] + (W.shape[1],))
    for t, off in enumerate(_taps()):
        y += _win(xp, off, D) @ W[t].T
    return y if b is None else y + b


def conv3d_bwd_data(dy, W):
    """dx[q] = sum_t W[t]^T dy[q - off_t]."""
    D = dy.shape[1:4]
    dyp = _pad(dy)
    dx = np.zeros(dy.shape[:4] + (W.shape[2],))
    for t, off in enumerate(_taps()):
        dx += _win(dyp, tuple(-o for o in off), D) @ W[t]
    return dx


def conv3d_bwd_weight(dy, x):
    """dW[t] = sum_p dy[p] x[p + off_t]^T."""
    D = x.shape[1:4]
    xp = _pad(x)
    dW = np.zeros((27, dy.shape[-1], x.shape[-1]))
    for t, off in enumerate(_taps()):
        dW[t] = np.einsum("ndhwo,ndhwi->oi", dy, _win(xp, off, D))
    return dW


def up2(x):
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def pool2_sum(g):
    n, D, _, _, C = g.shape
    return g.reshape(n, D // 2, 2, D // 2, 2, D // 2, 2, C).sum(axis=(2, 4, 6))


def grid_axis(n, dx):
    return (np.arange(n) - (n - 1) / 2.0) * dx


def log_prior(p, n, dx):
    """ln of the normalised anisotropic Gaussian, [batch, n, n, n]."""
    x = grid_axis(n, dx)
    nu = p[:, :3]
    lp = 0.25 * np.log(nu / math.pi).sum(axis=1)[:, None, None, None]
    lp = lp - 0.5 * (nu[:, 0, None, None, None] * x[None, :, None, None] ** 2
                     + nu[:, 1, None, None, None] * x[None, None, :, None] ** 2
                     + nu[:, 2, None, None, None] * x[None, None, None, :] ** 2)
    return lp


def features(p, a: Arch):
    """(nu_x, nu_y, nu_z, g) -> standardised (nu_x, nu_y, nu_z, ln g)."""
    q = np.array(p, dtype=np.float64).copy()
    q[:, 3] = np.log(q[:, 3])
    return (q - np.array(a.in_mean)) / np.array(a.in_std)


# ---------------------------------------------------------------- network
def forward(w: dict, p, a: Arch):
    """p: [batch, 4] raw (nu_x, nu_y, nu_z, g).  Returns psi [batch, n, n, n] and a cache."""
    p = np.asarray(p, dtype=np.float64)
    n = p.shape[0]
    cache = {"p": p}
    z0 = features(p, a)
    h1 = z0 @ w["W1"].T + w["b1"]
    a1 = silu(h1)
    h2 = a1 @ w["W2"].T + w["b2"]
    a2 = silu(h2).reshape(n, a.base, a.base, a.base, a.ch[0])
    cache.update(z0=z0, h1=h1, a1=a1, h2=h2)
    act = a2
    for s in range(1, a.stages + 1):
        u = up2(act)
        h = conv3d(u, w[f"C{s}"], w[f"c{s}"])
        cache[f"u{s}"], cache[f"h{s + 2}"] = u, h
        act = silu(h)
    cache["aL"] = act
    f = act @ w["wh"] + w["bh"] + log_prior(p, a.n_out, a.dx)
    psi = np.exp(np.minimum(f, FMAX))
    cache["f"], cache["psi"] = f, psi
    return psi, cache


def loss(psi, target, a: Arch):
    n = psi.shape[0]
    return float(((psi - target) ** 2).sum() * a.dx ** 3 / n)


def backward(w: dict, cache: dict, target, a: Arch):
    """Gradients of the loss with respect to every parameter (chain rule, layer by layer)."""
    psi, f = cache["psi"], cache["f"]
    n = psi.shape[0]
    g = {}
    dpsi = 2.0 * (psi - target) * a.dx ** 3 / n
    df = dpsi * psi * (f < FMAX)
    aL = cache["aL"]
    g["wh"] = np.einsum("ndhw,ndhwc->c", df, aL)
    g["bh"] = np.array(df.sum())
    dact = df[..., None] * w["wh"]
    for s in range(a.stages, 0, -1):
        dh = dact * silu_grad(cache[f"h{s + 2}"])
        g[f"C{s}"] = conv3d_bwd_weight(dh, cache[f"u{s}"])
        g[f"c{s}"] = dh.sum(axis=(0, 1, 2, 3))
        du = conv3d_bwd_data(dh, w[f"C{s}"])
        dact = pool2_sum(du)
    dh2 = dact.reshape(n, -1) * silu_grad(cache["h2"])
    g["W2"] = dh2.T @ cache["a1"]
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ w["W2"]) * silu_grad(cache["h1"])
    g["W1"] = dh1.T @ cache["z0"]
    g["b1"] = dh1.sum(axis=0)
    return g


def adam(wv, gv, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * gv
    v = b2 * v + (1 - b2) * gv * gv
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return wv - lr * mh / (np.sqrt(vh) + eps), m, v
