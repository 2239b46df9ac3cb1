"""Learned initial density (the machine-learned warm start of the SCF; the
paper's SCF starts from a superposition of atomic densities, Sec. 2.1, and
names machine-learning methods as a direction, Sec. 4): CPU reference of the
feature map, the three-layer periodic convolutional network, its gradient and
the Adam update.  Test infrastructure only: nothing in the GPU library or
its binding imports this module.

Network (float64 here; the GPU computes in float32):
    f_c(x)  = sum_I sum_images exp(-|x - R_I - n L|^2 / (2 w_c^2)),
              terms with |x - R_I - n L| <= 6 w_c, widths w = (0.5, 1.0, 2.0)
    a1 = relu(conv(W1, f) + b1)        3 -> 16 channels
    a2 = relu(conv(W2, a1) + b2)      16 -> 16
    z  = conv(W3, a2) + b3            16 -> 1
    s  = softplus(z),   rho = N_e s / (dV sum s)
    conv(W, u)[o, p] = sum_i sum_{k in {-1,0,1}^3} W[o, i, k] u[i, p + k]
    (cross-correlation with circular padding; tap index (kz, ky, kx) + 1).
Loss: mean over grid points of (rho - rho_target)^2.
Parameters are one flat vector: W1 (16,3,3,3,3), b1 (16), W2 (16,16,3,3,3),
b2 (16), W3 (1,16,3,3,3), b3 (1) -- 8673 values.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (0.5, 1.0, 2.0)
LAYERS = ((3, 16), (16, 16), (16, 1))
CUTOFF_WIDTHS = 6.0


def n_params() -> int:
    return sum(co * ci * 27 + co for ci, co in LAYERS)


def unpack(w: np.ndarray):
    """[(W (co, ci, 3, 3, 3), b (co,)), ...] views of the flat vector."""
    out, o = [], 0
    for ci, co in LAYERS:
        W = w[o:o + co * ci * 27].reshape(co, ci, 3, 3, 3)
        o += co * ci * 27
        b = w[o:o + co]
        o += co
        out.append((W, b))
    return out


def features(sys, widths=WIDTHS) -> np.ndarray:
    """(3, Nz, Ny, Nx) Gaussian features of the atoms."""
    nx, ny, nz = sys.n
    hx, hy, hz = sys.h
    Lx, Ly, Lz = sys.L
    X = np.arange(nx) * hx
    Y = np.arange(ny) * hy
    Z = np.arange(nz) * hz
    out = np.zeros((len(widths), nz, ny, nx))
    for c, w in enumerate(widths):
        rcut = CUTOFF_WIDTHS * w
        for R in sys.pos:
            ks = [range(-int(np.ceil((rcut + L) / L)), int(np.ceil((rcut + L) / L)) + 1) for L in (Lx, Ly, Lz)]
            for a in ks[0]:
                for b in ks[1]:
                    for cc in ks[2]:
                        dx = X - R[0] - a * Lx
                        dy = Y - R[1] - b * Ly
                        dz = Z - R[2] - cc * Lz
                        r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
                        out[c] += np.where(r2 <= rcut * rcut, np.exp(-r2 / (2 * w * w)), 0.0)
    return out


def conv(W: np.ndarray, u: np.ndarray, b=None) -> np.ndarray:
    """Circular cross-correlation: u (ci, Nz, Ny, Nx) -> (co, Nz, Ny, Nx)."""
    co = W.shape[0]
    out = np.zeros((co,) + u.shape[1:])
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                # shifted[i, p] = u[i, p + k]
                sh = np.roll(u, shift=(-(kz - 1), -(ky - 1), -(kx - 1)), axis=(1, 2, 3))
                out += np.tensordot(W[:, :, kz, ky, kx], sh, axes=(1, 0))
    if b is not None:
        out += b[:, None, None, None]
    return out


def conv_transpose(W: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Adjoint of conv in its input: g (co, ...) -> (ci, ...),
    out[i, p] = sum_o sum_k W[o, i, k] g[o, p - k]."""
    ci = W.shape[1]
    out = np.zeros((ci,) + g.shape[1:])
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                sh = np.roll(g, shift=(kz - 1, ky - 1, kx - 1), axis=(1, 2, 3))
                out += np.tensordot(W[:, :, kz, ky, kx].T, sh, axes=(1, 0))
    return out


def conv_weight_grad(u: np.ndarray, g: np.ndarray) -> np.ndarray:
    """dW[o, i, k] = sum_p g[o, p] u[i, p + k]."""
    co, ci = g.shape[0], u.shape[0]
    dW = np.zeros((co, ci, 3, 3, 3))
    gf = g.reshape(co, -1)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                sh = np.roll(u, shift=(-(kz - 1), -(ky - 1), -(kx - 1)), axis=(1, 2, 3)).reshape(ci, -1)
                dW[:, :, kz, ky, kx] = gf @ sh.T
    return dW


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(sys, w: np.ndarray, f: np.ndarray):
    """Returns (rho (Nz, Ny, Nx), cache)."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(w)
    a1 = np.maximum(conv(W1, f, b1), 0.0)
    a2 = np.maximum(conv(W2, a1, b2), 0.0)
    z = conv(W3, a2, b3)[0]
    s = softplus(z)
    S = s.sum()
    rho = sys.n_electrons * s / (sys.dV * S)
    return rho, dict(f=f, a1=a1, a2=a2, z=z, s=s, S=S)


def loss(rho, target) -> float:
    return float(np.mean((rho - target) ** 2))


def backward(sys, w: np.ndarray, rho, target, cache) -> np.ndarray:
    """Gradient of loss(forward(w), target) with respect to the flat w."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(w)
    f, a1, a2, z, s, S = (cache[k] for k in ("f", "a1", "a2", "z", "s", "S"))
    g = 2.0 * (rho - target) / rho.size             # dL/drho
    c = sys.n_electrons / (sys.dV * S)               # rho = c s
    ds = c * g - (c / S) * np.sum(g * s)
    dz = (ds * sigmoid(z))[None]
    dW3 = conv_weight_grad(a2, dz)
    db3 = dz.sum(axis=(1, 2, 3))
    d2 = conv_transpose(W3, dz) * (a2 > 0)
    dW2 = conv_weight_grad(a1, d2)
    db2 = d2.sum(axis=(1, 2, 3))
    d1 = conv_transpose(W2, d2) * (a1 > 0)
    dW1 = conv_weight_grad(f, d1)
    db1 = d1.sum(axis=(1, 2, 3))
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])


def adam(w, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba): returns new (w, m, v); t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def l1_distance(sys, a, b) -> float:
    """dV sum |a - b| / N_e (fallback test of the predicted density)."""
    return float(sys.dV * np.sum(np.abs(a - b)) / sys.n_electrons)
