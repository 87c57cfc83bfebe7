"""FP64 reference of the learned filter-weight network (test infrastructure).

The weight function is free (Section 2.2: the method is not tied to the
weight of eq. weightf; Section 2.2 also states the design goal
|beta(omega)| >> |beta(omega~)| for sought omega and unsought omega~).  In the
normalised variable x = tau*omega/2 the whole design depends on tau only
through products with tau:

* q_l(omega) = cos((l + 1/2) phi) / cos(phi/2) with phi = 2 arcsin(x)
  (the scalar recurrence of Section 2.3 solved in closed form);
* the Fourier weights w_l = tau*alpha(l*tau) of eq. weightf are
  w_0 = 2(c - a)/pi, w_l = 4/(pi l) sin(l(c - a)/2) cos(l(c + a)/2) with
  a = tau*omega_min, c = tau*omega_max, for l < L.

Network: features f = [a/pi, c/pi, x_max, L/512] (x_max = tau*sqrt(lambda_max)/2),
three GELU layers of width 128 and a linear output of 512 values;
w = w_Fourier + s * out (masked to l < L), s = 0.01, so the untrained
network (output layer at zero) reproduces the Fourier weights.  The parameter
vector stores the first layer in a 64 x 128 slot of which the rows of the four
features are used (the rest multiplies nothing and gets a zero gradient).

Precision: by default every product is float64.  With ``bf16=True`` the
operands of the network's matrix products (the four layers forward, and the
weight-gradient and back-propagation products) are first rounded to bfloat16
(round to nearest, ties to even), the stated training precision of the
learned filter (bfloat16 operands, wider accumulation); everything else
stays float64.

Loss per sample on the fixed grid x_g = 0.95 g / (G-1), g < G:
J = mean over the band [x_lo, x_hi] of (beta~ - 1)^2
  + gamma * mean over {x <= x_max, x outside [x_lo - d, x_hi + d]} of beta~^2,
d = pi / (2 L), gamma = 1 (the quadratic leakage criterion; the transition
band is half of one main-lobe width of an L-term filter).
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from synth import netinit

HIDDEN = 128
LMAX = 512
G = 512
XMAX_GRID = 0.95
OUT_SCALE = 0.01
GAMMA = 1.0
NFEAT = 4
SHAPES = [(64, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, LMAX), (LMAX,)]


def n_params() -> int:
    return int(sum(np.prod(s) for s in SHAPES))


def unpack(theta: np.ndarray):
    out, off = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(theta[off : off + k].reshape(s))
        off += k
    return out


def x_grid() -> np.ndarray:
    return XMAX_GRID * np.arange(G) / (G - 1)


def q_matrix() -> np.ndarray:
    """Q[l, g] = q_l at x_g (closed form of the scalar recurrence)."""
    phi = 2.0 * np.arcsin(x_grid())
    ell = np.arange(LMAX)[:, None]
    return np.cos((ell + 0.5) * phi[None, :]) / np.cos(0.5 * phi[None, :])


def sample_params(omega_min, omega_max, tau, lambda_max):
    a, c = tau * omega_min, tau * omega_max
    L = int(math.ceil(2.0 * math.pi / a))
    xm = 0.5 * tau * math.sqrt(lambda_max)
    return a, c, L, xm


def features(omega_min, omega_max, tau, lambda_max) -> np.ndarray:
    a, c, L, xm = sample_params(omega_min, omega_max, tau, lambda_max)
    return np.array([a / math.pi, c / math.pi, xm, L / LMAX])


def bf16_round(x) -> np.ndarray:
    """Nearest bfloat16 value (8 significant bits, ties to even) of each
    entry, as float64; the entries are first taken to float32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(A, B, bf16):
    """Matrix product of the network, with bfloat16 operands when asked."""
    return (bf16_round(A) @ bf16_round(B)) if bf16 else A @ B


def fourier_weights_normalised(a: float, c: float, L: int) -> np.ndarray:
    w = np.zeros(LMAX)
    ell = np.arange(1, L)
    w[0] = 2.0 * (c - a) / math.pi
    w[1:L] = 4.0 / (math.pi * ell) * np.sin(0.5 * ell * (c - a)) * np.cos(0.5 * ell * (c + a))
    return w


def masks(a: float, c: float, L: int, xm: float):
    x = x_grid()
    lo, hi = 0.5 * a, 0.5 * c
    d = math.pi / (2.0 * L)
    inb = (x >= lo) & (x <= hi)
    outb = (x <= xm) & ((x < lo - d) | (x > hi + d))
    return inb.astype(float), outb.astype(float)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, samples, bf16=False):
    """samples: (B, 4) rows (omega_min, omega_max, tau, lambda_max).
    Returns (weights (B, LMAX), loss per sample (B,), cache)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    X = np.stack([features(*s) for s in samples])
    prm = [sample_params(*s) for s in samples]
    z1 = _mm(X, W1[:NFEAT], bf16) + b1
    h1 = gelu(z1)
    z2 = _mm(h1, W2, bf16) + b2
    h2 = gelu(z2)
    z3 = _mm(h2, W3, bf16) + b3
    h3 = gelu(z3)
    out = _mm(h3, W4, bf16) + b4
    lmask = np.stack([(np.arange(LMAX) < L).astype(float) for (_a, _c, L, _x) in prm])
    wF = np.stack([fourier_weights_normalised(a, c, L) for (a, c, L, _x) in prm])
    w = (wF + OUT_SCALE * out) * lmask
    Q = q_matrix()
    beta = w @ Q
    mi = np.stack([masks(a, c, L, x)[0] for (a, c, L, x) in prm])
    mo = np.stack([masks(a, c, L, x)[1] for (a, c, L, x) in prm])
    ni = np.maximum(mi.sum(1), 1.0)
    no = np.maximum(mo.sum(1), 1.0)
    J = (mi * (beta - 1.0) ** 2).sum(1) / ni + GAMMA * (mo * beta**2).sum(1) / no
    cache = dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, lmask=lmask, beta=beta, mi=mi, mo=mo, ni=ni, no=no,
                 Q=Q)
    return w, J, cache


def loss_and_grad(theta, samples, bf16=False):
    """Mean loss over the batch and its gradient (backpropagation)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    w, J, c = forward(theta, samples, bf16)
    B = len(samples)
    dbeta = (2.0 * c["mi"] * (c["beta"] - 1.0) / c["ni"][:, None] + 2.0 * GAMMA * c["mo"] * c["beta"] / c["no"][:, None]) / B
    dw = (dbeta @ c["Q"].T) * c["lmask"]
    dout = OUT_SCALE * dw
    gW4 = _mm(c["h3"].T, dout, bf16)
    gb4 = dout.sum(0)
    dz3 = _mm(dout, W4.T, bf16) * gelu_grad(c["z3"])
    gW3 = _mm(c["h2"].T, dz3, bf16)
    gb3 = dz3.sum(0)
    dz2 = _mm(dz3, W3.T, bf16) * gelu_grad(c["z2"])
    gW2 = _mm(c["h1"].T, dz2, bf16)
    gb2 = dz2.sum(0)
    dz1 = _mm(dz2, W2.T, bf16) * gelu_grad(c["z1"])
    gW1 = np.zeros_like(W1)
    gW1[:NFEAT] = _mm(c["X"].T, dz1, bf16)
    gb1 = dz1.sum(0)
    grad = np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])
    return float(J.mean()), grad


def init_params(seed: int) -> np.ndarray:
    """The seeded initial parameters (drawn by the shared input generator)."""
    return netinit.init_params(seed, SHAPES)


def teacher(sample, ridge: float = 1e-6) -> np.ndarray:
    """Per-sample optimum of the quadratic loss over the L free weights
    (ridge least squares): the lower bound the network is measured against."""
    a, c, L, xm = sample_params(*sample)
    Q = q_matrix()[:L]
    mi, mo = masks(a, c, L, xm)
    ni, no = max(mi.sum(), 1.0), max(mo.sum(), 1.0)
    Wd = mi / ni + GAMMA * mo / no
    A = (Q * Wd[None, :]) @ Q.T + ridge * np.eye(L)
    rhs = Q @ (mi / ni)
    w = np.zeros(LMAX)
    w[:L] = np.linalg.solve(A, rhs)
    return w


def loss_of_weights(sample, w) -> float:
    a, c, L, xm = sample_params(*sample)
    beta = w @ q_matrix()
    mi, mo = masks(a, c, L, xm)
    return float((mi * (beta - 1) ** 2).sum() / max(mi.sum(), 1) + GAMMA * (mo * beta**2).sum() / max(mo.sum(), 1))
