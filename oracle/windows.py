"""Alternative weight functions (Section 4.3).  TEST INFRASTRUCTURE.

Section 2.2 builds the weight as the inverse cosine transform of a target
function on the frequency axis (eq. filterf with the indicator of
[omega_min, omega_max]) truncated to [0, T] (eq. weightf); with

    alpha(t) = (2/pi) * integral_0^inf g(omega) cos(omega t) d omega

the filter beta(omega) = integral_0^inf alpha(t) cos(omega t) dt returns g.
Section 4.3 names smoother or more localised targets (a triangle impulse, a
Gaussian peak) and weights adapted to the spectrum, whose filter is small
where unwanted eigenvalues of high multiplicity are expected.

Targets here, with centre c = (omega_min + omega_max)/2, half-width
d = (omega_max - omega_min)/2 and a width factor s > 0:

* ``indicator``: g = 1 on [omega_min, omega_max] (eq. weightf);
* ``triangle``: g(omega) = T(omega - c) + T(omega + c) with
  T(u) = max(0, 1 - |u|/h), h = s*d (s = 2: g = 1/2 at the interval ends);
* ``gaussian``: g(omega) = G(omega - c) + G(omega + c) with
  G(u) = exp(-u^2 / (2 sigma^2)), sigma = s*d / sqrt(2 ln 2) (s = 1: g = 1/2
  at the interval ends).

The mirrored second term makes g the restriction of an even function, so the
integral has a closed form; it only matters when the peak reaches omega = 0.
The rectangle rule then gives w_l = tau*alpha(l*tau), l < L (eq.
disc_filtercoeff).

``notch_weights`` is the spectrum-adapted form: the smallest change of given
weights w (in the 2-norm) after which the discrete filter of Lemma 2.3
vanishes at the given frequencies, beta~(omega_j) = sum_l w_l q_l(omega_j) = 0.
"""

from __future__ import annotations

import math

import numpy as np

from .filter import q_sequence

KINDS = ("indicator", "triangle", "gaussian")


def alpha_window(t, kind: str, omega_min: float, omega_max: float, width: float = 1.0):
    """alpha(t) for the target ``kind`` (untruncated)."""
    t = np.asarray(t, dtype=np.float64)
    c = 0.5 * (omega_min + omega_max)
    d = 0.5 * (omega_max - omega_min)
    if kind == "indicator":
        out = np.empty_like(t)
        z = t == 0.0
        out[z] = 2.0 * (omega_max - omega_min) / math.pi
        tz = t[~z]
        out[~z] = 2.0 / math.pi * (np.sin(omega_max * tz) - np.sin(omega_min * tz)) / tz
        return out
    if kind == "triangle":
        h = width * d
        # integral over the triangle of cos(omega t) = h cos(c t) sinc^2(h t / 2)
        x = 0.5 * h * t
        sinc = np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))
        return 2.0 / math.pi * h * np.cos(c * t) * sinc**2
    if kind == "gaussian":
        sigma = width * d / math.sqrt(2.0 * math.log(2.0))
        return 2.0 / math.pi * sigma * math.sqrt(2.0 * math.pi) * np.exp(-0.5 * (sigma * t) ** 2) * np.cos(c * t)
    raise ValueError(f"unknown window {kind!r}")


def target(omega, kind: str, omega_min: float, omega_max: float, width: float = 1.0):
    """The target function g(omega) whose transform alpha_window is."""
    om = np.asarray(omega, dtype=np.float64)
    c = 0.5 * (omega_min + omega_max)
    d = 0.5 * (omega_max - omega_min)
    if kind == "indicator":
        return ((om >= omega_min) & (om <= omega_max)).astype(float)
    if kind == "triangle":
        h = width * d
        return np.maximum(0.0, 1.0 - np.abs(om - c) / h) + np.maximum(0.0, 1.0 - np.abs(om + c) / h)
    if kind == "gaussian":
        sigma = width * d / math.sqrt(2.0 * math.log(2.0))
        return np.exp(-0.5 * ((om - c) / sigma) ** 2) + np.exp(-0.5 * ((om + c) / sigma) ** 2)
    raise ValueError(f"unknown window {kind!r}")


def window_weights(kind: str, omega_min: float, omega_max: float, tau: float, L: int, width: float = 1.0):
    """w_l = tau * alpha(l tau), l = 0..L-1 (alpha truncated at T = L tau)."""
    if L < 1 or tau <= 0:
        raise ValueError("need L >= 1 and tau > 0")
    return tau * alpha_window(np.arange(L) * tau, kind, omega_min, omega_max, width)


def notch_weights(w, tau: float, omegas) -> np.ndarray:
    """argmin ||w' - w||_2 subject to beta~(omega_j) = 0 for every j."""
    w = np.asarray(w, dtype=np.float64)
    Q = q_sequence(np.asarray(omegas, dtype=np.float64), tau, w.size).T  # k x L, Q[j, l] = q_l(omega_j)
    # the projection of w onto the null space of Q
    coef = np.linalg.solve(Q @ Q.T, Q @ w)
    return w - Q.T @ coef
