"""The operator C of Section 2.3, from its definition (eq. 2stepmethod and
eq. disc_filtercoeff).

For a start vector r (or a block of them, one per column) the explicit
two-step scheme defines the sequence

    y_{-1} = y_0 = r,
    y_{l+1} = -tau^2 M^{-1} S y_l + 2 y_l - y_{l-1},

and the rectangle rule with nodes l*tau, l = 0..L-1, defines

    C r = sum_{l=0}^{L-1} w_l y_l,      w_l = tau*alpha(l*tau).

M is diagonal (lumped), given as the vector m.  Forming y_0 .. y_{L-1}
takes L-1 products with S.

Remark 2.4 and Section 4.2 allow any explicit scheme whose iteration matrix
is a function of M^{-1} S (so that the pencil's eigenvectors stay those of
C), naming high-order variants of leapfrog.  ``order=4`` selects the
fourth-order two-step scheme obtained by adding the next term of the
expansion of cos(tau sqrt(M^{-1} S)):

    y_{l+1} = 2 y_l - y_{l-1} - tau^2 M^{-1} S y_l + (tau^4 / 12) (M^{-1} S)^2 y_l,

two products with S per step, same start values and weights.
"""

from __future__ import annotations

import numpy as np


def leapfrog_sequence(S, m: np.ndarray, tau: float, r: np.ndarray, count: int, order: int = 2):
    """Yield y_0, y_1, ..., y_{count-1} of the two-step scheme (order 2:
    eq. 2stepmethod; order 4: with the tau^4 term) started from
    y_{-1} = y_0 = r (float64)."""
    if order not in (2, 4):
        raise ValueError("order must be 2 or 4")
    r = np.asarray(r, dtype=np.float64)
    minv = 1.0 / np.asarray(m, dtype=np.float64)
    if r.ndim == 2:
        minv = minv[:, None]
    y_before = r.copy()  # y_{-1}
    y_now = r.copy()  # y_0
    for ell in range(count):
        yield y_now
        if ell + 1 < count:
            a_y = tau * tau * (minv * (S @ y_now))  # tau^2 M^{-1} S y_l
            y_next = 2.0 * y_now - y_before - a_y
            if order == 4:
                y_next = y_next + (tau * tau * (minv * (S @ a_y))) / 12.0
            y_before, y_now = y_now, y_next


def apply_filter(S, m: np.ndarray, tau: float, w: np.ndarray, r: np.ndarray, order: int = 2) -> np.ndarray:
    """Return C r = sum_l w_l y_l for a vector (N,) or block (N, b), in float64."""
    w = np.asarray(w, dtype=np.float64)
    total = np.zeros(np.shape(r), dtype=np.float64)
    for ell, y in enumerate(leapfrog_sequence(S, m, tau, r, len(w), order)):
        total = total + w[ell] * y
    return total
