"""The operator C of Section 2.3 (eq. 2stepmethod, eq. disc_filtercoeff),
applied exactly as the time loop of Algorithm 2.5 does it.

For a start vector r (or a block of them, one per column):

    y_{-1} = y_0 = r
    y_{l+1} = -tau^2 M^{-1} S y_l + 2 y_l - y_{l-1}
    C r = sum_{l=0}^{L-1} w_l y_l,      w_l = tau*alpha(l*tau)

M is diagonal (lumped), given as the vector m.  L-1 products with S.
"""

from __future__ import annotations

import numpy as np


def apply_filter(S, m: np.ndarray, tau: float, w: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Return C r for a vector (N,) or block (N, b), in float64."""
    r = np.asarray(r, dtype=np.float64)
    minv = 1.0 / np.asarray(m, dtype=np.float64)
    if r.ndim == 2:
        minv = minv[:, None]
    y_old = r.copy()  # y_{l-1}
    y_cur = r.copy()  # y_l
    acc = w[0] * y_cur  # first term of the rectangle rule
    for ell in range(1, len(w)):
        y_new = -tau * tau * (minv * (S @ y_cur)) + 2.0 * y_cur - y_old
        acc = acc + w[ell] * y_new
        y_old, y_cur = y_cur, y_new
    return acc
