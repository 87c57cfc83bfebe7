"""Fixed-dimension filtered subspace iteration (Section 4.4: instead of a
growing Krylov space, a space of fixed dimension, which makes the method a
FEAST-type algorithm with the time-domain filter).  TEST INFRASTRUCTURE.

One iteration, for a block X of p columns:

1. Q = C X, the operator C of Section 2.3 applied to every column;
2. Q is M-orthonormalised (classical Gram-Schmidt twice in the M inner
   product, a column losing all but ``drop_tol`` of its M-norm is dropped);
3. the pencil is projected onto span(Q) as in eq. projevp,
   H = Q^T S Q, G = Q^T M Q, and solved (scipy.linalg.eigh);
4. X <- Q Y, all Ritz vectors (the dimension stays p unless columns were
   dropped);
5. Ritz values with omega in [omega_min, omega_max] get residuals as in
   eq. res, relative to ||S v||_2; those at or below tol are accepted.

The iteration stops when ``target`` pairs are accepted, when every Ritz value
in the interval is accepted (target = 0), or after ``max_iters`` iterations.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .krylov import _m_norms, _orthonormalize_block
from .timestep import apply_filter


@dataclass
class SubspaceResult:
    omega2: np.ndarray
    residual: np.ndarray
    ritz: np.ndarray
    iterations: int
    dimension: int
    history: list = field(default_factory=list)  # (iteration, accepted count)
    block: np.ndarray | None = None


def subspace_solve(S, m, tau, w, X0, omega_min, omega_max, tol=1e-9, max_iters=20, target=0, drop_tol=1e-10,
                   keep_block=False):
    m = np.asarray(m, dtype=np.float64)
    X = np.asarray(X0, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    history = []
    theta = th_c = res = np.zeros(0)
    it = 0
    while it < max_iters:
        Q = apply_filter(S, m, tau, w, X)
        it += 1
        Q = _orthonormalize_block(Q, m, None, _m_norms(Q, m), drop_tol)
        if Q.shape[1] == 0:
            break
        SQ = S @ Q
        H = Q.T @ SQ
        G = Q.T @ (m[:, None] * Q)
        theta, Y = sla.eigh(0.5 * (H + H.T), 0.5 * (G + G.T))
        X = Q @ Y
        om = np.sqrt(np.maximum(theta, 0.0))
        inside = (om >= omega_min) & (om <= omega_max)
        th_c = theta[inside]
        V = X[:, inside]
        SV = SQ @ Y[:, inside]
        num = np.linalg.norm(SV - (m[:, None] * V) * th_c[None, :], axis=0)
        den = np.linalg.norm(SV, axis=0)
        den = np.where(den > 0.0, den, np.maximum(np.abs(th_c) * np.linalg.norm(m[:, None] * V, axis=0), 1e-300))
        res = num / den
        acc = int(np.count_nonzero(res <= tol))
        history.append((it, acc))
        if (target > 0 and acc >= target) or (target <= 0 and th_c.size > 0 and acc == th_c.size):
            break
    keep = res <= tol
    return SubspaceResult(
        omega2=th_c[keep],
        residual=res[keep],
        ritz=theta,
        iterations=it,
        dimension=X.shape[1],
        history=history,
        block=X if keep_block else None,
    )
