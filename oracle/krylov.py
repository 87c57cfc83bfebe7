"""Krylov loop, projection and acceptance (Section 2.1 eq. projevp;
Algorithm 2.5; Section 2.4 eq. res and the stopping rule after it).

Two forms of the Krylov loop:

``krylov_basis_euclidean``  an orthonormal basis, in the Euclidean inner
    product, of the Krylov space K_m(C, r_0) of Section 2.1 (def. ArnoldiEWP),
    the orthogonalisation the paper uses; a column that vanishes ends the
    space (it is invariant).  Used by the tests to show that the projected
    pencil does not depend on the choice of basis.

``krylov_solve``  the form the GPU library computes (readings of the paper
    are listed in the design notes):
    * block of b start vectors (the block Krylov remedy of the outlook);
    * orthogonalisation in the M inner product, classical Gram-Schmidt applied
      twice against the basis, then twice against the already kept columns of
      the same block, column by column;
    * a column whose M-norm after orthogonalisation is at most
      ``drop_tol`` times its M-norm before it is dropped (breakdown, the
      "exact eigenspace found" branch with a tolerance); when a whole block is
      dropped the loop stops;
    * every ``check_every`` iterations: the projected pencil
      H = B^T S B, G = B^T M B is solved (scipy.linalg.eigh), Ritz values with
      omega in [omega_min, omega_max] get Ritz vectors v = B y and residuals
      ||S v - omega^2 M v||_2 / ||S v||_2; those at or below ``tol`` are
      accepted;
    * stop when ``target`` pairs are accepted, the basis reaches ``m_max``
      columns, or breakdown.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .timestep import apply_filter


@dataclass
class KrylovResult:
    omega2: np.ndarray
    omega: np.ndarray
    residual: np.ndarray
    vectors: np.ndarray | None
    ritz: np.ndarray
    krylov_steps: int
    basis_size: int
    leapfrog_vector_steps: int  # sum over filter applications of b*(L-1)
    breakdown: bool
    basis: np.ndarray | None = None
    history: list = field(default_factory=list)


def krylov_basis_euclidean(S, m, tau, w, r0, mdim):
    """Euclidean-orthonormal basis of K_mdim(C, r0) (Section 2.1): column k+1
    is C applied to column k with its components along the earlier columns
    removed one at a time (modified Gram-Schmidt), then scaled to unit 2-norm.
    Fewer than mdim columns when the space becomes invariant (a zero column)."""
    columns = [np.asarray(r0, dtype=np.float64) / np.linalg.norm(r0)]
    while len(columns) < mdim:
        v = apply_filter(S, m, tau, w, columns[-1])
        for q in columns:
            v = v - (q @ v) * q
        length = np.linalg.norm(v)
        if length == 0.0:
            break
        columns.append(v / length)
    return np.column_stack(columns)


def _orthonormalize_block(X, m, B, ref, drop_tol):
    """CGS2 of the columns of X against B (M inner product), then column by
    column CGS2 against the kept columns of the block, normalisation, and the
    relative drop test.  Returns the kept columns (N x k)."""
    X = X.copy()
    if B is not None and B.shape[1] > 0:
        for _ in range(2):
            X = X - B @ (B.T @ (m[:, None] * X))
    kept = []
    for j in range(X.shape[1]):
        x = X[:, j]
        if kept:
            Q = np.column_stack(kept)
            for _ in range(2):
                x = x - Q @ (Q.T @ (m * x))
        nrm = math.sqrt(max(float(x @ (m * x)), 0.0))
        if nrm <= drop_tol * ref[j] or nrm == 0.0:
            continue
        kept.append(x / nrm)
    if not kept:
        return np.zeros((X.shape[0], 0))
    return np.column_stack(kept)


def _m_norms(X, m):
    return np.sqrt(np.maximum(np.einsum("ij,ij->j", X, m[:, None] * X), 0.0))


def rayleigh_ritz(S, m, B, omega_min, omega_max, want_vectors=True):
    """Projected pencil of eq. projevp on span(B), Ritz values, and for the
    Ritz values in the interval their Ritz vectors and relative residuals.

    Returns (theta_all, theta_c, res_c, V_c) with theta_c ascending."""
    SB = S @ B
    H = B.T @ SB
    G = B.T @ (m[:, None] * B)
    H = 0.5 * (H + H.T)
    G = 0.5 * (G + G.T)
    theta, Y = sla.eigh(H, G)
    om = np.sqrt(np.maximum(theta, 0.0))
    sel = (om >= omega_min) & (om <= omega_max)
    th_c = theta[sel]
    Yc = Y[:, sel]
    V = B @ Yc
    SV = SB @ Yc
    MV = m[:, None] * V
    num = np.linalg.norm(SV - MV * th_c[None, :], axis=0)
    den = np.linalg.norm(SV, axis=0)
    den = np.where(den > 0.0, den, np.maximum(np.abs(th_c) * np.linalg.norm(MV, axis=0), 1e-300))
    res = num / den
    return theta, th_c, res, (V if want_vectors else None)


def krylov_solve(
    S,
    m,
    tau,
    w,
    V0,
    omega_min,
    omega_max,
    tol=1e-9,
    m_max=200,
    target=None,
    check_every=1,
    drop_tol=1e-10,
    max_iters=None,
    keep_basis=False,
    want_vectors=False,
):
    """Block Krylov eigensolver with the filtered time-domain operator C.

    V0 is the N x b start block (row-major float64), the same numbers the GPU
    path receives.  ``max_iters`` caps the number of filter applications
    (Krylov iterations); ``m_max`` caps the basis size.
    """
    m = np.asarray(m, dtype=np.float64)
    V0 = np.asarray(V0, dtype=np.float64)
    if V0.ndim == 1:
        V0 = V0[:, None]
    L = len(w)
    B = _orthonormalize_block(V0, m, None, _m_norms(V0, m), drop_tol)
    Q = B
    iters = 0
    lf_steps = 0
    breakdown = B.shape[1] == 0
    history = []
    last = None

    def check():
        theta, th_c, res, V = rayleigh_ritz(S, m, B, omega_min, omega_max, want_vectors)
        acc = res <= tol
        history.append((B.shape[1], int(acc.sum())))
        return theta, th_c[acc], res[acc], (V[:, acc] if V is not None else None)

    while not breakdown:
        if max_iters is not None and iters >= max_iters:
            break
        if B.shape[1] >= m_max:
            break
        R = apply_filter(S, m, tau, w, Q)
        iters += 1
        lf_steps += Q.shape[1] * (L - 1)
        ref = _m_norms(R, m)
        Qn = _orthonormalize_block(R, m, B, ref, drop_tol)
        room = m_max - B.shape[1]
        Qn = Qn[:, :room]
        if Qn.shape[1] == 0:
            breakdown = True
            break
        B = np.column_stack([B, Qn])
        Q = Qn
        if iters % check_every == 0:
            last = check()
            if target is not None and last[1].size >= target:
                break
    if last is None or history[-1][0] != B.shape[1]:
        last = check()
    theta, th, res, V = last
    return KrylovResult(
        omega2=th,
        omega=np.sqrt(np.maximum(th, 0.0)),
        residual=res,
        vectors=V,
        ritz=theta,
        krylov_steps=iters,
        basis_size=B.shape[1],
        leapfrog_vector_steps=lf_steps,
        breakdown=breakdown,
        basis=B if keep_basis else None,
        history=history,
    )
