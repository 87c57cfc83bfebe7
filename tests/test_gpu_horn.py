"""The horn (Neumann, jittered P1, clustered eigenvalues) with blocks of 16
Krylov vectors: float32 stepping with float64 projection, and float64.

* small horn (4 x 4 cross-section cells, 60 layers, 1,525 DOFs): every
  eigenvalue of the pencil in the interval, from a dense generalized
  eigensolve (the plain definition), is found;
* 16 x 200 horn (58,089 DOFs, L = 448 steps): the block filter equals the
  oracle's;
* the full horn (752,845 DOFs, 4.0 M tetrahedra): properties that hold at
  any size -- the constants are the omega = 0 eigenvector, so C 1 =
  beta~(0) 1; C is M-self-adjoint.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from synth import power_start, start_block
from synth.horn import horn_pencil, horn_problem

pytestmark = pytest.mark.gpu


def _kf():
    from paper_2402_08515_amd import kf

    return kf


@pytest.fixture(scope="module")
def small_horn():
    S, m = horn_pencil(4, 60)
    lam = sl.eigh(S.toarray(), np.diag(m), eigvals_only=True)
    lmax = oracle.power_lambda_max(S, m, power_start(S.shape[0], 2), 30)
    return S, m, lam, lmax


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_small_horn_block16_finds_every_eigenvalue(small_horn, precision, bar):
    kf = _kf()
    S, m, lam, lmax = small_horn
    lo, hi = 200.0, 260.0
    ref = lam[(lam >= lo**2) & (lam <= hi**2)]
    tau, L = oracle.time_step_rule(lmax, lo)
    print(f"case small horn {precision} b=16 target={ref.size} L={L}", flush=True)
    # checks every second step (no growth wait): the basis limit of 600 columns
    # is tight for the float32 loop on this clustered spectrum
    prob = kf.Problem(S, m, lo, hi, tau, L, precision=precision, target=int(ref.size), check_every=2, check_growth=0.0)
    got = prob.solve(start_block(S.shape[0], 16, 2), m_max=600, tol=1e-9 if precision == "fp64" else 1e-6)
    # every accepted pair is an eigenpair of the pencil
    err = np.array([np.min(np.abs(ref - v)) / v for v in got.omega2])
    print(f"found {got.omega2.size} of {ref.size}; per-pair relative error vs dense:", np.array2string(err, precision=1))
    assert err.max() <= bar
    assert got.residual.max() <= (1e-9 if precision == "fp64" else 1e-6)
    # float32 stepping leaves a residual floor (about 1e-4 here) above the
    # gaps inside the cluster near omega = 205 (relative 1e-4): one float64
    # refinement pass resolves 37 of the 43, the second pass the rest
    assert got.omega2.size == ref.size
    np.testing.assert_allclose(got.omega2, ref, rtol=bar)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-5)])
def test_horn_block16_filter_matches_oracle(precision, tol):
    import torch

    kf = _kf()
    S, m = horn_pencil(16, 200)
    lmax = oracle.power_lambda_max(S, m, power_start(S.shape[0], 2), 30)
    tau, L = oracle.time_step_rule(lmax, 200.0)
    print(f"case horn 16x200 filter {precision} L={L}", flush=True)
    w = oracle.discrete_weights(200.0, 600.0, tau, L)
    X = start_block(S.shape[0], 16, 5)
    ref = oracle.apply_filter(S, m, tau, w, X)
    P = kf.Problem(S, m, 200.0, 600.0, tau, L, precision=precision)
    y = P.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    err = np.abs(y - ref).max(axis=0) / np.abs(ref).max(axis=0)
    assert err.max() <= tol, err


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("mixed", 1e-4)])
def test_full_horn_filter_properties(precision, tol):
    import torch

    kf = _kf()
    P = horn_problem()
    lmax = kf.estimate_lambda_max(P.S, P.m, 30, power_start(P.n, P.seed))
    tau, L = kf.time_step_rule(lmax, P.omega_min)
    print(f"case horn_4m filter properties {precision} n={P.n} L={L}", flush=True)
    prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, precision=precision)
    X = start_block(P.n, 16, 7)
    X[:, 0] = 1.0
    Y = prob.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    b0 = float(oracle.beta_tilde(np.array([0.0]), tau, prob.weights())[0])
    assert np.abs(Y[:, 0] - b0).max() <= tol * max(abs(b0), np.abs(Y[:, 1:]).max() / math.sqrt(P.n))
    # M-self-adjointness on the random columns: (x_i, C x_j)_M = (C x_i, x_j)_M
    A = X[:, 1:].T @ (P.m[:, None] * Y[:, 1:])
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() <= tol * scale
