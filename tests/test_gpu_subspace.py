"""The fixed-dimension filtered subspace iteration (Section 4.4, FEAST-type
variant) on the GPU against the oracle's (oracle.subspace_solve, plain CGS2
and scipy eigh) and the closed-form spectrum: every eigenvalue of the
interval with its multiplicity, in float64 (relative error <= 1e-10) and in
mixed precision (float32 then float64 stepping, <= 1e-6)."""

import math

import numpy as np
import pytest

import oracle
from synth import grid_spectrum, power_start, start_block, workload

pytestmark = pytest.mark.gpu


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def _grid2d():
    P = workload("grid2d_64")
    lam = oracle.power_lambda_max(P.S, P.m, power_start(P.n, P.seed), 30)
    tau, L = oracle.time_step_rule(lam, P.omega_min)
    return P, tau, L


def _inside(vals, lo, hi):
    om = np.sqrt(np.maximum(vals, 0.0))
    return np.sort(vals[(om >= lo) & (om <= hi)])


@pytest.mark.parametrize("precision,tol,bar", [("fp64", 1e-9, 1e-10), ("mixed", 1e-6, 1e-6)])
def test_subspace_grid2d_matches_oracle_and_closed_form(precision, tol, bar):
    kf = _kf()
    P, tau, L = _grid2d()
    ref_vals = _inside(grid_spectrum(2, 64), P.omega_min, P.omega_max)
    X0 = start_block(P.n, 32, 0)
    w = oracle.discrete_weights(P.omega_min, P.omega_max, tau, L)
    ref = oracle.subspace_solve(P.S, P.m, tau, w, X0, P.omega_min, P.omega_max, tol=1e-9, max_iters=40)
    print(f"case subspace grid2d_64 {precision}: oracle {ref.omega2.size} pairs in {ref.iterations} iterations",
          flush=True)
    prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, precision=precision)
    got = prob.subspace_solve(X0, max_iters=40, tol=tol)
    print(f"gpu: {got.omega2.size} pairs in {got.krylov_steps} iterations, dim {got.basis_size}, "
          f"float64 vector steps {got.refine_vector_steps}")
    assert got.status == 0
    assert got.omega2.size == ref.omega2.size == ref_vals.size == 20
    err = np.abs(np.sort(got.omega2) - np.sort(ref.omega2)) / ref_vals
    print("per-pair relative error vs the oracle:", np.array2string(err, precision=2))
    assert err.max() <= bar
    assert np.abs(np.sort(got.omega2) - ref_vals).max() / ref_vals.max() <= bar
    assert got.residual.max() <= tol
    if precision == "fp64":
        # the same arithmetic up to rounding order: the same iteration count
        assert abs(got.krylov_steps - ref.iterations) <= 1
    else:
        assert got.refine_vector_steps > 0 and got.t_refine > 0


def test_subspace_jittered_3d_matches_oracle():
    kf = _kf()
    from synth.grids import jittered_problem

    # Neumann, no exact multiplicities; [6, 7.5] holds 9 eigenvalues (three
    # near-triple clusters from the cube's triple ones)
    S, m = jittered_problem(3, 12, 0.1, seed=4)
    lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], 3), 30)
    lo, hi = 6.0, 7.5
    tau, L = oracle.time_step_rule(lam, lo)
    w = oracle.discrete_weights(lo, hi, tau, L)
    X0 = start_block(S.shape[0], 24, 6)
    ref = oracle.subspace_solve(S, m, tau, w, X0, lo, hi, tol=1e-9, max_iters=60)
    assert ref.omega2.size == 9
    print(f"case subspace jittered 3D n=12: oracle {ref.omega2.size} pairs, {ref.iterations} iterations", flush=True)
    got = kf.Problem(S, m, lo, hi, tau, L).subspace_solve(X0, max_iters=60, tol=1e-9)
    assert got.omega2.size == ref.omega2.size
    np.testing.assert_allclose(np.sort(got.omega2), np.sort(ref.omega2), rtol=1e-10)


def test_subspace_target_stops_early_and_small_space_reports_not_converged():
    kf = _kf()
    P, tau, L = _grid2d()
    prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, target=5)
    got = prob.subspace_solve(start_block(P.n, 32, 0), max_iters=40, tol=1e-9)
    assert got.omega2.size >= 5 and got.status == 0
    # 8 columns cannot hold the 20 eigenvalues of the interval
    few = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L).subspace_solve(start_block(P.n, 8, 0), max_iters=3,
                                                                                tol=1e-9)
    assert few.status == kf.KF_ENOTCONV and few.krylov_steps == 3


def test_subspace_rejects_bad_arguments():
    kf = _kf()
    P, tau, L = _grid2d()
    prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L)
    for args in ((start_block(P.n, 4, 0), 0, 1e-9), (start_block(P.n, 4, 0), 5, 0.0)):
        with pytest.raises(kf.KfError) as ei:
            prob.subspace_solve(*args)
        assert ei.value.code == kf.KF_EINVAL
    bad = start_block(P.n, 4, 0)
    bad[3, 2] = np.nan
    with pytest.raises(kf.KfError):
        prob.subspace_solve(bad, 5, 1e-9)
