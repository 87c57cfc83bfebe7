"""GPU parity of the several-steps-per-launch time loop (matrix-powers form
of eq. 2stepmethod for banded operators) against the CPU oracle's filter
(Lemma 2.3's C applied by the plain time loop) and against the one-step
kernel.

Bars: float64 stepping 1e-12 of the largest output entry (the sums are
formed in another order than the oracle's); float32 stepping 2e-5 (the
one-step kernel's float32 bar)."""

import numpy as np
import pytest

import oracle
from synth import grid_spectrum, distinct_target, power_start, start_block, workload
from synth.grids import grid_problem, jittered_problem

pytestmark = pytest.mark.gpu


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def _setup(S, m, lo, hi, seed):
    lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], seed), 30)
    tau, L = oracle.time_step_rule(lam, lo)
    return tau, L, oracle.discrete_weights(lo, hi, tau, L)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("mixed", 2e-5)])
@pytest.mark.parametrize("steps", [1, 2, 5, 16, -1])
def test_whole_problem_in_one_workgroup_matches_oracle(precision, bar, steps):
    """grid2d_64 (3,969 rows, band 63): the problem fits one workgroup's LDS,
    so every launch advances `steps` steps (-1: the whole filter)."""
    import torch

    kf = _kf()
    P = workload("grid2d_64")
    tau, L, w = _setup(P.S, P.m, P.omega_min, P.omega_max, P.seed)
    x = start_block(P.n, 1, 11)
    print(f"case multistep grid2d_64 {precision} steps={steps} L={L}", flush=True)
    ref = oracle.apply_filter(P.S, P.m, tau, w, x)
    prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, precision=precision, multistep=steps)
    y = prob.apply_filter(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.abs(y - ref).max() <= bar * np.abs(ref).max()


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("mixed", 2e-5)])
@pytest.mark.parametrize("steps", [2, 4, 7])
def test_halo_windows_of_several_workgroups_match_oracle(precision, bar, steps):
    """A 255 x 255 square (65,025 rows, band 255): too large for one
    workgroup, so each owns a range of row slices plus steps*255 halo rows on
    either side; the output equals the oracle's and the one-step kernel's."""
    import torch

    kf = _kf()
    S, m, h = grid_problem(2, 256)
    lo, hi = 30.0, 45.0
    tau, L, w = _setup(S, m, lo, hi, 5)
    x = start_block(S.shape[0], 1, 12)
    print(f"case multistep square n=256 {precision} steps={steps} L={L}", flush=True)
    ref = oracle.apply_filter(S, m, tau, w, x)
    one = kf.Problem(S, m, lo, hi, tau, L, precision=precision)
    many = kf.Problem(S, m, lo, hi, tau, L, precision=precision, multistep=steps)
    xd = torch.from_numpy(x).cuda()
    y1 = one.apply_filter(xd).cpu().numpy()
    ys = many.apply_filter(xd).cpu().numpy()
    assert np.abs(ys - ref).max() <= bar * np.abs(ref).max()
    assert np.abs(ys - y1).max() <= 2 * bar * np.abs(ref).max()


def test_jittered_unstructured_mesh_matches_oracle():
    """A jittered 3D mesh (natural vertex ordering: band of one layer of
    vertices), float64."""
    import torch

    kf = _kf()
    S, m = jittered_problem(3, 14, 0.05, seed=3)
    lo, hi = 6.0, 9.0
    tau, L, w = _setup(S, m, lo, hi, 2)
    x = start_block(S.shape[0], 1, 13)
    print(f"case multistep jittered n={S.shape[0]} L={L}", flush=True)
    ref = oracle.apply_filter(S, m, tau, w, x)
    prob = kf.Problem(S, m, lo, hi, tau, L, multistep=4)
    y = prob.apply_filter(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_solve_with_the_whole_filter_per_launch_finds_the_closed_form():
    """The eigensolver on grid2d_64 with one launch per filter application:
    all 11 distinct eigenvalues of [10, 20] at the float64 bar."""
    kf = _kf()
    P = workload("grid2d_64")
    tau, L, w = _setup(P.S, P.m, P.omega_min, P.omega_max, P.seed)
    tgt, vals, mult = distinct_target(grid_spectrum(2, 64), P.omega_min, P.omega_max, 1)
    print(f"case multistep solve grid2d_64 target={tgt}", flush=True)
    prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, multistep=-1)
    got = prob.solve(start_block(P.n, 1, P.seed), m_max=40, tol=1e-9)
    assert got.omega2.size == tgt
    assert np.max(np.abs(got.omega2 - vals) / vals) <= 1e-10


def test_band_too_wide_for_lds_is_an_error():
    """grid3d_96: the band is 9,216 rows, two levels of the halo alone exceed
    a workgroup's LDS: KF_EINVAL, and the problem still works without it."""
    import torch

    kf = _kf()
    S, m, h = grid_problem(3, 96)
    lam = 4.0 * 3 / h**2
    tau, L = kf.time_step_rule(lam, 30.0)
    print(f"case multistep grid3d_96 band too wide", flush=True)
    prob = kf.Problem(S, m, 30.0, 40.0, tau, L, multistep=2)
    with pytest.raises(kf.KfError) as e:
        prob.apply_filter(torch.from_numpy(start_block(S.shape[0], 1, 1)).cuda())
    assert e.value.code == kf.KF_EINVAL
