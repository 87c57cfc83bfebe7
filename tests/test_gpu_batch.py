"""Batches of uneven problems: the batched, graph-captured filter
application equals the oracle's operator C of each member, and a batched
solve returns what each member's own solve returns."""

import math

import numpy as np
import pytest

import oracle
from synth import distinct_target, grid_spectrum, power_start, start_block
from synth.grids import grid_problem, jittered_problem

pytestmark = pytest.mark.gpu


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def _members(spec):
    out = []
    for dim, n, ofrac_lo, ofrac_hi, L in spec:
        S, m, h = grid_problem(dim, n)
        lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], n), 30)
        tau, Lr = oracle.time_step_rule(lam, ofrac_lo * math.sqrt(lam))
        out.append((S, m, ofrac_lo * math.sqrt(lam), ofrac_hi * math.sqrt(lam), tau, L or Lr))
    return out


# L = 1 and 2 (no step, one step), 4, 5 and 7 (last steps with two, three and
# one pending levels of the weighted sum), and the time-step rule's L
SPEC = [(2, 20, 0.3, 0.5, 1), (2, 33, 0.2, 0.3, 2), (3, 9, 0.3, 0.6, 5), (2, 41, 0.1, 0.2, 0), (3, 12, 0.25, 0.4, 0),
        (2, 25, 0.3, 0.4, 4), (3, 8, 0.3, 0.5, 7)]


@pytest.mark.parametrize("precision,b", [("fp64", 1), ("fp64", 3), ("mixed", 4)])
def test_batched_filter_matches_oracle(precision, b):
    import torch

    kf = _kf()
    mem = _members(SPEC)
    print(f"case batch apply_filter {precision} b={b} L={[x[5] for x in mem]}", flush=True)
    bt = kf.Batch([(S, m, lo, hi, tau, L, 0) for S, m, lo, hi, tau, L in mem], precision=precision)
    xs = [start_block(S.shape[0], b, 100 + i) for i, (S, *_rest) in enumerate(mem)]
    ys = bt.apply_filter([torch.from_numpy(x).cuda() for x in xs])
    tol = 1e-12 if precision == "fp64" else 2e-5
    for (S, m, lo, hi, tau, L), x, y in zip(mem, xs, ys):
        ref = oracle.apply_filter(S, m, tau, oracle.discrete_weights(lo, hi, tau, L), x)
        err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= tol, (L, err)


@pytest.mark.parametrize("workers", [1, 0])
def test_batched_solve_equals_member_solves(workers):
    """Member projections one after another (workers 1) or on concurrent
    streams driven by host threads (workers 0 = default pool)."""
    kf = _kf()
    spec = [(2, 24, 15.0, 24.0), (2, 31, 12.0, 20.0), (3, 10, 9.0, 14.0), (2, 40, 25.0, 30.0)]
    members, starts, targets = [], [], []
    b = 2
    for i, (dim, n, lo, hi) in enumerate(spec):
        S, m, h = grid_problem(dim, n)
        lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], i), 30)
        tau, L = oracle.time_step_rule(lam, lo)
        tgt = distinct_target(grid_spectrum(dim, n), lo, hi, b)[0]
        members.append((S, m, lo, hi, tau, L, tgt))
        starts.append(start_block(S.shape[0], b, 50 + i))
        targets.append(tgt)
    print(f"case batch solve targets={targets}", flush=True)
    # checks in line in the batch and in the single solves: the same steps
    bt = kf.Batch(members, check_every=1, batch_workers=workers, overlap_checks=False)
    got = bt.solve(starts, m_max=200, tol=1e-9)
    # the default: every member's checks beside the batched loop
    bo = kf.Batch(members, check_every=1, batch_workers=workers)
    gov = bo.solve(starts, m_max=200, tol=1e-9)
    for (S, m, lo, hi, tau, L, tgt), V0, g, go, (dim, n, _, _) in zip(members, starts, got, gov, spec):
        single = kf.Problem(S, m, lo, hi, tau, L, target=tgt, overlap_checks=False).solve(V0, m_max=200, tol=1e-9)
        assert g.omega2.size == single.omega2.size == go.omega2.size == tgt
        np.testing.assert_allclose(g.omega2, single.omega2, rtol=1e-12)
        tg, vals, mult = distinct_target(grid_spectrum(dim, n), lo, hi, b)
        np.testing.assert_allclose(g.omega2, np.repeat(vals, np.minimum(mult, b)), rtol=1e-10)
        np.testing.assert_allclose(go.omega2, np.repeat(vals, np.minimum(mult, b)), rtol=1e-10)
        assert g.krylov_steps == single.krylov_steps
        assert g.overlapped_checks == 0 and go.overlapped_checks >= 1


def test_batched_solve_mixed_on_jittered_members():
    kf = _kf()
    members, starts, refs = [], [], []
    for i, (n, lo, hi) in enumerate([(14, 6.0, 9.0), (10, 5.0, 8.0), (12, 7.0, 10.0)]):
        S, m = jittered_problem(3, n, 0.05, seed=10 + i)
        lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], i), 30)
        tau, L = oracle.time_step_rule(lam, lo)
        V0 = start_block(S.shape[0], 2, 60 + i)
        ref = oracle.krylov_solve(S, m, tau, oracle.discrete_weights(lo, hi, tau, L), V0, lo, hi, tol=1e-10,
                                  m_max=240, check_every=10)
        members.append((S, m, lo, hi, tau, L, int(ref.omega2.size)))
        starts.append(V0)
        refs.append(ref)
    bt = kf.Batch(members, precision="mixed", check_every=2, batch_workers=3)
    got = bt.solve(starts, m_max=240, tol=1e-6)
    for g, ref in zip(got, refs):
        assert g.residual.max() <= 1e-6
        err = np.array([np.min(np.abs(g.omega2 - v)) / v for v in ref.omega2])
        print("member per-pair relative error vs FP64 oracle:", np.array2string(err, precision=2))
        assert err.max() <= 1e-6


def test_member_weights_can_be_replaced():
    """kf_batch_set_weights: the batched filter of a member follows its new
    coefficients (here the Fourier weights of another interval)."""
    import torch

    kf = _kf()
    mem = _members(SPEC[:3])
    bt = kf.Batch([(S, m, lo, hi, tau, L, 0) for S, m, lo, hi, tau, L in mem], precision="fp64")
    S, m, lo, hi, tau, L = mem[1]
    w_new = oracle.discrete_weights(0.5 * lo, 0.8 * hi, tau, L)
    bt.set_weights(1, w_new)
    xs = [start_block(M[0].shape[0], 2, 200 + i) for i, M in enumerate(mem)]
    ys = bt.apply_filter([torch.from_numpy(x).cuda() for x in xs])
    for i, ((S, m, lo, hi, tau, L), x, y) in enumerate(zip(mem, xs, ys)):
        w = w_new if i == 1 else oracle.discrete_weights(lo, hi, tau, L)
        ref = oracle.apply_filter(S, m, tau, w, x)
        assert np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max() <= 1e-12
    with pytest.raises(kf.KfError):
        bt.set_weights(1, w_new[:-1])


def test_mixed_batch_restarts_cube_members_in_the_float64_stack():
    """Cube members with eigenvalues of multiplicity 3 and 6 and one start
    vector: float32 round-off seeds the extra copies, the float64
    refinement misses the target, and the member restarts with float64
    stepping inside the batched loop (the batch's float64 stack).  Every
    member ends with all distinct eigenvalues of its interval, equal to the
    closed form at the float64 bar."""
    kf = _kf()
    spec = [(3, 12, 15.0, 19.0), (3, 14, 12.0, 15.0), (2, 30, 10.0, 16.0), (3, 16, 20.0, 23.0)]
    members, starts, refs = [], [], []
    for i, (dim, n, lo, hi) in enumerate(spec):
        S, m, h = grid_problem(dim, n)
        lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], i), 30)
        tau, L = oracle.time_step_rule(lam, lo)
        tgt, vals, mult = distinct_target(grid_spectrum(dim, n), lo, hi, 1)
        members.append((S, m, lo, hi, tau, L, tgt))
        starts.append(start_block(S.shape[0], 1, 70 + i))
        refs.append(vals)
    print("case mixed batch with float64 restarts, targets", [x[6] for x in members], flush=True)
    bt = kf.Batch(members, precision="mixed", check_every=2, check_growth=0.15)
    got = bt.solve(starts, m_max=600, tol=1e-6)
    esc = [bool(g.escalated) for g in got]
    print("escalated", esc, "steps", [g.krylov_steps for g in got])
    assert any(esc)
    for g, vals, (S, m, lo, hi, tau, L, tgt) in zip(got, refs, members):
        assert g.omega2.size == tgt
        assert np.max(np.abs(g.omega2 - vals) / vals) <= 1e-10
        assert g.residual.max() <= 1e-6


def test_slices_of_one_operator_restart_together():
    """Three slices of one cube's interval (the same operator arrays) and a
    square: once float32 stepping fails for one slice, the others restart
    with float64 stepping too; every slice ends complete at the float64
    bar."""
    kf = _kf()
    S, m, h = grid_problem(3, 16)
    lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], 0), 30)
    members, starts, refs = [], [], []
    for i, (lo, hi) in enumerate([(20.0, 21.0), (21.0, 22.0), (22.0, 23.0)]):
        tau, L = oracle.time_step_rule(lam, lo)
        tgt, vals, mult = distinct_target(grid_spectrum(3, 16), lo, hi, 1)
        members.append((S, m, lo, hi, tau, L, tgt))
        starts.append(start_block(S.shape[0], 1, 80 + i))
        refs.append(vals)
    S2, m2, h2 = grid_problem(2, 30)
    lam2 = oracle.power_lambda_max(S2, m2, power_start(S2.shape[0], 1), 30)
    tau2, L2 = oracle.time_step_rule(lam2, 10.0)
    tgt2, vals2, mult2 = distinct_target(grid_spectrum(2, 30), 10.0, 16.0, 1)
    members.append((S2, m2, 10.0, 16.0, tau2, L2, tgt2))
    starts.append(start_block(S2.shape[0], 1, 83))
    refs.append(vals2)
    print("case mixed batch, three slices of one cube and a square, targets", [x[6] for x in members], flush=True)
    got = kf.Batch(members, precision="mixed", check_every=2, check_growth=0.15).solve(starts, m_max=600, tol=1e-6)
    esc = [bool(g.escalated) for g in got]
    print("escalated", esc, "steps", [g.krylov_steps for g in got])
    # the slices of the cube restart together
    assert esc[0] and esc[1] and esc[2]
    for g, vals, mem in zip(got, refs, members):
        assert g.omega2.size == mem[6]
        assert np.max(np.abs(g.omega2 - vals) / vals) <= 1e-10
