"""GPU parity of the fused time-stepping filter, the weights, the filter
response and the power iteration against the CPU oracle (same inputs,
element by element).

Tolerances: float64 stepping is compared at 1e-12 relative to the largest
entry of the oracle's result (L <= 63 steps, each adding a few ulps of
rounding; the eigensolver's bar is 1e-10 on eigenvalues).  float32 stepping
(mixed precision) at 2e-5: the per-step rounding of 6e-8 grows at most
linearly over the L steps of a stable scheme and the filter sum is formed
from O(1) terms.
"""

import math

import numpy as np
import pytest

import oracle
from synth import power_start, start_block
from synth.grids import grid_problem, jittered_problem

pytestmark = pytest.mark.gpu


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def _case(dim, n, omin_frac=0.3, omax_frac=0.5, L=None):
    S, m, h = grid_problem(dim, n)
    lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], 0), 30)
    tau, Lr = oracle.time_step_rule(lam, omin_frac * math.sqrt(lam))
    return S, m, tau, (L or Lr), omin_frac * math.sqrt(lam), omax_frac * math.sqrt(lam)


@pytest.mark.parametrize(
    "dim,n,b,L,index_bytes,remap",
    [
        (2, 64, 1, 63, 0, 1),  # the 2D workload size, 3969 DOFs (ragged last slice)
        (2, 37, 1, 17, 4, 0),
        (2, 37, 3, 17, 2, 1),
        (2, 20, 2, 1, 0, 1),  # L = 1: no time step
        (2, 20, 4, 2, 0, 1),  # L = 2: the first step is also the last
        (3, 13, 8, 9, 0, 1),
        (3, 9, 16, 5, 4, 1),
        (3, 11, 5, 6, 2, 0),
        # the weighted sum is taken every third step: L - 1 = 2, 3, 6, 9
        # cover last steps with one, two and three pending levels
        (2, 37, 1, 3, 0, 1),
        (2, 37, 1, 4, 0, 1),
        (2, 37, 2, 7, 2, 1),
        (3, 9, 4, 10, 0, 0),
        # a single float64 vector is read in place by the first two steps
        (2, 20, 1, 2, 0, 1),  # L = 2: the in-place first step is also the last
        (2, 5, 1, 9, 0, 1),  # 16 DOFs: less than one 64-row slice
    ],
)
def test_apply_filter_fp64_matches_oracle(dim, n, b, L, index_bytes, remap):
    import torch

    kf = _kf()
    print(f"case apply_filter fp64 dim={dim} n={n} b={b} L={L} idx={index_bytes} remap={remap}", flush=True)
    S, m, tau, _, omin, omax = _case(dim, n)
    w = oracle.discrete_weights(omin, omax, tau, L)
    X = start_block(S.shape[0], b, 17)
    ref = oracle.apply_filter(S, m, tau, w, X)
    P = kf.Problem(S, m, omin, omax, tau, L, index_bytes=index_bytes, xcd_remap=bool(remap))
    np.testing.assert_allclose(P.weights(), w, rtol=1e-14, atol=1e-300)
    x = torch.from_numpy(X).cuda()
    y = P.apply_filter(x).cpu().numpy()
    torch.cuda.synchronize()
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err <= 1e-12, err


def test_apply_filter_unstructured_neumann_fp64():
    import torch

    kf = _kf()
    S, m = jittered_problem(3, 7, 0.2, seed=3)
    lam = oracle.power_lambda_max(S, m, power_start(S.shape[0], 3), 30)
    tau, L = oracle.time_step_rule(lam, 5.0)
    w = oracle.discrete_weights(5.0, 9.0, tau, L)
    X = start_block(S.shape[0], 2, 5)
    ref = oracle.apply_filter(S, m, tau, w, X)
    P = kf.Problem(S, m, 5.0, 9.0, tau, L)
    y = P.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("b", [1, 4, 16])
def test_apply_filter_mixed_matches_oracle(b):
    import torch

    kf = _kf()
    print(f"case apply_filter mixed b={b}", flush=True)
    S, m, tau, L, omin, omax = _case(2, 64)
    w = oracle.discrete_weights(omin, omax, tau, L)
    X = start_block(S.shape[0], b, 3)
    ref = oracle.apply_filter(S, m, tau, w, X)
    P = kf.Problem(S, m, omin, omax, tau, L, precision="mixed")
    y = P.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err <= 2e-5, err


def test_filter_response_matches_oracle():
    kf = _kf()
    S, m, tau, L, omin, omax = _case(2, 20)
    P = kf.Problem(S, m, omin, omax, tau, L)
    om = np.linspace(0.0, 1.99 / tau, 513)
    ref = oracle.beta_tilde(om, tau, oracle.discrete_weights(omin, omax, tau, L))
    np.testing.assert_allclose(P.filter_response(om), ref, atol=1e-12 * np.abs(ref).max())


def test_set_weights_changes_the_operator():
    import torch

    kf = _kf()
    S, m, tau, L, omin, omax = _case(2, 16)
    w = np.random.default_rng(4).standard_normal(L) * tau
    P = kf.Problem(S, m, omin, omax, tau, L)
    P.set_weights(w)
    X = start_block(S.shape[0], 1, 2)
    ref = oracle.apply_filter(S, m, tau, w, X)
    y = P.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dim,n", [(2, 64), (3, 12)])
def test_power_iteration_matches_oracle(dim, n):
    kf = _kf()
    S, m, h = grid_problem(dim, n)
    x0 = power_start(S.shape[0], 7)
    ref = oracle.power_lambda_max(S, m, x0, 30)
    got = kf.estimate_lambda_max(S, m, 30, x0)
    assert got == pytest.approx(ref, rel=1e-12)




@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_and_cached_load_variants_match_oracle(precision):
    """Every fused-step variant the autotuner chooses among (cached or
    non-temporal operator loads, either XCD mapping, 2- or 4-byte indices)
    computes the same operator C."""
    import torch

    kf = _kf()
    S, m, tau, _, omin, omax = _case(3, 13)
    L = 9
    w = oracle.discrete_weights(omin, omax, tau, L)
    X = start_block(S.shape[0], 3, 21)
    ref = oracle.apply_filter(S, m, tau, w, X)
    tol = 1e-12 if precision == "fp64" else 2e-5
    print(f"case autotune precision={precision}", flush=True)
    P = kf.Problem(S, m, omin, omax, tau, L, precision=precision, autotune=True)
    t = P.tuning()
    assert t["us_per_step"] > 0 and t["index_bytes"] in (2, 4) and t["nt_loads"] in (0, 1)
    assert t["gather_unroll"] in (2, 3, 4, 6)
    y = P.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.abs(y - ref).max() / np.abs(ref).max() <= tol
    for ib in (2, 4):
        for remap in (0, 1):
            Q = kf.Problem(S, m, omin, omax, tau, L, precision=precision, nt_loads=False, index_bytes=ib,
                           xcd_remap=bool(remap))
            assert Q.tuning()["nt_loads"] == 0 and Q.tuning()["us_per_step"] == 0
            y = Q.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
            assert np.abs(y - ref).max() / np.abs(ref).max() <= tol, (ib, remap)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dim,n", [(2, 37), (3, 13)])
@pytest.mark.parametrize("unroll", [2, 3, 4, 6])
def test_gather_unroll_variants_match_oracle(precision, dim, n, unroll):
    """Each unroll factor of the single-vector step's loop over a slice's
    entries (2D rows hold up to 7 entries, 3D rows up to 15; both grids end in
    a ragged slice) computes the same operator C."""
    import torch

    kf = _kf()
    S, m, tau, _, omin, omax = _case(dim, n)
    L = 8
    w = oracle.discrete_weights(omin, omax, tau, L)
    X = start_block(S.shape[0], 1, 23)
    ref = oracle.apply_filter(S, m, tau, w, X)
    tol = 1e-12 if precision == "fp64" else 2e-5
    print(f"case gather_unroll={unroll} precision={precision} dim={dim} n={n}", flush=True)
    P = kf.Problem(S, m, omin, omax, tau, L, precision=precision, gather_unroll=unroll)
    assert P.tuning()["gather_unroll"] == unroll
    y = P.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.abs(y - ref).max() / np.abs(ref).max() <= tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dim,n", [(2, 37), (3, 13)])
@pytest.mark.parametrize("b", [2, 4, 16])
@pytest.mark.parametrize("lpr", [1, 2, 4])
def test_lds_band_variants_match_oracle(precision, dim, n, b, lpr):
    """Blocks gathering from the LDS copy of each workgroup's band of rows
    (block_band = 1) compute the same operator C.  On the square every copy
    fits in 64 KB; on the cube (offsets up to 144 rows) the float64 block of
    16 with one lane per row does not, and those launches gather from the
    caches instead."""
    import torch

    kf = _kf()
    S, m, tau, _, omin, omax = _case(dim, n)
    L = 8
    w = oracle.discrete_weights(omin, omax, tau, L)
    X = start_block(S.shape[0], b, 29)
    ref = oracle.apply_filter(S, m, tau, w, X)
    tol = 1e-12 if precision == "fp64" else 2e-5
    print(f"case block_band precision={precision} dim={dim} n={n} b={b} lpr={lpr}", flush=True)
    P = kf.Problem(S, m, omin, omax, tau, L, precision=precision, block_band=1, lanes_per_row=lpr)
    y = P.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.abs(y - ref).max() / np.abs(ref).max() <= tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("b", [2, 4, 8, 16])
@pytest.mark.parametrize("lpr", [1, 2, 4])
def test_lanes_per_row_variants_match_oracle(precision, b, lpr):
    """Blocks of b vectors with 1, 2 or 4 lanes sharing a row (capped at b),
    on a ragged cube (last slice partly empty)."""
    import torch

    kf = _kf()
    S, m, tau, _, omin, omax = _case(3, 11)
    L = 7
    w = oracle.discrete_weights(omin, omax, tau, L)
    X = start_block(S.shape[0], b, 30 + b)
    ref = oracle.apply_filter(S, m, tau, w, X)
    print(f"case lanes_per_row={lpr} b={b} {precision}", flush=True)
    P = kf.Problem(S, m, omin, omax, tau, L, precision=precision, lanes_per_row=lpr)
    y = P.apply_filter(torch.from_numpy(X).cuda()).cpu().numpy()
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert np.abs(y - ref).max() / np.abs(ref).max() <= tol
