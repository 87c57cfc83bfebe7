"""kf_apply_filter_noalloc (time-stepping blocks in the library's fixed device
array, no allocation) against kf_apply_filter on the same inputs: the two run
the same kernels on the same values, so the results must agree bit for bit.
Two calls in a row, the second with a smaller input, so that what the first
call left in the shared array cannot leak into the second."""

import numpy as np
import pytest
import torch

import oracle
from synth.grids import grid_problem

pytestmark = pytest.mark.gpu


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def _problem(kf, dim, n, precision, omin=10.0, omax=20.0):
    S, m, h = grid_problem(dim, n)
    lam = oracle.power_lambda_max(S, m, np.random.default_rng(1000 + n).standard_normal(S.shape[0]), 30)
    tau, L = oracle.time_step_rule(lam, omin)
    return kf.Problem(S, m, omin, omax, tau, L, precision=precision), S, m, tau, L


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_equals_allocating_filter_twice_second_smaller(precision):
    kf = _kf()
    big, S1, m1, tau1, L1 = _problem(kf, 3, 30, precision)        # 24,389 DOFs
    small, S2, m2, tau2, L2 = _problem(kf, 2, 24, precision)      # 529 DOFs, ragged last slice
    g = torch.Generator(device="cpu").manual_seed(5)
    x1 = torch.randn(big.n, 4, generator=g, dtype=torch.float64).cuda()
    x2 = torch.randn(small.n, 1, generator=g, dtype=torch.float64).cuda()
    print(f"case {precision}: call 1 n={big.n} b=4 L={L1}; call 2 n={small.n} b=1 L={L2}", flush=True)
    y1 = torch.full_like(x1, np.nan)
    big.apply_filter_noalloc(x1, y1)
    y2 = torch.full_like(x2, np.nan)
    small.apply_filter_noalloc(x2, y2)
    torch.cuda.synchronize()
    r1 = big.apply_filter(x1)
    r2 = small.apply_filter(x2)
    torch.cuda.synchronize()
    assert torch.equal(y1, r1)
    assert torch.equal(y2, r2)
    # and both against the oracle, to the precision of the stepping
    tol = 1e-12 if precision == "fp64" else 2e-5
    for prob, S, m, tau, x, y in ((big, S1, m1, tau1, x1, y1), (small, S2, m2, tau2, x2, y2)):
        ref = oracle.apply_filter(S, m, tau, prob.weights(), x.cpu().numpy())
        err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= tol, err


def test_noalloc_rejects_blocks_beyond_the_fixed_array():
    kf = _kf()
    # 3 x 175,616 x 16 x 8 bytes > 64 MiB
    S, m, h = grid_problem(3, 57)
    prob = kf.Problem(S, m, 10.0, 20.0, 1e-3, 3)
    x = torch.zeros(prob.n, 16, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(kf.KfError) as ei:
        prob.apply_filter_noalloc(x, y)
    assert ei.value.code == kf.KF_EINVAL and "64 MiB" in str(ei.value)
    # a block that fits on the same problem works
    x1 = torch.ones(prob.n, 1, dtype=torch.float64, device="cuda")
    y1 = torch.zeros_like(x1)
    prob.apply_filter_noalloc(x1, y1)
    torch.cuda.synchronize()
    assert torch.equal(y1, prob.apply_filter(x1))
