"""The window entry points (Section 4.3: triangle, Gaussian and spectrum-
adapted weights) against the oracle's: host arithmetic through the C ABI
(CPU), then the filter they define applied on the GPU and a full solve."""

import numpy as np
import pytest

import oracle
from oracle import windows
from synth import power_start, start_block, workload


def _kf():
    from paper_2402_08515_amd import kf

    return kf


@pytest.mark.parametrize("kind,width", [("indicator", 1.0), ("triangle", 2.0), ("triangle", 0.6), ("gaussian", 1.0),
                                        ("gaussian", 3.0)])
@pytest.mark.parametrize("lo,hi,tau,L", [(10.0, 20.0, 0.01, 63), (0.0, 3.0, 0.0056, 300), (30.0, 40.0, 0.0055, 1)])
def test_window_weights_match_oracle(kind, width, lo, hi, tau, L):
    kf = _kf()
    got = kf.window_weights(kind, lo, hi, tau, L, width)
    ref = windows.window_weights(kind, lo, hi, tau, L, width)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_notch_weights_match_oracle_and_zero_the_filter():
    kf = _kf()
    tau, L = 0.0055, 39
    w = oracle.discrete_weights(30.0, 40.0, tau, L)
    om = [0.0, 47.3, 52.0]
    got = kf.notch_weights(w, tau, om)
    np.testing.assert_allclose(got, windows.notch_weights(w, tau, om), rtol=1e-10, atol=1e-13)
    assert np.abs(oracle.beta_tilde(np.array(om), tau, got)).max() <= 1e-12
    assert np.array_equal(kf.notch_weights(w, tau, []), w)


def test_window_arguments_are_checked():
    kf = _kf()
    for call in (lambda: kf.window_weights("gaussian", 10.0, 20.0, 0.01, 10, 0.0),
                 lambda: kf.window_weights("triangle", 20.0, 10.0, 0.01, 10),
                 lambda: kf.window_weights("indicator", 10.0, 20.0, -1.0, 10),
                 lambda: kf.notch_weights(np.ones(10), 0.01, [5.0, 5.0]),
                 lambda: kf.notch_weights(np.ones(3), 0.01, [1.0, 2.0, 3.0, 4.0])):
        with pytest.raises(kf.KfError) as ei:
            call()
        assert ei.value.code == kf.KF_EINVAL
    with pytest.raises(KeyError):
        kf.window_weights("hann", 10.0, 20.0, 0.01, 10)


@pytest.mark.gpu
@pytest.mark.parametrize("kind,width", [("triangle", 2.0), ("gaussian", 1.0)])
def test_window_filter_on_gpu_matches_oracle_and_solves(kind, width):
    import torch

    kf = _kf()
    P = workload("grid2d_64")
    lam = oracle.power_lambda_max(P.S, P.m, power_start(P.n, P.seed), 30)
    tau, L = oracle.time_step_rule(lam, P.omega_min)
    w = kf.window_weights(kind, P.omega_min, P.omega_max, tau, L, width)
    # checks in line: the solve stops where the oracle's does (a check beside
    # the loop reports a later basis, where second copies of the square's
    # double eigenvalues may also have converged)
    prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, target=11, overlap_checks=False)
    prob.set_weights(w)
    x = torch.from_numpy(start_block(P.n, 3, 12)).cuda()
    y = prob.apply_filter(x).cpu().numpy()
    ref = oracle.apply_filter(P.S, P.m, tau, w, x.cpu().numpy())
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    om = np.linspace(0.0, 40.0, 81)
    np.testing.assert_allclose(prob.filter_response(om), oracle.beta_tilde(om, tau, w), rtol=1e-12, atol=1e-14)
    print(f"case window {kind} width {width} on grid2d_64", flush=True)
    r = prob.solve(start_block(P.n, 1, P.seed), m_max=120, tol=1e-9)
    ref_s = oracle.krylov_solve(P.S, P.m, tau, w, start_block(P.n, 1, P.seed), P.omega_min, P.omega_max, tol=1e-9,
                                m_max=120, target=11)
    assert r.omega2.size == ref_s.omega2.size == 11
    np.testing.assert_allclose(r.omega2, ref_s.omega2, rtol=1e-10)
    print(f"{kind}: {r.krylov_steps} Krylov steps (oracle {ref_s.krylov_steps})")
