"""The learned filter network on the GPU against the FP64 reference
(oracle.mlp): loss and gradient (bfloat16 matrix products, so compared at
bfloat16 accuracy), the Fourier-weight fallback, and training that lands
between the Fourier weights and the per-sample least-squares optimum."""

import numpy as np
import pytest

from oracle import mlp
from synth.workloads import filter_samples

pytestmark = pytest.mark.gpu


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def test_untrained_network_loss_equals_fourier_loss():
    kf = _kf()
    s = filter_samples(64, stream=1)
    theta = mlp.init_params(0)
    net = kf.Mlp(theta.astype(np.float32))
    loss, _ = net.loss_grad(s, want_grad=False)
    ref = np.mean([mlp.loss_of_weights(r, mlp.fourier_weights_normalised(*mlp.sample_params(*r)[:3])) for r in s])
    assert loss == pytest.approx(ref, rel=1e-4)


def _blocks(v):
    out, off = [], 0
    for shape in mlp.SHAPES:
        k = int(np.prod(shape))
        out.append((shape, v[off:off + k]))
        off += k
    return out


def test_gradient_matches_reference_element_by_element():
    """Every gradient entry against the FP64 reference with the same bfloat16
    operands (oracle.mlp with bf16=True): the rest of the arithmetic (float32
    accumulation, GELU and filter response in float32) moves an entry by far
    less than 1e-3 of its layer's largest entry."""
    kf = _kf()
    s = filter_samples(128, stream=0)
    rng = np.random.default_rng(3)
    theta = mlp.init_params(1)
    theta[-(128 * 512 + 512):] = 0.3 * rng.standard_normal(128 * 512 + 512)  # non-zero output layer
    theta32 = theta.astype(np.float32)
    net = kf.Mlp(theta32)
    loss, g = net.loss_grad(s)
    ref_loss, ref_g = mlp.loss_and_grad(theta32.astype(np.float64), s, bf16=True)
    print(f"loss gpu {loss:.8e} reference {ref_loss:.8e}")
    assert loss == pytest.approx(ref_loss, rel=1e-5)
    for (shape, a), (_, b) in zip(_blocks(g.astype(np.float64)), _blocks(ref_g)):
        scale = np.abs(b).max()
        err = np.abs(a - b).max() / scale
        print(f"layer block {shape}: max |gpu - ref| / max |ref| = {err:.2e}")
        assert err <= 1e-3, shape
    assert np.all(g[4 * 128:64 * 128] == 0.0)


def test_network_weights_match_reference_element_by_element():
    kf = _kf()
    s = filter_samples(100, stream=1)  # 100 rows: padded to 128 inside
    rng = np.random.default_rng(8)
    theta = mlp.init_params(2)
    theta[-(128 * 512 + 512):] = 0.3 * rng.standard_normal(128 * 512 + 512)
    theta32 = theta.astype(np.float32)
    got = kf.Mlp(theta32).batch_weights(s)
    ref, _, _ = mlp.forward(theta32.astype(np.float64), s, bf16=True)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    print(f"weights: max |gpu - ref| / max |ref| = {err:.2e}")
    assert err <= 1e-5
    for row, (_, _, L, _) in zip(got, [mlp.sample_params(*r) for r in s]):
        assert np.all(row[L:] == 0.0)


def test_training_beats_fourier_and_the_gate_keeps_the_better_weights():
    kf = _kf()
    train = filter_samples(8192, stream=0)
    valid = filter_samples(16, stream=1)
    net = kf.Mlp(mlp.init_params(4).astype(np.float32))
    rng = np.random.default_rng(np.random.SeedSequence(4).spawn(3)[2])
    epochs = 6
    order = np.concatenate([rng.permutation(len(train)) for _ in range(epochs)]).astype(np.int32)
    hist = net.train(train, order, epochs, 256, 1e-3)
    print("epoch losses", np.array2string(hist, precision=4))
    assert hist[-1] < hist[0]
    better = 0
    for r in valid:
        a, c, L, xm = mlp.sample_params(*r)
        w, used, jl, jf = net.weights(*r, L)
        jF = mlp.loss_of_weights(r, mlp.fourier_weights_normalised(a, c, L))
        wt = np.zeros(mlp.LMAX)
        wt[:L] = w
        j = mlp.loss_of_weights(r, wt)
        jT = mlp.loss_of_weights(r, mlp.teacher(r))
        # the acceptance gate never returns weights worse than the Fourier ones
        assert j <= jF * (1 + 1e-3)
        assert jT <= j * (1 + 1e-6)
        better += used
    print(f"learned weights used for {better}/16 validation problems")
    assert better >= 8


def test_model_gate_keeps_the_learned_path_no_slower_than_fourier():
    """End to end on the 3D cube with 64 cells per axis: for each interval the
    convergence model (kf_select_weights on the cube's distinct closed-form
    spectrum) chooses between the Fourier weights and the network's; every
    solve finds every pair, and in aggregate the chosen weights need no more
    Krylov steps than the Fourier weights (the network's weights alone are
    printed beside them)."""
    kf = _kf()
    from synth import distinct_target, grid_spectrum, power_start, start_block
    from synth.grids import grid_problem

    train = filter_samples(8192, stream=0)
    net = kf.Mlp(mlp.init_params(4).astype(np.float32))
    rng = np.random.default_rng(7)
    net.train(train, np.concatenate([rng.permutation(8192) for _ in range(4)]).astype(np.int32), 4, 256, 1e-3)
    n = 64
    S, m, h = grid_problem(3, n)
    lam = kf.estimate_lambda_max(S, m, 30, power_start(S.shape[0], 4))
    spec = np.sort(grid_spectrum(3, n))
    om = np.sqrt(spec[np.concatenate([[True], np.diff(spec) > 1e-10 * spec[1:]])])
    V0 = start_block(S.shape[0], 1, 4)
    tot = {"fourier": 0, "network": 0, "chosen": 0}
    for lo, hi in ((19.36, 25.11), (31.0, 38.0), (12.5, 20.0)):
        tau, L = kf.time_step_rule(lam, lo)
        tgt, vals, mult = distinct_target(spec, lo, hi, 1)
        four = kf.window_weights("indicator", lo, hi, tau, L)
        wnet = net.batch_weights(np.array([[lo, hi, tau, lam]]))[0, :L]
        pick, pred = kf.select_weights([four, wnet], tau, lo, hi, om, np.ones(om.size), kmax=1500, margin=0.02)
        steps = {}
        for name, w in (("fourier", four), ("network", wnet)):
            # checks in line: the step counts compared are the basis each
            # weight set needs, not when an overlapped check's result arrived
            prob = kf.Problem(S, m, lo, hi, tau, L, target=tgt, check_every=2, overlap_checks=False)
            prob.set_weights(w)
            r = prob.solve(V0, m_max=800, tol=1e-6)
            assert r.omega2.size == tgt
            np.testing.assert_allclose(r.omega2, vals, rtol=1e-10)
            steps[name] = r.krylov_steps
        steps["chosen"] = steps["network" if pick == 1 else "fourier"]
        for k in tot:
            tot[k] += steps[k]
        print(f"[{lo}, {hi}] target {tgt}: predicted {pred.tolist()} -> {'network' if pick else 'fourier'}; "
              f"measured {steps}")
    print("aggregate Krylov steps", tot)
    assert tot["chosen"] <= 1.05 * tot["fourier"]
