#!/usr/bin/env python3
"""Benchmark of the filtered time-domain Krylov eigensolver on one MI355X.

Workload (default ``grid3d_96``): 3D unit cube, Dirichlet, Kuhn P1 with
lumped mass, 96 cells per axis (857,375 DOFs, 5,947,475 stored entries),
interval omega in [30, 40], one N(0,1) start vector from seed 1, float64.
tau = 0.9*2/sqrt(lambda_est) with lambda_est from 30 power iterations,
L = ceil(2*pi/(omega_min*tau)).

One step = one complete eigensolve (kf_solve): filter applications (the fused
leapfrog kernels), M-inner CGS2, projected-pencil updates, Rayleigh-Ritz
checks and residuals, until all 110 eigenpairs the start vector can reach are
accepted at relative residual <= 1e-6.  Inputs (operator, start vector) are
resident in device memory before the timed region.

value = DOF*timesteps per second of the whole solve:
        n * (leapfrog vector steps) / wall time of the solve.
The JSON line also carries the seconds to all eigenpairs, the
leapfrog-only rate, the roofline of the dominant kernel (k_leapfrog) and the
CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF·timesteps/s of fused leapfrog; s to all eigenpairs in interval at res 1e-6"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_per_step(n: int, nnz: int, b: int, value_bytes: int, L: int) -> float:
    """Average bytes one fused step must move over a filter application of L
    time levels, with the operator stored once: every stored entry (value +
    4-byte column index) and the row pointers at each step; per vector-DOF,
    cur read, prev read (not at the first step), next written (not at the
    last), the accumulator written at the first step and read and written at
    the steps that bring the weighted sum up to date (every third step: a step
    sees three consecutive time levels), read at the last step, which writes
    the float64 result instead of next."""
    mat = nnz * (value_bytes + 4) + 4 * (n + 1)
    total = 0.0
    for l in range(1, L):
        first, last = l == 1, l == L - 1
        u = 1 + 3 * ((l - 2) // 3) if l >= 2 else 1
        update = first or last or l - u == 3
        vec = value_bytes * (1 + (not first) + (not last))
        if first and not last:
            vec += value_bytes
        elif update and not last:
            vec += 2 * value_bytes
        elif last and not first:
            vec += value_bytes
        if last:
            vec += 8
        total += mat + vec * n * b
    return total / max(L - 1, 1)


def scope_bytes_per_step(n: int, nnz: int, b: int, value_bytes: int) -> float:
    """Algorithmic bytes of one fused step by the scope table's per-unit
    figure: [nnz (s_v + 4) + 4 (N + 1)] / (N b) + 5 s_v bytes per vector-DOF
    (the operator stored once with 4-byte indices; cur read, prev read, next
    written, accumulator read and written), times N b."""
    per_unit = (nnz * (value_bytes + 4) + 4 * (n + 1)) / (n * b) + 5 * value_bytes
    return per_unit * n * b


def measured_copy_gbs() -> float:
    """Bandwidth of a plain device-to-device copy of 1 GiB (bytes read plus
    bytes written per second), the practical HBM rate beside the 8 TB/s peak."""
    import torch

    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbs = 2 * a.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def traffic_from_profile(kernel_src_hash: str, workload: str):
    """HBM bytes per launch of k_leapfrog from committed rocprofv3 counter
    summaries, or None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"leapfrog_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256") != kernel_src_hash:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(P, tau, L, V0, krylov_iters: int):
    """The CPU oracle, untuned, on a bounded sample: the first
    ``krylov_iters`` filter applications (+ its Gram-Schmidt) of the same
    workload."""
    import oracle
    from threadpoolctl import threadpool_info

    w = oracle.discrete_weights(P.omega_min, P.omega_max, tau, L)
    t0 = time.perf_counter()
    r = oracle.krylov_solve(P.S, P.m, tau, w, V0, P.omega_min, P.omega_max, tol=1e-6, m_max=10**6,
                            max_iters=krylov_iters, check_every=10**9)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {
        "value": P.n * r.leapfrog_vector_steps / dt,
        "unit": "DOF·timesteps/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{krylov_iters} Krylov iterations ({r.leapfrog_vector_steps} leapfrog steps) of {P.name} "
                  f"with Gram-Schmidt, one final Rayleigh-Ritz; {dt:.1f} s; sparse products single-threaded, "
                  f"BLAS on {threads} threads",
    }


def bench_batch(args):
    """The uneven batch: 64 squares/cubes (seed 3), block width 4, float32
    time stepping, float64 projection, every member solved to all its
    eigenpairs (23,172 in total).  Intervals holding more than
    --slice-target pairs are cut into slices (between eigenvalues of the
    closed form) that enter the batch as members of their own; a slice of
    width d gets T >= 2 pi / (3 d) (the filter's transition at most three
    times the slice, as the rule's T gives the 3D cube), the other members
    the rule's L.  Timed: the batched mixed solve (one kf_solve_batch call),
    the same with the network's weights where the gate takes them, and the
    plain float64 method slice by slice; every problem is created before its
    timed region."""
    import math

    import numpy as np
    import torch

    from paper_2402_08515_amd import kf
    from synth import distinct_target, grid_spectrum, power_start, start_block
    from synth.netinit import init_params
    from synth.workloads import batch64_slices, filter_samples

    os.environ.setdefault("KF_PROGRESS", "1")  # the library reports the batched loop's progress on stderr
    slices = batch64_slices(args.slice_target, args.batch_count)
    lam_of, members, starts, meta = {}, [], [], []
    multiple = []  # the slice holds an eigenvalue of multiplicity above the block width
    for (i, P, lo, hi, tgt) in slices:
        if i not in lam_of:
            lam_of[i] = kf.estimate_lambda_max(P.S, P.m, 30, power_start(P.n, P.seed))
        tau, L_rule = kf.time_step_rule(lam_of[i], lo)
        L = max(L_rule, int(math.ceil(2 * math.pi / (args.slice_transition * (hi - lo) * tau))))
        members.append((P.S, P.m, lo, hi, tau, L, tgt))
        starts.append(start_block(P.n, P.block, P.seed))
        meta.append((i, P, lo, hi, tgt, lam_of[i]))
        t_, vals_, mult_ = distinct_target(grid_spectrum(P.meta["dim"], P.meta["n"]), lo, hi, P.block)
        multiple.append(bool(mult_.size and mult_.max() > P.block))
    total = sum(m[6] for m in members)
    print(f"[bench] batch: {args.batch_count} members in {len(members)} slices, L in "
          f"[{min(m[5] for m in members)}, {max(m[5] for m in members)}], {total} pairs", file=sys.stderr, flush=True)

    def count(res):
        found = sum(min(r.omega2.size, m[6]) for r, m in zip(res, members))
        errs = []
        for r, (i, P, lo, hi, tgt, lam) in zip(res, meta):
            if r.omega2.size:
                t, vals, mult = distinct_target(grid_spectrum(P.meta["dim"], P.meta["n"]), lo, hi, P.block)
                near = vals[np.abs(r.omega2[:, None] - vals[None, :]).argmin(axis=1)]
                errs.append(float(np.max(np.abs(r.omega2 - near) / near)))
        return int(found), max(errs) if errs else None

    opts = dict(check_every=2, check_growth=args.batch_check_growth)
    bopts = dict(opts, batch_workers=args.batch_workers)
    runs = {}
    sel_runs = set(args.batch_runs.split(","))
    # mixed, batched (the slices' problems and the stacked operator are built,
    # and the batched step variant timed, before the timed region)
    bt = kf.Batch([m for m in members], precision="mixed", autotune=True,
                  **(dict(bopts, escalate=False) if args.batch_no_restart else bopts))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = bt.solve(starts, m_max=args.m_max, tol=args.tol)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    found, err = count(res)
    esc = int(sum(r.escalated for r in res))
    steps = sum(P.n * r.leapfrog_vector_steps for (i, P, *_), r in zip(meta, res))
    def short(res):
        out = []
        for r, (i, P, lo, hi, tgt, lam), mm in zip(res, meta, members):
            if r.omega2.size < tgt:
                out.append({"member": i, "dim": P.meta["dim"], "n": P.meta["n"], "interval": [lo, hi], "L": mm[5],
                            "target": tgt, "found": int(r.omega2.size), "basis": r.basis_size,
                            "krylov_steps": r.krylov_steps, "escalated": bool(r.escalated), "status": r.status})
        return out

    def phases(res):
        # per-member event times summed over the members (a batch member's
        # t_leapfrog is the shared batched stepping time plus its own after
        # an escalation)
        return {"gram_schmidt": sum(r.t_gs for r in res), "rayleigh_ritz": sum(r.t_rr for r in res),
                "refine": sum(r.t_refine for r in res),
                "escalated_leapfrog": sum(max(r.t_leapfrog - res[0].t_leapfrog, 0.0) for r in res if r.escalated)}

    runs["mixed_batched"] = {"seconds": wall, "pairs": found, "max_rel_err": err, "escalated_slices": esc,
                             "batched_leapfrog_s": res[0].t_leapfrog, "phase_seconds_summed": phases(res),
                             "incomplete": short(res)}
    print(f"[bench] mixed batched: {wall:.2f}s, {found}/{total} pairs, max err {err}, {esc} slices escalated",
          file=sys.stderr, flush=True)
    bt.close()
    del bt
    # mixed, batched, with the members whose slice holds eigenvalues of
    # multiplicity above the block width stepping in float64 from the start
    # (the remedy for what float32 stepping cannot resolve; the closed-form
    # spectrum tells which slices they are)
    mem_fp64 = [m + (f,) for m, f in zip(members, multiple)]
    if "fp64members" in sel_runs:
        bt = kf.Batch(mem_fp64, precision="mixed", autotune=True, **bopts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res_mf = bt.solve(starts, m_max=args.m_max, tol=args.tol)
        torch.cuda.synchronize()
        wmf = time.perf_counter() - t0
        fmf, emf = count(res_mf)
        runs["mixed_batched_fp64_members"] = {"seconds": wmf, "pairs": fmf, "max_rel_err": emf,
                                              "fp64_members": int(sum(multiple)),
                                              "escalated_slices": int(sum(r.escalated for r in res_mf)),
                                              "batched_leapfrog_s": res_mf[0].t_leapfrog, "incomplete": short(res_mf)}
        print(f"[bench] mixed batched, {sum(multiple)} slices with multiplicity > 4 in float64: "
              f"{wmf:.2f}s, {fmf}/{total} pairs", file=sys.stderr, flush=True)
        bt.close()
        del bt
    if "fp64batched" in sel_runs:
        # the plain method batched: float64 stepping in one stacked operator
        bt = kf.Batch([m for m in members], precision="fp64", autotune=True, **bopts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res_b64 = bt.solve(starts, m_max=args.m_max, tol=args.tol)
        torch.cuda.synchronize()
        wb64 = time.perf_counter() - t0
        fb64, eb64 = count(res_b64)
        runs["fp64_batched"] = {"seconds": wb64, "pairs": fb64, "max_rel_err": eb64,
                                "batched_leapfrog_s": res_b64[0].t_leapfrog, "incomplete": short(res_b64)}
        print(f"[bench] fp64 batched: {wb64:.2f}s, {fb64}/{total} pairs", file=sys.stderr, flush=True)
        bt.close()
        del bt
    # learned weights where the gate takes them, mixed, batched
    if not args.no_learned:
        # trained on the batch's own spectral range (the members' lambda_max),
        # intervals from the evaluation law (omega_min ~ U[5, 50], width ~ U[5, 20])
        lams = [lam for (_, _, _, _, _, lam) in meta]
        lam_rng = (0.9 * min(lams), 1.1 * max(lams))
        train = filter_samples(args.mlp_samples, stream=0, lam_range=lam_rng)
        net = kf.Mlp(init_params(4).astype(np.float32))
        rng = np.random.default_rng(np.random.SeedSequence(4).spawn(3)[2])
        order = np.concatenate([rng.permutation(len(train)) for _ in range(args.mlp_epochs)]).astype(np.int32)
        net.train(train, order, args.mlp_epochs, 256, 1e-3)
        bt = kf.Batch(mem_fp64, precision="mixed", autotune=True, **bopts)
        used = 0
        t_sel = time.perf_counter()
        wn_all = net.batch_weights(np.array([[lo, hi, tau, lam] for (_, _, lo, hi, _, lam) in meta]))
        spec_of = {}
        for q, ((S, m, lo, hi, tau, L, tgt), (i, P, _, _, _, lam)) in enumerate(zip(members, meta)):
            # the network's weights where the Krylov convergence model (on the
            # member's closed-form spectrum) predicts fewer steps
            if i not in spec_of:
                spec_of[i] = model_spectrum(P.meta["dim"], P.meta["n"], hi * 1.5)
            om, wt = spec_of[i]
            # only inputs inside the range the network was trained on (its
            # samples' interval widths; the slices cut from wide intervals are
            # narrower), and only a prediction that resolves the slice within
            # the model's step limit
            if not (lam_rng[0] <= lam <= lam_rng[1] and 5.0 <= hi - lo <= 20.0):
                continue
            four = kf.window_weights("indicator", lo, hi, tau, L)
            kmax = 1500
            pick, pred = kf.select_weights([four, wn_all[q, :L]], tau, lo, hi, om, wt, kmax=kmax, margin=0.02)
            if pick == 1 and pred[1] < kmax:
                bt.set_weights(q, wn_all[q, :L])
                used += 1
        t_sel = time.perf_counter() - t_sel
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        resl = bt.solve(starts, m_max=args.m_max, tol=args.tol)
        torch.cuda.synchronize()
        wl = time.perf_counter() - t0
        fl, el = count(resl)
        runs["learned_mixed_batched"] = {"seconds": wl, "pairs": fl, "max_rel_err": el, "gate_took_network": used,
                                         "selection_seconds_untimed": t_sel, "fp64_members": int(sum(multiple)),
                                         "escalated_slices": int(sum(r.escalated for r in resl))}
        print(f"[bench] learned mixed batched: {wl:.2f}s, {fl}/{total} pairs, network weights on {used} slices",
              file=sys.stderr, flush=True)
        bt.close()
        del bt
    # the plain method: float64 stepping, Fourier weights, one slice after another
    if not args.no_sequential:
        singles = [kf.Problem(S, m, lo, hi, tau, L, target=tgt, autotune=True, **opts)
                   for (S, m, lo, hi, tau, L, tgt) in members]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res64 = [pr.solve(V0, m_max=args.m_max, tol=args.tol) for pr, V0 in zip(singles, starts)]
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t0
        f64, e64 = count(res64)
        runs["plain_fp64_one_by_one"] = {"seconds": w64, "pairs": f64, "max_rel_err": e64,
                                         "phase_seconds_summed": {"leapfrog": sum(r.t_leapfrog for r in res64),
                                                                  "gram_schmidt": sum(r.t_gs for r in res64),
                                                                  "rayleigh_ritz": sum(r.t_rr for r in res64)},
                                         "incomplete": short(res64)}
        print(f"[bench] plain fp64 one by one: {w64:.2f}s, {f64}/{total} pairs", file=sys.stderr, flush=True)
        del singles
    out = {
        "metric": METRIC,
        "value": steps / wall,
        "unit": "DOF·timesteps/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-step/f64-proj",
        "data": "synthetic",
        "config": {"workload": f"batch64[:{args.batch_count}]", "slices": len(members), "block": 4,
                   "tol": args.tol, "m_max": args.m_max, "slice_target": args.slice_target, "check_growth": args.batch_check_growth,
                   "target_pairs": int(total), "parallelism": "1 GPU"},
        "s_to_all_eigenpairs": wall if found >= total else None,
        "pairs_accepted": found,
        "runs": runs,
        "batched_leapfrog_dof_steps_per_s": steps / res[0].t_leapfrog,
    }
    print(json.dumps(out))


def bench_horn(args):
    """The horn: 752,845 DOFs (3,999,744 jittered P1 tetrahedra, Neumann), a
    block of 16 start vectors (seed 2), float32 time stepping with float64
    projection, tau and L by the rule at omega_min = 200 (the filter of the
    interval [200, 600]).  [200, 600] holds 6,542 eigenpairs (inertia count,
    tests/golden/horn_4m_counts.json), beyond a Krylov basis of 2,048 columns,
    so the time to all eigenpairs is taken on the sub-interval [200, 220]
    (146 eigenpairs by the inertia count) with the same tau and L, for the
    mixed form and for float64 stepping; the line also reports the fused block
    step against the HBM roofline."""
    import numpy as np
    import torch

    from paper_2402_08515_amd import kf
    from synth import power_start, start_block
    from synth.horn import horn_problem

    t0 = time.perf_counter()
    P = horn_problem()
    t_mesh = time.perf_counter() - t0
    lam = kf.estimate_lambda_max(P.S, P.m, 30, power_start(P.n, P.seed))
    tau, L = kf.time_step_rule(lam, P.omega_min)
    lo, hi = args.horn_interval
    with open(os.path.join(ROOT, "tests", "golden", "horn_4m_counts.json")) as f:
        counts = json.load(f)["counts"]
    tgt = counts[repr(float(hi))] - counts[repr(float(lo))]
    print(f"[bench] horn: n={P.n} nnz={P.nnz} (built in {t_mesh:.1f}s) lambda_est={lam:.6g} tau={tau:.6g} L={L}; "
          f"[{lo}, {hi}] holds {tgt} eigenpairs (inertia count)", file=sys.stderr, flush=True)
    V0 = start_block(P.n, P.block, P.seed)
    if args.probe_traffic:
        # counter calibration: one device-to-device copy of exactly 1 GiB read
        # + 1 GiB written, then one filter application of the block (L-1 fused
        # steps) in the variant the autotuner picks here (2 lanes per row)
        prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, precision="mixed", autotune=False,
                          lanes_per_row=2)
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").normal_()
        b = torch.empty_like(a)
        b.copy_(a)
        x = torch.from_numpy(V0).cuda()
        prob.apply_filter(x)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "traffic", "copy_bytes": a.numel() * 8, "workload": "horn_4m", "L": L}))
        return
    V0d = torch.from_numpy(V0).cuda()  # inputs resident in HBM before the timed region
    runs = {}
    for prec in ("mixed", "fp64"):
        prob = kf.Problem(P.S, P.m, lo, hi, tau, L, precision=prec, target=tgt, check_every=2,
                          check_growth=0.15, autotune=not args.no_autotune)
        tuning = prob.tuning()
        # set-up outside the timed region: the block width's step variant
        # (lanes per row, LDS band copy) is timed on its first use
        prob.apply_filter(V0d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = prob.solve(V0d, m_max=2048, tol=args.tol)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        runs[prec] = (r, wall, tuning)
        print(f"[bench] horn {prec}: {r.omega2.size}/{tgt} pairs in {wall:.2f}s ({r.krylov_steps} block iterations, "
              f"basis {r.basis_size}; stepping {r.t_leapfrog:.2f}s, gs {r.t_gs:.2f}s, rr {r.t_rr:.2f}s, refine "
              f"{r.t_refine:.2f}s, escalated {r.escalated})", file=sys.stderr, flush=True)
        del prob
    r, wall, tuning = runs["mixed"]
    r64, wall64, _ = runs["fp64"]
    launches = r.krylov_steps * (L - 1)
    per_launch = r.t_leapfrog / max(launches, 1)
    bytes_step = scope_bytes_per_step(P.n, P.nnz, P.block, 4)
    achieved = bytes_step / per_launch / 1e9
    src = open(os.path.join(ROOT, "paper_2402_08515_amd", "csrc", "kf_step.hip"), "rb").read()
    traffic = traffic_from_profile(hashlib.sha256(src).hexdigest(), "horn_4m")
    out = {
        "metric": METRIC,
        "value": P.n * r.leapfrog_vector_steps / wall,
        "unit": "DOF·timesteps/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-step/f64-proj",
        "data": "synthetic",
        "config": {"workload": "horn_4m", "n": P.n, "nnz": P.nnz, "tets": 3999744, "interval": [lo, hi],
                   "full_interval": [200.0, 600.0], "block": P.block, "tau": tau, "L": L,
                   "target_pairs_inertia": tgt, "parallelism": "1 GPU"},
        "s_to_all_eigenpairs": wall if r.omega2.size >= tgt else None,
        "pairs_accepted": int(r.omega2.size),
        "fp64_s_to_all_eigenpairs": wall64 if r64.omega2.size >= tgt else None,
        "fp64_pairs_accepted": int(r64.omega2.size),
        "mixed_speedup_vs_fp64": wall64 / wall,
        "max_residual": float(r.residual.max()) if r.omega2.size else None,
        "krylov_iters": r.krylov_steps,
        "basis_size": r.basis_size,
        "escalated": bool(r.escalated),
        "leapfrog_only_dof_steps_per_s": P.n * r.leapfrog_vector_steps / r.t_leapfrog,
        "phase_seconds": {"leapfrog": r.t_leapfrog, "gram_schmidt": r.t_gs, "rayleigh_ritz": r.t_rr,
                          "refine": r.t_refine},
        "roofline": {"bound": "hbm", "kernel": "k_leapfrog (block 16, float32)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_step, "avg_launch_us": per_launch * 1e6, "variant": tuning},
    }
    print(json.dumps(out))


def bench_multistep(args):
    """The time loop with several steps per launch (matrix-powers form for
    banded operators) against the one-step kernel: seconds per filter
    application and the scope table's algorithmic bytes per step over that
    time (the one-step roofline; a kernel that keeps the levels on chip can
    pass it).  Cases: the 2D square with 63 cells per side (3,969 rows, band
    63: one workgroup holds the whole problem, the filter is one launch),
    the square with 255 cells per side (65,025 rows, band 255: workgroups
    with halo windows), float64 and float32 stepping; grid3d_96 (band 9,216
    rows) and the horn's block of 16 do not fit a workgroup's LDS and are
    reported as such."""
    import numpy as np
    import torch

    from paper_2402_08515_amd import kf
    from synth import power_start, start_block, workload
    from synth.grids import grid_problem

    cases = []
    P = workload("grid2d_64")
    cases.append(("grid2d_64", P.S, P.m, P.omega_min, P.omega_max, P.seed))
    S, m, h = grid_problem(2, 256)
    cases.append(("grid2d_256", S, m, 30.0, 45.0, 5))
    out = {}
    reps = 20
    for name, S, m, lo, hi, seed in cases:
        n, nnz = S.shape[0], S.nnz
        lam = kf.estimate_lambda_max(S, m, 30, power_start(n, seed))
        tau, L = kf.time_step_rule(lam, lo)
        x = torch.from_numpy(start_block(n, 1, seed)).cuda()
        for prec, vb in (("fp64", 8), ("mixed", 4)):
            row = {}
            for ms in (0, 2, 4, 8, -1):
                try:
                    prob = kf.Problem(S, m, lo, hi, tau, L, precision=prec, multistep=ms)
                    prob.apply_filter(x)  # set-up and warm-up
                except kf.KfError as e:
                    row[str(ms)] = {"error": str(e)}
                    continue
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    prob.apply_filter(x)
                e1.record()
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) * 1e-3 / reps
                bstep = scope_bytes_per_step(n, nnz, 1, vb)
                row[str(ms)] = {"us_per_filter": t * 1e6, "dof_steps_per_s": n * (L - 1) / t,
                                "scope_gbs": bstep * (L - 1) / t / 1e9,
                                "frac_of_hbm_peak": bstep * (L - 1) / t / 1e9 / HBM_PEAK_GBS}
                del prob
            base = row["0"]["us_per_filter"]
            for k, v in row.items():
                if "us_per_filter" in v:
                    v["speedup_vs_one_step"] = base / v["us_per_filter"]
            out[f"{name}/{prec}"] = {"n": n, "nnz": int(nnz), "L": L, "steps_per_launch": row}
            print(f"[bench] multistep {name} {prec} L={L}: " + ", ".join(
                f"s={k}: {v['us_per_filter']:.1f}us" if "us_per_filter" in v else f"s={k}: n/a"
                for k, v in row.items()), file=sys.stderr, flush=True)
    # the benchmark problems whose band does not fit
    P = workload("grid3d_96")
    lam = kf.estimate_lambda_max(P.S, P.m, 30, power_start(P.n, P.seed))
    tau, L = kf.time_step_rule(lam, P.omega_min)
    try:
        prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, multistep=2)
        prob.apply_filter(torch.from_numpy(start_block(P.n, 1, P.seed)).cuda())
        out["grid3d_96"] = {"fits": True}
    except kf.KfError as e:
        out["grid3d_96"] = {"fits": False, "reason": str(e)}
    print(json.dumps({"metric": METRIC, "workload": "multistep", "cases": out}))


def bench_forms(args):
    """The project's forms against the plain method on the same problems:
    the squares of the uneven batch (seed 3; Dirichlet, so every eigenvalue's
    multiplicity is at most 2 and a block of 4 sees whole eigenspaces), each
    solved to all eigenpairs in its interval at residual <= tol:
      plain   float64 stepping, Fourier weights, one problem after another;
      mixed   float32 stepping + float64 projection, all problems batched;
      learned the same with the network's weights where the gate accepts
              them (network trained first, on the spectral range of these
              squares; training time reported separately).
    Every accepted eigenvalue is compared with the closed form."""
    import numpy as np
    import torch

    from paper_2402_08515_amd import kf
    from synth import distinct_target, grid_spectrum, power_start, start_block
    from synth.netinit import init_params
    from synth.workloads import batch64_problems, filter_samples

    probs = [P for P in batch64_problems() if P.meta["dim"] == 2][: args.forms_count]
    members, starts, targets, refs = [], [], [], []
    for P in probs:
        lam = kf.estimate_lambda_max(P.S, P.m, 30, power_start(P.n, P.seed))
        tau, L = kf.time_step_rule(lam, P.omega_min)
        tgt, vals, mult = distinct_target(grid_spectrum(2, P.meta["n"]), P.omega_min, P.omega_max, P.block)
        members.append((P.S, P.m, P.omega_min, P.omega_max, tau, L, tgt, lam))
        starts.append(start_block(P.n, P.block, P.seed))
        targets.append(tgt)
        refs.append(np.repeat(vals, np.minimum(mult, P.block)))
    print(f"[bench] forms: {len(probs)} squares, n in [{min(p.n for p in probs)}, {max(p.n for p in probs)}], "
          f"targets {sum(targets)}", file=sys.stderr, flush=True)

    def score(res):
        found = sum(min(r.omega2.size, t) for r, t in zip(res, targets))
        errs = [np.max(np.abs(r.omega2 - ref) / ref) for r, ref, t in zip(res, refs, targets)
                if r.omega2.size == t and t > 0]
        return int(found), float(max(errs)) if errs else None

    mm = args.m_max
    # plain float64, one by one (problems created before the timed region, as
    # the batches below are)
    probs = [kf.Problem(S, m, lo, hi, tau, L, target=tgt, check_every=2, check_growth=0.1)
             for (S, m, lo, hi, tau, L, tgt, lam) in members]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [pr.solve(V0, m_max=mm, tol=args.tol) for pr, V0 in zip(probs, starts)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # mixed, batched
    opts = dict(precision="mixed", check_every=2, check_growth=0.1)
    bt = kf.Batch([x[:7] for x in members], **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mixed = bt.solve(starts, m_max=mm, tol=args.tol)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    # learned weights, mixed, batched
    lams = [x[7] for x in members]
    train = filter_samples(args.mlp_samples, stream=0, lam_range=(0.9 * min(lams), 1.1 * max(lams)))
    net = kf.Mlp(init_params(4).astype(np.float32))
    rng = np.random.default_rng(np.random.SeedSequence(4).spawn(3)[2])
    order = np.concatenate([rng.permutation(len(train)) for _ in range(args.mlp_epochs)]).astype(np.int32)
    t0 = time.perf_counter()
    net.train(train, order, args.mlp_epochs, 256, 1e-3)
    t_train = time.perf_counter() - t0
    bt2 = kf.Batch([x[:7] for x in members], **opts)
    used = 0
    for q, (S, m, lo, hi, tau, L, tgt, lam) in enumerate(members):
        if L <= 512:
            w, u, jl, jf = net.weights(lo, hi, tau, lam, L)
            bt2.set_weights(q, w)
            used += int(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    learned = bt2.solve(starts, m_max=mm, tol=args.tol)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    rows = {}
    for name, res, t in (("plain_fp64_one_by_one", plain, t_plain), ("mixed_batched", mixed, t_mixed),
                         ("learned_mixed_batched", learned, t_learned)):
        found, err = score(res)
        rows[name] = {"seconds": t, "pairs": found, "max_rel_err_vs_closed_form": err,
                      "krylov_steps": int(sum(r.krylov_steps for r in res)),
                      "dof_steps": float(sum(P.n * r.leapfrog_vector_steps for P, r in zip(probs, res)))}
        print(f"[bench] {name}: {t:.2f}s pairs {found}/{sum(targets)} max err {err}", file=sys.stderr, flush=True)
    rows["learned_mixed_batched"]["members_with_learned_weights"] = used
    rows["learned_mixed_batched"]["train_seconds"] = t_train
    out = {
        "metric": METRIC,
        "value": t_learned,
        "unit": "s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": t_learned * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-step/f64-proj",
        "data": "synthetic",
        "config": {"workload": f"squares of batch64 [:{len(probs)}]", "block": 4, "tol": args.tol, "m_max": mm,
                   "target_pairs": int(sum(targets)), "parallelism": "1 GPU"},
        "forms": rows,
        "speedup_vs_plain": {k: t_plain / v["seconds"] for k, v in rows.items()},
    }
    print(json.dumps(out))


def model_spectrum(dim: int, n: int, top: float, far_every: int = 20):
    """Model spectrum of the convergence model for the square or cube with n
    cells per side: its distinct eigenvalues up to omega = top, every
    far_every-th beyond, standing for far_every eigenvalues each."""
    import numpy as np

    from synth import grid_spectrum

    lam = np.sort(grid_spectrum(dim, n))
    om = np.sqrt(lam[np.concatenate([[True], np.diff(lam) > 1e-10 * lam[1:]])])
    near = om <= top
    far = np.where(~near)[0][::far_every]
    return (np.concatenate([om[near], om[far]]),
            np.concatenate([np.ones(int(near.sum())), far_every * np.ones(far.size)]))


def cube_model_spectrum(n: int, top: float, far_every: int = 20):
    """Model spectrum for the convergence model on the cube with n cells per
    axis: its distinct eigenvalues (a single start vector sees one direction
    per eigenspace), all of them up to omega = top and every far_every-th
    beyond, standing for far_every eigenvalues each."""
    import numpy as np

    from synth import grid_spectrum

    lam = np.sort(grid_spectrum(3, n))
    om = np.sqrt(lam[np.concatenate([[True], np.diff(lam) > 1e-10 * lam[1:]])])
    near = om <= top
    far = np.where(~near)[0][::far_every]
    return (np.concatenate([om[near], om[far]]),
            np.concatenate([np.ones(int(near.sum())), far_every * np.ones(far.size)]))


def bench_learned(args):
    """Learned filter weights on the 3D cube with 128 cells per axis
    (2,048,383 DOFs), float32 time stepping (the mixed form: float64
    refinement, float64 restart when the cube's multiplicities defeat the
    refinement).  The network is trained on the GPU (50,000 samples of
    (omega_min, omega_max, tau, lambda_max), seed 4 stream 0); intervals come
    from the evaluation law (seed 4 stream 1), those holding more than
    --learned-max-target distinct eigenvalues are skipped.  For every interval
    the candidates are the Fourier weights, the network's, and the Gaussian and
    triangle windows; the Krylov convergence model (kf_select_weights, on the
    cube's distinct closed-form spectrum) picks one, the Fourier weights unless
    another is predicted faster.  Timed solves: Fourier, the network's weights
    on their own, and the selected weights."""
    import numpy as np
    import torch

    from paper_2402_08515_amd import kf
    from synth import distinct_target, grid_spectrum, power_start, start_block
    from synth.grids import grid_problem
    from synth.netinit import init_params
    from synth.workloads import filter_samples, grid3d_128_intervals

    train = filter_samples(args.mlp_samples, stream=0)
    net = kf.Mlp(init_params(4).astype(np.float32))
    rng = np.random.default_rng(np.random.SeedSequence(4).spawn(3)[2])
    order = np.concatenate([rng.permutation(len(train)) for _ in range(args.mlp_epochs)]).astype(np.int32)
    t0 = time.perf_counter()
    hist = net.train(train, order, args.mlp_epochs, 256, 1e-3)
    t_train = time.perf_counter() - t0
    print(f"[bench] trained {args.mlp_epochs} epochs on {len(train)} samples in {t_train:.2f}s, "
          f"loss {hist[0]:.4f} -> {hist[-1]:.4f}", file=sys.stderr, flush=True)
    n = args.learned_n
    S, m, h = grid_problem(3, n)
    lam = kf.estimate_lambda_max(S, m, 30, power_start(S.shape[0], 4))
    spec = grid_spectrum(3, n)
    V0 = torch.from_numpy(start_block(S.shape[0], 1, 4)).cuda()  # resident before the timed solves
    names = ["fourier", "network", "gaussian", "triangle"]
    rows = []
    for (lo, hi) in grid3d_128_intervals(32):
        tgt, vals, _ = distinct_target(spec, lo, hi, 1)
        if tgt == 0 or tgt > args.learned_max_target:
            continue
        tau, L = kf.time_step_rule(lam, lo)
        four = kf.window_weights("indicator", lo, hi, tau, L)
        wnet = net.batch_weights(np.array([[lo, hi, tau, lam]]))[0, :L]
        cands = [four, wnet, kf.window_weights("gaussian", lo, hi, tau, L, 1.0),
                 kf.window_weights("triangle", lo, hi, tau, L, 2.0)]
        omod, wmod = cube_model_spectrum(n, 3.0 * hi)
        t1 = time.perf_counter()
        pick, pred = kf.select_weights(cands, tau, lo, hi, omod, wmod, eps=args.tol, kmax=args.learned_m_max,
                                       margin=0.02)
        t_sel = time.perf_counter() - t1
        rec = {"interval": [lo, hi], "target": tgt, "L": L, "selected": names[pick],
               "predicted_steps": dict(zip(names, [int(x) for x in pred])), "select_seconds": t_sel}
        for kind, w in (("fourier", four), ("network", wnet), ("selected", cands[pick])):
            if kind == "selected" and pick in (0, 1):
                rec["selected_run"] = rec["fourier" if pick == 0 else "network"]
                continue
            # set-up (operator, autotuned step) outside the timed region, for every weight set alike
            prob = kf.Problem(S, m, lo, hi, tau, L, precision=args.learned_precision, target=tgt, check_every=2,
                              check_growth=args.learned_check_growth, autotune=True)
            prob.set_weights(w)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = prob.solve(V0, m_max=args.learned_m_max, tol=args.tol)
            dt = time.perf_counter() - t1
            err = None
            if r.omega2.size:
                near = vals[np.abs(r.omega2[:, None] - vals[None, :]).argmin(axis=1)]
                err = float(np.max(np.abs(r.omega2 - near) / near))
            res = {"pairs": int(r.omega2.size), "krylov_steps": r.krylov_steps, "seconds": dt,
                   "escalated": bool(r.escalated), "max_rel_err_vs_closed_form": err}
            rec["selected_run" if kind == "selected" else kind] = res
            del prob
        rows.append(rec)
        print(f"[bench] [{lo:.2f}, {hi:.2f}] target {tgt}: predicted {rec['predicted_steps']} -> "
              f"{rec['selected']}; fourier {rec['fourier']['krylov_steps']} steps {rec['fourier']['seconds']:.2f}s, "
              f"network {rec['network']['krylov_steps']} steps {rec['network']['seconds']:.2f}s, selected "
              f"{rec['selected_run']['seconds']:.2f}s", file=sys.stderr, flush=True)
        if len(rows) >= args.learned_count:
            break
    tot = lambda key, f: sum(r[key][f] for r in rows)  # noqa: E731
    out = {
        "metric": METRIC,
        "value": None,
        "unit": "s",
        "n_gpus": 1,
        "config": {"workload": f"grid3d_{n} learned-vs-Fourier", "intervals": len(rows), "tol": args.tol,
                   "precision": args.learned_precision, "max_target": args.learned_max_target,
                   "m_max": args.learned_m_max, "check_growth": args.learned_check_growth},
        "train_seconds": t_train,
        "train_loss_first_last": [float(hist[0]), float(hist[-1])],
        "fourier_seconds": tot("fourier", "seconds"),
        "network_seconds": tot("network", "seconds"),
        "selected_seconds": tot("selected_run", "seconds"),
        "fourier_krylov_steps": tot("fourier", "krylov_steps"),
        "network_krylov_steps": tot("network", "krylov_steps"),
        "selected_krylov_steps": tot("selected_run", "krylov_steps"),
        "selected_counts": {k: sum(1 for r in rows if r["selected"] == k) for k in names},
        "pairs_all_met": all(r[k]["pairs"] >= r["target"] for r in rows for k in ("fourier", "network", "selected_run")),
        "intervals": rows,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid3d_96")
    ap.add_argument("--m-max", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=2)
    ap.add_argument("--check-growth", type=float, default=0.3)
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--proj-every", type=int, default=12,
                    help="single vectors: steps between projections onto the whole basis")
    ap.add_argument("--no-overlap", action="store_true",
                    help="every Rayleigh-Ritz check stops the Krylov loop (no check on a second stream)")
    ap.add_argument("--gather-unroll", type=int, default=0,
                    help="single vectors: unroll factor (2, 3, 4 or 6) of the fused step's loop over a slice "
                         "(0 = autotuned)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default fused-step variant instead of timing all of them at set-up")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--slice-target", type=int, default=150,
                    help="batch: intervals with more pairs are cut into slices of at most this many")
    ap.add_argument("--no-learned", action="store_true", help="batch: skip the learned-weights run")
    ap.add_argument("--slice-transition", type=float, default=3.0,
                    help="batch: a slice of width d gets L >= 2 pi / (this * d * tau), i.e. a filter transition "
                         "of at most this many slice widths")
    ap.add_argument("--batch-runs", default="mixed,fp64members,fp64batched",
                    help="batch: which batched forms to time (mixed, fp64members, fp64batched; the learned form "
                         "and the one-by-one float64 run have their own switches)")
    ap.add_argument("--batch-check-growth", type=float, default=0.75,
                    help="batch: basis growth between Rayleigh-Ritz checks of a member (their tridiagonalisation and "
                         "inverse iteration dominate the members' device time at small growth)")
    ap.add_argument("--batch-no-restart", action="store_true",
                    help="batch: in the first (mixed) form a member whose float64 refinement misses ends there "
                         "instead of restarting with float64 stepping (the float32 stack alone)")
    ap.add_argument("--batch-workers", type=int, default=0,
                    help="batch: host threads driving the members' projection work (0: min(8, members))")
    ap.add_argument("--mlp-samples", type=int, default=50000)
    ap.add_argument("--mlp-epochs", type=int, default=8)
    ap.add_argument("--learned-n", type=int, default=128)
    ap.add_argument("--learned-count", type=int, default=32)
    ap.add_argument("--learned-max-target", type=int, default=450,
                    help="learned: intervals holding more distinct eigenvalues are skipped (three of the 32 hold "
                         "538-618, beyond what a 2048-column basis resolves with one start vector)")
    ap.add_argument("--learned-m-max", type=int, default=2048, help="learned: basis columns per solve")
    ap.add_argument("--learned-check-growth", type=float, default=0.1,
                    help="learned: basis growth between Rayleigh-Ritz checks")
    ap.add_argument("--learned-precision", default="mixed", choices=("mixed", "fp64"))
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--forms-count", type=int, default=16, help="squares in the forms comparison")
    ap.add_argument("--horn-interval", type=float, nargs=2, default=(200.0, 220.0),
                    help="horn sub-interval solved to completion (ends must be keys of the stored inertia counts)")
    ap.add_argument("--probe-traffic", action="store_true",
                    help="for hardware-counter runs: a few filter applications and a plain copy of known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: one GPU only (--gpus 1); runs on several GPUs are not supported",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        bench_batch(args)
        return
    if args.workload == "learned":
        bench_learned(args)
        return
    if args.workload == "horn_4m":
        bench_horn(args)
        return
    if args.workload == "multistep":
        bench_multistep(args)
        return
    if args.workload == "forms":
        bench_forms(args)
        return

    import numpy as np
    import torch

    from paper_2402_08515_amd import kf
    from synth import distinct_target, grid_spectrum, power_start, start_block, workload

    P = workload(args.workload)
    dim, ncell = P.meta["dim"], P.meta["n"]
    target, vals, mult = distinct_target(grid_spectrum(dim, ncell), P.omega_min, P.omega_max, P.block)
    print(f"[bench] workload {P.name}: n={P.n} nnz={P.nnz} target={target}", file=sys.stderr, flush=True)

    lam = kf.estimate_lambda_max(P.S, P.m, 30, power_start(P.n, P.seed))
    tau, L = kf.time_step_rule(lam, P.omega_min)
    print(f"[bench] lambda_est={lam:.6g} tau={tau:.6g} L={L}", file=sys.stderr, flush=True)
    prob = kf.Problem(P.S, P.m, P.omega_min, P.omega_max, tau, L, precision=P.precision, target=target,
                      check_every=args.check_every, check_growth=args.check_growth, autotune=not args.no_autotune,
                      gather_unroll=args.gather_unroll, overlap_checks=not args.no_overlap,
                      proj_every=args.proj_every)
    tuning = prob.tuning()
    print(f"[bench] fused-step variant {tuning}", file=sys.stderr, flush=True)
    V0 = start_block(P.n, P.block, P.seed)

    if args.probe_traffic:
        # counter calibration: one device-to-device copy of exactly 1 GiB read
        # + 1 GiB written, then 3 filter applications (3*(L-1) fused steps)
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").normal_()
        b = torch.empty_like(a)
        b.copy_(a)
        x = torch.from_numpy(V0).cuda()
        for _ in range(3):
            prob.apply_filter(x)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "traffic", "copy_bytes": a.numel() * 8, "workload": P.name, "L": L}))
        return

    results = []
    V0d = torch.from_numpy(V0).cuda()  # inputs resident in HBM before the timed region
    for i in range(args.warmup):
        r = prob.solve(V0d, m_max=args.m_max, tol=args.tol)
        print(f"[bench] warmup {i}: {r.t_total:.3f}s pairs={r.omega2.size} basis={r.basis_size}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = prob.solve(V0d, m_max=args.m_max, tol=args.tol)
        results.append(r)
        print(f"[bench] step {i}: {r.t_total:.3f}s pairs={r.omega2.size} basis={r.basis_size} "
              f"steps={r.krylov_steps} lf={r.t_leapfrog:.3f}s gs={r.t_gs:.3f}s rr={r.t_rr:.3f}s "
              f"rr beside the loop={r.t_rr_overlapped:.3f}s ({r.overlapped_checks} checks)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    steps_total = sum(r.leapfrog_vector_steps for r in results)
    value = P.n * steps_total / wall
    last = results[-1]
    err = float("nan")
    if last.omega2.size == target:
        expect = np.repeat(vals, np.minimum(mult, P.block))
        err = float(np.max(np.abs(last.omega2 - expect) / expect))

    vb = 8 if P.precision == "fp64" else 4
    launches = sum(r.krylov_steps for r in results) * (L - 1)
    t_lf = sum(r.t_leapfrog for r in results)
    per_launch_s = t_lf / max(launches, 1)
    # the scope table's per-unit figure (five vector streams at every step);
    # the kernel itself touches the weighted sum every third step only, which
    # the second figure counts
    bytes_step = scope_bytes_per_step(P.n, P.nnz, P.block, vb)
    kernel_bytes_step = algorithmic_bytes_per_step(P.n, P.nnz, P.block, vb, L)
    achieved = bytes_step / per_launch_s / 1e9
    src = open(os.path.join(ROOT, "paper_2402_08515_amd", "csrc", "kf_step.hip"), "rb").read()
    traffic = traffic_from_profile(hashlib.sha256(src).hexdigest(), P.name)
    copy_gbs = measured_copy_gbs()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF·timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if P.precision == "fp64" else "f32-step/f64-proj",
        "data": "synthetic",
        "config": {
            "workload": P.name,
            "n": P.n,
            "nnz": P.nnz,
            "interval": [P.omega_min, P.omega_max],
            "block": P.block,
            "tau": tau,
            "L": L,
            "tol": args.tol,
            "target_pairs": target,
            "parallelism": "1 GPU",
        },
        "s_to_all_eigenpairs": wall / args.steps,
        "pairs_accepted": int(last.omega2.size),
        "max_rel_eig_err_vs_closed_form": err,
        "max_residual": float(last.residual.max()) if last.omega2.size else None,
        "krylov_steps": last.krylov_steps,
        "basis_size": last.basis_size,
        "leapfrog_only_dof_steps_per_s": P.n * steps_total / t_lf,
        "phase_seconds_per_solve": {
            "leapfrog": t_lf / args.steps,
            "gram_schmidt": sum(r.t_gs for r in results) / args.steps,
            "rayleigh_ritz": sum(r.t_rr for r in results) / args.steps,
            "rayleigh_ritz_overlapped": sum(r.t_rr_overlapped for r in results) / args.steps,
        },
        "overlapped_checks": last.overlapped_checks,
        # share of the solve's wall time outside the fused time steps
        # (Gram-Schmidt, the Rayleigh-Ritz work the loop waits for, launch
        # and host gaps)
        "non_leapfrog_fraction": 1.0 - t_lf / wall,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_leapfrog",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": bytes_step,
            "bytes_per_launch_model": "scope table per vector-DOF-step figure x N x b",
            "kernel_bytes_per_launch": kernel_bytes_step,
            "kernel_bytes_frac": kernel_bytes_step / per_launch_s / 1e9 / HBM_PEAK_GBS,
            "avg_launch_us": per_launch_s * 1e6,
            "variant": tuning,
            "copy_measured": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, tau, L, V0, args.cpu_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
