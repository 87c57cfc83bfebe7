"""ctypes binding of libkf.so (argument marshalling only).

Every computation happens in the HIP library; this module converts NumPy /
SciPy / torch objects to the plain pointers and sizes of ``include/kf.h`` and
back.  torch is imported first so that the process has one HIP runtime (the
one torch loaded) and so that device blocks can be handed over as torch
tensors on the current stream.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

import torch  # loads torch's HIP runtime before libkf.so; device start blocks

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkf.so")

KF_OK, KF_EINVAL, KF_ENOMEM, KF_EHIP, KF_EUNSTABLE, KF_EBREAKDOWN, KF_ENOTCONV = range(7)
KF_FP64, KF_MIXED = 0, 1
_PREC = {"fp64": KF_FP64, "mixed": KF_MIXED}


class KfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[kf status {code}] {msg}")
        self.code = code


class CsrT(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("nnz", C.c_int64),
        ("rowptr", C.c_void_p),
        ("col", C.c_void_p),
        ("val", C.c_void_p),
        ("on_device", C.c_int32),
    ]


class OptionsT(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("check_every", C.c_int32),
        ("check_growth", C.c_double),
        ("full_reorth", C.c_int32),
        ("target", C.c_int32),
        ("max_iters", C.c_int32),
        ("drop_tol", C.c_double),
        ("reorth_tol", C.c_double),
        ("proj_every", C.c_int32),
        ("refine", C.c_int32),
        ("escalate", C.c_int32),
        ("want_vectors", C.c_int32),
        ("index_bytes", C.c_int32),
        ("xcd_remap", C.c_int32),
        ("nt_loads", C.c_int32),
        ("autotune", C.c_int32),
        ("batch_workers", C.c_int32),
        ("lanes_per_row", C.c_int32),
        ("gather_unroll", C.c_int32),
        ("block_band", C.c_int32),
        ("stepper", C.c_int32),
        ("overlap_checks", C.c_int32),
        ("multistep", C.c_int32),
        ("stream", C.c_void_p),
    ]


class ResultT(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("n_pairs", C.c_int32),
        ("omega2", C.POINTER(C.c_double)),
        ("omega", C.POINTER(C.c_double)),
        ("residual", C.POINTER(C.c_double)),
        ("vectors", C.POINTER(C.c_double)),
        ("n_ritz", C.c_int32),
        ("ritz", C.POINTER(C.c_double)),
        ("krylov_steps", C.c_int32),
        ("basis_size", C.c_int32),
        ("breakdown", C.c_int32),
        ("status", C.c_int32),
        ("leapfrog_vector_steps", C.c_int64),
        ("t_total", C.c_double),
        ("t_leapfrog", C.c_double),
        ("t_gs", C.c_double),
        ("t_rr", C.c_double),
        ("t_refine", C.c_double),
        ("orth_error", C.c_double),
        ("full_passes", C.c_int32),
        ("refine_vector_steps", C.c_int64),
        ("escalated", C.c_int32),
        ("t_rr_overlapped", C.c_double),
        ("overlapped_checks", C.c_int32),
    ]


class ProblemDescT(C.Structure):
    _fields_ = [
        ("S", CsrT),
        ("m_diag", C.c_void_p),
        ("omega_min", C.c_double),
        ("omega_max", C.c_double),
        ("tau", C.c_double),
        ("L", C.c_int32),
        ("target", C.c_int32),
        ("step_fp64", C.c_int32),
    ]


_lib = None

_SIGNATURES = {
    "kf_default_options": (None, [C.POINTER(OptionsT)]),
    "kf_last_error": (C.c_char_p, []),
    "kf_create": (
        C.c_int,
        [C.POINTER(CsrT), C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int32, C.POINTER(OptionsT),
         C.POINTER(C.c_void_p)],
    ),
    "kf_destroy": (C.c_int, [C.c_void_p]),
    "kf_set_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "kf_get_weights": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kf_estimate_lambda_max": (
        C.c_int, [C.POINTER(CsrT), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
    ),
    "kf_time_step_rule": (C.c_int, [C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "kf_filter_response": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "kf_window_weights": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_double,
                                    C.c_void_p]),
    "kf_predict_steps": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_double, C.c_int32,
                                   C.c_double, C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_int32)]),
    "kf_select_weights": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_double,
                                    C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_double,
                                    C.POINTER(C.c_int32), C.c_void_p]),
    "kf_notch_weights": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_int32, C.c_void_p]),
    "kf_apply_filter": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "kf_apply_filter_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "kf_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.POINTER(C.POINTER(ResultT))]),
    "kf_result_free": (C.c_int, [C.POINTER(ResultT)]),
    "kf_subspace_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_double,
                                    C.POINTER(C.POINTER(ResultT))]),
    "kf_tune_steps": (C.c_int, [C.POINTER(CsrT), C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.POINTER(OptionsT),
                                C.POINTER(C.c_int32), C.c_void_p, C.c_void_p]),
    "kf_copy_basis": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "kf_sym_eig": (C.c_int, [C.c_int32, C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.POINTER(C.c_int32),
                             C.c_void_p, C.c_void_p]),
    "kf_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "kf_create_batch": (C.c_int, [C.c_int32, C.c_void_p, C.POINTER(OptionsT), C.POINTER(C.c_void_p)]),
    "kf_destroy_batch": (C.c_int, [C.c_void_p]),
    "kf_batch_set_weights": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    "kf_batch_apply_filter": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "kf_solve_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_void_p]),
    "kf_mlp_param_count": (C.c_int32, []),
    "kf_mlp_create": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "kf_mlp_destroy": (C.c_int, [C.c_void_p]),
    "kf_mlp_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kf_mlp_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_void_p]),
    "kf_mlp_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_double,
                               C.c_void_p]),
    "kf_mlp_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "kf_weights_from_mlp": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                                      C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
}


def lib():
    """Load libkf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().kf_last_error().decode()


def _check(code: int):
    if code not in (KF_OK,):
        raise KfError(code, last_error())


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _host_csr(S):
    import scipy.sparse as sp

    S = sp.csr_matrix(S)
    rowptr = np.ascontiguousarray(S.indptr, dtype=np.int32)
    col = np.ascontiguousarray(S.indices, dtype=np.int32)
    val = np.ascontiguousarray(S.data, dtype=np.float64)
    keep = (rowptr, col, val)
    c = CsrT(S.shape[0], int(S.nnz), _ptr(rowptr), _ptr(col), _ptr(val), 0)
    return c, keep


def _stream_handle() -> int:
    # the legacy default stream (0) when torch sees no device: validation
    # errors are raised before any device call
    if not torch.cuda.is_available():
        return 0
    return torch.cuda.current_stream().cuda_stream


def sym_eig(A, lo: float = 0.0, hi: float = -1.0, vectors: bool = False):
    """All eigenvalues (ascending) of the dense symmetric matrix A with the
    library's GPU eigensolver; with vectors=True also the eigenvectors of the
    eigenvalues in [lo, hi] (k x count)."""
    a = np.asfortranarray(A, dtype=np.float64)
    k = a.shape[0]
    if a.shape != (k, k):
        raise ValueError("A must be square")
    theta = np.empty(k)
    nsel = C.c_int32(0)
    Y = np.empty((k, k), order="F") if vectors else None
    _check(lib().kf_sym_eig(k, _ptr(a), lo, hi, _ptr(theta), C.byref(nsel), _ptr(Y) if vectors else None,
                            _stream_handle()))
    if vectors:
        return theta, np.ascontiguousarray(Y[:, : nsel.value])
    return theta


def tune_steps(S, m, omega_min: float, omega_max: float, tau: float, L_candidates, start, m_max: int, tol: float,
               **options):
    """The L among the candidates whose solve meets options['target'] fastest;
    returns (L_best, seconds per candidate, Krylov steps per candidate)."""
    c, keep = _host_csr(S)
    m = np.ascontiguousarray(m, dtype=np.float64)
    Lc = np.ascontiguousarray(L_candidates, dtype=np.int32)
    V0 = np.ascontiguousarray(start, dtype=np.float64)
    if V0.ndim == 1:
        V0 = V0[:, None]
    opt = _options(**options)
    best = C.c_int32()
    secs = np.zeros(Lc.size)
    its = np.zeros(Lc.size, dtype=np.int32)
    _check(lib().kf_tune_steps(C.byref(c), _ptr(m), float(omega_min), float(omega_max), float(tau), _ptr(Lc),
                               int(Lc.size), _ptr(V0), int(V0.shape[1]), int(m_max), float(tol), C.byref(opt),
                               C.byref(best), _ptr(secs), _ptr(its)))
    return best.value, secs, its


WINDOWS = {"indicator": 0, "triangle": 1, "gaussian": 2}


def window_weights(kind: str, omega_min: float, omega_max: float, tau: float, L: int, width: float = 1.0):
    """Filter coefficients tau*alpha(l tau), l < L, of an analytic window."""
    out = np.empty(int(L))
    _check(lib().kf_window_weights(WINDOWS[kind], float(omega_min), float(omega_max), float(tau), int(L),
                                   float(width), _ptr(out)))
    return out


def predict_steps(omega, weight, w, tau: float, omega_min: float, omega_max: float, eps: float = 1e-6,
                  kmax: int = 2000, stepper: int = 2) -> int:
    """Krylov steps the convergence model predicts for the weights w."""
    om = np.ascontiguousarray(omega, dtype=np.float64)
    wt = np.ascontiguousarray(weight, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = C.c_int32()
    _check(lib().kf_predict_steps(_ptr(om), _ptr(wt), int(om.size), _ptr(w), int(w.size), float(tau), int(stepper),
                                  float(omega_min), float(omega_max), float(eps), int(kmax), C.byref(out)))
    return out.value


def select_weights(candidates, tau: float, omega_min: float, omega_max: float, omega, weight, eps: float = 1e-6,
                   kmax: int = 2000, margin: float = 0.0, stepper: int = 2):
    """Index of the candidate weight set to use (0, the Fourier weights, unless
    another is predicted faster) and the predicted steps of each."""
    cs = [np.ascontiguousarray(c, dtype=np.float64) for c in candidates]
    L = cs[0].size
    if any(c.size != L for c in cs):
        raise ValueError("candidates must have the same length")
    arr = (C.c_void_p * len(cs))(*[c.ctypes.data for c in cs])
    om = np.ascontiguousarray(omega, dtype=np.float64)
    wt = np.ascontiguousarray(weight, dtype=np.float64)
    chosen = C.c_int32()
    steps = np.zeros(len(cs), dtype=np.int32)
    _check(lib().kf_select_weights(C.cast(arr, C.c_void_p), len(cs), L, float(tau), int(stepper), float(omega_min),
                                   float(omega_max), _ptr(om), _ptr(wt), int(om.size), float(eps), int(kmax),
                                   float(margin), C.byref(chosen), _ptr(steps)))
    return chosen.value, steps


def notch_weights(w, tau: float, omegas):
    """The weights nearest to w whose filter vanishes at the given omegas."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    om = np.ascontiguousarray(np.atleast_1d(omegas), dtype=np.float64)
    out = np.empty_like(w)
    _check(lib().kf_notch_weights(_ptr(w), int(w.size), float(tau), _ptr(om), int(om.size), _ptr(out)))
    return out


def time_step_rule(lambda_est: float, omega_min: float, safety: float = 0.9):
    tau = C.c_double()
    L = C.c_int32()
    _check(lib().kf_time_step_rule(lambda_est, omega_min, safety, C.byref(tau), C.byref(L)))
    return tau.value, L.value


def estimate_lambda_max(S, m, iters: int, x0) -> float:
    c, keep = _host_csr(S)
    m = np.ascontiguousarray(m, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    out = C.c_double()
    _check(lib().kf_estimate_lambda_max(C.byref(c), _ptr(m), iters, _ptr(x0), _stream_handle(), C.byref(out)))
    return out.value


@dataclass
class SolveResult:
    omega2: np.ndarray
    omega: np.ndarray
    residual: np.ndarray
    vectors: np.ndarray | None
    ritz: np.ndarray
    krylov_steps: int
    basis_size: int
    breakdown: bool
    status: int
    leapfrog_vector_steps: int
    t_total: float
    t_leapfrog: float
    t_gs: float
    t_rr: float
    t_refine: float
    orth_error: float
    full_passes: int
    refine_vector_steps: int
    escalated: bool
    t_rr_overlapped: float = 0.0
    overlapped_checks: int = 0


def _take_result(res, n: int) -> SolveResult:
    """Copy a library-owned kf_result into Python objects and free it."""
    try:
        r = res.contents
        na = r.n_pairs
        vec = None
        if r.vectors:
            vec = np.ctypeslib.as_array(r.vectors, shape=(na, n)).T.copy()
        return SolveResult(
            omega2=np.ctypeslib.as_array(r.omega2, shape=(na,)).copy() if na else np.zeros(0),
            omega=np.ctypeslib.as_array(r.omega, shape=(na,)).copy() if na else np.zeros(0),
            residual=np.ctypeslib.as_array(r.residual, shape=(na,)).copy() if na else np.zeros(0),
            vectors=vec,
            ritz=np.ctypeslib.as_array(r.ritz, shape=(r.n_ritz,)).copy() if r.n_ritz else np.zeros(0),
            krylov_steps=r.krylov_steps,
            basis_size=r.basis_size,
            breakdown=bool(r.breakdown),
            status=r.status,
            leapfrog_vector_steps=r.leapfrog_vector_steps,
            t_total=r.t_total,
            t_leapfrog=r.t_leapfrog,
            t_gs=r.t_gs,
            t_rr=r.t_rr,
            t_refine=r.t_refine,
            orth_error=r.orth_error,
            full_passes=r.full_passes,
            refine_vector_steps=r.refine_vector_steps,
            escalated=bool(r.escalated),
            t_rr_overlapped=r.t_rr_overlapped,
            overlapped_checks=r.overlapped_checks,
        )
    finally:
        lib().kf_result_free(res)


def _options(precision="fp64", check_every=1, check_growth=0.3, full_reorth=False, target=0, max_iters=0,
             drop_tol=1e-10, refine=None, want_vectors=False, index_bytes=0, xcd_remap=True, nt_loads=False,
             autotune=False, reorth_tol=None, lanes_per_row=0, batch_workers=0, proj_every=None, gather_unroll=0,
             block_band=0, escalate=None, stepper=2, overlap_checks=None, multistep=0):
    opt = OptionsT()
    lib().kf_default_options(C.byref(opt))
    opt.precision = _PREC[precision]
    opt.check_every = check_every
    opt.check_growth = check_growth
    opt.full_reorth = int(full_reorth)
    opt.target = target
    opt.max_iters = max_iters
    opt.drop_tol = drop_tol
    if reorth_tol is not None:
        opt.reorth_tol = reorth_tol
    if proj_every is not None:
        opt.proj_every = proj_every
    if refine is not None:
        opt.refine = int(refine)
    if escalate is not None:
        opt.escalate = int(escalate)
    opt.want_vectors = int(want_vectors)
    opt.index_bytes = index_bytes
    opt.xcd_remap = int(xcd_remap)
    opt.nt_loads = int(nt_loads)
    opt.autotune = int(autotune)
    opt.lanes_per_row = int(lanes_per_row)
    opt.gather_unroll = int(gather_unroll)
    opt.block_band = int(block_band)
    opt.stepper = int(stepper)
    if overlap_checks is not None:
        opt.overlap_checks = int(overlap_checks)
    opt.multistep = int(multistep)
    opt.batch_workers = int(batch_workers)
    opt.stream = _stream_handle()
    return opt


class Batch:
    """Handle of ``kf_create_batch``: independent problems whose time loops
    advance in one batched launch.  ``members`` is a list of tuples
    (S, m, omega_min, omega_max, tau, L, target[, step_fp64]); members that
    pass the same S and m objects share one converted copy (the library
    then knows them as slices of one operator)."""

    def __init__(self, members, **options):
        L_ = lib()
        self._h = C.c_void_p()
        self._keep = []
        descs = (ProblemDescT * len(members))()
        self.n = []
        conv = {}
        for i, mem in enumerate(members):
            S, m, omin, omax, tau, L, target = mem[:7]
            fp64 = int(bool(mem[7])) if len(mem) > 7 else 0
            key = (id(S), id(m))
            if key not in conv:
                c, keep = _host_csr(S)
                mm = np.ascontiguousarray(m, dtype=np.float64)
                conv[key] = (c, keep, mm)
            c, keep, mm = conv[key]
            self._keep.append((keep, mm))
            descs[i] = ProblemDescT(c, _ptr(mm), float(omin), float(omax), float(tau), int(L), int(target), fp64)
            self.n.append(S.shape[0])
        opt = _options(**options)
        _check(L_.kf_create_batch(len(members), C.cast(descs, C.c_void_p), C.byref(opt), C.byref(self._h)))
        self._keep = None
        self.P = len(members)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().kf_destroy_batch(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, q: int, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        _check(lib().kf_batch_set_weights(self._h, int(q), _ptr(w), int(w.size)))

    def apply_filter(self, xs):
        """ys[p] = C_p xs[p] for device blocks xs[p] of shape (n_p, b),
        float64; one batched application."""
        b = int(xs[0].shape[1])
        cols = [x.t().contiguous() for x in xs]  # column-major n x b
        outs = [torch.empty_like(c) for c in cols]
        xp = (C.c_void_p * self.P)(*[c.data_ptr() for c in cols])
        yp = (C.c_void_p * self.P)(*[o.data_ptr() for o in outs])
        _check(lib().kf_batch_apply_filter(self._h, C.cast(xp, C.c_void_p), C.cast(yp, C.c_void_p), b))
        return [o.t().contiguous() for o in outs]

    def solve(self, starts, m_max: int, tol: float):
        arrs = [np.ascontiguousarray(v[:, None] if v.ndim == 1 else v, dtype=np.float64) for v in starts]
        b = arrs[0].shape[1]
        sp = (C.c_void_p * self.P)(*[a.ctypes.data for a in arrs])
        res = (C.POINTER(ResultT) * self.P)()
        _check(lib().kf_solve_batch(self._h, C.cast(sp, C.c_void_p), int(b), int(m_max), float(tol),
                                    C.cast(res, C.c_void_p)))
        return [_take_result(res[i], self.n[i]) for i in range(self.P)]


class Problem:
    """Handle of ``kf_create``: pencil, interval, tau, L and options."""

    def __init__(self, S, m, omega_min: float, omega_max: float, tau: float, L: int, **options):
        L_ = lib()
        self._h = C.c_void_p()
        opt = _options(**options)
        precision = options.get("precision", "fp64")
        c, keep = _host_csr(S)
        m = np.ascontiguousarray(m, dtype=np.float64)
        _check(L_.kf_create(C.byref(c), _ptr(m), omega_min, omega_max, tau, L, C.byref(opt), C.byref(self._h)))
        self.n = S.shape[0]
        self.L = L
        self.tau = tau
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().kf_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tuning(self) -> dict:
        r, nt, ib, u = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        us = C.c_double()
        _check(lib().kf_get_tuning(self._h, C.byref(r), C.byref(nt), C.byref(ib), C.byref(u), C.byref(us)))
        return {"xcd_remap": r.value, "nt_loads": nt.value, "index_bytes": ib.value, "gather_unroll": u.value,
                "us_per_step": us.value}

    def weights(self) -> np.ndarray:
        w = np.empty(self.L)
        _check(lib().kf_get_weights(self._h, _ptr(w)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        _check(lib().kf_set_weights(self._h, _ptr(w), int(w.size)))

    def filter_response(self, omega) -> np.ndarray:
        om = np.ascontiguousarray(np.atleast_1d(omega), dtype=np.float64)
        out = np.empty_like(om)
        _check(lib().kf_filter_response(self._h, _ptr(om), int(om.size), _ptr(out)))
        return out

    def apply_filter(self, x: torch.Tensor) -> torch.Tensor:
        """y = C x for a device block x (n x b float64, contiguous)."""
        if x.dim() == 1:
            x = x[:, None]
        if x.device.type != "cuda" or x.dtype != torch.float64 or not x.is_contiguous() or x.shape[0] != self.n:
            raise ValueError("x must be a contiguous float64 CUDA tensor with n rows")
        y = torch.empty_like(x)
        _check(lib().kf_apply_filter(self._h, x.data_ptr(), y.data_ptr(), int(x.shape[1])))
        return y

    def apply_filter_noalloc(self, x: torch.Tensor, y: torch.Tensor) -> None:
        """y = C x into the caller's device block y (both n x b float64,
        contiguous), with no device allocation in the library."""
        if x.dim() == 1:
            x, y = x[:, None], y[:, None]
        for t in (x, y):
            if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous() or t.shape[0] != self.n:
                raise ValueError("x and y must be contiguous float64 CUDA tensors with n rows")
        if x.shape != y.shape:
            raise ValueError("x and y must have the same shape")
        _check(lib().kf_apply_filter_noalloc(self._h, x.data_ptr(), y.data_ptr(), int(x.shape[1])))

    def solve(self, start, m_max: int, tol: float) -> SolveResult:
        """start: n x b float64 block, a host array or a contiguous CUDA tensor."""
        if isinstance(start, torch.Tensor) and start.is_cuda:
            V0 = start if start.dim() == 2 else start[:, None]
            if V0.dtype != torch.float64 or not V0.is_contiguous() or V0.shape[0] != self.n:
                raise ValueError("start must be a contiguous float64 tensor with n rows")
            ptr, b = V0.data_ptr(), int(V0.shape[1])
        else:
            V0 = np.ascontiguousarray(start, dtype=np.float64)
            if V0.ndim == 1:
                V0 = V0[:, None]
            ptr, b = _ptr(V0), int(V0.shape[1])
        res = C.POINTER(ResultT)()
        _check(lib().kf_solve(self._h, ptr, b, int(m_max), float(tol), C.byref(res)))
        return _take_result(res, self.n)

    def subspace_solve(self, start, max_iters: int, tol: float) -> SolveResult:
        """Fixed-dimension filtered subspace iteration from the n x ncols block
        start (host array or contiguous CUDA tensor, float64)."""
        if isinstance(start, torch.Tensor) and start.is_cuda:
            X0 = start if start.dim() == 2 else start[:, None]
            if X0.dtype != torch.float64 or not X0.is_contiguous() or X0.shape[0] != self.n:
                raise ValueError("start must be a contiguous float64 tensor with n rows")
            ptr, nc = X0.data_ptr(), int(X0.shape[1])
        else:
            X0 = np.ascontiguousarray(start, dtype=np.float64)
            if X0.ndim == 1:
                X0 = X0[:, None]
            ptr, nc = _ptr(X0), int(X0.shape[1])
        res = C.POINTER(ResultT)()
        _check(lib().kf_subspace_solve(self._h, ptr, nc, int(max_iters), float(tol), C.byref(res)))
        return _take_result(res, self.n)

    def basis(self, max_cols: int) -> np.ndarray:
        out = np.empty((max_cols, self.n))
        nc = C.c_int32()
        _check(lib().kf_copy_basis(self._h, _ptr(out), int(max_cols), C.byref(nc)))
        return out[: nc.value].T.copy()


class Mlp:
    """Handle of ``kf_mlp_create``: the learned filter-weight network
    (parameters float32, layout W1[64x128] b1 W2 b2 W3 b3 W4[128x512] b4)."""

    def __init__(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != lib().kf_mlp_param_count():
            raise ValueError("wrong parameter count")
        self._h = C.c_void_p()
        _check(lib().kf_mlp_create(_ptr(p), C.byref(self._h)))

    @staticmethod
    def param_count() -> int:
        return int(lib().kf_mlp_param_count())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().kf_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(self.param_count(), dtype=np.float32)
        _check(lib().kf_mlp_get_params(self._h, _ptr(out)))
        return out

    def loss_grad(self, samples, want_grad=True):
        s = np.ascontiguousarray(samples, dtype=np.float64)
        loss = C.c_double()
        g = np.empty(self.param_count(), dtype=np.float32) if want_grad else None
        _check(lib().kf_mlp_loss_grad(self._h, _ptr(s), int(s.shape[0]), C.byref(loss), _ptr(g) if want_grad else None))
        return loss.value, g

    def train(self, samples, order, epochs: int, batch: int, lr: float) -> np.ndarray:
        s = np.ascontiguousarray(samples, dtype=np.float64)
        o = np.ascontiguousarray(order, dtype=np.int32)
        hist = np.zeros(epochs)
        _check(lib().kf_mlp_train(self._h, _ptr(s), int(s.shape[0]), _ptr(o), int(epochs), int(batch), float(lr),
                                  _ptr(hist)))
        return hist

    def batch_weights(self, samples) -> np.ndarray:
        """The network's weights (n x 512, no gate) for n sample rows."""
        s = np.ascontiguousarray(samples, dtype=np.float64)
        out = np.empty((s.shape[0], 512))
        _check(lib().kf_mlp_weights(self._h, _ptr(s), int(s.shape[0]), _ptr(out)))
        return out

    def weights(self, omega_min, omega_max, tau, lambda_max, L):
        w = np.empty(int(L))
        used = C.c_int32()
        jl = C.c_double()
        jf = C.c_double()
        _check(lib().kf_weights_from_mlp(self._h, omega_min, omega_max, tau, lambda_max, int(L), _ptr(w),
                                         C.byref(used), C.byref(jl), C.byref(jf)))
        return w, bool(used.value), jl.value, jf.value
