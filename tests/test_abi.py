"""The C-ABI library on the CPU: it loads, exports every entry point that
include/kf.h declares, and rejects invalid input before touching a device."""

import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from synth.grids import grid_problem


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def _declared(repo_root):
    txt = open(os.path.join(repo_root, "include", "kf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(kf_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(repo_root):
    kf = _kf()
    names = _declared(repo_root)
    assert len(names) >= 13
    lib = kf.lib()
    for nm in names:
        assert hasattr(lib, nm), nm
    out = subprocess.run(["nm", "-D", "--defined-only", kf.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (kf_[a-z_]+)", out))
    assert set(names) <= exported


def test_time_step_rule_matches_oracle():
    kf = _kf()
    for lam, om in [(32028.459056753818, 10.0), (1.1e5, 30.0), (4.0, 0.5)]:
        assert kf.time_step_rule(lam, om) == pytest.approx(oracle.time_step_rule(lam, om))
    with pytest.raises(kf.KfError):
        kf.time_step_rule(-1.0, 10.0)
    with pytest.raises(kf.KfError):
        kf.time_step_rule(1.0, 0.0)


@pytest.fixture(scope="module")
def small():
    S, m, h = grid_problem(2, 8)
    return S, m


def _expect_einval(fn):
    kf = _kf()
    with pytest.raises(kf.KfError) as ei:
        fn()
    assert ei.value.code == kf.KF_EINVAL
    return str(ei.value)


def test_create_rejects_bad_pencils(small):
    kf = _kf()
    S, m = small
    assert "m_diag" in _expect_einval(lambda: kf.Problem(S, -m, 1.0, 2.0, 0.01, 10))
    m2 = m.copy()
    m2[3] = np.inf
    _expect_einval(lambda: kf.Problem(S, m2, 1.0, 2.0, 0.01, 10))
    S2 = S.copy()
    S2.indices[3], S2.indices[4] = S2.indices[4], S2.indices[3]
    assert "increasing" in _expect_einval(lambda: kf.Problem(S2, m, 1.0, 2.0, 0.01, 10))
    S3 = S.copy()
    S3.data[5] = np.nan
    assert "non-finite" in _expect_einval(lambda: kf.Problem(S3, m, 1.0, 2.0, 0.01, 10))
    S4 = S.copy()
    S4.indices[0] = S.shape[0]
    assert "range" in _expect_einval(lambda: kf.Problem(S4, m, 1.0, 2.0, 0.01, 10))


def test_create_rejects_bad_parameters(small):
    kf = _kf()
    S, m = small
    _expect_einval(lambda: kf.Problem(S, m, 2.0, 1.0, 0.01, 10))
    _expect_einval(lambda: kf.Problem(S, m, -1.0, 1.0, 0.01, 10))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.0, 10))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, float("nan"), 10))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 0))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 10, index_bytes=3))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 10, reorth_tol=-1.0))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 10, reorth_tol=float("inf")))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 10, lanes_per_row=3))
    assert "gather_unroll" in _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 10, gather_unroll=1))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 10, gather_unroll=5))
    _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 10, gather_unroll=8))
    assert "block_band" in _expect_einval(lambda: kf.Problem(S, m, 1.0, 2.0, 0.01, 10, block_band=2))


def test_default_options_fill_the_bindings_structure():
    """kf_default_options writes through the binding's copy of kf_options:
    every default lands in its own field, so the two layouts agree."""
    import ctypes

    kf = _kf()
    o = kf.OptionsT()
    kf.lib().kf_default_options(ctypes.byref(o))
    got = {f: getattr(o, f) for f, _ in kf.OptionsT._fields_}
    want = {"precision": 0, "check_every": 1, "check_growth": 0.3, "full_reorth": 0, "target": 0, "max_iters": 0,
            "drop_tol": 1e-10, "reorth_tol": 1e-9, "proj_every": 12, "refine": 8, "escalate": 1, "want_vectors": 0,
            "index_bytes": 0, "xcd_remap": 1, "nt_loads": 0, "autotune": 0, "batch_workers": 0, "lanes_per_row": 0,
            "gather_unroll": 0, "block_band": 0, "stepper": 2, "overlap_checks": 1, "multistep": 0, "stream": None}
    assert got == want


def test_last_error_is_a_string():
    kf = _kf()
    assert isinstance(kf.last_error(), str)


def test_sym_eig_validation():
    from paper_2402_08515_amd import kf

    _expect_einval(lambda: kf.sym_eig(np.zeros((0, 0))))
    A = np.eye(3)
    A[1, 2] = np.nan
    assert "non-finite" in _expect_einval(lambda: kf.sym_eig(A))
    _expect_einval(lambda: kf.sym_eig(np.eye(2049)))
