"""Eigenvalue counts by Sylvester's law of inertia (TEST INFRASTRUCTURE).

The pencil (S, M) of Section 2 has S symmetric positive semi-definite and M
diagonal positive (Remark 2.1); S - sigma M = L D L^T is congruent to D, so
its negative pivots count the eigenvalues omega^2 < sigma.  The count pins
the completeness of a solve on meshes without a closed-form spectrum: the
number of eigenvalues in [omega_min, omega_max] is
count(omega_max^2 (1 + eps)) - count(omega_min^2 (1 - eps)).

The factorisation is the plain C routine in ``inertia.c`` (banded, no
pivoting), compiled with gcc into ``_inertia.so`` next to this file on first
use (``build()`` compiles it beforehand).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "inertia.c")
_LIB = os.path.join(_HERE, "_inertia.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-O3", "-march=native", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        lib.kf_oracle_inertia.restype = C.c_int64
        lib.kf_oracle_inertia.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                          C.c_int32]
        _lib = lib
    return _lib


def bandwidth(S) -> int:
    S = sp.coo_matrix(S)
    return int(np.abs(S.row - S.col).max()) if S.nnz else 0


def count_below(S, m, sigma: float) -> int:
    """Number of eigenvalues omega^2 < sigma of S v = omega^2 diag(m) v."""
    S = sp.csr_matrix(S)
    rowptr = np.ascontiguousarray(S.indptr, dtype=np.int32)
    col = np.ascontiguousarray(S.indices, dtype=np.int32)
    val = np.ascontiguousarray(S.data, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.float64)
    r = _load().kf_oracle_inertia(S.shape[0], rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, m.ctypes.data,
                                  float(sigma), bandwidth(S))
    if r == -2:
        raise ArithmeticError(f"zero pivot at sigma = {sigma}: move sigma off the eigenvalue")
    if r < 0:
        raise RuntimeError(f"inertia count failed ({r})")
    return int(r)


def count_in_interval(S, m, omega_min: float, omega_max: float, rel: float = 1e-9) -> int:
    """Eigenvalues with omega in [omega_min, omega_max] (closed, widened by
    ``rel`` relative on the omega^2 axis so that a pair on an end counts)."""
    return count_below(S, m, omega_max**2 * (1 + rel)) - count_below(S, m, omega_min**2 * (1 - rel))
