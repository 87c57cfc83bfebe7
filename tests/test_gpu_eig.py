"""The projected-pencil eigensolver (kf_sym_eig: Householder
tridiagonalisation on one workgroup below order 48 and one launch per
reflector above, bisection, inverse iteration, back-transformation) on
matrices whose spectrum is fixed by construction, A = Q diag(lam) Q^T."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def _matrix(k, seed, clusters=True):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(-3.0, 5.0, size=k))
    if clusters and k >= 8:
        lam[k // 3 : k // 3 + 3] = lam[k // 3]  # a triple eigenvalue
        lam[k // 2 + 1] = lam[k // 2] * (1 + 1e-11)  # a tight pair
        lam = np.sort(lam)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return (Q * lam) @ Q.T, lam


@pytest.mark.parametrize("k", [1, 2, 3, 17, 47, 48, 49, 160, 457, 1100])
def test_eigenvalues_and_vectors(k):
    kf = _kf()
    print(f"case sym_eig k={k}", flush=True)
    A, lam = _matrix(k, 40 + k)
    lo, hi = np.quantile(lam, 0.3), np.quantile(lam, 0.6)
    theta, Y = kf.sym_eig(A, lo, hi, vectors=True)
    scale = np.abs(lam).max()
    assert np.abs(theta - lam).max() <= 1e-12 * scale * max(1.0, np.sqrt(k) / 8)
    sel = theta[(theta >= lo) & (theta <= hi)]
    assert Y.shape == (k, sel.size)
    if sel.size:
        R = A @ Y - Y * sel
        assert np.abs(R).max() <= 1e-11 * scale
        assert np.abs(Y.T @ Y - np.eye(sel.size)).max() <= 1e-10


@pytest.mark.parametrize("k", [40, 300, 900])
def test_large_clusters_get_orthonormal_vectors(k):
    # an 8-fold and a 4-fold eigenvalue and three exact pairs inside the
    # selected range: every member of a cluster is found from its own start
    # vector, then the cluster's vectors are orthonormalised
    kf = _kf()
    print(f"case sym_eig clusters k={k}", flush=True)
    rng = np.random.default_rng(500 + k)
    lam = np.sort(rng.uniform(-3.0, 5.0, size=k))
    i0 = k // 3
    lam[i0 : i0 + 8] = lam[i0]
    lam[i0 + 10 : i0 + 14] = lam[i0 + 10]
    for j in (i0 + 16, i0 + 19, i0 + 22):
        lam[j + 1] = lam[j]
    lam = np.sort(lam)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    A = (Q * lam) @ Q.T
    lo, hi = lam[max(i0 - 3, 0)] - 1e-3, lam[min(i0 + 30, k - 1)] + 1e-3
    theta, Y = kf.sym_eig(A, lo, hi, vectors=True)
    scale = np.abs(lam).max()
    assert np.abs(theta - lam).max() <= 1e-12 * scale * max(1.0, np.sqrt(k) / 8)
    sel = theta[(theta >= lo) & (theta <= hi)]
    assert sel.size >= 20
    R = A @ Y - Y * sel
    assert np.abs(R).max() <= 1e-11 * scale
    assert np.abs(Y.T @ Y - np.eye(sel.size)).max() <= 1e-10


def test_values_only_and_asymmetric_input_is_averaged():
    kf = _kf()
    A, lam = _matrix(200, 7, clusters=False)
    rng = np.random.default_rng(8)
    E = 1e-3 * rng.standard_normal(A.shape)
    theta = kf.sym_eig(A + E)
    ref = np.linalg.eigvalsh(A + 0.5 * (E + E.T))
    assert np.abs(theta - ref).max() <= 1e-12 * np.abs(ref).max()
