"""Pins of stage 2 (band -> tridiagonal bulge chase, C).

* b >= n-1: one reflector per sweep, which is LAPACK's tridiagonalisation of
  the (full) band matrix: dsytrd / zhetrd ('L') give the same d, e, tau and v.
* The windowed C chase equals a dense brute force that applies every
  reflector to whole rows and columns (tiny n).
* spec(T) = spec(B) (LAPACK dsbevd / zhbevd on B's band storage).
* Q2 = BT1(I) satisfies Q2^H Q2 = I and Q2^H B Q2 = T: this ties the reflector
  layout, the application order and the conjugation convention of the
  back-transformation to the reduction that produced them.
* Slot counts equal a brute-force enumeration and the layout generator.
"""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

import workload as W
from oracle import bt, stage1, stage2
from oracle.householder import larfg


def banded(A, b):
    A = A.copy()
    i, k = np.indices(A.shape)
    A[np.abs(i - k) > b] = 0
    return A


def dense_chase(B, b):
    """Brute force: same slot sequence, whole-matrix two-sided updates."""
    A = np.array(B, dtype=B.dtype, copy=True)
    n = A.shape[0]
    hh, taus = [], []
    for s in range(n - 1):
        J = -(-(n - 1 - s) // b)
        for j in range(J):
            r = s + 1 + j * b
            L = min(b, n - r)
            c = s if j == 0 else r - b
            v, t, beta = larfg(A[r:r + L, c].copy())
            vf = np.zeros(n, dtype=A.dtype)
            vf[r:r + L] = v
            H = np.eye(n, dtype=A.dtype) - t * np.outer(vf, vf.conj())
            A = H.conj().T @ A @ H
            A[r, c] = beta
            A[c, r] = beta
            A[r + 1:r + L, c] = 0
            A[c, r + 1:r + L] = 0
            pad = np.zeros(b, dtype=A.dtype)
            pad[:L] = v
            hh.append(pad)
            taus.append(t)
    return (np.real(np.diag(A)), np.real(np.diag(A, -1)),
            np.concatenate(hh), np.array(taus, dtype=A.dtype), A)


@pytest.mark.parametrize("n,b", [(2, 1), (3, 1), (9, 2), (20, 3), (25, 6), (18, 17), (12, 40)])
def test_slot_counts(orc, n, b):
    brute = sum(-(-(n - 1 - s) // b) for s in range(n - 1))
    assert stage2.num_reflectors(n, b) == brute
    ss, jj, rr, LL = W.reflector_layout(n, b)
    assert LL.size == brute
    assert int(LL.sum()) == n * (n - 1) // 2
    assert np.all(LL >= 1) and np.all(rr + LL <= n)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,b", [(19, 18), (12, 30)])
def test_full_band_is_lapack_tridiagonalisation(orc, n, b, cplx):
    A = W.herm_gaussian(n, 11) if cplx else W.sym_gaussian(n, 11)
    d, e, hh, tau = stage2.band_to_tridiag(A, b)
    fn = lapack.zhetrd if cplx else lapack.dsytrd
    c, dl, el, tl, info = fn(A, lower=1)
    assert np.allclose(d, dl, atol=1e-13)
    assert np.allclose(e, el, atol=1e-13)
    assert np.allclose(tau, tl, atol=1e-13)
    H = hh.reshape(-1, b)
    for s in range(n - 1):
        L = n - 1 - s
        assert H[s, 0] == 1
        assert np.allclose(H[s, 1:L], c[s + 2:, s], atol=1e-12)
        assert np.all(H[s, L:] == 0)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,b", [(13, 3), (20, 4), (17, 5), (16, 1), (11, 2)])
def test_windowed_chase_equals_dense_brute_force(orc, n, b, cplx):
    A = W.herm_gaussian(n, 3 * n + b) if cplx else W.sym_gaussian(n, 3 * n + b)
    B = banded(A, b)
    d, e, hh, tau = stage2.band_to_tridiag(B, b)
    d2, e2, hh2, tau2, T = dense_chase(B, b)
    assert np.allclose(d, d2, atol=1e-12)
    assert np.allclose(e, e2, atol=1e-12)
    assert np.allclose(hh, hh2, atol=1e-11)
    assert np.allclose(tau, tau2, atol=1e-12)
    # the brute-force result is tridiagonal
    assert np.max(np.abs(np.tril(T, -2))) < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,b", [(40, 6), (33, 8), (64, 16)])
def test_spectrum_and_similarity(orc, n, b, cplx):
    A = W.herm_gaussian(n, n * b) if cplx else W.sym_gaussian(n, n * b)
    B, _ = stage1.full_to_band(A, b)
    d, e, hh, tau = stage2.band_to_tridiag(B, b)
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    # LAPACK band eigensolver on the lower band storage of B
    ab = np.zeros((b + 1, n), dtype=B.dtype)
    for k in range(b + 1):
        ab[k, :n - k] = np.diag(B, -k)
    fn = lapack.zhbevd if cplx else lapack.dsbevd
    w = fn(ab, compute_v=0, lower=1)[0]
    assert np.allclose(np.sort(np.linalg.eigvalsh(T)), np.sort(w), atol=1e-12)
    Q2 = bt.bt_tridiag_to_band(hh, tau, np.eye(n, dtype=B.dtype), n, b)
    assert np.allclose(Q2.conj().T @ Q2, np.eye(n), atol=1e-13)
    assert np.allclose(Q2.conj().T @ B @ Q2, T, atol=1e-12)


def test_orthogonality_error_bound_grows_slowly(orc):
    n, b = 256, 16
    A = W.sym_gaussian(n, 77)
    B, _ = stage1.full_to_band(A, b)
    d, e, hh, tau = stage2.band_to_tridiag(B, b)
    Q2 = bt.bt_tridiag_to_band(hh, tau, np.eye(n), n, b)
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    eps = 2.0 ** -52
    assert np.linalg.norm(Q2.T @ Q2 - np.eye(n), 1) / (n * eps) < 50
    assert np.linalg.norm(Q2.T @ B @ Q2 - T, 1) / (np.linalg.norm(B, 1) * n * eps) < 50
