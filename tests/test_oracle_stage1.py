"""Pins of stage 1 (full -> band).

* b = 1 is LAPACK's Householder tridiagonalisation: dsytrd / zhetrd ('L')
  give the same d, e, tau and reflector vectors to rounding.
* blocked (compact WY) == unblocked (per reflector two-sided).
* B is banded, B = Q1^H A Q1, and spec(B) = spec(A).
"""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

import workload as W
from oracle import stage1


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("blocked", [False, True])
def test_b1_is_lapack_tridiagonalisation(cplx, blocked):
    n = 23
    A = W.herm_gaussian(n, 5) if cplx else W.sym_gaussian(n, 5)
    B, panels = stage1.full_to_band(A, 1, blocked=blocked)
    fn = lapack.zhetrd if cplx else lapack.dsytrd
    c, d, e, tau, info = fn(A, lower=1)
    assert info == 0
    assert np.allclose(np.real(np.diag(B)), d, atol=1e-13)
    assert np.allclose(np.real(np.diag(B, -1)), e, atol=1e-13)
    assert np.allclose(np.imag(np.diag(B, -1)), 0, atol=1e-14)
    taus = np.array([t[0] for _, _, t in panels])
    assert np.allclose(taus, tau, atol=1e-13)
    for p, V, _ in panels:
        assert np.allclose(V[1:, 0], c[p + 2:, p], atol=1e-12)


@pytest.mark.parametrize("n,b", [(30, 4), (41, 6), (17, 16), (16, 20), (50, 7)])
@pytest.mark.parametrize("cplx", [False, True])
def test_band_similarity_spectrum(n, b, cplx):
    A = W.herm_gaussian(n, n + b) if cplx else W.sym_gaussian(n, n + b)
    Bb, pb = stage1.full_to_band(A, b, blocked=True)
    Bu, pu = stage1.full_to_band(A, b, blocked=False)
    assert np.allclose(Bb, Bu, atol=1e-12)
    i, k = np.indices(Bb.shape)
    assert np.all(Bb[np.abs(i - k) > b] == 0)
    assert np.allclose(Bb, Bb.conj().T, atol=0)
    # Q1 explicitly: B = Q1^H A Q1
    Q1 = np.eye(n, dtype=Bb.dtype)
    for p, V, taus in pb:
        for q in range(V.shape[1]):
            H = np.eye(n, dtype=Bb.dtype)
            v = np.zeros(n, dtype=Bb.dtype)
            v[p + b:] = V[:, q]
            H -= taus[q] * np.outer(v, v.conj())
            Q1 = Q1 @ H
    assert np.allclose(Q1.conj().T @ Q1, np.eye(n), atol=1e-13)
    assert np.allclose(Q1.conj().T @ A @ Q1, Bb, atol=1e-12)
    assert np.allclose(np.linalg.eigvalsh(Bb), np.linalg.eigvalsh(A), atol=1e-12)
