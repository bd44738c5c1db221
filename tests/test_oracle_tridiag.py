"""Pins of the tridiagonal eigensolver (bisection + inverse iteration, C).

* Closed form: tridiag(1, 0, 1) has lambda_k = 2 cos(k pi/(n+1)) and
  v_k[i] = sqrt(2/(n+1)) sin((i+1) k pi/(n+1)); also the hand-derived n = 5
  fixture tests/golden/toeplitz_n5.json.
* Library: scipy.linalg.eigh_tridiagonal (LAPACK stemr/stebz).
* Brute force: cyclic Jacobi (pure Python) for n <= 16; Sturm counts against
  a direct count of eigvalsh below x.
* Invariants: residual and orthogonality ratios < 50 with clusters present.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import checks, tridiag

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def T_of(d, e):
    return np.diag(d) + np.diag(e, -1) + np.diag(e, 1)


def test_golden_toeplitz_n5(orc):
    g = json.load(open(os.path.join(GOLD, "toeplitz_n5.json")))
    w, Z = tridiag.eigh_tridiag(np.array(g["d"]), np.array(g["e"]))
    assert np.allclose(w, g["eigenvalues"], atol=1e-15)
    assert np.allclose(np.abs(Z[:, 0]), g["v_for_lambda_0_abs"], atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 7, 100, 513])
def test_toeplitz_closed_form(orc, n):
    d = np.zeros(n)
    e = np.ones(n - 1)
    w, Z = tridiag.eigh_tridiag(d, e)
    k = np.arange(n, 0, -1)
    lam = 2 * np.cos(k * np.pi / (n + 1))
    assert np.allclose(w, lam, atol=4e-15 * max(1, n) ** 0.5)
    i = np.arange(1, n + 1)[:, None]
    V = np.sqrt(2.0 / (n + 1)) * np.sin(i * k[None, :] * np.pi / (n + 1))
    # the closed-form vectors have exact magnitude ties (v[i] = +-v[n-1-i]),
    # so compare up to sign and check the sign rule on the computed vectors
    s = np.sign(np.sum(Z * V, axis=0))
    assert np.allclose(Z, V * s[None, :], atol=1e-12)
    big = np.argmax(np.abs(Z), axis=0)
    assert np.all(Z[big, np.arange(n)] > 0)


@pytest.mark.parametrize("n,seed", [(10, 1), (200, 2), (1000, 3)])
def test_against_lapack(orc, n, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    w, Z = tridiag.eigh_tridiag(d, e)
    wl, Zl = sla.eigh_tridiagonal(d, e)
    assert np.allclose(w, wl, atol=1e-13 * np.max(np.abs(wl)))
    # eigenvectors agree up to sign
    s = np.sign(np.sum(Z * Zl, axis=0))
    assert np.allclose(Z, Zl * s[None, :], atol=1e-9)
    T = T_of(d, e)
    assert checks.residual_ratio(T, Z, w) < 50
    assert checks.orth_ratio(Z) < 50


@pytest.mark.parametrize("n", [2, 5, 9, 16])
def test_against_jacobi(orc, n):
    rng = np.random.default_rng(40 + n)
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    wj, Vj = checks.jacobi_eigh(T_of(d, e))
    w, Z = tridiag.eigh_tridiag(d, e)
    assert np.allclose(w, wj, atol=1e-13)
    s = np.sign(np.sum(Z * Vj, axis=0))
    assert np.allclose(Z, Vj * s[None, :], atol=1e-10)


def test_sturm_counts(orc):
    rng = np.random.default_rng(9)
    n = 60
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    lam = np.linalg.eigvalsh(T_of(d, e))
    for x in np.linspace(-5, 5, 41):
        assert tridiag.sturm_count(d, e, x) == int(np.sum(lam < x))


def test_partial_spectrum_and_clusters(orc):
    # Wilkinson-like matrix W21+: pairs of nearly equal eigenvalues
    m = 10
    d = np.abs(np.arange(-m, m + 1)).astype(float)
    e = np.ones(2 * m)
    n = d.size
    w, Z = tridiag.eigh_tridiag(d, e)
    T = T_of(d, e)
    assert np.allclose(w, np.linalg.eigvalsh(T), atol=1e-13)
    assert checks.residual_ratio(T, Z, w) < 50
    assert checks.orth_ratio(Z) < 50
    wl, Zl = tridiag.eigh_tridiag(d, e, nev=7)
    assert np.allclose(wl, w[:7], atol=0)
    assert np.allclose(np.abs(Zl), np.abs(Z[:, :7]), atol=1e-10)


def test_gaussian_band_tridiagonal_invariants(orc):
    """GOE-like spectrum at moderate n (dense, many near-clusters)."""
    rng = np.random.default_rng(12)
    n = 1500
    d = rng.standard_normal(n) * np.sqrt(n) / 10
    e = np.abs(rng.standard_normal(n - 1)) * np.sqrt(n) / 10
    w, Z = tridiag.eigh_tridiag(d, e)
    T = T_of(d, e)
    assert checks.residual_ratio(T, Z, w) < 50
    assert checks.orth_ratio(Z) < 50
