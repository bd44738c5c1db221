"""End-to-end pins of the whole two-stage oracle.

* Closed form: A = Q_H diag(lambda) Q_H^T with Haar Q_H gives back sort(lambda)
  and, for well separated lambda, the columns of Q_H up to sign.
* Brute force: cyclic Jacobi for n <= 16 (complex via the real 2n x 2n
  embedding).
* Invariants res < 50 and orth < 50 on the first workload (n = 512, nbw = 32).
"""
import numpy as np
import pytest

import workload as W
from oracle import checks, solve


def test_known_spectrum(orc):
    n, b = 96, 8
    A = W.haar_spectrum(n, 201, 202)
    rng = np.random.Generator(np.random.PCG64(202))
    lam = np.sort(rng.uniform(-1.0, 1.0, n))
    r = solve.solve_two_stage(A, b)
    assert np.allclose(r["lam"], lam, atol=n * 2.0 ** -52 * 4)
    X = np.random.Generator(np.random.PCG64(201)).standard_normal((n, n))
    Qh, R = np.linalg.qr(X)
    Qh = Qh * np.sign(np.diag(R))[None, :]
    order = np.argsort(np.random.Generator(np.random.PCG64(202)).uniform(-1, 1, n))
    Qs = Qh[:, order]
    gaps = np.minimum(np.diff(lam, prepend=-np.inf), np.diff(lam, append=np.inf))
    ok = gaps > 1e-3
    s = np.sign(np.sum(r["Z"] * Qs, axis=0))
    assert np.allclose((r["Z"] * s[None, :])[:, ok], Qs[:, ok], atol=1e-9)


@pytest.mark.parametrize("n,b", [(6, 2), (11, 3), (16, 4)])
def test_against_jacobi_real(orc, n, b):
    A = W.sym_gaussian(n, 1000 + n)
    wj, Vj = checks.jacobi_eigh(A)
    r = solve.solve_two_stage(A, b)
    assert np.allclose(r["lam"], wj, atol=1e-13)
    s = np.sign(np.sum(r["Z"] * Vj, axis=0))
    assert np.allclose(r["Z"], Vj * s[None, :], atol=1e-9)


@pytest.mark.parametrize("n,b", [(5, 2), (12, 3)])
def test_against_jacobi_complex(orc, n, b):
    A = W.herm_gaussian(n, 2000 + n)
    wj = checks.jacobi_eigvals_hermitian(A)
    r = solve.solve_two_stage(A, b)
    assert np.allclose(r["lam"], wj, atol=1e-13)
    assert checks.residual_ratio(A, r["Z"], r["lam"]) < 50


@pytest.mark.parametrize("cplx", [False, True])
def test_first_workload_invariants(orc, cplx):
    n, b = 512, 32
    A = W.herm_gaussian(n, 101) if cplx else W.sym_gaussian(n, 101)
    r = solve.solve_two_stage(A, b)
    assert checks.residual_ratio(A, r["Z"], r["lam"]) < 50
    assert checks.orth_ratio(r["Z"]) < 50
    assert checks.residual_ratio(r["B"], r["Zb"], r["lam"]) < 50
    assert np.allclose(r["lam"], np.linalg.eigvalsh(A), atol=1e-12)


def test_partial_nev(orc):
    n, b = 200, 16
    A = W.sym_gaussian(n, 55)
    r = solve.solve_two_stage(A, b, nev=20)
    assert r["Z"].shape == (n, 20)
    assert np.allclose(r["lam"], np.linalg.eigvalsh(A)[:20], atol=1e-12)
    assert checks.residual_ratio(A, r["Z"], r["lam"]) < 50
