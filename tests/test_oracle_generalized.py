"""Pins of the oracle's generalized eigenproblem (oracle/generalized.py)
against values fixed by the mathematics: a factor with integer entries, its
inverse worked by hand, LAPACK's failure index, problems that reduce to known
ones (B = I, diagonal B, A = B), and the invariants A V = B V Lambda,
V^H B V = I."""
import numpy as np
import pytest

import workload as W
from oracle import generalized as G


def spd(n, seed, cplx=False):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, n)) + (1j * g.standard_normal((n, n)) if cplx else 0)
    return X @ np.conj(X.T) / n + np.eye(n)


def test_cholesky_integer_factor():
    # B = L L^T with L = [[2,0,0],[6,1,0],[-8,5,3]]: an exact factor
    B = np.array([[4.0, 12, -16], [12, 37, -43], [-16, -43, 98]])
    L, info = G.cholesky(B)
    assert info == 0
    assert np.array_equal(L, np.array([[2.0, 0, 0], [6, 1, 0], [-8, 5, 3]]))


def test_cholesky_reads_lower_triangle_only():
    B = np.array([[4.0, 12, -16], [12, 37, -43], [-16, -43, 98]])
    Bu = np.tril(B) + np.triu(np.full((3, 3), np.nan), 1)
    L, info = G.cholesky(Bu)
    assert info == 0 and np.array_equal(L, np.array([[2.0, 0, 0], [6, 1, 0], [-8, 5, 3]]))


def test_inverse_worked_by_hand():
    L = np.array([[2.0, 0, 0], [6, 1, 0], [-8, 5, 3]])
    X = G.inverse_lower(L)
    ref = np.array([[0.5, 0, 0], [-3, 1, 0], [19 / 3, -5 / 3, 1 / 3]])
    assert np.max(np.abs(X - ref)) <= 4 * np.finfo(float).eps * 19 / 3
    assert np.array_equal(np.triu(X, 1), np.zeros((3, 3)))


@pytest.mark.parametrize("B,info", [
    (np.diag([1.0, 2.0, -1.0, 5.0]), 3),
    (np.array([[1.0, 2.0], [2.0, 1.0]]), 2),
    (np.array([[0.0, 0.0], [0.0, 1.0]]), 1),
    (np.diag([1.0, np.nan, 1.0]), 2),
])
def test_cholesky_failure_index(B, info):
    assert G.cholesky(B)[1] == info


@pytest.mark.parametrize("cplx", [False, True])
def test_factor_and_inverse_invariants(cplx):
    n = 40
    B = spd(n, 5, cplx)
    L, info = G.cholesky(B)
    assert info == 0
    assert np.array_equal(np.triu(L, 1), np.zeros_like(L))
    assert np.all(np.diag(L).real > 0) and np.all(np.diag(L).imag == 0)
    assert np.max(np.abs(L @ np.conj(L.T) - B)) <= 1e-13 * np.max(np.abs(B))
    X = G.inverse_lower(L)
    assert np.max(np.abs(X @ L - np.eye(n))) <= 1e-12
    assert np.max(np.abs(X @ B @ np.conj(X.T) - np.eye(n))) <= 1e-12


def test_identity_b_is_the_standard_problem():
    A = W.sym_gaussian(30, 7)
    r = G.generalized_eigh(A, np.eye(30), 8)
    assert np.max(np.abs(r["lam"] - np.linalg.eigvalsh(A))) <= 1e-12 * np.max(np.abs(A)) * 30


def test_diagonal_b_scales_the_problem():
    # B = D: the problem is D^{-1/2} A D^{-1/2}, whose eigenvalues numpy gives
    n = 25
    A = W.sym_gaussian(n, 8)
    dg = np.linspace(0.5, 3.0, n)
    r = G.generalized_eigh(A, np.diag(dg), 8)
    S = A / np.sqrt(np.outer(dg, dg))
    assert np.max(np.abs(r["lam"] - np.linalg.eigvalsh(S))) <= 1e-12 * np.max(np.abs(S)) * n


def test_a_equal_b_gives_unit_eigenvalues():
    B = spd(20, 9)
    r = G.generalized_eigh(B, B, 4)
    assert np.max(np.abs(r["lam"] - 1.0)) <= 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_generalized_invariants_and_reuse(cplx):
    n, nbw = 60, 8
    A = W.herm_gaussian(n, 10) if cplx else W.sym_gaussian(n, 10)
    B = spd(n, 11, cplx)
    r = G.generalized_eigh(A, B, nbw)
    V, lam = r["V"], r["lam"]
    scale = np.linalg.norm(A, 2) + np.linalg.norm(B, 2) * np.max(np.abs(lam))
    assert np.max(np.abs(A @ V - B @ V * lam)) <= 1e-11 * scale
    assert np.max(np.abs(np.conj(V.T) @ B @ V - np.eye(n))) <= 1e-11
    # the same eigenvalues as scipy's generalized solver
    import scipy.linalg
    assert np.max(np.abs(lam - scipy.linalg.eigh(A, B, eigvals_only=True))) <= 1e-11 * scale
    # a second A with the same B, reusing the inverted factor
    A2 = W.herm_gaussian(n, 12) if cplx else W.sym_gaussian(n, 12)
    r2 = G.generalized_eigh(A2, None, nbw, Linv=r["Linv"])
    V2, lam2 = r2["V"], r2["lam"]
    assert np.max(np.abs(A2 @ V2 - B @ V2 * lam2)) <= 1e-11 * scale
