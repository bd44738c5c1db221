"""Generalized Hermitian-definite eigenproblem A V = B V Lambda on the CPU
(Sec. 2, Eq. (1) and the Cholesky, forward-transformation and
back-transformation equations there; Sec. 4 "Generalized EVP problem" for the
inverted factor kept in B between calls).

Test infrastructure: plain, slow, obviously correct fp64 / complex128 code that
the GPU path is checked against; nothing in the library imports it.

    B = L L^H                      cholesky()       (column recurrence)
    Linv = L^{-1}                  inverse_lower()  (forward substitution)
    A~ = Linv A Linv^H             to_standard()
    (lambda, V~) of A~             solve.solve_two_stage()
    V = Linv^H V~                  back()
"""
import numpy as np

from . import solve


def cholesky(B):
    """Lower Cholesky factor of the Hermitian matrix B (only its lower triangle
    is read), by the column recurrence
        L[j, j] = sqrt(B[j, j] - sum_{k<j} |L[j, k]|^2)
        L[i, j] = (B[i, j] - sum_{k<j} L[i, k] conj(L[j, k])) / L[j, j],  i > j.
    Returns (L, info): info = 0, or j + 1 (1-based, LAPACK's convention) when
    the leading minor of order j + 1 is not positive definite, in which case
    L holds the columns before j."""
    B = np.asarray(B)
    n = B.shape[0]
    L = np.zeros_like(B, dtype=np.result_type(B.dtype, np.float64))
    for j in range(n):
        d = B[j, j].real - np.sum(np.abs(L[j, :j]) ** 2)
        if not d > 0.0:
            return L, j + 1
        L[j, j] = np.sqrt(d)
        if j + 1 < n:
            L[j + 1:, j] = (B[j + 1:, j] - L[j + 1:, :j] @ np.conj(L[j, :j])) / L[j, j]
    return L, 0


def inverse_lower(L):
    """L^{-1} for a lower triangular L with nonzero diagonal: column j of X
    solves L x = e_j by forward substitution (zero above row j)."""
    L = np.asarray(L)
    n = L.shape[0]
    X = np.zeros_like(L)
    for j in range(n):
        X[j, j] = 1.0 / L[j, j]
        for i in range(j + 1, n):
            X[i, j] = -(L[i, j:i] @ X[j:i, j]) / L[i, i]
    return X


def to_standard(A, Linv):
    """The standard problem's matrix Linv A Linv^H."""
    return Linv @ A @ np.conj(Linv.T)


def back(Linv, Vt):
    """Eigenvectors of the generalized problem from the standard problem's:
    Linv^H V~."""
    return np.conj(Linv.T) @ Vt


def generalized_eigh(A, B, nbw, nev=None, Linv=None, seed=12345):
    """The whole generalized solve on the two-stage path.  With Linv given
    (the inverted factor of an earlier call with the same B) the Cholesky
    factorisation and inversion are skipped.  Returns dict(lam, V, Linv, At)."""
    if Linv is None:
        L, info = cholesky(B)
        if info:
            raise np.linalg.LinAlgError(f"leading minor of order {info} is not positive definite")
        Linv = inverse_lower(L)
    At = to_standard(A, Linv)
    At = (At + np.conj(At.T)) / 2
    r = solve.solve_two_stage(At, nbw, nev, seed=seed)
    return dict(lam=r["lam"], V=back(Linv, r["Z"]), Linv=Linv, At=At)
