"""Invariants, error metrics and a brute-force Jacobi eigensolver.

Residual and orthogonality ratios (eps = 2^-52, 1-norms):
    res  = ||A Z - Z Lambda||_1 / (||A||_1 * n * eps)
    orth = ||Z^H Z - I||_1 / (n * eps)
Both must stay below 50 for a correct solve.

Parity metric between a result and the oracle:
    err = max |X - X_ref| / max |X_ref|  (max-abs relative).
"""
import numpy as np

EPS = 2.0 ** -52


def norm1(M):
    return float(np.max(np.sum(np.abs(M), axis=0))) if M.size else 0.0


def residual_ratio(A, Z, lam):
    n = A.shape[0]
    R = A @ Z - Z * np.asarray(lam)[None, :]
    return norm1(R) / (norm1(A) * n * EPS)


def orth_ratio(Z):
    n = Z.shape[0]
    G = Z.conj().T @ Z - np.eye(Z.shape[1])
    return norm1(G) / (n * EPS)


def max_rel_err(X, Xref):
    ref = float(np.max(np.abs(Xref)))
    if ref == 0.0:
        return float(np.max(np.abs(X)))
    return float(np.max(np.abs(np.asarray(X) - Xref))) / ref


def fro_rel_err(X, Xref):
    ref = float(np.linalg.norm(Xref))
    return float(np.linalg.norm(np.asarray(X) - Xref)) / (ref if ref else 1.0)


def jacobi_eigh(A, sweeps=60, tol=None):
    """Cyclic Jacobi for a small real symmetric matrix (pure Python loops).

    Returns (ascending eigenvalues, eigenvectors as columns).  Each rotation
    annihilates A[p, q] exactly in exact arithmetic (the classical two-sided
    2x2 symmetric Schur decomposition).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    fro = np.sqrt(np.sum(A * A))
    tol = EPS * fro if tol is None else tol
    for _ in range(sweeps):
        off = np.sqrt(max(0.0, np.sum(A * A) - np.sum(np.diag(A) ** 2)))
        if off <= tol:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if abs(apq) <= 1e-300:
                    continue
                theta = (A[q, q] - A[p, p]) / (2.0 * apq)
                t = (1.0 if theta >= 0 else -1.0) / (abs(theta) + np.hypot(theta, 1.0))
                c = 1.0 / np.sqrt(t * t + 1.0)
                s = t * c
                for k in range(n):
                    akp, akq = A[k, p], A[k, q]
                    A[k, p] = c * akp - s * akq
                    A[k, q] = s * akp + c * akq
                for k in range(n):
                    apk, aqk = A[p, k], A[q, k]
                    A[p, k] = c * apk - s * aqk
                    A[q, k] = s * apk + c * aqk
                for k in range(n):
                    vkp, vkq = V[k, p], V[k, q]
                    V[k, p] = c * vkp - s * vkq
                    V[k, q] = s * vkp + c * vkq
    w = np.diag(A).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def jacobi_eigvals_hermitian(A):
    """Eigenvalues of a small complex Hermitian matrix through the real
    2n x 2n embedding [[Re, -Im], [Im, Re]], whose spectrum is that of A with
    every eigenvalue doubled."""
    Ar, Ai = np.real(A), np.imag(A)
    M = np.block([[Ar, -Ai], [Ai, Ar]])
    w, _ = jacobi_eigh(M)
    return w[0::2]
