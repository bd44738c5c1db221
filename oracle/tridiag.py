"""Tridiagonal eigensolver (Eq. Esolv of the paper: T V^ = V^ Lambda).

The paper does not name its tridiagonal solver.  Reading used here: Sturm
sequence bisection for the wanted eigenvalues (the nev smallest, ascending,
since the applications want the lower part of the spectrum), then inverse
iteration with partial-pivoting LU of T - lambda I, modified Gram-Schmidt
inside clusters of eigenvalues closer than ||T||_1 / n, and the sign fixed so
that the largest-magnitude entry is positive.  fp64 throughout (C code).
"""
import numpy as np

from .native import lib, ptr


def sturm_count(d, e, x):
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    piv = np.finfo(np.float64).tiny * max(1.0, float(np.max(e * e)) if e.size else 1.0)
    return int(lib().orc_sturm_count(d.size, ptr(d), ptr(e), float(x), piv))


def eigvals(d, e, il=0, iu=None, nthreads=0):
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = d.size
    iu = n - 1 if iu is None else iu
    w = np.zeros(iu - il + 1)
    rc = lib().orc_tridiag_bisect(n, ptr(d), ptr(e), il, iu, ptr(w), nthreads)
    if rc != 0:
        raise RuntimeError("bisection failed: %d" % rc)
    return w


def eigvecs(d, e, w, seed=12345, nthreads=0):
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = d.size
    Z = np.zeros((n, w.size), order="F")
    rc = lib().orc_tridiag_invit(n, ptr(d), ptr(e), w.size, ptr(w), ptr(Z), n,
                                 seed, nthreads)
    if rc != 0:
        raise RuntimeError("inverse iteration failed: %d" % rc)
    return Z


def eigh_tridiag(d, e, nev=None, seed=12345, nthreads=0):
    """The nev smallest eigenpairs of the symmetric tridiagonal (d, e)."""
    n = len(d)
    nev = n if nev is None else nev
    w = eigvals(d, e, 0, nev - 1, nthreads)
    return w, eigvecs(d, e, w, seed, nthreads)
