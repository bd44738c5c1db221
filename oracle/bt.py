"""The two eigenvector back-transformations of the two-stage method.

Sec. 2 of the paper: the eigenvectors of T are back-transformed as
V~ = Q^H V^ (the equation after Eq. Esolv), and the two-stage variant has to
transform every eigenvector twice.

``bt_tridiag_to_band`` is the hot path's definition, written out plainly in C
(oracle/csrc/oracle.c, orc_bt1_*): Q <- H(0,0) H(0,1) ... H(n-2, J-1) Q, i.e.
every band->tridiagonal reflector, the last generated first, applied to every
column.  This is the paper's Q^H V^ with Q = Q_n ... Q_1 and the paper's Q_i
equal to our H^H.

``bt_band_to_full`` applies the stage-1 panels the same way
(Z <- Q_0 Q_1 ... Z, last panel first) with numpy.
"""
import numpy as np

from .native import lib, ptr


def bt_tridiag_to_band(hh, tau, Z, n, b, nthreads=0):
    """Return H(0,0)...H(n-2,J-1) Z for reflectors in the boundary layout."""
    cplx = np.iscomplexobj(hh) or np.iscomplexobj(tau) or np.iscomplexobj(Z)
    dt = np.complex128 if cplx else np.float64
    Q = np.array(Z, dtype=dt, order="F", copy=True)
    if Q.ndim == 1:
        Q = Q.reshape(-1, 1, order="F")
    hh = np.ascontiguousarray(hh, dtype=dt)
    tau = np.ascontiguousarray(tau, dtype=dt)
    nev = Q.shape[1]
    if Q.shape[0] != n:
        raise ValueError("Z must have n rows")
    fn = lib().orc_bt1_z if cplx else lib().orc_bt1_d
    rc = fn(n, nev, b, ptr(hh), ptr(tau), ptr(Q), n, nthreads)
    if rc != 0:
        raise RuntimeError("bt1 failed: %d" % rc)
    return Q


def bt_band_to_full(panels, Z, b):
    """Return Q1 Z with Q1 = Q_0 Q_1 ... from stage1.full_to_band's panels."""
    cplx = np.iscomplexobj(Z) or any(np.iscomplexobj(V) for _, V, _ in panels)
    Z = np.array(Z, dtype=np.complex128 if cplx else np.float64, copy=True)
    for p, V, taus in reversed(panels):
        r0 = p + b
        k = V.shape[1]
        for i in reversed(range(k)):
            v = V[:, i]
            X = Z[r0:, :]
            w = v.conj() @ X
            X -= taus[i] * np.outer(v, w)
    return Z
