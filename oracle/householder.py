"""Householder reflector generation in the LAPACK ``larfg`` convention.

The paper represents each Householder matrix only by its vector (Sec. 2, text
after Eq. tridiagonalization: Q_i = I - beta_i v_i v_i^H, never formed).  It
fixes no normalisation; the reading used here is LAPACK's: v[0] = 1,
H = I - tau v v^H and H^H x = beta e_0 with beta real (so a complex Hermitian
matrix reduces to a real tridiagonal one).  The paper's beta_i is conj(tau).
The LAPACK safe-minimum rescaling loop is omitted.
"""
import numpy as np


def larfg(x):
    """Return (v, tau, beta) with H^H x = beta e_0, H = I - tau v v^H, v[0] = 1."""
    x = np.asarray(x)
    cplx = np.iscomplexobj(x)
    alpha = x[0]
    xnorm = float(np.sqrt(np.sum(np.abs(x[1:]) ** 2))) if x.size > 1 else 0.0
    v = np.zeros_like(x)
    v[0] = 1.0
    ai = float(np.imag(alpha)) if cplx else 0.0
    if xnorm == 0.0 and ai == 0.0:
        return v, (0.0 + 0.0j if cplx else 0.0), float(np.real(alpha))
    ar = float(np.real(alpha))
    h = float(np.sqrt(ar * ar + ai * ai + xnorm * xnorm))
    beta = -h if ar >= 0.0 else h
    if cplx:
        tau = complex((beta - ar) / beta, -ai / beta)
    else:
        tau = (beta - ar) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def apply_left(v, tau, X):
    """X <- H^H X for H = I - tau v v^H (in place on a view)."""
    w = v.conj() @ X
    X -= np.conj(tau) * np.outer(v, w)


def apply_right(v, tau, X):
    """X <- X H for H = I - tau v v^H (in place on a view)."""
    w = X @ v
    X -= tau * np.outer(w, v.conj())
