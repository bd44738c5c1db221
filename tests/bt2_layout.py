"""Conversion between the first stage's panels (oracle.stage1.full_to_band:
a list of (p, V, taus), V (n-p-nbw) x k with column i holding its reflector
on rows [i, n-p-nbw)) and the column layout of include/elpa_bt2.h (column c
of V holds v_c from row c+nbw down).  Test glue only: no arithmetic of the
method."""
import numpy as np


def panels_to_abi(panels, n, nbw, dtype):
    """(V, tau) in the library layout from stage1.full_to_band's panels."""
    N = max(0, n - nbw)
    V = np.full((n, max(N, 1)), np.nan, dtype=dtype, order="F")
    tau = np.zeros(max(N, 1), dtype=dtype)
    for p, Vp, taus in panels:
        for i in range(Vp.shape[1]):
            c = p + i
            V[c + nbw + 1:, c] = Vp[i + 1:, i]
            tau[c] = taus[i]
    return V, tau


def abi_to_panels(V, tau, n, nbw):
    """The oracle's panel format from the library layout (unit leads and
    zeros written explicitly)."""
    panels = []
    p = 0
    while p + nbw < n:
        m = n - p - nbw
        k = min(nbw, m)
        Vp = np.zeros((m, k), dtype=V.dtype)
        for i in range(k):
            Vp[i, i] = 1.0
            Vp[i + 1:, i] = V[p + nbw + i + 1:, p + i]
        panels.append((p, Vp, tau[p:p + k].copy()))
        p += nbw
    return panels
