"""Stage 1 of the two-stage reduction: full Hermitian matrix -> band.

Sec. 2 of the paper: the first step reduces the matrix to banded form so that
BLAS level 3 can be used; the paper gives no further detail.  Reading used
here (textbook panel algorithm):

  for panel p = 0, b, 2b, ... while p + b < n:
      Householder QR of the panel A[p+b:n, p:p+b] (one larfg per column,
      k = min(b, n-p-b) reflectors, reflector i acting on rows [p+b+i, n));
      the trailing block A[p+b:, p+b:] <- Q_p^H A[p+b:, p+b:] Q_p with
      Q_p = H_0 H_1 ... H_{k-1};
      the panel and its mirror image are written back.

After all panels A[i, k] = 0 for |i - k| > b.  The whole transformation is
B = Q1^H A Q1 with Q1 = Q_0 Q_1 ... (generation order).

Two variants compute the same thing: ``blocked=False`` applies every reflector
two-sided on its own (rank-1 numpy updates, for small n); ``blocked=True``
applies each panel's product as I - V T V^H (compact WY, T from the forward
column-wise recurrence), using numpy matmul as the only library primitive.
"""
import numpy as np

from .householder import larfg, apply_left, apply_right


def _larft(V, taus):
    """Forward column-wise T with H_0 H_1 ... H_{k-1} = I - V T V^H."""
    k = V.shape[1]
    T = np.zeros((k, k), dtype=V.dtype)
    for i in range(k):
        T[i, i] = taus[i]
        if i > 0:
            T[:i, i] = -taus[i] * (T[:i, :i] @ (V[:, :i].conj().T @ V[:, i]))
    return T


def full_to_band(A, b, blocked=True):
    """Return (B, panels) with B = Q1^H A Q1 banded (semi-bandwidth b).

    ``panels`` is a list of (p, V, taus): V is (n-p-b) x k, column i holds the
    reflector vector on rows [i, n-p-b) of the panel (zeros above), taus its
    tau values.  A is not modified.
    """
    A = np.array(A, dtype=np.result_type(A, np.float64), order="F", copy=True)
    n = A.shape[0]
    if b < 1:
        raise ValueError("b must be >= 1")
    panels = []
    p = 0
    while p + b < n:
        m = n - p - b
        k = min(b, m)
        r0 = p + b
        V = np.zeros((m, k), dtype=A.dtype)
        taus = np.zeros(k, dtype=A.dtype)
        if blocked:
            P = A[r0:, p:p + b].copy()
            for i in range(k):
                v, t, beta = larfg(P[i:, i])
                if i + 1 < b:
                    apply_left(v, t, P[i:, i + 1:])
                P[i, i] = beta
                P[i + 1:, i] = 0.0
                V[i:, i] = v
                taus[i] = t
            T = _larft(V, taus)
            A22 = A[r0:, r0:]
            A22 -= V @ (T.conj().T @ (V.conj().T @ A22))
            A22 -= (A22 @ V) @ (T @ V.conj().T)
            A[r0:, p:p + b] = P
            A[p:p + b, r0:] = P.conj().T
        else:
            for i in range(k):
                r = r0 + i
                v, t, beta = larfg(A[r:, p + i].copy())
                # two-sided on every row / column that can be non-zero
                apply_left(v, t, A[r:, p:])
                apply_right(v, t, A[p:, r:])
                A[r, p + i] = beta
                A[p + i, r] = beta
                A[r + 1:, p + i] = 0.0
                A[p + i, r + 1:] = 0.0
                V[i:, i] = v
                taus[i] = t
        panels.append((p, V, taus))
        p += b
    # exact band structure
    i, k = np.indices(A.shape)
    A[np.abs(i - k) > b] = 0.0
    return A, panels
