"""Stage 2 of the two-stage reduction: band -> tridiagonal (bulge chasing).

Sec. 2 of the paper names the step (the banded matrix is further reduced to
tridiagonal form) but not the algorithm.  Reading used here: the
one-column-per-step Householder bulge chase.  Sweep s = 0..n-2 eliminates
column s; chase step j = 0..J(s)-1, J(s) = ceil((n-1-s)/b), reduces column
c (= s for j = 0, else r - b) below row r = s+1+j*b with a reflector of
length L = min(b, n-r) applied two-sided.  The reflectors are emitted in the
library's boundary layout: slot-major in generation order (s, then j), v[0] = 1
stored, zero padded to b, one tau per slot.

The work itself is in C (oracle/csrc/oracle.c, orc_band_to_tridiag_*).
"""
import numpy as np

from .native import lib, ptr


def num_reflectors(n, b):
    return int(lib().orc_num_reflectors(n, b))


def num_steps(n, b, s):
    return int(lib().orc_num_steps(n, b, s))


def band_to_tridiag(B, b):
    """Return (d, e, hh, tau) for a Hermitian band matrix B (full storage)."""
    cplx = np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    A = np.array(B, dtype=dt, order="F", copy=True)
    n = A.shape[0]
    nr = num_reflectors(n, b)
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0))
    hh = np.zeros(max(nr, 1) * b, dtype=dt)
    tau = np.zeros(max(nr, 1), dtype=dt)
    fn = lib().orc_band_to_tridiag_z if cplx else lib().orc_band_to_tridiag_d
    rc = fn(n, b, ptr(A), n, ptr(d), ptr(e), ptr(hh), ptr(tau))
    if rc != 0:
        raise RuntimeError("band_to_tridiag failed: %d" % rc)
    return d, e, hh[:nr * b].copy(), tau[:nr].copy()
