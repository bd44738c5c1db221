"""Host logic of the band -> tridiagonal reduction's launch schedule (CPU).

Chase step (s, j) runs in launch t = j + 3 s (include/elpa_b2t.h).  A step
re-implemented here in numpy (the one-column bulge-chase step with LAPACK's
larfg convention) is run once in the sequential order (sweep by sweep, step
by step) and once launch by launch, with the steps of a launch in increasing
and in decreasing sweep order (they run concurrently on the GPU); the matrix
and every reflector must be bitwise equal, which holds only if the launches
reorder steps that touch disjoint entries.  A lag of 2 sweeps, where they do
not, is shown to fail.  The active-sweep ranges the library computes per launch are
checked against a brute-force enumeration."""
import numpy as np
import pytest


def chase_step(A, n, b, s, j):
    r = s + 1 + j * b
    L = min(b, n - r)
    c = s if j == 0 else r - b
    x = A[r:r + L, c].copy()
    alpha = x[0]
    ss = float(np.sum(x[1:] ** 2))
    if ss == 0.0:
        t, beta, v = 0.0, alpha, np.eye(1, L).ravel()
    else:
        h = np.sqrt(alpha * alpha + ss)
        beta = -h if alpha >= 0 else h
        t = (beta - alpha) / beta
        v = x / (alpha - beta)
        v[0] = 1.0
    lo, hi = max(r - b, 0), min(r + L + b, n)
    if t != 0.0:
        for k in range(lo, hi):
            A[r:r + L, k] -= v * (t * np.dot(v, A[r:r + L, k]))
        for i in range(lo, hi):
            A[i, r:r + L] -= (t * np.dot(A[i, r:r + L], v)) * v
    A[r, c] = A[c, r] = beta
    A[r + 1:r + L, c] = 0.0
    A[c, r + 1:r + L] = 0.0
    return v, t


def steps(n, b, s):
    return -(-(n - 1 - s) // b)


LAG = 3   # launch t runs the steps (s, t - LAG s)


def launches(n, b, lag=LAG):
    """The library's launch loop: (t, s_lo, s_hi) for every non-empty launch."""
    T = max(lag * s + steps(n, b, s) for s in range(n - 1))
    out, s_lo = [], 0
    for t in range(T):
        while s_lo <= n - 2 and lag * s_lo + steps(n, b, s_lo) <= t:
            s_lo += 1
        s_hi = min(t // lag, n - 2)
        if s_hi >= s_lo:
            out.append((t, s_lo, s_hi))
    return out


def band(n, b):
    rng = np.random.default_rng(n * 100 + b)
    G = rng.standard_normal((n, n))
    A0 = (G + G.T) / 2.0
    A0[np.abs(np.subtract.outer(np.arange(n), np.arange(n))) > b] = 0.0
    return A0


def sequential(A0, n, b):
    A1 = A0.copy()
    seq = {}
    for s in range(n - 1):
        for j in range(steps(n, b, s)):
            seq[(s, j)] = chase_step(A1, n, b, s, j)
    return A1, seq


def wavefront(A0, n, b, lag, reverse):
    A2 = A0.copy()
    par = {}
    for t, s_lo, s_hi in launches(n, b, lag):
        ss = range(s_hi, s_lo - 1, -1) if reverse else range(s_lo, s_hi + 1)
        for s in ss:
            par[(s, t - lag * s)] = chase_step(A2, n, b, s, t - lag * s)
    return A2, par


@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("n,b", [(40, 3), (50, 7), (33, 1), (64, 16), (30, 29), (12, 4),
                                 (45, 2)])
def test_wavefront_equals_sequential_bitwise(n, b, reverse):
    A0 = band(n, b)
    A1, seq = sequential(A0, n, b)
    A2, par = wavefront(A0, n, b, LAG, reverse)
    assert set(par) == set(seq)
    assert np.array_equal(A1, A2)
    for k in seq:
        assert np.array_equal(seq[k][0], par[k][0]) and seq[k][1] == par[k][1], k


@pytest.mark.parametrize("n,b", [(40, 3), (64, 16)])
def test_lag_two_conflicts(n, b):
    """With a lag of 2 sweeps the steps of a launch share entries, and running
    them in decreasing sweep order changes the result: the check above would
    catch a schedule that reorders conflicting steps."""
    A0 = band(n, b)
    A1, _ = sequential(A0, n, b)
    A2, _ = wavefront(A0, n, b, 2, True)
    assert not np.array_equal(A1, A2)


@pytest.mark.parametrize("n,b", [(2, 1), (3, 2), (100, 7), (257, 64), (1000, 32)])
def test_launch_ranges_brute_force(n, b):
    got = {(t, s) for t, lo, hi in launches(n, b) for s in range(lo, hi + 1)}
    want = {(j + LAG * s, s) for s in range(n - 1) for j in range(steps(n, b, s))}
    assert got == want
