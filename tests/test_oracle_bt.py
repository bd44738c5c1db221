"""Pins of the back-transformations, above all the hot path's definition
(tridiagonal -> band, oracle/csrc/oracle.c orc_bt1_*).

* Brute force: the explicit dense product H(0,0) H(0,1) ... H(n-2,J-1) of all
  reflectors as n x n matrices, times Z (n <= 32).
* Identity input: BT1(I) = Q2 with Q2^H B Q2 = T (in test_oracle_stage2).
* Band eigen-residual: B BT1(Z^) = BT1(Z^) Lambda for the eigenvectors of T.
* tau == 0 is the identity; columns are independent; a NaN stays in its column.
* Any order that respects the dependency lemma (sweep blocks descending, chase
  steps ascending inside a block, sweeps descending inside a step group) gives
  the bitwise same result as strict reverse generation order.
* BT2: Q1 BT1 output solves A Z = Z Lambda.
"""
import numpy as np
import pytest

import workload as W
from oracle import bt, checks, stage1, stage2, tridiag


def dense_product(hh, tau, n, b):
    ss, jj, rr, LL = W.reflector_layout(n, b)
    H = hh.reshape(-1, b)
    P = np.eye(n, dtype=hh.dtype)
    for k in range(LL.size):
        v = np.zeros(n, dtype=hh.dtype)
        v[rr[k]:rr[k] + LL[k]] = H[k, :LL[k]]
        P = P @ (np.eye(n, dtype=hh.dtype) - tau[k] * np.outer(v, v.conj()))
    return P


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,b", [(2, 1), (5, 2), (17, 4), (32, 6), (12, 12), (9, 20)])
def test_bt1_equals_dense_product(orc, n, b, cplx):
    hh, tau = W.synthetic_reflectors(n, b, complex_=cplx, seed=n * b)
    Z = W.gaussian_block(n, 7, complex_=cplx, seed=3)
    got = bt.bt_tridiag_to_band(hh, tau, Z, n, b)
    ref = dense_product(hh, tau, n, b) @ Z
    assert np.allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("cplx", [False, True])
def test_bt1_real_reflectors_dense_product(orc, cplx):
    n, b = 24, 5
    A = W.herm_gaussian(n, 4) if cplx else W.sym_gaussian(n, 4)
    B, _ = stage1.full_to_band(A, b)
    d, e, hh, tau = stage2.band_to_tridiag(B, b)
    Z = W.gaussian_block(n, n, complex_=cplx, seed=8)
    got = bt.bt_tridiag_to_band(hh, tau, Z, n, b)
    assert np.allclose(got, dense_product(hh, tau, n, b) @ Z, atol=1e-13)


def test_zero_tau_is_identity(orc):
    n, b = 40, 7
    hh, tau = W.synthetic_reflectors(n, b, seed=1)
    Z = W.gaussian_block(n, 5, seed=2)
    got = bt.bt_tridiag_to_band(hh, np.zeros_like(tau), Z, n, b)
    assert np.array_equal(got, Z)


def test_column_independence_and_nan_isolation(orc):
    n, b = 60, 8
    hh, tau = W.synthetic_reflectors(n, b, seed=5)
    Z = np.asfortranarray(W.gaussian_block(n, 9, seed=6))
    full = bt.bt_tridiag_to_band(hh, tau, Z, n, b)
    for c in (0, 4, 8):
        one = bt.bt_tridiag_to_band(hh, tau, Z[:, c:c + 1], n, b)
        assert np.array_equal(one[:, 0], full[:, c])
    Zn = Z.copy()
    Zn[10, 3] = np.nan
    out = bt.bt_tridiag_to_band(hh, tau, Zn, n, b)
    assert np.all(np.isnan(out[:, 3]) | (np.arange(n) < 1))
    keep = [c for c in range(9) if c != 3]
    assert np.array_equal(out[:, keep], full[:, keep])


def grouped_order(n, b, k):
    """Slot order: sweep blocks of k descending, chase step ascending inside a
    block, sweep descending inside a (block, step) group."""
    ss, jj, rr, LL = W.reflector_layout(n, b)
    idx = {(int(s), int(j)): i for i, (s, j) in enumerate(zip(ss, jj))}
    order = []
    top = n - 2
    while top >= 0:
        s0 = max(0, top - k + 1)
        Jmax = -(-(n - 1 - s0) // b)
        for j in range(Jmax):
            for s in range(top, s0 - 1, -1):
                if (s, j) in idx:
                    order.append(idx[(s, j)])
        top = s0 - 1
    return order


def apply_in_order(hh, tau, Z, n, b, order):
    ss, jj, rr, LL = W.reflector_layout(n, b)
    H = hh.reshape(-1, b)
    Q = np.array(Z, copy=True)
    for k in order:
        r, L = rr[k], LL[k]
        v = H[k, :L]
        for c in range(Q.shape[1]):
            x = Q[r:r + L, c]
            w = 0.0
            for i in range(L):
                w += np.conj(v[i]) * x[i]
            w *= tau[k]
            for i in range(L):
                x[i] -= v[i] * w
    return Q


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("k", [1, 2, 4, 6, 7, 12])
def test_grouped_orders_bitwise_equal(orc, k, cplx):
    n, b = 41, 6
    hh, tau = W.synthetic_reflectors(n, b, complex_=cplx, seed=9)
    Z = W.gaussian_block(n, 3, complex_=cplx, seed=10)
    strict = list(reversed(range(len(tau))))
    ref = apply_in_order(hh, tau, Z, n, b, strict)
    got = apply_in_order(hh, tau, Z, n, b, grouped_order(n, b, k))
    assert np.array_equal(got, ref)
    # and the C oracle agrees with the strict order
    assert np.allclose(bt.bt_tridiag_to_band(hh, tau, Z, n, b), ref, atol=1e-14)


def test_wrong_order_is_detected(orc):
    """Chase steps descending inside a block violates the lemma: O(1) error."""
    n, b = 41, 6
    hh, tau = W.synthetic_reflectors(n, b, seed=9)
    Z = W.gaussian_block(n, 3, seed=10)
    ref = bt.bt_tridiag_to_band(hh, tau, Z, n, b)
    bad = apply_in_order(hh, tau, Z, n, b, list(range(len(tau))))  # generation order
    assert checks.max_rel_err(bad, ref) > 1e-2


@pytest.mark.parametrize("cplx", [False, True])
def test_band_eigen_residual(orc, cplx):
    n, b = 120, 12
    A = W.herm_gaussian(n, 21) if cplx else W.sym_gaussian(n, 21)
    B, panels = stage1.full_to_band(A, b)
    d, e, hh, tau = stage2.band_to_tridiag(B, b)
    lam, Zt = tridiag.eigh_tridiag(d, e)
    Zb = bt.bt_tridiag_to_band(hh, tau, Zt.astype(hh.dtype), n, b)
    assert checks.residual_ratio(B, Zb, lam) < 50
    assert checks.orth_ratio(Zb) < 50
    Z = bt.bt_band_to_full(panels, Zb, b)
    assert checks.residual_ratio(A, Z, lam) < 50
    assert checks.orth_ratio(Z) < 50
