"""Pins of the oracle's reflector generation (Python and C twins).

Pinned against: a hand-worked example (tests/golden/larfg_3_4.json), LAPACK
dlarfg / zlarfg through scipy, and the defining properties H^H x = beta e_0,
H^H H = I.
"""
import ctypes as C
import json
import os

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from oracle.householder import larfg
from oracle.native import ptr

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def c_larfg(orc, x):
    x = np.array(x, copy=True)
    if np.iscomplexobj(x):
        t = np.zeros(1, dtype=np.complex128)
        b = np.zeros(1)
        orc.orc_larfg_z(x.size, ptr(x), ptr(t), ptr(b))
    else:
        t = np.zeros(1)
        b = np.zeros(1)
        orc.orc_larfg_d(x.size, ptr(x), ptr(t), ptr(b))
    return x, t[0], b[0]


def test_golden_worked_example(orc):
    g = json.load(open(os.path.join(GOLD, "larfg_3_4.json")))
    for fn in (lambda x: larfg(np.array(x)), lambda x: c_larfg(orc, x)):
        v, tau, beta = fn(g["x"])
        assert np.allclose(v, g["v"], rtol=0, atol=1e-15)
        assert abs(tau - g["tau"]) < 1e-15
        assert abs(beta - g["beta"]) < 1e-15


@pytest.mark.parametrize("L", [1, 2, 5, 33, 64])
@pytest.mark.parametrize("cplx", [False, True])
def test_matches_lapack(orc, L, cplx):
    rng = np.random.default_rng(L + 100 * cplx)
    x = rng.standard_normal(L) + (1j * rng.standard_normal(L) if cplx else 0)
    if cplx:
        a, xs, t = lapack.zlarfg(L, x[0], x[1:].copy() if L > 1 else np.zeros(1, complex))
    else:
        a, xs, t = lapack.dlarfg(L, x[0], x[1:].copy() if L > 1 else np.zeros(1))
    for v, tau, beta in (larfg(x), c_larfg(orc, x)):
        assert abs(tau - t) <= 1e-14 * max(1, abs(t))
        assert abs(beta - np.real(a)) <= 1e-14 * abs(a)
        if L > 1:
            assert np.allclose(v[1:], xs[:L - 1], rtol=1e-13, atol=1e-15)
        assert v[0] == 1.0


@pytest.mark.parametrize("cplx", [False, True])
def test_defining_properties(orc, cplx):
    rng = np.random.default_rng(7)
    for L in (2, 3, 17, 64):
        x = rng.standard_normal(L) + (1j * rng.standard_normal(L) if cplx else 0)
        for v, tau, beta in (larfg(x), c_larfg(orc, x)):
            H = np.eye(L) - tau * np.outer(v, v.conj())
            e0 = np.zeros(L)
            e0[0] = beta
            assert np.allclose(H.conj().T @ x, e0, atol=1e-13)
            assert np.allclose(H.conj().T @ H, np.eye(L), atol=1e-14)
            assert np.imag(beta) == 0


def test_zero_tail_real_is_identity(orc):
    for v, tau, beta in (larfg(np.array([2.5, 0.0, 0.0])), c_larfg(orc, [2.5, 0.0, 0.0])):
        assert tau == 0 and beta == 2.5 and list(v) == [1.0, 0.0, 0.0]


def test_length_one_complex_makes_real(orc):
    x = np.array([1.0 + 2.0j])
    for v, tau, beta in (larfg(x), c_larfg(orc, x)):
        assert tau != 0
        assert abs(np.conj(1 - tau) * x[0] - beta) < 1e-15
