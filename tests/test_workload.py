"""Seeded input generators and traces (CPU)."""
import numpy as np

import workload as W


def test_scf_trace_share_and_precision_switch():
    t, sq, st, f32 = W.scf_trace(nseq=8, steps=30, rate=100.0, p32=0.25)
    assert np.all(np.diff(t) >= 0) and t[0] == 0.0
    assert set(sq) == set(range(8)) and st.max() == 29
    assert 0.1 < f32.mean() < 0.4                     # the random fp32 share
    # switching: single precision for the first steps of every sequence only
    _, sq2, st2, f2 = W.scf_trace(nseq=8, steps=30, rate=100.0, switch_step=20)
    assert np.array_equal(f2, st2 < 20)
    assert f2.sum() == 8 * 20


def test_synthetic_stage1_reflectors_are_unitary():
    for cplx in (False, True):
        V, tau = W.synthetic_stage1(50, 7, complex_=cplx, seed=3)
        assert V.shape == (50, 43) and tau.shape == (43,)
        for c in (0, 20, 42):
            v = V[c + 7:, c]
            assert v[0] == 1.0 and np.all(V[:c + 7, c] == 0)
            H = np.eye(v.size) - tau[c] * np.outer(v, v.conj())
            assert np.abs(H @ H.conj().T - np.eye(v.size)).max() < 1e-13
