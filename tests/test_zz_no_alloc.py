"""GPU test of the allocation-free entry point elpa_hh_trafo_noalloc (through
the C ABI): two calls in a row, the second on a smaller problem, each equal to
elpa_hh_trafo on the same inputs to the parity bar (1e-12 max-abs relative for
fp64, 5e-5 for fp32), and checked against the oracle on sampled columns; a
problem whose workspace exceeds the fixed scratch is refused with
ELPA_ERR_ADMIT and Q is left untouched; nbw without a two-lane kernel runs the
reference kernel.
"""
import numpy as np
import pytest

import workload as W
from oracle import bt, checks

pytestmark = pytest.mark.gpu

TOL = {"r64": 1e-12, "c64": 1e-12, "r32": 5e-5}


@pytest.fixture(scope="module")
def torch_dev():
    import time
    t0 = time.time()
    print("importing torch", flush=True)
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1811_01277_amd as P
    P.library()
    print(f"torch ready after {time.time() - t0:.1f} s", flush=True)
    return torch, torch.device("cuda:0")


def npdt(dt):
    return {"r64": np.float64, "r32": np.float32, "c64": np.complex128}[dt]


def inputs(torch, dev, n, nbw, nev, dt, seed):
    cplx = dt == "c64"
    hh, tau = W.synthetic_reflectors(n, nbw, complex_=cplx, seed=seed)
    Z = np.asfortranarray(W.gaussian_block(n, nev, complex_=cplx, seed=seed + 1))
    h = torch.from_numpy(hh.astype(npdt(dt))).to(dev)
    t = torch.from_numpy(tau.astype(npdt(dt))).to(dev)
    q = torch.from_numpy(np.ascontiguousarray(Z.T).astype(npdt(dt))).to(dev).t()
    return (hh, tau, Z), (h, t, q)


def rounded(x, dt):
    return x.astype(np.float32).astype(np.float64) if dt == "r32" else x


def code(P, dt):
    return {"r64": P.R64, "r32": P.R32, "c64": P.C64}[dt]


@pytest.mark.parametrize("dt", ["r64", "r32", "c64"])
def test_noalloc_equals_allocating_entry_two_calls(torch_dev, dt):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    # first call larger than the second: the scratch keeps the first call's
    # contents when the second runs
    for (n, nbw, nev, seed) in [(1500, 64, 1000, 11), (700, 32, 300, 12)]:
        print(f"noalloc {dt} n={n} nbw={nbw} nev={nev}", flush=True)
        assert P.workspace_bytes(n, nev, nbw, code(P, dt), P.PATH_SPLIT) <= P.NOALLOC_SCRATCH_BYTES
        (hh, tau, Z), (h, t, q) = inputs(torch, dev, n, nbw, nev, dt, seed)
        q_ref = q.t().clone().t()
        P.hh_trafo(q_ref, h, t, nbw)
        rc = P.hh_trafo_noalloc_ptr(n, nev, nbw, h.data_ptr(), t.data_ptr(), q.data_ptr(),
                                    q.stride(1), code(P, dt),
                                    torch.cuda.current_stream(dev).cuda_stream)
        assert rc == 0, P.strerror(rc)
        torch.cuda.synchronize()
        a = q.cpu().numpy().astype(np.complex128 if dt == "c64" else np.float64)
        b = q_ref.cpu().numpy().astype(a.dtype)
        err = checks.max_rel_err(a, b)
        print(f"  vs elpa_hh_trafo: max-abs rel diff {err:.3e}, bitwise {np.array_equal(a, b)}",
              flush=True)
        assert err <= TOL[dt]
        cols = sorted({0, 31, 32, nev // 2, nev - 1})
        ref = bt.bt_tridiag_to_band(rounded(hh, dt), rounded(tau, dt),
                                    rounded(np.asfortranarray(Z[:, cols]), dt), n, nbw)
        assert checks.max_rel_err(a[:, cols], ref) <= TOL[dt]


def test_noalloc_refuses_beyond_scratch_and_runs_reference_nbw(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 20000, 64, 2000           # stripe copy alone ~320 MB
    assert P.workspace_bytes(n, nev, nbw, P.R64, P.PATH_SPLIT) > P.NOALLOC_SCRATCH_BYTES
    q = torch.zeros(64, device=dev, dtype=torch.float64)
    before = q.clone()
    rc = P.hh_trafo_noalloc_ptr(n, nev, nbw, q.data_ptr(), q.data_ptr(), q.data_ptr(), n, P.R64)
    assert rc == -7, rc
    torch.cuda.synchronize()
    assert torch.equal(q, before)
    # nbw = 7 has no two-lane kernel: the reference kernel, no workspace
    (hh, tau, Z), (h, t, qq) = inputs(torch, dev, 300, 7, 50, "r64", 21)
    rc = P.hh_trafo_noalloc_ptr(300, 50, 7, h.data_ptr(), t.data_ptr(), qq.data_ptr(),
                                qq.stride(1), P.R64)
    assert rc == 0
    torch.cuda.synchronize()
    ref = bt.bt_tridiag_to_band(hh, tau, Z, 300, 7)
    assert checks.max_rel_err(qq.cpu().numpy(), ref) <= 1e-12
