"""GPU tests of the batched entry point elpa_hh_trafo_batched.

* every problem of a batch matches the oracle (same bar as single calls);
* a problem gives the bitwise same result alone and inside a batch (same
  kernel variant, same per-task arithmetic);
* mixed element types and nbw in one call; an invalid problem rejects the
  whole call before anything runs.
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


def make(torch, dev, n, nbw, nev, dt, seed):
    cplx = dt == "c64"
    hh, tau = W.synthetic_reflectors(n, nbw, complex_=cplx, seed=seed)
    Z = np.asfortranarray(W.gaussian_block(n, nev, complex_=cplx, seed=seed + 1))
    q = torch.from_numpy(np.ascontiguousarray(Z.T).astype(npdt(dt))).to(dev).t()
    h = torch.from_numpy(hh.astype(npdt(dt))).to(dev)
    t = torch.from_numpy(tau.astype(npdt(dt))).to(dev)
    return (q, h, t, nbw), (hh, tau, Z)


def rounded(x, dt):
    return x.astype(np.float32).astype(np.float64) if dt == "r32" else x


def test_batch_matches_oracle_and_single_calls(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    sizes = [(65, 32, 65), (200, 32, 200), (333, 32, 101), (97, 32, 97), (512, 32, 512),
             (130, 64, 129), (260, 64, 64)]
    probs, host = [], []
    for i, (n, nbw, nev) in enumerate(sizes):
        p, h = make(torch, dev, n, nbw, nev, "r64", 1000 + i)
        probs.append(p)
        host.append(h)
    singles = []
    for (q, h, t, nbw) in probs:
        qq = q.clone()  # new storage, same column-major strides
        assert qq.data_ptr() != q.data_ptr() and qq.stride() == q.stride()
        P.hh_trafo(qq, h, t, nbw)
        singles.append(qq)
    print("batch of", len(probs), "problems", flush=True)
    P.hh_trafo_batched(probs)
    torch.cuda.synchronize()
    for (q, _, _, nbw), (hh, tau, Z), s, (n, _, nev) in zip(probs, host, singles, sizes):
        ref = bt.bt_tridiag_to_band(hh, tau, Z, n, nbw)
        got = q.cpu().numpy()
        assert checks.max_rel_err(got, ref) <= TOL["r64"]
        assert torch.equal(q, s), "batched result differs from the single call"


@pytest.mark.parametrize("family", ["default", "wy"])
def test_fp32_batch_equals_single_calls(torch_dev, family):
    """fp32 problems (library choice: the two-lane kernel; and the compact-WY
    MFMA path) give bitwise the same result in a batch as alone, and match the
    oracle."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    path = P.PATH_WY if family == "wy" else None
    sizes = [(300, 64, 150), (517, 64, 517), (130, 32, 33), (260, 64, 97)]
    probs, host = [], []
    for i, (n, nbw, nev) in enumerate(sizes):
        p, h = make(torch, dev, n, nbw, nev, "r32", 4000 + i)
        probs.append(p)
        host.append(h)
    singles = []
    for (q, h, t, nbw) in probs:
        qq = q.clone()
        P.hh_trafo(qq, h, t, nbw, path=path)
        singles.append(qq)
    P.profile_enable(True)
    try:
        P.hh_trafo_batched(probs, path=path)
        pr = P.profile_last()
    finally:
        P.profile_enable(False)
    torch.cuda.synchronize()
    assert pr["path"] == P.PATH_AUTO or pr["launches"] > 0
    for (q, _, _, nbw), (hh, tau, Z), s, (n, _, nev) in zip(probs, host, singles, sizes):
        assert torch.equal(q, s), "batched fp32 result differs from the single call"
        ref = bt.bt_tridiag_to_band(rounded(hh, "r32"), rounded(tau, "r32"), rounded(Z, "r32"),
                                    n, nbw)
        assert checks.max_rel_err(q.cpu().numpy().astype(np.float64), ref) <= TOL["r32"]


def test_batch_mixed_dtypes(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    spec = [(150, 32, 90, "r64"), (150, 32, 90, "r32"), (120, 32, 70, "c64"),
            (90, 7, 40, "r64"), (77, 64, 33, "r32")]
    probs, host = [], []
    for i, (n, nbw, nev, dt) in enumerate(spec):
        p, h = make(torch, dev, n, nbw, nev, dt, 2000 + i)
        probs.append(p)
        host.append(h)
    print("mixed batch", flush=True)
    P.hh_trafo_batched(probs)
    torch.cuda.synchronize()
    for (q, _, _, nbw), (hh, tau, Z), (n, _, nev, dt) in zip(probs, host, spec):
        ref = bt.bt_tridiag_to_band(rounded(hh, dt), rounded(tau, dt), rounded(Z, dt), n, nbw)
        err = checks.max_rel_err(q.cpu().numpy(), ref)
        assert err <= TOL[dt], (n, nbw, dt, err)


def test_invalid_problem_rejects_whole_batch(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    a, _ = make(torch, dev, 100, 32, 40, "r64", 3000)
    b, _ = make(torch, dev, 100, 32, 40, "r64", 3001)
    before = a[0].clone()
    bad = (b[0], b[1], b[2], 0)  # nbw = 0
    with pytest.raises(P.ElpaError) as e:
        P.hh_trafo_batched([a, bad])
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert torch.equal(a[0], before)


def test_batched_workload_sampled(torch_dev):
    """The batched workload shape: 256 problems, n ~ U{200..2000}, nbw = 32,
    nev = n, one call; four problems (smallest, largest, two others) checked
    completely against the oracle, every problem's column norms checked."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    sizes = W.batched_sizes(256, 200, 2000, seed=401)
    probs, host = [], {}
    check = {int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 200}
    norms0 = []
    for i, n in enumerate(sizes):
        n = int(n)
        hh, tau = W.synthetic_reflectors(n, 32, seed=401000 + i)
        Z = np.asfortranarray(W.gaussian_block(n, n, seed=402000 + i))
        q = torch.from_numpy(np.ascontiguousarray(Z.T)).to(dev).t()
        probs.append((q, torch.from_numpy(hh).to(dev), torch.from_numpy(tau).to(dev), 32))
        norms0.append(torch.linalg.vector_norm(q, dim=0))
        if i in check:
            host[i] = (hh, tau, Z)
    print("batched workload: 256 problems", flush=True)
    P.hh_trafo_batched(probs)
    torch.cuda.synchronize()
    for i, (q, _, _, _) in enumerate(probs):
        rel = ((torch.linalg.vector_norm(q, dim=0) - norms0[i]).abs() / norms0[i]).max().item()
        assert rel < 1e-12, (i, rel)
    for i, (hh, tau, Z) in host.items():
        n = int(sizes[i])
        ref = bt.bt_tridiag_to_band(hh, tau, Z, n, 32)
        assert checks.max_rel_err(probs[i][0].cpu().numpy(), ref) <= TOL["r64"], i
