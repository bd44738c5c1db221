"""GPU tests of the batched entry point elpa_hh_trafo_batched.

* every problem of a batch matches the oracle (same bar as single calls);
* a problem gives the bitwise same result alone and inside a batch (same
  kernel variant, same per-column arithmetic);
* the problems of a batch that run the two-lane kernel run in one launch
  (the batched workload included);
* mixed element types and nbw in one call; an invalid problem rejects the
  whole call before anything runs.
"""
import numpy as np
import pytest

import workload as W
from oracle import bt, checks

pytestmark = pytest.mark.gpu


def batched_k(q, nbw, path=None):
    """k of the kernel a batched call runs for this problem (the batched
    choice can differ from a single call's: k = 96 at nbw = 32)."""
    import paper_1811_01277_amd as P
    from paper_1811_01277_amd import binding as B
    n, nev = q.shape
    return P.chosen_plan(n, nev, nbw, B._dtype_code(q), batched=True, path=path)["k"]

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


@pytest.mark.parametrize("sched", ["one_launch", "one_launch_linear", "diagonal", "auto"])
def test_batch_matches_oracle_and_single_calls(torch_dev, sched):
    """one_launch deals each problem's stripes to one die (the default order);
    one_launch_linear numbers them problem by problem in workgroup order."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    batch = {"one_launch": P.BATCH_ONE_LAUNCH, "one_launch_linear": P.BATCH_ONE_LAUNCH,
             "diagonal": P.BATCH_DIAGONAL, "auto": 0}[sched]
    order = P.ORDER_LINEAR if sched == "one_launch_linear" else 0
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
        # the kernel batched calls run
        P.hh_trafo(qq, h, t, nbw, path=P.PATH_SPLIT, k=batched_k(q, nbw))
        singles.append(qq)
    print("batch of", len(probs), "problems", flush=True)
    P.profile_enable(True)
    try:
        P.hh_trafo_batched(probs, batch=batch, order=order)
        pr = P.profile_last()
    finally:
        P.profile_enable(False)
    torch.cuda.synchronize()
    # every problem runs the two-lane kernel: one group per nbw (32 and 64),
    # each one launch or its diagonal sequence
    if sched.startswith("one_launch"):
        assert pr["launches"] == 2, pr
    elif sched == "diagonal":
        assert pr["launches"] > 2, pr
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
    path = P.PATH_WY if family == "wy" else P.PATH_SPLIT
    sizes = [(300, 64, 150), (517, 64, 517), (130, 32, 33), (260, 64, 97)]
    probs, host = [], []
    for i, (n, nbw, nev) in enumerate(sizes):
        p, h = make(torch, dev, n, nbw, nev, "r32", 4000 + i)
        probs.append(p)
        host.append(h)
    singles = []
    for (q, h, t, nbw) in probs:
        qq = q.clone()
        P.hh_trafo(qq, h, t, nbw, path=path, k=batched_k(q, nbw, path))
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
    # single calls of the checked problems, for bitwise comparison
    singles = {}
    for i in check:
        q, h, t, nbw = probs[i]
        qq = q.clone()
        P.hh_trafo(qq, h, t, nbw, path=P.PATH_SPLIT, k=batched_k(q, nbw))
        singles[i] = qq
    print("batched workload: 256 problems", flush=True)
    P.profile_enable(True)
    try:
        P.hh_trafo_batched(probs)
        pr = P.profile_last()
    finally:
        P.profile_enable(False)
    torch.cuda.synchronize()
    print(f"  one launch: {pr['launches']} launch(es), {pr['kernel_ms']:.2f} ms", flush=True)
    assert pr["launches"] == 1, pr
    for i in check:
        assert torch.equal(probs[i][0], singles[i]), i
    for i, (q, _, _, _) in enumerate(probs):
        rel = ((torch.linalg.vector_norm(q, dim=0) - norms0[i]).abs() / norms0[i]).max().item()
        assert rel < 1e-12, (i, rel)
    for i, (hh, tau, Z) in host.items():
        n = int(sizes[i])
        ref = bt.bt_tridiag_to_band(hh, tau, Z, n, 32)
        assert checks.max_rel_err(probs[i][0].cpu().numpy(), ref) <= TOL["r64"], i


@pytest.mark.parametrize("dt", ["r32", "c64"])
def test_one_launch_batch_other_dtypes(torch_dev, dt):
    """fp32 and complex problems of the two-lane kernel: one launch per
    (dtype, nbw) group, each result bitwise the single call's and within the
    oracle's bar; problems of uneven n and nev, ragged stripes."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    sizes = [(257, 64, 100), (1000, 64, 33), (70, 64, 70), (400, 64, 65)]
    probs, host = [], []
    for i, (n, nbw, nev) in enumerate(sizes):
        p, h = make(torch, dev, n, nbw, nev, dt, 5000 + i)
        probs.append(p)
        host.append(h)
    singles = []
    for (q, h, t, nbw) in probs:
        qq = q.clone()
        P.hh_trafo(qq, h, t, nbw, path=P.PATH_SPLIT)
        singles.append(qq)
    P.profile_enable(True)
    try:
        P.hh_trafo_batched(probs, batch=P.BATCH_ONE_LAUNCH)
        pr = P.profile_last()
    finally:
        P.profile_enable(False)
    torch.cuda.synchronize()
    assert pr["path"] == P.PATH_SPLIT and pr["launches"] == 1, pr
    for (q, _, _, nbw), (hh, tau, Z), s, (n, _, nev) in zip(probs, host, singles, sizes):
        assert torch.equal(q, s), (n, nev)
        ref = bt.bt_tridiag_to_band(rounded(hh, dt), rounded(tau, dt), rounded(Z, dt), n, nbw)
        assert checks.max_rel_err(q.cpu().numpy().astype(ref.dtype), ref) <= TOL[dt]


def test_few_large_problems_take_the_diagonal_schedule(torch_dev):
    """Two large problems have too few stripes to fill the device in one
    launch: the library's model picks the diagonal sequence, and the result
    equals the forced single launch bitwise (same per-column arithmetic)."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    sizes = [(3000, 64, 3000), (2500, 64, 1200)]
    probs, probs2 = [], []
    for i, (n, nbw, nev) in enumerate(sizes):
        p, _ = make(torch, dev, n, nbw, nev, "r64", 6000 + i)
        probs.append(p)
        probs2.append((p[0].clone(), p[1], p[2], p[3]))
    P.profile_enable(True)
    try:
        P.hh_trafo_batched(probs)
        auto = P.profile_last()
        P.hh_trafo_batched(probs2, batch=P.BATCH_ONE_LAUNCH)
        one = P.profile_last()
    finally:
        P.profile_enable(False)
    torch.cuda.synchronize()
    print(f"  auto: {auto['launches']} launches {auto['kernel_ms']:.2f} ms; one launch "
          f"{one['kernel_ms']:.2f} ms", flush=True)
    assert auto["launches"] > 1 and one["launches"] == 1
    for a, b in zip(probs, probs2):
        assert torch.equal(a[0], b[0])
