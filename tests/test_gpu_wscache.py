"""Workspace cache of the back-transformation calls (GPU).

* calls on three streams, issued back to back from one host thread and from
  three threads, reusing cached blocks across sizes and streams: every
  result equals the same call made alone on one stream, bitwise;
* the cache's accounting: a call leaves its block cached, a repeated call of
  the same size on the same stream reuses it, and release frees idle blocks.
"""
import threading

import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu


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


def _problems(torch, dev, spec, seed):
    out = []
    for i, (n, nev, dt) in enumerate(spec):
        tdt = {"r64": torch.float64, "r32": torch.float32}[dt]
        hh, tau = W.synthetic_reflectors(n, 64, seed=seed + i)
        Z = W.gaussian_block(n, nev, seed=seed + 50 + i)
        q = torch.from_numpy(np.ascontiguousarray(Z.T)).to(dev).to(tdt).t()
        out.append((q, torch.from_numpy(hh).to(dev).to(tdt),
                    torch.from_numpy(tau).to(dev).to(tdt)))
    return out


SPEC = [(700, 300, "r64"), (1500, 200, "r64"), (3200, 160, "r64"), (900, 400, "r32"),
        (3100, 100, "r32"), (650, 650, "r64")]


@pytest.mark.parametrize("threads", [False, True])
def test_concurrent_streams_equal_alone(torch_dev, threads):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    probs = _problems(torch, dev, SPEC, 3000)
    # reference: one at a time on one stream
    ref = []
    for q, h, t in probs:
        x = q.clone()
        P.hh_trafo(x, h, t, 64)
        ref.append(x)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(device=dev) for _ in range(3)]
    print(f"concurrent streams, threads={threads}", flush=True)
    for rep in range(3):
        outs = [q.clone() for q, _, _ in probs]
        torch.cuda.synchronize()

        def issue(k):
            torch.cuda.set_device(dev)
            for i in range(k, len(probs), 3):
                P.hh_trafo(outs[i], probs[i][1], probs[i][2], 64, stream=streams[k])

        if threads:
            ts = [threading.Thread(target=issue, args=(k,)) for k in range(3)]
            for t_ in ts:
                t_.start()
            for t_ in ts:
                t_.join()
        else:
            for k in range(3):
                issue(k)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (rep, i)


def test_cache_accounting_and_release(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    torch.cuda.synchronize()
    P.workspace_release()
    base = P.workspace_cached()
    (q, h, t), = _problems(torch, dev, [(2000, 500, "r64")], 3100)
    s = torch.cuda.Stream(device=dev)
    P.hh_trafo(q, h, t, 64, stream=s)
    one = P.workspace_cached()
    need = P.workspace_bytes(2000, 500, 64, P.R64)
    assert one - base >= need > 0
    for _ in range(3):                        # same size, same stream: reused
        P.hh_trafo(q, h, t, 64, stream=s)
    assert P.workspace_cached() == one
    torch.cuda.synchronize()
    freed = P.workspace_release()
    assert freed >= one - base and P.workspace_cached() == 0


def test_cache_evicts_idle_blocks_beyond_its_bound(torch_dev):
    """Idle blocks beyond 8 GiB are freed, least recently used first, before a
    new block is allocated: a large call's block (n = nev = 20000) is evicted
    when a smaller call that cannot reuse it (less than half its size) would
    take the idle total past the bound."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    bound = 8 << 30
    na, nb_ = 20000, 12000
    wa = P.workspace_bytes(na, na, 64, P.R64)
    wb = P.workspace_bytes(nb_, nb_, 64, P.R64)
    assert wb < wa // 2 and wa > bound - wb, (wa, wb)   # the case this test needs
    torch.cuda.synchronize()
    P.workspace_release()
    g = torch.Generator(device=dev)
    g.manual_seed(3200)
    print(f"eviction: workspaces {wa / 1e9:.2f} and {wb / 1e9:.2f} GB", flush=True)
    for n in (na, nb_):
        hh, tau = W.device_reflectors(torch, n, 64, dev, g)
        q = W.device_block(torch, n, n, dev, g)
        P.hh_trafo(q, hh, tau, 64)
        torch.cuda.synchronize()
        held = P.workspace_cached()
        if n == na:
            assert held >= wa
        else:
            assert wb <= held < wa, held       # the large block was freed
        del hh, tau, q
    P.workspace_release()
    assert P.workspace_cached() == 0
