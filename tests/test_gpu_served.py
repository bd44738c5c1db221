"""GPU tests of the served stream (paper_1811_01277_amd.serve): continuous
batching over several streams with admission by device-memory footprint.

* every result of a concurrent, batched run equals the same request run
  alone on the plain one-call-at-a-time path (within the parity tolerance)
  and, on a sample, the CPU oracle;
* the work overlapped (several batches in flight, batches of several
  requests) and the sequence order held (step k+1 started after step k);
* a memory budget below two requests' workspace keeps one batch in flight.
"""
import numpy as np
import pytest

import workload as W
from oracle import bt, checks

pytestmark = pytest.mark.gpu

TOL = {"r64": 1e-12, "r32": 5e-5}


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


def make_stream(torch, dev, nseq=6, steps=3, rate=2000.0, seed=700):
    """Small SCF-like stream: nseq sequences of `steps` solves, n in [130, 420],
    nbw 64, nev = n, a quarter fp32; every request has its own buffers."""
    from paper_1811_01277_amd.serve import Request
    sizes = W.scf_sequence_sizes(nseq, 130, 420, seed=seed)
    t, sq, st, f32 = W.scf_trace(nseq, steps, rate=rate, p32=0.25, seed_arrivals=seed + 1,
                                 seed_dtypes=seed + 2)
    reqs, host, last = [], [], {}
    for i in range(len(t)):
        n = int(sizes[sq[i]])
        dt = "r32" if f32[i] else "r64"
        hh, tau = W.synthetic_reflectors(n, 64, seed=seed * 1000 + i)
        Z = np.asfortranarray(W.gaussian_block(n, n, seed=seed * 1000 + 500 + i))
        npdt = np.float32 if dt == "r32" else np.float64
        q = torch.from_numpy(np.ascontiguousarray(Z.T).astype(npdt)).to(dev).t()
        h = torch.from_numpy(hh.astype(npdt)).to(dev)
        ta = torch.from_numpy(tau.astype(npdt)).to(dev)
        r = Request(rid=i, q=q, hh=h, tau=ta, nbw=64, arrival=float(t[i]),
                    after=last.get(int(sq[i]), -1), seq=int(sq[i]), step=int(st[i]))
        last[int(sq[i])] = i
        reqs.append(r)
        host.append((hh, tau, Z, dt))
    return reqs, host


def test_served_results_equal_alone_and_overlap(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    from paper_1811_01277_amd.serve import Server, latency_stats
    # arrivals close together: more ready requests than slots, so batches form
    reqs, host = make_stream(torch, dev, rate=1e5)
    inputs = [r.q.clone() for r in reqs]
    print(f"served: {len(reqs)} requests", flush=True)
    srv = Server(dev, slots=3, max_batch=8)
    srv.run(reqs)
    torch.cuda.synchronize()
    print("served stats", latency_stats(reqs), "batches", srv.batches, flush=True)
    assert srv.max_busy >= 2, "no two batches ever ran at once"
    assert max(b[1] for b in srv.batches) >= 2, "no batch held more than one request"
    by_rid = {r.rid: r for r in reqs}
    for r in reqs:
        assert r.t_done >= r.t_start >= r.t_ready >= r.arrival
        if r.after >= 0:
            assert r.t_start >= by_rid[r.after].t_done
    for i, r in enumerate(reqs):
        dt = host[i][3]
        q = inputs[i].t().contiguous().t()   # same values, new column-major storage
        assert q.data_ptr() != r.q.data_ptr()
        P.hh_trafo(q, r.hh, r.tau, r.nbw)
        torch.cuda.synchronize()
        err = checks.max_rel_err(r.q.cpu().numpy().astype(np.float64),
                                 q.cpu().numpy().astype(np.float64))
        assert err <= TOL[dt], (i, dt, err)
    for i in (0, len(reqs) // 2, len(reqs) - 1):
        hh, tau, Z, dt = host[i]
        rd = (lambda x: x.astype(np.float32).astype(np.float64)) if dt == "r32" else (lambda x: x)
        n = Z.shape[0]
        ref = bt.bt_tridiag_to_band(rd(hh), rd(tau), rd(Z), n, 64)
        assert checks.max_rel_err(reqs[i].q.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


def test_memory_budget_limits_inflight_work(torch_dev):
    torch, dev = torch_dev
    from paper_1811_01277_amd.serve import Server, footprint
    reqs, _ = make_stream(torch, dev, nseq=4, steps=2, seed=800)
    fps = [footprint(r) for r in reqs]
    srv = Server(dev, slots=3, budget_bytes=min(fps), max_batch=8)
    srv.run(reqs)
    torch.cuda.synchronize()
    print("batches", srv.batches, flush=True)
    # no two requests fit the budget together (a larger one runs alone on an
    # idle device): one request in flight at a time
    assert srv.max_busy == 1 and all(b[1] == 1 for b in srv.batches)
    assert srv.max_in_use <= max(fps)
    assert all(r.t_done is not None for r in reqs)
