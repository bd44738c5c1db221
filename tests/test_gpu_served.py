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
    slack = 1e-4   # host clock vs device event times (same time base to a few us)
    for r in reqs:
        assert r.t_done >= r.t_start                       # both device events
        assert r.t_start >= r.t_ready - slack and r.t_ready >= r.arrival
        if r.after >= 0:
            assert r.t_start >= by_rid[r.after].t_done     # both device events
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


def test_scf_precision_switching_through_device_reductions(torch_dev):
    """An SCF-like stream with precision switching (single precision for the
    first steps of a sequence, double for the rest), every request derived
    from its own matrix A_k = A_0 + 1e-3 k (E + E^T) by the device reductions
    (full -> band, band -> tridiagonal, divide and conquer, all fp64; the
    fp32 requests get those results rounded), served with continuous
    batching.  Every result against the oracle on the same reflectors and
    tridiagonal eigenvectors (fp64: 1e-12; fp32: 5e-5 against the oracle of
    the rounded inputs, error against the unrounded fp64 oracle printed), and
    each step's full eigenvectors (band -> full on the device) satisfy
    A_k Z = Z Lambda to the precision of the request."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    from paper_1811_01277_amd.serve import Request, Server, latency_stats
    nbw, steps, switch = 32, 4, 2
    sizes = [200, 260, 330]
    reqs, meta, last = [], [], {}
    rid = 0
    for step in range(steps):
        for sq, n in enumerate(sizes):
            A0 = W.sym_gaussian(n, 900 + sq)
            E = np.random.Generator(np.random.PCG64(950 + sq)).standard_normal((n, n))
            A = A0 + 1e-3 * step * (E + E.T)
            a = torch.from_numpy(A.copy()).to(dev).t()       # symmetric: column-major view
            v, t1 = P.full_to_band(a, nbw)
            d, e, hh, tau = P.band_to_tridiag(a, nbw)
            lam, z = P.tridiag_eigh(d, e, n)
            torch.cuda.synchronize()
            f32 = step < switch
            host = (hh.cpu().numpy(), tau.cpu().numpy(), np.asfortranarray(z.cpu().numpy()))
            if f32:
                q, h, ta = z.t().float().t(), hh.float(), tau.float()
            else:
                q, h, ta = z.t().contiguous().t(), hh, tau
            r = Request(rid=rid, q=q, hh=h, tau=ta, nbw=nbw, arrival=0.0,
                        after=last.get(sq, -1), seq=sq, step=step)
            last[sq] = rid
            reqs.append(r)
            meta.append((A, host, v, t1, lam, f32, n))
            rid += 1
    srv = Server(dev, slots=3, max_batch=8)
    srv.run(reqs)
    torch.cuda.synchronize()
    print("switching stream", latency_stats(reqs), "batches", srv.batches, flush=True)
    for r, (A, (hh, tau, z), v, t1, lam, f32, n) in zip(reqs, meta):
        got = r.q.cpu().numpy().astype(np.float64)
        ref64 = bt.bt_tridiag_to_band(hh, tau, z, n, nbw)
        if f32:
            rd = lambda x: x.astype(np.float32).astype(np.float64)
            ref = bt.bt_tridiag_to_band(rd(hh), rd(tau), rd(z), n, nbw)
            err = checks.max_rel_err(got, ref)
            print(f"  seq {r.seq} step {r.step} fp32: {err:.2e} vs rounded-input oracle, "
                  f"{checks.max_rel_err(got, ref64):.2e} vs fp64 oracle", flush=True)
            assert err <= 5e-5
        else:
            assert checks.max_rel_err(got, ref64) <= 1e-12
        # the request's band eigenvectors to the full matrix's on the device
        if f32:
            P.bt2_trafo(r.q, v.float(), t1.float(), nbw)
        else:
            P.bt2_trafo(r.q, v, t1, nbw)
        torch.cuda.synchronize()
        Z = r.q.cpu().numpy().astype(np.float64)
        lamh = lam.cpu().numpy()
        R = A @ Z - Z * lamh[None, :]
        eps = 2.0 ** -24 if f32 else 2.0 ** -52
        ratio = np.abs(R).sum(0).max() / (np.abs(A).sum(0).max() * n * eps)
        assert ratio < 50, (r.seq, r.step, f32, ratio)


def test_served_with_graphs_equals_alone(torch_dev):
    """Served stream whose lone requests replay per-sequence graphs of
    prepared batches: every result equals the request run alone, and graphs
    were replayed."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    from paper_1811_01277_amd.serve import Server, latency_stats
    reqs, host = make_stream(torch, dev, nseq=4, steps=3, rate=300.0, seed=1100)
    inputs = [r.q.clone() for r in reqs]
    srv = Server(dev, slots=3, max_batch=8)
    held = srv.prepare_graphs(reqs)
    srv.run(reqs)
    torch.cuda.synchronize()
    print("served with graphs", latency_stats(reqs), "replays", srv.replays, "held", held,
          flush=True)
    assert srv.replays > 0 and held > 0
    vias = {r.via for r in reqs}
    assert "graph" in vias and vias <= {"graph", "single", "batched"}
    for i, r in enumerate(reqs):
        q = inputs[i].t().contiguous().t()
        # a replay or a lone call runs the library's single-call kernel; a
        # batched call runs the two-lane kernel, bitwise equal to that kernel
        # called alone
        if r.via == "batched":
            P.hh_trafo(q, r.hh, r.tau, r.nbw, path=P.PATH_SPLIT)
        else:
            P.hh_trafo(q, r.hh, r.tau, r.nbw)
        torch.cuda.synchronize()
        assert torch.equal(q, r.q), (i, r.via)
    srv.close_graphs()
