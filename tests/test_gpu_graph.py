"""A single-problem call captured into a HIP graph (torch.cuda.graph) and
replayed: the capture records the library's stream-ordered workspace
allocation, the fork/join of its stripe-group streams and every launch.
Each replay runs on fresh input (written eagerly between replays, with other
eager work and synchronizations in between) and must equal the eager call
bitwise."""
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


@pytest.mark.parametrize("dt,path", [("r64", 3), ("c64", 3), ("r32", 4), ("r64", 2)])
def test_graph_replay_equals_eager(torch_dev, dt, path):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 600, 64, 190
    tdt = {"r64": torch.float64, "r32": torch.float32, "c64": torch.complex128}[dt]
    cplx = dt == "c64"
    hh, tau = W.synthetic_reflectors(n, nbw, complex_=cplx, seed=1500)
    h = torch.from_numpy(hh).to(dev).to(tdt)
    t = torch.from_numpy(tau).to(dev).to(tdt)
    inputs = [torch.from_numpy(np.ascontiguousarray(
        W.gaussian_block(n, nev, complex_=cplx, seed=1501 + i).T)).to(dev).to(tdt).t()
        for i in range(3)]
    eager = []
    for z in inputs:
        q = z.clone()
        P.hh_trafo(q, h, t, nbw, path=path)
        eager.append(q)
    torch.cuda.synchronize()
    q = inputs[0].clone()                      # the graph's fixed buffer
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        P.hh_trafo(q, h, t, nbw, path=path, stream=s)   # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print(f"capturing dt={dt} path={path}", flush=True)
    with torch.cuda.graph(g, stream=s):
        P.hh_trafo(q, h, t, nbw, path=path, stream=s)
    torch.cuda.synchronize()
    for rep in range(2):
        for i, z in enumerate(inputs):
            q.copy_(z)                         # eager work between replays
            junk = torch.randn(1000, device=dev).sum()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(q, eager[i]), (rep, i)
            assert torch.isfinite(junk)


@pytest.mark.parametrize("sched", ["one_launch", "diagonal", "single", "single_wy"])
def test_prepared_batch_graph_replay_equals_eager(torch_dev, sched):
    """A prepared batch (elpa_hh_batch_create: tables and workspace on the
    device once) captured into a graph: every replay, with fresh input and
    other eager work in between, equals the eager batched call bitwise.
    Schedules: the one-launch and diagonal batched forms, and a single
    problem (the single-call kernel choice, compact-WY here for complex and
    for fp64 at n >= 3000 with nev >= 1024, its stripe groups forked and
    joined inside the capture), which equals the single-problem call
    bitwise."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    spec = {"one_launch": [(300, 64, 120, "r64"), (520, 64, 70, "r64"), (200, 64, 200, "r64")],
            "diagonal": [(300, 32, 120, "r32"), (700, 32, 90, "r32")],
            "single": [(900, 64, 400, "c64")],
            "single_wy": [(3100, 64, 1100, "r64")]}[sched]
    batch = {"one_launch": P.BATCH_ONE_LAUNCH, "diagonal": P.BATCH_DIAGONAL, "single": 0,
             "single_wy": 0}[sched]
    tdt = {"r64": torch.float64, "r32": torch.float32, "c64": torch.complex128}
    probs, inputs = [], []
    for i, (n, nbw, nev, dt) in enumerate(spec):
        cplx = dt == "c64"
        hh, tau = W.synthetic_reflectors(n, nbw, complex_=cplx, seed=1600 + i)
        h = torch.from_numpy(hh).to(dev).to(tdt[dt])
        t = torch.from_numpy(tau).to(dev).to(tdt[dt])
        zs = [torch.from_numpy(np.ascontiguousarray(
            W.gaussian_block(n, nev, complex_=cplx, seed=1700 + 10 * i + r).T)).to(dev)
            .to(tdt[dt]).t() for r in range(3)]
        q = zs[0].clone()
        probs.append((q, h, t, nbw))
        inputs.append(zs)
    # eager reference: the plain batched call on each input set; a batch of
    # one problem runs the single-problem call (the library's kernel choice)
    eager = []
    for r in range(3):
        cur = [(zs[r].clone(), h, t, nbw) for zs, (_, h, t, nbw) in zip(inputs, probs)]
        if len(cur) == 1:
            P.hh_trafo(*cur[0])
        else:
            P.hh_trafo_batched(cur, batch=batch)
        eager.append([c[0] for c in cur])
    torch.cuda.synchronize()
    B = P.Batch(probs, batch=batch)
    assert B.nbytes > 0
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        B.run(s)                                # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print(f"capturing prepared batch {sched}", flush=True)
    with torch.cuda.graph(g, stream=s):
        B.run(s)
    torch.cuda.synchronize()
    for rep in range(2):
        for r in range(3):
            for (q, _, _, _), zs in zip(probs, inputs):
                q.copy_(zs[r])
            junk = torch.randn(1000, device=dev).sum()
            P.hh_trafo_batched([(inputs[0][r].clone(), probs[0][1], probs[0][2], probs[0][3])])
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for (q, _, _, _), e in zip(probs, eager[r]):
                assert torch.equal(q, e), (sched, rep, r)
            assert torch.isfinite(junk)
    # eager runs of the prepared batch equal the batched call too
    for (q, _, _, _), zs in zip(probs, inputs):
        q.copy_(zs[1])
    B.run()
    torch.cuda.synchronize()
    for (q, _, _, _), e in zip(probs, eager[1]):
        assert torch.equal(q, e)
    B.close()
