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
