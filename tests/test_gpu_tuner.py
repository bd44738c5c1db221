"""GPU tests of the plan tuner: elpa_hh_tune leaves Q untouched and caches a
runnable plan; calls without a plan then run it; a batch whose problems have
plans with different kernels runs them as separate launch sequences with the
same results as single calls; the batch tuner leaves every Q untouched and
returns a uniform plan whose batched run equals single calls under it."""
import numpy as np
import pytest

import workload as W
from oracle import bt, checks

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


@pytest.fixture(autouse=True)
def clean():
    import paper_1811_01277_amd as P
    P.tuner_clear()
    yield
    P.tuner_clear()


def make(torch, dev, n, nbw, nev, seed):
    hh, tau = W.synthetic_reflectors(n, nbw, seed=seed)
    Z = np.asfortranarray(W.gaussian_block(n, nev, seed=seed + 1))
    q = torch.from_numpy(np.ascontiguousarray(Z.T)).to(dev).t()
    return q, torch.from_numpy(hh).to(dev), torch.from_numpy(tau).to(dev), (hh, tau, Z)


@pytest.mark.parametrize("level", [0, 1])
def test_tune_keeps_q_and_plan_is_used(torch_dev, level):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 700, 64, 300
    q, h, t, (hh, tau, Z) = make(torch, dev, n, nbw, nev, 1100 + level)
    before = q.clone()
    print(f"tune level {level}", flush=True)
    plan = P.tune(q, h, t, nbw, level=level)
    torch.cuda.synchronize()
    print("tuned plan", plan, flush=True)
    assert torch.equal(q, before), "tuning modified Q"
    assert P.tuner_get(P.R64, nbw, n, nev) == plan
    assert P.plan_supported(nbw, P.R64, plan["path"], plan["k"])
    P.profile_enable(True)
    try:
        P.hh_trafo(q, h, t, nbw)                 # no plan: the tuned one
        pr = P.profile_last()
    finally:
        P.profile_enable(False)
    assert pr["path"] == plan["path"]
    if plan["k"]:
        assert pr["k"] == plan["k"]
    assert pr["streams"] == (plan["streams"] or 2)
    ref = bt.bt_tridiag_to_band(hh, tau, Z, n, nbw)
    assert checks.max_rel_err(q.cpu().numpy(), ref) <= 1e-12


def test_batch_with_tuned_plans_of_different_kernels(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    # two size classes with different k: two launch sequences in one call
    P.tuner_set(P.R64, 64, 300, 300, path=P.PATH_SPLIT, k=48)
    P.tuner_set(P.R64, 64, 900, 900, path=P.PATH_SPLIT, k=80)
    sizes = [300, 900, 290, 880]      # size classes floor(4 log2 n): 32, 39, 32, 39
    probs, host, singles = [], [], []
    for i, n in enumerate(sizes):
        q, h, t, hst = make(torch, dev, n, 64, n, 1200 + i)
        probs.append((q, h, t, 64))
        host.append(hst)
    for (q, h, t, nbw) in probs:
        qq = q.clone()
        P.hh_trafo(qq, h, t, nbw, path=P.PATH_SPLIT,
                   k=P.tuner_get(P.R64, 64, q.shape[0], q.shape[1])["k"])
        singles.append(qq)
    P.hh_trafo_batched(probs)
    torch.cuda.synchronize()
    for (q, _, _, _), s, (hh, tau, Z), n in zip(probs, singles, host, sizes):
        assert torch.equal(q, s)
        ref = bt.bt_tridiag_to_band(hh, tau, Z, n, 64)
        assert checks.max_rel_err(q.cpu().numpy(), ref) <= 1e-12


def test_tune_batched_keeps_q_and_plan_runs(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    sizes = [200, 333, 470, 610, 257, 700]
    probs, host, before = [], [], []
    for i, n in enumerate(sizes):
        q, h, t, hst = make(torch, dev, n, 32, n, 1300 + i)
        probs.append((q, h, t, 32))
        host.append(hst)
        before.append(q.clone())
    print("tune batched level 1", flush=True)
    plan = P.tune_batched(probs, level=1)
    torch.cuda.synchronize()
    print("tuned batch plan", plan, flush=True)
    assert P.tuner_size() == 0, "batch plans are not cached"
    for q, b in zip(probs, before):
        assert torch.equal(q[0], b), "tuning modified Q"
    assert plan["path"] in (P.PATH_SPLIT, P.PATH_WY, P.PATH_STRIPE)
    singles = []
    for (q, h, t, nbw) in probs:
        qq = q.clone()
        P.hh_trafo(qq, h, t, nbw, **plan)
        singles.append(qq)
    P.hh_trafo_batched(probs, **plan)
    torch.cuda.synchronize()
    for (q, _, _, _), s, (hh, tau, Z), n in zip(probs, singles, host, sizes):
        assert torch.equal(q, s), n
        ref = bt.bt_tridiag_to_band(hh, tau, Z, n, 32)
        assert checks.max_rel_err(q.cpu().numpy(), ref) <= 1e-12, n


def test_autotune_over_a_solve_sequence(torch_dev, tmp_path):
    """SCF-like sequence: every step is a correct back-transformation whichever
    candidate runs; tuning ends after the warm-up and one step per candidate;
    the state can be saved, reloaded and finished; set_best puts the winner in
    the plan cache."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 600, 64, 200
    q, h, t, (hh, tau, Z) = make(torch, dev, n, nbw, nev, 1400)
    ref = bt.bt_tridiag_to_band(hh, tau, Z, n, nbw)
    zq = q.clone()
    at = P.Autotune(P.AUTOTUNE_MEDIUM, n, nev, nbw, P.R64, path=P.PATH_SPLIT, k=64)
    cands = at.candidates
    assert cands == 10
    steps, tuning = 0, True
    while tuning and steps < 4:
        q.copy_(zq)
        tuning = at.step(q, h, t)
        torch.cuda.synchronize()
        assert checks.max_rel_err(q.cpu().numpy(), ref) <= 1e-12, steps
        steps += 1
    f = tmp_path / "at.txt"
    at.save(str(f))
    at.close()
    at = P.Autotune.load(str(f))
    while tuning:
        q.copy_(zq)
        tuning = at.step(q, h, t)
        torch.cuda.synchronize()
        assert checks.max_rel_err(q.cpu().numpy(), ref) <= 1e-12, steps
        steps += 1
        assert steps <= cands + 1
    assert steps == cands + 1                         # warm-up + one per candidate
    best = at.best()
    assert best["path"] == P.PATH_SPLIT and best["k"] == 64
    at.set_best()
    assert P.tuner_get(P.R64, nbw, n, nev) == best
    q.copy_(zq)
    assert not at.step(q, h, t)                       # runs the best from now on
    torch.cuda.synchronize()
    assert checks.max_rel_err(q.cpu().numpy(), ref) <= 1e-12
