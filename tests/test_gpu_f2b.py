"""GPU full -> band reduction (include/elpa_f2b.h) against the oracle's
full_to_band, and the whole eigenvector chain with every stage but the
tridiagonal solve on the device."""
import numpy as np
import pytest

import workload as W
from oracle import checks, stage1, tridiag

from bt2_layout import panels_to_abi

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


def to_dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(dev).t()


CASES = [(97, 32, 501), (130, 64, 502), (300, 32, 503), (600, 64, 504), (50, 7, 505),
         (20, 19, 506), (65, 64, 507)]


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}_b{c[1]}" for c in CASES])
def test_f2b_matches_oracle(torch_dev, case, cplx):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, b, seed = case
    A = W.herm_gaussian(n, seed) if cplx else W.sym_gaussian(n, seed)
    B0, panels = stage1.full_to_band(A, b)
    V0, t0 = panels_to_abi(panels, n, b, np.complex128 if cplx else np.float64)
    print(f"f2b n={n} b={b} cplx={cplx}", flush=True)
    a = to_dev(torch, dev, A)
    v, tau = P.full_to_band(a, b)
    torch.cuda.synchronize()
    B = a.cpu().numpy()
    scale = float(np.max(np.abs(A)))
    # band structure, Hermitian storage, and the spectrum kept
    far = np.abs(np.subtract.outer(np.arange(n), np.arange(n))) > b
    assert np.all(B[far] == 0)
    assert np.max(np.abs(B - B.conj().T)) <= 1e-13 * scale * n
    lam = np.linalg.eigvalsh(A)
    assert np.max(np.abs(np.linalg.eigvalsh(B) - lam)) <= 50 * n * np.finfo(float).eps * \
        np.linalg.norm(A, 2)
    # the oracle's band matrix and reflectors
    assert np.max(np.abs(B - B0)) <= 1e-11 * scale * n ** 0.5
    N = n - b
    Vg, tg = v.cpu().numpy(), tau.cpu().numpy()
    for c in range(N):
        ref = V0[c + b + 1:, c]
        assert np.max(np.abs(Vg[c + b + 1:, c] - ref), initial=0.0) <= 1e-9 * max(1.0, np.max(np.abs(ref), initial=0.0))
    assert np.max(np.abs(tg[:N] - t0[:N])) <= 1e-10


@pytest.mark.parametrize("cplx", [False, True])
def test_eigenvectors_all_stages_but_the_tridiagonal_solve_on_gpu(torch_dev, cplx):
    """full -> band, band -> tridiagonal, tridiagonal -> band and band -> full
    on the GPU (reflectors and band matrix never leave the device), the
    tridiagonal eigenpairs from the oracle: A Z = Z Lambda, Z^H Z = I."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, b = 500, 32
    A = W.herm_gaussian(n, 511) if cplx else W.sym_gaussian(n, 511)
    a = to_dev(torch, dev, A)
    v, tau_v = P.full_to_band(a, b)
    d, e, hh, tau_h = P.band_to_tridiag(a, b)
    lam, Zt = tridiag.eigh_tridiag(d.cpu().numpy(), e.cpu().numpy())
    dt = np.complex128 if cplx else np.float64
    q = to_dev(torch, dev, Zt.astype(dt))
    P.hh_trafo(q, hh, tau_h, b)
    P.bt2_trafo(q, v, tau_v, b)
    torch.cuda.synchronize()
    Z = q.cpu().numpy()
    assert checks.residual_ratio(A, Z, lam) < 50
    assert checks.orth_ratio(Z) < 50
    assert np.max(np.abs(lam - np.linalg.eigvalsh(A))) <= 50 * n * np.finfo(float).eps * \
        np.linalg.norm(A, 2)
