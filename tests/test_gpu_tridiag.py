"""GPU divide-and-conquer tridiagonal eigensolver (include/elpa_tridiag.h)
against the oracle's bisection + inverse iteration (oracle/tridiag.py) and
against closed forms: eigenvalues to a few n eps ||T||, the residual and
orthogonality invariants, and, for eigenvalues separated from their
neighbours, the eigenvectors themselves up to sign.  Then the whole standard
solve with every step on the GPU."""
import numpy as np
import pytest

import workload as W
from oracle import checks, tridiag

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


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


def make(kind, n, seed):
    g = np.random.default_rng(seed)
    if kind == "gauss":
        return g.standard_normal(n), g.standard_normal(max(n - 1, 0))
    if kind == "wilkinson":     # pairs of nearly equal eigenvalues
        return np.abs(np.arange(n) - (n - 1) / 2.0), np.ones(max(n - 1, 0))
    if kind == "split":         # zeros on the off-diagonal: independent blocks
        d, e = g.standard_normal(n), g.standard_normal(max(n - 1, 0))
        e[::7] = 0.0
        return d, e
    if kind == "laplace":       # 2 - 2 cos(k pi / (n + 1)), closed form
        return 2.0 * np.ones(n), -np.ones(max(n - 1, 0))
    if kind == "repeated":      # every eigenvalue of a 1-2-1 block repeated
        d = np.tile([1.0, 2.0, 1.0], (n + 2) // 3)[:n]
        e = np.tile([0.5, 0.5, 0.0], (n + 2) // 3)[:max(n - 1, 0)]
        return d, e
    if kind == "semicircle":    # the tridiagonal of a Gaussian symmetric matrix
        A = W.sym_gaussian(n, seed)
        from oracle import stage1, stage2
        B, _ = stage1.full_to_band(A, 8)
        d, e, _, _ = stage2.band_to_tridiag(B, 8)
        return d, e
    raise ValueError(kind)


def gpu_solve(torch, dev, d, e, nev=None, dtype=None):
    import paper_1811_01277_amd as P
    lam, z = P.tridiag_eigh(torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev), nev, dtype)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), z.cpu().numpy()


def check_solution(d, e, lam, Z, what):
    n = d.shape[0]
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    nrm = max(np.max(np.abs(np.linalg.eigvalsh(T))), 1e-300)
    ref = tridiag.eigvals(d, e)
    assert np.all(np.diff(lam) >= 0), what
    # absolute floor for the zero matrix (bisection stops within ~1e-308 of 0)
    assert np.max(np.abs(lam - ref)) <= 8 * n * EPS * nrm + 1e-300, what
    R = T @ Z - Z * lam[None, :Z.shape[1]]
    assert checks.norm1(R) <= 50 * n * EPS * max(checks.norm1(T), 1e-300), what
    assert checks.orth_ratio(Z) < 50, what
    return T, nrm, ref


CASES = [(k, n) for k in ("gauss", "wilkinson", "split", "laplace", "repeated", "semicircle")
         for n in (1, 2, 3, 7, 100, 257, 600)]


@pytest.mark.parametrize("kind,n", CASES, ids=[f"{k}-{n}" for k, n in CASES])
def test_dc_matches_oracle(torch_dev, kind, n):
    torch, dev = torch_dev
    d, e = make(kind, n, 700 + n)
    print(f"tridiag_eigh kind={kind} n={n}", flush=True)
    lam, Z = gpu_solve(torch, dev, d, e)
    T, nrm, ref = check_solution(d, e, lam, Z, (kind, n))
    if kind == "laplace":
        k = np.arange(1, n + 1)
        exact = 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))
        assert np.max(np.abs(lam - exact)) <= 8 * n * EPS * 4
    # well separated eigenvalues: the eigenvector is unique up to sign
    gap = np.full(n, np.inf)
    if n > 1:
        dl = np.diff(ref)
        gap[:-1] = dl
        gap[1:] = np.minimum(gap[1:], dl)
    sep = np.nonzero(gap > 1e-3 * nrm)[0]
    if sep.size:
        _, Zo = tridiag.eigh_tridiag(d, e)
        dots = np.abs(np.sum(Z[:, sep] * Zo[:, sep], axis=0))
        assert np.max(np.abs(dots - 1.0)) <= 1e-9, (kind, n)


def test_dc_dtypes_and_nev(torch_dev):
    """float32 and complex128 outputs are the float64 eigenvectors converted;
    nev < n returns the leading columns; nev = 0 the eigenvalues alone."""
    torch, dev = torch_dev
    d, e = make("gauss", 300, 801)
    lam, Z = gpu_solve(torch, dev, d, e)
    lam32, Z32 = gpu_solve(torch, dev, d, e, dtype=torch.float32)
    assert np.array_equal(lam32, lam) and np.array_equal(Z32, Z.astype(np.float32))
    lamc, Zc = gpu_solve(torch, dev, d, e, nev=40, dtype=torch.complex128)
    assert np.array_equal(lamc, lam) and np.array_equal(Zc, Z[:, :40].astype(np.complex128))
    lam0, Z0 = gpu_solve(torch, dev, d, e, nev=0)
    assert np.array_equal(lam0, lam) and Z0.shape == (300, 0)


def test_dc_large_sampled(torch_dev):
    """n = 20000, the tridiagonal of the full-size workload's distribution
    (diagonal and off-diagonal of a reduced Gaussian symmetric matrix have
    the semicircle spectrum of radius 2 sqrt(n)); a Gaussian stand-in with the
    same scale: sampled eigenvalues against bisection, residual of sampled
    columns, and Z^T Z = I checked on the GPU."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n = 20000
    g = np.random.default_rng(811)
    d = g.standard_normal(n) * np.sqrt(n) / 4
    e = g.standard_normal(n - 1) * np.sqrt(n) / 4
    print("tridiag_eigh n=20000", flush=True)
    lam_t, z_t = P.tridiag_eigh(torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev))
    G = z_t.t() @ z_t
    G.diagonal().sub_(1.0)
    orth = float(G.abs().sum(0).max()) / (n * EPS)
    lam = lam_t.cpu().numpy()
    idx = np.array([0, 1, 777, 5000, 12345, n - 2, n - 1])
    Zs = z_t[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
    del G, z_t
    torch.cuda.empty_cache()
    assert orth < 50
    assert np.all(np.diff(lam) >= 0)
    nrm = float(np.max(np.abs(lam)))
    for i in idx:
        ref = tridiag.eigvals(d, e, int(i), int(i))[0]
        assert abs(lam[i] - ref) <= 8 * n * EPS * nrm
    TZ = d[:, None] * Zs
    TZ[1:] += e[:, None] * Zs[:-1]
    TZ[:-1] += e[:, None] * Zs[1:]
    R = TZ - Zs * lam[idx]
    assert np.max(np.sum(np.abs(R), axis=0)) / (nrm * 3 * n * EPS) < 50


@pytest.mark.parametrize("cplx", [False, True])
def test_whole_solve_on_gpu(torch_dev, cplx):
    """A -> band -> tridiagonal -> eigenpairs -> band vectors -> full vectors,
    every step on the GPU: A Z = Z Lambda, Z^H Z = I, eigenvalues as numpy's."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw = 500, 32
    A = W.herm_gaussian(n, 821) if cplx else W.sym_gaussian(n, 821)
    a = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev).t()
    v, t1 = P.full_to_band(a, nbw)
    d, e, hh, tau = P.band_to_tridiag(a, nbw)
    lam, q = P.tridiag_eigh(d, e, dtype=torch.complex128 if cplx else torch.float64)
    P.hh_trafo(q, hh, tau, nbw)
    P.bt2_trafo(q, v, t1, nbw)
    torch.cuda.synchronize()
    Z, lam = q.cpu().numpy(), lam.cpu().numpy()
    assert checks.residual_ratio(A, Z, lam) < 50
    assert checks.orth_ratio(Z) < 50
    assert np.max(np.abs(lam - np.linalg.eigvalsh(A))) <= 8 * n * EPS * np.linalg.norm(A, 2)


def test_padded_ldz_through_the_c_abi(torch_dev):
    """elpa_tridiag_eigh with ldz > n: the eigenvectors land in rows [0, n) of
    each column and the padding rows are left as they were."""
    torch, dev = torch_dev
    import ctypes as C
    import paper_1811_01277_amd as P
    n, nev, ldz = 130, 37, 141
    d, e = make("gauss", n, 901)
    lam0, Z0 = gpu_solve(torch, dev, d, e)
    dt = torch.from_numpy(d).to(dev)
    et = torch.from_numpy(e).to(dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    buf = torch.full((nev, ldz), float("nan"), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    rc = P.library().elpa_tridiag_eigh(n, nev, C.c_void_p(dt.data_ptr()), C.c_void_p(et.data_ptr()),
                                       C.c_void_p(lam.data_ptr()), C.c_void_p(buf.data_ptr()), ldz,
                                       P.R64, C.c_void_p(st))
    assert rc == 0
    torch.cuda.synchronize()
    got = buf.cpu().numpy().T
    assert np.array_equal(got[:n], Z0[:, :nev]) and np.array_equal(lam.cpu().numpy(), lam0)
    assert np.all(np.isnan(got[n:]))


def test_whole_solve_full_size(torch_dev):
    """n = 20000, nbw = 64, nev = 2000, every stage on the device: for sampled
    eigenpairs of the original matrix the residual ratio
    ||A z - lambda z||_1 / (||A||_1 n eps) stays below 50, the sampled
    columns are orthonormal to n eps, and the eigenvalues ascend and lie in
    the spectrum's bounds (|lambda| <= ||A||_1)."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 20000, 64, 2000
    g = torch.Generator(device=dev)
    g.manual_seed(931)
    A = torch.randn(n, n, device=dev, dtype=torch.float64, generator=g)
    A = (A + A.t()) * 0.5
    a = A.clone().t()
    print("whole solve n=20000", flush=True)
    v, t1 = P.full_to_band(a, nbw)
    d, e, hh, tau = P.band_to_tridiag(a, nbw)
    del a
    lam, q = P.tridiag_eigh(d, e, nev)
    P.hh_trafo(q, hh, tau, nbw)
    P.bt2_trafo(q, v, t1, nbw)
    del v, t1, hh, tau
    idx = torch.tensor([0, 1, 500, 1234, nev - 2, nev - 1], device=dev)
    Z = q[:, idx]
    R = A @ Z - Z * lam[idx]
    norm1 = float(A.abs().sum(0).max())
    res = float(R.abs().sum(0).max()) / (norm1 * n * EPS)
    G = Z.t() @ Z - torch.eye(len(idx), dtype=torch.float64, device=dev)
    orth = float(G.abs().sum(0).max()) / (n * EPS)
    lam_h = lam.cpu().numpy()
    del A, q, Z, R
    torch.cuda.empty_cache()
    assert res < 50 and orth < 50, (res, orth)
    assert np.all(np.diff(lam_h) >= 0) and np.max(np.abs(lam_h)) <= norm1


@pytest.mark.parametrize("n,nbw,nev,cplx", [(300, 32, 100, False), (300, 32, 300, True),
                                            (5, 64, 5, False), (1, 64, 1, False)])
def test_eigenvectors_api(torch_dev, n, nbw, nev, cplx):
    """paper_1811_01277_amd.eigenvectors: the whole solve in one call (band
    width clamped to n - 1 for small n): A Z = Z Lambda, Z^H Z = I,
    eigenvalues as numpy's."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    A = W.herm_gaussian(n, 941) if cplx else W.sym_gaussian(n, 941)
    a = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev).t()
    lam, z = P.eigenvectors(a, nev, nbw)
    torch.cuda.synchronize()
    lam, Z = lam.cpu().numpy(), z.cpu().numpy()
    assert Z.shape == (n, nev)
    ref = np.linalg.eigvalsh(A)
    assert np.max(np.abs(lam - ref)) <= 8 * n * EPS * max(np.linalg.norm(A, 2), 1e-300)
    assert checks.norm1(A @ Z - Z * lam[None, :nev]) <= 50 * n * EPS * checks.norm1(A)
    assert checks.orth_ratio(Z) < 50
