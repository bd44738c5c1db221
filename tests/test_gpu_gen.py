"""GPU generalized eigenproblem steps (include/elpa_gen.h) against the
oracle's (oracle/generalized.py): the inverted Cholesky factor, the forward
transformation Linv A Linv^H, the back-transformation Linv^H V, and the whole
generalized solve with every step but the tridiagonal solve on the GPU, first
with the factorisation and then reusing the inverted factor for a second A."""
import numpy as np
import pytest

import workload as W
from oracle import checks, generalized as G, tridiag

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


def spd(n, seed, cplx=False):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, n)) + (1j * g.standard_normal((n, n)) if cplx else 0)
    return X @ np.conj(X.T) / n + np.eye(n)


def dev_cm(torch, dev, M, ld=None):
    """Column-major device copy of M with leading dimension ld (padding rows
    filled with NaN); returns (buffer, view)."""
    rows, cols = M.shape
    ld = ld or rows
    buf = np.full((cols, ld), np.nan, dtype=M.dtype)
    buf[:, :rows] = M.T
    t = torch.from_numpy(buf).to(dev)
    return t, t.t()[:rows]


def host(x):
    return x.cpu().numpy()


NS = [1, 2, 7, 130, 256, 257, 600]


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", NS)
def test_cholesky_inverse_matches_oracle(torch_dev, n, cplx):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    B = spd(n, 100 + n, cplx)
    L, info = G.cholesky(B)
    ref = G.inverse_lower(L)
    # the strict upper triangle is not read: NaN there
    Bn = np.tril(B) + np.triu(np.full((n, n), np.nan), 1)
    print(f"cholesky_inverse n={n} cplx={cplx}", flush=True)
    buf, b = dev_cm(torch, dev, Bn.astype(B.dtype), ld=n + 3)
    P.cholesky_inverse(b)
    got = host(b)
    assert np.array_equal(np.triu(got, 1), np.zeros_like(got))
    assert checks.max_rel_err(got, ref) <= 1e-11
    assert np.max(np.abs(got @ B @ np.conj(got.T) - np.eye(n))) <= 1e-11
    assert np.all(np.isnan(host(buf.t()[n:])))   # padding rows untouched


@pytest.mark.parametrize("B,info", [
    (np.diag([1.0, 2.0, -1.0, 5.0]), 3),
    (np.array([[1.0, 2.0], [2.0, 1.0]]), 2),
    (np.array([[0.0, 0.0], [0.0, 1.0]]), 1),
])
def test_cholesky_failure_index(torch_dev, B, info):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    assert G.cholesky(B)[1] == info
    _, b = dev_cm(torch, dev, B)
    assert int(P.cholesky_inverse(b, check=False).item()) == info
    _, b = dev_cm(torch, dev, B)
    with pytest.raises(np.linalg.LinAlgError):
        P.cholesky_inverse(b)


def test_cholesky_failure_in_a_later_panel(torch_dev):
    """A minor that fails past the first 256-column panel: the same index as
    the oracle's."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n = 600
    B = spd(n, 7)
    B[400, 400] = -5.0
    info0 = G.cholesky(B)[1]
    assert info0 == 401
    _, b = dev_cm(torch, dev, B)
    assert int(P.cholesky_inverse(b, check=False).item()) == info0


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [1, 33, 300])
def test_transforms_match_oracle(torch_dev, n, cplx):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    A = W.herm_gaussian(n, 200 + n) if cplx else W.sym_gaussian(n, 200 + n)
    B = spd(n, 300 + n, cplx)
    Linv = G.inverse_lower(G.cholesky(B)[0])
    ref = G.to_standard(A, Linv)
    _, a = dev_cm(torch, dev, A, ld=n + 1)
    _, li = dev_cm(torch, dev, Linv)
    print(f"to_standard n={n} cplx={cplx}", flush=True)
    P.generalized_to_standard(a, li)
    got = host(a)
    assert np.array_equal(got, np.conj(got.T)), "not exactly Hermitian"
    assert checks.max_rel_err(got, ref) <= 1e-12
    nev = max(1, n // 3)
    Vt = W.gaussian_block(n, nev, complex_=cplx, seed=400 + n)
    qbuf, q = dev_cm(torch, dev, np.asarray(Vt), ld=n + 2)
    P.generalized_back(q, li)
    assert checks.max_rel_err(host(q), G.back(Linv, Vt)) <= 1e-12
    assert np.all(np.isnan(host(qbuf.t()[n:])))


@pytest.mark.parametrize("cplx", [False, True])
def test_generalized_solve_on_gpu(torch_dev, cplx):
    """Cholesky inverse, forward transformation, full -> band, band ->
    tridiagonal, both back-transformations and the generalized
    back-transformation on the GPU (the tridiagonal solve on the oracle):
    A V = B V Lambda, V^H B V = I, eigenvalues as the oracle's.  Then a second
    A with the inverted factor kept from the first call."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw = 400, 32
    dt = np.complex128 if cplx else np.float64
    B = spd(n, 500, cplx)
    _, b = dev_cm(torch, dev, B)
    P.cholesky_inverse(b)
    for rep, seed in enumerate((501, 502)):
        A = W.herm_gaussian(n, seed) if cplx else W.sym_gaussian(n, seed)
        print(f"generalized solve rep={rep} cplx={cplx}", flush=True)
        _, a = dev_cm(torch, dev, A)
        P.generalized_to_standard(a, b)
        v, t1 = P.full_to_band(a, nbw)
        d, e, hh, tau = P.band_to_tridiag(a, nbw)
        lam, Zt = tridiag.eigh_tridiag(host(d), host(e))
        _, q = dev_cm(torch, dev, Zt.astype(dt))
        P.hh_trafo(q, hh, tau, nbw)
        P.bt2_trafo(q, v, t1, nbw)
        P.generalized_back(q, b)
        V = host(q)
        scale = np.linalg.norm(A, 2) + np.linalg.norm(B, 2) * np.max(np.abs(lam))
        assert np.max(np.abs(A @ V - B @ V * lam)) <= 1e-11 * scale
        assert np.max(np.abs(np.conj(V.T) @ B @ V - np.eye(n))) <= 1e-10
        ref = G.generalized_eigh(A, B, nbw)
        assert np.max(np.abs(lam - ref["lam"])) <= 1e-11 * scale


@pytest.mark.parametrize("cplx", [False, True])
def test_generalized_eigenvectors_api(torch_dev, cplx):
    """paper_1811_01277_amd.generalized_eigenvectors, every step on the GPU
    (the tridiagonal solve included): the first call factors B and leaves
    the inverted factor in b; the second, with is_already_decomposed=True and
    another A, reuses it.  A V = B V Lambda, V^H B V = I, eigenvalues as
    scipy's generalized solver."""
    torch, dev = torch_dev
    import scipy.linalg
    import paper_1811_01277_amd as P
    n, nbw, nev = 300, 32, 120
    B = spd(n, 951, cplx)
    _, b = dev_cm(torch, dev, B)
    for rep, seed in enumerate((952, 953)):
        A = W.herm_gaussian(n, seed) if cplx else W.sym_gaussian(n, seed)
        _, a = dev_cm(torch, dev, A)
        print(f"generalized_eigenvectors rep={rep} cplx={cplx}", flush=True)
        lam, v = P.generalized_eigenvectors(a, b, nev, nbw, is_already_decomposed=rep > 0)
        torch.cuda.synchronize()
        lam, V = host(lam), host(v)
        ref = scipy.linalg.eigh(A, B, eigvals_only=True)
        scale = np.linalg.norm(A, 2) + np.linalg.norm(B, 2) * np.max(np.abs(ref))
        assert np.max(np.abs(lam - ref)) <= 1e-11 * scale
        assert np.max(np.abs(A @ V - B @ V * lam[:nev])) <= 1e-11 * scale
        assert np.max(np.abs(np.conj(V.T) @ B @ V - np.eye(nev))) <= 1e-10
