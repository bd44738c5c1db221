"""GPU parity of the band -> full back-transformation (include/elpa_bt2.h)
against the oracle's bt_band_to_full on the first stage's own panels.

The panels are converted to the library's layout (column c of V holds v_c
from row c+nbw down); every entry the library must not read (the unit lead
and everything above it) is NaN, so reading one shows up as NaN in Q."""
import numpy as np
import pytest

import workload as W
from oracle import bt, checks, solve, stage1

from bt2_layout import abi_to_panels, panels_to_abi

pytestmark = pytest.mark.gpu

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


def npdtype(dt):
    return {"r64": np.float64, "r32": np.float32, "c64": np.complex128}[dt]


def rounded(x, dt):
    return x.astype(np.float32).astype(np.float64) if dt == "r32" else x


def to_dev(torch, dev, a, dt, ld=None):
    """Column-major device copy (leading dimension ld >= rows)."""
    a = np.asarray(a)
    rows, cols = a.shape
    ld = ld or rows
    buf = np.zeros((cols, ld), dtype=npdtype(dt))
    buf[:, :rows] = a.T.astype(npdtype(dt))
    t = torch.from_numpy(buf).to(dev)
    return t, t.t()[:rows]


def run_gpu(torch, dev, V, tau, Z, nbw, dt, block=0, ldq=None):
    import paper_1811_01277_amd as P
    n = Z.shape[0]
    vbuf, v = to_dev(torch, dev, V, dt)
    qbuf, q = to_dev(torch, dev, Z, dt, ldq)
    t = torch.from_numpy(np.ascontiguousarray(tau).astype(npdtype(dt))).to(dev)
    P.bt2_trafo(q, v, t, nbw, block=block)
    torch.cuda.synchronize()
    return qbuf.cpu().numpy().T   # (ld, nev)


CASES = [
    # (n, nbw, nev, seed)
    (97, 32, 40, 301),    # ragged last panel
    (130, 64, 129, 302),
    (300, 32, 65, 303),
    (65, 64, 3, 304),     # a single reflector
]


@pytest.mark.parametrize("dt", ["r64", "r32", "c64"])
@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}_b{c[1]}_e{c[2]}" for c in CASES])
def test_bt2_parity_blocks(torch_dev, case, dt):
    torch, dev = torch_dev
    n, nbw, nev, seed = case
    cplx = dt == "c64"
    A = W.herm_gaussian(n, seed) if cplx else W.sym_gaussian(n, seed)
    _, panels = stage1.full_to_band(A, nbw)
    V, tau = panels_to_abi(panels, n, nbw, np.complex128 if cplx else np.float64)
    Z = np.asfortranarray(W.gaussian_block(n, nev, complex_=cplx, seed=seed + 1))
    Vr = np.where(np.isnan(V), 0, V)
    ref = bt.bt_band_to_full(abi_to_panels(rounded(Vr, dt), rounded(tau, dt), n, nbw),
                             rounded(Z, dt), nbw)
    for block in (0, 1, 7, 64, 128, 512):
        print(f"bt2 n={n} nbw={nbw} nev={nev} dt={dt} block={block}", flush=True)
        got = run_gpu(torch, dev, V, tau, Z, nbw, dt, block)
        assert np.all(np.isfinite(got)), "a NaN entry of V was read"
        err = checks.max_rel_err(got.astype(ref.dtype), ref)
        assert err <= TOL[dt], (block, err)


def test_bt2_padding_and_noop(torch_dev):
    torch, dev = torch_dev
    n, nbw, nev, ldq = 150, 32, 30, 171
    A = W.sym_gaussian(n, 311)
    _, panels = stage1.full_to_band(A, nbw)
    V, tau = panels_to_abi(panels, n, nbw, np.float64)
    Z = np.asfortranarray(W.gaussian_block(n, nev, seed=312))
    ref = bt.bt_band_to_full(panels, Z, nbw)
    got = run_gpu(torch, dev, V, tau, Z, nbw, "r64", ldq=ldq)
    assert np.all(got[n:] == 0), "padding rows written"
    assert checks.max_rel_err(got[:n], ref) <= TOL["r64"]
    # n <= nbw: identity
    Z2 = np.asfortranarray(W.gaussian_block(40, 5, seed=313))
    got2 = run_gpu(torch, dev, np.zeros((40, 1)), np.zeros(1), Z2, 64, "r64")
    assert np.array_equal(got2, Z2)


@pytest.mark.parametrize("cplx", [False, True])
def test_eigenvector_chain_on_gpu(torch_dev, cplx):
    """Tridiagonal eigenvectors -> band (elpa_hh_trafo) -> full (elpa_bt2_trafo)
    on the GPU: equal to the oracle's eigenvectors, and they satisfy the
    eigen-residual and orthogonality invariants of A."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw = 256, 32
    dt = "c64" if cplx else "r64"
    A = W.herm_gaussian(n, 321) if cplx else W.sym_gaussian(n, 321)
    r = solve.solve_two_stage(A, nbw)
    V, tau = panels_to_abi(r["panels"], n, nbw, np.complex128 if cplx else np.float64)
    Zt = r["Zt"].astype(np.complex128 if cplx else np.float64)
    qbuf, q = to_dev(torch, dev, Zt, dt)
    h = torch.from_numpy(r["hh"].astype(npdtype(dt))).to(dev)
    t = torch.from_numpy(r["tau"].astype(npdtype(dt))).to(dev)
    P.hh_trafo(q, h, t, nbw)
    vbuf, v = to_dev(torch, dev, V, dt)
    t2 = torch.from_numpy(tau.astype(npdtype(dt))).to(dev)
    P.bt2_trafo(q, v, t2, nbw)
    torch.cuda.synchronize()
    Z = qbuf.cpu().numpy().T
    assert checks.max_rel_err(Z, r["Z"]) <= 1e-12
    assert checks.residual_ratio(A, Z, r["lam"]) < 50
    assert checks.orth_ratio(Z) < 50


def test_bt2_full_size_sampled(torch_dev):
    """n = 20000, nbw = 64, nev = 2000 with the library's default block (384
    reflectors), synthetic unit-lead reflectors with tau = 2 / |v|^2; four
    sampled columns against the oracle."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 20000, 64, 2000
    V, tau = W.synthetic_stage1(n, nbw, seed=331)
    Z = W.gaussian_block(n, nev, seed=332)
    cols = [0, 777, 1500, nev - 1]
    print("oracle on sampled columns", flush=True)
    ref = bt.bt_band_to_full(abi_to_panels(V, tau, n, nbw), np.asfortranarray(Z[:, cols]), nbw)
    print("gpu", flush=True)
    vbuf, v = to_dev(torch, dev, V, "r64")
    qbuf, q = to_dev(torch, dev, Z, "r64")
    t = torch.from_numpy(tau).to(dev)
    P.bt2_trafo(q, v, t, nbw)
    torch.cuda.synchronize()
    got = q[:, cols].cpu().numpy()
    assert checks.max_rel_err(got, ref) <= TOL["r64"]
