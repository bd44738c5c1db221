"""GPU parity of elpa_hh_trafo (through the C ABI) against the CPU oracle.

Bar (max-abs error divided by max |Q_ref|): 1e-12 for real and complex fp64,
5e-5 for fp32.  fp32 inputs are the fp64 inputs rounded to fp32; the oracle
applies those rounded values in fp64, so the measured error is the kernel's
fp32 arithmetic alone.  The fp32 error against the unrounded fp64 oracle is
printed beside it.

Small sizes compare every element and span several 64-column stripes and a
ragged column / row tail; the full sizes (n = 8192 and 20000) compare sampled
columns, which the oracle computes one by one.
"""
import numpy as np
import pytest

import workload as W
from oracle import bt, checks, solve

pytestmark = pytest.mark.gpu

TOL = {"r64": 1e-12, "c64": 1e-12, "r32": 5e-5}
KS = [1, 2, 4, 6, 8, 16, 24, 32, 40, 48, 64]
SPLIT_KS = [16, 24, 32, 48, 64, 80, 96, 128]
WY_KS = [16, 32, 48, 64, 96, 112, 128, 144, 160, 192]


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


def tdtype(torch, dt):
    return {"r64": torch.float64, "r32": torch.float32, "c64": torch.complex128}[dt]


def npdtype(dt):
    return {"r64": np.float64, "r32": np.float32, "c64": np.complex128}[dt]


def upload_q(torch, dev, Z, dt, ldq=None):
    """Column-major (n, nev) device tensor, optionally with padding rows."""
    n, nev = Z.shape
    ldq = n if ldq is None else ldq
    buf = torch.zeros((nev, ldq), dtype=tdtype(torch, dt))
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(Z.T).astype(npdtype(dt)))
    buf = buf.to(dev)
    return buf, buf[:, :n].t()


def run_gpu(torch, dev, hh, tau, Z, nbw, dt, path=None, k=0, ldq=None, steps=0, order=0,
            streams=0):
    import paper_1811_01277_amd as P
    buf, q = upload_q(torch, dev, Z, dt, ldq)
    h = torch.from_numpy(hh.astype(npdtype(dt))).to(dev)
    t = torch.from_numpy(tau.astype(npdtype(dt))).to(dev)
    P.hh_trafo(q, h, t, nbw, path=path, k=k, steps=steps, order=order, streams=streams)
    torch.cuda.synchronize()
    return buf.cpu().numpy().T  # (ldq, nev)


def oracle_inputs(n, nbw, nev, dt, seed, real_pipeline=False):
    cplx = dt == "c64"
    if real_pipeline:
        A = W.herm_gaussian(n, seed) if cplx else W.sym_gaussian(n, seed)
        r = solve.solve_two_stage(A, nbw, nev)
        hh, tau = r["hh"], r["tau"]
        Z = r["Zt"].astype(np.complex128 if cplx else np.float64)
    else:
        hh, tau = W.synthetic_reflectors(n, nbw, complex_=cplx, seed=seed)
        Z = np.asfortranarray(W.gaussian_block(n, nev, complex_=cplx, seed=seed + 1))
    return hh, tau, Z


def rounded(x, dt):
    """The values the kernel receives, back in fp64 for the oracle."""
    if dt == "r32":
        return x.astype(np.float32).astype(np.float64)
    return x


def plans(nbw, dt):
    import paper_1811_01277_amd as P
    code = {"r64": P.R64, "r32": P.R32, "c64": P.C64}[dt]
    out = [(None, 0), (P.PATH_REF, 0)]
    out += [(P.PATH_STRIPE, k) for k in KS if P.plan_supported(nbw, code, P.PATH_STRIPE, k)]
    out += [(P.PATH_SPLIT, k) for k in SPLIT_KS if P.plan_supported(nbw, code, P.PATH_SPLIT, k)]
    out += [(P.PATH_WY, k) for k in WY_KS if P.plan_supported(nbw, code, P.PATH_WY, k)]
    return out


SMALL = [
    # (n, nbw, nev, seed, real pipeline)
    (512, 32, 512, 101, True),    # the first workload: full oracle pipeline
    (97, 32, 70, 11, False),      # ragged rows and one partial stripe
    (130, 64, 129, 12, False),    # 3 stripes, last with one column
    (300, 64, 65, 13, True),
    (65, 64, 64, 14, False),      # one chase step per sweep except the first
    (64, 64, 3, 15, False),       # nbw >= n-1
    (2, 32, 1, 16, False),        # a single reflector
    (3, 1, 5, 17, False),         # nbw = 1 (generic path)
    (200, 7, 33, 18, True),       # nbw without a stripe kernel
]


@pytest.mark.parametrize("dt", ["r64", "r32", "c64"])
@pytest.mark.parametrize("case", SMALL, ids=[f"n{c[0]}_b{c[1]}_e{c[2]}" for c in SMALL])
def test_parity_small_all_plans(torch_dev, case, dt):
    torch, dev = torch_dev
    n, nbw, nev, seed, real = case
    hh, tau, Z = oracle_inputs(n, nbw, nev, dt, seed, real)
    ref = bt.bt_tridiag_to_band(rounded(hh, dt), rounded(tau, dt), rounded(Z, dt), n, nbw)
    ref_unrounded = bt.bt_tridiag_to_band(hh, tau, Z, n, nbw) if dt == "r32" else ref
    for path, k in plans(nbw, dt):
        print(f"case n={n} nbw={nbw} nev={nev} dt={dt} path={path} k={k}", flush=True)
        got = run_gpu(torch, dev, hh, tau, Z, nbw, dt, path, k)[:n]
        err = checks.max_rel_err(got, ref)
        assert err <= TOL[dt], (path, k, err)
        if dt == "r32":
            print(f"  fp32 err vs fp64 oracle of unrounded inputs: "
                  f"{checks.max_rel_err(got, ref_unrounded):.3e} (vs rounded: {err:.3e})")


@pytest.mark.parametrize("dt", ["r64", "c64"])
def test_padding_rows_untouched_and_replay_bitwise(torch_dev, dt):
    torch, dev = torch_dev
    n, nbw, nev, ldq = 150, 32, 100, 173
    hh, tau, Z = oracle_inputs(n, nbw, nev, dt, 21)
    ref = bt.bt_tridiag_to_band(hh, tau, Z, n, nbw)
    a = run_gpu(torch, dev, hh, tau, Z, nbw, dt, ldq=ldq)
    b = run_gpu(torch, dev, hh, tau, Z, nbw, dt, ldq=ldq)
    assert np.array_equal(a, b)
    assert np.all(a[n:] == 0)
    assert checks.max_rel_err(a[:n], ref) <= TOL[dt]


@pytest.mark.parametrize("nbw,k", [(64, 48), (64, 64), (64, 80), (32, 32), (32, 64), (32, 96)])
def test_split_steps_per_tile(torch_dev, nbw, k):
    """Two-lane kernel with tiles of 1, 3 and 16 chase steps: group
    boundaries inside a block (carried rows written back and reloaded), the
    last group of a block shorter than the others, n - 1 not a multiple of k."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nev = 1000, 97
    hh, tau, Z = oracle_inputs(n, nbw, nev, "r64", 51 + k)
    ref = bt.bt_tridiag_to_band(hh, tau, Z, n, nbw)
    outs = []
    for steps in (1, 3, 16):
        print(f"split n={n} nbw={nbw} k={k} steps={steps}", flush=True)
        got = run_gpu(torch, dev, hh, tau, Z, nbw, "r64", P.PATH_SPLIT, k, steps=steps)
        assert checks.max_rel_err(got, ref) <= TOL["r64"], steps
        outs.append(got)
    # the tiling changes only which wave runs a step, not the arithmetic
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("dt,path,k", [("r64", 3, 64), ("r64", 2, 32), ("r32", 2, 32),
                                       ("c64", 2, 4)])
def test_tile_order_does_not_change_results(torch_dev, dt, path, k):
    """Linear and die-grouped tile orders run the same tiles: bitwise equal."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 900, 64, 333
    hh, tau, Z = oracle_inputs(n, nbw, nev, dt, 71)
    ref = bt.bt_tridiag_to_band(rounded(hh, dt), rounded(tau, dt), rounded(Z, dt), n, nbw)
    got = [run_gpu(torch, dev, hh, tau, Z, nbw, dt, path, k, steps=2, order=o)
           for o in (P.ORDER_LINEAR, P.ORDER_XCD)]
    assert np.array_equal(got[0], got[1])
    assert checks.max_rel_err(got[0], ref) <= TOL[dt]


def test_stripe_groups_on_streams(torch_dev):
    """Stripe groups on 2, 3 and 8 library streams (more groups than
    stripes is clamped): bitwise equal to one stream, and the caller's stream
    is ordered behind all groups (the result is read right after the call)."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 800, 64, 161   # 6 stripes of 32 columns, the last one ragged
    hh, tau, Z = oracle_inputs(n, nbw, nev, "r64", 81)
    ref = bt.bt_tridiag_to_band(hh, tau, Z, n, nbw)
    one = run_gpu(torch, dev, hh, tau, Z, nbw, "r64", P.PATH_SPLIT, 64, steps=3, streams=1)
    assert checks.max_rel_err(one, ref) <= TOL["r64"]
    P.profile_enable(True)
    try:
        for ns in (2, 3, 8):
            print(f"streams={ns}", flush=True)
            got = run_gpu(torch, dev, hh, tau, Z, nbw, "r64", P.PATH_SPLIT, 64, steps=3,
                          streams=ns)
            assert np.array_equal(got, one), ns
            pr = P.profile_last()
            M, J0 = -(-(n - 1) // 64), -(-(n - 1) // nbw)
            assert pr["launches"] == min(ns, 6) * (M + -(-J0 // 3) - 1)
    finally:
        P.profile_enable(False)


@pytest.mark.parametrize("dt,nbw,k", [("r64", 64, 64), ("r64", 64, 32), ("r64", 32, 96),
                                       ("r32", 64, 64), ("r32", 32, 64)])
def test_wy_path_tilings(torch_dev, dt, nbw, k):
    """Compact-WY MFMA path: tiles of 1, 3 and 16 chase steps and two stripe
    groups give bitwise equal results that match the oracle."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nev = 1000, 83
    hh, tau, Z = oracle_inputs(n, nbw, nev, dt, 91 + k)
    ref = bt.bt_tridiag_to_band(rounded(hh, dt), rounded(tau, dt), rounded(Z, dt), n, nbw)
    outs = []
    for steps, ns in ((1, 1), (3, 1), (16, 2)):
        print(f"wy n={n} nbw={nbw} k={k} dt={dt} steps={steps} streams={ns}", flush=True)
        got = run_gpu(torch, dev, hh, tau, Z, nbw, dt, P.PATH_WY, k, steps=steps, streams=ns)
        assert checks.max_rel_err(got, ref) <= TOL[dt], steps
        outs.append(got)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("nbw,k", [(64, 64), (64, 80), (64, 96), (32, 64), (32, 96), (32, 128)])
def test_split_fp32_tilings(torch_dev, nbw, k):
    """Two-lane kernel on fp32 values (reflector pairs): tiles of 1, 3 and 16
    chase steps and two stripe groups give bitwise equal results that match
    the oracle on the fp32-rounded inputs."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nev = 900, 77
    hh, tau, Z = oracle_inputs(n, nbw, nev, "r32", 151 + k)
    ref = bt.bt_tridiag_to_band(rounded(hh, "r32"), rounded(tau, "r32"), rounded(Z, "r32"), n, nbw)
    outs = []
    for steps, ns in ((1, 1), (3, 1), (16, 2)):
        print(f"split r32 n={n} nbw={nbw} k={k} steps={steps} streams={ns}", flush=True)
        got = run_gpu(torch, dev, hh, tau, Z, nbw, "r32", P.PATH_SPLIT, k, steps=steps,
                      streams=ns)
        assert checks.max_rel_err(got, ref) <= TOL["r32"], steps
        outs.append(got)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("nbw,k", [(64, 16), (64, 24), (32, 32), (32, 48)])
def test_split_complex_tilings(torch_dev, nbw, k):
    """Two-lane kernel on complex values: tiles of 1, 3 and 16 chase steps and
    two stripe groups give bitwise equal results that match the oracle."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nev = 900, 77
    hh, tau, Z = oracle_inputs(n, nbw, nev, "c64", 131 + k)
    ref = bt.bt_tridiag_to_band(hh, tau, Z, n, nbw)
    outs = []
    for steps, ns in ((1, 1), (3, 1), (16, 2)):
        print(f"split c64 n={n} nbw={nbw} k={k} steps={steps} streams={ns}", flush=True)
        got = run_gpu(torch, dev, hh, tau, Z, nbw, "c64", P.PATH_SPLIT, k, steps=steps,
                      streams=ns)
        assert checks.max_rel_err(got, ref) <= TOL["c64"], steps
        outs.append(got)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_profile_reports_main_kernel_sequence(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 700, 64, 300
    hh, tau, Z = oracle_inputs(n, nbw, nev, "r64", 61)
    P.profile_enable(True)
    try:
        run_gpu(torch, dev, hh, tau, Z, nbw, "r64", P.PATH_SPLIT, 64, steps=2, streams=1)
        a = P.profile_last()
        run_gpu(torch, dev, hh, tau, Z, nbw, "r64", P.PATH_SPLIT, 64, steps=2)
        a2 = P.profile_last()   # library default: two stripe groups
        run_gpu(torch, dev, hh, tau, Z, nbw, "r64", P.PATH_REF)
        b = P.profile_last()
    finally:
        P.profile_enable(False)
    # diagonal schedule: M + ceil(J0 / steps) - 1 launches (M = ceil((n-1)/k) blocks)
    M, J0 = -(-(n - 1) // 64), -(-(n - 1) // nbw)
    assert a["path"] == P.PATH_SPLIT and a["k"] == 64 and a["steps"] == 2
    assert a["launches"] == M + -(-J0 // 2) - 1 and a["kernel_ms"] > 0 and a["streams"] == 1
    assert 0 < a["sum_launch_ms"] <= a["kernel_ms"] * 1.01
    assert a2["streams"] == 2 and a2["launches"] == 2 * a["launches"]
    assert b["path"] == P.PATH_REF and b["launches"] == 1 and b["kernel_ms"] > 0
    with pytest.raises(P.ElpaError):
        P.profile_last()


def test_column_independence_nan_isolation_identity(torch_dev):
    torch, dev = torch_dev
    n, nbw, nev = 260, 64, 140
    hh, tau, Z = oracle_inputs(n, nbw, nev, "r64", 31)
    full = run_gpu(torch, dev, hh, tau, Z, nbw, "r64")
    sub = run_gpu(torch, dev, hh, tau, np.asfortranarray(Z[:, 70:75]), nbw, "r64")
    assert np.array_equal(sub, full[:, 70:75])
    Zn = Z.copy()
    Zn[100, 7] = np.nan
    got = run_gpu(torch, dev, hh, tau, Zn, nbw, "r64")
    keep = [c for c in range(nev) if c != 7]
    assert np.array_equal(got[:, keep], full[:, keep])
    assert np.isnan(got[:, 7]).any()
    ident = run_gpu(torch, dev, hh, np.zeros_like(tau), Z, nbw, "r64")
    assert np.array_equal(ident, Z)


def test_error_leaves_q_untouched(torch_dev):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev = 40, 8, 10
    hh, tau, Z = oracle_inputs(n, nbw, nev, "r64", 41)
    buf, q = upload_q(torch, dev, Z, "r64")
    h = torch.from_numpy(hh).to(dev)
    t = torch.from_numpy(tau).to(dev)
    before = buf.clone()
    rc = P.hh_trafo_ptr(n, nev, nbw, h.data_ptr(), t.data_ptr(), q.data_ptr(), n - 1, P.R64)
    assert rc == -1
    rc = P.hh_trafo_ptr(n, nev, nbw, h.data_ptr(), t.data_ptr(), q.data_ptr() + 4, n, P.R64)
    assert rc == -3
    torch.cuda.synchronize()
    assert torch.equal(buf, before)


def sampled_columns(nev):
    cols = {0, 1, 31, 32, 63, 64, nev // 2, nev - 1}
    return sorted(c for c in cols if 0 <= c < nev)


FULL = [
    # (n, nbw, nev, dtype, plan (path, k) or None for the library choice)
    (8192, 64, 819, "r64", None), (8192, 64, 4096, "r64", None),
    (20000, 64, 2000, "r64", None), (20000, 64, 10000, "r64", None),
    (20000, 64, 20000, "r64", None),
    (20000, 64, 2000, "r64", (2, 32)),   # one-lane stripe kernel at full size
    (20000, 64, 2000, "r64", (4, 64)),   # compact-WY MFMA path
    (20000, 64, 2000, "r32", (4, 64)),
    (20000, 64, 2000, "c64", (4, 32)),   # compact-WY MFMA path, complex (planar)
    (20000, 64, 2000, "c64", (2, 4)),    # one-lane stripe kernel, complex
    (20000, 64, 2000, "r32", None), (20000, 64, 2000, "c64", None),
]


@pytest.mark.parametrize("case", FULL, ids=[f"n{c[0]}_e{c[2]}_{c[3]}" + (
    f"_p{c[4][0]}k{c[4][1]}" if c[4] else "") for c in FULL])
def test_parity_full_size_sampled(torch_dev, case):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev, dt, plan = case
    path, k = plan if plan else (None, 0)
    cplx = dt == "c64"
    hh, tau = W.synthetic_reflectors(n, nbw, complex_=cplx, seed=n + nev)
    Z = W.gaussian_block(n, nev, complex_=cplx, seed=n + nev + 1)
    print(f"full case n={n} nev={nev} dt={dt} plan={plan}", flush=True)
    q = torch.from_numpy(np.ascontiguousarray(Z.T).astype(npdtype(dt))).to(dev).t()
    h = torch.from_numpy(hh.astype(npdtype(dt))).to(dev)
    t = torch.from_numpy(tau.astype(npdtype(dt))).to(dev)
    P.hh_trafo(q, h, t, nbw, path=path, k=k)
    torch.cuda.synchronize()
    cols = sampled_columns(nev)
    got = q[:, cols].cpu().numpy()
    ref = bt.bt_tridiag_to_band(rounded(hh, dt), rounded(tau, dt),
                                rounded(np.asfortranarray(Z[:, cols]), dt), n, nbw)
    err = checks.max_rel_err(got, ref)
    print(f"  sampled max-abs rel err = {err:.3e}")
    assert err <= TOL[dt]
    # orthogonal reflectors preserve every column norm (all columns checked)
    nq = torch.linalg.vector_norm(q.to(torch.complex128 if cplx else torch.float64), dim=0)
    nz = torch.linalg.vector_norm(torch.from_numpy(Z.T.copy()).to(dev), dim=1)
    rel = ((nq - nz).abs() / nz).max().item()
    assert rel <= (1e-4 if dt == "r32" else 1e-11), rel


def oracle_columns(hh, tau, Zc, n, nbw):
    """The oracle on each sampled column in its own thread (the oracle runs one
    thread per 8-column block; its calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, Zc.shape[1])) as ex:
        cols = list(ex.map(lambda c: bt.bt_tridiag_to_band(hh, tau, Zc[:, c:c + 1], n, nbw,
                                                           nthreads=1),
                           range(Zc.shape[1])))
    return np.concatenate(cols, axis=1)


# The remaining stated full sizes: n = 8192 with every eigenvector, and fp32
# and complex fp64 at n = 20000 with 10000 and 20000 eigenvectors (the tile
# heights and stripe counts of those launch schedules).  Inputs are drawn on
# the device (workload.device_*, same structure and distribution as the numpy
# generators); the oracle gets the same values copied back (fp32: the rounded
# values, in fp64).
FULL_DEVICE = [
    (8192, 64, 8192, "r64"),
    (20000, 64, 10000, "r32"), (20000, 64, 20000, "r32"),
    (20000, 64, 10000, "c64"), (20000, 64, 20000, "c64"),
]


@pytest.mark.parametrize("case", FULL_DEVICE, ids=[f"n{c[0]}_e{c[2]}_{c[3]}" for c in FULL_DEVICE])
def test_parity_full_size_device_inputs(torch_dev, case):
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw, nev, dt = case
    cplx = dt == "c64"
    print(f"full case n={n} nev={nev} dt={dt} (device inputs)", flush=True)
    g = torch.Generator(device=dev)
    g.manual_seed(7000 + n + nev + (1 if dt == "r32" else 2 if cplx else 0))
    hh, tau = W.device_reflectors(torch, n, nbw, dev, g, complex_=cplx)
    Z = W.device_block(torch, n, nev, dev, g, complex_=cplx)
    if dt == "r32":
        hh, tau, Z = hh.float(), tau.float(), Z.t().float().t()
    q = Z.t().clone().t()                          # column major, the call's Q
    cols = sampled_columns(nev) + [nev // 3, (2 * nev) // 3]
    cols = sorted(set(cols))
    Zc = Z[:, cols].cpu().numpy().astype(np.complex128 if cplx else np.float64)
    hh_h = hh.cpu().numpy().astype(np.complex128 if cplx else np.float64)
    tau_h = tau.cpu().numpy().astype(np.complex128 if cplx else np.float64)
    P.profile_enable(True)
    try:
        P.hh_trafo(q, hh, tau, nbw)
        pr = P.profile_last()
    finally:
        P.profile_enable(False)
    torch.cuda.synchronize()
    print(f"  plan path={pr['path']} k={pr['k']} steps={pr['steps']} streams={pr['streams']} "
          f"launches={pr['launches']} kernel {pr['kernel_ms']:.1f} ms", flush=True)
    got = q[:, cols].cpu().numpy()
    ref = oracle_columns(hh_h, tau_h, Zc, n, nbw)
    err = checks.max_rel_err(got.astype(ref.dtype), ref)
    print(f"  sampled max-abs rel err = {err:.3e} over {len(cols)} columns", flush=True)
    assert err <= TOL[dt]
    # orthogonal / unitary reflectors preserve every column norm (all columns)
    wide = torch.complex128 if cplx else torch.float64
    nq = torch.linalg.vector_norm(q.to(wide), dim=0)
    nz = torch.linalg.vector_norm(Z.to(wide), dim=0)
    rel = ((nq - nz).abs() / nz).max().item()
    assert rel <= (1e-4 if dt == "r32" else 1e-11), rel


def test_workspace_beyond_device_memory_is_nomem(torch_dev):
    """A call whose workspace exceeds the device's memory returns
    ELPA_ERR_NOMEM with nothing enqueued (the library refuses such a size
    before asking the allocator, so no kernel can run); Q is untouched and
    the next calls work."""
    torch, dev = torch_dev
    import paper_1811_01277_amd as P
    n, nbw = 20000, 64
    total = torch.cuda.get_device_properties(dev).total_memory
    nev = 4_000_000                                   # stripe copy alone ~640 GB
    need = P.workspace_bytes(n, nev, nbw, P.R64)
    assert need > 2 * total, (need, total)
    q = torch.zeros(64, device=dev, dtype=torch.float64)
    h = torch.zeros(64, device=dev, dtype=torch.float64)
    before = q.clone()
    rc = P.hh_trafo_ptr(n, nev, nbw, h.data_ptr(), h.data_ptr(), q.data_ptr(), n, P.R64)
    assert rc == -4, rc
    rc = P.hh_trafo_batched_ptr([(n, nev, nbw, n, h.data_ptr(), h.data_ptr(), q.data_ptr(),
                                  P.R64)])
    assert rc == -4, rc
    torch.cuda.synchronize()
    assert torch.equal(q, before)
    # the library and torch keep working
    hh, tau, Z = oracle_inputs(100, 32, 40, "r64", 51)
    got = run_gpu(torch, dev, hh, tau, Z, 32, "r64")
    assert checks.max_rel_err(got, bt.bt_tridiag_to_band(hh, tau, Z, 100, 32)) <= 1e-12
