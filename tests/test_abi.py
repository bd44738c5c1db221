"""Host-side tests of the C ABI (no GPU needed, no compute call is made).

* The library loads and exports every function include/*.h declares.
* Slot arithmetic equals a brute-force enumeration.
* Every invalid argument returns its error code before anything is enqueued
  (checked with host buffers that must stay untouched), n <= 1 and nev == 0
  are no-ops.
"""
import ctypes as C
import glob
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1811_01277_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(elpa_\w+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = P.library()
    names = header_functions()
    assert "elpa_hh_trafo" in names and "elpa_bt2_trafo" in names and len(names) >= 9
    for nm in names:
        assert hasattr(lib, nm), nm
    out = subprocess.run(["nm", "-D", "--defined-only", P.library_path()],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (elpa_\w+)", out))
    assert set(names) <= exported


@pytest.mark.parametrize("n,b", [(0, 1), (1, 4), (2, 1), (3, 2), (17, 4), (64, 64), (65, 64),
                                 (512, 32), (8192, 64), (1000, 7)])
def test_slot_arithmetic_brute_force(n, b):
    J = [-(-(n - 1 - s) // b) for s in range(max(n - 1, 0))]
    assert P.num_reflectors(n, b) == sum(J)
    acc = 0
    for s in range(max(n - 1, 0)):
        assert P.slot_offset(n, b, s) == acc
        acc += J[s]
    if n >= 1:
        assert P.slot_offset(n, b, n - 1) == acc


def test_slot_arithmetic_large():
    assert P.num_reflectors(20000, 64) == 3134695
    assert P.num_reflectors(8192, 64) == 528256
    assert P.num_reflectors(2000, 32) == 63441
    assert P.num_reflectors(5, 0) == -1


def _buf(nbytes, fill=7):
    a = np.full(nbytes, fill, dtype=np.uint8)
    return a, a.ctypes.data


def test_error_codes_and_untouched_buffers():
    q, qp = _buf(4096)
    h, hp = _buf(4096)
    t, tp = _buf(512)
    snap = q.copy()
    E = {"arg": -1, "dtype": -2, "align": -3}
    cases = [
        (dict(n=10, nev=5, nbw=0), E["arg"]),          # nbw < 1
        (dict(n=-1, nev=5, nbw=2), E["arg"]),          # n < 0
        (dict(n=10, nev=-1, nbw=2), E["arg"]),         # nev < 0
        (dict(n=10, nev=5, nbw=2, ldq=9), E["arg"]),   # ldq < n
        (dict(n=10, nev=5, nbw=2, dtype=7), E["dtype"]),
        (dict(n=10, nev=5, nbw=2, dtype=-1), E["dtype"]),
        (dict(n=10, nev=5, nbw=2, q=0), E["arg"]),     # null pointers
        (dict(n=10, nev=5, nbw=2, hh=0), E["arg"]),
        (dict(n=10, nev=5, nbw=2, tau=0), E["arg"]),
        (dict(n=10, nev=5, nbw=2, q=qp + 4), E["align"]),
        (dict(n=10, nev=5, nbw=2, hh=hp + 8, dtype=2), E["align"]),
        (dict(n=10, nev=5, nbw=2, tau=tp + 2, dtype=1), E["align"]),
        (dict(n=10, nev=5, nbw=2, path=9), -6),        # unknown plan path
        (dict(n=10, nev=5, nbw=5, path=2, k=3), -6),   # stripe not built for nbw=5
        (dict(n=10, nev=2, nbw=2, ldq=2 ** 62), E["arg"]),  # address overflow
    ]
    for kw, want in cases:
        a = dict(n=10, nev=5, nbw=2, hh=hp, tau=tp, q=qp, ldq=None, dtype=0, path=None, k=0)
        a.update(kw)
        ldq = a["n"] if a["ldq"] is None else a["ldq"]
        rc = P.hh_trafo_ptr(a["n"], a["nev"], a["nbw"], a["hh"], a["tau"], a["q"], ldq,
                            a["dtype"], 0, a["path"], a["k"])
        assert rc == want, (kw, rc)
        assert P.strerror(rc) and P.strerror(rc) != "unknown error code"
    assert np.array_equal(q, snap)


def test_noops_touch_nothing():
    # n <= 1 or nev == 0: success without dereferencing anything (null pointers)
    assert P.hh_trafo_ptr(1, 5, 3, 0, 0, 0, 1, 0) == 0
    assert P.hh_trafo_ptr(0, 5, 3, 0, 0, 0, 1, 0) == 0
    assert P.hh_trafo_ptr(10, 0, 3, 0, 0, 0, 10, 0) == 0


def test_plan_support_table():
    assert P.plan_supported(64, P.R64, P.PATH_STRIPE, 16)
    assert P.plan_supported(32, P.R32, P.PATH_STRIPE, 32)
    assert P.plan_supported(5, P.R64, P.PATH_REF)
    assert P.plan_supported(5, P.R64, P.PATH_AUTO)
    assert not P.plan_supported(5, P.R64, P.PATH_STRIPE, 4)
    assert not P.plan_supported(64, 9, P.PATH_AUTO)
    # two-lane kernel: real fp64, nbw 32 / 64, even k
    for nbw, k in [(64, 48), (64, 64), (64, 80), (32, 32), (32, 64), (32, 96)]:
        assert P.plan_supported(nbw, P.R64, P.PATH_SPLIT, k), (nbw, k)
    assert P.plan_supported(64, P.R64, P.PATH_SPLIT)          # library default k
    # fp32 two-lane kernel (four waves per SIMD): nbw 64 with k 64..96, nbw 32 up to 128
    for nbw, k in [(64, 64), (64, 80), (64, 96), (32, 64), (32, 96), (32, 128)]:
        assert P.plan_supported(nbw, P.R32, P.PATH_SPLIT, k), (nbw, k)
    assert not P.plan_supported(64, P.R32, P.PATH_SPLIT, 48)
    assert P.plan_supported(64, P.C64, P.PATH_SPLIT)           # complex: k = 24 default
    assert P.plan_supported(64, P.C64, P.PATH_SPLIT, 16)
    assert not P.plan_supported(64, P.C64, P.PATH_SPLIT, 80)
    assert not P.plan_supported(64, P.R64, P.PATH_SPLIT, 63)
    assert not P.plan_supported(16, P.R64, P.PATH_SPLIT)
    assert not P.plan_supported(64, P.R64, 5)                # no such path
    # compact-WY MFMA path: real fp64 / fp32 and complex fp64, nbw 32 / 64, k a
    # multiple of 16
    for nbw, k, dt in [(64, 32, P.R64), (64, 64, P.R64), (32, 64, P.R64), (64, 64, P.R32),
                       (64, 32, P.C64), (64, 16, P.C64), (32, 32, P.C64)]:
        assert P.plan_supported(nbw, dt, P.PATH_WY, k), (nbw, k, dt)
    assert P.plan_supported(64, P.C64, P.PATH_WY)            # library default k
    assert not P.plan_supported(64, P.R64, P.PATH_WY, 40)
    assert not P.plan_supported(64, P.C64, P.PATH_WY, 64)
    rc = P.hh_trafo_ptr(10, 5, 2, 8, 8, 8, 10, P.R64, 0, None, 0, 0, 3)   # unknown order
    assert rc == -6
    rc = P.hh_trafo_ptr(10, 5, 2, 8, 8, 8, 10, P.R64, 0, None, 0, 0, 0, 9)  # > 8 streams
    assert rc == -6
    pl = P.binding._Plan(0, 0, 0, 0, 0, 3)                                  # unknown batch
    assert P.library().elpa_hh_trafo_plan(10, 5, 2, 8, 8, 8, 10, P.R64, None, C.byref(pl)) == -6


def split_ws_brute(n, nev, nbw, k, es):
    """Workspace of the two-lane kernel by direct summation: the stripe copy
    of Q and the packed step records of every sweep block's existing steps."""
    al = lambda x: -(-x // 256) * 256
    rows_pad = -(-(n + nbw + k) // 64) * 64
    M = -(-(n - 1) // k)
    steps = sum(-(-(n - 1 - m * k) // nbw) for m in range(M))
    rs = 2 * (nbw // 2 + 2)
    return al((steps * k * rs + 32) * es) + al(M * 8) + al(rows_pad * (-(-nev // 32)) * 32 * es)


def wy_ws_brute(n, nev, nbw, k, es, planes, tiles):
    """Workspace of the compact-WY kernel by direct summation: per sweep block
    and existing chase step, k/16 sub-group records of 2 x planes x 4 (nbw/16+1)
    fragments of 64 values; the block table; the stripe copy of Q in stripes of
    16 x tiles columns."""
    al = lambda x: -(-x // 256) * 256
    rows_pad = -(-(n + nbw + k) // 64) * 64
    M = -(-(n - 1) // k)
    steps = sum(-(-(n - 1 - m * k) // nbw) for m in range(M))
    rec = 2 * planes * 4 * (nbw // 16 + 1) * 64
    sw = 16 * tiles
    return (al(steps * (k // 16) * rec * es) + al(M * 8) +
            al(rows_pad * (-(-nev // sw)) * sw * es * (2 if planes == 2 else 1)))


@pytest.mark.parametrize("dt,nbw,k,planes,tiles", [("r64", 64, 160, 1, 2), ("r64", 64, 64, 1, 2),
                                                  ("r64", 32, 96, 1, 2), ("r32", 64, 96, 1, 2),
                                                  ("c64", 64, 48, 2, 1)])
def test_wy_workspace_matches_direct_sum(dt, nbw, k, planes, tiles):
    code = {"r64": P.R64, "r32": P.R32, "c64": P.C64}[dt]
    es = {"r64": 8, "r32": 4, "c64": 8}[dt]
    for n in list(range(2, 300, 7)) + [1000, 4097, 20000]:
        assert P.workspace_bytes(n, 70, nbw, code, P.PATH_WY, k) == \
            wy_ws_brute(n, 70, nbw, k, es, planes, tiles), n


@pytest.mark.parametrize("nbw,k", [(64, 48), (64, 64), (64, 80), (32, 32), (32, 64), (32, 96)])
def test_split_workspace_matches_direct_sum(nbw, k):
    # the library sums the blocks' step counts in closed form (a floor sum);
    # every n from 2 to 400 plus a spread of large ones against the direct sum
    for n in list(range(2, 401)) + [1000, 4097, 8192, 12345, 20000, 65537]:
        assert P.workspace_bytes(n, 33, nbw, P.R64, P.PATH_SPLIT, k) == \
            split_ws_brute(n, 33, nbw, k, 8), n


def test_workspace_bytes():
    # reference path and no-ops allocate nothing; invalid arguments give -1
    assert P.workspace_bytes(100, 10, 7, P.R64) == 0
    assert P.workspace_bytes(1, 10, 64, P.R64) == 0
    assert P.workspace_bytes(100, 10, 0, P.R64) == -1
    assert P.workspace_bytes(100, 10, 64, 9) == -1
    assert P.workspace_bytes(100, 10, 64, P.R64, P.PATH_SPLIT, 63) == -1
    # split path at n = nev = 20000, k = 80: stripe copy (rows_pad x 625 x 32 fp64)
    # plus packed reflectors: one record set of k records of 68 values per
    # (sweep block m, existing chase step j < J0(m)), +32 values, and the
    # table of each block's first record (M int64)
    n, nev, nbw, k = 20000, 20000, 64, 80
    want = split_ws_brute(n, nev, nbw, k, 8)
    assert P.workspace_bytes(n, nev, nbw, P.R64, P.PATH_SPLIT, k) == want
    # the library default at this size: the compact-WY kernel, k = 160
    assert P.workspace_bytes(n, nev, nbw, P.R64) == wy_ws_brute(n, nev, nbw, 160, 8, 1, 2)
    assert P.workspace_bytes(2000, 2000, nbw, P.R64) == split_ws_brute(2000, 2000, nbw, 80, 8)
    assert P.workspace_bytes(n, nev, nbw, P.C64) > 0
    # batched: the kernels a batched call picks, plus descriptor tables
    one = P.workspace_bytes_batched([(n, nev, nbw, P.R64)])
    assert one >= want and one < want + (1 << 20)
    two = P.workspace_bytes_batched([(n, nev, nbw, P.R64), (500, 300, 32, P.R32)])
    assert two > one
    assert P.workspace_bytes_batched([(500, 300, 32, P.R32)]) >= \
        P.workspace_bytes(500, 300, 32, P.R32)
    assert P.workspace_bytes_batched([(500, 300, 32, P.R32)], path=P.PATH_WY) >= \
        P.workspace_bytes(500, 300, 32, P.R32, P.PATH_WY)
    assert P.workspace_bytes_batched([(500, 300, 0, P.R32)]) == -1
    assert P.workspace_bytes_batched([]) == 0


def test_profile_api_without_calls():
    P.profile_enable(False)
    with pytest.raises(P.ElpaError) as e:
        P.profile_last()                  # nothing recorded
    assert e.value.code == -1
    assert P.strerror(12345) == "unknown error code"


def test_bt2_argument_errors_and_workspace():
    """Band -> full back-transformation: argument checks run before anything
    touches a device; no-op sizes succeed; workspace sizes."""
    lib = P.library()
    nul = None
    # n <= nbw or nev == 0: nothing to do
    assert lib.elpa_bt2_trafo(64, 10, 64, nul, 64, nul, nul, 64, P.R64, nul, 0) == 0
    assert lib.elpa_bt2_trafo(100, 0, 32, nul, 100, nul, nul, 100, P.R64, nul, 0) == 0
    assert lib.elpa_bt2_trafo(100, 5, 32, nul, 100, nul, nul, 100, 7, nul, 0) == -2
    assert lib.elpa_bt2_trafo(100, 5, 0, nul, 100, nul, nul, 100, P.R64, nul, 0) == -1
    assert lib.elpa_bt2_trafo(100, 5, 32, nul, 100, nul, nul, 99, P.R64, nul, 0) == -1   # ldq
    assert lib.elpa_bt2_trafo(100, 5, 32, nul, 99, nul, nul, 100, P.R64, nul, 0) == -1   # ldv
    assert lib.elpa_bt2_trafo(100, 5, 32, nul, 100, nul, nul, 100, P.R64, nul, 0) == -1  # nulls
    assert lib.elpa_bt2_trafo(100, 5, 32, nul, 100, nul, nul, 100, P.R64, nul, 513) == -1
    assert P.bt2_workspace_bytes(100, 5, 32, P.R64) > 0
    assert P.bt2_workspace_bytes(32, 5, 32, P.R64) == 0
    assert P.bt2_workspace_bytes(100, 5, 32, 9) == -1
    # V block (68 x 64) + G + M (64 x 64 each) + W (64 x 5) + partial products
    # (68 rows: one K chunk, the larger of W's and G's), 256-byte aligned
    al = lambda x: -(-x // 256) * 256
    assert P.bt2_workspace_bytes(100, 5, 32, P.R64, 64) == \
        al(68 * 64 * 8) + 2 * al(64 * 64 * 8) + al(64 * 5 * 8) + al(64 * 64 * 8)


def test_band_to_tridiag_argument_errors():
    """Bulge chasing: argument checks before anything touches a device."""
    lib = P.library()
    nul = None
    assert lib.elpa_band_to_tridiag(10, 2, nul, 10, nul, nul, nul, nul, P.R32, nul) == -2
    assert lib.elpa_band_to_tridiag(10, 2, nul, 10, nul, nul, nul, nul, 9, nul) == -2
    assert lib.elpa_band_to_tridiag(0, 2, nul, 10, nul, nul, nul, nul, P.R64, nul) == -1
    assert lib.elpa_band_to_tridiag(10, 0, nul, 10, nul, nul, nul, nul, P.R64, nul) == -1
    assert lib.elpa_band_to_tridiag(10, 513, nul, 10, nul, nul, nul, nul, P.R64, nul) == -1
    assert lib.elpa_band_to_tridiag(10, 2, nul, 9, nul, nul, nul, nul, P.R64, nul) == -1
    assert lib.elpa_band_to_tridiag(10, 2, nul, 10, nul, nul, nul, nul, P.R64, nul) == -1


def test_full_to_band_argument_errors():
    lib = P.library()
    nul = None
    assert lib.elpa_full_to_band(10, 2, nul, 10, nul, 10, nul, P.R32, nul) == -2
    assert lib.elpa_full_to_band(0, 2, nul, 10, nul, 10, nul, P.R64, nul) == -1
    assert lib.elpa_full_to_band(10, 0, nul, 10, nul, 10, nul, P.R64, nul) == -1
    assert lib.elpa_full_to_band(10, 257, nul, 10, nul, 10, nul, P.R64, nul) == -1
    assert lib.elpa_full_to_band(10, 2, nul, 9, nul, 10, nul, P.R64, nul) == -1
    assert lib.elpa_full_to_band(10, 2, nul, 10, nul, 9, nul, P.R64, nul) == -1
    assert lib.elpa_full_to_band(10, 2, nul, 10, nul, 10, nul, P.R64, nul) == -1


def test_generalized_argument_errors():
    """Cholesky inverse and the two generalized transformations: argument
    checks before anything touches a device; n = 0 is a no-op."""
    lib = P.library()
    nul = None
    assert lib.elpa_cholesky_inverse(10, nul, 10, P.R32, nul, nul) == -2
    assert lib.elpa_cholesky_inverse(-1, nul, 10, P.R64, nul, nul) == -1
    assert lib.elpa_cholesky_inverse(10, nul, 9, P.R64, nul, nul) == -1
    assert lib.elpa_cholesky_inverse(1 << 31, nul, 1 << 31, P.R64, nul, nul) == -1
    assert lib.elpa_cholesky_inverse(10, nul, 10, P.R64, nul, nul) == -1
    assert lib.elpa_cholesky_inverse(0, nul, 1, P.C64, nul, nul) == 0
    assert lib.elpa_generalized_to_standard(10, nul, 10, nul, 10, P.R32, nul) == -2
    assert lib.elpa_generalized_to_standard(10, nul, 9, nul, 10, P.R64, nul) == -1
    assert lib.elpa_generalized_to_standard(10, nul, 10, nul, 9, P.R64, nul) == -1
    assert lib.elpa_generalized_to_standard(10, nul, 10, nul, 10, P.C64, nul) == -1
    assert lib.elpa_generalized_to_standard(0, nul, 1, nul, 1, P.R64, nul) == 0
    assert lib.elpa_generalized_back(10, 3, nul, 10, nul, 10, 7, nul) == -2
    assert lib.elpa_generalized_back(10, -1, nul, 10, nul, 10, P.R64, nul) == -1
    assert lib.elpa_generalized_back(10, 3, nul, 10, nul, 9, P.R64, nul) == -1
    assert lib.elpa_generalized_back(10, 3, nul, 10, nul, 10, P.R64, nul) == -1
    assert lib.elpa_generalized_back(10, 0, nul, 10, nul, 10, P.R64, nul) == 0


def test_tridiag_eigh_argument_errors():
    lib = P.library()
    nul = None
    assert lib.elpa_tridiag_eigh(10, 3, nul, nul, nul, nul, 10, 5, nul) == -2
    assert lib.elpa_tridiag_eigh(-1, 0, nul, nul, nul, nul, 10, P.R64, nul) == -1
    assert lib.elpa_tridiag_eigh(10, 11, nul, nul, nul, nul, 10, P.R64, nul) == -1
    assert lib.elpa_tridiag_eigh(10, 3, nul, nul, nul, nul, 9, P.R64, nul) == -1
    assert lib.elpa_tridiag_eigh(10, 3, nul, nul, nul, nul, 10, P.R64, nul) == -1
    assert lib.elpa_tridiag_eigh(1 << 31, 0, nul, nul, nul, nul, 1 << 31, P.R64, nul) == -1
    assert lib.elpa_tridiag_eigh(0, 0, nul, nul, nul, nul, 1, P.R64, nul) == 0


def test_chosen_plan_single_and_batched():
    """The kernel choice a call would make, without a device: the compact-WY
    kernel for large fp64 single calls, the two-lane kernel below n = 3000 and
    in batched calls (k = 96 at nbw = 32 there, 64 for a single call)."""
    P.tuner_clear()
    assert P.chosen_plan(20000, 20000, 64, P.R64)["path"] == P.PATH_WY
    assert P.chosen_plan(20000, 20000, 64, P.R64)["k"] == 160
    # few columns: the T-build would dominate, the two-lane kernel runs
    assert P.chosen_plan(8192, 819, 64, P.R64)["path"] == P.PATH_SPLIT
    assert P.chosen_plan(8192, 1024, 64, P.R64)["path"] == P.PATH_WY
    assert P.chosen_plan(8192, 819, 64, P.R32)["path"] == P.PATH_WY
    assert P.chosen_plan(20000, 20000, 64, P.R32)["k"] == 160
    assert P.chosen_plan(4000, 4000, 64, P.R32)["k"] == 96
    one = P.chosen_plan(1000, 1000, 64, P.R64)
    assert one["path"] == P.PATH_SPLIT and one["k"] == 80
    assert P.chosen_plan(20000, 20000, 64, P.R64, batched=True)["path"] == P.PATH_SPLIT
    assert P.chosen_plan(1000, 1000, 32, P.R64)["k"] == 64
    big32 = P.chosen_plan(4000, 4000, 32, P.R64)
    assert big32["path"] == P.PATH_WY and big32["k"] == 96
    assert P.chosen_plan(4000, 4000, 32, P.R32)["path"] == P.PATH_WY
    assert P.chosen_plan(4000, 4000, 32, P.C64)["path"] == P.PATH_SPLIT
    assert P.chosen_plan(1000, 1000, 32, P.R64, batched=True)["k"] == 96
    assert P.chosen_plan(1000, 1000, 32, P.R64, path=P.PATH_SPLIT, k=32)["k"] == 32
    assert P.chosen_plan(100, 100, 7, P.R64)["path"] == P.PATH_REF
    with pytest.raises(P.ElpaError) as e:
        P.chosen_plan(100, 100, 64, P.R64, path=P.PATH_SPLIT, k=63)
    assert e.value.code == -6
    with pytest.raises(P.ElpaError) as e:
        P.chosen_plan(100, 100, 64, 9)
    assert e.value.code == -2


@pytest.mark.parametrize("dt,nbw,n,nev,path,k", [
    ("r64", 64, 2999, 2999, "split", 80), ("r64", 64, 3000, 3000, "wy", 128),
    ("r64", 64, 5999, 5999, "wy", 128), ("r64", 64, 6000, 6000, "wy", 160),
    ("r64", 64, 20000, 1023, "split", 80), ("r64", 64, 20000, 1024, "wy", 160),
    ("r32", 64, 5999, 5999, "wy", 96), ("r32", 64, 6000, 6000, "wy", 160),
    ("r32", 64, 500, 100, "wy", 96), ("c64", 64, 500, 100, "wy", 48),
    ("r64", 32, 1999, 1999, "split", 64), ("r64", 32, 2000, 2000, "wy", 96),
    ("r32", 32, 2000, 1023, "split", 64), ("r32", 32, 2000, 1024, "wy", 96),
    ("c64", 32, 8000, 8000, "split", 48),
])
def test_library_choice_boundaries(dt, nbw, n, nev, path, k):
    """The single-call kernel choice at the edges of its size rules (no tuned
    plan): compact-WY for fp64 from n = 3000 with nev >= 1024 (k = 160 from
    n = 6000), fp32 and complex at nbw = 64 (fp32 k = 160 from n = 6000), real
    data at nbw = 32 from n = 2000 with nev >= 1024; the two-lane kernel
    otherwise."""
    P.tuner_clear()
    code = {"r64": P.R64, "r32": P.R32, "c64": P.C64}[dt]
    got = P.chosen_plan(n, nev, nbw, code)
    want = {"split": P.PATH_SPLIT, "wy": P.PATH_WY}[path]
    assert (got["path"], got["k"]) == (want, k), got
