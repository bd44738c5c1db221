"""Plan tuner cache (CPU): explicit entries, size classes, save / load round
trip, refusal of malformed files and of plans that cannot run."""
import os

import pytest

import paper_1811_01277_amd as P


@pytest.fixture(autouse=True)
def clean():
    P.tuner_clear()
    yield
    P.tuner_clear()


def test_set_get_size_classes():
    assert P.tuner_size() == 0 and P.tuner_get(P.R64, 64, 20000, 20000) is None
    P.tuner_set(P.R64, 64, 20000, 20000, path=P.PATH_SPLIT, k=64, steps=8, streams=2)
    got = P.tuner_get(P.R64, 64, 20000, 20000)
    assert got == {"path": P.PATH_SPLIT, "k": 64, "steps": 8, "order": 0, "streams": 2, "batch": 0}
    # quarter-octave classes: 4 log2(20000) = 57.15, [19504, 23193) shares it
    assert P.tuner_get(P.R64, 64, 21000, 19600) == got
    assert P.tuner_get(P.R64, 64, 24000, 20000) is None
    assert P.tuner_get(P.R64, 32, 20000, 20000) is None          # other nbw
    assert P.tuner_get(P.R32, 64, 20000, 20000) is None          # other dtype
    assert P.tuner_size() == 1
    P.tuner_set(P.R64, 64, 20500, 20000, path=P.PATH_SPLIT, k=80)  # same class: replaced
    assert P.tuner_size() == 1 and P.tuner_get(P.R64, 64, 20000, 20000)["k"] == 80


def test_set_refuses_plans_that_cannot_run():
    with pytest.raises(P.ElpaError) as e:
        P.tuner_set(P.R64, 64, 1000, 1000, path=P.PATH_SPLIT, k=63)
    assert e.value.code == -6
    with pytest.raises(P.ElpaError) as e:
        P.tuner_set(P.C64, 64, 1000, 1000, path=P.PATH_WY, k=64)   # no such complex WY k
    assert e.value.code == -6
    with pytest.raises(P.ElpaError) as e:
        P.tuner_set(P.R64, 64, 1000, 1000, path=P.PATH_SPLIT, k=64, streams=9)
    assert e.value.code == -1
    assert P.tuner_size() == 0


def test_save_load_round_trip(tmp_path):
    P.tuner_set(P.R64, 64, 20000, 2000, path=P.PATH_SPLIT, k=80, steps=2, streams=2)
    P.tuner_set(P.R32, 64, 20000, 2000, path=P.PATH_WY, k=64)
    P.tuner_set(P.C64, 64, 8192, 8192, path=P.PATH_STRIPE, k=4, order=P.ORDER_XCD)
    f = tmp_path / "plans.txt"
    P.tuner_save(str(f))
    text = f.read_text().splitlines()
    assert text[0] == "elpa_hh_tuner 1" and len([l for l in text if not l.startswith("#")]) == 4
    before = {k: P.tuner_get(*k) for k in [(P.R64, 64, 20000, 2000), (P.R32, 64, 20000, 2000),
                                           (P.C64, 64, 8192, 8192)]}
    P.tuner_clear()
    assert P.tuner_size() == 0
    P.tuner_load(str(f))
    assert P.tuner_size() == 3
    for k, v in before.items():
        assert P.tuner_get(*k) == v


@pytest.mark.parametrize("body", [
    "not a tuner file\n",
    "elpa_hh_tuner 1\n0 64 57 57 3 64 8 0\n",            # a field missing
    "elpa_hh_tuner 1\n0 64 57 57 3 63 8 0 2\n",          # no k = 63 kernel
    "elpa_hh_tuner 1\n0 64 57 57 9 64 8 0 2\n",          # no such path
])
def test_load_refuses_bad_files_whole(tmp_path, body):
    P.tuner_set(P.R64, 64, 100, 100, path=P.PATH_REF)
    f = tmp_path / "bad.txt"
    f.write_text(body)
    with pytest.raises(P.ElpaError) as e:
        P.tuner_load(str(f))
    assert e.value.code == -1
    assert P.tuner_size() == 1                           # cache unchanged
    with pytest.raises(P.ElpaError):
        P.tuner_load(os.path.join(str(tmp_path), "missing.txt"))


def test_workspace_queries_follow_tuned_plan():
    # a call without a plan runs the tuned plan, so its workspace is that plan's
    n, nev = 20000, 20000
    wy = P.workspace_bytes(n, nev, 64, P.R64, path=P.PATH_WY, k=32)
    assert P.workspace_bytes(n, nev, 64, P.R64) != wy
    P.tuner_set(P.R64, 64, n, nev, path=P.PATH_WY, k=32)
    assert P.workspace_bytes(n, nev, 64, P.R64) == wy
    one = [(n, nev, 64, P.R64)]
    assert (P.workspace_bytes_batched(one) ==
            P.workspace_bytes_batched(one, path=P.PATH_WY, k=32))


def test_tune_batched_argument_errors():
    # rejected before anything touches a device
    with pytest.raises(P.ElpaError) as e:
        P.tune_batched([], level=0, stream=0)
    assert e.value.code == -1
    import ctypes as C
    from paper_1811_01277_amd import binding as B
    arr = (B._Problem * 1)()
    arr[0] = B._Problem(100, 10, 32, 100, None, None, None, P.R64, 0)
    out = B._Plan()
    assert B.library().elpa_hh_tune_batched(arr, 1, None, 3, C.byref(out)) == -1   # level
    arr[0] = B._Problem(100, 10, 32, 99, None, None, None, P.R64, 0)
    assert B.library().elpa_hh_tune_batched(arr, 1, None, 0, C.byref(out)) == -1   # ldq < n
    arr[0] = B._Problem(100, 10, 32, 100, None, None, None, 7, 0)
    assert B.library().elpa_hh_tune_batched(arr, 1, None, 0, C.byref(out)) == -2   # dtype


def test_autotune_setup_levels_fixed_and_state_round_trip(tmp_path):
    """On-the-fly autotuning state (no device call is made here)."""
    fast = P.Autotune(P.AUTOTUNE_FAST, 20000, 20000, 64, P.R64)
    med = P.Autotune(P.AUTOTUNE_MEDIUM, 20000, 20000, 64, P.R64)
    split = P.Autotune(P.AUTOTUNE_MEDIUM, 20000, 20000, 64, P.R64, path=P.PATH_SPLIT)
    k80 = P.Autotune(P.AUTOTUNE_MEDIUM, 20000, 20000, 64, P.R64, path=P.PATH_SPLIT, k=80)
    # FAST: one candidate per kernel family; MEDIUM: also k, tile height, streams
    assert fast.candidates == 3
    assert med.candidates > split.candidates > k80.candidates == 10
    f = tmp_path / "state.txt"
    split.save(str(f))
    text = f.read_text().splitlines()
    assert text[0] == "elpa_hh_autotune 1" and len(text) == 2 + split.candidates
    assert all(line.split()[0] == "3" for line in text[2:])      # the fixed family only
    back = P.Autotune.load(str(f))
    g = tmp_path / "again.txt"
    back.save(str(g))
    assert g.read_text() == f.read_text()
    with pytest.raises(P.ElpaError):
        back.best()                                    # nothing timed yet
    bad = tmp_path / "bad.txt"
    bad.write_text("elpa_hh_autotune 1\n0 0 100 100 64 0 1\n3 63 0 0 1 -1\n")   # k = 63
    with pytest.raises(P.ElpaError):
        P.Autotune.load(str(bad))
    with pytest.raises(P.ElpaError):
        P.Autotune(5, 1000, 1000, 64, P.R64)
    with pytest.raises(P.ElpaError):
        P.Autotune(P.AUTOTUNE_FAST, 1000, 1000, 64, P.R64, path=P.PATH_WY, k=63)


def test_plan_with_only_streams_set_takes_tuned_kernel():
    """A plan that sets only streams (or order) leaves the kernel open: it runs
    the tuned plan's kernel, so its workspace is that plan's."""
    import ctypes as C
    from paper_1811_01277_amd import binding as B
    n, nev = 20000, 20000
    wy = P.workspace_bytes(n, nev, 64, P.R64, path=P.PATH_WY, k=32)
    streams_only = B._Plan(0, 0, 0, 0, 1, 0)
    lib = B.library()
    before = lib.elpa_hh_workspace_bytes(n, nev, 64, P.R64, C.byref(streams_only))
    assert before != wy
    P.tuner_set(P.R64, 64, n, nev, path=P.PATH_WY, k=32)
    assert lib.elpa_hh_workspace_bytes(n, nev, 64, P.R64, C.byref(streams_only)) == wy
    # an explicit kernel field keeps the caller's plan
    k80 = B._Plan(0, 80, 0, 0, 1, 0)
    assert lib.elpa_hh_workspace_bytes(n, nev, 64, P.R64, C.byref(k80)) != wy
