"""The C-ABI library loads and exports every symbol include/lhaf.h declares;
host-only entry points (planner, term counts) work without a GPU."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lhaf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)
    skip = {"if", "sizeof", "defined"}
    return sorted({n for n in names if n not in skip and (n.startswith("lh"))})


@pytest.fixture(scope="module")
def L():
    from paper_2108_01622_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        from paper_2108_01622_amd import build
        build.build()
    return _binding


def test_exports_every_declared_symbol(L):
    lib = L.lib()
    decl = declared_functions()
    assert "lhaf" in decl and "lhaf_backward" in decl and "lhaf_batched" in decl
    for name in decl:
        assert hasattr(lib, name), name
    assert set(L.EXPORTED) == set(decl)


def test_status_strings(L):
    assert L.lib().lh_status_string(0) == b"ok"
    assert b"too large" in L.lib().lh_status_string(2)
    assert L.lib().lhaf_schedule_count() >= 4


def test_planner_worked_example(L):
    """(2,1,0,3) -> pairs (3,0) x 2 and (3,1) x 1: 6 repeated-pair terms (Sec. 2)."""
    pos, eta = L.plan_pairs(4, [2, 1, 0, 3])
    H = len(eta)
    pairs = sorted((max(pos[p], pos[H + p]), min(pos[p], pos[H + p]), eta[p]) for p in range(H))
    assert pairs == [(3, 0, 2), (3, 1, 1)]
    assert L.term_count(4, [2, 1, 0, 3], sum="et") == 6
    # FDS halves on the first pair with odd eta: (2+1) * (1//2+1) = 3
    assert L.term_count(4, [2, 1, 0, 3], sum="fds") == 3


def test_planner_matches_oracle_greedy(L, orc):
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(200):
        M = int(rng.integers(1, 10))
        r = rng.integers(0, 5, size=M).astype(np.int32)
        if r.sum() == 0 or r.sum() > 64:
            continue
        pos, eta = L.plan_pairs(M, r)
        pairs, left = orc.matched_reps(r)
        want = [(a, b, e) for a, b, e in pairs] + ([(left, -1, 1)] if left is not None else [])
        H = len(eta)
        got = [(int(pos[p]), int(pos[H + p]), int(eta[p])) for p in range(H)]
        assert got == want, (r, got, want)
        for mode in ("et", "fds"):
            assert L.term_count(M, r, sum=mode) == orc.term_count([w[2] for w in want], mode=mode)


def test_plain_pairs_and_padding(L):
    pos, eta = L.plan_pairs(5)
    assert list(pos) == [0, 1, 2, 3, 4, -1] and list(eta) == [1, 1, 1]
    assert L.term_count(40) == 2 ** 19
    assert L.term_count(40, sum="et") == 2 ** 20


def test_invalid_arguments(L):
    import ctypes
    lib = L.lib()
    o = L.make_opts()
    # N > 64 is rejected synchronously, before any device work
    assert lib.lhaf(None, 65, None, 65, None, None, ctypes.byref(o), None) == 1  # null out -> EINVAL
    assert L.lib().lhaf_plan_pairs(65, None, ctypes.c_void_p(np.zeros(200, np.int32).ctypes.data),
                                   ctypes.c_void_p(np.zeros(200, np.int32).ctypes.data)) == -2
    r = np.array([1, -1], dtype=np.int32)
    assert L.lib().lhaf_term_count(2, L.host_ptr(r), 1) == -1


def test_compensated_mode_gating(L):
    """acc = LH_ACC_DD_COMP is accepted by the value entry points only; the
    others refuse it before any device work (LH_EUNSUPPORTED), and an unknown
    accumulation mode is an invalid argument."""
    import ctypes
    src = open(os.path.join(ROOT, "include", "lhaf.h")).read()
    assert int(re.search(r"#define LH_ACC_DD_COMP (\d+)", src).group(1)) == L.LH_ACC_DD_COMP
    lib = L.lib()
    o = L.make_opts(acc="ddc")
    EUNS = 5
    assert lib.lhaf_backward(1, None, 2, 4, None, 2, None, None, None, None, None, None, 1, None, 0,
                             ctypes.byref(o), None) == EUNS
    assert lib.lhaf_real(None, 2, None, None, 1, None, None, ctypes.byref(o), None) == EUNS
    assert lib.lhaf_chain(None, 2, None, None, 1, 0, 2, None, None, ctypes.byref(o), None) == EUNS
    assert lib.lhaf_gammas(None, 2, None, 2, None, 1, 1, None, None, ctypes.byref(o), None) == EUNS
    og = L.make_opts(acc="ddc")
    og.grads = ctypes.c_void_p(16)
    og.grads_count = 1
    assert lib.lhaf_batched(1, None, 2, 4, None, 2, None, None, None, None, None, None, 0,
                            ctypes.byref(og), None) == EUNS
    os_ = L.make_opts(acc="ddc")
    os_.saved = ctypes.c_void_p(16)
    os_.saved_count = 1
    assert lib.lhaf(None, 2, None, 2, None, None, ctypes.byref(os_), None) == EUNS
    bad = L.make_opts()
    bad.acc = 3
    assert lib.lhaf(None, 2, None, 2, None, None, ctypes.byref(bad), None) == 1
    # the value entry points accept it (a null output is then the first error)
    assert lib.lhaf(None, 2, None, 2, None, None, ctypes.byref(o), None) == 1


def test_saved_count(L):
    """Entries of the per-term coefficient store: sum over problems of terms x n."""
    import ctypes
    lib = L.lib()
    for s in ("fds", "et"):
        o = L.make_opts(sum=s)
        off = np.array([0, 40, 80, 91], dtype=np.int64)  # N = 40, 40, 11 (padded to 12)
        want = 2 * L.term_count(40, sum=s) * 20 + L.term_count(11, sum=s) * 6
        assert lib.lhaf_saved_count(3, L.host_ptr(off), None, ctypes.byref(o)) == want
        r = np.array([2, 1, 3, 0, 1], dtype=np.int32)  # one repeated problem, n = 7/2 -> 4
        off = np.array([0, 5], dtype=np.int64)
        assert lib.lhaf_saved_count(1, L.host_ptr(off), L.host_ptr(r), ctypes.byref(o)) == \
            L.term_count(5, r, sum=s) * 4
        off = np.array([0, 0], dtype=np.int64)  # empty problem: no terms stored
        assert lib.lhaf_saved_count(1, L.host_ptr(off), None, ctypes.byref(o)) == 0
    bad = np.array([0, 65], dtype=np.int64)
    assert lib.lhaf_saved_count(1, L.host_ptr(bad), None, ctypes.byref(L.make_opts())) == -2
