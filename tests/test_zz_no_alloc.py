"""lhaf_batched_noalloc (the entry point for callers that cannot allocate)
against lhaf_batched, through the C ABI: two calls in a row, the second on a
smaller batch, each compared with the existing entry point on the same
inputs; plus the size limit.  The two entry points share the planner and the
kernels, so the results agree bit for bit."""
import ctypes

import numpy as np
import pytest

from paper_2108_01622_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _call(T, name, A, g, idx, off, sum_mode="fds", acc="dd"):
    from paper_2108_01622_amd import _binding as Bn
    L = Bn.lib()
    B = len(off) - 1
    out = T.empty(B, dtype=T.complex128, device="cuda")
    err = T.empty(B, dtype=T.float64, device="cuda")
    o = Bn.make_opts(sum_mode, acc)
    st = ctypes.c_void_p(T.cuda.current_stream().cuda_stream)
    lda = A.shape[-1]
    sA = 0 if A.dim() == 2 else A.shape[1] * A.shape[2]
    sg = 0 if g.dim() == 1 else g.shape[1]
    offh = np.ascontiguousarray(off, dtype=np.int64)
    ip = ctypes.c_void_p(idx.data_ptr()) if idx is not None else None
    args = [B, ctypes.c_void_p(A.data_ptr()), lda, sA, ctypes.c_void_p(g.data_ptr()), sg, ip,
            Bn.host_ptr(offh), None, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(err.data_ptr())]
    if name == "lhaf_batched":
        need = int(L.lhaf_batched_workspace(B, Bn.host_ptr(offh), None, ctypes.byref(o)))
        ws = T.empty(need, dtype=T.uint8, device="cuda")
        status = L.lhaf_batched(*args, ctypes.c_void_p(ws.data_ptr()), need, ctypes.byref(o), st)
    else:
        status = L.lhaf_batched_noalloc(*args, ctypes.byref(o), st)
    T.cuda.synchronize()
    return status, out.cpu().numpy(), err.cpu().numpy()


def test_noalloc_matches_batched_two_calls(T):
    rng = np.random.Generator(np.random.PCG64(707))
    # call 1: dense stack of 6 N = 30 Gaussian-state matrices
    mats = [I.gaussian_state_matrix(30, rng) for _ in range(6)]
    A1 = T.as_tensor(np.stack([m[0] for m in mats]), device="cuda")
    g1 = T.as_tensor(np.stack([m[1] for m in mats]), device="cuda")
    off1 = np.arange(7, dtype=np.int64) * 30
    # call 2 (smaller): 3 index lists N = 9, 14, 20 into one shared 100-mode base
    st = I.state100(0)
    A2 = T.as_tensor(st["B"], device="cuda")
    g2 = T.as_tensor(st["gamma"], device="cuda")
    lists = [rng.permutation(100)[:k] for k in (9, 14, 20)]
    idx2 = T.as_tensor(np.concatenate(lists).astype(np.int32), device="cuda")
    off2 = np.array([0, 9, 23, 43], dtype=np.int64)
    for A, g, idx, off in ((A1, g1, None, off1), (A2, g2, idx2, off2)):
        for mode in ("fds", "et"):
            # "ddc": the double-double recurrence kernels, with their larger LDS
            for acc in ("dd", "ddc"):
                s0, want, werr = _call(T, "lhaf_batched", A, g, idx, off, mode, acc)
                s1, got, gerr = _call(T, "lhaf_batched_noalloc", A, g, idx, off, mode, acc)
                print(f"[case] noalloc B={len(off) - 1} {mode} {acc} status {s0} {s1}", flush=True)
                assert s0 == 0 and s1 == 0
                assert np.array_equal(got, want), np.max(np.abs(got - want) / np.abs(want))
                assert np.array_equal(gerr, werr)


def test_noalloc_rejects_oversize_batch(T):
    from paper_2108_01622_amd import _binding as Bn
    L = Bn.lib()
    limit = int(L.lhaf_noalloc_scratch_bytes())
    assert limit == 64 << 20
    # 2048 problems of N = 64 pack 2048 x (64^2 + 64) x 16 B = 136 MB of reduced matrices
    B, N = 2048, 64
    off = np.arange(B + 1, dtype=np.int64) * N
    o = Bn.make_opts("fds")
    need = int(L.lhaf_batched_workspace(B, Bn.host_ptr(off), None, ctypes.byref(o)))
    assert need > limit
    A = T.zeros((N, N), dtype=T.complex128, device="cuda")
    g = T.zeros(N, dtype=T.complex128, device="cuda")
    idx = T.as_tensor(np.tile(np.arange(N, dtype=np.int32), B), device="cuda")
    out = T.full((B,), 7.0 + 0j, dtype=T.complex128, device="cuda")
    st = ctypes.c_void_p(T.cuda.current_stream().cuda_stream)
    status = L.lhaf_batched_noalloc(B, ctypes.c_void_p(A.data_ptr()), N, 0, ctypes.c_void_p(g.data_ptr()),
                                    0, ctypes.c_void_p(idx.data_ptr()), Bn.host_ptr(off), None,
                                    ctypes.c_void_p(out.data_ptr()), None, ctypes.byref(o), st)
    T.cuda.synchronize()
    assert status == 6  # LH_ESCRATCH: nothing queued
    assert b"fixed device scratch" in L.lh_status_string(status)
    assert bool((out == 7.0).all())
