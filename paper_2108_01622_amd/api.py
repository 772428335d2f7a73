"""PyTorch-facing wrappers of the C ABI (same names as include/lhaf.h).

Tensors must be complex128 on a ROCm device; results are complex128 device
tensors.  Work is queued on torch's current HIP stream.  The functions only
marshal arguments: planning, the term sums and every reduction run in the
HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _binding as Bn


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_c128(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a ROCm device (got {t.device})")
    if t.dtype != torch.complex128:
        t = t.to(torch.complex128)
    return t.contiguous()


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def lhaf(A: torch.Tensor, gamma: torch.Tensor | None = None, r=None, *, sum: str = "fds",
         acc: str = "dd", term_begin: int = 0, term_end: int = -1, scaled: bool = True,
         schedule: int = -1, return_error: bool = False, return_lo: bool = False,
         workspace: torch.Tensor | None = None):
    """Loop hafnian of one matrix.  gamma=None takes gamma = diag(A).  With r
    (host integer multiplicities) this is lhaf_repeated: lhaf(A_r, gamma_r).
    acc: "dd" double-double accumulation of the signed sum (default), "fp64"
    plain, "ddc" double-double accumulation and each term's characteristic
    polynomial and series recurrences in double-double (ill-conditioned sums;
    values only, not with gradients)."""
    A = _dev_c128(A, "A")
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    N = A.shape[0]
    gamma = torch.diagonal(A).contiguous() if gamma is None else _dev_c128(gamma, "gamma")
    out = torch.empty((), dtype=torch.complex128, device=A.device)
    err = torch.empty((), dtype=torch.float64, device=A.device)
    lo = torch.zeros((), dtype=torch.complex128, device=A.device) if return_lo else None
    o = Bn.make_opts(sum, acc, term_begin, term_end, scaled, schedule, workspace, lo)
    with torch.cuda.device(A.device):
        st = _stream_ptr(A.device)
        if r is None:
            Bn.check(Bn.lib().lhaf(_p(A), N, _p(gamma), N, _p(out), _p(err), ctypes.byref(o), st))
        else:
            rr = np.ascontiguousarray(np.asarray(r), dtype=np.int32)
            if len(rr) != N:
                raise ValueError("r must have one entry per row of A")
            Bn.check(Bn.lib().lhaf_repeated(_p(A), N, _p(gamma), Bn.host_ptr(rr), N, _p(out),
                                            _p(err), ctypes.byref(o), st))
    res = [out]
    if return_error:
        res.append(err)
    if return_lo:
        res.append(lo)
    return res[0] if len(res) == 1 else tuple(res)


def lhaf_repeated(A, gamma, r, **kw):
    return lhaf(A, gamma, r, **kw)


def _batch_args(A, gamma, idx, idx_off, r):
    A = _dev_c128(A, "A")
    gamma = _dev_c128(gamma, "gamma")
    if A.dim() == 3:  # dense stack: problem b = A[b], identity indices
        Bsz, N, N2 = A.shape
        if N != N2 or gamma.shape != (Bsz, N):
            raise ValueError("dense batch needs A (B,N,N) and gamma (B,N)")
        lda, sA, sg = N, N * N, N
        off = np.arange(Bsz + 1, dtype=np.int64) * N if idx_off is None else np.asarray(idx_off, np.int64)
        idx_t = None if idx is None else _idx_tensor(idx, A.device)
    else:
        if idx_off is None:
            raise ValueError("a shared base matrix needs idx_off")
        Bsz = len(idx_off) - 1
        lda, sA, sg = A.shape[1], 0, 0
        off = np.ascontiguousarray(idx_off, dtype=np.int64)
        idx_t = None if idx is None else _idx_tensor(idx, A.device)
    rr = None if r is None else np.ascontiguousarray(np.asarray(r), dtype=np.int32)
    return A, gamma, Bsz, lda, sA, sg, off, idx_t, rr


def _idx_tensor(idx, device):
    if isinstance(idx, torch.Tensor):
        return idx.to(device=device, dtype=torch.int32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32), device=device)


def lhaf_batched_workspace(idx_off, r=None, **kw) -> int:
    off = np.ascontiguousarray(idx_off, dtype=np.int64)
    rr = None if r is None else np.ascontiguousarray(r, dtype=np.int32)
    o = Bn.make_opts(kw.get("sum", "fds"), kw.get("acc", "dd"), kw.get("term_begin", 0),
                     kw.get("term_end", -1), kw.get("scaled", True), kw.get("schedule", -1))
    return int(Bn.lib().lhaf_batched_workspace(len(off) - 1, Bn.host_ptr(off), Bn.host_ptr(rr),
                                               ctypes.byref(o)))


def lhaf_real(A, gamma=None, r=None, *, sum="fds", acc="dd", term_begin=0, term_end=-1,
              scaled=True, schedule=-1, return_error=False, workspace=None):
    """Loop hafnian of a real symmetric matrix with real loop weights, in real
    FP64 (float64 device tensors; gamma=None takes diag(A))."""
    if not isinstance(A, torch.Tensor) or A.device.type != "cuda":
        raise ValueError("A must be a ROCm device tensor")
    A = A.to(torch.float64).contiguous()
    M = A.shape[0]
    if A.dim() != 2 or A.shape[1] != M:
        raise ValueError("A must be square")
    gamma = torch.diagonal(A).contiguous() if gamma is None else gamma.to(torch.float64).contiguous()
    out = torch.empty((), dtype=torch.float64, device=A.device)
    err = torch.empty((), dtype=torch.float64, device=A.device)
    rr = None if r is None else np.ascontiguousarray(np.asarray(r), dtype=np.int32)
    o = Bn.make_opts(sum, acc, term_begin, term_end, scaled, schedule, workspace)
    with torch.cuda.device(A.device):
        Bn.check(Bn.lib().lhaf_real(_p(A), M, _p(gamma), Bn.host_ptr(rr), M, _p(out), _p(err),
                                    ctypes.byref(o), _stream_ptr(A.device)))
    return (out, err) if return_error else out


def lhaf_mixed(A, gamma, n, *, sum="fds", acc="dd", term_begin=0, term_end=-1, scaled=True,
               schedule=-1, return_error=False, workspace=None):
    """Mixed-state lhafmix(A, gamma, n): A (2M, 2M), gamma (2M,), n host photon
    numbers (M,); row i paired with row M+i, n_i times."""
    A = _dev_c128(A, "A")
    gamma = _dev_c128(gamma, "gamma")
    nn = np.ascontiguousarray(np.asarray(n), dtype=np.int32)
    M = len(nn)
    if A.dim() != 2 or A.shape != (2 * M, 2 * M) or gamma.shape != (2 * M,):
        raise ValueError("A (2M,2M) and gamma (2M,) required for M photon numbers")
    out = torch.empty((), dtype=torch.complex128, device=A.device)
    err = torch.empty((), dtype=torch.float64, device=A.device)
    o = Bn.make_opts(sum, acc, term_begin, term_end, scaled, schedule, workspace)
    with torch.cuda.device(A.device):
        Bn.check(Bn.lib().lhaf_mixed(_p(A), 2 * M, _p(gamma), Bn.host_ptr(nn), M, _p(out), _p(err),
                                     ctypes.byref(o), _stream_ptr(A.device)))
    return (out, err) if return_error else out


def lhaf_chain(A, gamma, r, mode_b: int, n_cut: int, *, acc="dd", schedule=-1,
               return_error=False, workspace=None):
    """One chain-rule step: out[k] = lhaf of the pattern r with mode_b at k
    photons, k = 0..n_cut (ET sum; one pass serves every k).  r: host ints,
    one per row of A, r[mode_b] = 0."""
    A = _dev_c128(A, "A")
    gamma = _dev_c128(gamma, "gamma")
    M = A.shape[0]
    rr = np.ascontiguousarray(np.asarray(r), dtype=np.int32)
    if A.dim() != 2 or A.shape[1] != M or gamma.shape != (M,) or len(rr) != M:
        raise ValueError("A (M,M), gamma (M,) and r (M,) required")
    out = torch.empty(n_cut + 1, dtype=torch.complex128, device=A.device)
    err = torch.empty(n_cut + 1, dtype=torch.float64, device=A.device)
    o = Bn.make_opts("et", acc, 0, -1, True, schedule, workspace)
    with torch.cuda.device(A.device):
        Bn.check(Bn.lib().lhaf_chain(_p(A), M, _p(gamma), Bn.host_ptr(rr), M, int(mode_b),
                                     int(n_cut), _p(out), _p(err), ctypes.byref(o),
                                     _stream_ptr(A.device)))
    return (out, err) if return_error else out


def lhaf_gammas(A, gammas, r=None, *, sum="fds", acc="dd", schedule=-1, return_error=False,
                workspace=None):
    """Sub-detector batching: out[g] = lhaf(A_r, gammas[g]) for G <= 64 loop
    weight vectors (gammas (G, M)) of one matrix, one pass over the terms."""
    A = _dev_c128(A, "A")
    gammas = _dev_c128(gammas, "gammas")
    M = A.shape[0]
    if A.dim() != 2 or A.shape[1] != M or gammas.dim() != 2 or gammas.shape[1] != M:
        raise ValueError("A (M,M) and gammas (G,M) required")
    G = gammas.shape[0]
    rr = None if r is None else np.ascontiguousarray(np.asarray(r), dtype=np.int32)
    if rr is not None and len(rr) != M:
        raise ValueError("r must have one entry per row of A")
    out = torch.empty(G, dtype=torch.complex128, device=A.device)
    err = torch.empty(G, dtype=torch.float64, device=A.device)
    o = Bn.make_opts(sum, acc, 0, -1, True, schedule, workspace)
    with torch.cuda.device(A.device):
        Bn.check(Bn.lib().lhaf_gammas(_p(A), M, _p(gammas), M, Bn.host_ptr(rr), M, G, _p(out),
                                      _p(err), ctypes.byref(o), _stream_ptr(A.device)))
    return (out, err) if return_error else out


def lhaf_saved_count(idx_off, r=None, sum="fds", term_begin=0, term_end=-1) -> int:
    """Entries of the per-term coefficient store of a batch (complex128) over
    the term range [term_begin, term_end) of every problem."""
    off = np.ascontiguousarray(idx_off, dtype=np.int64)
    rr = None if r is None else np.ascontiguousarray(r, dtype=np.int32)
    o = Bn.make_opts(sum, term_begin=term_begin, term_end=term_end)
    v = int(Bn.lib().lhaf_saved_count(len(off) - 1, Bn.host_ptr(off), Bn.host_ptr(rr),
                                      ctypes.byref(o)))
    if v < 0:
        Bn.check(-v)
    return v


def _saved_tensor(saved, device):
    if saved is None:
        return None
    if saved.dtype != torch.complex128 or saved.device != device or not saved.is_contiguous():
        raise ValueError("saved / grads must be a contiguous complex128 tensor on the problems' "
                         "device")
    return saved


def lhaf_grads_count(idx_off, r=None) -> int:
    """Entries of the per-problem reduced-gradient buffer (complex128) of a
    batch, for the fused pass (lhaf_batched(..., grads=...))."""
    off = np.ascontiguousarray(idx_off, dtype=np.int64)
    rr = None if r is None else np.ascontiguousarray(r, dtype=np.int32)
    v = int(Bn.lib().lhaf_grads_count(len(off) - 1, Bn.host_ptr(off), Bn.host_ptr(rr)))
    if v < 0:
        Bn.check(-v)
    return v


def lhaf_batched(A, gamma, idx=None, idx_off=None, r=None, *, sum="fds", acc="dd",
                 term_begin=0, term_end=-1, scaled=True, schedule=-1, return_error=False,
                 return_lo=False, workspace=None, saved=None, grads=None):
    """Many loop hafnians in one persistent launch.  Either a dense stack
    A (B,N,N), gamma (B,N), or a shared base A (M,M), gamma (M) with index
    lists idx[idx_off[b]:idx_off[b+1]] (r: optional multiplicities packed like
    idx).  saved: optional complex128 tensor of lhaf_saved_count(...) entries
    that receives the per-term coefficients for lhaf_backward.  grads:
    optional complex128 tensor of lhaf_grads_count(...) entries: the fused
    pass, which also leaves each problem's gradient there for
    lhaf_backward(..., grads=...)."""
    A, gamma, Bsz, lda, sA, sg, off, idx_t, rr = _batch_args(A, gamma, idx, idx_off, r)
    out = torch.empty(Bsz, dtype=torch.complex128, device=A.device)
    err = torch.empty(Bsz, dtype=torch.float64, device=A.device)
    lo = torch.zeros(Bsz, dtype=torch.complex128, device=A.device) if return_lo else None
    o = Bn.make_opts(sum, acc, term_begin, term_end, scaled, schedule, None, lo,
                     _saved_tensor(saved, A.device), _saved_tensor(grads, A.device))
    need = int(Bn.lib().lhaf_batched_workspace(Bsz, Bn.host_ptr(off), Bn.host_ptr(rr), ctypes.byref(o)))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    with torch.cuda.device(A.device):
        Bn.check(Bn.lib().lhaf_batched(Bsz, _p(A), lda, sA, _p(gamma), sg, _p(idx_t),
                                       Bn.host_ptr(off), Bn.host_ptr(rr), _p(out), _p(err),
                                       _p(workspace), workspace.numel(), ctypes.byref(o),
                                       _stream_ptr(A.device)))
    res = [out]
    if return_error:
        res.append(err)
    if return_lo:
        res.append(lo)
    return res[0] if len(res) == 1 else tuple(res)


def lhaf_backward(A, gamma, grad_out, idx=None, idx_off=None, r=None, *, sum="fds",
                  acc="dd", term_begin=0, term_end=-1, schedule=-1, workspace=None, saved=None,
                  grads=None):
    """Gradients (dA, dgamma) of the batch in PyTorch's complex convention:
    grad_out * conj(d lhaf / d input).  With a term range, the share of the
    gradient from those terms of every problem (disjoint ranges add up).
    saved: the coefficient store written by lhaf_batched on the same batch,
    sum and term range (skips the Hessenberg phase).  grads: the gradients a
    fused lhaf_batched(..., grads=...) pass left (skips the term pass)."""
    A, gamma, Bsz, lda, sA, sg, off, idx_t, rr = _batch_args(A, gamma, idx, idx_off, r)
    grad_out = _dev_c128(grad_out, "grad_out").reshape(-1)
    if grad_out.numel() != Bsz:
        raise ValueError("grad_out needs one value per problem")
    base_dim = A.shape[-1]
    dA = torch.empty_like(A)
    dg = torch.empty_like(gamma)
    o = Bn.make_opts(sum, acc, term_begin, term_end, True, schedule,
                     saved=_saved_tensor(saved, A.device), grads=_saved_tensor(grads, A.device))
    need = int(Bn.lib().lhaf_backward_workspace(Bsz, Bn.host_ptr(off), Bn.host_ptr(rr), base_dim,
                                                ctypes.byref(o)))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    with torch.cuda.device(A.device):
        Bn.check(Bn.lib().lhaf_backward(Bsz, _p(A), lda, sA, _p(gamma), sg, _p(idx_t),
                                        Bn.host_ptr(off), Bn.host_ptr(rr), _p(grad_out), _p(dA),
                                        _p(dg), base_dim, _p(workspace), workspace.numel(),
                                        ctypes.byref(o), _stream_ptr(A.device)))
    return dA, dg


def _store_fits(count: int, device, fraction: float) -> bool:
    """Whether a coefficient store of `count` entries fits in the given
    fraction of the device's free memory."""
    free, _ = torch.cuda.mem_get_info(device)
    return count * 16 <= fraction * free


class LhafFunction(torch.autograd.Function):
    """lhaf of a dense batch (A (B,N,N), gamma (B,N)) with the adjoint kernels
    as backward.  Modes when gradients are needed:
      "fused" (default): the forward runs the fused pass -- every term's value
        and adjoint in one launch -- and keeps only each problem's reduced
        gradient (LD^2 + 64 complex per problem); the backward maps it to
        dA, dgamma with grad_out.
      "recompute": plain forward; the backward repeats every term's spectral
        work (nothing kept between the passes but A, gamma).
      "store": the forward keeps every term's series coefficients (16 n bytes
        per term) when they fit in store_fraction of free device memory, and
        the backward reads them (else it recomputes)."""

    @staticmethod
    def forward(ctx, A, gamma, sum="fds", acc="dd", r=None, mode="fused", store_fraction=0.5):
        saved = grads = None
        need_grad = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        off = np.arange(A.shape[0] + 1, dtype=np.int64) * A.shape[1]
        rr = None if r is None else np.asarray(r, dtype=np.int32).reshape(-1)
        if need_grad and mode == "fused":
            grads = torch.empty(lhaf_grads_count(off, rr), dtype=torch.complex128, device=A.device)
        elif need_grad and mode == "store":
            count = lhaf_saved_count(off, rr, sum)
            if count > 0 and _store_fits(count, A.device, store_fraction):
                saved = torch.empty(count, dtype=torch.complex128, device=A.device)
        elif mode not in ("fused", "recompute", "store"):
            raise ValueError(f"unknown mode {mode!r}")
        ctx.save_for_backward(A, gamma)
        ctx.store, ctx.grads = saved, grads
        ctx.opts = (sum, acc, r)
        return lhaf_batched(A, gamma, r=r, sum=sum, acc=acc, saved=saved, grads=grads)

    @staticmethod
    def backward(ctx, grad_out):
        A, gamma = ctx.saved_tensors
        sum, acc, r = ctx.opts
        # the buffers stay with the graph (a retained graph's second backward
        # must give the same bits)
        dA, dg = lhaf_backward(A, gamma, grad_out.contiguous(), r=r, sum=sum, acc=acc,
                               saved=ctx.store, grads=ctx.grads)
        return dA, dg, None, None, None, None, None


def lhaf_autograd(A, gamma, sum="fds", acc="dd", r=None, mode="fused", store_fraction=0.5):
    """Differentiable lhaf of one matrix (A (N,N)) or a dense batch (A (B,N,N));
    mode "fused" (default), "recompute" or "store" (see LhafFunction)."""
    squeeze = A.dim() == 2
    if squeeze:
        A, gamma = A.unsqueeze(0), gamma.unsqueeze(0)
    out = LhafFunction.apply(A, gamma, sum, acc, r, mode, store_fraction)
    return out[0] if squeeze else out
