#!/usr/bin/env python
"""Loop-hafnian throughput on one MI355X.

    python bench.py [--steps K] [--warmup W] [--pass fwdbwd|fwd]

A step is one pass of the hot path over one batch of synthetic input: the
256 N=40 Gaussian-state matrices of the differentiation workload (U Haar
40x40, r ~ U[0.5,1.5], gamma ~ CN(0,0.1)), finite-difference-sieve sum with
double-double accumulation, forward (lhaf) and backward (d lhaf/dA,
d lhaf/d gamma).  `value` is lhaf terms of the batch per second of the whole
step (2^19 terms per matrix, each evaluated once forward and once in the
adjoint).  The forward keeps the per-term series coefficients in a store
in HBM (43 GB at this size) that the backward reads (--no-store recomputes
them in the backward).  Inputs are resident in HBM before the timed region.  One extra,
untimed-for-value measurement runs a full N=52 block-diagonal lhaf (the
paper's accuracy protocol) for the N=52 throughput and error.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6


def canonical_flops(m: int, n: int) -> float:
    """Algorithmic FP64 flops of one term: complex Householder Hessenberg
    reduction of the m x m matrix (40/3 m^3) plus n complex mat-vecs for the
    loop moments (8 n m^2)."""
    return 40.0 / 3.0 * m ** 3 + 8.0 * n * m * m


def ps_products(n: int) -> int:
    """Matrix products of the Paterson-Stockmeyer evaluation of a degree n-1
    polynomial: s = ceil(sqrt n) powers, ceil(n/s) - 1 Horner steps."""
    s = 1
    while s * s < n:
        s += 1
    return (s - 1) + (n + s - 1) // s - 1


def canonical_flops_bwd(m: int, n: int, store: bool) -> float:
    """Algorithmic FP64 flops of one adjoint term: the Paterson-Stockmeyer
    products of P(W) (8 m^3 each), the Krylov sequence, the rank-one terms and
    the two power-sum contractions (24 n m^2), plus the forward's spectral
    work when the per-term coefficients are recomputed instead of read."""
    return (0.0 if store else canonical_flops(m, n)) + 8.0 * m ** 3 * ps_products(n) + 24.0 * n * m * m


def cpu_baseline(A, g, budget_s: float = 12.0):
    """The oracle (explicit matrix powers, OpenMP over term ranges) on a
    bounded sample of the same workload: the first S terms of matrix 0."""
    from oracle import oracle as O
    threads = os.cpu_count() or 1
    O.set_threads(threads)
    t = time.perf_counter()
    probe = 8 * threads
    O.lhaf_sum(A, g, mode="fds", t0=0, t1=probe, scaled=False)
    dt = time.perf_counter() - t
    S = int(max(probe, min(2 ** 19, probe * budget_s / max(dt, 1e-6))))
    t = time.perf_counter()
    O.lhaf_sum(A, g, mode="fds", t0=0, t1=S, scaled=False)
    dt = time.perf_counter() - t
    return dict(value=S / dt, unit="terms/s", cores=O.get_threads(), kind="oracle",
                sample=f"FDS terms [0,{S}) of matrix 0 of the N=40 batch (explicit matrix powers, "
                       f"double + Neumaier), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="grad40")
    ap.add_argument("--pass", dest="passes", default="fwdbwd", choices=["fwd", "fwdbwd"])
    ap.add_argument("--no-n52", action="store_true")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="run one plain device copy of this size before timing (a known-size "
                         "reference for memory-traffic counters)")
    ap.add_argument("--sum", default="fds", choices=["fds", "et"])
    ap.add_argument("--acc", default="dd", choices=["dd", "fp64"])
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-chain", action="store_true",
                    help="skip the 4096-problem chain-rule forward (N = 20..40 submatrices)")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the multi-output measurements (sub-detector and chain-rule batching)")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the forward precision-mode table (ET/FDS x FP64/DD)")
    ap.add_argument("--no-store", action="store_true",
                    help="recompute the per-term coefficients in the backward instead of keeping "
                         "the forward's coefficient store")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (across GPUs "
                                   "the term sum shards by term ranges: each GPU evaluates its "
                                   "term_begin/term_end share unscaled and the partial sums are added)"}))
        sys.exit(2)

    import torch
    from paper_2108_01622_amd import api, inputs
    from paper_2108_01622_amd import _binding
    from paper_2108_01622_amd.profiling import stored_traffic

    dev = torch.device("cuda", 0)
    A_np, g_np = inputs.grad40(count=args.batch)
    N = A_np.shape[1]
    n, m = N // 2, N
    A = torch.as_tensor(A_np, device=dev)
    g = torch.as_tensor(g_np, device=dev)
    terms_per_problem = _binding.term_count(N, sum=args.sum)
    terms = args.batch * terms_per_problem
    stream = torch.cuda.current_stream(dev)

    if args.copy_ref_mib > 0:
        src = torch.ones(args.copy_ref_mib * (1 << 17), dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    fwd_ms, bwd_ms = [], []
    out = None
    # workspaces allocated once, outside the timed region
    off = np.arange(args.batch + 1, dtype=np.int64) * N
    ws_fwd = torch.empty(api.lhaf_batched_workspace(off, sum=args.sum, acc=args.acc),
                         dtype=torch.uint8, device=dev)
    ws_bwd = None
    store = None
    ones = torch.ones(args.batch, dtype=torch.complex128, device=dev)
    if args.passes == "fwdbwd" and not args.no_store:
        store = torch.empty(api.lhaf_saved_count(off, sum=args.sum), dtype=torch.complex128,
                            device=dev)
    if args.passes == "fwdbwd":
        nb = int(_binding.lib().lhaf_backward_workspace(args.batch, _binding.host_ptr(off), None, N,
                                                         ctypes.byref(_binding.make_opts(args.sum, args.acc))))
        ws_bwd = torch.empty(nb, dtype=torch.uint8, device=dev)

    def step(timed: bool):
        nonlocal out
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = api.lhaf_batched(A, g, sum=args.sum, acc=args.acc, workspace=ws_fwd, saved=store)
        e1.record(stream)
        if args.passes == "fwdbwd":
            e2 = torch.cuda.Event(enable_timing=True)
            e2.record(stream)
            api.lhaf_backward(A, g, ones, sum=args.sum, acc=args.acc, workspace=ws_bwd, saved=store)
            e3 = torch.cuda.Event(enable_timing=True)
            e3.record(stream)
        if timed:
            torch.cuda.synchronize()
            fwd_ms.append(e0.elapsed_time(e1))
            if args.passes == "fwdbwd":
                bwd_ms.append(e2.elapsed_time(e3))

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    passes = 2 if args.passes == "fwdbwd" else 1
    value = terms * args.steps / elapsed
    fwd_s = np.mean(fwd_ms) / 1e3
    fwd_tf = canonical_flops(m, n) * terms / fwd_s / 1e12
    if bwd_ms:
        bwd_s = np.mean(bwd_ms) / 1e3
        bwd_flops = canonical_flops_bwd(m, n, store is not None)
        bwd_tf = bwd_flops * terms / bwd_s / 1e12
        dom = {"bound": "alu", "kernel": "backward_kernel<5>", "achieved": bwd_tf,
               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": bwd_tf / FP64_PEAK_TFLOPS,
               "traffic": stored_traffic("backward_kernel<5>", terms), "per_term_flops": bwd_flops,
               "terms_per_launch": terms, "launch_ms": bwd_s * 1e3}
    else:
        dom = {"bound": "alu", "kernel": "forward_kernel<5>", "achieved": fwd_tf,
               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": fwd_tf / FP64_PEAK_TFLOPS,
               "traffic": stored_traffic("forward_kernel<5>", terms), "per_term_flops": canonical_flops(m, n),
               "terms_per_launch": terms, "launch_ms": fwd_s * 1e3}
    res = {
        "metric": "lhaf terms/sec (N=40, FDS, double-double; " +
                  ("forward + backward" if passes == 2 else "forward") + ")",
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian-state matrices)",
        "config": {"workload": f"grad40: {args.batch} x lhaf N={N} complex128, {args.sum.upper()} "
                               f"{args.acc} accumulation, " + ("fwd+bwd" if passes == 2 else "fwd"),
                   "global_batch": args.batch, "N": N, "terms_per_lhaf": terms_per_problem,
                   "sum": args.sum, "acc": args.acc,
                   "backward_coefficients": "forward store" if store is not None else "recomputed"},
        "roofline": dom,
        "lhafs_per_s": args.batch * args.steps / elapsed,
        "time_to_solution_s": elapsed / args.steps,
        "forward": {"kernel": "forward_kernel<5>", "terms_per_s": terms / fwd_s, "tflops": fwd_tf,
                    "frac": fwd_tf / FP64_PEAK_TFLOPS, "launch_ms": fwd_s * 1e3,
                    "per_term_flops": canonical_flops(m, n)},
    }
    if bwd_ms:
        res["backward"] = {"kernel": "backward_kernel<5>", "terms_per_s": terms / bwd_s,
                           "tflops": bwd_tf, "frac": bwd_tf / FP64_PEAK_TFLOPS,
                           "launch_ms": bwd_s * 1e3, "per_term_flops": bwd_flops,
                           "coefficient_store": store is not None,
                           "store_bytes": 0 if store is None else store.numel() * 16}
    # relative error against stored oracle values (tests/golden, oracle-only)
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    if os.path.exists(gold_path) and args.sum == "fds":
        gold = json.load(open(gold_path))
        o = out.cpu().numpy()
        errs = []
        for key, ent in gold.items():
            if key.startswith("grad40/") and key.count("/") == 1:
                b = int(key.split("/")[1])
                if b < args.batch:
                    ref = complex(*ent["value"])
                    errs.append(abs(o[b] - ref) / abs(ref))
        if errs:
            res["rel_err_vs_oracle"] = {"max": max(errs), "count": len(errs),
                                        "oracle": "FDS double, explicit matrix powers"}
    if not args.no_n52:
        # N = 52 forward: one full block-diagonal lhaf (2^25 terms, tile B = 7)
        A52, g52, _, _ = inputs.block_diagonal_stress(52, 0)
        a52 = torch.as_tensor(A52, device=dev)
        q52 = torch.as_tensor(g52, device=dev)
        api.lhaf(a52, q52)  # warm
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        v52 = api.lhaf(a52, q52)
        e1.record(stream)
        torch.cuda.synchronize()
        t52 = e0.elapsed_time(e1) / 1e3
        T52 = _binding.term_count(52)
        tf52 = canonical_flops(52, 26) * T52 / t52 / 1e12
        ent = {"workload": "block52/0 (A1 (+) A2, N=52, FDS dd)", "terms_per_s": T52 / t52,
               "tflops": tf52, "frac": tf52 / FP64_PEAK_TFLOPS, "seconds": t52}
        if os.path.exists(gold_path):
            gold = json.load(open(gold_path))
            if "block52/0" in gold:
                ref = complex(*gold["block52/0"]["value"])
                ent["rel_err_vs_oracle"] = abs(v52.item() - ref) / abs(ref)
                ent["oracle"] = "__float128 FDS of both halves, multiplied"
        res["n52_forward"] = ent
        print("[bench] N=52 done", file=sys.stderr, flush=True)
    if not args.no_modes:
        # forward precision modes on the first 8 matrices of the batch
        A8, g8 = A[:8], g[:8]
        modes = {}
        for sm in ("fds", "et"):
            for am in ("dd", "fp64"):
                api.lhaf_batched(A8, g8, sum=sm, acc=am)
                torch.cuda.synchronize()
                t = time.perf_counter()
                api.lhaf_batched(A8, g8, sum=sm, acc=am)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                T8 = 8 * _binding.term_count(N, sum=sm)
                modes[f"{sm}/{am}"] = {"terms_per_s": T8 / dt, "lhafs_per_s": 8 / dt,
                                       "frac": canonical_flops(m, n) * T8 / dt / 1e12 / FP64_PEAK_TFLOPS}
        res["forward_modes_n40"] = modes
        print("[bench] precision modes done", file=sys.stderr, flush=True)
    if not args.no_chain:
        # chain-rule batch: 4096 submatrices N = 20..40 of the 100-mode state, one launch
        ch = inputs.chain4096()
        Bc = torch.as_tensor(ch["B"], device=dev)
        gc = torch.as_tensor(ch["gamma"], device=dev)
        api.lhaf_batched(Bc, gc, idx=ch["idx"][:ch["idx_off"][64]], idx_off=ch["idx_off"][:65])
        torch.cuda.synchronize()
        t = time.perf_counter()
        api.lhaf_batched(Bc, gc, idx=ch["idx"], idx_off=ch["idx_off"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        Tc = sum(_binding.term_count(int(k)) for k in ch["sizes"])
        fl = sum(_binding.term_count(int(k)) * canonical_flops(int(k), int(k) // 2) for k in ch["sizes"])
        res["chain4096_forward"] = {"workload": "4096 submatrices N=20..40 (even) of the 100-mode state, "
                                                "FDS dd, one persistent launch",
                                    "terms": Tc, "seconds": dt, "terms_per_s": Tc / dt,
                                    "lhafs_per_s": 4096 / dt, "tflops": fl / dt / 1e12,
                                    "frac": fl / dt / 1e12 / FP64_PEAK_TFLOPS}
        print("[bench] chain4096 done", file=sys.stderr, flush=True)
    if not args.no_multi:
        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            return time.perf_counter() - t
        # sub-detector batching: 12 loop-weight vectors of one N = 40 matrix
        rng = np.random.Generator(np.random.PCG64(4040))
        gs = g_np[0][None, :] + 0.05 * (rng.normal(size=(12, N)) + 1j * rng.normal(size=(12, N)))
        gst = torch.as_tensor(gs, device=dev)
        A12 = A[:1].expand(12, N, N).contiguous()
        t_one = timed(lambda: api.lhaf_gammas(A[0], gst))
        t_sep = timed(lambda: api.lhaf_batched(A12, gst))
        res["gamma_batch_n40"] = {"workload": "one N=40 grad40 matrix, 12 loop-weight vectors, FDS dd",
                                  "seconds": t_one, "separate_seconds": t_sep,
                                  "speedup": t_sep / t_one,
                                  "output_terms_per_s": 12 * terms_per_problem / t_one}
        # chain-rule step: the 100-mode state's 40-photon pattern fixed, one
        # empty mode batched up to 8 photons (9 outputs, ET)
        st = inputs.state100(0)
        rfix = st["r"].astype(np.int32).copy()
        b = int(np.nonzero(rfix == 0)[0][0])
        Bt = torch.as_tensor(st["B"], device=dev)
        gt = torch.as_tensor(st["gamma"], device=dev)
        t_chain = timed(lambda: api.lhaf_chain(Bt, gt, rfix, b, 8))
        def separate():
            for k in range(9):
                rk = rfix.copy()
                rk[b] = k
                api.lhaf(Bt, gt, r=rk, sum="et")
        t_sep = timed(separate)
        res["chain_step_state100"] = {"workload": "state100 pattern (40 photons, 28 modes) fixed, "
                                                  "one empty mode batched k = 0..8, ET dd",
                                      "seconds": t_chain, "separate_seconds": t_sep,
                                      "speedup": t_sep / t_chain}
        # mixed-state lhafmix (App. B.2): 2M x 2M with M = 20, N = 2 sum(n) <= 40
        Am, gm, nm = inputs.mixed_state(20, 0)
        while 2 * nm.sum() > 40:
            nm[np.argmax(nm)] -= 1
        Amt = torch.as_tensor(Am, device=dev)
        gmt = torch.as_tensor(gm, device=dev)
        t_mix = timed(lambda: api.lhaf_mixed(Amt, gmt, nm))
        Tm = int(np.prod(nm[nm > 0] + 1))
        Tm = Tm // 2 if np.any(nm % 2) else Tm // 2 + 1  # FDS halving (first odd pair, else pair 0)
        t_greedy = timed(lambda: api.lhaf(Amt, gmt, r=np.concatenate([nm, nm])))
        res["mixed_state_m20"] = {"workload": f"lhafmix, 2M x 2M with M = 20, n = {nm.tolist()}, "
                                              f"N = {2 * int(nm.sum())}, FDS dd",
                                  "seconds": t_mix, "greedy_repeated_seconds": t_greedy,
                                  "terms": Tm,
                                  "terms_per_s": Tm / t_mix}
        # real non-negative N = 40 lhaf (real FP64 kernel) against the complex
        # kernels on the same entries
        rng = np.random.Generator(np.random.PCG64(4041))
        Ar = rng.uniform(0.0, 0.2, size=(N, N))
        Ar = 0.5 * (Ar + Ar.T)
        gr = rng.uniform(0.0, 1.0, size=N)
        Art, grt = torch.as_tensor(Ar, device=dev), torch.as_tensor(gr, device=dev)
        t_real = timed(lambda: api.lhaf_real(Art, grt))
        t_cplx = timed(lambda: api.lhaf(Art.to(torch.complex128), grt.to(torch.complex128)))
        res["real_nonneg_n40"] = {"workload": "one real non-negative N=40 lhaf, FDS dd",
                                  "seconds": t_real, "complex_kernel_seconds": t_cplx,
                                  "terms_per_s": terms_per_problem / t_real,
                                  "speedup_vs_complex": t_cplx / t_real}
        print("[bench] multi-output done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(A_np[0], g_np[0])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
