#!/usr/bin/env python
"""Loop-hafnian throughput on one MI355X.

    python bench.py [--steps K] [--warmup W] [--budget-s S] [--mode fused|recompute|store]

Workload (differentiation workload): 256 Gaussian-state matrices N = 40
(U Haar 40x40, r ~ U[0.5,1.5], gamma ~ CN(0,0.1)), finite-difference-sieve
sum, double-double accumulation, values (lhaf) and gradients (d lhaf/dA,
d lhaf/d gamma).  Each matrix has 2^19 terms.  A step is one pass of the hot
path over one contiguous term slice of every matrix: terms
[s 2^14, (s+1) 2^14) of all 256 matrices, s = step mod 32 (each term is
independent, so a slice is a full-size share of the work at full m; 32
consecutive steps cover every term).  Modes:
  fused (default): one persistent launch evaluates every term's value and
    adjoint (the spectral work of a term done once, nothing stored per
    term), then the per-problem gradients are mapped to dA, dgamma;
  recompute: a forward launch, then a backward launch that repeats every
    term's spectral work;
  store: the forward keeps every term's series coefficients (16 n bytes per
    term), the backward reads them.
`value` is terms of the step (256 x 2^14) per second of the whole step.
Inputs are resident in HBM before the timed region.

After the timed steps, secondary measurements run while a wall-clock budget
(--budget-s, counted from the end of the timed steps) lasts, each skipped
with a note once it is spent: the stored oracle error of the batch, the CPU
oracle on a bounded sample, the other two modes, N = 52 values + gradients
on a term slice, the N = 16 latency, the forward precision modes, the full
N = 52 block-diagonal lhaf against its __float128 reference, the
multi-output kernels and the 4096-problem chain batch.  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6


def canonical_flops(m: int, n: int) -> float:
    """Algorithmic FP64 flops of one forward term: complex Householder
    Hessenberg reduction of the m x m matrix (40/3 m^3) plus n complex
    mat-vecs for the loop moments (8 n m^2)."""
    return 40.0 / 3.0 * m ** 3 + 8.0 * n * m * m


def canonical_flops_bwd(m: int, n: int, store: bool) -> float:
    """Algorithmic FP64 flops of one adjoint term: about 2 sqrt(n) dense
    m x m complex products for the matrix polynomial (8 m^3 each,
    ceil(2 sqrt n) of them), the Krylov sequence, rank-one terms and
    power-sum contractions (24 n m^2), plus the forward's spectral work when
    the per-term coefficients are recomputed instead of read."""
    return (0.0 if store else canonical_flops(m, n)) + 8.0 * m ** 3 * math.ceil(2 * math.sqrt(n)) \
        + 24.0 * n * m * m


def et_flops_per_lhaf(N: int) -> float:
    """Algorithmic FP64 flops of a plain ET lhaf with pair deletion: a term
    keeping k of the n = N/2 pairs works at m = 2k, so the sum is
    sum_k C(n, k) F(2k, n)."""
    n = N // 2
    return float(sum(math.comb(n, k) * canonical_flops(2 * k, n) for k in range(1, n + 1)))


def ps_products(n: int) -> int:
    """Matrix products the kernel executes for the degree n-1 polynomial:
    Paterson-Stockmeyer with s = ceil(sqrt n) powers and ceil(n/s) - 1 Horner
    steps."""
    s = 1
    while s * s < n:
        s += 1
    return (s - 1) + (n + s - 1) // s - 1


def cpu_baseline(A, g, budget_s: float):
    """The oracle (explicit matrix powers, OpenMP over term ranges) on a
    bounded sample of the same workload: the first S terms of matrix 0, on
    all host cores and on one thread."""
    from oracle import oracle as O
    res = {}
    for label, threads in (("all", os.cpu_count() or 1), ("one", 1)):
        O.set_threads(threads)
        probe = 8 * threads
        t = time.perf_counter()
        O.lhaf_sum(A, g, mode="fds", t0=0, t1=probe, scaled=False)
        dt = time.perf_counter() - t
        S = int(max(probe, min(2 ** 19, probe * budget_s / max(dt, 1e-6))))
        t = time.perf_counter()
        O.lhaf_sum(A, g, mode="fds", t0=0, t1=S, scaled=False)
        dt = time.perf_counter() - t
        res[label] = dict(value=S / dt, cores=O.get_threads(), terms=S, seconds=dt)
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    a = res["all"]
    return dict(value=a["value"], unit="terms/s", cores=a["cores"], kind="oracle",
                sample=f"FDS terms [0,{a['terms']}) of matrix 0 of the N=40 batch (explicit matrix "
                       f"powers, double + Neumaier), {a['seconds']:.1f} s on {a['cores']} threads",
                single_thread={"value": res["one"]["value"], "cores": 1,
                               "sample": f"FDS terms [0,{res['one']['terms']}) of the same matrix, "
                                         f"{res['one']['seconds']:.1f} s"},
                cpu_model=cpu, nproc=os.cpu_count())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--slice-log2", type=int, default=14,
                    help="terms per matrix per step = 2^slice_log2 (of 2^19)")
    ap.add_argument("--sum", default="fds", choices=["fds", "et"])
    ap.add_argument("--acc", default="dd", choices=["dd", "fp64"])
    ap.add_argument("--pass", dest="passes", default="fwdbwd", choices=["fwd", "fwdbwd"])
    ap.add_argument("--mode", default="fused", choices=["fused", "recompute", "store"],
                    help="fused: one pass evaluates every term's value and adjoint (the per-"
                         "problem gradient is then mapped to dA, dgamma); recompute: forward "
                         "pass, then a backward pass that repeats every term's spectral work; "
                         "store: the forward keeps every term's series coefficients and the "
                         "backward reads them")
    ap.add_argument("--budget-s", type=float, default=150.0,
                    help="wall-clock budget (s, after the timed steps) for the secondary "
                         "measurements")
    ap.add_argument("--no-extras", action="store_true", help="skip every secondary measurement")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="run one plain device copy of this size before timing (a known-size "
                         "reference for memory-traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 (across "
                                   "GPUs the term sum shards by term ranges: each GPU evaluates "
                                   "its term_begin/term_end share unscaled and the partial sums "
                                   "are added)"}))
        sys.exit(2)
    t_start = time.time()
    t_extras = [None]

    def budget_left():
        return args.budget_s - (time.time() - t_extras[0])

    import torch
    from paper_2108_01622_amd import api, inputs
    from paper_2108_01622_amd import _binding
    from paper_2108_01622_amd.profiling import stored_traffic

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    A_np, g_np = inputs.grad40(count=args.batch)
    N = A_np.shape[1]
    n, m = N // 2, N
    A = torch.as_tensor(A_np, device=dev)
    g = torch.as_tensor(g_np, device=dev)
    T_full = _binding.term_count(N, sum=args.sum)
    S = min(1 << args.slice_log2, T_full)
    nslices = (T_full + S - 1) // S
    terms = args.batch * S
    off = np.arange(args.batch + 1, dtype=np.int64) * N

    if args.copy_ref_mib > 0:
        src = torch.ones(args.copy_ref_mib * (1 << 17), dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # workspaces and buffers, allocated once outside the timed region
    ones = torch.ones(args.batch, dtype=torch.complex128, device=dev)
    grads = torch.empty(api.lhaf_grads_count(off), dtype=torch.complex128, device=dev)

    def workspaces(mode):
        kw = dict(sum=args.sum, acc=args.acc, term_begin=0, term_end=S)
        if mode == "fused":
            o = _binding.make_opts(args.sum, args.acc, 0, S, grads=grads)
            nf = int(_binding.lib().lhaf_batched_workspace(args.batch, _binding.host_ptr(off), None,
                                                           ctypes.byref(o)))
        else:
            nf = api.lhaf_batched_workspace(off, **kw)
        o_b = _binding.make_opts(args.sum, args.acc, 0, S, grads=grads if mode == "fused" else None)
        nb = int(_binding.lib().lhaf_backward_workspace(args.batch, _binding.host_ptr(off), None, N,
                                                        ctypes.byref(o_b)))
        return (torch.empty(max(nf, 1), dtype=torch.uint8, device=dev),
                torch.empty(max(nb, 1), dtype=torch.uint8, device=dev))

    def make_store():
        return torch.empty(api.lhaf_saved_count(off, sum=args.sum, term_begin=0, term_end=S),
                           dtype=torch.complex128, device=dev)

    def make_step(mode):
        ws_fwd, ws_bwd = workspaces(mode)
        st = make_store() if mode == "store" else None
        gr = grads if mode == "fused" else None

        def run_step(i, fwd_ms=None, bwd_ms=None):
            s = i % nslices
            t0, t1 = s * S, min((s + 1) * S, T_full)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record(stream)
            out = api.lhaf_batched(A, g, sum=args.sum, acc=args.acc, term_begin=t0, term_end=t1,
                                   scaled=False, workspace=ws_fwd, saved=st,
                                   grads=gr if args.passes == "fwdbwd" else None)
            e[1].record(stream)
            if args.passes == "fwdbwd":
                e[2].record(stream)
                api.lhaf_backward(A, g, ones, sum=args.sum, acc=args.acc, term_begin=t0,
                                  term_end=t1, workspace=ws_bwd, saved=st, grads=gr)
                e[3].record(stream)
            if fwd_ms is not None:
                torch.cuda.synchronize()
                fwd_ms.append(e[0].elapsed_time(e[1]))
                if args.passes == "fwdbwd":
                    bwd_ms.append(e[2].elapsed_time(e[3]))
            return out
        return run_step, st

    run_step, store = make_step(args.mode)

    for i in range(args.warmup):
        run_step(i)
        torch.cuda.synchronize()
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    fwd_ms, bwd_ms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        run_step(i, fwd_ms, bwd_ms)
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    value = terms * args.steps / elapsed
    fwd_s = float(np.mean(fwd_ms)) / 1e3
    F = canonical_flops(m, n)
    fwd_tf = F * terms / fwd_s / 1e12
    tile = math.ceil(N / 8)
    fwd_kernel = f"forward_kernel<{tile}, {'true' if args.sum == 'et' else 'false'}>"
    # the backward instance the library selects: LDS-staged up to tile 5 when
    # it reads the coefficient store, up to tile 3 when it recomputes them
    staged = tile <= (5 if args.mode == "store" else 3)
    bwd_kernel = f"backward_kernel<{tile}, {'true' if staged else 'false'}>"
    fused = args.mode == "fused" and args.passes == "fwdbwd"
    if fused:
        # one launch (backward_kernel) evaluates every term's value and adjoint;
        # the "backward" call only maps the per-problem gradients
        fwd_kernel = bwd_kernel
        f_s = fwd_s
        Fb = canonical_flops_bwd(m, n, False)
        f_tf = Fb * terms / f_s / 1e12
        dom = {"bound": "alu", "kernel": bwd_kernel, "achieved": f_tf,
               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": f_tf / FP64_PEAK_TFLOPS,
               "traffic": stored_traffic(bwd_kernel, terms), "per_term_flops": Fb,
               "terms_per_launch": terms, "launch_ms": f_s * 1e3}
    elif bwd_ms:
        bwd_s = float(np.mean(bwd_ms)) / 1e3
        Fb = canonical_flops_bwd(m, n, args.mode == "store")
        bwd_tf = Fb * terms / bwd_s / 1e12
        dom = {"bound": "alu", "kernel": bwd_kernel, "achieved": bwd_tf,
               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": bwd_tf / FP64_PEAK_TFLOPS,
               "traffic": stored_traffic(bwd_kernel, terms), "per_term_flops": Fb,
               "terms_per_launch": terms, "launch_ms": bwd_s * 1e3}
    else:
        dom = {"bound": "alu", "kernel": fwd_kernel, "achieved": fwd_tf,
               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": fwd_tf / FP64_PEAK_TFLOPS,
               "traffic": stored_traffic(fwd_kernel, terms), "per_term_flops": F,
               "terms_per_launch": terms, "launch_ms": fwd_s * 1e3}
    coeffs = {"fused": "computed once per term in the fused value+adjoint pass; nothing stored "
                       "per term",
              "recompute": "recomputed per term in a separate backward pass",
              "store": "forward store (16 n bytes per term)"}[args.mode]
    res = {
        "metric": "lhaf terms/sec (N=40, FDS, double-double; " +
                  ("forward + backward" if bwd_ms else "forward") + ")",
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
                               f"{args.acc} accumulation, " + ("fwd+bwd" if bwd_ms else "fwd") +
                               f"; a step = term slice [s*{S}, (s+1)*{S}) of every matrix "
                               f"(s = step mod {nslices}, {T_full} terms per matrix)",
                   "global_batch": args.batch, "N": N, "terms_per_lhaf": T_full,
                   "terms_per_step": terms, "slice_terms": S, "sum": args.sum, "acc": args.acc,
                   "mode": args.mode, "backward_coefficients": coeffs},
        "roofline": dom,
        "lhafs_per_s": args.batch * args.steps / elapsed * S / T_full,
        "time_to_solution_s": elapsed / args.steps * nslices,
    }
    if fused:
        res["fused_pass"] = {"kernel": bwd_kernel, "terms_per_s": terms / fwd_s,
                             "launch_ms": fwd_s * 1e3, "per_term_flops": Fb,
                             "frac": dom["frac"],
                             "gradient_map_ms": float(np.mean(bwd_ms)),
                             "products_executed": ps_products(n)}
    else:
        res["forward"] = {"kernel": fwd_kernel, "terms_per_s": terms / fwd_s, "tflops": fwd_tf,
                          "frac": fwd_tf / FP64_PEAK_TFLOPS, "launch_ms": fwd_s * 1e3,
                          "per_term_flops": F}
    if bwd_ms and not fused:
        res["backward"] = {"kernel": bwd_kernel, "terms_per_s": terms / bwd_s, "tflops": bwd_tf,
                           "frac": bwd_tf / FP64_PEAK_TFLOPS, "launch_ms": bwd_s * 1e3,
                           "per_term_flops": Fb, "coefficients": coeffs,
                           "products_executed": ps_products(n),
                           "per_term_flops_executed_products":
                               (F if args.mode == "recompute" else 0.0)
                               + 8.0 * m ** 3 * ps_products(n) + 24.0 * n * m * m}
    print(f"[bench] timed steps done: {value / 1e6:.3f} M terms/s", file=sys.stderr, flush=True)

    skipped = []
    t_extras[0] = time.time()

    def extra(name, need_s, fn):
        if args.no_extras:
            return
        if budget_left() < need_s:
            skipped.append(name)
            return
        t = time.time()
        try:
            res[name] = fn()
        except Exception as ex:  # a failed secondary measurement is reported, not fatal
            res[name] = {"error": f"{type(ex).__name__}: {ex}"}
        print(f"[bench] {name} done ({time.time() - t:.1f} s)", file=sys.stderr, flush=True)

    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else {}

    def timed_once(fn, reps=1):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    def rel_err_grad40():
        # full forward of the matrices whose oracle value is stored
        keys = [k for k in gold if k.startswith("grad40/") and k.count("/") == 1
                and int(k.split("/")[1]) < args.batch]
        bs = [int(k.split("/")[1]) for k in keys]
        out = api.lhaf_batched(A[bs], g[bs], sum=args.sum, acc=args.acc).cpu().numpy()
        errs = [abs(out[i] - complex(*gold[k]["value"])) / abs(complex(*gold[k]["value"]))
                for i, k in enumerate(keys)]
        return {"max": max(errs), "count": len(errs), "matrices": bs,
                "oracle": "FDS double, explicit matrix powers (stored oracle values)"}

    if args.sum == "fds":
        extra("rel_err_vs_oracle", 10, rel_err_grad40)

    def cpu():
        return cpu_baseline(A_np[0], g_np[0], budget_s=8.0)

    extra("cpu_baseline", 20, cpu)

    def other_mode(mode):
        def fn():
            step, st = make_step(mode)
            fm, bm = [], []
            step(0)
            for i in range(3):
                step(i, fm, bm)
            f_ms, b_ms = float(np.mean(fm)), float(np.mean(bm))
            ent = {"workload": f"same step (slice of {S} terms x {args.batch}), mode {mode}: " +
                               {"fused": "one pass for values and adjoints",
                                "recompute": "forward pass, then a backward pass that repeats "
                                             "every term's spectral work",
                                "store": "the forward keeps every term's series coefficients, "
                                         "the backward reads them"}[mode],
                   "step_terms_per_s": terms / ((f_ms + b_ms) / 1e3),
                   "forward_ms": f_ms, "backward_ms": b_ms}
            if mode != "fused":
                Fm = canonical_flops_bwd(m, n, mode == "store")
                ent.update({"forward_terms_per_s": terms / (f_ms / 1e3),
                            "forward_frac": F * terms / (f_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                            "backward_terms_per_s": terms / (b_ms / 1e3),
                            "backward_per_term_flops": Fm,
                            "backward_frac": Fm * terms / (b_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS})
            if mode == "store":
                ent["store_bytes"] = st.numel() * 16
                ent["store_bytes_per_term"] = 16 * n
            return ent
        return fn

    if args.passes == "fwdbwd":
        for mode in ("fused", "recompute", "store"):
            if mode != args.mode:
                extra(f"{mode}_variant", 12, other_mode(mode))

    def n52():
        A52, g52, _, _ = inputs.block_diagonal_stress(52, 0)
        a52 = torch.as_tensor(A52, device=dev)[None]
        q52 = torch.as_tensor(g52, device=dev)[None]
        T52 = _binding.term_count(52)
        S52 = 1 << 17
        one = torch.ones(1, dtype=torch.complex128, device=dev)
        tf = timed_once(lambda: api.lhaf_batched(a52, q52, term_begin=0, term_end=S52, scaled=False))
        tb = timed_once(lambda: api.lhaf_backward(a52, q52, one, term_begin=0, term_end=S52))
        g52 = torch.empty(api.lhaf_grads_count(np.array([0, 52])), dtype=torch.complex128,
                          device=dev)

        def fused52():
            api.lhaf_batched(a52, q52, term_begin=0, term_end=S52, scaled=False, grads=g52)
            api.lhaf_backward(a52, q52, one, grads=g52)
        tfu = timed_once(fused52)
        F52 = canonical_flops(52, 26)
        Fb52 = canonical_flops_bwd(52, 26, False)
        ent = {"workload": f"block52/0 (A1 (+) A2, N=52, FDS dd): terms [0, {S52}) of {T52}: "
                           f"forward then backward (coefficients recomputed), and the fused pass",
               "forward_terms_per_s": S52 / tf, "forward_frac": F52 * S52 / tf / 1e12 / FP64_PEAK_TFLOPS,
               "backward_terms_per_s": S52 / tb,
               "backward_frac": Fb52 * S52 / tb / 1e12 / FP64_PEAK_TFLOPS,
               "two_pass_step_terms_per_s": S52 / (tf + tb), "forward_per_term_flops": F52,
               "backward_per_term_flops": Fb52, "fused_step_terms_per_s": S52 / tfu,
               "fused_frac": Fb52 * S52 / tfu / 1e12 / FP64_PEAK_TFLOPS}
        return ent

    extra("n52_fwd_bwd", 20, n52)

    def n52_full():
        A52, g52, _, _ = inputs.block_diagonal_stress(52, 0)
        a52 = torch.as_tensor(A52, device=dev)
        q52 = torch.as_tensor(g52, device=dev)
        T52 = _binding.term_count(52)
        torch.cuda.synchronize()
        t = time.perf_counter()
        v52 = api.lhaf(a52, q52).item()
        t52 = time.perf_counter() - t
        tf52 = canonical_flops(52, 26) * T52 / t52 / 1e12
        ent = {"workload": "block52/0 (A1 (+) A2, N=52, FDS dd), full sum", "terms_per_s": T52 / t52,
               "tflops": tf52, "frac": tf52 / FP64_PEAK_TFLOPS, "seconds": t52}
        # the same sum with the characteristic polynomial and the series in
        # double-double (acc "ddc")
        torch.cuda.synchronize()
        t = time.perf_counter()
        v52c = api.lhaf(a52, q52, acc="ddc").item()
        t52c = time.perf_counter() - t
        ent["ddc_terms_per_s"] = T52 / t52c
        if "block52/0" in gold:
            ref = complex(*gold["block52/0"]["value"])
            ent["rel_err_vs_oracle"] = abs(v52 - ref) / abs(ref)
            ent["ddc_rel_err_vs_oracle"] = abs(v52c - ref) / abs(ref)
            ent["oracle"] = "__float128 FDS of both halves, multiplied"
        return ent

    extra("n52_forward_full", 35, n52_full)

    def modes():
        A8, g8 = A[:8], g[:8]
        out = {}
        for sm in ("fds", "et"):
            for am in ("dd", "fp64", "ddc"):
                dt = timed_once(lambda: api.lhaf_batched(A8, g8, sum=sm, acc=am))
                T8 = 8 * _binding.term_count(N, sum=sm)
                fl = 8 * (et_flops_per_lhaf(N) if sm == "et" else F * _binding.term_count(N))
                out[f"{sm}/{am}"] = {"terms_per_s": T8 / dt, "lhafs_per_s": 8 / dt,
                                     "frac": fl / dt / 1e12 / FP64_PEAK_TFLOPS}
        return out

    extra("forward_modes_n40", 10, modes)

    def latency16():
        A16, g16 = inputs.single16()
        a = torch.as_tensor(A16, device=dev)
        q = torch.as_tensor(g16, device=dev)
        for _ in range(5):
            api.lhaf(a, q)
        torch.cuda.synchronize()
        lat = []
        for _ in range(50):
            t = time.perf_counter()
            api.lhaf(a, q)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t)
        lat.sort()
        return {"workload": "single16: one N=16 lhaf (FDS dd), call to result on the host",
                "median_us": 1e6 * lat[len(lat) // 2], "min_us": 1e6 * lat[0],
                "p90_us": 1e6 * lat[int(0.9 * len(lat))]}

    extra("latency_n16", 3, latency16)

    def chain():
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
        return {"workload": "4096 submatrices N=20..40 (even) of the 100-mode state, FDS dd, "
                            "one persistent launch",
                "terms": Tc, "seconds": dt, "terms_per_s": Tc / dt, "lhafs_per_s": 4096 / dt,
                "tflops": fl / dt / 1e12, "frac": fl / dt / 1e12 / FP64_PEAK_TFLOPS}

    extra("chain4096_forward", 45, chain)

    def multi():
        out = {}
        _, gs = inputs.subdetector_gammas(12)
        gst = torch.as_tensor(gs, device=dev)
        A12 = A[:1].expand(12, N, N).contiguous()
        t_one = timed_once(lambda: api.lhaf_gammas(A[0], gst))
        t_sep = timed_once(lambda: api.lhaf_batched(A12, gst))
        out["gamma_batch_n40"] = {"workload": "one N=40 grad40 matrix, 12 loop-weight vectors, FDS dd",
                                  "seconds": t_one, "separate_seconds": t_sep,
                                  "speedup": t_sep / t_one,
                                  "output_terms_per_s": 12 * T_full / t_one}
        st = inputs.state100(0)
        rfix = st["r"].astype(np.int32).copy()
        b = int(np.nonzero(rfix == 0)[0][0])
        Bt = torch.as_tensor(st["B"], device=dev)
        gt = torch.as_tensor(st["gamma"], device=dev)
        t_chain = timed_once(lambda: api.lhaf_chain(Bt, gt, rfix, b, 8))

        def separate():
            for k in range(9):
                rk = rfix.copy()
                rk[b] = k
                api.lhaf(Bt, gt, r=rk, sum="et")
        t_sep = timed_once(separate)
        out["chain_step_state100"] = {"workload": "state100 pattern (40 photons, 28 modes) fixed, "
                                                  "one empty mode batched k = 0..8, ET dd",
                                      "seconds": t_chain, "separate_seconds": t_sep,
                                      "speedup": t_sep / t_chain}
        Am, gm, nm = inputs.mixed_state(20, 0)
        while 2 * nm.sum() > 40:
            nm[np.argmax(nm)] -= 1
        Amt = torch.as_tensor(Am, device=dev)
        gmt = torch.as_tensor(gm, device=dev)
        t_mix = timed_once(lambda: api.lhaf_mixed(Amt, gmt, nm))
        Tm = int(np.prod(nm[nm > 0] + 1))
        Tm = Tm // 2 if np.any(nm % 2) else Tm // 2 + 1  # FDS halving (first odd pair, else pair 0)
        out["mixed_state_m20"] = {"workload": f"lhafmix, 2M x 2M with M = 20, n = {nm.tolist()}, "
                                              f"N = {2 * int(nm.sum())}, FDS dd",
                                  "seconds": t_mix, "terms": Tm, "terms_per_s": Tm / t_mix}
        Ar, gr = inputs.real_nonneg(N, 0)
        Art, grt = torch.as_tensor(Ar, device=dev), torch.as_tensor(gr, device=dev)
        t_real = timed_once(lambda: api.lhaf_real(Art, grt))
        t_cplx = timed_once(lambda: api.lhaf(Art.to(torch.complex128), grt.to(torch.complex128)))
        out["real_nonneg_n40"] = {"workload": "one real non-negative N=40 lhaf, FDS dd",
                                  "seconds": t_real, "complex_kernel_seconds": t_cplx,
                                  "terms_per_s": T_full / t_real,
                                  "speedup_vs_complex": t_cplx / t_real}
        return out

    extra("multi_output", 8, multi)

    if skipped:
        res["skipped_for_time_budget"] = skipped
    res["wall_s"] = time.time() - t_start
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
