"""Accuracy of the signed term sum against stored __float128 references.

    python -m paper_2108_01622_amd.precision [--n52 K] [--n60 K] [--modes fds/dd ...] > table.md

The paper's accuracy protocol (App. B.4): block-diagonal C = A1 (+) A2 with
both halves drawn iid CN(0, 1/N), so that lhaf(C) = lhaf(A1) lhaf(A2) is
known exactly from the halves (evaluated by the oracle in __float128 and
stored in tests/golden/oracle_values.json by tests/golden/make_golden.py).
Each listed lhaf is evaluated on the GPU in the requested sum / accumulation
modes and its relative error against the stored reference is tabulated with
the library's own error estimate.  This module only reads the stored values;
it never runs the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
GOLD = os.path.join(ROOT, "tests", "golden", "oracle_values.json")


def _sliced(api, _binding, At, gt, N, sm, am, slices, label, log):
    """lhaf as `slices` consecutive term ranges (each scaled: its share of the
    sum), combined exactly from their double-double parts; a progress line
    per range.  Returns (value, summed err_est)."""
    import math
    T = _binding.term_count(N, sum=sm)
    re, im, est = [], [], 0.0
    for i in range(slices):
        t0, t1 = i * T // slices, (i + 1) * T // slices
        v, e, lo = api.lhaf(At, gt, sum=sm, acc=am, term_begin=t0, term_end=t1,
                            return_error=True, return_lo=True)
        v, lo = complex(v.item()), complex(lo.item())
        re += [v.real, lo.real]
        im += [v.imag, lo.imag]
        est += e.item()
        print(f"[precision] {label} terms [{t0}, {t1}) done", file=log, flush=True)
    return complex(math.fsum(re), math.fsum(im)), est


def measure(N: int, instances, modes, log=sys.stderr, slices=1):
    import torch
    from . import _binding, api, inputs
    gold = json.load(open(GOLD))
    rows = []
    for k in instances:
        key = f"block{N}/{k}"
        if key not in gold:
            continue
        ref = complex(*gold[key]["value"])
        A, g, _, _ = inputs.block_diagonal_stress(N, k)
        At = torch.as_tensor(A, device="cuda")
        gt = torch.as_tensor(g, device="cuda")
        for mode in modes:
            sm, am = mode.split("/")
            print(f"[precision] {key} {mode} ...", file=log, flush=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            if slices > 1:
                v, e = _sliced(api, _binding, At, gt, N, sm, am, slices, f"{key} {mode}", log)
            else:
                v, e = api.lhaf(At, gt, sum=sm, acc=am, return_error=True)
                v, e = v.item(), e.item()
            dt = time.perf_counter() - t
            rel = abs(v - ref) / abs(ref)
            rows.append(dict(key=key, mode=mode, rel=rel, err_est_rel=e / abs(ref), seconds=dt))
            print(f"[precision] {key} {mode} rel {rel:.3e} est {e / abs(ref):.3e} {dt:.1f} s",
                  file=log, flush=True)
    return rows


def table(rows) -> str:
    out = ["| lhaf | mode | rel. error vs __float128 | library err_est / abs | seconds |",
           "|:--|:--|--:|--:|--:|"]
    for r in rows:
        out.append(f"| {r['key']} | {r['mode']} | {r['rel']:.2e} | {r['err_est_rel']:.2e} | "
                   f"{r['seconds']:.1f} |")
    by = {}
    for r in rows:
        n = r["key"].split("/")[0]
        by.setdefault((n, r["mode"]), []).append(r["rel"])
    out += ["", "| set | mode | max rel. error | median | count |", "|:--|:--|--:|--:|--:|"]
    for (n, mode), v in sorted(by.items()):
        out.append(f"| {n} | {mode} | {max(v):.2e} | {float(np.median(v)):.2e} | {len(v)} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n52", type=int, default=10, help="block52 instances (stored: 10)")
    ap.add_argument("--n60", type=int, default=1, help="block60 instances (stored: 4)")
    ap.add_argument("--from60", type=int, default=0, help="first block60 instance")
    ap.add_argument("--modes", nargs="*", default=["fds/dd", "fds/fp64", "et/dd", "et/fp64"])
    ap.add_argument("--modes60", nargs="*", default=["fds/dd", "fds/fp64"])
    ap.add_argument("--slices60", type=int, default=1,
                    help="evaluate each N = 60 sum as this many term ranges (progress per range)")
    a = ap.parse_args(argv)
    rows = measure(52, range(a.n52), a.modes)
    if a.n60 > 0:
        rows += measure(60, range(a.from60, a.from60 + a.n60), a.modes60, slices=a.slices60)
    sys.stdout.write(table(rows))


if __name__ == "__main__":
    main()
