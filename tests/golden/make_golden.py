"""Write tests/golden/oracle_values.json: reference values for the full-size
workloads, computed by the CPU oracle only (never by the HIP library).

    python tests/golden/make_golden.py [--only KEY ...] [--threads N]

Each entry records how it was computed.  Methods:
  memo_f128      definition, memoised recursion, __float128
  fds_f64        finite-difference sieve, explicit matrix powers, double + Neumaier
  fds_f128       same in __float128
  fds_f128 lhafmix  mixed-state lhafmix (App. B.2), FDS in __float128
  block_f128     block-diagonal A1 (+) A2: lhaf(A1) * lhaf(A2), each half FDS in
                 __float128 (the paper's own accuracy protocol, App. B.4)
The file is updated incrementally (existing keys are kept unless --force).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2108_01622_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "oracle_values.json")

GRAD40_SAMPLE = [0, 37, 101, 255]
CHAIN_PER_SIZE = 2
DENSE52_BLOCK = 10
DENSE60_BLOCK = 4
GAMMAS40_SAMPLE = [0, 5, 11]


def cx(z):
    return [float(np.real(z)), float(np.imag(z))]


def jobs():
    J = {}
    A, g = I.single16()
    J["single16"] = lambda A=A, g=g: dict(method="memo_f128", value=cx(O.lhaf_memo(A, g, prec="f128")),
                                          sha256=I.sha256_of(A, g))
    st = I.state100(0)
    def rep(st=st):
        v, ab = O.lhaf_repeated(st["B"], st["gamma"], st["r"], method="sum", mode="fds", prec="f64",
                                with_abs=True)
        pairs, left = O.matched_reps(st["r"])
        return dict(method="fds_f64 repeated pairs (greedy matching)", value=cx(v), abs_sum=ab,
                    pattern_counts=[int((st["r"] == k).sum()) for k in (1, 2, 3)],
                    eta=[p[2] for p in pairs] + ([1] if left is not None else []),
                    sha256=I.sha256_of(st["B"], st["gamma"], st["r"]))
    J["state100"] = rep
    def rep128(st=st):
        v = O.lhaf_repeated(st["B"], st["gamma"], st["r"], method="sum", mode="fds", prec="f128")
        return dict(method="fds_f128 repeated pairs (greedy matching)", value=cx(v))
    J["state100/f128"] = rep128
    A40, g40 = I.grad40()
    for b in GRAD40_SAMPLE:
        def g40job(b=b):
            v, ab = O.lhaf_sum(A40[b], g40[b], mode="fds", prec="f64", with_abs=True)
            return dict(method="fds_f64", value=cx(v), abs_sum=ab, sha256=I.sha256_of(A40[b], g40[b]))
        J[f"grad40/{b}"] = g40job
    # closed-form derivatives of grad40[0]: d/d gamma_3 = lhaf(A_-3),
    # d/d A_12 (entry of the full matrix read through sym(A)) = lhaf(A_-1,-2) / 2
    def d_gamma(b=0, i=3):
        Ar, gr = O.remove(A40[b], g40[b], [i])
        return dict(method="fds_f64 of the minor", value=cx(O.lhaf_sum(Ar, gr, mode="fds", prec="f64")))
    def d_a(b=0, i=1, j=2):
        Ar, gr = O.remove(A40[b], g40[b], [i, j])
        return dict(method="fds_f64 of the minor, halved", value=cx(0.5 * O.lhaf_sum(Ar, gr, mode="fds", prec="f64")))
    J["grad40/0/dgamma3"] = d_gamma
    J["grad40/0/dA1_2"] = d_a
    ch = I.chain4096()
    sizes = ch["sizes"]
    for N in range(20, 41, 2):
        picks = [int(i) for i in np.nonzero(sizes == N)[0][:CHAIN_PER_SIZE]]
        for b in picks:
            def chjob(b=b):
                ix = ch["idx"][ch["idx_off"][b]:ch["idx_off"][b + 1]]
                A = ch["B"][np.ix_(ix, ix)]
                g = ch["gamma"][ix]
                v, ab = O.lhaf_sum(A, g, mode="fds", prec="f64", with_abs=True)
                return dict(method="fds_f64", value=cx(v), abs_sum=ab, N=int(len(ix)))
            J[f"chain4096/{b}"] = chjob
    def ch128(b=0):
        ix = ch["idx"][ch["idx_off"][b]:ch["idx_off"][b + 1]]
        v = O.lhaf_sum(ch["B"][np.ix_(ix, ix)], ch["gamma"][ix], mode="fds", prec="f128")
        return dict(method="fds_f128", value=cx(v), N=int(len(ix)))
    J["chain4096/0/f128"] = ch128
    for n, cnt in ((52, DENSE52_BLOCK), (60, DENSE60_BLOCK)):
        for k in range(cnt):
            def bjob(n=n, k=k):
                A, g, (a1, g1), (a2, g2) = I.block_diagonal_stress(n, k)
                v1 = O.lhaf_sum(a1, g1, mode="fds", prec="f128")
                v2 = O.lhaf_sum(a2, g2, mode="fds", prec="f128")
                return dict(method="block_f128", value=cx(v1 * v2), halves=[cx(v1), cx(v2)],
                            sha256=I.sha256_of(A, g))
            J[f"block{n}/{k}"] = bjob
    A1, gs = I.subdetector_gammas()
    for k in GAMMAS40_SAMPLE:
        def gjob(k=k):
            v, ab = O.lhaf_sum(A1, gs[k], mode="fds", prec="f64", with_abs=True)
            return dict(method="fds_f64", value=cx(v), abs_sum=ab, sha256=I.sha256_of(A1, gs[k]))
        J[f"gammas40/{k}"] = gjob
    # mixed state of 14 modes, photon numbers capped at 2 sum n = 40, in the
    # pairing (i, M + i) of lhafmix (App. B.2): kappa = 4.4e6
    def mixjob(inst=0):
        A, g, n = I.mixed_state(14, inst)
        while 2 * n.sum() > 40:
            n[np.argmax(n)] -= 1
        v = O.lhafmix(A, g, n, mode="fds", prec="f128")
        return dict(method="fds_f128 lhafmix", value=cx(v), n=[int(x) for x in n],
                    sha256=I.sha256_of(A, g))
    J["mixed14/0/f128"] = mixjob
    for n in (24, 40):
        def rjob(n=n):
            a, g = I.real_nonneg(n, 0)
            v, ab = O.lhaf_sum(a.astype(complex), g.astype(complex), mode="fds", prec="f64",
                               with_abs=True)
            return dict(method="fds_f64", value=cx(v), abs_sum=ab, sha256=I.sha256_of(a, g))
        J[f"real{n}/0"] = rjob
    return J


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--force", action="store_true")
    a = ap.parse_args()
    O.set_threads(a.threads)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data.setdefault("_about", "written by tests/golden/make_golden.py from oracle/ only")
    for key, fn in jobs().items():
        if a.only and not any(key.startswith(o) for o in a.only):
            continue
        if key in data and not a.force:
            continue
        t = time.time()
        res = fn()
        res["seconds"] = round(time.time() - t, 2)
        res["threads"] = a.threads
        # merge with what other runs wrote meanwhile
        data = json.load(open(OUT)) if os.path.exists(OUT) else data
        data[key] = res
        json.dump(data, open(OUT + ".tmp", "w"), indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)
        print(f"{key}: {res['value']} ({res['seconds']} s)", flush=True)


if __name__ == "__main__":
    main()
