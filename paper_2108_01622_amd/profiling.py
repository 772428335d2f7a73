"""Summaries of rocprofv3 runs of the loop-hafnian kernels (host-side text
processing only; run the profiler itself with the program directly after
`--`, e.g. `rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o
run -- python bench.py`).

    python -m paper_2108_01622_amd.profiling stats DIR/run_kernel_stats.csv \\
        --command "..." --title "..."                      > profiles/NAME.md
    python -m paper_2108_01622_amd.profiling traffic \\
        --fetch DIR/f_counter_collection.csv --write DIR/w_counter_collection.csv \\
        --kernel "backward_kernel<5>" --terms T --copy-bytes 1073741824 \\
        --command "..." --title "..."                      > profiles/NAME.md
    python -m paper_2108_01622_amd.profiling issue DIR/a_counter_collection.csv \\
        DIR/b_counter_collection.csv --kernel "forward_kernel<5, false>" --terms T \\
        --command "..." --title "..."                      > profiles/NAME.md

`traffic` turns the FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch)
into HBM bytes: each counter is scaled by the factor that makes it read the
known size of the largest plain copy in the same run (the run must contain
one, e.g. bench.py --copy-ref-mib 1024), and the per-term bytes are recorded
in profiles/traffic.json together with a hash of the kernel sources, so that
bench.py reports them only for the code they were measured on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash() -> str:
    """SHA-256 over the sources the persistent kernels are compiled from (the
    kernel files, device and internal headers, the per-tile unit and the
    public header) and the shipped schedule table, which sets their launch
    shape.  The host API unit (lhaf_api.hip: validation, planning, small
    set-up kernels) and the planner are left out, so a host-side change does
    not invalidate a traffic record of an unchanged kernel."""
    h = hashlib.sha256()
    files = sorted([f for f in glob.glob(os.path.join(HERE, "csrc", "*.hip"))
                    if os.path.basename(f) != "lhaf_api.hip"] +
                   glob.glob(os.path.join(HERE, "csrc", "*.h")) +
                   glob.glob(os.path.join(ROOT, "include", "*.h")) +
                   [os.path.join(HERE, "tune", "mi355x.txt")])
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def stored_traffic(kernel: str, terms: int):
    """HBM bytes of one launch of `kernel` processing `terms` terms, from
    profiles/traffic.json; None if absent or taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    ent = json.load(open(TRAFFIC_JSON)).get(kernel)
    if not ent or ent.get("src_sha256") != kernel_source_hash():
        return None
    return (ent["fetch_bytes_per_term"] + ent["write_bytes_per_term"]) * terms


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").replace("lh::", "")


def stats_md(path: str, command: str, title: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {title}", "", "Command (from /tmp, TMPDIR=/tmp):", f"`{command}`", "",
           "| Kernel | Calls | Total (ms) | Average (ms) | Min (ms) | Max (ms) | Percent |",
           "|:--|--:|--:|--:|--:|--:|--:|"]
    for r in rows[:top]:
        out.append("| {} | {} | {:.3f} | {:.3f} | {:.3f} | {:.3f} | {:.2f} |".format(
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6, float(r["MaxNs"]) / 1e6,
            float(r["Percentage"])))
    return "\n".join(out) + "\n"


def _counter_rows(path: str, counter: str):
    res = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            res.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]),
                        float(r["Counter_Value"])))
    return res


def _copy_factor(rows, copy_bytes: int) -> tuple[float, str]:
    """Known bytes / counter bytes of the largest plain copy dispatch."""
    cands = [r for r in rows if "copyBuffer" in r[1] or "copy" in r[1].lower()]
    if not cands:
        raise SystemExit("no copy dispatch in the counter file (run with --copy-ref-mib)")
    d = max(cands, key=lambda r: r[3])
    return copy_bytes / (d[3] * 1024.0), f"{_short(d[1])} (dispatch {d[0]}, {d[3]:.1f} KiB)"


def traffic_md(fetch_csv: str, write_csv: str, kernel: str, terms: int, copy_bytes: int,
               command: str, title: str, update_json: bool = True) -> str:
    fr = _counter_rows(fetch_csv, "FETCH_SIZE")
    wr = _counter_rows(write_csv, "WRITE_SIZE")
    ff, fdesc = _copy_factor(fr, copy_bytes)
    wf, wdesc = _copy_factor(wr, copy_bytes)
    fk = [r for r in fr if _short(r[1]) == kernel]
    wk = [r for r in wr if _short(r[1]) == kernel]
    if not fk or not wk:
        raise SystemExit(f"kernel {kernel} not found in the counter files")
    fetch_b = fk[-1][3] * 1024.0 * ff
    write_b = wk[-1][3] * 1024.0 * wf
    out = [f"# {title}", "", "Commands (each its own rocprofv3 run, from /tmp, TMPDIR=/tmp):",
           f"`{command}`", "",
           f"Copy reference ({copy_bytes} bytes read and written): FETCH_SIZE factor {ff:.4f} "
           f"from {fdesc}; WRITE_SIZE factor {wf:.4f} from {wdesc}.", "",
           "| Kernel dispatch | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM read (B) | HBM write (B) "
           "| Terms | Read B/term | Write B/term |",
           "|:--|--:|--:|--:|--:|--:|--:|--:|",
           f"| {kernel} | {fk[-1][3]:.1f} | {wk[-1][3]:.1f} | {fetch_b:.4g} | {write_b:.4g} | {terms} "
           f"| {fetch_b / terms:.1f} | {write_b / terms:.1f} |"]
    if update_json:
        data = json.load(open(TRAFFIC_JSON)) if os.path.exists(TRAFFIC_JSON) else {}
        data[kernel] = {"src_sha256": kernel_source_hash(),
                        "fetch_bytes_per_term": fetch_b / terms,
                        "write_bytes_per_term": write_b / terms,
                        "fetch_factor": ff, "write_factor": wf, "command": command}
        os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
        json.dump(data, open(TRAFFIC_JSON, "w"), indent=1, sort_keys=True)
    return "\n".join(out) + "\n"


ISSUE_COUNTERS = ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU",
                  "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_WAIT_INST_ANY", "SQ_INSTS_VALU_FMA_F64",
                  "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64"]


def issue_md(csvs, kernel: str, terms: int, command: str, title: str) -> str:
    """Instruction-issue summary of the last dispatch of `kernel` from SQ
    counter files (one or more rocprofv3 --pmc passes): instructions per term
    by class and the fraction of each wavefront's cycles spent issuing VALU
    instructions."""
    val = {}
    for path in csvs:
        last = {}
        for r in csv.DictReader(open(path)):
            if _short(r["Kernel_Name"]) != kernel:
                continue
            d = int(r["Dispatch_Id"])
            last.setdefault(r["Counter_Name"], {})[d] = float(r["Counter_Value"])
        for c, by in last.items():
            val[c] = by[max(by)]
    if not val:
        raise SystemExit(f"kernel {kernel} not found in the counter files")
    out = [f"# {title}", "", "Commands (one rocprofv3 --pmc pass per counter set, from /tmp, "
           "TMPDIR=/tmp):", f"`{command}`", "", f"Terms in the dispatch: {terms}.", "",
           "| Counter | Value | Per term |", "|:--|--:|--:|"]
    for c in ISSUE_COUNTERS:
        if c in val:
            out.append(f"| {c} | {val[c]:.4g} | {val[c] / terms:.4g} |")
    if "SQ_ACTIVE_INST_VALU" in val and "SQ_WAVE_CYCLES" in val:
        out += ["", "VALU issue per wavefront cycle (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES): "
                f"{val['SQ_ACTIVE_INST_VALU'] / val['SQ_WAVE_CYCLES']:.3f}"]
    if "SQ_INSTS_VALU_FMA_F64" in val and "SQ_INSTS_VALU" in val:
        out.append("FP64 FMA share of the VALU instructions: "
                   f"{val['SQ_INSTS_VALU_FMA_F64'] / val['SQ_INSTS_VALU']:.3f}")
    if all(c in val for c in ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64",
                              "SQ_INSTS_VALU_MUL_F64")):
        # every wavefront instruction issues 64 lanes (masked lanes included)
        flops = 64.0 * (2.0 * val["SQ_INSTS_VALU_FMA_F64"] + val["SQ_INSTS_VALU_ADD_F64"]
                        + val["SQ_INSTS_VALU_MUL_F64"])
        out.append(f"Executed FP64 flops per term (64 lanes x (2 FMA + ADD + MUL)): "
                   f"{flops / terms:.4g}")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="rocprofv3 kernel trace summary")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--terms", type=int, required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--command", required=True)
    t.add_argument("--title", default="rocprofv3 memory traffic")
    t.add_argument("--no-json", action="store_true")
    i = sub.add_parser("issue")
    i.add_argument("csv", nargs="+")
    i.add_argument("--kernel", required=True)
    i.add_argument("--terms", type=int, required=True)
    i.add_argument("--command", required=True)
    i.add_argument("--title", default="rocprofv3 instruction issue")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        sys.stdout.write(stats_md(a.csv, a.command, a.title))
    elif a.cmd == "issue":
        sys.stdout.write(issue_md(a.csv, a.kernel, a.terms, a.command, a.title))
    else:
        sys.stdout.write(traffic_md(a.fetch, a.write, a.kernel, a.terms, a.copy_bytes, a.command,
                                    a.title, not a.no_json))


if __name__ == "__main__":
    main()
