"""Host logic of the measurement tooling (no GPU): rocprofv3 counter files are
turned into HBM bytes with the copy-kernel factors, recorded per kernel with
the hash of the kernel sources, and reported only for those sources; the
benchmark's Paterson-Stockmeyer product count."""
import csv
import importlib
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        for d, name, grid, val in rows:
            w.writerow([d, name, grid, counter, val])


@pytest.fixture
def prof(tmp_path, monkeypatch):
    from paper_2108_01622_amd import profiling
    monkeypatch.setattr(profiling, "TRAFFIC_JSON", str(tmp_path / "traffic.json"))
    return profiling


def test_copy_factor_scaling_and_hash_gate(prof, tmp_path, monkeypatch):
    kib = 1 << 20  # 1 GiB copy in KiB
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    kname = "void lh::backward_kernel<5>(lh::Prob const*, int)"
    # the counter reads half of the copied bytes on FETCH, all of them on WRITE
    write_counters(fetch, "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", 512, kib / 2),
                                         (2, kname, 64, 1000.0)])
    write_counters(write, "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", 512, kib),
                                         (2, kname, 64, 300.0)])
    md = prof.traffic_md(str(fetch), str(write), "backward_kernel<5>", 10, 1 << 30, "cmd", "t")
    assert "factor 2.0000" in md and "factor 1.0000" in md
    got = prof.stored_traffic("backward_kernel<5>", 10)
    assert got == pytest.approx(1000 * 1024 * 2.0 + 300 * 1024 * 1.0)
    assert prof.stored_traffic("forward_kernel<5>", 10) is None
    # other kernel sources: the stored counters no longer apply
    monkeypatch.setattr(prof, "kernel_source_hash", lambda: "different")
    assert prof.stored_traffic("backward_kernel<5>", 10) is None


def test_missing_copy_reference_is_an_error(prof, tmp_path):
    fetch = tmp_path / "f.csv"
    write_counters(fetch, "FETCH_SIZE", [(1, "lh::forward_kernel<5>(x)", 64, 5.0)])
    with pytest.raises(SystemExit):
        prof.traffic_md(str(fetch), str(fetch), "forward_kernel<5>", 1, 1 << 30, "c", "t")


def test_paterson_stockmeyer_products():
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    # s = ceil(sqrt n) powers W^2..W^s, then ceil(n/s) - 1 Horner steps
    assert [bench.ps_products(n) for n in (1, 2, 4, 5, 9, 20, 26, 32)] == [0, 1, 2, 3, 4, 7, 9, 10]
    assert bench.canonical_flops(40, 20) == pytest.approx(40 / 3 * 40 ** 3 + 8 * 20 * 1600)


def test_issue_summary_takes_last_dispatch_of_each_pass(prof, tmp_path):
    """Counters of the kernel's last dispatch, from two passes, per term."""
    kname = "void lh::forward_kernel<5, false>(lh::Prob const*, int)"
    a = tmp_path / "a.csv"
    b = tmp_path / "b.csv"
    with open(a, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writerow([1, kname, 64, "SQ_INSTS_VALU", 999.0])        # earlier dispatch: ignored
        w.writerow([3, kname, 64, "SQ_INSTS_VALU", 4000.0])
        w.writerow([3, kname, 64, "SQ_ACTIVE_INST_VALU", 4000.0])
        w.writerow([3, kname, 64, "SQ_WAVE_CYCLES", 10000.0])
        w.writerow([2, "void lh::pack_kernel(int)", 64, "SQ_INSTS_VALU", 5.0])
    with open(b, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writerow([3, kname, 64, "SQ_INSTS_VALU_FMA_F64", 1000.0])
    md = prof.issue_md([str(a), str(b)], "forward_kernel<5, false>", 100, "cmd", "t")
    assert "| SQ_INSTS_VALU | 4000 | 40 |" in md
    assert "| SQ_INSTS_VALU_FMA_F64 | 1000 | 10 |" in md
    assert "SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES): 0.400" in md
    assert "FP64 FMA share of the VALU instructions: 0.250" in md
    assert "Executed FP64 flops" not in md  # needs the ADD and MUL counts too
    with pytest.raises(SystemExit):
        prof.issue_md([str(a)], "backward_kernel<5>", 100, "cmd", "t")


def test_issue_summary_executed_flops(prof, tmp_path):
    kname = "void lh::forward_kernel<5, false>(lh::Prob const*, int)"
    a = tmp_path / "a.csv"
    with open(a, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        for c, v in (("SQ_INSTS_VALU_FMA_F64", 10.0), ("SQ_INSTS_VALU_ADD_F64", 3.0),
                     ("SQ_INSTS_VALU_MUL_F64", 2.0)):
            w.writerow([1, kname, 64, c, v])
    md = prof.issue_md([str(a)], "forward_kernel<5, false>", 4, "cmd", "t")
    # 64 lanes x (2 x 10 + 3 + 2) = 1600 flops over 4 terms
    assert "Executed FP64 flops per term (64 lanes x (2 FMA + ADD + MUL)): 400" in md
