"""Build the HIP library in-tree: paper_2108_01622_amd/_lib/liblhaf.so (gfx950).

    python -m paper_2108_01622_amd.build [--force] [-j N]   # or build.build()

The library is self-contained (host planner + kernels + C ABI) and links
only against the HIP runtime.  The persistent kernels are compiled one
(family, register tile) per translation unit (csrc/lhaf_tile.hip with
-DLH_FAMILY / -DLH_TILE), in parallel; objects go to _build/ and are reused
when neither the command nor any source they include has changed (force=True
recompiles everything).
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(HERE, "_lib")
OBJDIR = os.path.join(ROOT, "_build", "lhaf")
LIB = os.path.join(LIBDIR, "liblhaf.so")
ARCH = os.environ.get("LHAF_OFFLOAD_ARCH", "gfx950")

# family 4: the forward with compensated recurrences (its kernels are in lhaf_forward.hip)
FAMILIES = {0: "lhaf_forward.hip", 1: "lhaf_backward.hip", 2: "lhaf_multi.hip", 3: "lhaf_real.hip",
            4: "lhaf_forward.hip"}
TILES = range(1, 9)
BWD_SPLIT_TILES = (4, 5)  # backward tiles with a staged and an unstaged instance
_COMMON = ["lhaf.h", "lhaf_device.h", "lhaf_internal.h", "lhaf_forward.hip", "lhaf_launch.h"]


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _src(name: str) -> str:
    return os.path.join(INCLUDE if name == "lhaf.h" else CSRC, name)


def _flags(extra=()):
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # keep hipcc from forming packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC, "-Wno-unused-result", *extra]


def _units(extra=()):
    """(object path, compile command, source files it depends on)."""
    units = []
    cc = hipcc()
    for fam, ffile in FAMILIES.items():
        deps = _COMMON + ["lhaf_tile.hip"] + ([ffile] if fam else [])
        for b in sorted(TILES, reverse=True):  # largest tiles compile longest: start them first
            # the backward tile with both an LDS-staged and an unstaged instance
            # compiles them in separate units, so that the two occupancy targets
            # do not meet in shared device functions
            parts = [("", 0)] if not (fam == 1 and b in BWD_SPLIT_TILES) else [("", 1), ("u", 2)]
            for suffix, unit in parts:
                obj = os.path.join(OBJDIR, f"tile_f{fam}_b{b}{suffix}.o")
                cmd = [cc, *_flags(extra), f"-DLH_FAMILY={fam}", f"-DLH_TILE={b}",
                       f"-DLH_BWD_UNIT={unit}", "-c", _src("lhaf_tile.hip"), "-o", obj]
                units.append((obj, cmd, deps))
    api_deps = sorted(set(_COMMON + list(FAMILIES.values()) + ["lhaf_api.hip"]))
    units.append((os.path.join(OBJDIR, "api.o"),
                  [cc, *_flags(extra), "-c", _src("lhaf_api.hip"), "-o", os.path.join(OBJDIR, "api.o")],
                  api_deps))
    units.append((os.path.join(OBJDIR, "planner.o"),
                  [cc, *_flags(extra), "-c", _src("planner.cpp"), "-o", os.path.join(OBJDIR, "planner.o")],
                  ["planner.cpp", "lhaf_internal.h"]))
    return units


def _stamp(cmd, deps) -> str:
    h = hashlib.sha256(" ".join(cmd).encode())
    for d in sorted(deps):
        h.update(d.encode())
        h.update(open(_src(d), "rb").read())
    return h.hexdigest()


def _compile(obj, cmd, deps, force, verbose):
    stamp_path = obj + ".stamp"
    stamp = _stamp(cmd, deps)
    if not force and os.path.exists(obj) and os.path.exists(stamp_path) and \
            open(stamp_path).read() == stamp:
        return obj, 0.0, False
    t = time.time()
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the device-only target feature: not an error
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    if out.strip() and verbose:
        print(out, flush=True)
    open(stamp_path, "w").write(stamp)
    return obj, time.time() - t, True


def build(verbose: bool = False, extra=(), force: bool = False, jobs: int | None = None) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    os.makedirs(OBJDIR, exist_ok=True)
    units = _units(extra)
    jobs = jobs or int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 4)
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, 16))) as ex:
        futs = [ex.submit(_compile, o, c, d, force, verbose) for o, c, d in units]
        done = [f.result() for f in futs]
    rebuilt = [(os.path.basename(o), dt) for o, dt, r in done if r]
    tmp = LIB + ".tmp"
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *[o for o, _, _ in units], "-o", tmp]
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    if verbose:
        slow = sorted(rebuilt, key=lambda x: -x[1])[:4]
        print(f"built {LIB}: {len(rebuilt)}/{len(units)} units compiled in {time.time() - t0:.1f} s "
              f"(slowest: {', '.join(f'{n} {dt:.0f}s' for n, dt in slow)})", flush=True)
    return LIB


if __name__ == "__main__":
    args = sys.argv[1:]
    force = "--force" in args
    jobs = None
    if "-j" in args:
        jobs = int(args[args.index("-j") + 1])
    extra = [a for i, a in enumerate(args) if a != "--force" and a != "-j" and (i == 0 or args[i - 1] != "-j")]
    build(verbose=True, extra=extra, force=force, jobs=jobs)
    print(LIB)
