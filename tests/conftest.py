import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_sessionstart(session):
    """For GPU runs, import torch and create the HIP context before any test
    starts, so per-test time limits do not include a cold first import."""
    expr = session.config.getoption("markexpr", default="") or ""
    if "gpu" in expr and "not gpu" not in expr:
        import time
        t = time.time()
        import torch
        ok = torch.cuda.is_available()
        if ok:
            torch.zeros(1, device="cuda").sum().item()
        print(f"[session] torch {torch.__version__} cuda={ok} warm-up {time.time() - t:.1f}s", flush=True)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    O.build()
    O.set_threads(min(8, os.cpu_count() or 1))
    return O
