"""Loop hafnians on MI355X (gfx950): the hot path of arXiv:2108.01622.

C ABI: include/lhaf.h, built into paper_2108_01622_amd/_lib/liblhaf.so.
Python: ``paper_2108_01622_amd.api`` (torch tensors in, torch tensors out).
Workload generators: ``paper_2108_01622_amd.inputs`` (no GPU needed).
"""
__all__ = ["api", "inputs", "build"]


def __getattr__(name):
    if name in ("lhaf", "lhaf_repeated", "lhaf_batched", "lhaf_backward", "lhaf_autograd",
                "LhafFunction", "lhaf_batched_workspace"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
