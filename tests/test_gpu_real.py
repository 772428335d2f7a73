"""GPU parity of lhaf_real (real FP64 kernel for real symmetric matrices,
e.g. the non-negative ones of the MIS independence proposal, App. C) with the
oracle's definition on the same matrix, and with the complex kernels."""
import numpy as np
import pytest

from paper_2108_01622_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def api():
    from paper_2108_01622_amd import api as A
    return A


def nonneg(rng, N):
    A = rng.uniform(0.0, 1.0, size=(N, N))
    A = 0.5 * (A + A.T)
    return A, rng.uniform(0.0, 1.0, size=N)


def rel(a, b):
    return abs(complex(a) - complex(b)) / max(abs(complex(b)), 1e-300)


@pytest.mark.parametrize("mode", ["fds", "et"])
@pytest.mark.parametrize("N", [1, 2, 3, 6, 9, 12])
def test_real_small_vs_definition(T, api, orc, N, mode):
    rng = np.random.Generator(np.random.PCG64(3000 + N))
    A, g = nonneg(rng, N)
    got, err = api.lhaf_real(T.as_tensor(A, device="cuda"), T.as_tensor(g, device="cuda"), sum=mode,
                             return_error=True)
    want = orc.lhaf_memo(A.astype(complex), g.astype(complex), prec="f128")
    assert rel(got.item(), want) < 1e-12
    assert abs(got.item() - want.real) <= err.item() + 1e-300


def test_real_signed_and_repeated(T, api, orc):
    rng = np.random.Generator(np.random.PCG64(3100))
    A = rng.normal(size=(5, 5))
    A = A + A.T
    g = rng.normal(size=5)
    r = [2, 0, 3, 1, 1]
    got = api.lhaf_real(T.as_tensor(A, device="cuda"), T.as_tensor(g, device="cuda"), r=r).item()
    want = orc.lhaf_repeated(A.astype(complex), g.astype(complex), r, method="explicit", prec="f128")
    assert rel(got, want) < 1e-12
    assert abs(api.lhaf_real(T.zeros((0, 0), dtype=T.float64, device="cuda"),
                             T.zeros(0, dtype=T.float64, device="cuda")).item() - 1.0) == 0.0


@pytest.mark.parametrize("N", [24, 40])
def test_real_matches_complex_kernel(T, api, N):
    """Non-negative N x N matrix: the real kernel against the complex kernel
    on the same entries (both within their error estimates)."""
    rng = np.random.Generator(np.random.PCG64(3200 + N))
    A, g = nonneg(rng, N)
    A *= 0.2
    got, e1 = api.lhaf_real(T.as_tensor(A, device="cuda"), T.as_tensor(g, device="cuda"),
                            return_error=True)
    ref, e2 = api.lhaf(T.as_tensor(A.astype(complex), device="cuda"),
                       T.as_tensor(g.astype(complex), device="cuda"), return_error=True)
    assert abs(got.item() - ref.item()) <= e1.item() + e2.item()
    assert rel(got.item(), ref.item()) < 1e-11


@pytest.mark.parametrize("N", [24, 40])
def test_real_vs_stored_oracle(T, api, N):
    """Real non-negative N = 24 / 40 lhaf in the real kernel against the
    oracle's FDS sum stored in tests/golden (oracle only); bound
    max(1e-11, 4 kappa u)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))
    key = f"real{N}/0"
    if key not in gold:
        pytest.skip(f"no stored oracle value for {key}")
    A, g = I.real_nonneg(N, 0)
    got = api.lhaf_real(T.as_tensor(A, device="cuda"), T.as_tensor(g, device="cuda")).item()
    want = complex(*gold[key]["value"])
    assert abs(want.imag) <= 1e-14 * abs(want.real)
    kappa = gold[key]["abs_sum"] / abs(want)
    r = abs(got - want.real) / abs(want)
    print(f"[measure] {key} rel {r:.3e} kappa {kappa:.3e}", flush=True)
    assert r < max(1e-11, 4 * kappa * 2.0 ** -53)
