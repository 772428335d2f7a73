"""Contracts of the C ABI beyond parity: every schedule gives the same
result to rounding and a fixed schedule gives the same bits on every call
(values and gradients); non-finite inputs give NaN with err_est = +Inf for
the problem that reads them and leave the others untouched."""
import math

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


def dev(T, x):
    return T.as_tensor(np.ascontiguousarray(x), dtype=T.complex128, device="cuda")


def _batch(T):
    rng = np.random.Generator(np.random.PCG64(9090))
    mats = [I.gaussian_state_matrix(n, rng) for n in (24,) * 5]
    A = np.stack([m[0] for m in mats])
    g = np.stack([m[1] for m in mats])
    return dev(T, A), dev(T, g)


@pytest.mark.parametrize("mode", ["fds", "et"])
def test_schedules_agree_and_repeat_bitwise(T, api, mode):
    from paper_2108_01622_amd import _binding as Bn
    A, g = _batch(T)
    nsched = int(Bn.lib().lhaf_schedule_count())
    assert nsched >= 2
    go = dev(T, np.array([1.0, -0.5j, 0.25, 2.0, 1 + 1j]))
    vals, grads = [], []
    for s in range(nsched):
        v1 = api.lhaf_batched(A, g, sum=mode, schedule=s)
        v2 = api.lhaf_batched(A, g, sum=mode, schedule=s)
        assert T.equal(v1, v2), f"schedule {s}: values differ between calls"
        d1 = api.lhaf_backward(A, g, go, sum=mode, schedule=s)
        d2 = api.lhaf_backward(A, g, go, sum=mode, schedule=s)
        assert T.equal(d1[0], d2[0]) and T.equal(d1[1], d2[1]), f"schedule {s}: gradients differ"
        vals.append(v1)
        grads.append(d1)
    tol = 1e-13 if mode == "fds" else 1e-11
    for s in range(1, nsched):
        assert float((vals[s] - vals[0]).abs().max()) <= tol * float(vals[0].abs().max()), s
        for a, b in zip(grads[s], grads[0]):
            assert float((a - b).abs().max()) <= 10 * tol * float(b.abs().max()), s


@pytest.mark.parametrize("acc", ["dd", "fp64"])
def test_nonfinite_inputs(T, api, acc):
    A, g = _batch(T)
    ref, ref_err = api.lhaf_batched(A, g, acc=acc, return_error=True)
    A2, g2 = A.clone(), g.clone()
    A2[1, 3, 7] = complex(math.nan, 0.0)      # read (off-diagonal)
    g2[3, 5] = complex(math.inf, 1.0)         # read (loop weight)
    A2[4, 2, 2] = complex(math.nan, math.nan)  # plain problem: the diagonal is not read
    out, err = api.lhaf_batched(A2, g2, acc=acc, return_error=True)
    out, err = out.cpu().numpy(), err.cpu().numpy()
    ref, ref_err = ref.cpu().numpy(), ref_err.cpu().numpy()
    for b in (1, 3):
        assert math.isnan(out[b].real) and math.isnan(out[b].imag), b
        assert err[b] == math.inf, b
    for b in (0, 2, 4):
        assert out[b] == ref[b] and err[b] == ref_err[b], b
    # single-problem entry points follow the same rule
    v, e = api.lhaf(A2[1], g2[1], return_error=True)
    assert math.isnan(v.item().real) and e.item() == math.inf
    r = np.array([2, 1, 1, 0, 2], dtype=np.int32)
    Ar, gr = I.random_symmetric(5, 5151)
    Ar = Ar.copy()
    Ar[0, 0] = math.inf  # repeated problems read A_ii (coupling of two copies)
    v, e = api.lhaf(dev(T, Ar), dev(T, gr), r=r, return_error=True)
    assert math.isnan(v.item().real) and e.item() == math.inf
