"""GPU parity of lhaf_mixed (mixed-state lhafmix, App. B.2) with the oracle:
the definition on the explicitly repeated matrix (small), the paper's lhafmix
sum in double (moderate), and the library's greedy repeated route."""
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


def rel(a, b):
    return abs(complex(a) - complex(b)) / max(abs(complex(b)), 1e-300)


@pytest.mark.parametrize("mode", ["fds", "et"])
@pytest.mark.parametrize("n", [[1, 0, 2], [2, 2, 1], [3, 0, 0], [1, 1, 1, 1], [0, 0], [0, 2, 0, 3]])
def test_mixed_small_vs_definition(T, api, orc, n, mode):
    M = len(n)
    A, g, _ = I.mixed_state(M, 11)
    got, err = api.lhaf_mixed(dev(T, A), dev(T, g), n, sum=mode, return_error=True)
    want = orc.lhafmix(A, g, n, method="explicit", prec="f128") if sum(n) else 1.0
    assert rel(got.item(), want) < 1e-11, (got.item(), want)
    assert abs(got.item() - want) <= err.item() + 1e-300


@pytest.mark.parametrize("inst", [0, 1])
def test_mixed_state_moderate(T, api, orc, inst):
    """M = 14 modes, photon numbers 0..3 (N = 2 sum n up to 40 after the cap)."""
    A, g, n = I.mixed_state(14, inst)
    while 2 * n.sum() > 40:
        n[np.argmax(n)] -= 1
    # reference: the oracle's lhafmix sum (explicit powers, Neumaier), whose
    # own error is far below the kernels' (6.6e-11 against __float128 on
    # instance 0, where the pairing (i, M+i) has kappa = 4.4e6)
    want, ab = orc.lhafmix(A, g, n, mode="fds", prec="f64", with_abs=True)
    got, err = api.lhaf_mixed(dev(T, A), dev(T, g), n, return_error=True)
    got, err = got.item(), err.item()
    # the library's estimate takes a per-term rounding of 8(m+1) u of
    # |c_t f_t|, so the bound scales with this pairing's kappa (instance 0:
    # kappa 4.4e6, m = 20, measured 6.6e-8 relative = 6 (m+1) u kappa; the
    # double-double recurrences of acc="ddc" are tested on this case in
    # test_gpu_compensated.py)
    assert abs(got - want) <= err, (got, want, err)
    assert rel(got, want) < max(1e-10, 2e-14 * ab / abs(want))
    # the greedy pairing of the same (n, n) pattern is far better conditioned
    v_g, ab_g = orc.lhaf_repeated(A, g, np.concatenate([n, n]), method="sum", mode="fds",
                                  prec="f64", with_abs=True)
    greedy = api.lhaf(dev(T, A), dev(T, g), r=np.concatenate([n, n])).item()
    assert rel(greedy, v_g) < max(1e-10, 1e-15 * ab_g / abs(v_g))
    et = api.lhaf_mixed(dev(T, A), dev(T, g), n, sum="et").item()
    want_et, ab_et = orc.lhafmix(A, g, n, mode="et", prec="f64", with_abs=True)
    assert rel(et, want_et) < max(1e-12, 1e-14 * ab_et / abs(want_et))
