"""GPU parity of the adjoint (lhaf_backward) with the oracle's closed forms:
  d lhaf / d gamma_i = lhaf(A without row/col i)
  d lhaf / d A_ij    = lhaf(A without rows/cols i, j) / 2   (i != j; A read as sym(A))
  repeated rows: r_i lhaf(A_{r-e_i}), r_i r_j lhaf(A_{r-e_i-e_j}) / 2,
                 C(r_i, 2) lhaf(A_{r-2e_i}) on the diagonal
and with identities that hold at any size (row expansion, Euler homogeneity,
exact central differences: lhaf is affine in each symmetric entry).
Returned values follow PyTorch's convention: grad_out * conj(derivative)."""
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


def rel(a, b):
    return abs(complex(a) - complex(b)) / max(abs(complex(b)), 1e-300)


def dev(T, x):
    return T.as_tensor(np.ascontiguousarray(x), dtype=T.complex128, device="cuda")


def grads(T, api, A, g, r=None, mode="fds"):
    one = T.ones(1, dtype=T.complex128, device="cuda")
    dA, dg = api.lhaf_backward(dev(T, A)[None], dev(T, g)[None], one, r=r, sum=mode)
    return np.conj(dA[0].cpu().numpy()), np.conj(dg[0].cpu().numpy())


@pytest.mark.parametrize("mode", ["fds", "et"])
@pytest.mark.parametrize("N", [2, 3, 5, 8, 11])
def test_closed_forms_small(T, api, orc, N, mode):
    A, g = I.random_symmetric(N, 7000 + N)
    A = A.copy()
    np.fill_diagonal(A, 0.3 - 0.2j)
    dA, dg = grads(T, api, A, g, mode=mode)
    for i in range(N):
        want = orc.lhaf_memo(*orc.remove(A, g, [i]), prec="f128")
        assert rel(dg[i], want) < 1e-10, ("gamma", i)
        assert abs(dA[i, i]) < 1e-13
        for j in range(i + 1, N):
            want = 0.5 * orc.lhaf_memo(*orc.remove(A, g, [i, j]), prec="f128")
            assert rel(dA[i, j], want) < 1e-10, (i, j)
            assert rel(dA[j, i], want) < 1e-10, (j, i)


def test_gaussian_state_16(T, api, orc):
    A, g = I.single16()
    dA, dg = grads(T, api, A, g)
    for i in (0, 7, 15):
        assert rel(dg[i], orc.lhaf_memo(*orc.remove(A, g, [i]), prec="f128")) < 1e-10
    for (i, j) in ((0, 1), (3, 12), (14, 15)):
        assert rel(dA[i, j], 0.5 * orc.lhaf_memo(*orc.remove(A, g, [i, j]), prec="f128")) < 1e-10


def reduce_r(r, *idx):
    r = list(r)
    for i in idx:
        r[i] -= 1
    return r


@pytest.mark.parametrize("r", [[2, 1], [3, 2, 1], [2, 1, 0, 3], [4, 1], [2, 2, 1]])
def test_repeated_closed_forms(T, api, orc, r):
    M = len(r)
    A, g = I.random_symmetric(M, 8000 + 17 * sum(r) + M)
    dA, dg = grads(T, api, A, g, r=r)

    def lr(rr):
        if sum(rr) == 0:
            return 1.0
        return orc.lhaf_repeated(A, g, rr, method="explicit", prec="f128")

    for i in range(M):
        if r[i] == 0:
            assert abs(dg[i]) < 1e-13 and np.all(np.abs(dA[i]) < 1e-13)
            continue
        assert rel(dg[i], r[i] * lr(reduce_r(r, i))) < 1e-10, ("gamma", i)
        if r[i] >= 2:
            assert rel(dA[i, i], math.comb(r[i], 2) * lr(reduce_r(r, i, i))) < 1e-10, ("diag", i)
        for j in range(M):
            if j != i and r[j] > 0:
                want = 0.5 * r[i] * r[j] * lr(reduce_r(r, i, j))
                assert rel(dA[i, j], want) < 1e-10, (i, j)


def test_identities_n24(T, api, orc):
    """Row expansion gamma_i dg_i + sum_j A_ij (2 dA_ij) = lhaf for every i;
    Euler: sum_{i<j} A_ij (2 dA_ij) + sum_i gamma_i dg_i / 2 = (N/2) lhaf."""
    A, g = I.gaussian_state_matrix(24, np.random.Generator(np.random.PCG64(2424)))
    val = api.lhaf(dev(T, A), dev(T, g)).item()
    dA, dg = grads(T, api, A, g)
    N = 24
    for i in range(N):
        s = g[i] * dg[i] + sum(A[i, j] * 2 * dA[i, j] for j in range(N) if j != i)
        assert rel(s, val) < 1e-10, i
    e = sum(A[i, j] * 2 * dA[i, j] for i in range(N) for j in range(i + 1, N)) + 0.5 * np.dot(g, dg)
    assert rel(e, N / 2 * val) < 1e-10


def test_central_differences(T, api):
    """lhaf is affine in each symmetric entry and in each gamma_i, so a central
    difference has no truncation error; h = 1e-6 leaves roundoff ~ eps/h."""
    A, g = I.gaussian_state_matrix(14, np.random.Generator(np.random.PCG64(1414)))
    dA, dg = grads(T, api, A, g)
    h = 1e-6
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(6):
        i, j = sorted(rng.choice(14, 2, replace=False))
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Ap[j, i] += h
        Am[i, j] -= h
        Am[j, i] -= h
        fd = (api.lhaf(dev(T, Ap), dev(T, g)).item() - api.lhaf(dev(T, Am), dev(T, g)).item()) / (2 * h)
        assert rel(fd, 2 * dA[i, j]) < 1e-6, (i, j)
    for i in (0, 9):
        gp, gm = g.copy(), g.copy()
        gp[i] += h
        gm[i] -= h
        fd = (api.lhaf(dev(T, A), dev(T, gp)).item() - api.lhaf(dev(T, A), dev(T, gm)).item()) / (2 * h)
        assert rel(fd, dg[i]) < 1e-6


def test_batched_dense_and_grad_out(T, api, orc):
    rng = np.random.Generator(np.random.PCG64(99))
    mats = [I.gaussian_state_matrix(n, rng) for n in (10, 10, 10)]
    A = np.stack([m[0] for m in mats])
    g = np.stack([m[1] for m in mats])
    go = np.array([1.0, 0.5 - 2j, -1j])
    dA, dg = api.lhaf_backward(dev(T, A), dev(T, g), dev(T, go))
    dA, dg = dA.cpu().numpy(), dg.cpu().numpy()
    for b in range(3):
        want = orc.lhaf_memo(*orc.remove(A[b], g[b], [4]), prec="f128")
        assert rel(dg[b, 4], go[b] * np.conj(want)) < 1e-10
        want = 0.5 * orc.lhaf_memo(*orc.remove(A[b], g[b], [1, 8]), prec="f128")
        assert rel(dA[b, 1, 8], go[b] * np.conj(want)) < 1e-10


def test_shared_base_accumulates(T, api, orc):
    base = I.state100(0)
    Bm, gam = base["B"], base["gamma"]
    idx = [np.array([3, 7, 10, 20, 51, 60]), np.array([7, 10, 33, 51]), np.array([3, 10, 99])]
    off = np.array([0, 6, 10, 13], dtype=np.int64)
    go = np.ones(3, dtype=complex)
    dA, dg = api.lhaf_backward(dev(T, Bm), dev(T, gam), dev(T, go), idx=np.concatenate(idx), idx_off=off)
    dA, dg = np.conj(dA.cpu().numpy()), np.conj(dg.cpu().numpy())
    # gamma_10 appears in all three problems
    want = 0.0
    for ix in idx:
        sub = list(ix)
        k = sub.index(10)
        As, gs = Bm[np.ix_(ix, ix)], gam[ix]
        want += orc.lhaf_memo(*orc.remove(As, gs, [k]), prec="f128")
    assert rel(dg[10], want) < 1e-10
    # entry (7, 51) appears in problems 0 and 1
    want = 0.0
    for ix in idx[:2]:
        sub = list(ix)
        As, gs = Bm[np.ix_(ix, ix)], gam[ix]
        want += 0.5 * orc.lhaf_memo(*orc.remove(As, gs, [sub.index(7), sub.index(51)]), prec="f128")
    assert rel(dA[7, 51], want) < 1e-10
    assert abs(dA[0, 1]) == 0 and abs(dg[1]) == 0


def test_autograd_gradcheck(T, api):
    A, g = I.random_symmetric(6, 606)
    At = dev(T, A).requires_grad_(True)
    gt = dev(T, g).requires_grad_(True)
    assert T.autograd.gradcheck(lambda a, b: api.lhaf_autograd(a, b), (At, gt), eps=1e-6, atol=1e-7,
                                rtol=1e-5, fast_mode=False)


def _saved_vs_recomputed(T, api, A, g, idx=None, idx_off=None, r=None, mode="fds", go=None):
    At, gt = dev(T, A), dev(T, g)
    off = idx_off if idx_off is not None else np.arange(A.shape[0] + 1, dtype=np.int64) * A.shape[1]
    count = api.lhaf_saved_count(off, r, sum=mode)
    store = T.empty(count, dtype=T.complex128, device="cuda")
    nb = len(off) - 1
    gout = dev(T, go if go is not None else np.ones(nb))
    out_s = api.lhaf_batched(At, gt, idx=idx, idx_off=idx_off, r=r, sum=mode, saved=store)
    out = api.lhaf_batched(At, gt, idx=idx, idx_off=idx_off, r=r, sum=mode)
    assert T.equal(out_s, out)  # saving does not change the forward result
    dA_s, dg_s = api.lhaf_backward(At, gt, gout, idx=idx, idx_off=idx_off, r=r, sum=mode, saved=store)
    dA, dg = api.lhaf_backward(At, gt, gout, idx=idx, idx_off=idx_off, r=r, sum=mode)
    # both paths are correct to rounding; the ET sum cancels more than FDS
    tol = 1e-12 if mode == "fds" else 1e-10
    scale_A = max(float(dA.abs().max()), 1e-300)
    scale_g = max(float(dg.abs().max()), 1e-300)
    assert float((dA_s - dA).abs().max()) / scale_A < tol
    assert float((dg_s - dg).abs().max()) / scale_g < tol


@pytest.mark.parametrize("mode", ["fds", "et"])
def test_saved_store_dense(T, api, mode):
    """Backward from the forward's coefficient store equals the backward that
    recomputes the Hessenberg phase (N = 24, 25 and 7 in one dense batch of
    the largest size is not possible, so three batches)."""
    rng = np.random.Generator(np.random.PCG64(4242))
    for N, cnt in ((24, 3), (25, 2), (7, 4)):
        mats = [I.gaussian_state_matrix(N, rng) for _ in range(cnt)]
        A = np.stack([m[0] for m in mats])
        g = np.stack([m[1] for m in mats])
        _saved_vs_recomputed(T, api, A, g, mode=mode, go=np.linspace(1, 2, cnt) - 0.5j)


def test_saved_store_shared_and_repeated(T, api):
    base = I.state100(0)
    Bm, gam = base["B"], base["gamma"]
    idx = np.concatenate([np.arange(0, 30, 2), np.arange(5, 41), np.array([3, 10, 99])])
    off = np.array([0, 15, 51, 54], dtype=np.int64)
    _saved_vs_recomputed(T, api, Bm, gam, idx=idx, idx_off=off)
    r = np.array([2, 1, 3, 0, 1, 2, 1], dtype=np.int32)
    A, g = I.random_symmetric(7, 777)
    _saved_vs_recomputed(T, api, A[None], g[None], r=r)


def test_saved_store_errors(T, api):
    from paper_2108_01622_amd._binding import LhafError
    A, g = I.random_symmetric(12, 1212)
    At, gt = dev(T, A)[None], dev(T, g)[None]
    count = api.lhaf_saved_count(np.array([0, 12]))
    small = T.empty(count - 1, dtype=T.complex128, device="cuda")
    with pytest.raises(LhafError, match="workspace too small"):
        api.lhaf_batched(At, gt, saved=small)
    # a term range needs a store of that range only
    assert api.lhaf_saved_count(np.array([0, 12]), term_begin=3, term_end=8) == 5 * 6
    part = T.empty(5 * 6 - 1, dtype=T.complex128, device="cuda")
    with pytest.raises(LhafError, match="workspace too small"):
        api.lhaf_batched(At, gt, saved=part, term_begin=3, term_end=8, scaled=False)
    with pytest.raises(LhafError, match="workspace too small"):
        api.lhaf_backward(At, gt, T.ones(1, dtype=T.complex128, device="cuda"), saved=small)


def test_autograd_modes_agree(T, api):
    """The three autograd modes (fused pass, recomputation, coefficient store)
    give the same values and gradients to rounding."""
    rng = np.random.Generator(np.random.PCG64(31))
    mats = [I.gaussian_state_matrix(16, rng) for _ in range(3)]
    A = np.stack([m[0] for m in mats])
    g = np.stack([m[1] for m in mats])
    res = []
    for mode in ("fused", "store", "recompute"):
        At = dev(T, A).requires_grad_(True)
        gt = dev(T, g).requires_grad_(True)
        out = api.lhaf_autograd(At, gt, mode=mode)
        (out * dev(T, np.array([1.0, -1j, 0.5]))).sum().real.backward()
        res.append((out.detach().clone(), At.grad.clone(), gt.grad.clone()))
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert float((a - b).abs().max()) <= 1e-12 * float(b.abs().max())


@pytest.mark.parametrize("mode", ["fds", "et"])
@pytest.mark.parametrize("acc", ["dd", "fp64"])
def test_fused_pass_matches_separate_passes(T, api, orc, mode, acc):
    """The fused pass (values and per-problem gradients in one launch) against
    lhaf_batched and lhaf_backward on a shared base with index lists of mixed
    sizes (several tiles in one launch) and on a repeated pattern; the values
    also against the oracle."""
    base = I.state100(0)
    Bm, gam = dev(T, base["B"]), dev(T, base["gamma"])
    lists = [np.arange(0, 30, 2), np.arange(5, 41), np.array([3, 10, 99]), np.arange(60, 78)]
    idx = np.concatenate(lists)
    off = np.cumsum([0] + [len(x) for x in lists]).astype(np.int64)
    go = dev(T, np.array([1.0, 0.5 - 0.25j, -2j, 0.75]))
    grads = T.empty(api.lhaf_grads_count(off), dtype=T.complex128, device="cuda")
    v_f, e_f = api.lhaf_batched(Bm, gam, idx=idx, idx_off=off, sum=mode, acc=acc, grads=grads,
                                return_error=True)
    v_s, e_s = api.lhaf_batched(Bm, gam, idx=idx, idx_off=off, sum=mode, acc=acc,
                                return_error=True)
    dA_f, dg_f = api.lhaf_backward(Bm, gam, go, idx=idx, idx_off=off, sum=mode, grads=grads)
    dA_s, dg_s = api.lhaf_backward(Bm, gam, go, idx=idx, idx_off=off, sum=mode)
    tol = 1e-12 if mode == "fds" else 1e-10
    assert float((v_f - v_s).abs().max()) <= tol * float(v_s.abs().max())
    assert float((dA_f - dA_s).abs().max()) <= tol * float(dA_s.abs().max())
    assert float((dg_f - dg_s).abs().max()) <= tol * float(dg_s.abs().max())
    vv = v_f.cpu().numpy()
    for b in (0, 2):
        ix = lists[b]
        want = orc.lhaf_memo(base["B"][np.ix_(ix, ix)], base["gamma"][ix], prec="f128") \
            if len(ix) <= 16 else None
        if want is not None:
            assert abs(vv[b] - want) <= max(1e-10 * abs(want), 4 * float(e_f[b])), b
    # repeated rows, dense stack of one
    A, g = I.random_symmetric(7, 777)
    r = np.array([2, 1, 3, 0, 1, 2, 1], dtype=np.int32)
    At, gt = dev(T, A)[None], dev(T, g)[None]
    grads = T.empty(api.lhaf_grads_count(np.array([0, 7]), r), dtype=T.complex128, device="cuda")
    v_f = api.lhaf_batched(At, gt, r=r, sum=mode, acc=acc, grads=grads)
    want = orc.lhaf_memo(*orc.repeat_matrix(A, g, r), prec="f128")
    assert abs(v_f.item() - want) <= 1e-10 * abs(want)
    one = T.ones(1, dtype=T.complex128, device="cuda")
    dA_f, dg_f = api.lhaf_backward(At, gt, one, r=r, sum=mode, grads=grads)
    dA_s, dg_s = api.lhaf_backward(At, gt, one, r=r, sum=mode)
    assert float((dA_f - dA_s).abs().max()) <= tol * float(dA_s.abs().max())
    assert float((dg_f - dg_s).abs().max()) <= tol * float(dg_s.abs().max())


def test_fused_pass_term_slices(T, api):
    """Fused pass over term slices: raw value partials and gradient shares
    add up to the full value and gradient."""
    rng = np.random.Generator(np.random.PCG64(5151))
    mats = [I.gaussian_state_matrix(18, rng) for _ in range(2)]
    A = dev(T, np.stack([m[0] for m in mats]))
    g = dev(T, np.stack([m[1] for m in mats]))
    off = np.arange(3, dtype=np.int64) * 18
    Tn = int(api.Bn.term_count(18))
    go = dev(T, np.array([1.0, -1j]))
    v_full = api.lhaf_batched(A, g)
    dA_full, dg_full = api.lhaf_backward(A, g, go)
    grads = T.empty(api.lhaf_grads_count(off), dtype=T.complex128, device="cuda")
    vs = T.zeros_like(v_full)
    sA, sg = T.zeros_like(dA_full), T.zeros_like(dg_full)
    for a, b in ((0, 3), (3, Tn // 2), (Tn // 2, Tn)):
        vs += api.lhaf_batched(A, g, term_begin=a, term_end=b, scaled=False, grads=grads)
        pA, pg = api.lhaf_backward(A, g, go, grads=grads)
        sA += pA
        sg += pg
    vs *= 2.0 ** -9
    assert float((vs - v_full).abs().max()) <= 1e-12 * float(v_full.abs().max())
    assert float((sA - dA_full).abs().max()) <= 1e-12 * float(dA_full.abs().max())
    assert float((sg - dg_full).abs().max()) <= 1e-12 * float(dg_full.abs().max())


@pytest.mark.parametrize("mode", ["fds", "et"])
def test_backward_term_slices_add_up(T, api, mode):
    """The gradient of disjoint term ranges covering all terms adds up to the
    full gradient (each term is independent), with and without the store,
    for a dense batch of mixed sizes and a shared base with index lists."""
    rng = np.random.Generator(np.random.PCG64(5150))
    mats = [I.gaussian_state_matrix(14, rng) for _ in range(3)]
    A = np.stack([m[0] for m in mats])
    g = np.stack([m[1] for m in mats])
    At, gt = dev(T, A), dev(T, g)
    go = dev(T, np.array([1.0, 0.25 - 1j, 2j]))
    dA, dg = api.lhaf_backward(At, gt, go, sum=mode)
    Tn = int(api.Bn.term_count(14, sum=mode))
    cuts = [0, 1, 17, Tn // 2 + 5, Tn - 3, Tn]
    assert cuts == sorted(cuts) and len(set(cuts)) == len(cuts)
    off = np.arange(4, dtype=np.int64) * 14
    sA, sg = T.zeros_like(dA), T.zeros_like(dg)
    sA2, sg2 = T.zeros_like(dA), T.zeros_like(dg)
    for a, b in zip(cuts[:-1], cuts[1:]):
        pA, pg = api.lhaf_backward(At, gt, go, sum=mode, term_begin=a, term_end=b)
        sA += pA
        sg += pg
        store = T.empty(api.lhaf_saved_count(off, sum=mode, term_begin=a, term_end=b),
                        dtype=T.complex128, device="cuda")
        api.lhaf_batched(At, gt, sum=mode, term_begin=a, term_end=b, scaled=False, saved=store)
        qA, qg = api.lhaf_backward(At, gt, go, sum=mode, term_begin=a, term_end=b, saved=store)
        sA2 += qA
        sg2 += qg
    tol = 1e-12 if mode == "fds" else 1e-10
    for x, y in ((sA, dA), (sg, dg), (sA2, dA), (sg2, dg)):
        assert float((x - y).abs().max()) <= tol * float(y.abs().max())
    # a range past the end contributes nothing
    zA, zg = api.lhaf_backward(At, gt, go, sum=mode, term_begin=Tn, term_end=Tn + 5)
    assert float(zA.abs().max()) == 0.0 and float(zg.abs().max()) == 0.0


def test_dense_stack_with_index_lists(T, api, orc):
    """A dense stack with index lists: problem b is the submatrix of A_b on
    the rows idx_b (a permuted subset of fewer rows than A_b has).  Gradients
    land on those rows of dA_b / dgamma_b; every other entry is 0."""
    rng = np.random.Generator(np.random.PCG64(8080))
    M = 12
    mats = [I.random_symmetric(M, 8100 + b) for b in range(3)]
    A = np.stack([m[0] for m in mats])
    g = np.stack([m[1] for m in mats])
    idx = [rng.permutation(M)[:k] for k in (9, 12, 7)]
    off = np.array([0, 9, 21, 28], dtype=np.int64)
    go = np.array([1.0, -0.5 + 1j, 0.75j])
    dA, dg = api.lhaf_backward(dev(T, A), dev(T, g), dev(T, go), idx=np.concatenate(idx), idx_off=off)
    dA, dg = dA.cpu().numpy(), dg.cpu().numpy()
    for b in range(3):
        ix = list(idx[b])
        As, gs = A[b][np.ix_(ix, ix)], g[b][ix]
        As = 0.5 * (As + As.T)
        unused = sorted(set(range(M)) - set(ix))
        for x in unused:
            assert dg[b, x] == 0 and np.all(dA[b, x, :] == 0) and np.all(dA[b, :, x] == 0)
        for k in (0, len(ix) - 1):
            want = go[b] * np.conj(orc.lhaf_memo(*orc.remove(As, gs, [k]), prec="f128"))
            assert rel(dg[b, ix[k]], want) < 1e-10, (b, k)
        k, l = 1, len(ix) - 2
        want = go[b] * np.conj(0.5 * orc.lhaf_memo(*orc.remove(As, gs, [k, l]), prec="f128"))
        assert rel(dA[b, ix[k], ix[l]], want) < 1e-10
        assert rel(dA[b, ix[l], ix[k]], want) < 1e-10
        assert np.all(np.diag(dA[b]) == 0)
