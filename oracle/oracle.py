"""CPU oracle for complex loop hafnians (Python side).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may use this module; the product path never does.  It shares
no code with the HIP library ``paper_2108_01622_amd``.

Two implementations of the paper's power-trace sums live here:

* ``lhaf_sum`` -- the C++ oracle (``lhaf_oracle.cpp``): explicit repeated
  matrix products for Tr((CX)^k), double or __float128;
* ``lhaf_eig_sum`` -- numpy: the traces from the eigenvalues of CX, which is
  the route the paper describes (App. B.1, "finding the eigenvalues of CX"),
  batched over terms with ``numpy.linalg.eigvals``.

plus the definition itself (matching enumeration, memoised), Ryser's
permanent, the loop repeated-moment sum, the greedy pair matching of
App. B.3, and exact integer closed forms used as pins.

Term enumeration shared *by specification* (not by code) with the library:
pairs p = 0..H-1 with repeat counts eta_p; mixed-radix digits with pair 0
fastest; FDS halving pair = first pair with odd eta (else pair 0) with radix
floor(eta/2)+1; see ``lhaf_oracle.cpp`` for the coefficients.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblhaf_oracle.so")
_SRC = os.path.join(_HERE, "lhaf_oracle.cpp")


def build(force: bool = False) -> str:
    """Compile the C++ oracle with g++ (OpenMP, libquadmath not needed for
    plain __float128 arithmetic)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _SO + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_lhaf_enum.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp]
        L.orc_lhaf_memo.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp]
        L.orc_lhaf_sum.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ip, ip, ip, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                   ctypes.c_int, dp, dp]
        L.orc_term_count.argtypes = [ctypes.c_int, ip, ctypes.c_int, ctypes.c_int]
        L.orc_term_count.restype = ctypes.c_int64
        L.orc_perm_ryser.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp]
        L.orc_lhaf_rep_moment.argtypes = [ctypes.c_int, dp, dp, ip, ctypes.c_int, dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def _cd(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ci(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _prec(p):
    return {"f64": 0, "f128": 1}[p]


def _result(out, hi_lo):
    hi = complex(out[0], out[1])
    lo = complex(out[2], out[3])
    return (hi, lo) if hi_lo else hi + lo


def pad_odd(A, g):
    """Odd N: append one vertex with zero couplings and loop weight 1; by the
    definition lhaf(A (+) [1]) = lhaf(A)."""
    N = A.shape[0]
    if N % 2 == 0:
        return A, g
    A2 = np.zeros((N + 1, N + 1), dtype=np.complex128)
    A2[:N, :N] = A
    g2 = np.concatenate([np.asarray(g, dtype=np.complex128), [1.0 + 0j]])
    return A2, g2


# ---------------------------------------------------------------------------
# the definition
def lhaf_enum(A, g, prec="f64", hi_lo=False):
    A, pa = _cd(A)
    g, pg = _cd(g)
    out = np.zeros(4)
    rc = lib().orc_lhaf_enum(A.shape[0], pa, pg, _prec(prec), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, rc
    return _result(out, hi_lo)


def lhaf_memo(A, g, prec="f64", hi_lo=False):
    A, pa = _cd(A)
    g, pg = _cd(g)
    out = np.zeros(4)
    rc = lib().orc_lhaf_memo(A.shape[0], pa, pg, _prec(prec), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, rc
    return _result(out, hi_lo)


# ---------------------------------------------------------------------------
# power-trace sums (C++)
def plain_pairs(N):
    """Fixed perfect matching of App. B.1/B.2: position i pairs with N/2 + i."""
    n = N // 2
    return np.arange(n), np.arange(n, 2 * n), np.ones(n, dtype=np.int32)


def lhaf_sum(A, g, pairs=None, mode="fds", halve=True, t0=0, t1=-1, scaled=True, prec="f64",
             hi_lo=False, with_abs=False):
    """Power-trace sum (ET or FDS) over `pairs` = (u, w, eta).  Default pairs:
    the plain matching of the (odd-padded) matrix."""
    if pairs is None:
        A, g = pad_odd(np.asarray(A), np.asarray(g))
        pairs = plain_pairs(A.shape[0])
    u, w, eta = pairs
    A, pa = _cd(A)
    g, pg = _cd(g)
    u, pu = _ci(u)
    w, pw = _ci(w)
    eta, pe = _ci(eta)
    out = np.zeros(4)
    ab = np.zeros(1)
    rc = lib().orc_lhaf_sum(A.shape[0], pa, pg, len(u), pu, pw, pe, 1 if mode == "fds" else 0,
                            1 if halve else 0, int(t0), int(t1), 1 if scaled else 0, _prec(prec),
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            ab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, rc
    r = _result(out, hi_lo)
    return (r, float(ab[0])) if with_abs else r


def term_count(eta, mode="fds", halve=True):
    eta, pe = _ci(eta)
    return int(lib().orc_term_count(len(eta), pe, 1 if mode == "fds" else 0, 1 if halve else 0))


def perm_ryser(B, prec="f64"):
    B, pb = _cd(B)
    out = np.zeros(4)
    rc = lib().orc_perm_ryser(B.shape[0], pb, _prec(prec), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0
    return _result(out, False)


def lhaf_rep_moment(A, g, r, prec="f128"):
    """Loop repeated-moment sum for lhaf(A_r) (prod (r_i+1) terms)."""
    A, pa = _cd(A)
    g, pg = _cd(g)
    r, pr = _ci(r)
    out = np.zeros(4)
    rc = lib().orc_lhaf_rep_moment(A.shape[0], pa, pg, pr, _prec(prec), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0
    return _result(out, False)


# ---------------------------------------------------------------------------
# repeated rows (App. A: A_n repeats row/column i n_i times; the diagonal is
# replaced by the repeated gamma; two copies of mode i couple with A_ii)
def repeat_matrix(A, g, r):
    idx = np.repeat(np.arange(len(r)), np.asarray(r, dtype=np.int64))
    Ar = np.asarray(A)[np.ix_(idx, idx)].copy()
    gr = np.asarray(g)[idx].copy()
    np.fill_diagonal(Ar, gr)
    return Ar, gr


def matched_reps(r):
    """Greedy pair matching (App. B.3).  Ties in the sort are broken by mode
    index (ascending).  Returns (pairs [(m1, m2, eta)], leftover mode or None)."""
    cnt = {i: int(v) for i, v in enumerate(r) if v > 0}
    pairs = []
    while sum(cnt.values()) > 1:
        order = sorted(cnt.items(), key=lambda kv: (-kv[1], kv[0]))
        m1, n1 = order[0]
        m2, n2 = order[1] if len(order) > 1 else (None, 0)
        if n1 >= 2 * n2:
            k = n1 // 2
            pairs.append((m1, m1, k))
            cnt[m1] -= 2 * k
        else:
            pairs.append((m1, m2, n2))
            cnt[m1] -= n2
            cnt[m2] -= n2
        cnt = {i: v for i, v in cnt.items() if v > 0}
    left = next(iter(cnt)) if cnt else None
    return pairs, left


def repeated_pairs_system(A, g, r):
    """Matrix, loop vector and pair spec for the repeated-pairs sum of
    lhaf(A_r): the modes plus (for odd total) one dummy vertex with zero
    couplings and loop weight 1 paired with the leftover photon."""
    pairs, left = matched_reps(r)
    M = len(r)
    A = np.asarray(A, dtype=np.complex128)  # diagonal A_ii = coupling of copies
    g = np.asarray(g, dtype=np.complex128)
    if left is not None:
        A2 = np.zeros((M + 1, M + 1), dtype=np.complex128)
        A2[:M, :M] = A
        g2 = np.concatenate([g, [1.0 + 0j]])
        pairs = pairs + [(left, M, 1)]
        A, g = A2, g2
    u = np.array([p[0] for p in pairs], dtype=np.int32)
    w = np.array([p[1] for p in pairs], dtype=np.int32)
    eta = np.array([p[2] for p in pairs], dtype=np.int32)
    return A, g, (u, w, eta)


def lhaf_repeated(A, g, r, method="sum", **kw):
    """lhaf(A_r).  method 'sum': repeated-pairs power-trace sum (kw: mode,
    prec ...); 'explicit': memoised definition on the repeated matrix;
    'moment': loop repeated-moment sum."""
    if method == "explicit":
        Ar, gr = repeat_matrix(A, g, r)
        return lhaf_memo(Ar, gr, prec=kw.get("prec", "f64"))
    if method == "moment":
        return lhaf_rep_moment(A, g, r, prec=kw.get("prec", "f128"))
    if method == "eig":
        A2, g2, ps = repeated_pairs_system(A, g, r)
        return lhaf_eig_sum(A2, g2, ps, mode=kw.get("mode", "fds"))
    A2, g2, ps = repeated_pairs_system(A, g, r)
    return lhaf_sum(A2, g2, ps, **kw)


def lhafmix(A, g, n, method="sum", **kw):
    """Mixed-state lhafmix(A, g, n) (App. B.2): A is 2M x 2M, row i paired
    with row M+i, n_i times.  method 'sum': the paper's sum over z_i in
    [0, n_i] with that pairing (kw: mode, prec, ...); 'explicit': the
    definition on the matrix with rows i and M+i repeated n_i times."""
    n = np.asarray(n, dtype=np.int64)
    M = len(n)
    if method == "explicit":
        return lhaf_repeated(A, g, np.concatenate([n, n]), method="explicit", **kw)
    keep = np.nonzero(n > 0)[0]
    u = keep.astype(np.int32)
    w = (keep + M).astype(np.int32)
    return lhaf_sum(np.asarray(A, dtype=np.complex128), np.asarray(g, dtype=np.complex128),
                    (u, w, n[keep].astype(np.int32)), **kw)


def lhaf_chain_outputs(A, g, r, mode_b, n_cut, method="explicit", **kw):
    """Outputs of one chain-rule step by their definition (App. B.5): lhaf of
    the pattern r with mode_b set to k photons, for k = 0..n_cut."""
    out = []
    for k in range(n_cut + 1):
        rk = np.array(r, dtype=np.int64).copy()
        rk[mode_b] = k
        out.append(lhaf_repeated(A, g, rk, method=method, **kw) if rk.sum() > 0 else 1.0 + 0j)
    return np.array(out, dtype=np.complex128)


def lhaf_gamma_outputs(A, gammas, r=None, method="explicit", **kw):
    """Sub-detector outputs by their definition (App. B.5): lhaf(A_r, gamma_g)
    for every row gamma_g of gammas (r = None: the plain matrix)."""
    out = []
    for gv in np.asarray(gammas):
        if r is None:
            if method == "explicit":
                out.append(lhaf_memo(A, gv, prec=kw.get("prec", "f64")))
            else:
                out.append(lhaf_sum(A, gv, **kw))
        else:
            out.append(lhaf_repeated(A, gv, r, method=method, **kw))
    return np.array(out, dtype=np.complex128)


# ---------------------------------------------------------------------------
# numpy: traces from eigenvalues (the route App. B.1 names), batched
def _digits(t, radix):
    out = np.empty((len(t), len(radix)), dtype=np.int64)
    r = t.copy()
    for p, R in enumerate(radix):
        out[:, p] = r % R
        r //= R
    return out


def lhaf_eig_sum(A, g, pairs=None, mode="fds", halve=True, t0=0, t1=-1, scaled=True, chunk=2048,
                 with_abs=False):
    """Same sum as ``lhaf_sum`` (same enumeration), with Tr((CX)^k) = sum of
    the k-th powers of the eigenvalues of CX; f is the lambda^n coefficient of
    sum_j G^j / j! (App. B.1, Eq. ET_poly).  Plain float64."""
    A = np.asarray(A, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    if pairs is None:
        A, g = pad_odd(A, g)
        pairs = plain_pairs(A.shape[0])
    u, w, eta = (np.asarray(x, dtype=np.int64) for x in pairs)
    H = len(u)
    n = int(eta.sum())
    if n == 0:  # lhaf of the empty matrix: one empty matching
        return (1.0 + 0j, 1.0) if with_abs else 1.0 + 0j
    fds = mode == "fds"
    hp = next((p for p in range(H) if eta[p] % 2 == 1), 0)
    radix = [(eta[p] // 2 + 1) if (fds and halve and p == hp) else (eta[p] + 1) for p in range(H)]
    T = int(np.prod(radix)) if H else 1
    if t1 < 0 or t1 > T:
        t1 = T
    idx = np.concatenate([u, w])
    C = A[np.ix_(idx, idx)].copy()  # keeps A_ii: coupling of two copies of mode i
    v = g[idx]
    m = 2 * H
    binom = np.array([[math.comb(int(e), s) for s in range(33)] for e in eta], dtype=np.float64)
    total_parts = []
    abs_parts = []
    fact = np.array([math.factorial(j) for j in range(n + 1)], dtype=np.float64)
    for c0 in range(t0, t1, chunk):
        c1 = min(t1, c0 + chunk)
        t = np.arange(c0, c1, dtype=np.int64)
        s = _digits(t, radix)
        coef = np.ones(len(t))
        for p in range(H):
            coef *= binom[p][s[:, p]]
        if fds:
            coef *= np.where(s.sum(1) % 2 == 1, -1.0, 1.0)
            if halve and H:
                coef *= np.where(2 * s[:, hp] != eta[hp], 2.0, 1.0)
            x = (eta[None, :] - 2 * s).astype(np.float64)
        else:
            coef *= np.where((n - s.sum(1)) % 2 == 1, -1.0, 1.0)
            x = s.astype(np.float64)
        xx = np.concatenate([x, x], axis=1)  # weight of column j's pair
        # W = C X_x : column j = x_{pair(j)} * column partner(j) of C
        perm = np.concatenate([np.arange(H, m), np.arange(0, H)])
        W = C[None, :, perm] * xx[:, None, :]
        ev = np.linalg.eigvals(W)
        vx = xx * v[perm][None, :]
        y = np.broadcast_to(v, (len(t), m)).copy()
        G = np.zeros((len(t), n + 1), dtype=np.complex128)
        evk = np.ones_like(ev)
        for k in range(1, n + 1):
            evk = evk * ev
            G[:, k] = evk.sum(1) / (2 * k) + 0.5 * np.einsum("ti,ti->t", vx, y)
            y = np.einsum("tij,tj->ti", W, y)
        # sum_j G^j / j!, keep the lambda^n coefficient
        Gp = G.copy()
        f = Gp[:, n].copy()
        for j in range(2, n + 1):
            new = np.zeros_like(Gp)
            for d in range(j, n + 1):
                new[:, d] = np.einsum("ta,ta->t", Gp[:, 1:d], G[:, d - 1:0:-1])
            Gp = new
            f += Gp[:, n] / fact[j]
        if not fds:
            f = np.where(s.sum(1) == 0, 0.0, f)
        cf = coef * f
        total_parts.append(cf)
        abs_parts.append(np.abs(cf))
    if total_parts:
        allv = np.concatenate(total_parts)
        res = complex(math.fsum(allv.real), math.fsum(allv.imag))
        ab = float(np.sum(np.concatenate(abs_parts)))
    else:
        res, ab = 0j, 0.0
    if fds and scaled:
        res *= 2.0 ** (-n)
        ab *= 2.0 ** (-n)
    return (res, ab) if with_abs else res


# ---------------------------------------------------------------------------
# exact closed forms (Python integers)
def telephone(N: int) -> int:
    """Involution numbers: lhaf of the all-ones N x N matrix (A = J, gamma = 1)
    counts single-pair matchings; T(N) = T(N-1) + (N-1) T(N-2)."""
    a, b = 1, 1
    for k in range(2, N + 1):
        a, b = b, b + (k - 1) * a
    return b if N >= 1 else 1


def double_factorial_odd(n: int) -> int:
    """(2n-1)!! = number of perfect matchings of 2n vertices."""
    r = 1
    for k in range(1, 2 * n, 2):
        r *= k
    return r


def single_mode_repeated(a: complex, gamma: complex, r: int) -> complex:
    """lhaf of one mode repeated r times: sum_k C(r, 2k) (2k-1)!! a^k gamma^(r-2k)."""
    s = 0j
    for k in range(r // 2 + 1):
        s += math.comb(r, 2 * k) * double_factorial_odd(k) * a ** k * gamma ** (r - 2 * k)
    return s


def remove(A, g, rows):
    keep = [i for i in range(A.shape[0]) if i not in set(rows)]
    return np.asarray(A)[np.ix_(keep, keep)], np.asarray(g)[keep]
