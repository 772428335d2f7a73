"""Seeded synthetic workloads for the loop-hafnian path.

This module only draws random numbers and assembles matrices from them; it
holds none of the loop-hafnian arithmetic, so both the HIP path and the CPU
oracle can take their inputs from it.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` with
``seed = 1622*1000 + 100*workload + instance`` so that any consumer rebuilds
the same bytes.  ``sha256_of`` fingerprints the arrays.

Workloads (shapes and distributions follow the paper's benchmark family of
Sec. 3 and the Gaussian-state construction of App. A):

* ``single16``   -- one N=16 Gaussian-state matrix A = U diag(tanh r) U^T,
  U Haar, r_i ~ U[0.5, 1.5], loop weights gamma_i ~ CN(0, 0.1).
* ``state100``   -- a 100-mode pure-state matrix B from 50 squeezed inputs
  (r = 1.5) behind uniform transmission 0.3 and a Haar 100x100 interferometer,
  split into pure part + classical displacement noise (App. A.1, Williamson),
  plus a 40-photon collision pattern on 28 modes with multiplicities in {1,2,3}.
* ``chain4096``  -- 4096 submatrices of ``state100`` with even sizes in
  [20, 40], indexed by prefixes of seeded mode permutations.
* ``dense52/60`` -- complex symmetric iid CN(0, 1/N) matrices (N = 52, 60)
  and block-diagonal A1 (+) A2 analogues of the paper's accuracy test (App. B.4).
* ``grad40``     -- 256 N=40 Gaussian-state matrices built like ``single16``.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

SEED_BASE = 1622 * 1000


def seed_for(workload: int, instance: int = 0) -> int:
    return SEED_BASE + 100 * workload + instance


def rng_for(workload: int, instance: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(workload, instance)))


def sha256_of(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def complex_normal(rng: np.random.Generator, shape, var: float) -> np.ndarray:
    """CN(0, var): real and imaginary parts iid N(0, var/2)."""
    s = math.sqrt(var / 2.0)
    return rng.standard_normal(shape) * s + 1j * (rng.standard_normal(shape) * s)


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary: QR of a complex Ginibre matrix with the phases of
    R's diagonal moved into Q (Mezzadri's correction)."""
    z = complex_normal(rng, (n, n), 1.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def gaussian_state_matrix(n: int, rng: np.random.Generator):
    """A = U diag(tanh r) U^T with U Haar, r_i ~ U[0.5, 1.5]; gamma ~ CN(0, 0.1)."""
    u = haar_unitary(n, rng)
    r = rng.uniform(0.5, 1.5, n)
    a = (u * np.tanh(r)[None, :]) @ u.T
    a = 0.5 * (a + a.T)
    gamma = complex_normal(rng, n, 0.1)
    return a.astype(np.complex128), gamma.astype(np.complex128)


# --------------------------------------------------------------------------
# workload 1: one N=16 matrix
def single16(instance: int = 0):
    rng = rng_for(1, instance)
    return gaussian_state_matrix(16, rng)


# --------------------------------------------------------------------------
# workload 2: 100-mode lossy squeezed state + collision pattern
STATE100_MODES = 100
STATE100_SQUEEZED = 50
STATE100_R = 1.5
STATE100_ETA = 0.3


def _pure_part_parameters(r: float, eta: float):
    """Single-mode lossy squeezed vacuum, hbar = 2 (vacuum covariance I):
    V = diag(a, b) with a = eta e^{-2r} + 1 - eta, b = eta e^{2r} + 1 - eta.
    Williamson: V = nu S S^T with nu = sqrt(ab), S = diag(e^{-r'}, e^{r'}),
    r' = ln(b/a)/4.  Pure part T = S S^T; noise W = (nu - 1) S S^T."""
    a = eta * math.exp(-2 * r) + 1 - eta
    b = eta * math.exp(2 * r) + 1 - eta
    nu = math.sqrt(a * b)
    rp = 0.25 * math.log(b / a)
    return a, b, nu, rp


def state100(instance: int = 0):
    """Returns dict with B (100x100 complex symmetric), gamma (100), the
    collision pattern r (int32[100]) and the generator parameters."""
    rng = rng_for(2, instance)
    m = STATE100_MODES
    k = STATE100_SQUEEZED
    u = haar_unitary(m, rng)
    a, b, nu, rp = _pure_part_parameters(STATE100_R, STATE100_ETA)
    t = math.tanh(rp)
    uk = u[:, :k]
    bmat = (uk * t) @ uk.T
    bmat = 0.5 * (bmat + bmat.T)
    # classical displacement noise of the pure-state ensemble (App. A.1)
    x = rng.standard_normal(k) * math.sqrt((nu - 1.0) * math.exp(-2 * rp))
    p = rng.standard_normal(k) * math.sqrt((nu - 1.0) * math.exp(2 * rp))
    alpha_in = (x + 1j * p) / 2.0
    alpha = uk @ alpha_in
    gamma = alpha - bmat @ np.conj(alpha)
    # detection pattern: 28 distinct modes at 1 photon, then 12 more photons
    # added one at a time to uniformly chosen modes still below 3
    modes = rng.choice(m, size=28, replace=False)
    pattern = np.zeros(m, dtype=np.int32)
    pattern[modes] = 1
    for _ in range(12):
        cand = [int(i) for i in modes if pattern[i] < 3]
        j = cand[int(rng.integers(len(cand)))]
        pattern[j] += 1
    return dict(B=bmat.astype(np.complex128), gamma=gamma.astype(np.complex128),
                r=pattern, params=dict(a=a, b=b, nu=nu, r_prime=rp, tanh_r_prime=t))


# --------------------------------------------------------------------------
# workload 3: chain-rule-step batch of submatrices of state100
def chain4096(count: int = 4096):
    base = state100(0)
    rng = rng_for(3, 0)
    sizes = 2 * rng.integers(10, 21, size=count)
    idx = []
    for b in range(count):
        perm = rng.permutation(STATE100_MODES)
        idx.append(np.sort(perm[: sizes[b]]).astype(np.int32))
    offs = np.zeros(count + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(i) for i in idx])
    return dict(B=base["B"], gamma=base["gamma"], idx=np.concatenate(idx).astype(np.int32),
                idx_off=offs, sizes=sizes.astype(np.int32))


def mixed_state(M: int, instance: int = 0):
    """Stand-in for a mixed Gaussian state's 2M x 2M loop-hafnian matrix: the
    block form [[B, C], [C^T, conj(B)]] with B = U diag(t) U^T (squeezing,
    t_i = tanh r_i, r ~ U[0.5, 1.5] scaled by 0.6) and C = U diag(c) U^dagger
    Hermitian PSD (thermal part, c ~ U[0, 0.3]), U Haar; gamma = (beta,
    conj(beta)) with beta ~ CN(0, 0.1).  Photon numbers n: M modes, each 0..3
    drawn with probabilities (0.2, 0.45, 0.25, 0.1)."""
    rng = rng_for(6, instance)
    U = haar_unitary(M, rng)
    t = 0.6 * np.tanh(rng.uniform(0.5, 1.5, size=M))
    c = rng.uniform(0.0, 0.3, size=M)
    Bm = (U * t) @ U.T
    Cm = (U * c) @ U.conj().T
    A = np.block([[Bm, Cm], [Cm.T, Bm.conj()]]).astype(np.complex128)
    beta = complex_normal(rng, M, 0.1)
    gamma = np.concatenate([beta, beta.conj()]).astype(np.complex128)
    n = rng.choice(4, size=M, p=[0.2, 0.45, 0.25, 0.1]).astype(np.int32)
    return A, gamma, n


# --------------------------------------------------------------------------
# workload 4: precision stress
def dense_symmetric(n: int, rng: np.random.Generator, var: float):
    a = complex_normal(rng, (n, n), var)
    a = np.triu(a, 1)
    a = a + a.T
    gamma = complex_normal(rng, n, var)
    np.fill_diagonal(a, 0.0)
    return a.astype(np.complex128), gamma.astype(np.complex128)


def dense_stress(n: int, instance: int):
    """iid CN(0, 1/n) complex symmetric matrix and loop vector."""
    rng = rng_for(4, (0 if n == 52 else 50) + instance)
    return dense_symmetric(n, rng, 1.0 / n)


def block_diagonal_stress(n: int, instance: int):
    """A1 (+) A2 with each half drawn iid CN(0, 1/n) (n = full size).
    Returns (A, gamma, (A1, g1), (A2, g2))."""
    rng = rng_for(4, (20 if n == 52 else 70) + instance)
    h = n // 2
    a1, g1 = dense_symmetric(h, rng, 1.0 / n)
    a2, g2 = dense_symmetric(h, rng, 1.0 / n)
    a = np.zeros((n, n), dtype=np.complex128)
    a[:h, :h] = a1
    a[h:, h:] = a2
    return a, np.concatenate([g1, g2]), (a1, g1), (a2, g2)


# --------------------------------------------------------------------------
# workload 5: differentiation batch
def grad40(count: int = 256, n: int = 40):
    rng = rng_for(5, 0)
    a = np.empty((count, n, n), dtype=np.complex128)
    g = np.empty((count, n), dtype=np.complex128)
    for b in range(count):
        a[b], g[b] = gaussian_state_matrix(n, rng)
    return a, g


def random_symmetric(n: int, seed: int, var: float = 1.0):
    """Generic small test matrix (iid CN(0, var) entries, symmetric)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = complex_normal(rng, (n, n), var)
    a = 0.5 * (a + a.T)
    g = complex_normal(rng, n, var)
    return a.astype(np.complex128), g.astype(np.complex128)


# --------------------------------------------------------------------------
# sub-detector batching: loop-weight vectors around one grad40 matrix's
def subdetector_gammas(count: int = 12):
    """grad40 matrix 0 and `count` loop-weight vectors gamma_0 + 0.05 (x + i y),
    x, y iid N(0, 1) (the loop vectors of neighbouring sub-detector outcomes)."""
    A, g = grad40(count=1)
    rng = rng_for(6, 0)
    n = A.shape[1]
    gs = g[0][None, :] + 0.05 * (rng.normal(size=(count, n)) + 1j * rng.normal(size=(count, n)))
    return A[0], gs.astype(np.complex128)


# real non-negative matrices (independence-proposal weights)
def real_nonneg(n: int, instance: int = 0):
    """Symmetric A with A_ij ~ U[0, 0.2] (i < j), gamma_i ~ U[0, 1], real."""
    rng = rng_for(7, instance)
    a = rng.uniform(0.0, 0.2, size=(n, n))
    a = 0.5 * (a + a.T)
    g = rng.uniform(0.0, 1.0, size=n)
    return a, g
