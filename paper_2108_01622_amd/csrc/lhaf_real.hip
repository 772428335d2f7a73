// Real loop hafnians (real symmetric A, real gamma), e.g. the non-negative
// matrices whose lhaf the independence proposal of the MIS sampler needs
// (App. C of arXiv:2108.01622).  Same method as the complex kernels -- the
// power-trace sum over a fixed matching, ET or FDS, repeated pairs -- in real
// FP64: one real FMA where the complex path needs four, half the registers
// and LDS per wavefront.  The term enumeration, the weights and the
// coefficients are those of the complex kernels.
namespace lh {
namespace real {

// LDS layout of one wavefront (doubles)
struct Lds {
  double* wv;    // [65] Householder vector
  double* sc;    // [8]
  double* col;   // [65] current Hessenberg column
  double* wb;    // [64] characteristic-polynomial weights
  double* xb;    // [2][64] Krylov vectors
  double* mu;    // [33] loop moments
  double* ser;   // [2][33] series
  double* ring;  // [NR][NP]
  int NP, NR;
};

__device__ inline Lds carve(char* base, int nmax) {
  Lds L;
  double* c = reinterpret_cast<double*>(base);
  L.wv = c;
  L.sc = c + 65;
  L.col = c + 73;
  L.wb = c + 138;
  L.xb = c + 202;
  L.mu = c + 330;
  L.ser = c + 363;
  L.ring = c + 429;
  L.NP = nmax + 1;
  L.NR = nmax + 2;
  return L;
}

inline size_t lds_bytes(int nmax) {
  return sizeof(double) * (429 + (size_t)(nmax + 1) * (nmax + 2));
}

// Householder step (real): P = I - tau w w^T, w = x + sign(x_1) |x| e_1
template <int B, int kb>
__device__ __forceinline__ void householder_step(double (&W)[B][B], const int jj, const int j,
                                                 const int p, const int q, Lds& L) {
  double nrm2 = 0.0;
#pragma unroll
  for (int a = 0; a < B; ++a) {
    if (a < kb) continue;
    if (8 * a + p > j) nrm2 = fma(W[a][kb], W[a][kb], nrm2);
  }
  nrm2 = sum_col8(nrm2);
  if (q == jj) {
#pragma unroll
    for (int a = 0; a < B; ++a) {
      const int i = 8 * a + p;
      double x = (a >= kb && i > j) ? W[a][kb] : 0.0;
      if (i == j + 1) {
        const double nrm = sqrt(nrm2);
        const double ax = fabs(x);
        double tau = 0.0, beta = x;
        if (nrm > 0.0) {
          const double ph = x < 0.0 ? -1.0 : 1.0;
          x = fma(ph, nrm, x);
          tau = 1.0 / (nrm * (nrm + ax));
          beta = -ph * nrm;
        }
        L.sc[0] = tau;
        L.sc[1] = beta;
      }
      L.wv[i] = x;
    }
  }
  wave_sync();
  const double tau = L.sc[0];
  {
    double wr[B];
#pragma unroll
    for (int a = 0; a < B; ++a) wr[a] = (a >= kb) ? L.wv[8 * a + p] : 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      if (k < kb) continue;
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < B; ++a) {
        if (a < kb) continue;
        s = fma(wr[a], W[a][k], s);
      }
      s = tau * sum_col8(s);
#pragma unroll
      for (int a = 0; a < B; ++a) {
        if (a < kb) continue;
        W[a][k] = fma(-wr[a], s, W[a][k]);
      }
    }
  }
  if (q == jj) {
    const double beta = L.sc[1];
#pragma unroll
    for (int a = 0; a < B; ++a) {
      if (a < kb) continue;
      const int i = 8 * a + p;
      if (i == j + 1) W[a][kb] = beta;
      else if (i > j + 1) W[a][kb] = 0.0;
    }
  }
  {
    double wc[B];
#pragma unroll
    for (int k = 0; k < B; ++k) wc[k] = (k >= kb) ? L.wv[8 * k + q] : 0.0;
#pragma unroll
    for (int a = 0; a < B; ++a) {
      double y = 0.0;
#pragma unroll
      for (int k = 0; k < B; ++k) {
        if (k < kb) continue;
        y = fma(W[a][k], wc[k], y);
      }
      y = tau * sum_row8(y);
#pragma unroll
      for (int k = 0; k < B; ++k) {
        if (k < kb) continue;
        W[a][k] = fma(-y, wc[k], W[a][k]);
      }
    }
  }
}

// characteristic polynomial of the leading (J+1) x (J+1) Hessenberg block
// (the cofactor recursion of the complex kernel, in real arithmetic)
template <int B, int kb>
__device__ __forceinline__ void charpoly_step(const double (&W)[B][B], const int jj, const int J,
                                              const int p, const int q, const int lane,
                                              const int n, double& pi, double& hsub, Lds& L) {
  if (q == jj) {
#pragma unroll
    for (int a = 0; a < B; ++a) L.col[8 * a + p] = W[a][kb];
  }
  if (lane == 0) L.col[64] = 0.0;
  wave_sync();
  const double hJJ = L.col[J];
  const double hnext = L.col[J + 1];
  if (J >= 1) {
    if (lane < J - 1) pi *= hsub;
    else if (lane == J - 1) pi = hsub;
  }
  if (lane < J) L.wb[lane] = L.col[lane] * pi;
  wave_sync();
  const int t = (lane & 31) + 1;
  const int slot = lane >> 5;
  double acc = 0.0, acc2 = 0.0;
  if (t <= n) {
    const int ilo = (J + 1 - t) > 0 ? (J + 1 - t) : 0;
    int i = J - 1 - slot;
    for (; i - 2 >= ilo; i -= 4) {
      const double* Tp = L.ring + ring_slot(i - 1, L.NR) * L.NP;
      const double* Tq = L.ring + ring_slot(i - 3, L.NR) * L.NP;
      acc = fma(L.wb[i], Tp[t - (J - i + 1)], acc);
      acc2 = fma(L.wb[i - 2], Tq[t - (J - i + 3)], acc2);
    }
    if (i >= ilo) {
      const double* Tp = L.ring + ring_slot(i - 1, L.NR) * L.NP;
      acc = fma(L.wb[i], Tp[t - (J - i + 1)], acc);
    }
  }
  acc = sum_xor32(acc + acc2);
  const double* Tprev = L.ring + ring_slot(J - 1, L.NR) * L.NP;
  double* Tcur = L.ring + ring_slot(J, L.NR) * L.NP;
  double val = 0.0;
  if (slot == 0 && t <= n) val = fma(-hJJ, Tprev[t - 1], Tprev[t]) - acc;
  wave_sync();
  if (slot == 0 && t <= n) Tcur[t] = val;
  if (lane == 32) Tcur[0] = 1.0;
  wave_sync();
  hsub = hnext;
}

template <int B, int KB>
struct HessLoop {
  __device__ __forceinline__ static void run(double (&W)[B][B], const int m, const int n,
                                             const int p, const int q, const int lane, double& pi,
                                             double& hsub, Lds& L) {
#pragma unroll 1
    for (int jj = 0; jj < 8; ++jj) {
      const int j = 8 * KB + jj;
      if (j >= m) return;
      int ln = lane;  // optionally opaque per step, as in the complex kernel
      LH_OPAQUE(LH_OPAQUE_STEP, ln);
      const int pp = ln >> 3, qq = ln & 7;
      if (j <= m - 3) householder_step<B, KB>(W, jj, j, pp, qq, L);
      charpoly_step<B, KB>(W, jj, j, pp, qq, ln, n, pi, hsub, L);
    }
    HessLoop<B, KB + 1>::run(W, m, n, p, q, lane, pi, hsub, L);
  }
};
template <int B>
struct HessLoop<B, B> {
  __device__ __forceinline__ static void run(double (&)[B][B], const int, const int, const int,
                                             const int, const int, double&, double&, Lds&) {}
};

// loop moments mu_k = u^T W^{k-1} v (u = X_d v) from x_i = W^i v with the
// symmetry of X_d W: mu_{2i+1} = x_i^T X_d x_i, mu_{2i+2} = x_i^T X_d x_{i+1}
template <int B>
__device__ __forceinline__ void loop_moments(const double (&W)[B][B], const double (&dcol)[B],
                                             const double* __restrict__ vp, const int m,
                                             const int H, const int n, const int p, const int q,
                                             const int lane, Lds& L) {
  double xc[B];
#pragma unroll
  for (int k = 0; k < B; ++k) xc[k] = vp[8 * k + q];
  L.xb[lane] = vp[lane];
  wave_sync();
  int cur = 0;
  for (int i = 0; 2 * i + 1 <= n; ++i) {
    const double* xcur = L.xb + 64 * cur;
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int c = 8 * k + q;
      const int pc = c < H ? c + H : c - H;
      if (c < m) part = fma(dcol[k] * xc[k], xcur[pc & 63], part);
    }
    part = sum_row8(part);
    if (lane == 0) L.mu[2 * i + 1] = part;
    wave_sync();
    if (2 * i + 2 <= n) {
      double* xnext = L.xb + 64 * (cur ^ 1);
      double y[B];
#pragma unroll
      for (int a = 0; a < B; ++a) {
        y[a] = 0.0;
#pragma unroll
        for (int k = 0; k < B; ++k) y[a] = fma(W[a][k], xc[k], y[a]);
        y[a] = sum_row8(y[a]);
      }
      if (q == 0) {
#pragma unroll
        for (int a = 0; a < B; ++a) xnext[8 * a + p] = y[a];
      }
      wave_sync();
      double part2 = 0.0;
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int c = 8 * k + q;
        const int pc = c < H ? c + H : c - H;
        if (c < m) part2 = fma(dcol[k] * xc[k], xnext[pc & 63], part2);
      }
      part2 = sum_row8(part2);
      if (lane == 0) L.mu[2 * i + 2] = part2;
#pragma unroll
      for (int k = 0; k < B; ++k) xc[k] = xnext[8 * k + q];
      cur ^= 1;
      wave_sync();
    }
  }
}

// k y_k = sum_{j=1..k} (al k + j/2) x_j y_{k-j}: lanes 0..31 the series of
// c(lambda)^{-1/2} (al = -1), lanes 32..63 exp(sum mu_j lambda^j / 2)
__device__ __forceinline__ void two_series(const double* x0, double* y0, const double* x1,
                                           double* y1, const int n, const int lane) {
  const int h = lane >> 5, j = (lane & 31) + 1;
  const double* xs = h == 0 ? x0 : x1;
  double* ys = h == 0 ? y0 : y1;
  const double xj = j <= n ? xs[j] : 0.0;
  const double al = h == 0 ? -1.0 : 0.0;
  if ((lane & 31) == 0) ys[0] = 1.0;
  wave_sync();
  for (int k = 1; k <= n; ++k) {
    double t = 0.0;
    if (j <= k) t = fma(al, (double)k, 0.5 * j) * xj * ys[k - j];
    t = sum_half32(t);
    if ((lane & 31) == 0) ys[k] = t / k;
    wave_sync();
  }
}

template <int B>
__device__ __forceinline__ void run_item(const Prob& P, const int64_t t0, const int64_t t1,
                                         const double* __restrict__ Cp,
                                         const double* __restrict__ vp,
                                         Partial* __restrict__ out, Lds& L, const int acc_dd) {
  constexpr int LD = 8 * B;
  const int lane0 = threadIdx.x & 63;
  const int m = P.m, H = P.H, n = P.n;
  TermIter it = term_begin(P, t0, lane0);
  dd acc = {0.0, 0.0};
  double sabs = 0.0;
  for (int64_t t = t0; t < t1; ++t) {
    // lane index of this term (optionally opaque, see LH_OPAQUE_TERM)
    int lane = lane0;
    LH_OPAQUE(LH_OPAQUE_TERM, lane);
    const int p = lane >> 3, q = lane & 7;
    if (t != t0) term_next(it, H, lane);
    double coef;
    bool empty;
    const double wl = term_weight(it, P, lane, coef, empty);
    if (empty) {
      wave_sync();
      continue;
    }
    double dcol[B];
    column_weights<B>(wl, m, H, q, dcol);
    double W[B][B];
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int k = 0; k < B; ++k) W[a][k] = Cp[(8 * a + p) * LD + 8 * k + q] * dcol[k];
    loop_moments<B>(W, dcol, vp, m, H, n, p, q, lane, L);
    if (lane <= n) L.ring[lane] = lane == 0 ? 1.0 : 0.0;  // T_{-1}
    wave_sync();
    double pi = 0.0, hsub = 0.0;
    HessLoop<B, 0>::run(W, m, n, p, q, lane, pi, hsub, L);
    two_series(L.ring + ring_slot(m - 1, L.NR) * L.NP, L.ser, L.mu, L.ser + 33, n, lane);
    double f = 0.0;
    if (lane <= n) f = L.ser[lane] * L.ser[33 + n - lane];
    f = sum_col8(sum_row8(f));
    if (acc_dd) dd_add_prod(acc, coef, f);
    else acc.hi = fma(coef, f, acc.hi);
    sabs = fma(fabs(coef), fabs(f), sabs);
    wave_sync();
  }
  if (lane0 == 0) {
    Partial pr;
    pr.hr = acc.hi;
    pr.lr = acc.lo;
    pr.hi = pr.li = 0.0;
    pr.abs_sum = sabs;
    pr.pad0 = pr.pad1 = pr.pad2 = 0.0;
    *out = pr;
  }
}

#ifndef LH_REAL_WAVES
#define LH_REAL_WAVES(bmax) ((bmax) <= 2 ? 4 : ((bmax) <= 5 ? 3 : 2))
#endif

template <int BMAX>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(LH_REAL_WAVES(BMAX), LH_REAL_WAVES(BMAX)))) void real_kernel(
    const Prob* __restrict__ probs, const Item* __restrict__ items, int n_items, int* counter,
    const double* __restrict__ ws, Partial* __restrict__ parts, int acc_dd, int nmax) {
  extern __shared__ __align__(16) char lds_raw[];
  Lds L = carve(lds_raw, nmax);
  const int lane = threadIdx.x & 63;
  for (;;) {
    // every lane issues the atomic (see forward_kernel)
    const int it = __builtin_amdgcn_readfirstlane(atomicAdd(counter, lane == 0 ? 1 : 0));
    if (it >= n_items) break;
    const Item I = items[it];
    const Prob& P = probs[I.prob];
    const int LD = 8 * P.B;
    const double* Cp = ws + 2 * P.c_off;  // the complex-sized slot holds doubles
    const double* vp = Cp + LD * LD;
    switch (P.B) {
#define LH_RCASE(BB)                                                                       \
  case BB:                                                                                 \
    if (BB <= BMAX) run_item<(BB <= BMAX ? BB : 1)>(P, I.t0, I.t1, Cp, vp, parts + I.pad, L, acc_dd); \
    break;
      LH_RCASE(1)
      LH_RCASE(2)
      LH_RCASE(3)
      LH_RCASE(4)
      LH_RCASE(5)
      LH_RCASE(6)
      LH_RCASE(7)
      LH_RCASE(8)
#undef LH_RCASE
      default:
        break;
    }
  }
}

#ifdef LH_COMMON_KERNELS
// reduced matrix and loop vector of one real problem (the rules of
// pack_kernel), stored as doubles at twice the complex offset
__global__ void pack_kernel(const Prob* __restrict__ probs, const double* __restrict__ A,
                            int64_t lda, const double* __restrict__ g, double* __restrict__ ws,
                            int* counter) {
  const Prob& P = probs[blockIdx.x];
  const int LD = 8 * P.B;
  double* Cp = ws + 2 * P.c_off;
  for (int e = threadIdx.x; e < LD * LD; e += blockDim.x) {
    const int i = e / LD, c = e % LD;
    double val = 0.0;
    if (i < P.m && c < P.m) {
      const int j = c < P.H ? c + P.H : c - P.H;
      const int pi = P.pos[i], pj = P.pos[j];
      if (pi >= 0 && pj >= 0) {
        val = 0.5 * (A[(int64_t)pi * lda + pj] + A[(int64_t)pj * lda + pi]);
        if (i == j) {
          const int pr = i < P.H ? i : i - P.H;
          if (!((P.diag_keep_mask >> pr) & 1)) val = 0.0;
        }
      }
    }
    Cp[e] = val;
  }
  double* v = Cp + LD * LD;
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    double val = 0.0;
    if (i < P.m) {
      const int pi = P.pos[i];
      val = pi < 0 ? 1.0 : g[pi];
    }
    v[i] = val;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

// result and error estimate of the single real problem
__global__ void finalize_kernel(const Prob* __restrict__ probs, const Partial* __restrict__ parts,
                                double* out, double* err, int acc_dd) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const Prob& P = probs[0];
  dd s = {0.0, 0.0};
  double sabs = 0.0;
  if (P.n == 0 && P.t0 < P.t1) {
    s.hi = 1.0;
    sabs = 1.0;
  }
  for (int k = 0; k < P.n_items; ++k) {
    const Partial pr = parts[P.first_item + k];
    dd_add(s, pr.hr, pr.lr);
    sabs += pr.abs_sum;
  }
  double v = (s.hi + s.lo) * P.scale;
  const bool bad = !isfinite(v) || !isfinite(sabs);
  if (bad) v = NAN;  // non-finite input or overflow
  *out = v;
  if (err) {
    const double eps = 1.1102230246251565e-16;
    double rel_term = kTermErrPerDim * (P.m + 1) * eps;
    // plain FP64 sums each item's terms in order in one wavefront and the
    // item partials in double-double: the longest item bounds its rounding
    if (!acc_dd) rel_term += (double)lh_longest_item(P) * eps;
    double e = sabs * P.scale * rel_term;
    if (bad || !isfinite(e)) e = INFINITY;
    *err = e;
  }
}

#endif  // LH_COMMON_KERNELS

}  // namespace real
}  // namespace lh
