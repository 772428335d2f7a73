// Forward loop-hafnian kernels for gfx950.
//
// One wavefront evaluates one term of the power-trace sum at a time
// (App. B.1 / B.2 / B.4 of arXiv:2108.01622):
//   W = C X_d (C: reduced matrix of the problem, X_d: weighted fixed matching)
//   t_k = Tr(W^k),  mu_k = u^T W^{k-1} v  (u = X_d v),  k = 1..n
//   f = lambda^n coefficient of exp(sum_k (t_k/(2k) + mu_k/2) lambda^k)
//     = [lambda^n]  det(I - lambda W)^{-1/2} * exp(sum_k mu_k lambda^k / 2)
// and the signed sum over terms is accumulated in double-double.
//
// The power traces come from the characteristic polynomial of a Householder
// Hessenberg form of W (any exact-arithmetic equivalent of the eigenvalue
// route of App. B.1 gives the same t_k).  W lives in VGPRs: the 64 lanes form
// an 8 x 8 grid and lane (p, q) holds the entries (8a+p, 8k+q), a, k < B, so
// the active trailing block shrinks evenly over all lanes.  Row sums and
// column sums of the grid are DPP / permlane butterflies; the Householder
// vector goes through LDS.
#include <hip/hip_runtime.h>

#include "lhaf.h"
#include "lhaf_device.h"
#include "lhaf_internal.h"

namespace lh {

// LDS layout of one wavefront (dynamic shared memory).
struct LdsView {
  cd* wv;      // [65] Householder vector (by row)
  double* sc;  // [8] scalars of the current reflector
  cd* col;     // [65] current Hessenberg column
  cd* wb;      // [64] characteristic-polynomial weights
  cd* xb;      // [2][64] Krylov vectors
  cd* mu;      // [33] loop moments
  cd* ser;     // [2][33] q / L series
  cd* ring;    // [NR][NP] characteristic polynomials of leading blocks
  // compensated-recurrence instances only (beyond lds_bytes_for): the low
  // parts of the ring's and the series' double-double values
  cd* ring_lo;  // [NR][NP]
  cd* ser_lo;   // [2][33]
  int NP, NR;
};


__device__ inline LdsView carve(char* base, int nmax) {
  LdsView L;
  cd* c = reinterpret_cast<cd*>(base);
  L.wv = c;
  L.col = c + 65;
  L.wb = c + 130;
  L.xb = c + 194;
  L.mu = c + 322;
  L.ser = c + 355;
  L.sc = reinterpret_cast<double*>(c + 421);
  L.ring = reinterpret_cast<cd*>(L.sc + 8);
  L.NP = nmax + 1;
  L.NR = nmax + 2;
  L.ring_lo = L.ring + L.NP * L.NR;
  L.ser_lo = L.ring_lo + L.NP * L.NR;
  return L;
}

// Slot of T_k in the ring of NR = nmax + 2 polynomials.  k + 1 < 2 NR
// (k < m = 2H <= 2n <= 2 nmax), so one conditional subtraction replaces the
// integer remainder.
__device__ __forceinline__ int ring_slot(int k, int NR) {
  const int s = k + 1;
  return s >= NR ? s - NR : s;
}

#ifndef LH_FUSED_CONJ_UPDATE
#define LH_FUSED_CONJ_UPDATE 1
#endif

// -------------------------------------------------------------------------
// One Householder step of the Hessenberg reduction: column j (= 8*kb + jj)
// is reduced below the subdiagonal by W <- P W P, P = I - tau w w^* (P is
// Hermitian and unitary), w = x + e^{i arg x_1} |x| e_1 (x = W[j+1:, j]),
// tau = 1 / (|x| (|x| + |x_1|)).  Applied as two rank-1 passes, left then
// right, so only one reduction vector is live at a time:
//   W <- W - w (tau s),  s = w^* W        (column sums over the lane grid)
//   W <- W - (tau y) w^*, y = W w         (row sums over the lane grid)
template <int B, int kb>
__device__ __forceinline__ void householder_step(double (&Wr)[B][B], double (&Wi)[B][B],
                                                 const int jj, const int j, const int p,
                                                 const int q, LdsView& L) {
  // |x|^2 of every lane-column's column below row j (only column j is used)
  double nrm2 = 0.0;
#pragma unroll
  for (int a = 0; a < B; ++a) {
    if (a < kb) continue;
    const int i = 8 * a + p;
    if (i > j) nrm2 = fma(Wr[a][kb], Wr[a][kb], fma(Wi[a][kb], Wi[a][kb], nrm2));
  }
  nrm2 = sum_col8(nrm2);
  if (q == jj) {
#pragma unroll
    for (int a = 0; a < B; ++a) {
      const int i = 8 * a + p;
      cd x = czero();
      if (a >= kb && i > j) x = mk(Wr[a][kb], Wi[a][kb]);
      if (i == j + 1) {
        const double nrm = sqrt(nrm2);
        const double ax = sqrt(cabs2(x));
        double tau = 0.0;
        cd beta = x;
        if (nrm > 0.0) {
          cd ph = ax > 0.0 ? mk(x.r / ax, x.i / ax) : mk(1.0, 0.0);
          x = mk(fma(ph.r, nrm, x.r), fma(ph.i, nrm, x.i));
          tau = 1.0 / (nrm * (nrm + ax));
          beta = mk(-ph.r * nrm, -ph.i * nrm);
        }
        L.sc[0] = tau;
        L.sc[1] = beta.r;
        L.sc[2] = beta.i;
      }
      L.wv[i] = x;
    }
  }
  wave_sync();
  const double tau = L.sc[0];
  // ---- left: W <- W - w (tau w^* W), rows >= 8kb, columns >= 8kb
  {
    cd wr[B];
#pragma unroll
    for (int a = 0; a < B; ++a) wr[a] = (a >= kb) ? L.wv[8 * a + p] : czero();
#pragma unroll
    for (int k = 0; k < B; ++k) {
      if (k < kb) continue;
      cd s = czero();
#pragma unroll
      for (int a = 0; a < B; ++a) {
        if (a < kb) continue;
        s = cjfma(wr[a], mk(Wr[a][k], Wi[a][k]), s);
      }
      s = cscale(tau, sum_col8(s));
#pragma unroll
      for (int a = 0; a < B; ++a) {
        if (a < kb) continue;
        const cd w_ = cfnma(wr[a], s, mk(Wr[a][k], Wi[a][k]));
        Wr[a][k] = w_.r;
        Wi[a][k] = w_.i;
      }
    }
  }
  // column j is now (.., beta, 0, ..) below row j; set it exactly
  if (q == jj) {
    const cd beta = mk(L.sc[1], L.sc[2]);
#pragma unroll
    for (int a = 0; a < B; ++a) {
      if (a < kb) continue;
      const int i = 8 * a + p;
      if (i == j + 1) {
        Wr[a][kb] = beta.r;
        Wi[a][kb] = beta.i;
      } else if (i > j + 1) {
        Wr[a][kb] = 0.0;
        Wi[a][kb] = 0.0;
      }
    }
  }
  // ---- right: W <- W - (tau W w) w^*, all rows, columns >= 8kb
  {
    cd wc[B];
#pragma unroll
    for (int k = 0; k < B; ++k) wc[k] = (k >= kb) ? L.wv[8 * k + q] : czero();
#pragma unroll
    for (int a = 0; a < B; ++a) {
      cd y = czero();
#pragma unroll
      for (int k = 0; k < B; ++k) {
        if (k < kb) continue;
        y = cfma(mk(Wr[a][k], Wi[a][k]), wc[k], y);
      }
      y = cscale(tau, sum_row8(y));
#pragma unroll
      for (int k = 0; k < B; ++k) {
        if (k < kb) continue;
        const cd w_ = LH_FUSED_CONJ_UPDATE ? cfnmaj(y, wc[k], mk(Wr[a][k], Wi[a][k]))
                                           : csub(mk(Wr[a][k], Wi[a][k]), cmulj(y, wc[k]));
        Wr[a][k] = w_.r;
        Wi[a][k] = w_.i;
      }
    }
  }
}

// -------------------------------------------------------------------------
// Characteristic polynomial of the leading (J+1) x (J+1) block of the upper
// Hessenberg H, as T_J(lambda) = det(I - lambda H_J) truncated at degree n:
//   T_J = (1 - lambda h_JJ) T_{J-1}
//         - sum_{i<J} h_iJ (prod_{l=i+1..J} h_{l,l-1}) lambda^{J-i+1} T_{i-1}
// (cofactor expansion along the last column), T_{-1} = 1.
// kComp: every new coefficient is a compensated dot product (formed as in
// twice the working precision, rounded once when stored).
template <int B, int kb, bool kComp = false>
__device__ __forceinline__ void charpoly_step(const double (&Wr)[B][B], const double (&Wi)[B][B],
                                              const int jj, const int J, const int p, const int q,
                                              const int lane, const int n, cd& pi, cd& hsub,
                                              LdsView& L) {
  if (q == jj) {
#pragma unroll
    for (int a = 0; a < B; ++a) L.col[8 * a + p] = mk(Wr[a][kb], Wi[a][kb]);
  }
  if (lane == 0) L.col[64] = czero();
  wave_sync();
  const cd hJJ = L.col[J];
  const cd hnext = L.col[J + 1];
  if (J >= 1) {
    if (lane < J - 1) pi = cmul(pi, hsub);
    else if (lane == J - 1) pi = hsub;
  }
  if (lane < J) L.wb[lane] = cmul(L.col[lane], pi);
  wave_sync();
  const int t = (lane & 31) + 1;
  const int slot = lane >> 5;
  if constexpr (kComp) {
    // the ring holds double-double values (high parts in ring, low parts in
    // ring_lo); each new coefficient is formed from them exactly up to a
    // relative u^2 and kept unrounded
    const cd* Rl = L.ring_lo;
    cdd acc = cdd_zero(), acc2 = cdd_zero();
    if (t <= n) {
      const int ilo = (J + 1 - t) > 0 ? (J + 1 - t) : 0;
      int i = J - 1 - slot;
      for (; i - 2 >= ilo; i -= 4) {
        const int o1 = ring_slot(i - 1, L.NR) * L.NP + t - (J - i + 1);
        const int o2 = ring_slot(i - 3, L.NR) * L.NP + t - (J - i + 3);
        cdd_fma_hl(acc, L.wb[i], L.ring[o1], Rl[o1]);
        cdd_fma_hl(acc2, L.wb[i - 2], L.ring[o2], Rl[o2]);
      }
      if (i >= ilo) {
        const int o1 = ring_slot(i - 1, L.NR) * L.NP + t - (J - i + 1);
        cdd_fma_hl(acc, L.wb[i], L.ring[o1], Rl[o1]);
      }
    }
    acc = cdd_plus_xor32(cdd_plus(acc, acc2));
    const int op = ring_slot(J - 1, L.NR) * L.NP, oc = ring_slot(J, L.NR) * L.NP;
    cd vh = czero(), vl = czero();
    if (slot == 0 && t <= n) {
      cdd v = {L.ring[op + t].r, Rl[op + t].r, L.ring[op + t].i, Rl[op + t].i};
      cdd_fma_hl(v, mk(-hJJ.r, -hJJ.i), L.ring[op + t - 1], Rl[op + t - 1]);
      cdd_split(cdd_plus(v, cdd_neg(acc)), vh, vl);
    }
    wave_sync();
    if (slot == 0 && t <= n) {
      L.ring[oc + t] = vh;
      L.ring_lo[oc + t] = vl;
    }
    if (lane == 32) {
      L.ring[oc] = mk(1.0, 0.0);
      L.ring_lo[oc] = czero();
    }
    wave_sync();
    hsub = hnext;
    return;
  }
  cd acc = czero(), acc2 = czero();
  if (t <= n) {
    const int ilo = (J + 1 - t) > 0 ? (J + 1 - t) : 0;
    int i = J - 1 - slot;
    // two independent chains so the LDS loads of one overlap the other's FMAs
    for (; i - 2 >= ilo; i -= 4) {
      const cd* Tp = L.ring + ring_slot(i - 1, L.NR) * L.NP;
      const cd* Tq = L.ring + ring_slot(i - 3, L.NR) * L.NP;
      acc = cfma(L.wb[i], Tp[t - (J - i + 1)], acc);
      acc2 = cfma(L.wb[i - 2], Tq[t - (J - i + 3)], acc2);
    }
    if (i >= ilo) {
      const cd* Tp = L.ring + ring_slot(i - 1, L.NR) * L.NP;
      acc = cfma(L.wb[i], Tp[t - (J - i + 1)], acc);
    }
  }
  acc = sum_xor32(cadd(acc, acc2));
  const cd* Tprev = L.ring + ring_slot(J - 1, L.NR) * L.NP;
  cd* Tcur = L.ring + ring_slot(J, L.NR) * L.NP;
  cd val = czero();
  if (slot == 0 && t <= n) val = csub(cfnma(hJJ, Tprev[t - 1], Tprev[t]), acc);
  wave_sync();
  if (slot == 0 && t <= n) Tcur[t] = val;
  if (lane == 32) Tcur[0] = mk(1.0, 0.0);
  wave_sync();
  hsub = hnext;
}

// -------------------------------------------------------------------------
// Column blocks of 8: block KB is a compile-time constant, so every register
// index stays static while the 8 steps inside a block run as a loop.
template <int B, int KB, bool kComp = false>
struct HessLoop {
  __device__ __forceinline__ static void run(double (&Wr)[B][B], double (&Wi)[B][B], const int m,
                                             const int n, const int p, const int q,
                                             const int lane, cd& pi, cd& hsub, LdsView& L) {
#pragma unroll 1
    for (int jj = 0; jj < 8; ++jj) {
      const int j = 8 * KB + jj;
      if (j >= m) return;
      // lane index of this step (optionally opaque, see LH_OPAQUE_STEP)
      int ln = lane;
      LH_OPAQUE(LH_OPAQUE_STEP, ln);
      const int pp = ln >> 3, qq = ln & 7;
      if (j <= m - 3) householder_step<B, KB>(Wr, Wi, jj, j, pp, qq, L);
      charpoly_step<B, KB, kComp>(Wr, Wi, jj, j, pp, qq, ln, n, pi, hsub, L);
    }
    HessLoop<B, KB + 1, kComp>::run(Wr, Wi, m, n, p, q, lane, pi, hsub, L);
  }
};
template <int B, bool kComp>
struct HessLoop<B, B, kComp> {
  __device__ __forceinline__ static void run(double (&)[B][B], double (&)[B][B], const int,
                                             const int, const int, const int, const int, cd&,
                                             cd&, LdsView&) {}
};

// -------------------------------------------------------------------------
// Term enumeration state: lane p (< H) holds the digit of pair p; pair 0 is
// the fastest digit.
struct TermIter {
  int digit, eta_l, radix_l;
};

__device__ __forceinline__ TermIter term_begin(const Prob& P, const int64_t t0, const int lane) {
  TermIter it;
  it.eta_l = lane < P.H ? (int)P.eta[lane] : 0;
  it.radix_l = lane < P.H ? (int)P.radix[lane] : 1;
  it.digit = 0;
  int64_t r = t0;
  for (int pp = 0; pp < P.H; ++pp) {
    const int R = P.radix[pp];
    const int d = (int)(r % R);
    r /= R;
    if (lane == pp) it.digit = d;
  }
  return it;
}

__device__ __forceinline__ void term_next(TermIter& it, const int H, const int lane) {
  const unsigned long long can = __ballot(lane < H && it.digit != it.radix_l - 1);
  const int k = __ffsll((long long)can) - 1;
  if (lane < k) it.digit = 0;
  else if (lane == k) it.digit += 1;
}

// Weight of the lane's pair (d_p for FDS, z_p for ET) and the term's exact
// integer coefficient c_t; `empty` marks the ET term with no pair (f = 0).
__device__ __forceinline__ double term_weight(const TermIter& it, const Prob& P, const int lane,
                                              double& coef, bool& empty) {
  const bool fds = P.mode == 1;
  double wl, fl;
  if (fds) {
    wl = (double)(it.eta_l - 2 * it.digit);
    fl = ((it.digit & 1) ? -1.0 : 1.0) * c_binom.v[it.eta_l][it.digit];
    if (lane == P.hp && 2 * it.digit != it.eta_l) fl *= 2.0;
  } else {
    wl = (double)it.digit;
    fl = (((it.eta_l - it.digit) & 1) ? -1.0 : 1.0) * c_binom.v[it.eta_l][it.digit];
  }
  if (lane >= P.H) {
    wl = 0.0;
    fl = 1.0;
  }
  coef = prod_wave(fl, lane);
  empty = !fds && __ballot(lane < P.H && it.digit != 0) == 0ull;
  return wl;
}

// d of the pairs of the lane's columns c = 8k+q (0 beyond m)
template <int B>
__device__ __forceinline__ void column_weights(const double wl, const int m, const int H,
                                               const int q, double (&dcol)[B]) {
#pragma unroll
  for (int k = 0; k < B; ++k) {
    const int c = 8 * k + q;
    const int pc = c < H ? c : c - H;
    const double d = shfl_d(wl, pc & 63);
    dcol[k] = c < m ? d : 0.0;
  }
}

// W = C X_d: packed Cp holds C with partner-permuted columns
template <int B>
__device__ __forceinline__ void load_w(const cd* __restrict__ Cp, const double (&dcol)[B],
                                       const int p, const int q, double (&Wr)[B][B],
                                       double (&Wi)[B][B]) {
  const int LD = 8 * B;
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const cd c = Cp[(8 * a + p) * LD + 8 * k + q];
      Wr[a][k] = c.r * dcol[k];
      Wi[a][k] = c.i * dcol[k];
    }
}

// Loop moments mu_k = u^T W^{k-1} v (u = X_d v) into L.mu[1..n], from the
// Krylov vectors x_i = W^i v: X_d W is symmetric, so
//   mu_{2i+1} = x_i^T X_d x_i,  mu_{2i+2} = x_i^T X_d x_{i+1}.
template <int B>
__device__ __forceinline__ void loop_moments(const double (&Wr)[B][B], const double (&Wi)[B][B],
                                             const double (&dcol)[B], const cd* __restrict__ vp,
                                             const int m, const int H, const int n, const int p,
                                             const int q, const int lane, LdsView& L) {
  cd xc[B];
#pragma unroll
  for (int k = 0; k < B; ++k) xc[k] = vp[8 * k + q];
  L.xb[lane] = vp[lane];
  wave_sync();
  int cur = 0;
  for (int i = 0; 2 * i + 1 <= n; ++i) {
    const cd* xcur = L.xb + 64 * cur;
    cd part = czero();
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int c = 8 * k + q;
      const int pc = c < H ? c + H : c - H;
      if (c < m) part = cfma(cscale(dcol[k], xc[k]), xcur[pc & 63], part);
    }
    part = sum_row8(part);
    if (lane == 0) L.mu[2 * i + 1] = part;
    wave_sync();
    if (2 * i + 2 <= n) {
      cd* xnext = L.xb + 64 * (cur ^ 1);
      cd y[B];
#pragma unroll
      for (int a = 0; a < B; ++a) {
        y[a] = czero();
#pragma unroll
        for (int k = 0; k < B; ++k) y[a] = cfma(mk(Wr[a][k], Wi[a][k]), xc[k], y[a]);
        y[a] = sum_row8(y[a]);
      }
      if (q == 0) {
#pragma unroll
        for (int a = 0; a < B; ++a) xnext[8 * a + p] = y[a];
      }
      wave_sync();
      cd part2 = czero();
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int c = 8 * k + q;
        const int pc = c < H ? c + H : c - H;
        if (c < m) part2 = cfma(cscale(dcol[k], xc[k]), xnext[pc & 63], part2);
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

// Two power-series recurrences at once, lanes 0..31 for (x0 -> y0) and lanes
// 32..63 for (x1 -> y1), y[0] = 1 and
//   k y_k = sum_{j=1..k} (al k + j/2) x_j y_{k-j},   k = 1..n:
// al = -1 gives y = c(lambda)^{-1/2} from the coefficients c_j of
// c(lambda) = det(I - lambda W); al = 0 gives y = exp(sum_j x_j lambda^j / 2).
// Step k is a 32-lane dot product over j = 1..k (lane j-1 of the half)
// reduced by a butterfly inside the half, so the serial chain is n steps.
// kComp: each step is a compensated dot product (the weight al k + j/2 is
// exact, its product with x_j is split exactly, and the sum is rounded once
// after the division by k).
// (x0_lo, y0_lo, y1_lo: the low parts of the double-double values, used by
// the kComp instance only; x1 has none)
template <bool kComp = false>
__device__ __forceinline__ void two_series(const cd* x0, cd* y0, const double al0, const cd* x1,
                                           cd* y1, const double al1, const int n, const int lane,
                                           const cd* x0_lo = nullptr, cd* y0_lo = nullptr,
                                           cd* y1_lo = nullptr) {
  const int h = lane >> 5, j = (lane & 31) + 1;
  const cd* xs = h == 0 ? x0 : x1;
  cd* ys = h == 0 ? y0 : y1;
  const cd xj = j <= n ? xs[j] : czero();
  const double al = h == 0 ? al0 : al1;
  if ((lane & 31) == 0) ys[0] = mk(1.0, 0.0);
  [[maybe_unused]] cd* ys_lo = nullptr;
  [[maybe_unused]] cd xjl = czero();
  if constexpr (kComp) {
    ys_lo = h == 0 ? y0_lo : y1_lo;
    if (h == 0 && j <= n) xjl = x0_lo[j];
    if ((lane & 31) == 0) ys_lo[0] = czero();
  }
  wave_sync();
  for (int k = 1; k <= n; ++k) {
    if constexpr (kComp) {
      // x and y double-double (x1 = the loop moments, exact in double); the
      // weight al k + j/2 is exact and its product with x_j is split exactly
      cdd t = cdd_zero();
      if (j <= k) {
        const double w = fma(al, (double)k, 0.5 * j);
        const cd yh = ys[k - j], yl = ys_lo[k - j];
        const cd wx = mk(w * xj.r, w * xj.i);
        const cd wxl = mk(fma(w, xj.r, -wx.r) + w * xjl.r, fma(w, xj.i, -wx.i) + w * xjl.i);
        cdd_fma_hl2(t, wx, wxl, yh, yl);
      }
      t = cdd_sum_half32(t);
      if ((lane & 31) == 0) {
        cd qh, ql;
        cdd_split(cdd_div(t, (double)k), qh, ql);
        ys[k] = qh;
        ys_lo[k] = ql;
      }
    } else {
      cd t = czero();
      if (j <= k) t = cmul(cscale(fma(al, (double)k, 0.5 * j), xj), ys[k - j]);
      t = sum_half32(t);
      if ((lane & 31) == 0) ys[k] = cscale(1.0 / k, t);
    }
    wave_sync();
  }
}

// Hessenberg reduction (destroys W) and characteristic polynomial of W, then
// the two series of f(lambda) = c(lambda)^{-1/2} exp(M(lambda)),
// M = sum_k mu_k lambda^k / 2:
//   L.ser[0..n]      q_k, k q_k = -sum_{j=1..k} (k - j/2) c_j q_{k-j}
//   L.ser[33..33+n]  L_k, k L_k = sum_{j=1..k} (j/2) mu_j L_{k-j}
template <int B, bool kComp = false>
__device__ __forceinline__ void spectral_series(double (&Wr)[B][B], double (&Wi)[B][B],
                                                const int m, const int n, const int p,
                                                const int q, const int lane, LdsView& L) {
  if (lane <= n) L.ring[lane] = lane == 0 ? mk(1.0, 0.0) : czero();  // T_{-1} in slot 0
  if constexpr (kComp) {
    if (lane <= n) L.ring_lo[lane] = czero();
  }
  wave_sync();
  cd pi = czero(), hsub = czero();
  HessLoop<B, 0, kComp>::run(Wr, Wi, m, n, p, q, lane, pi, hsub, L);
  const int co = ring_slot(m - 1, L.NR) * L.NP;
  two_series<kComp>(L.ring + co, L.ser, -1.0, L.mu, L.ser + 33, 0.0, n, lane, L.ring_lo + co,
                    L.ser_lo, L.ser_lo + 33);
}

// Lane k (1 <= k <= n): a_k = e_{n-k} / 2, where e_j = sum_{i<=j} q_i L_{j-i}
// is the lambda^j coefficient of f(lambda) (the weights of the power sums in
// the adjoint: d f / d g_k = e_{n-k}).
__device__ __forceinline__ cd series_coef(const LdsView& L, const int n, const int lane) {
  const int j = n - lane;
  cd e0 = czero(), e1 = czero();
  int i = 0;
  for (; i + 1 <= j; i += 2) {
    e0 = cfma(L.ser[i], L.ser[33 + j - i], e0);
    e1 = cfma(L.ser[i + 1], L.ser[33 + j - i - 1], e1);
  }
  if (i <= j) e0 = cfma(L.ser[i], L.ser[33 + j - i], e0);
  return cscale(0.5, cadd(e0, e1));
}

// -------------------------------------------------------------------------
// ET pair deletion (App. B.2): a pair with weight z_p = 0 contributes zero
// columns to W = C X_z and a zero entry to u = X_z v, so the term's traces
// and loop moments are those of the reduced problem on the kept pairs, with
// m = 2 H' (H' kept pairs) and the same lambda degree n.  km receives the
// full-problem position of every reduced position -- kept pairs' first ends
// in pair order, then their partners -- and -1 beyond 2 H'.  Returns H'.
__device__ __forceinline__ int kept_map(const TermIter& it, const int H, const int lane,
                                        int* __restrict__ km) {
  const bool kept = lane < H && it.digit != 0;
  const unsigned long long keep = __ballot(kept);
  const int Hk = __popcll(keep);
  if (kept) {
    const int r = __popcll(keep & ((1ull << lane) - 1ull));
    km[r] = lane;
    km[Hk + r] = H + lane;
  }
  if (lane >= 2 * Hk) km[lane] = -1;
  wave_sync();
  return Hk;
}

// One term at register tile b: W = C X (every pair, or through km only the
// kept pairs of an ET term), loop moments and the two series into L.ser;
// returns f = [lambda^n] of the product of the series on every lane.
template <int b, bool kComp = false>
__device__ __forceinline__ cd term_f(const cd* __restrict__ Cp, const int LDp,
                                     const cd* __restrict__ vp, const int* __restrict__ km,
                                     const double wl, const int mt, const int Ht, const int H,
                                     const int n, const int p, const int q, const int lane,
                                     LdsView& L) {
  double dcol[b];
  double Wr[b][b], Wi[b][b];
  if (km) {
    int oc[b];
#pragma unroll
    for (int k = 0; k < b; ++k) {
      const int c = 8 * k + q;
      oc[k] = c < mt ? km[c] : -1;
      const int pr = oc[k] < 0 ? 0 : (oc[k] < H ? oc[k] : oc[k] - H);
      const double d = shfl_d(wl, pr & 63);
      dcol[k] = oc[k] >= 0 ? d : 0.0;
    }
#pragma unroll
    for (int a = 0; a < b; ++a) {
      const int i = 8 * a + p;
      const int oi = i < mt ? km[i] : -1;
#pragma unroll
      for (int k = 0; k < b; ++k) {
        cd c = czero();
        if (oi >= 0 && oc[k] >= 0) c = Cp[oi * LDp + oc[k]];
        Wr[a][k] = c.r * dcol[k];
        Wi[a][k] = c.i * dcol[k];
      }
    }
  } else {
    column_weights<b>(wl, mt, Ht, q, dcol);
    load_w<b>(Cp, dcol, p, q, Wr, Wi);
  }
  loop_moments<b>(Wr, Wi, dcol, vp, mt, Ht, n, p, q, lane, L);
  spectral_series<b, kComp>(Wr, Wi, mt, n, p, q, lane, L);
  // f = sum_k q_k L_{n-k}: lanes over k, full-wave sum (every lane gets f)
  if constexpr (kComp) {
    cdd fc = cdd_zero();
    if (lane <= n)
      cdd_fma_hl2(fc, L.ser[lane], L.ser_lo[lane], L.ser[33 + n - lane], L.ser_lo[33 + n - lane]);
    return cdd_round(cdd_sum_wave(fc));
  }
  cd f = czero();
  if (lane <= n) f = cmul(L.ser[lane], L.ser[33 + n - lane]);
  return mk(sum_col8(sum_row8(f.r)), sum_col8(sum_row8(f.i)));
}

// term_f at the runtime tile bt (1 <= bt <= BMAX; uniform over the wavefront)
template <int BMAX, bool kComp = false>
__device__ __forceinline__ cd term_f_at(const int bt, const cd* __restrict__ Cp, const int LDp,
                                        const cd* __restrict__ vp, const int* __restrict__ km,
                                        const double wl, const int mt, const int Ht, const int H,
                                        const int n, const int p, const int q, const int lane,
                                        LdsView& L) {
  cd f = czero();
  switch (bt) {
#define LH_TCASE(BB)                                                                 \
  case BB:                                                                           \
    if constexpr (BB <= BMAX)                                                        \
      f = term_f<BB, kComp>(Cp, LDp, vp, km, wl, mt, Ht, H, n, p, q, lane, L);       \
    break;
    LH_TCASE(1) LH_TCASE(2) LH_TCASE(3) LH_TCASE(4) LH_TCASE(5) LH_TCASE(6) LH_TCASE(7)
    LH_TCASE(8)
#undef LH_TCASE
    default:
      break;
  }
  return f;
}

// -------------------------------------------------------------------------
// Evaluate terms [t0, t1) of problem P; writes the item's partial sum (and,
// with a coefficient store, the a_k of every term).  kET: an ET batch, whose
// terms run on their kept pairs only, at tile ceil(2H'/8) <= B chosen per
// term; otherwise every term runs at the problem's tile B = P.B.  (ET and
// FDS batches are separate kernels: the per-term tile switch would raise the
// register pressure of the FDS path.)
// kET with tile bounds [tlo, thi]: only the terms whose reduced tile
// ceil(2H'/8) lies in the bounds are evaluated (the ET term space split into
// tile classes, each launched at its own occupancy; the classes' partial sums
// add up).
template <int B, bool kET, bool kComp = false>
__device__ __forceinline__ void run_item(const Prob& P, const int64_t t0, const int64_t t1,
                                         const cd* __restrict__ Cp, const cd* __restrict__ vp,
                                         Partial* __restrict__ out, LdsView& L, const int acc_dd,
                                         cd* __restrict__ saved, const int tlo, const int thi) {
  const int lane0 = threadIdx.x & 63;
  const int m = P.m, H = P.H, n = P.n, LDp = 8 * P.B;
  int* km = reinterpret_cast<int*>(L.wv);  // free until the Hessenberg phase
  cd* vred = L.xb + 64;                    // overwritten only after loop_moments read it
  TermIter it = term_begin(P, t0, lane0);
  // The item's partial lives in LDS, in the scalar slots after the
  // reflector's (hr, lr, hi, li, abs), read and written by lane 0 only: in
  // registers it would stay live through the whole term.
  double* vacc = L.sc + 3;
  if (lane0 == 0) {
#pragma unroll
    for (int k = 0; k < 5; ++k) vacc[k] = 0.0;
  }

  for (int64_t t = t0; t < t1; ++t) {
    // lane index of this term (optionally opaque, see LH_OPAQUE_TERM)
    int lane = lane0;
    LH_OPAQUE(LH_OPAQUE_TERM, lane);
    const int p = lane >> 3, q = lane & 7;
    if (t != t0) term_next(it, H, lane);
    if constexpr (kET) {
      const int hk = __popcll(__ballot(lane < H && it.digit != 0));
      const int bt = (2 * hk + 7) >> 3;
      // (a term needing a larger tile than this instance's belongs to the
      // other launch of a split sum)
      if (hk == 0 || bt < tlo || bt > thi || bt > B) continue;  // uniform: no LDS touched
    }
    double coef;
    bool empty;
    const double wl = term_weight(it, P, lane, coef, empty);
    if (empty) {
      wave_sync();
      continue;
    }
    cd f;
    if constexpr (kET) {
      const int Hk = kept_map(it, H, lane, km);
      const int mk_ = 2 * Hk;
      vred[lane] = lane < mk_ ? vp[km[lane]] : czero();
      wave_sync();
      f = term_f_at<B, kComp>((mk_ + 7) >> 3, Cp, LDp, vred, km, wl, mk_, Hk, H, n, p, q, lane,
                              L);
    } else {
      f = term_f<B, kComp>(Cp, LDp, vp, nullptr, wl, m, H, H, n, p, q, lane, L);
    }
    if (lane0 == 0) {
      dd accr = {vacc[0], vacc[1]}, acci = {vacc[2], vacc[3]};
      if (acc_dd) {
        dd_add_prod(accr, coef, f.r);
        dd_add_prod(acci, coef, f.i);
      } else {
        accr.hi = fma(coef, f.r, accr.hi);
        acci.hi = fma(coef, f.i, acci.hi);
      }
      vacc[0] = accr.hi;
      vacc[1] = accr.lo;
      vacc[2] = acci.hi;
      vacc[3] = acci.lo;
      vacc[4] = fma(fabs(coef), sqrt(cabs2(f)), vacc[4]);
    }
    if (saved && lane >= 1 && lane <= n) saved[P.s_off + (t - P.t0) * n + (lane - 1)] = series_coef(L, n, lane);
    wave_sync();
  }
  if (lane0 == 0) {
    Partial pr;
    pr.hr = vacc[0];
    pr.hi = vacc[2];
    pr.lr = vacc[1];
    pr.li = vacc[3];
    pr.abs_sum = vacc[4];
    pr.pad0 = pr.pad1 = pr.pad2 = 0.0;
    *out = pr;
  }
}

#ifdef LH_COMMON_KERNELS
// -------------------------------------------------------------------------
// Pack the reduced matrix of every problem: Cp[i][c] = C[i][partner(c)] with
// C[i][j] = sym(A)[mode(i)][mode(j)]; C's diagonal is kept only for repeated
// pairs (it is the coupling of two copies of a mode and cancels otherwise).
// v[i] = gamma[mode(i)] (1 for the padding vertex).  Also resets the work
// counter.
__global__ void pack_kernel(const Prob* __restrict__ probs, const int64_t* __restrict__ aoff,
                            const int64_t* __restrict__ goff, const int64_t* __restrict__ ioff,
                            const lh_c128* __restrict__ A, int64_t lda,
                            const lh_c128* __restrict__ g, const int32_t* __restrict__ idx,
                            cd* __restrict__ ws, int* counter) {
  const int b = blockIdx.x;
  const Prob& P = probs[b];
  const int LD = 8 * P.B;
  const lh_c128* Ab = A + aoff[b];
  const lh_c128* gb = g + goff[b];
  const int32_t* ib = idx ? idx + ioff[b] : nullptr;
  cd* Cp = ws + P.c_off;
  for (int e = threadIdx.x; e < LD * LD; e += blockDim.x) {
    const int i = e / LD, c = e % LD;
    cd val = czero();
    if (i < P.m && c < P.m) {
      const int j = c < P.H ? c + P.H : c - P.H;
      const int pi = P.pos[i], pj = P.pos[j];
      if (pi >= 0 && pj >= 0) {
        const int mi = ib ? ib[pi] : pi;
        const int mj = ib ? ib[pj] : pj;
        const lh_c128 x = Ab[(int64_t)mi * lda + mj];
        const lh_c128 y = Ab[(int64_t)mj * lda + mi];
        val = mk(0.5 * (x.re + y.re), 0.5 * (x.im + y.im));
        if (i == j) {
          const int pr = i < P.H ? i : i - P.H;
          if (!((P.diag_keep_mask >> pr) & 1)) val = czero();
        }
      }
    }
    Cp[e] = val;
  }
  cd* v = Cp + LD * LD;
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    cd val = czero();
    if (i < P.m) {
      const int pi = P.pos[i];
      if (pi < 0) val = mk(1.0, 0.0);
      else {
        const lh_c128 x = gb[ib ? ib[pi] : pi];
        val = mk(x.re, x.im);
      }
    }
    v[i] = val;
  }
  if (b == 0 && threadIdx.x == 0) {
    counter[0] = 0;
    counter[kSecondCounter] = 0;  // queue of a second launch over the same items
  }
}

#endif  // LH_COMMON_KERNELS

// resident wavefronts per SIMD the register allocation aims for, by tile
#ifndef LH_FWD_WAVES
#define LH_FWD_WAVES(bmax) ((bmax) <= 3 ? 4 : ((bmax) <= 4 ? 3 : ((bmax) <= 6 ? 2 : 1)))
#endif

// The forward kernels: one wavefront per workgroup takes items from the
// work queue until it is empty.  forward_kernel evaluates in plain FP64;
// forward_comp_kernel (the compensated-recurrence mode) forms the
// characteristic polynomial, the two series and the final coefficient as
// compensated dot products, at the same occupancy.  One body, stamped twice.
#define LH_FORWARD_KERNEL(NAME, COMP)                                                          \
  template <int BMAX, bool kET>                                                                \
  __global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(                         \
      LH_FWD_WAVES(BMAX), LH_FWD_WAVES(BMAX)))) void NAME(const Prob* __restrict__ probs,      \
                                                          const Item* __restrict__ items,      \
                                                          int n_items, int* counter,           \
                                                          const cd* __restrict__ ws,           \
                                                          Partial* __restrict__ parts,         \
                                                          int acc_dd, int nmax,                \
                                                          cd* __restrict__ saved, int tlo,     \
                                                          int thi) {                           \
    extern __shared__ __align__(16) char lds_raw[];                                            \
    LdsView L = carve(lds_raw, nmax);                                                          \
    const int lane = threadIdx.x & 63;                                                         \
    for (;;) {                                                                                 \
      /* Every lane issues the atomic (only lane 0 adds 1), so no lane-divergent region     */ \
      /* precedes the cross-lane read at the loop head; the compiler may otherwise split    */ \
      /* the loop by lane and leave lanes reading an inactive lane 0.  Lane 0's return      */ \
      /* value is unique per wavefront either way.                                          */ \
      const int it = __builtin_amdgcn_readfirstlane(atomicAdd(counter, lane == 0 ? 1 : 0));    \
      if (it >= n_items) break;                                                                \
      const Item I = items[it];                                                                \
      const Prob& P = probs[I.prob];                                                           \
      const int LD = 8 * P.B;                                                                  \
      const cd* Cp = ws + P.c_off;                                                             \
      const cd* vp = Cp + LD * LD;                                                             \
      if constexpr (kET) {                                                                     \
        /* every problem: a term runs at its reduced tile, which the tile bounds keep     */   \
        /* within BMAX                                                                    */   \
        run_item<BMAX, true, COMP>(P, I.t0, I.t1, Cp, vp, parts + I.pad, L, acc_dd, saved,     \
                                   tlo, thi);                                                  \
      } else {                                                                                 \
        switch (P.B) {                                                                         \
          LH_FWD_CASE(1, COMP) LH_FWD_CASE(2, COMP) LH_FWD_CASE(3, COMP) LH_FWD_CASE(4, COMP)  \
          LH_FWD_CASE(5, COMP) LH_FWD_CASE(6, COMP) LH_FWD_CASE(7, COMP) LH_FWD_CASE(8, COMP)  \
          default:                                                                             \
            break;                                                                             \
        }                                                                                      \
      }                                                                                        \
    }                                                                                          \
  }
#define LH_FWD_CASE(BB, COMP)                                                               \
  case BB:                                                                                  \
    if constexpr (BB <= BMAX)                                                               \
      run_item<BB, false, COMP>(P, I.t0, I.t1, Cp, vp, parts + I.pad, L, acc_dd, saved, 1,  \
                                8);                                                         \
    break;
LH_FORWARD_KERNEL(forward_kernel, false)
LH_FORWARD_KERNEL(forward_comp_kernel, true)
#undef LH_FWD_CASE
#undef LH_FORWARD_KERNEL

#ifdef LH_COMMON_KERNELS
// Sum the item partials of each problem in item order (double-double),
// apply the FDS prefactor and write the result and an error estimate.
// With `raw` the prefactor is not applied (partial sums of a term range).
// parts2 (nullable): the partials of a second launch over the same items
// (the other tile class of a split ET sum), added after the first set.
__global__ void finalize_kernel(const Prob* __restrict__ probs, int nprob,
                                const Partial* __restrict__ parts,
                                const Partial* __restrict__ parts2, lh_c128* out, lh_c128* out_lo,
                                double* err, int acc_dd, int raw) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nprob) return;
  const Prob& P = probs[b];
  dd sr = {0.0, 0.0}, si = {0.0, 0.0};
  double sabs = 0.0;
  if (P.n == 0 && P.t0 < P.t1) {  // the empty matching: lhaf = 1
    sr.hi = 1.0;
    sabs = 1.0;
  }
  for (int set = 0; set < (parts2 ? 2 : 1); ++set) {
    const Partial* ps = set == 0 ? parts : parts2;
    for (int k = 0; k < P.n_items; ++k) {
      const Partial pr = ps[P.first_item + k];
      dd_add(sr, pr.hr, pr.lr);
      dd_add(si, pr.hi, pr.li);
      sabs += pr.abs_sum;
    }
  }
  const double sc = raw ? 1.0 : P.scale;  // power of two: exact
  sr.hi *= sc;
  sr.lo *= sc;
  si.hi *= sc;
  si.lo *= sc;
  sabs *= sc;
  // a non-finite input (an entry the problem reads) or an overflow makes the
  // whole result NaN, with err_est = +Inf
  const bool bad = !isfinite(sr.hi + sr.lo) || !isfinite(si.hi + si.lo) || !isfinite(sabs);
  if (bad) sr.hi = si.hi = sr.lo = si.lo = NAN;
  lh_c128 o;
  if (out_lo) {
    o.re = sr.hi;
    o.im = si.hi;
    lh_c128 ol;
    ol.re = sr.lo;
    ol.im = si.lo;
    out_lo[b] = ol;
  } else {
    o.re = sr.hi + sr.lo;
    o.im = si.hi + si.lo;
  }
  out[b] = o;
  if (err) {
    // per-term relative error of the Hessenberg / characteristic-polynomial
    // evaluation: kTermErrPerDim (m + 1) eps of every |c_t f_t|
    const double eps = 1.1102230246251565e-16;
    double rel_term = kTermErrPerDim * (P.m + 1) * eps;
    // plain FP64 sums each item's terms in order in one wavefront and the
    // item partials in double-double: the longest item bounds its rounding
    if (!acc_dd) rel_term += (double)lh_longest_item(P) * eps;
    double e = sabs * rel_term;
    if (bad || !isfinite(e)) e = INFINITY;
    err[b] = e;
  }
}

// Single-value writes for trivial problems (N = 0 gives 1).
__global__ void fill_one_kernel(lh_c128* out, lh_c128* out_lo, double* err, int count) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  lh_c128 one;
  one.re = 1.0;
  one.im = 0.0;
  out[b] = one;
  if (out_lo) {
    lh_c128 z;
    z.re = 0.0;
    z.im = 0.0;
    out_lo[b] = z;
  }
  if (err) err[b] = 0.0;
}

#endif  // LH_COMMON_KERNELS

}  // namespace lh
