// Multi-output loop-hafnian kernels: one pass over the terms of a problem
// serves several outputs (batching of probability calculations, App. B.5 of
// arXiv:2108.01622).
//
// Chain mode (one chain-rule step): outputs k = 0..n_cut are lhaf of the
// fixed pattern with the batched mode at k photons.  The problem's pairs are
// those of the fixed pattern, the batched mode paired with itself
// J = floor(n_cut/2) times, and the batched mode paired once with a padding
// vertex.  An ET term with weights z (App. B.1/B.2) serves output k when
// z_self <= floor(k/2) and z_pad <= k mod 2: the traces of W = C X_z are the
// same, only the binomial weights and the lambda degree
// n_k = n_fixed + floor(k/2) + (k mod 2) change, and every e_j, j <= n, comes
// out of the same series.  (The coupling of two copies of the batched mode is
// kept for the self pair; it cancels from the outputs where that pair repeats
// at most once.)
//
// Gamma mode (sub-detector batching): G loop-weight vectors for one matrix.
// W and its power traces do not depend on gamma, so per term the Hessenberg
// phase runs once and only the loop moments and the exponential series
// repeat per vector.
namespace lh {

struct MultiArgs {
  int32_t mode;      // 0 chain, 1 gamma
  int32_t nout;      // outputs (<= 64)
  int32_t pbb, pbp;  // chain: pair index of the self pair / the padding pair (-1: none)
  int32_t nf;        // chain: lambda degree of the fixed pairs
  int32_t pad;
  const cd* vg;      // gamma: packed loop vectors [nout][64]
};

// region after the forward layout (16-byte aligned)
__device__ __forceinline__ cd* lds_multi(const LdsView& L) { return L.ring + L.NP * L.NR; }

// LDS bytes of one multi-output wavefront: the forward layout, then for the
// gamma mode the exponential series of every vector plus one moment buffer.
inline size_t multi_lds_bytes(int nmax, int mode, int nout) {
  return lds_bytes_for(nmax) + (mode == 1 ? sizeof(cd) * 33 * (size_t)(nout + 2) : 0);
}

// lane's output accumulation of c * e (double-double or plain)
__device__ __forceinline__ void acc_term(dd& ar, dd& ai, double& sabs, const double c, const cd e,
                                         const int acc_dd) {
  if (acc_dd) {
    dd_add_prod(ar, c, e.r);
    dd_add_prod(ai, c, e.i);
  } else {
    ar.hi = fma(c, e.r, ar.hi);
    ai.hi = fma(c, e.i, ai.hi);
  }
  sabs = fma(fabs(c), sqrt(cabs2(e)), sabs);
}

template <int B, int MODE>
__device__ __forceinline__ void run_item_multi(const Prob& P, const int64_t t0, const int64_t t1,
                                               const cd* __restrict__ Cp,
                                               const cd* __restrict__ vp,
                                               Partial* __restrict__ out, LdsView& L,
                                               const int acc_dd, const MultiArgs& ma) {
  const int lane0 = threadIdx.x & 63;
  const int m = P.m, H = P.H, n = P.n;
  cd* Lbuf = lds_multi(L);   // gamma: [nout + 1][33] exponential series
  cd* mu2 = Lbuf + 33 * (ma.nout + 1);  // second moment buffer
  TermIter it = term_begin(P, t0, lane0);
  dd accr = {0.0, 0.0}, acci = {0.0, 0.0};  // lane o: output o
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
    if constexpr (MODE == 1) {
      double dcol[B];
      column_weights<B>(wl, m, H, q, dcol);
      double Wr[B][B], Wi[B][B];
      load_w<B>(Cp, dcol, p, q, Wr, Wi);
      // loop moments of every vector (W intact), exponential series two at a time
      for (int g = 0; g < ma.nout; g += 2) {
        LdsView La = L;
        loop_moments<B>(Wr, Wi, dcol, ma.vg + 64 * g, m, H, n, p, q, lane, La);
        const bool two = g + 1 < ma.nout;
        if (two) {
          LdsView Lb = L;
          Lb.mu = mu2;
          loop_moments<B>(Wr, Wi, dcol, ma.vg + 64 * (g + 1), m, H, n, p, q, lane, Lb);
        }
        two_series(L.mu, Lbuf + 33 * g, 0.0, mu2, Lbuf + 33 * (two ? g + 1 : ma.nout), 0.0, n,
                   lane);
      }
      spectral_series<B>(Wr, Wi, m, n, p, q, lane, L);  // q_k in L.ser[0..n]
      if (lane < ma.nout) {
        const cd* Lg = Lbuf + 33 * lane;
        cd f0 = czero(), f1 = czero();
        int j = 0;
        for (; j + 1 <= n; j += 2) {
          f0 = cfma(L.ser[j], Lg[n - j], f0);
          f1 = cfma(L.ser[j + 1], Lg[n - j - 1], f1);
        }
        if (j <= n) f0 = cfma(L.ser[j], Lg[n - j], f0);
        acc_term(accr, acci, sabs, coef, cadd(f0, f1), acc_dd);
      }
    } else {
      // chain outputs are ET sums: the term runs on its kept pairs only
      // (tile ceil(2H'/8) <= B), see kept_map; the series land in L.ser
      int* km = reinterpret_cast<int*>(L.wv);
      cd* vred = L.xb + 64;
      const int Hk = kept_map(it, H, lane, km);
      const int mk_ = 2 * Hk;
      vred[lane] = lane < mk_ ? vp[km[lane]] : czero();
      wave_sync();
      (void)term_f_at<B>((mk_ + 7) >> 3, Cp, 8 * P.B, vred, km, wl, mk_, Hk, H, n, p, q, lane, L);
      const int zbb = ma.pbb >= 0 ? __builtin_amdgcn_readlane(it.digit, ma.pbb) : 0;
      const int zbp = ma.pbp >= 0 ? __builtin_amdgcn_readlane(it.digit, ma.pbp) : 0;
      // binomial weights of the fixed pairs, parity of sum z
      const bool fixed = lane < H && lane != ma.pbb && lane != ma.pbp;
      const double cf = prod_wave(fixed ? c_binom.v[it.eta_l][it.digit] : 1.0, lane);
      const int zpar = __popcll(__ballot(lane < H && (it.digit & 1))) & 1;
      if (lane < ma.nout) {
        const int jk = lane >> 1, ok = lane & 1;
        const int nk = ma.nf + jk + ok;
        const double cb = c_binom.v[jk][zbb] * c_binom.v[ok][zbp];
        if (cb != 0.0 && nk >= 1) {
          cd e0 = czero(), e1 = czero();
          int i = 0;
          for (; i + 1 <= nk; i += 2) {
            e0 = cfma(L.ser[i], L.ser[33 + nk - i], e0);
            e1 = cfma(L.ser[i + 1], L.ser[33 + nk - i - 1], e1);
          }
          if (i <= nk) e0 = cfma(L.ser[i], L.ser[33 + nk - i], e0);
          const double sign = ((nk + zpar) & 1) ? -1.0 : 1.0;
          acc_term(accr, acci, sabs, sign * cf * cb, cadd(e0, e1), acc_dd);
        }
      }
    }
    wave_sync();
  }
  if (lane0 < ma.nout) {
    Partial pr;
    pr.hr = accr.hi;
    pr.hi = acci.hi;
    pr.lr = accr.lo;
    pr.li = acci.lo;
    pr.abs_sum = sabs;
    pr.pad0 = pr.pad1 = pr.pad2 = 0.0;
    out[lane0] = pr;
  }
}

template <int BMAX, int MODE>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(LH_FWD_WAVES(BMAX), LH_FWD_WAVES(BMAX)))) void multi_kernel(
    const Prob* __restrict__ probs, const Item* __restrict__ items, int n_items, int* counter,
    const cd* __restrict__ ws, Partial* __restrict__ parts, int acc_dd, int nmax, MultiArgs ma) {
  extern __shared__ __align__(16) char lds_raw[];
  LdsView L = carve(lds_raw, nmax);
  const int lane = threadIdx.x & 63;
  for (;;) {
    // every lane issues the atomic (see forward_kernel)
    const int it = __builtin_amdgcn_readfirstlane(atomicAdd(counter, lane == 0 ? 1 : 0));
    if (it >= n_items) break;
    const Item I = items[it];
    const Prob& P = probs[I.prob];
    const int LD = 8 * P.B;
    const cd* Cp = ws + P.c_off;
    const cd* vp = Cp + LD * LD;
    Partial* out = parts + (int64_t)I.pad * ma.nout;
    if constexpr (MODE == 0) {  // per-term tiles inside (pair deletion)
      if (P.B <= BMAX) run_item_multi<BMAX, 0>(P, I.t0, I.t1, Cp, vp, out, L, acc_dd, ma);
    } else {
      switch (P.B) {
#define LH_MCASE(BB)                                                                        \
  case BB:                                                                                  \
    if (BB <= BMAX) run_item_multi<(BB <= BMAX ? BB : 1), MODE>(P, I.t0, I.t1, Cp, vp, out, L, acc_dd, ma); \
    break;
        LH_MCASE(1)
        LH_MCASE(2)
        LH_MCASE(3)
        LH_MCASE(4)
        LH_MCASE(5)
        LH_MCASE(6)
        LH_MCASE(7)
        LH_MCASE(8)
#undef LH_MCASE
        default:
          break;
      }
    }
  }
}

#ifdef LH_COMMON_KERNELS
// gamma mode: vg[g][i] = gamma_g[mode of vertex i] (1 for padding, 0 beyond m)
__global__ void pack_gammas_kernel(const Prob* __restrict__ probs, const lh_c128* __restrict__ g,
                                   int64_t ldg, int G, cd* __restrict__ vg) {
  const Prob& P = probs[0];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 64 * G; e += gridDim.x * blockDim.x) {
    const int gi = e / 64, i = e % 64;
    cd val = czero();
    if (i < P.m) {
      const int pi = P.pos[i];
      if (pi < 0) val = mk(1.0, 0.0);
      else {
        const lh_c128 x = g[(int64_t)gi * ldg + pi];
        val = mk(x.re, x.im);
      }
    }
    vg[e] = val;
  }
}

// Output o = sum of the item partials in item order (double-double), times
// the FDS prefactor; chain outputs of lambda degree 0 are 1.
__global__ void finalize_multi_kernel(const Prob* __restrict__ probs,
                                      const Partial* __restrict__ parts, MultiArgs ma,
                                      lh_c128* out, double* err, int acc_dd) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= ma.nout) return;
  const Prob& P = probs[0];
  dd sr = {0.0, 0.0}, si = {0.0, 0.0};
  double sabs = 0.0;
  const bool empty_out = ma.mode == 0 ? (ma.nf + (o >> 1) + (o & 1) == 0) : (P.n == 0);
  if (empty_out && P.t0 < P.t1) {
    sr.hi = 1.0;
    sabs = 1.0;
  }
  for (int k = 0; k < P.n_items; ++k) {
    const Partial pr = parts[(int64_t)(P.first_item + k) * ma.nout + o];
    dd_add(sr, pr.hr, pr.lr);
    dd_add(si, pr.hi, pr.li);
    sabs += pr.abs_sum;
  }
  const double sc = P.scale;
  lh_c128 r;
  r.re = (sr.hi + sr.lo) * sc;
  r.im = (si.hi + si.lo) * sc;
  const bool bad = !isfinite(r.re) || !isfinite(r.im) || !isfinite(sabs);
  if (bad) r.re = r.im = NAN;  // non-finite input or overflow
  out[o] = r;
  if (err) {
    const double eps = 1.1102230246251565e-16;
    double rel_term = kTermErrPerDim * (P.m + 1) * eps;
    // plain FP64 sums each item's terms in order in one wavefront and the
    // item partials in double-double: the longest item bounds its rounding
    if (!acc_dd) rel_term += (double)lh_longest_item(P) * eps;
    double e = sabs * sc * rel_term;
    if (bad || !isfinite(e)) e = INFINITY;
    err[o] = e;
  }
}

#endif  // LH_COMMON_KERNELS

}  // namespace lh
