// Adjoint kernels: gradients of loop hafnians (the paper has none; this is
// the reverse pass of the per-term power-trace recursion of App. B.1/B.2).
//
// Per term, with W = C X_d, u = X_d v, g_k = Tr(W^k)/(2k) + u^T W^{k-1} v / 2
// and f = [lambda^n] exp(sum_k g_k lambda^k) = sum_j ... with coefficients
// e_j = [lambda^j] exp(G):
//   d f / d g_k = e_{n-k}                    (d exp(G)/d g_k = lambda^k exp(G))
//   a_k := e_{n-k} / 2
//   (d f / d W)^T = P(W) + sum_{i+j<=n-2} a_{i+j+2} b_j alpha_i^T
//       P(x) = sum_{k=1..n} a_k x^{k-1},  b_j = W^j v,  alpha_i = (W^T)^i u
//   d f / d v = sum_k a_k (alpha_{k-1} + X_d b_{k-1})
//   d f / d C = (d f / d W) X_d.
// P(W) is evaluated by Paterson-Stockmeyer (s = ceil(sqrt n): powers
// W^1..W^s, then Horner in W^s), the dense contraction of this path; the
// products keep one operand in registers (8 x 8 lane grid, row broadcasts by
// ds_bpermute) and stream the other.  For register tiles B <= kStageMaxB the
// streamed operand (W while the powers are formed, then W^s) and the Krylov
// vectors live in a per-wavefront LDS region X, so the products and the
// rank-one terms never wait on global memory; the powers that the Horner
// steps combine elementwise go to a per-wavefront scratch in global memory.
// Larger tiles (whose LDS share would cut occupancy) keep everything in the
// global scratch.  Terms are recomputed per subset; nothing is stored across
// terms except the running gradient of the item.
namespace lh {

constexpr int kMaxPS = 6;      // ceil(sqrt(32))
#ifndef LH_STAGE_MAX_B
#define LH_STAGE_MAX_B 5
#endif
constexpr int kStageMaxB = LH_STAGE_MAX_B;  // largest register tile with LDS staging

// The same address as p, opaque to the optimiser (forces a fresh load).
template <class T>
__device__ __forceinline__ const T* launder_ptr(const T* p) {
  uint64_t v = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(v));
  return reinterpret_cast<const T*>(v);
}

__host__ __device__ inline size_t bwd_wave_scratch_elems(int B) {
  const size_t LD = 8 * (size_t)B;
  return kMaxPS * LD * LD + 33 * 64;
}
__host__ __device__ inline size_t bwd_item_elems(int B) {
  const size_t LD = 8 * (size_t)B;
  return LD * LD + 64;
}
// Which instance runs a backward launch of largest tile bmax: the LDS-staged
// one (one wavefront per SIMD, the operand and Krylov vectors in LDS) for
// tiles up to kStageMaxB when the coefficients come from the store, but only
// up to LH_STAGE_RECOMPUTE_MAX_B when the launch recomputes them (fused pass
// or recomputing backward): there tiles 4 and 5 run unstaged at two
// wavefronts per SIMD, whose second wavefront hides the latency of the term's
// spectral phase (measured fused pass: N = 40 4.47 vs 4.19, N = 32 7.92 vs
// 6.95 M terms/s; three wavefronts at tile 4 6.71); from the store the
// staged instance stays ahead (N = 40 6.82 vs 5.51).
#ifndef LH_STAGE_RECOMPUTE_MAX_B
#define LH_STAGE_RECOMPUTE_MAX_B 3
#endif
__host__ __device__ constexpr bool bwd_staged(int bmax, bool from_store) {
  return bmax <= (from_store ? kStageMaxB : LH_STAGE_RECOMPUTE_MAX_B);
}
// complex elements of the LDS region X of a backward kernel instance (0
// without staging): the larger of one LD x LD matrix and nmax Krylov vectors
// of LD entries.
__host__ __device__ inline size_t bwd_x_elems(int bmax, int nmax, bool staged) {
  if (!staged) return 0;
  const size_t LD = 8 * (size_t)bmax;
  return LD * (LD > (size_t)nmax ? LD : (size_t)nmax);
}
inline size_t bwd_lds_bytes(int bmax, int nmax, bool staged) {
  return lds_bytes_for(nmax) + sizeof(cd) * bwd_x_elems(bmax, nmax, staged);
}
// Lanes of the wavefront exchange data through LDS only when staging (and
// through the global scratch otherwise, which needs the full barrier).
template <bool kLds>
__device__ __forceinline__ void lane_sync() {
  if constexpr (kLds) wave_sync();
  else __syncthreads();
}

// X starts after the forward layout (16-byte aligned)
__device__ __forceinline__ cd* lds_x(const LdsView& L) { return L.ring + L.NP * L.NR; }

// R <- R * M with R in registers (lane (p,q) holds R[8a+p][8k+q]) and M
// row-major LD x LD (global).  Output row i needs only input row i, so rows
// are done in groups of G local rows, in place: only the group's
// accumulators are live, and M is streamed once per group.
template <int B, int G, int A0>
__device__ __forceinline__ void mul_rows(double (&Rr)[B][B], double (&Ri)[B][B],
                                         const cd* __restrict__ M, const int p, const int q) {
  if constexpr (A0 < B) {
    constexpr int LD = 8 * B;
    constexpr int NG = (A0 + G <= B) ? G : (B - A0);
    double Or[NG][B], Oi[NG][B];
#pragma unroll
    for (int a = 0; a < NG; ++a)
#pragma unroll
      for (int k = 0; k < B; ++k) Or[a][k] = Oi[a][k] = 0.0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll 2
      for (int r = 0; r < 8; ++r) {
        const int l = 8 * b + r;
        cd mrow[B];
#pragma unroll
        for (int k = 0; k < B; ++k) mrow[k] = M[l * LD + 8 * k + q];
        const int src = (p << 3) | r;
#pragma unroll
        for (int a = 0; a < NG; ++a) {
          const cd x = mk(shfl_d(Rr[A0 + a][b], src), shfl_d(Ri[A0 + a][b], src));
#pragma unroll
          for (int k = 0; k < B; ++k) {
            const cd o = cfma(x, mrow[k], mk(Or[a][k], Oi[a][k]));
            Or[a][k] = o.r;
            Oi[a][k] = o.i;
          }
        }
      }
    }
#pragma unroll
    for (int a = 0; a < NG; ++a)
#pragma unroll
      for (int k = 0; k < B; ++k) {
        Rr[A0 + a][k] = Or[a][k];
        Ri[A0 + a][k] = Oi[a][k];
      }
    mul_rows<B, G, A0 + G>(Rr, Ri, M, p, q);
  }
}

// Row l of the product O += R[:, l] M[l, :] with compile-time l: R[8a+p][l]
// reaches the row group by a DPP broadcast from lane (p, l mod 8), with no
// LDS round trip; the operand row of M for l + 1 is fetched into the other
// buffer while row l is used, and a scheduling barrier keeps the live
// operands to two rows.
template <int B, int L>
__device__ __forceinline__ void product_rows(const double (&Rr)[B][B], const double (&Ri)[B][B],
                                             double (&Or)[B][B], double (&Oi)[B][B],
                                             cd (&mcur)[B], cd (&mnxt)[B],
                                             const cd* __restrict__ M, const int q) {
  constexpr int LD = 8 * B;
  if constexpr (L < LD) {
    constexpr int b = L / 8, r = L % 8;
    if constexpr (L + 1 < LD) {
#pragma unroll
      for (int k = 0; k < B; ++k) mnxt[k] = M[(L + 1) * LD + 8 * k + q];
    }
    double xr[B], xi[B];
#pragma unroll
    for (int a = 0; a < B; ++a) {
      xr[a] = bcast_row8_lo<r>(Rr[a][b]);
      xi[a] = bcast_row8_lo<r>(Ri[a][b]);
    }
#pragma unroll
    for (int a = 0; a < B; ++a) {
      xr[a] = bcast_row8_hi<r>(xr[a], Rr[a][b]);
      xi[a] = bcast_row8_hi<r>(xi[a], Ri[a][b]);
    }
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const cd o = cfma(mk(xr[a], xi[a]), mcur[k], mk(Or[a][k], Oi[a][k]));
        Or[a][k] = o.r;
        Oi[a][k] = o.i;
      }
    __builtin_amdgcn_sched_barrier(0);
    product_rows<B, L + 1>(Rr, Ri, Or, Oi, mnxt, mcur, M, q);
  }
}

// R <- R * M for the LDS-staged tiles: all output rows at once, M read once.
template <int B>
__device__ __forceinline__ void mul_right_dpp(double (&Rr)[B][B], double (&Ri)[B][B],
                                              const cd* __restrict__ M, const int q) {
  double Or[B][B], Oi[B][B];
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int k = 0; k < B; ++k) Or[a][k] = Oi[a][k] = 0.0;
  cd m0[B], m1[B];
#pragma unroll
  for (int k = 0; k < B; ++k) m0[k] = M[8 * k + q];
  product_rows<B, 0>(Rr, Ri, Or, Oi, m0, m1, M, q);
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int k = 0; k < B; ++k) {
      Rr[a][k] = Or[a][k];
      Ri[a][k] = Oi[a][k];
    }
}

// row-group size of the unstaged products: all row groups at once (M
// streamed once) up to B = 7; one at a time at B = 8, where a second full
// accumulator next to R does not fit the register file (measured: B = 7
// 0.62 vs 0.49 M terms/s all-at-once vs one group, B = 8 0.09 vs 0.24)
#ifndef LH_MULG
#define LH_MULG(B) ((B) <= 7 ? (B) : 1)
#endif
// opaque lane index per term in the backward kernels of the unstaged tiles
// (kernel BMAX >= 6; measured +7 % at B = 6, +16 % at B = 7, -3 % at
// B = 5).  Decided per kernel, not per item: every item path of a kernel
// shares its register allocation.
#ifndef LH_BWD_OPAQUE
#define LH_BWD_OPAQUE(unstaged) (unstaged)
#endif
__host__ __device__ constexpr int mul_group(int B) { return LH_MULG(B); }
// Products of the unstaged tiles 6 and 7 in the LDS-staged form (all row
// groups at once, DPP row broadcasts of R at compile-time rows, the next
// operand row prefetched) with the operand read from the global scratch
// instead of LDS: measured +9 % at B = 6 and +14 % at B = 7 over the
// ds_bpermute rows (fused pass N = 48 1.74 vs 1.59, N = 52 1.01 vs 0.89 M
// terms/s).  Tile 8 keeps one row group at a time (two full accumulators do
// not fit the register file).
#ifndef LH_UNSTAGED_DPP
#define LH_UNSTAGED_DPP(B) ((B) >= 4 && (B) <= 7)
#endif

template <int B>
__device__ __forceinline__ void mul_right(double (&Rr)[B][B], double (&Ri)[B][B],
                                          const cd* __restrict__ M, const int p, const int q) {
  mul_rows<B, mul_group(B), 0>(Rr, Ri, M, p, q);
}

template <int B>
__device__ __forceinline__ void store_mat(const double (&Rr)[B][B], const double (&Ri)[B][B],
                                          cd* __restrict__ M, const int p, const int q) {
  constexpr int LD = 8 * B;
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int k = 0; k < B; ++k) M[(8 * a + p) * LD + 8 * k + q] = mk(Rr[a][k], Ri[a][k]);
}

// Krylov sequence b_j = W^j v (0 <= j < n) into bv (vector j at bv + S j,
// entry = vertex; rows up to 8B are written, zero beyond m) and the loop
// moments mu_k = u . b_{k-1} (u = X_d v) into L.mu.  The second sequence
// alpha_i = (W^T)^i u needs no products: X_d W is symmetric, so
// (W^T)^i X_d = X_d W^i and alpha_i = X_d b_i, i.e.
// alpha_i[c] = d_{pair(c)} b_i[partner(c)].
template <int B, int S, bool kLds>
__device__ __forceinline__ void krylov_b(const double (&Wr)[B][B], const double (&Wi)[B][B],
                                         const double dlane, const cd* __restrict__ vp,
                                         const int m, const int H, const int n, const int p,
                                         const int q, const int lane, cd* __restrict__ bv,
                                         LdsView& L, const bool with_mu) {
  if (lane < 8 * B) bv[lane] = vp[lane];
  lane_sync<kLds>();
  for (int j = 0; j + 1 < n; ++j) {
    cd xc[B];
#pragma unroll
    for (int k = 0; k < B; ++k) xc[k] = bv[S * j + 8 * k + q];
#pragma unroll
    for (int a = 0; a < B; ++a) {
      cd y = czero();
#pragma unroll
      for (int k = 0; k < B; ++k) y = cfma(mk(Wr[a][k], Wi[a][k]), xc[k], y);
      y = sum_row8(y);
      if (q == 0) bv[S * (j + 1) + 8 * a + p] = y;
    }
    lane_sync<kLds>();
  }
  if (!with_mu) return;
  // mu_k = sum_c u_c b_{k-1}[c], u_c = d_{pair(c)} v_{partner(c)}
  const int pl = lane < H ? lane + H : lane - H;
  const cd ul = lane < m ? cscale(dlane, vp[pl & 63]) : czero();
  for (int k = 1; k <= n; ++k) {
    const cd t = lane < m ? cmul(ul, bv[S * (k - 1) + lane]) : czero();
    const double re = sum_col8(sum_row8(t.r));
    const double im = sum_col8(sum_row8(t.i));
    if (lane == 0) L.mu[k] = mk(re, im);
  }
  lane_sync<kLds>();
}

// R += sum_{i+j <= n-2} a_{i+j+2} b_j alpha_i^T = sum_i beta_i alpha_i^T with
// beta_i = sum_j a_{i+j+2} b_j (each lane forms beta_i at its own vertex and
// the grid reads it back through the LDS buffer xb).
template <int B, int S>
__device__ __forceinline__ void rank_terms(double (&Rr)[B][B], double (&Ri)[B][B],
                                           const cd* __restrict__ bv, const cd* __restrict__ acoef,
                                           const double (&dcol)[B], const int m, const int H,
                                           const int n, const int p, const int q,
                                           const int lane, cd* __restrict__ xb) {
  for (int i = 0; i + 2 <= n; ++i) {
    cd b0 = czero(), b1 = czero();
    if (lane < m) {
      int j = 0;
      for (; i + j + 3 <= n; j += 2) {
        b0 = cfma(acoef[i + j + 2], bv[S * j + lane], b0);
        b1 = cfma(acoef[i + j + 3], bv[S * (j + 1) + lane], b1);
      }
      if (i + j + 2 <= n) b0 = cfma(acoef[i + j + 2], bv[S * j + lane], b0);
    }
    cd* bb = xb + 64 * (i & 1);
    bb[lane] = cadd(b0, b1);
    wave_sync();
    cd al[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int c = 8 * k + q;
      const int pc = c < H ? c + H : c - H;
      al[k] = c < m ? cscale(dcol[k], bv[S * i + pc]) : czero();
    }
    // small tiles load every beta first (the LDS latencies overlap); larger
    // ones one row group at a time, so only its beta is live next to R
    constexpr int NB = B <= 5 ? B : 1;
    cd beta[NB];
    if constexpr (B <= 5) {
#pragma unroll
      for (int a = 0; a < B; ++a) beta[a] = bb[8 * a + p];
    }
#pragma unroll
    for (int a = 0; a < B; ++a) {
      const cd be = B <= 5 ? beta[a < NB ? a : 0] : bb[8 * a + p];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const cd o = cfma(be, al[k], mk(Rr[a][k], Ri[a][k]));
        Rr[a][k] = o.r;
        Ri[a][k] = o.i;
      }
    }
  }
}

// d of the pairs of the lane's rows i = 8a+p (0 beyond m)
template <int B>
__device__ __forceinline__ void row_weights(const double wl, const int m, const int H, const int p,
                                            double (&drow)[B]) {
#pragma unroll
  for (int a = 0; a < B; ++a) {
    const int i = 8 * a + p;
    const int pi = i < H ? i : i - H;
    const double d = shfl_d(wl, pi & 63);
    drow[a] = i < m ? d : 0.0;
  }
}

// G[row][col] += w_row R[row][col] (pointer laundered so the loads are not
// hoisted above the computation of R)
template <int B>
__device__ __forceinline__ void accumulate_g(cd* __restrict__ G, const double coef,
                                             const double (&drow)[B], const double (&Rr)[B][B],
                                             const double (&Ri)[B][B], const int p, const int q) {
  constexpr int LD = 8 * B;
  cd* Gl = const_cast<cd*>(launder_ptr(G));
#pragma unroll
  for (int a = 0; a < B; ++a) {
    const double w = coef * drow[a];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      cd* g = Gl + (8 * a + p) * LD + 8 * k + q;
      *g = cfma(mk(w, 0.0), mk(Rr[a][k], Ri[a][k]), *g);
    }
  }
}

// R <- B_q (reset) or R + B_q, B_q = a_{qs+1} I + sum_{r=1..s-1} a_{qs+r+1} W^r
// with W^r read from the wavefront scratch (one row block per batch of loads).
template <int B>
__device__ __forceinline__ void combine_powers(double (&Rr)[B][B], double (&Ri)[B][B],
                                               const bool reset, const cd* __restrict__ pw,
                                               const cd* __restrict__ acoef, const int qq,
                                               const int s, const int n, const int m,
                                               const int p, const int q) {
  constexpr int LD = 8 * B;
  const cd ak = acoef[qq * s + 1];
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int i = 8 * a + p, c = 8 * k + q;
      if (reset) Rr[a][k] = Ri[a][k] = 0.0;
      if (i == c && i < m) {
        Rr[a][k] += ak.r;
        Ri[a][k] += ak.i;
      }
    }
  for (int r = 1; r < s && qq * s + r + 1 <= n; ++r) {
    const cd a1 = acoef[qq * s + r + 1];
    const cd* P1 = pw + (r - 1) * LD * LD;
#pragma unroll
    for (int a = 0; a < B; ++a) {
      cd x1[B];
#pragma unroll
      for (int k = 0; k < B; ++k) x1[k] = P1[(8 * a + p) * LD + 8 * k + q];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const cd o = cfma(a1, x1[k], mk(Rr[a][k], Ri[a][k]));
        Rr[a][k] = o.r;
        Ri[a][k] = o.i;
      }
    }
  }
}

// Gradient of the terms [t0, t1) of problem P into the item slot
// G[LD*LD] (accumulated as sum_t c_t d_{pair(j)} M_t[j][c], M = (d f/d W)^T)
// and G[LD*LD + l] (d f / d v_l).  With a coefficient store written by the
// forward pass, the a_k are read instead of recomputed.
//
// With `part` (fused pass, no store), the item also accumulates its share of
// the value: the recomputed series give f = sum_k q_k L_{n-k} of every term,
// added as c_t f_t into a double-double (acc_dd) or plain partial, exactly as
// the forward kernel does.
template <int B, bool kStage, bool kRankLate = false>
__device__ __forceinline__ void run_item_bwd(const Prob& P, const int64_t t0, const int64_t t1,
                                             const cd* __restrict__ Cp,
                                             const cd* __restrict__ vp, cd* __restrict__ G,
                                             cd* __restrict__ scr, LdsView& L,
                                             const cd* __restrict__ saved,
                                             Partial* __restrict__ part, const int acc_dd) {
  constexpr int LD = 8 * B;
  constexpr int S = kStage ? LD : 64;    // stride of the Krylov vectors
  const int lane0 = threadIdx.x & 63;
  const int m = P.m, H = P.H, n = P.n;
  cd* pw = scr;                                          // [kMaxPS][LD*LD] powers
  cd* X = lds_x(L);                                      // staging region (kStage)
  cd* bv = kStage ? X : scr + kMaxPS * LD * LD;          // Krylov vectors
  cd* acoef = L.wb;                                      // a_1..a_n (index k)

  // The item's gradient accumulators: d f / d v in one register per lane,
  // the matrix part in the item's slot (a register copy next to the products
  // spills: measured 1.2 KB/lane at B = 5).
  cd gv = czero();
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int k = 0; k < B; ++k) G[(8 * a + (lane0 >> 3)) * LD + 8 * k + (lane0 & 7)] = czero();

  // Paterson-Stockmeyer split s = ceil(sqrt n); for tiles whose powers live
  // in the global scratch, lowered while the product count (s - 1) +
  // ceil(n / s) - 1 stays the same, so fewer powers are stored and re-read
  // (n = 26: s = 4 instead of 6, 3 stored powers instead of 5)
  int s = 1;
  while (s * s < n) ++s;
  if constexpr (!kStage)
    while (s > 2 && (s - 2) + (n + s - 2) / (s - 1) <= (s - 1) + (n + s - 1) / s) --s;
  const int Q = (n + s - 1) / s - 1;
  // The item's value partial (fused pass) lives in LDS, in the scalar slots
  // after the reflector's (hr, lr, hi, li, abs), read and written by lane 0
  // only: in registers it would stay live through the whole term.
  double* vacc = L.sc + 3;
  if (part && lane0 == 0) {
#pragma unroll
    for (int k = 0; k < 5; ++k) vacc[k] = 0.0;
  }

  TermIter it = term_begin(P, t0, lane0);
  for (int64_t t = t0; t < t1; ++t) {
    // lane index of this term (opaque for large tiles, see LH_BWD_OPAQUE)
    int lane = lane0;
    LH_OPAQUE(LH_BWD_OPAQUE(!kStage), lane);
    const int p = lane >> 3, q = lane & 7;
    if (t != t0) term_next(it, H, lane);
    double coef;
    bool empty;
    const double wl = term_weight(it, P, lane, coef, empty);
    if (empty) {
      lane_sync<kStage>();
      continue;
    }
    // The pair weights of the lane's rows and columns: held through the term
    // for the LDS-staged tiles, re-derived from wl (one value per lane) at
    // each use for the larger ones, where they would sit next to the
    // matrices in the register file.
    double dcol_k[B], drow_k[B];
    if constexpr (kStage) {
      column_weights<B>(wl, m, H, q, dcol_k);
      row_weights<B>(wl, m, H, p, drow_k);
    }
    const int lpair = lane < H ? lane : lane - H;
    const double dsh = shfl_d(wl, lpair & 63);
    const double dlane = lane < m ? dsh : 0.0;

    cd asaved = czero();
    if (saved && lane >= 1 && lane <= n) asaved = saved[P.s_off + (t - P.t0) * n + (lane - 1)];
    double Wr[B][B], Wi[B][B];
    if constexpr (kStage) {
      load_w<B>(Cp, dcol_k, p, q, Wr, Wi);
    } else {
      double dcol[B];
      column_weights<B>(wl, m, H, q, dcol);
      load_w<B>(Cp, dcol, p, q, Wr, Wi);
    }
    krylov_b<B, S, kStage>(Wr, Wi, dlane, vp, m, H, n, p, q, lane, bv, L, saved == nullptr);
    if (saved) {
      if (lane >= 1 && lane <= n) acoef[lane] = asaved;
    } else {
      spectral_series<B>(Wr, Wi, m, n, p, q, lane, L);
      if (lane >= 1 && lane <= n) acoef[lane] = series_coef(L, n, lane);
      if (part) {
        cd f = czero();
        if (lane <= n) f = cmul(L.ser[lane], L.ser[33 + n - lane]);
        f = mk(sum_col8(sum_row8(f.r)), sum_col8(sum_row8(f.i)));
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
      }
    }
    lane_sync<kStage>();

    double Rr[B][B], Ri[B][B];
    // ---- rank-one terms sum_i beta_i alpha_i^T.  Added to the item gradient
    // here, while the Krylov vectors are resident (a staged tile's P(W)
    // operand overwrites them in LDS); with kRankLate (unstaged, vectors in
    // the global scratch) they are added to P(W) in registers after the
    // products instead, one read-modify-write of the gradient slot per term.
    if constexpr (!kRankLate) {
#pragma unroll
      for (int a = 0; a < B; ++a)
#pragma unroll
        for (int k = 0; k < B; ++k) Rr[a][k] = Ri[a][k] = 0.0;
      if constexpr (kStage) {
        rank_terms<B, S>(Rr, Ri, bv, acoef, dcol_k, m, H, n, p, q, lane, L.xb);
      } else {
        double dcol[B];
        column_weights<B>(wl, m, H, q, dcol);
        rank_terms<B, S>(Rr, Ri, bv, acoef, dcol, m, H, n, p, q, lane, L.xb);
      }
      if constexpr (kStage) {
        accumulate_g<B>(G, coef, drow_k, Rr, Ri, p, q);
      } else {
        double drow[B];
        row_weights<B>(wl, m, H, p, drow);
        accumulate_g<B>(G, coef, drow, Rr, Ri, p, q);
      }
    }
    // ---- d f / d v_l = sum_k a_k (alpha_{k-1}[l] + d_{pair(l)} b_{k-1}[partner(l)])
    //                  = 2 sum_k a_k d_{pair(l)} b_{k-1}[partner(l)]
    if (lane < m) {
      const int pl = lane < H ? lane + H : lane - H;
      cd g0 = czero(), g1 = czero();
      int k = 1;
      for (; k + 1 <= n; k += 2) {
        g0 = cfma(acoef[k], bv[S * (k - 1) + pl], g0);
        g1 = cfma(acoef[k + 1], bv[S * k + pl], g1);
      }
      if (k <= n) g0 = cfma(acoef[k], bv[S * (k - 1) + pl], g0);
      gv = cfma(mk(2.0 * coef * dlane, 0.0), cadd(g0, g1), gv);
    }
    lane_sync<kStage>();

    // ---- P(W) = sum_{k=1..n} a_k W^{k-1} by Paterson-Stockmeyer.  W is
    // re-read from L2 (the pointer is hidden from the optimiser so it does
    // not keep the first copy live through the Hessenberg phase).
    const cd* Cp2 = launder_ptr(Cp);
    if constexpr (kStage) {
      load_w<B>(Cp2, dcol_k, p, q, Rr, Ri);
    } else {
      double dcol[B];
      column_weights<B>(wl, m, H, q, dcol);
      load_w<B>(Cp2, dcol, p, q, Rr, Ri);
    }
    if (kStage) store_mat<B>(Rr, Ri, X, p, q);
    if (s > 1) store_mat<B>(Rr, Ri, pw, p, q);  // W^1
    lane_sync<kStage>();
    const cd* Wop = kStage ? X : pw;
    cd* Yop = kStage ? X : pw + (s - 1) * LD * LD;
    // One product per step (a single call site keeps the unrolled product
    // code once): steps 0..s-2 form W^2..W^s (R = W^{step+2}); then R = B_Q
    // and steps s-1 .. s-2+Q are the Horner steps R <- R W^s + B_q,
    // q = Q-1 .. 0, where B_q = sum_{r=0..s-1} a_{qs+r+1} W^r.
    if (s == 1) combine_powers<B>(Rr, Ri, true, pw, acoef, Q, s, n, m, p, q);
    const int nsteps = (s - 1) + Q;
    for (int step = 0; step < nsteps; ++step) {
      if constexpr (kStage) mul_right_dpp<B>(Rr, Ri, X, q);
      else if constexpr (LH_UNSTAGED_DPP(B)) mul_right_dpp<B>(Rr, Ri, step < s - 1 ? Wop : Yop, q);
      else mul_right<B>(Rr, Ri, step < s - 1 ? Wop : Yop, p, q);
      if (step < s - 2) {
        store_mat<B>(Rr, Ri, pw + (step + 1) * LD * LD, p, q);  // W^{step+2}
        lane_sync<kStage>();
      } else if (step == s - 2) {
        lane_sync<kStage>();  // every read of W precedes its overwrite
        store_mat<B>(Rr, Ri, Yop, p, q);
        lane_sync<kStage>();
        combine_powers<B>(Rr, Ri, true, pw, acoef, Q, s, n, m, p, q);
      } else {
        combine_powers<B>(Rr, Ri, false, pw, acoef, Q - 1 - (step - (s - 1)), s, n, m, p, q);
      }
    }
    if constexpr (kStage) {
      accumulate_g<B>(G, coef, drow_k, Rr, Ri, p, q);
    } else {
      if constexpr (kRankLate) {
        double dcol[B];
        column_weights<B>(wl, m, H, q, dcol);
        rank_terms<B, S>(Rr, Ri, bv, acoef, dcol, m, H, n, p, q, lane, L.xb);
      }
      double drow[B];
      row_weights<B>(wl, m, H, p, drow);
      accumulate_g<B>(G, coef, drow, Rr, Ri, p, q);
    }
    lane_sync<kStage>();
  }
  G[LD * LD + lane0] = gv;
  if (part && lane0 == 0) {
    Partial pr;
    pr.hr = vacc[0];
    pr.hi = vacc[2];
    pr.lr = vacc[1];
    pr.li = vacc[3];
    pr.abs_sum = vacc[4];
    pr.pad0 = pr.pad1 = pr.pad2 = 0.0;
    *part = pr;
  }
}

// The unstaged instances add the rank-one terms to P(W) in registers and
// update the gradient slot once per term, at their own tile only (measured
// on MI355X, fused pass M terms/s, late vs separate: N = 40 4.54 vs 4.40,
// N = 48 1.80 vs 1.72, N = 64 0.270 vs 0.265); tile 7 keeps the separate
// update (N = 52 1.00 vs 1.04).
#ifndef LH_BWD_RANK_LATE
#define LH_BWD_RANK_LATE(bb, bmax, stg) (!(stg) && (bb) == (bmax) && (bmax) != 7)
#endif
#ifndef LH_BWD_WAVES
#define LH_BWD_WAVES(bmax, stg) \
  ((bmax) <= 1 ? 4 : ((bmax) <= 3 ? 2 : ((bmax) <= 5 && !(stg) ? 2 : 1)))
#endif
#ifndef LH_BWD_ATTR
#define LH_BWD_ATTR                   \
  __launch_bounds__(64) __attribute__( \
      (amdgpu_waves_per_eu(LH_BWD_WAVES(BMAX, kStg), LH_BWD_WAVES(BMAX, kStg))))
#endif
// kStg: operand and Krylov vectors in LDS (tiles <= kStageMaxB, see
// bwd_staged), otherwise in the per-wavefront global scratch
template <int BMAX, bool kStg>
__global__ LH_BWD_ATTR void backward_kernel(const Prob* __restrict__ probs,
                                                      const Item* __restrict__ items, int n_items,
                                                      int* counter, const cd* __restrict__ ws,
                                                      cd* __restrict__ gslots,
                                                      cd* __restrict__ scratch, int nmax,
                                                      const cd* __restrict__ saved,
                                                      Partial* __restrict__ parts, int acc_dd) {
  extern __shared__ __align__(16) char lds_raw[];
  LdsView L = carve(lds_raw, nmax);
  const int lane = threadIdx.x & 63;
  cd* scr = scratch + (size_t)blockIdx.x * bwd_wave_scratch_elems(BMAX);
  for (;;) {
    const int it = __builtin_amdgcn_readfirstlane(atomicAdd(counter, lane == 0 ? 1 : 0));
    if (it >= n_items) break;
    const Item I = items[it];
    const Prob& P = probs[I.prob];
    const int LD = 8 * P.B;
    const cd* Cp = ws + P.c_off;
    const cd* vp = Cp + LD * LD;
    cd* G = gslots + P.g_off + (int64_t)(I.pad - P.first_item) * (LD * LD + 64);
    switch (P.B) {
#define LH_BCASE(BB)                                                                   \
  case BB:                                                                             \
    if (BB <= BMAX)                                                                    \
      run_item_bwd<(BB <= BMAX ? BB : 1), kStg, LH_BWD_RANK_LATE(BB, BMAX, kStg)>(       \
          P, I.t0, I.t1, Cp, vp, G, scr, L, saved, parts ? parts + I.pad : nullptr, acc_dd); \
    break;
      LH_BCASE(1)
      LH_BCASE(2)
      LH_BCASE(3)
      LH_BCASE(4)
      LH_BCASE(5)
      LH_BCASE(6)
      LH_BCASE(7)
      LH_BCASE(8)
#undef LH_BCASE
      default:
        break;
    }
  }
}

#ifdef LH_COMMON_KERNELS
// Sum the item gradients of each problem (in item order) into the problem's
// reduced gradient at dst + r_off (0 when no item of the problem ran).
__global__ void greduce_kernel(const Prob* __restrict__ probs, const cd* __restrict__ gslots,
                               cd* __restrict__ dst) {
  const Prob& P = probs[blockIdx.x];
  const int LD = 8 * P.B;
  const int E = LD * LD + 64;
  const cd* base = gslots + P.g_off;
  cd* out = dst + P.r_off;
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    cd acc = czero();
    for (int k = 0; k < P.n_items; ++k) acc = cadd(acc, base[(int64_t)k * E + e]);
    out[e] = acc;
  }
}

// d lhaf / d C[c][i] from the reduced accumulator (see run_item_bwd):
// T[c][i] = scale * G[partner(i)][c].
__device__ __forceinline__ cd grad_c(const Prob& P, const cd* __restrict__ G, int LD, int c, int i) {
  const int pi = i < P.H ? i + P.H : i - P.H;
  return cscale(P.scale, G[pi * LD + c]);
}

// Dense batch: problem b owns dA_b (base_dim x base_dim, lda) and dgamma_b
// (base_dim); one block per problem writes every entry of both from the
// problem's reduced gradient (grads + r_off).  Entry
// (x, y) gathers the reduced-gradient entries of the vertices whose index
// list entry maps to matrix rows x and y (idx, or the identity without one);
// rows that no vertex maps to get 0.
__global__ void scatter_dense_kernel(const Prob* __restrict__ probs, const cd* __restrict__ grads,
                                     const int64_t* __restrict__ ioff,
                                     const int32_t* __restrict__ idx,
                                     const lh_c128* __restrict__ grad_out, lh_c128* dA, int64_t lda,
                                     int64_t strideA, lh_c128* dg, int64_t strideG, int base_dim) {
  __shared__ short first[kMaxRows];
  __shared__ short nxt[64];
  const int b = blockIdx.x;
  const Prob& P = probs[b];
  const int N = base_dim;
  const int32_t* ib = idx ? idx + ioff[b] : nullptr;
  for (int x = threadIdx.x; x < N; x += blockDim.x) first[x] = -1;
  if (threadIdx.x < 64) nxt[threadIdx.x] = -1;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = P.m - 1; c >= 0; --c) {
      const int x = P.pos[c];
      const int row = x < 0 ? -1 : (ib ? ib[x] : x);
      if (row >= 0 && row < N) {
        nxt[c] = first[row];
        first[row] = c;
      }
    }
  }
  __syncthreads();
  const int LD = 8 * P.B;
  const cd* G = grads + P.r_off;
  const lh_c128 go = grad_out[b];
  const cd gout = mk(go.re, go.im);
  lh_c128* dAb = dA + (int64_t)b * strideA;
  lh_c128* dgb = dg + (int64_t)b * strideG;
  for (int e = threadIdx.x; e < N * N + N; e += blockDim.x) {
    cd val = czero();
    if (e < N * N) {
      const int x = e / N, y = e % N;
      if (P.n > 0)
        for (int c = first[x]; c >= 0; c = nxt[c])
          for (int i = first[y]; i >= 0; i = nxt[i]) {
            if (c != i) {
              val = cadd(val, cscale(0.5, cadd(grad_c(P, G, LD, c, i), grad_c(P, G, LD, i, c))));
            } else {
              const int pr = c < P.H ? c : c - P.H;
              if ((P.diag_keep_mask >> pr) & 1) val = cadd(val, grad_c(P, G, LD, c, c));
            }
          }
      const cd o = cmulj(gout, val);  // grad_out * conj(d lhaf / d A)
      lh_c128 r;
      r.re = o.r;
      r.im = o.i;
      dAb[(int64_t)x * lda + y] = r;
    } else {
      const int x = e - N * N;
      if (P.n > 0)
        for (int c = first[x]; c >= 0; c = nxt[c]) val = cadd(val, cscale(P.scale, G[LD * LD + c]));
      const cd o = cmulj(gout, val);
      lh_c128 r;
      r.re = o.r;
      r.im = o.i;
      dgb[x] = r;
    }
  }
}

// Shared base matrix: entry (x, y) of dA (base_dim x base_dim) sums the
// contributions of every problem, in problem order.
__global__ void scatter_shared_kernel(const Prob* __restrict__ probs, int nprob,
                                      const int64_t* __restrict__ ioff,
                                      const int32_t* __restrict__ idx,
                                      const cd* __restrict__ grads,
                                      const lh_c128* __restrict__ grad_out, lh_c128* dA,
                                      int64_t lda, lh_c128* dg, int base_dim) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t E = (int64_t)base_dim * base_dim + base_dim;
  if (e >= E) return;
  cd tot = czero();
  for (int b = 0; b < nprob; ++b) {
    const Prob& P = probs[b];
    if (P.n == 0) continue;
    const int LD = 8 * P.B;
    const cd* G = grads + P.r_off;
    const int32_t* ib = idx ? idx + ioff[b] : nullptr;
    const lh_c128 go = grad_out[b];
    cd val = czero();
    if (e < (int64_t)base_dim * base_dim) {
      const int x = (int)(e / base_dim), y = (int)(e % base_dim);
      for (int c = 0; c < P.m; ++c) {
        const int pc = P.pos[c];
        if (pc < 0 || (ib ? ib[pc] : pc) != x) continue;
        for (int i = 0; i < P.m; ++i) {
          const int pi = P.pos[i];
          if (pi < 0 || (ib ? ib[pi] : pi) != y) continue;
          if (c != i) {
            val = cadd(val, cscale(0.5, cadd(grad_c(P, G, LD, c, i), grad_c(P, G, LD, i, c))));
          } else {
            const int pr = c < P.H ? c : c - P.H;
            if ((P.diag_keep_mask >> pr) & 1) val = cadd(val, grad_c(P, G, LD, c, c));
          }
        }
      }
    } else {
      const int x = (int)(e - (int64_t)base_dim * base_dim);
      for (int c = 0; c < P.m; ++c) {
        const int pc = P.pos[c];
        if (pc < 0 || (ib ? ib[pc] : pc) != x) continue;
        val = cadd(val, cscale(P.scale, G[LD * LD + c]));
      }
    }
    tot = cadd(tot, cmulj(mk(go.re, go.im), val));
  }
  lh_c128 r;
  r.re = tot.r;
  r.im = tot.i;
  if (e < (int64_t)base_dim * base_dim)
    dA[(e / base_dim) * lda + (e % base_dim)] = r;
  else
    dg[e - (int64_t)base_dim * base_dim] = r;
}

#endif  // LH_COMMON_KERNELS

}  // namespace lh
