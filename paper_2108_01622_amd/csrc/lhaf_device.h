// Device-side building blocks: complex FP64 arithmetic, wavefront reductions
// on the 8 x 8 lane grid, double-double accumulation.
#pragma once
#include <hip/hip_runtime.h>

namespace lh {

// Binomial coefficients C(a, b), 0 <= b <= a <= 32, exact in double (the
// largest, C(32, 16), is below 2^30).  Built at compile time, so every
// translation unit that includes this header has its own initialised copy.
struct BinomTable {
  double v[33][33];
};
constexpr BinomTable make_binom_table() {
  BinomTable t{};
  for (int a = 0; a <= 32; ++a) {
    unsigned long long c = 1;  // C(a, b), built up along the row
    for (int b = 0; b <= 32; ++b) {
      t.v[a][b] = b <= a ? (double)c : 0.0;
      if (b < a) c = c * (unsigned long long)(a - b) / (unsigned long long)(b + 1);
    }
  }
  return t;
}
static __constant__ BinomTable c_binom = make_binom_table();

// Opaque copies of the lane index.  Enabled, the persistent loops re-derive
// every per-lane address and mask once per term (LH_OPAQUE_TERM) or per
// Hessenberg step (LH_OPAQUE_STEP) instead of letting the compiler hoist them
// into registers held for the whole kernel: fewer registers, more
// instructions.  Off by default (measured faster where the hoisted values fit).
#ifndef LH_OPAQUE_TERM
#define LH_OPAQUE_TERM 0
#endif
#ifndef LH_OPAQUE_STEP
#define LH_OPAQUE_STEP 0
#endif
#define LH_OPAQUE(flag, v)              \
  do {                                  \
    if (flag) asm volatile("" : "+v"(v)); \
  } while (0)

// Per-term relative rounding error of the Hessenberg / characteristic-
// polynomial evaluation assumed by the error estimates, in units of u per
// matrix dimension m + 1.  Typical terms stay within a few u; the largest
// per-term error seen is about 6 (m + 1) u (mixed-state pairing (i, M + i),
// m = 20, where the signed sum cancels by 5e6), so the estimate takes 8.
constexpr double kTermErrPerDim = 8.0;

struct cd {
  double r, i;
};

__device__ __forceinline__ cd mk(double r, double i) {
  cd c;
  c.r = r;
  c.i = i;
  return c;
}
__device__ __forceinline__ cd czero() { return mk(0.0, 0.0); }
__device__ __forceinline__ cd cadd(cd a, cd b) { return mk(a.r + b.r, a.i + b.i); }
__device__ __forceinline__ cd csub(cd a, cd b) { return mk(a.r - b.r, a.i - b.i); }
__device__ __forceinline__ cd cscale(double s, cd a) { return mk(s * a.r, s * a.i); }
__device__ __forceinline__ cd cmul(cd a, cd b) {
  return mk(fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r));
}
// a*b + c
__device__ __forceinline__ cd cfma(cd a, cd b, cd c) {
  return mk(fma(a.r, b.r, fma(-a.i, b.i, c.r)), fma(a.r, b.i, fma(a.i, b.r, c.i)));
}
// c - a*b
__device__ __forceinline__ cd cfnma(cd a, cd b, cd c) {
  return mk(fma(-a.r, b.r, fma(a.i, b.i, c.r)), fma(-a.r, b.i, fma(-a.i, b.r, c.i)));
}
// conj(a)*b + c
__device__ __forceinline__ cd cjfma(cd a, cd b, cd c) {
  return mk(fma(a.r, b.r, fma(a.i, b.i, c.r)), fma(a.r, b.i, fma(-a.i, b.r, c.i)));
}
// c - a*conj(b)
__device__ __forceinline__ cd cfnmaj(cd a, cd b, cd c) {
  return mk(fma(-a.r, b.r, fma(-a.i, b.i, c.r)), fma(-a.i, b.r, fma(a.r, b.i, c.i)));
}
// a*conj(b)
__device__ __forceinline__ cd cmulj(cd a, cd b) {
  return mk(fma(a.r, b.r, a.i * b.i), fma(a.i, b.r, -a.r * b.i));
}
__device__ __forceinline__ double cabs2(cd a) { return fma(a.r, a.r, a.i * a.i); }

// ---------------------------------------------------------------------------
// Lane grid: lane = 8*p + q.  "Row group" = the 8 lanes sharing p (consecutive
// lanes), "column group" = the 8 lanes sharing q (stride 8).
// Value of a permuted lane for the lane permutations used below (quad
// permutes, row_ror, row_half_mirror), each of which reads a valid lane for
// every lane: with bound_ctrl and full masks the old value of the destination
// is never used, so the move needs no copy of its source.
#ifndef LH_DPP_BOUND
#define LH_DPP_BOUND 1
#endif
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  if constexpr (LH_DPP_BOUND) {
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  } else {
    lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
  }
  return __hiloint2double(hi, lo);
}

// x + (value of the lane 16 apart): permlane16_swap exchanges the odd 16-lane
// rows of its first operand with the even rows of its second, so with x in
// both the two outputs together hold every lane's value and its partner's.
__device__ __forceinline__ double sum_xor16(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  auto L = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto H = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double(H[0], L[0]) + __hiloint2double(H[1], L[1]);
}
__device__ __forceinline__ double sum_xor32(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  auto L = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  auto H = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(H[0], L[0]) + __hiloint2double(H[1], L[1]);
}
// Two different values through one swap: rows 0 and 2 receive a + (a of the
// lane 16 apart), rows 1 and 3 the same sum of b (no register copies).
__device__ __forceinline__ double sum_xor16_pair(double a, double b) {
  int alo = __double2loint(a), ahi = __double2hiint(a);
  int blo = __double2loint(b), bhi = __double2hiint(b);
  auto L = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
  auto H = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
  return __hiloint2double(H[0], L[0]) + __hiloint2double(H[1], L[1]);
}
// Inverse of the pairing: from x holding a in rows 0, 2 and b in rows 1, 3,
// a and b on every lane.
__device__ __forceinline__ void unpair_rows16(double x, double& a, double& b) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  auto L = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto H = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  a = __hiloint2double(H[0], L[0]);
  b = __hiloint2double(H[1], L[1]);
}

// Sum over the row group (xor 1, xor 2 by quad permutes, then lane i with
// lane 7-i inside each group of 8).  Every lane of the group ends with the
// same bits (IEEE addition is commutative).
__device__ __forceinline__ double sum_row8(double x) {
  x += dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_d<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_d<0x141>(x);  // row_half_mirror
  return x;
}
// Sum over the column group (xor 8 by a rotate of 8 inside 16-lane rows,
// then the 16- and 32-lane swaps).
__device__ __forceinline__ double sum_col8(double x) {
  x += dpp_d<0x128>(x);  // row_ror:8
  x = sum_xor16(x);
  x = sum_xor32(x);
  return x;
}
// sum over each half-wave (lanes 0..31 and 32..63 separately)
__device__ __forceinline__ double sum_half32(double x) {
  x = sum_row8(x);
  x += dpp_d<0x128>(x);  // row_ror:8
  return sum_xor16(x);
}
__device__ __forceinline__ cd sum_half32(cd a) { return mk(sum_half32(a.r), sum_half32(a.i)); }
__device__ __forceinline__ cd sum_row8(cd a) { return mk(sum_row8(a.r), sum_row8(a.i)); }
// Complex column-group sum: after the xor-8 step the real and imaginary parts
// share one register through the paired xor-16 swap, take the xor-32 step
// together and are separated again (every lane of a column group ends with
// the same bits).
#ifndef LH_COL_PAIR
#define LH_COL_PAIR 1
#endif
__device__ __forceinline__ cd sum_col8(cd a) {
  if constexpr (!LH_COL_PAIR) return mk(sum_col8(a.r), sum_col8(a.i));
  double r = a.r + dpp_d<0x128>(a.r);  // row_ror:8
  double i = a.i + dpp_d<0x128>(a.i);
  double x = sum_xor32(sum_xor16_pair(r, i));
  unpair_rows16(x, r, i);
  return mk(r, i);
}
__device__ __forceinline__ cd sum_xor32(cd a) { return mk(sum_xor32(a.r), sum_xor32(a.i)); }

// Value of lane 8p + r for every lane of row group p (r compile-time): DPP
// row_newbcast broadcasts one lane of each 16-lane row; the bank masks write
// lane r into the lower half-row (group 2j) and lane 8 + r into the upper
// half-row (group 2j + 1).
// (The lanes the first move leaves unwritten are written by the second, so
// the first needs no old value and no copy of x.)
template <int R>
__device__ __forceinline__ double bcast_row8_c(double x) {
  double y = __builtin_amdgcn_mov_dpp(x, 0x150 + R, 0xF, 0x3, false);
  return __builtin_amdgcn_update_dpp(y, x, 0x158 + R, 0xF, 0xC, false);
}
// The two halves of bcast_row8_c separately, so that a caller can issue all
// first halves before the second ones (the second reads the first's result).
template <int R>
__device__ __forceinline__ double bcast_row8_lo(double x) {
  return __builtin_amdgcn_mov_dpp(x, 0x150 + R, 0xF, 0x3, false);
}
template <int R>
__device__ __forceinline__ double bcast_row8_hi(double y, double x) {
  return __builtin_amdgcn_update_dpp(y, x, 0x158 + R, 0xF, 0xC, false);
}
// same with r folded to a constant by full unrolling of the caller's loop
__device__ __forceinline__ double bcast_row8(double x, const int r) {
  switch (r) {
    case 0: return bcast_row8_c<0>(x);
    case 1: return bcast_row8_c<1>(x);
    case 2: return bcast_row8_c<2>(x);
    case 3: return bcast_row8_c<3>(x);
    case 4: return bcast_row8_c<4>(x);
    case 5: return bcast_row8_c<5>(x);
    case 6: return bcast_row8_c<6>(x);
    default: return bcast_row8_c<7>(x);
  }
}

__device__ __forceinline__ double shfl_d(double x, int src) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_ds_bpermute(src << 2, lo);
  hi = __builtin_amdgcn_ds_bpermute(src << 2, hi);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double bcast0_d(double x) {
  int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
  int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cd bcast0(cd a) { return mk(bcast0_d(a.r), bcast0_d(a.i)); }

// product over all 64 lanes (exact for the integer factors used here); lane
// is the caller's lane index (0..63)
__device__ __forceinline__ double prod_wave(double x, const int lane) {
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) x *= shfl_d(x, lane ^ s);
  return x;
}

// Synchronisation of the lanes of one wavefront for kernels that run one
// wavefront per workgroup and exchange data between lanes only through LDS:
// a wavefront's LDS operations execute in issue order, so it suffices that
// the compiler keeps memory accesses on their side of this point.  Unlike
// __syncthreads() it does not wait for outstanding global loads and stores.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Double-double complex values for the compensated-recurrence mode: a complex
// value as unevaluated sums hi + lo per component.  cdd_fma adds a * b with
// every real product split exactly (FMA TwoProd) and every addition to the
// high parts exact (Knuth TwoSum), the rounding errors gathered in the low
// parts, so a dot product comes out as if formed in twice the working
// precision (the compensated dot product of Ogita, Rump and Oishi, 2005);
// cdd_fma_hl / cdd_fma_hl2 take double-double operands (their low-part
// cross products in plain FP64: relative error O(u^2)), and cdd_split
// renormalises a result into the (hi, lo) pair that is stored.
struct cdd {
  double rh, rl, ih, il;
};
__device__ __forceinline__ cdd cdd_zero() { return {0.0, 0.0, 0.0, 0.0}; }
__device__ __forceinline__ cdd cdd_of(const cd a) { return {a.r, 0.0, a.i, 0.0}; }
__device__ __forceinline__ cdd cdd_neg(const cdd a) { return {-a.rh, -a.rl, -a.ih, -a.il}; }
// s + e = a + b exactly (Knuth's TwoSum; the same bits for either order).
// The error-free transformations here and below turn off floating-point
// contraction: HIP contracts a product into a later addition by default,
// which would fuse x * y into the TwoSum of a TwoProd and count the
// product's rounding error twice.
__device__ __forceinline__ void two_sum(const double a, const double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
// h + l += x * y
__device__ __forceinline__ void dd_acc_prod(double& h, double& l, const double x, const double y) {
#pragma clang fp contract(off)
  const double p = x * y;
  const double pe = fma(x, y, -p);
  double s, e;
  two_sum(h, p, s, e);
  h = s;
  l += e + pe;
}
// acc += a * b
__device__ __forceinline__ void cdd_fma(cdd& acc, const cd a, const cd b) {
  dd_acc_prod(acc.rh, acc.rl, a.r, b.r);
  dd_acc_prod(acc.rh, acc.rl, -a.i, b.i);
  dd_acc_prod(acc.ih, acc.il, a.r, b.i);
  dd_acc_prod(acc.ih, acc.il, a.i, b.r);
}
// a + b; commutative to the bit, so two lanes that combine each other's
// values end with the same bits
__device__ __forceinline__ cdd cdd_plus(const cdd& a, const cdd& b) {
  cdd r;
  double e;
  two_sum(a.rh, b.rh, r.rh, e);
  r.rl = e + (a.rl + b.rl);
  two_sum(a.ih, b.ih, r.ih, e);
  r.il = e + (a.il + b.il);
  return r;
}
__device__ __forceinline__ cd cdd_round(const cdd& a) { return mk(a.rh + a.rl, a.ih + a.il); }
// acc += a * (bh + bl)
__device__ __forceinline__ void cdd_fma_hl(cdd& acc, const cd a, const cd bh, const cd bl) {
  cdd_fma(acc, a, bh);
  acc.rl += fma(a.r, bl.r, -a.i * bl.i);
  acc.il += fma(a.r, bl.i, a.i * bl.r);
}
// acc += (ah + al) * (bh + bl)
__device__ __forceinline__ void cdd_fma_hl2(cdd& acc, const cd ah, const cd al, const cd bh,
                                            const cd bl) {
  cdd_fma(acc, ah, bh);
  acc.rl += fma(ah.r, bl.r, -ah.i * bl.i) + fma(al.r, bh.r, -al.i * bh.i);
  acc.il += fma(ah.r, bl.i, ah.i * bl.r) + fma(al.r, bh.i, al.i * bh.r);
}
// (h + l) / k for a small positive integer k: the quotient of the high part,
// corrected by its exact remainder and the low part
__device__ __forceinline__ void dd_div(double& h, double& l, const double k) {
  const double q = h / k;
  const double r = fma(-q, k, h);
  h = q;
  l = (r + l) / k;
}
__device__ __forceinline__ cdd cdd_div(cdd a, const double k) {
  dd_div(a.rh, a.rl, k);
  dd_div(a.ih, a.il, k);
  return a;
}
// renormalised (hi, lo): hi = fl(hi + lo), lo the exact remainder (TwoSum:
// after a cancellation the low part can exceed the high one)
__device__ __forceinline__ void cdd_split(const cdd& a, cd& hi, cd& lo) {
  two_sum(a.rh, a.rl, hi.r, lo.r);
  two_sum(a.ih, a.il, hi.i, lo.i);
}
// a + (a of another lane) for the lane patterns of the plain sums above; the
// permlane swaps hand every lane of a pair its two values in the same order
template <int CTRL>
__device__ __forceinline__ cdd cdd_plus_dpp(const cdd& a) {
  return cdd_plus(a, {dpp_d<CTRL>(a.rh), dpp_d<CTRL>(a.rl), dpp_d<CTRL>(a.ih), dpp_d<CTRL>(a.il)});
}
__device__ __forceinline__ void swap16_d(const double x, double& v0, double& v1) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  auto L = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto H = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  v0 = __hiloint2double(H[0], L[0]);
  v1 = __hiloint2double(H[1], L[1]);
}
__device__ __forceinline__ void swap32_d(const double x, double& v0, double& v1) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  auto L = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  auto H = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  v0 = __hiloint2double(H[0], L[0]);
  v1 = __hiloint2double(H[1], L[1]);
}
__device__ __forceinline__ cdd cdd_plus_xor16(const cdd& a) {
  cdd u, v;
  swap16_d(a.rh, u.rh, v.rh);
  swap16_d(a.rl, u.rl, v.rl);
  swap16_d(a.ih, u.ih, v.ih);
  swap16_d(a.il, u.il, v.il);
  return cdd_plus(u, v);
}
__device__ __forceinline__ cdd cdd_plus_xor32(const cdd& a) {
  cdd u, v;
  swap32_d(a.rh, u.rh, v.rh);
  swap32_d(a.rl, u.rl, v.rl);
  swap32_d(a.ih, u.ih, v.ih);
  swap32_d(a.il, u.il, v.il);
  return cdd_plus(u, v);
}
// compensated sums over the row group, each half-wave and the whole wave
__device__ __forceinline__ cdd cdd_sum_row8(cdd a) {
  a = cdd_plus_dpp<0xB1>(a);   // quad_perm [1,0,3,2]
  a = cdd_plus_dpp<0x4E>(a);   // quad_perm [2,3,0,1]
  return cdd_plus_dpp<0x141>(a);  // row_half_mirror
}
__device__ __forceinline__ cdd cdd_sum_half32(cdd a) {
  a = cdd_sum_row8(a);
  a = cdd_plus_dpp<0x128>(a);  // row_ror:8
  return cdd_plus_xor16(a);
}
__device__ __forceinline__ cdd cdd_sum_wave(const cdd& a) { return cdd_plus_xor32(cdd_sum_half32(a)); }

// ---------------------------------------------------------------------------
// double-double accumulation (Knuth TwoSum, FMA TwoProd; no contraction, see
// two_sum)
struct dd {
  double hi, lo;
};
__device__ __forceinline__ void dd_add_prod(dd& acc, double c, double x) {
#pragma clang fp contract(off)
  double p = c * x;
  double pe = fma(c, x, -p);
  double s = acc.hi + p;
  double bb = s - acc.hi;
  double e = (acc.hi - (s - bb)) + (p - bb);
  double lo = acc.lo + (e + pe);
  double h2 = s + lo;
  acc.lo = lo - (h2 - s);
  acc.hi = h2;
}
__device__ __forceinline__ void dd_add(dd& acc, double hi, double lo) {
#pragma clang fp contract(off)
  double s = acc.hi + hi;
  double bb = s - acc.hi;
  double e = (acc.hi - (s - bb)) + (hi - bb);
  double l = acc.lo + (e + lo);
  double h2 = s + l;
  acc.lo = l - (h2 - s);
  acc.hi = h2;
}

}  // namespace lh
