// Internal structures shared by the host planner, the API layer and the HIP
// kernels of the loop-hafnian library.  Not part of the public ABI.
#pragma once
#include <stdint.h>

#include <vector>

namespace lh {

constexpr int kMaxN = 64;      // vertices per problem (after odd padding)
constexpr int kMaxPairs = 32;  // distinct pairs H
constexpr int kMaxB = 8;       // register tile: m <= 8*B, lane grid 8 x 8
constexpr int kMaxRows = 4096; // rows of one repeated problem's matrix (modes)

// One loop-hafnian problem as the kernels see it.
struct Prob {
  int64_t c_off;  // offset (lh_c128 units) of the packed reduced matrix in the workspace;
                  // the loop vector v (64 entries) follows the (8B)^2 matrix
  int64_t T;      // terms in the full enumeration
  int64_t t0, t1; // term range evaluated by this call
  int32_t m;      // reduced size 2H
  int32_t H;      // distinct pairs
  int32_t n;      // lambda degree = sum eta (= N/2 after padding)
  int32_t B;      // register tile, ceil(m/8)
  int32_t mode;   // 0 ET, 1 FDS
  int32_t hp;     // FDS halving pair (-1 for ET)
  int32_t first_item, n_items;
  int32_t Nvert;  // rows of the problem's matrix (entries of its index list)
  int64_t g_off;  // backward: offset (lh_c128 units) of the item gradient slots
  int64_t r_off;  // backward: offset of the problem's reduced gradient (LD^2 + 64 entries)
                  // in the per-problem gradient layout
  int64_t s_off;  // offset of the problem's block in the per-term coefficient store
  int32_t diag_keep_mask;  // bit p set: pair p repeats (eta >= 2), keep C's diagonal
  double scale;   // 2^-n for scaled FDS, 1 otherwise
  int8_t eta[kMaxPairs];
  int8_t radix[kMaxPairs];
  int16_t pos[kMaxN];  // entry index into the problem's index list, -1 = padding vertex
};

struct Item {
  int32_t prob;
  int32_t pad;
  int64_t t0, t1;
};

// Terms of the longest item of a problem: the planner cuts [t0, t1) into
// n_items ranges of equal length up to one term.
__host__ __device__ inline int64_t lh_longest_item(const Prob& P) {
  const int64_t k = P.n_items > 0 ? P.n_items : 1;
  return (P.t1 - P.t0 + k - 1) / k;
}

// Offset (ints) of the work counter of a second launch over the same items,
// on its own cache line in the 256-byte counter block of the workspace.
constexpr int kSecondCounter = 32;

// Partial sum of one item: double-double complex + sum of |c_t f_t|.
struct Partial {
  double hr, hi, lr, li, abs_sum, pad0, pad1, pad2;
};

// LDS bytes of one forward wavefront for lambda degree <= nmax
inline size_t lds_bytes_for(int nmax) {
  const size_t NP = nmax + 1, NR = nmax + 2;
  return 16 * (65 + 65 + 64 + 128 + 33 + 66) + 8 * 8 + 16 * NP * NR;
}
// the compensated-recurrence forward: also the low parts of the ring and of
// the two series
inline size_t lds_bytes_comp(int nmax) {
  const size_t NP = nmax + 1, NR = nmax + 2;
  return lds_bytes_for(nmax) + 16 * (NP * NR + 66);
}

// Host planner --------------------------------------------------------------
struct PairPlan {
  int H = 0;
  int n = 0;
  int N = 0;     // vertices before padding (photons for a repeated problem)
  int rows = 0;  // rows of the problem's matrix
  bool padded = false;
  std::vector<int> pos;  // 2H
  std::vector<int> eta;  // H
};

// plain problem of N vertices: position i pairs with n + i (padding if odd)
PairPlan plan_plain(int N);
// repeated problem: greedy matching on multiplicities r (App. B.3)
PairPlan plan_repeated(const int32_t* r, int M);
// mixed-state form (App. B.2): 2M rows, row i paired with row M + i, n_i times
PairPlan plan_mixed(const int32_t* n, int M);
// fill a Prob (without offsets / items) for `mode` over [t0, t1)
bool fill_prob(const PairPlan& pp, int mode, int64_t t0, int64_t t1, bool scaled, Prob* out);
int64_t term_count(const PairPlan& pp, int mode, int* hp_out);

}  // namespace lh
