// CPU oracle for complex loop hafnians.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file: only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark use it.  It shares no code with the HIP library.
//
// Everything here is deliberately plain and serial per term (OpenMP only
// splits term ranges across threads; partials are added in thread order).
// Arithmetic is templated on the real type: double, or __float128 (soft
// float, exact conversion from the double inputs).
//
// Implemented (paper = arXiv:2108.01622, "The boundary for quantum advantage
// in Gaussian boson sampling"):
//   * lhaf by the definition (App. B, sum over single-pair matchings):
//     recursive enumeration, and the same recursion memoised over the set of
//     still-unmatched vertices.
//   * the eigenvalue-trace inclusion/exclusion sum (App. B.1, Eqs. ET_loop and
//     ET_poly) with repeated pairs (App. B.2, lhafmix with weighted matching
//     X_z), power traces by explicit repeated matrix products.
//   * the finite-difference sieve (App. B.4, Eq. fdsieve) with repeated pairs
//     (delta of a pair with eta copies runs -eta..eta in steps of 2).
//   * Ryser's formula for the permanent (bipartite-hafnian pin).
//   * the loop repeated-moment sum obtained from the generating function
//     exp(x^T A x / 2 + gamma^T x) (pin for the repeated-row form).
//
// Matrices are row-major N x N, complex interleaved (re, im) doubles.
// lhaf(A, gamma) takes loops from gamma; A's own diagonal matters only where
// rows are repeated (it couples two copies of a mode, App. A), so the
// power-trace sums keep C's diagonal = A_ii and take v = gamma separately.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

template <class T> struct cx {
  T re, im;
  cx() : re(0), im(0) {}
  cx(T r, T i = 0) : re(r), im(i) {}
};
template <class T> inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T> inline cx<T>& operator+=(cx<T>& a, cx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <class T> inline cx<T>& operator-=(cx<T>& a, cx<T> b) { a.re -= b.re; a.im -= b.im; return a; }

template <class T> inline T tabs(T x) { return x < 0 ? -x : x; }

// Kahan-Babuska-Neumaier compensated complex sum.
template <class T> struct nsum {
  cx<T> s, c;
  void add(cx<T> x) {
    T t = s.re + x.re;
    if (tabs(s.re) >= tabs(x.re)) c.re += (s.re - t) + x.re; else c.re += (x.re - t) + s.re;
    s.re = t;
    t = s.im + x.im;
    if (tabs(s.im) >= tabs(x.im)) c.im += (s.im - t) + x.im; else c.im += (x.im - t) + s.im;
    s.im = t;
  }
  cx<T> get() const { return s + c; }
};

template <class T> std::vector<cx<T>> load(const double* p, int64_t count) {
  std::vector<cx<T>> v(count);
  for (int64_t i = 0; i < count; ++i) v[i] = cx<T>((T)p[2 * i], (T)p[2 * i + 1]);
  return v;
}

// write x as (hi, lo) double pairs: out[0..1] = hi(re, im), out[2..3] = lo(re, im)
template <class T> void store(cx<T> x, double* out, bool with_lo) {
  double hr = (double)x.re, hi = (double)x.im;
  out[0] = hr;
  out[1] = hi;
  if (with_lo) {
    out[2] = (double)(x.re - (T)hr);
    out[3] = (double)(x.im - (T)hi);
  }
}

// ---------------------------------------------------------------------------
// Definition: lhaf(A) = sum over single-pair matchings M of [N] of the product
// of A_ij over the pairs {i,j} in M and of gamma_i over the singles {i} in M
// (App. B, first equation; singles weighted by the diagonal, which App. A sets
// to gamma).  Expanding on the lowest unmatched vertex i: it is either a single
// (weight gamma_i) or paired with some other unmatched j (weight A_ij).
template <class T> struct Enum {
  int N;
  const std::vector<cx<T>>& A;
  const std::vector<cx<T>>& g;
  cx<T> rec(uint64_t rest) const {
    if (rest == 0) return cx<T>(1);
    int i = __builtin_ctzll(rest);
    uint64_t r = rest & ~(1ull << i);
    cx<T> s = g[i] * rec(r);
    for (uint64_t q = r; q; q &= q - 1) {
      int j = __builtin_ctzll(q);
      s += A[(size_t)i * N + j] * rec(r & ~(1ull << j));
    }
    return s;
  }
};

template <class T> struct Memo {
  int N;
  const std::vector<cx<T>>& A;
  const std::vector<cx<T>>& g;
  std::vector<cx<T>> val;
  std::vector<uint8_t> done;
  cx<T> rec(uint64_t rest) {
    if (rest == 0) return cx<T>(1);
    if (done[rest]) return val[rest];
    int i = __builtin_ctzll(rest);
    uint64_t r = rest & ~(1ull << i);
    cx<T> s = g[i] * rec(r);
    for (uint64_t q = r; q; q &= q - 1) {
      int j = __builtin_ctzll(q);
      s += A[(size_t)i * N + j] * rec(r & ~(1ull << j));
    }
    done[rest] = 1;
    val[rest] = s;
    return s;
  }
};

// ---------------------------------------------------------------------------
// f(C, v, x) for the power-trace sums (App. B.1, Eq. ET_poly; App. B.2 with the
// weighted matching X_x):  the lambda^n coefficient of
//     sum_{j=1..n} (1/j!) ( sum_{k=1..n} g_k lambda^k )^j,
//     g_k = Tr((C X)^k) / (2k) + v X (C X)^{k-1} v^T / 2,
// where X pairs position p with position h+p (h = size/2) with weight x_p.
// v is the loop vector (diag of A_n in Eq. ET_poly; gamma in lhafmix).  Tr((C X)^k) is taken from explicit products of C X, and the
// exponential series from explicit truncated polynomial powers.
template <class T>
cx<T> f_term(const std::vector<cx<T>>& C, const std::vector<cx<T>>& v, int m, const std::vector<T>& x,
             int n) {
  const int h = m / 2;
  // W = C X: column j of W is x_{pair(j)} times column partner(j) of C.
  std::vector<cx<T>> W((size_t)m * m), P((size_t)m * m), Q((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      int pj = j < h ? j + h : j - h;
      T w = x[j < h ? j : j - h];
      W[(size_t)i * m + j] = w * C[(size_t)i * m + pj];
    }
  std::vector<cx<T>> vx(m), y(m), y2(m);
  for (int j = 0; j < m; ++j) {  // row vector v X
    int pj = j < h ? j + h : j - h;
    vx[j] = x[j < h ? j : j - h] * v[pj];
  }
  std::vector<cx<T>> g(n + 1);
  P = W;
  y = v;  // (C X)^{k-1} v^T
  for (int k = 1; k <= n; ++k) {
    cx<T> tr;
    for (int i = 0; i < m; ++i) tr += P[(size_t)i * m + i];
    cx<T> mu;
    for (int i = 0; i < m; ++i) mu += vx[i] * y[i];
    g[k] = (T(1) / T(2 * k)) * tr + (T(1) / T(2)) * mu;
    if (k == n) break;
    // P <- P W ; y <- W y
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        cx<T> s;
        for (int l = 0; l < m; ++l) s += P[(size_t)i * m + l] * W[(size_t)l * m + j];
        Q[(size_t)i * m + j] = s;
      }
    P.swap(Q);
    for (int i = 0; i < m; ++i) {
      cx<T> s;
      for (int l = 0; l < m; ++l) s += W[(size_t)i * m + l] * y[l];
      y2[i] = s;
    }
    y.swap(y2);
  }
  // sum_{j=1..n} G^j / j!, truncated at degree n; return degree-n coefficient.
  std::vector<cx<T>> Gp(n + 1), tmp(n + 1);
  Gp = g;  // G^1 (g[0] = 0)
  cx<T> out = Gp[n];
  T fact = 1;
  for (int j = 2; j <= n; ++j) {
    for (int d = 0; d <= n; ++d) {
      cx<T> s;
      for (int a = 1; a < d; ++a) s += Gp[a] * g[d - a];
      tmp[d] = s;
    }
    Gp.swap(tmp);
    fact *= (T)j;
    out += (T(1) / fact) * Gp[n];
  }
  return out;
}

// binomial coefficient as an exact integer
inline double binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  double r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return std::round(r);
}

struct PairSpec {
  int H;
  std::vector<int> u, w, eta;
  int n;  // sum eta
};

// Reduced matrix for pairs: position p <-> row u_p, position h+p <-> row w_p,
// C[a][b] = A[idx_a][idx_b] including the diagonal.  In the repeated-pairs sum
// (App. B.2, lhafmix) the matrix keeps its own diagonal and the loop vector is
// passed separately: C_aa = A_ii is the coupling between two copies of mode i
// (App. A: rows of A_n are copies of rows of A), which a walk uses when it
// crosses between two repeats of the same pair.  v = gamma[idx].
template <class T>
std::vector<cx<T>> reduced(const std::vector<cx<T>>& A, int N, const std::vector<int>& idx) {
  int m = (int)idx.size();
  std::vector<cx<T>> C((size_t)m * m);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) C[(size_t)a * m + b] = A[(size_t)idx[a] * N + idx[b]];
  return C;
}

// Term of the documented enumeration (mixed radix, pair 0 fastest).
//  ET : radix eta_p + 1, z_p = digit, coefficient (-1)^{n - sum z} prod C(eta_p, z_p);
//       pairs with z_p = 0 are deleted (App. B.2); z = 0 gives f = 0.
//  FDS: radix eta_p + 1 except the halving pair hp (floor(eta/2) + 1), digit s_p,
//       weight d_p = eta_p - 2 s_p, coefficient prod (-1)^{s_p} C(eta_p, s_p),
//       times 2 for the halving pair unless 2 s_hp == eta_hp (App. B.4).
//  When `halve` is false the FDS runs over every digit (no symmetry halving).
template <class T>
cx<T> term_value(const std::vector<cx<T>>& A, const std::vector<cx<T>>& g, int N, const PairSpec& ps,
                 bool fds, bool halve, int hp, int64_t t, double* coef_out) {
  const int H = ps.H;
  std::vector<int> s(H);
  int64_t r = t;
  for (int p = 0; p < H; ++p) {
    int radix = ps.eta[p] + 1;
    if (fds && halve && p == hp) radix = ps.eta[p] / 2 + 1;
    s[p] = (int)(r % radix);
    r /= radix;
  }
  double coef = 1;
  std::vector<int> keep;
  std::vector<T> x;
  if (fds) {
    for (int p = 0; p < H; ++p) {
      coef *= ((s[p] & 1) ? -1.0 : 1.0) * binom(ps.eta[p], s[p]);
      keep.push_back(p);
      x.push_back((T)(ps.eta[p] - 2 * s[p]));
    }
    if (halve && H > 0 && 2 * s[hp] != ps.eta[hp]) coef *= 2;
  } else {
    int sz = 0;
    for (int p = 0; p < H; ++p) {
      coef *= binom(ps.eta[p], s[p]);
      sz += s[p];
      if (s[p] > 0) {
        keep.push_back(p);
        x.push_back((T)s[p]);
      }
    }
    if ((ps.n - sz) & 1) coef = -coef;
    if (keep.empty()) {
      *coef_out = coef;
      return cx<T>(0);
    }
  }
  int hk = (int)keep.size();
  std::vector<int> idx(2 * hk);
  for (int q = 0; q < hk; ++q) {
    idx[q] = ps.u[keep[q]];
    idx[hk + q] = ps.w[keep[q]];
  }
  std::vector<cx<T>> C = reduced(A, N, idx);
  std::vector<cx<T>> v(2 * hk);
  for (int a = 0; a < 2 * hk; ++a) v[a] = g[idx[a]];
  *coef_out = coef;
  return f_term(C, v, 2 * hk, x, ps.n);
}

int halving_pair(const PairSpec& ps) {
  for (int p = 0; p < ps.H; ++p)
    if (ps.eta[p] & 1) return p;
  return 0;
}

int64_t term_count(const PairSpec& ps, bool fds, bool halve) {
  int hp = halving_pair(ps);
  int64_t T = 1;
  for (int p = 0; p < ps.H; ++p) T *= (fds && halve && p == hp) ? (ps.eta[p] / 2 + 1) : (ps.eta[p] + 1);
  return T;
}

template <class T>
void power_trace_sum(int N, const double* A_, const double* g_, int H, const int* u, const int* w,
                     const int* eta, int fds, int halve, int64_t t0, int64_t t1, int scaled, double* out,
                     double* abs_sum) {
  auto A = load<T>(A_, (int64_t)N * N);
  auto g = load<T>(g_, N);
  PairSpec ps;
  ps.H = H;
  ps.n = 0;
  for (int p = 0; p < H; ++p) {
    ps.u.push_back(u[p]);
    ps.w.push_back(w[p]);
    ps.eta.push_back(eta[p]);
    ps.n += eta[p];
  }
  if (ps.n == 0) {  // lhaf of the empty matrix is 1 (one empty matching)
    store(cx<T>(1), out, true);
    if (abs_sum) *abs_sum = 1;
    return;
  }
  int hp = halving_pair(ps);
  int64_t T_all = term_count(ps, fds != 0, halve != 0);
  if (t1 < 0 || t1 > T_all) t1 = T_all;
  if (t0 < 0) t0 = 0;
  int nt = omp_get_max_threads();
  std::vector<nsum<T>> part(nt);
  std::vector<T> apart(nt, T(0));
#pragma omp parallel num_threads(nt)
  {
    int tid = omp_get_thread_num();
    int64_t len = t1 > t0 ? t1 - t0 : 0;
    int64_t b = t0 + len * tid / nt, e = t0 + len * (tid + 1) / nt;
    for (int64_t t = b; t < e; ++t) {
      double coef;
      cx<T> f = term_value(A, g, N, ps, fds != 0, halve != 0, hp, t, &coef);
      cx<T> cf = (T)coef * f;
      part[tid].add(cf);
      T a2 = cf.re * cf.re + cf.im * cf.im;
      apart[tid] += (T)std::sqrt((double)a2);
    }
  }
  nsum<T> tot;
  T at = 0;
  for (int i = 0; i < nt; ++i) {
    tot.add(part[i].get());
    at += apart[i];
  }
  cx<T> res = tot.get();
  if (fds && scaled) {
    T sc = 1;
    for (int i = 0; i < ps.n; ++i) sc = sc / 2;
    res = sc * res;
    at = sc * at;
  }
  store(res, out, true);
  if (abs_sum) *abs_sum = (double)at;
}

// Ryser: perm(B) = (-1)^n sum_{S subset [n]} (-1)^{|S|} prod_i sum_{j in S} B_ij
template <class T> cx<T> ryser(int n, const std::vector<cx<T>>& B) {
  nsum<T> tot;
  for (uint64_t S = 1; S < (1ull << n); ++S) {
    cx<T> prod(1);
    for (int i = 0; i < n; ++i) {
      cx<T> rs;
      for (int j = 0; j < n; ++j)
        if (S >> j & 1) rs += B[(size_t)i * n + j];
      prod = prod * rs;
    }
    int pc = __builtin_popcountll(S);
    if ((n - pc) & 1) prod = T(-1) * prod;
    tot.add(prod);
  }
  return tot.get();
}

// Loop repeated-moment sum.  With P(x) = exp(x^T A x / 2 + gamma^T x) the
// coefficient of prod x_i^{r_i} / r_i! is lhaf(A_r) (rows repeated r_i times,
// copies coupled by A_ii, loops gamma_i).  For the degree-N homogeneous part
// P_N, the mixed derivative d^r P_N equals
//   sum_{0<=nu<=r} (-1)^{|nu|} prod C(r_i, nu_i) P_N(r/2 - nu)
// (inclusion/exclusion over the N linear factors), and
//   P_N(h) = sum_{j = N mod 2, step 2} (h^T A h / 2)^{(N-j)/2} (gamma^T h)^j
//            / (((N-j)/2)! j!).
template <class T> cx<T> rep_moment(int M, const std::vector<cx<T>>& A, const std::vector<cx<T>>& g,
                                     const std::vector<int>& r) {
  int N = 0;
  for (int v : r) N += v;
  std::vector<int> nu(M, 0);
  nsum<T> tot;
  std::vector<T> h(M);
  while (true) {
    T sgn = 1, cb = 1;
    for (int i = 0; i < M; ++i) {
      h[i] = (T)r[i] / 2 - (T)nu[i];
      cb *= (T)binom(r[i], nu[i]);
      if (nu[i] & 1) sgn = -sgn;
    }
    cx<T> q, l;
    for (int i = 0; i < M; ++i) {
      if (h[i] == 0) continue;
      l += h[i] * g[i];
      for (int j = 0; j < M; ++j) q += (h[i] * h[j]) * A[(size_t)i * M + j];
    }
    q = T(0.5) * q;
    cx<T> pn;
    for (int j = N % 2; j <= N; j += 2) {
      int a = (N - j) / 2;
      cx<T> t(1);
      for (int e = 0; e < a; ++e) t = t * q;
      for (int e = 0; e < j; ++e) t = t * l;
      T fa = 1, fj = 1;
      for (int e = 2; e <= a; ++e) fa *= e;
      for (int e = 2; e <= j; ++e) fj *= e;
      pn += (T(1) / (fa * fj)) * t;
    }
    tot.add((sgn * cb) * pn);
    int i = 0;
    while (i < M && nu[i] == r[i]) nu[i++] = 0;
    if (i == M) break;
    nu[i]++;
  }
  return tot.get();
}

}  // namespace

extern "C" {

void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads() { return omp_get_max_threads(); }

// lhaf by recursive enumeration of single-pair matchings (N <= 20).
// prec: 0 = double, 1 = __float128.  out: 4 doubles (hi re, hi im, lo re, lo im).
int orc_lhaf_enum(int N, const double* A, const double* g, int prec, double* out) {
  if (N < 0 || N > 20) return 2;
  if (prec == 0) {
    auto a = load<double>(A, (int64_t)N * N);
    auto gg = load<double>(g, N);
    Enum<double> e{N, a, gg};
    store(e.rec(N ? (~0ull >> (64 - N)) : 0), out, true);
  } else {
    auto a = load<__float128>(A, (int64_t)N * N);
    auto gg = load<__float128>(g, N);
    Enum<__float128> e{N, a, gg};
    store(e.rec(N ? (~0ull >> (64 - N)) : 0), out, true);
  }
  return 0;
}

// lhaf by the same recursion memoised over unmatched-vertex sets (N <= 24).
int orc_lhaf_memo(int N, const double* A, const double* g, int prec, double* out) {
  if (N < 0 || N > 24) return 2;
  uint64_t full = N ? (~0ull >> (64 - N)) : 0;
  if (prec == 0) {
    auto a = load<double>(A, (int64_t)N * N);
    auto gg = load<double>(g, N);
    Memo<double> e{N, a, gg, std::vector<cx<double>>(1ull << N), std::vector<uint8_t>(1ull << N, 0)};
    store(e.rec(full), out, true);
  } else {
    auto a = load<__float128>(A, (int64_t)N * N);
    auto gg = load<__float128>(g, N);
    Memo<__float128> e{N, a, gg, std::vector<cx<__float128>>(1ull << N),
                       std::vector<uint8_t>(1ull << N, 0)};
    store(e.rec(full), out, true);
  }
  return 0;
}

// Power-trace sum over the pairs (u_p, w_p) repeated eta_p times.
// fds: 0 = eigenvalue-trace inclusion/exclusion, 1 = finite-difference sieve.
// halve: FDS symmetry halving on the documented halving pair.
// [t0, t1): term range of the documented enumeration (t1 < 0: to the end).
// scaled: multiply the FDS sum by 2^{-n} (set 0 for partial sums of ranges).
// out: 4 doubles (hi, lo); abs_sum: sum of |c_t f_t| (same scaling), nullable.
int orc_lhaf_sum(int N, const double* A, const double* g, int H, const int* u, const int* w,
                 const int* eta, int fds, int halve, int64_t t0, int64_t t1, int scaled, int prec,
                 double* out, double* abs_sum) {
  if (H < 0 || H > 32 || N > 128) return 2;
  if (prec == 0)
    power_trace_sum<double>(N, A, g, H, u, w, eta, fds, halve, t0, t1, scaled, out, abs_sum);
  else
    power_trace_sum<__float128>(N, A, g, H, u, w, eta, fds, halve, t0, t1, scaled, out, abs_sum);
  return 0;
}

int64_t orc_term_count(int H, const int* eta, int fds, int halve) {
  PairSpec ps;
  ps.H = H;
  ps.n = 0;
  for (int p = 0; p < H; ++p) {
    ps.eta.push_back(eta[p]);
    ps.n += eta[p];
  }
  return term_count(ps, fds != 0, halve != 0);
}

int orc_perm_ryser(int n, const double* B, int prec, double* out) {
  if (n < 0 || n > 24) return 2;
  if (prec == 0) store(ryser<double>(n, load<double>(B, (int64_t)n * n)), out, true);
  else store(ryser<__float128>(n, load<__float128>(B, (int64_t)n * n)), out, true);
  return 0;
}

int orc_lhaf_rep_moment(int M, const double* A, const double* g, const int* r, int prec, double* out) {
  std::vector<int> rv(r, r + M);
  if (prec == 0)
    store(rep_moment<double>(M, load<double>(A, (int64_t)M * M), load<double>(g, M), rv), out, true);
  else
    store(rep_moment<__float128>(M, load<__float128>(A, (int64_t)M * M), load<__float128>(g, M), rv),
          out, true);
  return 0;
}

}  // extern "C"
