// Host planner: fixed perfect matching, repeat counts and term enumeration
// parameters for one loop-hafnian problem.
//
// Plain problems use the matching of App. B.1/B.2 (position i with N/2 + i).
// Collision patterns use the greedy matching of App. B.3, which repeats pairs
// so that the repeated-pairs sum (App. B.2) needs prod (eta_i + 1) terms.
#include <algorithm>
#include <cmath>

#include "lhaf_internal.h"

namespace lh {

PairPlan plan_plain(int N) {
  PairPlan pp;
  pp.N = N;
  pp.rows = N;
  int Np = N + (N & 1);
  pp.padded = (N & 1) != 0;
  pp.n = Np / 2;
  pp.H = pp.n;
  pp.pos.resize(2 * pp.H);
  pp.eta.assign(pp.H, 1);
  for (int p = 0; p < pp.H; ++p) {
    pp.pos[p] = p;
    int w = pp.n + p;
    pp.pos[pp.H + p] = (w < N) ? w : -1;  // the last vertex of an odd N pairs with the pad
  }
  return pp;
}

// Greedy matching (App. B.3): repeatedly sort the remaining counts in
// descending order (ties: lower index first); if the largest count n1 is at
// least twice the second n2, pair the first mode with itself floor(n1/2)
// times, otherwise pair the first two modes n2 times; stop when at most one
// photon is left.  A single leftover photon is paired with a padding vertex.
PairPlan plan_repeated(const int32_t* r, int M) {
  PairPlan pp;
  struct Cnt {
    int mode, left;
  };
  std::vector<Cnt> live;
  int total = 0;
  for (int i = 0; i < M; ++i)
    if (r[i] > 0) {
      live.push_back({i, r[i]});
      total += r[i];
    }
  pp.N = total;
  pp.rows = M;
  std::vector<int> u, w;
  while (total > 1) {
    std::stable_sort(live.begin(), live.end(), [](const Cnt& a, const Cnt& b) {
      return a.left != b.left ? a.left > b.left : a.mode < b.mode;
    });
    int n1 = live[0].left;
    int n2 = live.size() > 1 ? live[1].left : 0;
    if (n1 >= 2 * n2) {
      int k = n1 / 2;
      u.push_back(live[0].mode);
      w.push_back(live[0].mode);
      pp.eta.push_back(k);
      live[0].left -= 2 * k;
      total -= 2 * k;
    } else {
      u.push_back(live[0].mode);
      w.push_back(live[1].mode);
      pp.eta.push_back(n2);
      live[0].left -= n2;
      live[1].left -= n2;
      total -= 2 * n2;
    }
    live.erase(std::remove_if(live.begin(), live.end(), [](const Cnt& c) { return c.left == 0; }),
               live.end());
  }
  if (total == 1) {
    u.push_back(live[0].mode);
    w.push_back(-1);
    pp.eta.push_back(1);
    pp.padded = true;
  }
  pp.H = (int)u.size();
  pp.n = 0;
  for (int e : pp.eta) pp.n += e;
  pp.pos.resize(2 * pp.H);
  for (int p = 0; p < pp.H; ++p) {
    pp.pos[p] = u[p];
    pp.pos[pp.H + p] = w[p];
  }
  return pp;
}

PairPlan plan_mixed(const int32_t* n, int M) {
  PairPlan pp;
  pp.rows = 2 * M;
  pp.N = 0;
  std::vector<int> u, w;
  for (int i = 0; i < M; ++i)
    if (n[i] > 0) {
      u.push_back(i);
      w.push_back(M + i);
      pp.eta.push_back(n[i]);
      pp.N += 2 * n[i];
    }
  pp.H = (int)u.size();
  pp.n = pp.N / 2;
  pp.pos.resize(2 * pp.H);
  for (int p = 0; p < pp.H; ++p) {
    pp.pos[p] = u[p];
    pp.pos[pp.H + p] = w[p];
  }
  return pp;
}

int64_t term_count(const PairPlan& pp, int mode, int* hp_out) {
  int hp = -1;
  if (mode == 1) {
    hp = 0;
    for (int p = 0; p < pp.H; ++p)
      if (pp.eta[p] & 1) {
        hp = p;
        break;
      }
  }
  int64_t T = 1;
  for (int p = 0; p < pp.H; ++p) {
    int radix = (p == hp) ? pp.eta[p] / 2 + 1 : pp.eta[p] + 1;
    T *= radix;
  }
  if (hp_out) *hp_out = hp;
  return T;
}

bool fill_prob(const PairPlan& pp, int mode, int64_t t0, int64_t t1, bool scaled, Prob* pr) {
  if (pp.H > kMaxPairs || 2 * pp.H > kMaxN) return false;
  *pr = Prob{};
  int hp;
  pr->T = term_count(pp, mode, &hp);
  pr->hp = (pp.H > 0) ? hp : -1;
  pr->t0 = t0 < 0 ? 0 : std::min<int64_t>(t0, pr->T);
  pr->t1 = (t1 < 0 || t1 > pr->T) ? pr->T : t1;
  if (pr->t1 < pr->t0) pr->t1 = pr->t0;
  pr->m = 2 * pp.H;
  pr->Nvert = pp.rows;
  pr->H = pp.H;
  pr->n = pp.n;
  pr->B = (pr->m + 7) / 8;
  if (pr->B < 1) pr->B = 1;
  pr->mode = mode;
  pr->scale = (mode == 1 && scaled) ? std::ldexp(1.0, -pp.n) : 1.0;
  pr->diag_keep_mask = 0;
  for (int p = 0; p < pp.H; ++p) {
    pr->eta[p] = (int8_t)pp.eta[p];
    pr->radix[p] = (int8_t)((p == pr->hp) ? pp.eta[p] / 2 + 1 : pp.eta[p] + 1);
    if (pp.eta[p] >= 2) pr->diag_keep_mask |= 1 << p;
  }
  for (int i = 0; i < kMaxN; ++i) pr->pos[i] = (i < 2 * pp.H) ? (int16_t)pp.pos[i] : (int16_t)-1;
  return true;
}

}  // namespace lh
