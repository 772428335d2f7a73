// C ABI of the loop-hafnian library: validation, planning, workspace layout
// and kernel launches.  No torch types; every buffer belongs to the caller
// (or, without a workspace, to one lazily grown per-device scratch buffer).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lhaf.h"
#include "lhaf_device.h"
#include "lhaf_internal.h"
// Kernel sources: this unit compiles only the small non-templated kernels
// (pack, finalize, reductions, scatters); the persistent kernels are
// instantiated per tile in their own units (lhaf_tile.hip) and reached
// through the launchers of lhaf_launch.h.
#define LH_COMMON_KERNELS
#include "lhaf_forward.hip"
#include "lhaf_backward.hip"
#include "lhaf_multi.hip"
#include "lhaf_real.hip"
#include "lhaf_launch.h"

namespace lh {

namespace {

std::mutex g_mu;
struct DevState {
  bool binom_ready = false;  // device attributes read
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  int cus = 0;
};
DevState g_dev[64];

lh_status ensure_device(int& dev) {
  if (hipGetDevice(&dev) != hipSuccess) return LH_EHIP;
  if (dev < 0 || dev >= 64) return LH_EHIP;
  DevState& S = g_dev[dev];
  if (!S.binom_ready) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return LH_EHIP;
    S.cus = cus > 0 ? cus : 1;
    S.binom_ready = true;
  }
  return LH_OK;
}

// Library-owned workspace of calls without one: reserved once per device at
// the first such call (256 MiB, or the call's need if larger), so later calls
// allocate nothing; a call that needs more replaces it by a buffer at least
// twice as large (waiting for the device first, since queued work may still
// use the old one).
lh_status get_scratch(int dev, size_t bytes, void** out) {
  DevState& S = g_dev[dev];
  if (S.scratch_bytes < bytes) {
    const size_t old = S.scratch_bytes;
    if (S.scratch) {
      (void)hipDeviceSynchronize();
      (void)hipFree(S.scratch);
      S.scratch = nullptr;
      S.scratch_bytes = 0;
    }
    size_t sz = std::max<size_t>(std::max<size_t>(bytes, 2 * old), (size_t)256 << 20);
    if (hipMalloc(&S.scratch, sz) != hipSuccess) return LH_ENOMEM;
    S.scratch_bytes = sz;
  }
  *out = S.scratch;
  return LH_OK;
}

// ---------------------------------------------------------------------------
// schedules: items (term ranges) queued per resident wavefront.  The grid of
// the persistent kernels is the number of wavefronts the chip keeps resident
// (CUs x occupancy of the kernel instance), so a schedule only sets how
// finely the term space is cut for load balance.
struct Schedule {
  int items_per_wave;
};
const Schedule kSchedules[] = {{1}, {2}, {4}, {8}, {16}, {32}};
const int kNumSchedules = (int)(sizeof(kSchedules) / sizeof(kSchedules[0]));
const int kDefaultSchedule = 2;

// schedule cache: lines "tile kind schedule" from $LHAF_TUNE_CACHE, kind 0 =
// ET forward, 1 = FDS forward, 2 = gradient pass (fused or backward, either
// sum)
struct TuneCache {
  bool loaded = false;
  int best[9][3];
};
TuneCache g_tune;

int pick_schedule(const lh_opts* o, int bmax, int kind) {
  if (o && o->schedule >= 0 && o->schedule < kNumSchedules) return o->schedule;
  if (!g_tune.loaded) {
    for (auto& r : g_tune.best) r[0] = r[1] = r[2] = -1;
    const char* path = std::getenv("LHAF_TUNE_CACHE");
    if (path) {
      if (FILE* f = std::fopen(path, "r")) {
        char line[256];
        while (std::fgets(line, sizeof(line), f)) {
          int b, md, s;
          if (line[0] == '#') continue;
          if (std::sscanf(line, "%d %d %d", &b, &md, &s) == 3 && b >= 1 && b <= 8 && md >= 0 &&
              md <= 2 && s >= 0 && s < kNumSchedules)
            g_tune.best[b][md] = s;
        }
        std::fclose(f);
      }
    }
    g_tune.loaded = true;
  }
  int s = g_tune.best[bmax][kind];
  return s >= 0 ? s : kDefaultSchedule;
}

// ---------------------------------------------------------------------------
struct ProblemIn {
  PairPlan plan;
  int64_t a_off, g_off, i_off;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t counter, probs, items, parts, parts2, aoff, goff, ioff, cdata, total;
};

Layout layout_for(int nprob, int nitems, size_t c_elems) {
  Layout L;
  size_t o = 0;
  L.counter = o;
  o = align_up(o + 256);
  L.probs = o;
  o = align_up(o + sizeof(Prob) * (size_t)std::max(nprob, 1));
  L.items = o;
  o = align_up(o + sizeof(Item) * (size_t)std::max(nitems, 1));
  L.parts = o;
  o = align_up(o + sizeof(Partial) * (size_t)std::max(nitems, 1));
  L.parts2 = o;  // partials of a second launch over the same items
  o = align_up(o + sizeof(Partial) * (size_t)std::max(nitems, 1));
  L.aoff = o;
  o = align_up(o + 8 * (size_t)std::max(nprob, 1));
  L.goff = o;
  o = align_up(o + 8 * (size_t)std::max(nprob, 1));
  L.ioff = o;
  o = align_up(o + 8 * (size_t)std::max(nprob, 1));
  L.cdata = o;
  o = align_up(o + sizeof(cd) * c_elems);
  L.total = o;
  return L;
}

struct Plan {
  std::vector<Prob> probs;
  std::vector<Item> items;
  std::vector<int64_t> aoff, goff, ioff;
  size_t c_elems = 0;
  int bmax = 1, nmax = 0;
  int grid = 1;
  int64_t saved_need = 0;  // entries of the per-term coefficient store
  int64_t grads_need = 0;  // entries of the per-problem reduced gradients
  Layout lay;
};

// wavefronts of one kernel instance resident per CU (occupancy query)
int resident_per_cu(bool bwd, int bmax, int nmax, int et, bool staged) {
  const size_t lds =
      bwd ? bwd_lds_bytes(bmax, std::max(nmax, 1), staged) : lds_bytes_for(std::max(nmax, 1));
  int blocks = 0;
  switch (bmax) {
#define LH_FN(BB)                                                      \
  case BB:                                                             \
    blocks = bwd ? resident_backward<BB>(lds, staged) : resident_forward<BB>(lds, et); \
    break;
    LH_FN(1) LH_FN(2) LH_FN(3) LH_FN(4) LH_FN(5) LH_FN(6) LH_FN(7)
    default: LH_FN(8)
#undef LH_FN
  }
  if (blocks < 1) blocks = 4;
  return blocks;
}

// relative cost of one term with register tile B (Householder ~ m^3)
double term_cost(int B) { return (double)B * B * B + 2.0; }

lh_status build_plan(std::vector<ProblemIn>& pin, const lh_opts& o, int dev, Plan& pl,
                     bool for_backward) {
  const int nprob = (int)pin.size();
  pl.probs.resize(nprob);
  pl.aoff.resize(nprob);
  pl.goff.resize(nprob);
  pl.ioff.resize(nprob);
  double total_cost = 0.0;
  int mode_any = o.sum;
  for (int b = 0; b < nprob; ++b) {
    Prob& P = pl.probs[b];
    if (!fill_prob(pin[b].plan, o.sum, o.term_begin, o.term_end, o.scaled != 0 || for_backward, &P))
      return LH_ESIZE;
    P.c_off = (int64_t)pl.c_elems;
    pl.c_elems += (size_t)(8 * P.B) * (8 * P.B) + 64;
    P.s_off = -1;
    if (P.n > 0) {
      P.s_off = pl.saved_need;
      pl.saved_need += (P.t1 - P.t0) * P.n;
    }
    P.r_off = pl.grads_need;
    pl.grads_need += (int64_t)bwd_item_elems(P.B);
    pl.aoff[b] = pin[b].a_off;
    pl.goff[b] = pin[b].g_off;
    pl.ioff[b] = pin[b].i_off;
    if (P.n > 0) {
      pl.bmax = std::max(pl.bmax, P.B);
      pl.nmax = std::max(pl.nmax, P.n);
      total_cost += (double)(P.t1 - P.t0) * term_cost(P.B);
    }
  }
  const int sched = pick_schedule(&o, pl.bmax, for_backward ? 2 : (mode_any ? 1 : 0));
  const Schedule S = kSchedules[sched];
  const int cus = g_dev[dev].cus;
  const int waves =
      std::max(1, cus * resident_per_cu(for_backward, pl.bmax, pl.nmax, o.sum == LH_SUM_ET,
                                        bwd_staged(pl.bmax, o.saved != nullptr)));
  const double target = std::max(total_cost / ((double)waves * S.items_per_wave), 1e-9);
  struct Tmp {
    int prob;
    int64_t t0, t1;
    double cost;
  };
  std::vector<Tmp> tmp;
  for (int b = 0; b < nprob; ++b) {
    Prob& P = pl.probs[b];
    const int64_t len = P.t1 - P.t0;
    if (P.n == 0 || len <= 0) continue;
    const double c = (double)len * term_cost(P.B);
    int64_t k = (int64_t)std::ceil(c / target);
    k = std::max<int64_t>(1, std::min<int64_t>(k, len));
    k = std::min<int64_t>(k, 1 << 22);
    for (int64_t s = 0; s < k; ++s) {
      const int64_t a = P.t0 + len * s / k, e = P.t0 + len * (s + 1) / k;
      tmp.push_back({b, a, e, (double)(e - a) * term_cost(P.B)});
    }
  }
  // longest-processing-time first; ties by problem and range (deterministic)
  std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& x, const Tmp& y) { return x.cost > y.cost; });
  // give every problem its items as a contiguous block of partial slots in
  // term order, independent of the processing order
  std::vector<int> count(nprob, 0);
  for (auto& t : tmp) count[t.prob]++;
  int acc = 0;
  for (int b = 0; b < nprob; ++b) {
    pl.probs[b].first_item = acc;
    pl.probs[b].n_items = count[b];
    acc += count[b];
  }
  // slot of each item = first_item + rank of its range inside the problem
  std::vector<std::vector<int64_t>> starts(nprob);
  for (auto& t : tmp) starts[t.prob].push_back(t.t0);
  for (auto& s : starts) std::sort(s.begin(), s.end());
  pl.items.resize(tmp.size());
  // processing order = LPT order; the kernel writes partial `slot`
  std::vector<Item> ordered(tmp.size());
  for (size_t r = 0; r < tmp.size(); ++r) {
    const Tmp& t = tmp[r];
    auto& st = starts[t.prob];
    const int rank = (int)(std::lower_bound(st.begin(), st.end(), t.t0) - st.begin());
    Item I;
    I.prob = t.prob;
    I.pad = pl.probs[t.prob].first_item + rank;  // partial slot
    I.t0 = t.t0;
    I.t1 = t.t1;
    ordered[r] = I;
  }
  pl.items = ordered;
  // every item must address a valid problem, slot and term range
  for (const Item& I : pl.items) {
    const Prob& P = pl.probs[I.prob];
    if (I.prob < 0 || I.prob >= nprob || I.t0 < P.t0 || I.t1 > P.t1 || I.t0 >= I.t1 ||
        I.pad < P.first_item || I.pad >= P.first_item + P.n_items)
      return LH_EINVAL;
  }
  pl.grid = (int)std::min<int64_t>((int64_t)waves, std::max<int64_t>(1, (int64_t)pl.items.size()));
  pl.lay = layout_for(nprob, (int)pl.items.size(), pl.c_elems);
  return LH_OK;
}

}  // namespace

// launch a planned forward evaluation
lh_status run_forward(Plan& pl, const lh_c128* A, int64_t lda, const lh_c128* g,
                      const int32_t* idx, lh_c128* out, double* err, const lh_opts& o,
                      void* ws, hipStream_t st, int dev, bool pageable = false);

// Plan tables reach the device through a small ring of pinned staging
// buffers per device.  Each buffer's copy is followed by an event; a buffer is
// reused only after its previous copy has completed, so a call never waits
// for earlier kernels on the stream (only, with more than kStageRing uploads
// in flight, for the oldest upload's copy).
constexpr int kStageRing = 8;
struct StageBuf {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};
// The entry point that allocates nothing (lhaf_batched_noalloc) stages
// through a separate ring of pageable host buffers (std::vector, no pinned
// or device allocation); the runtime copies those through its own staging.
struct PageBuf {
  std::vector<char> host;
  hipEvent_t done = nullptr;
  bool pending = false;
};
std::mutex g_stage_mu;
StageBuf g_stage[64][kStageRing];
int g_stage_next[64] = {0};
PageBuf g_pstage[64][kStageRing];
int g_pstage_next[64] = {0};

lh_status upload_plan(const Plan& pl, char* base, hipStream_t st, int dev, bool pageable) {
  const size_t nprob = pl.probs.size(), nit = pl.items.size();
  const size_t span = pl.lay.cdata;  // tables occupy [probs, cdata)
  std::lock_guard<std::mutex> lk(g_stage_mu);
  hipEvent_t* done;
  bool* pending;
  char* h;
  if (pageable) {
    PageBuf& S = g_pstage[dev][g_pstage_next[dev]];
    g_pstage_next[dev] = (g_pstage_next[dev] + 1) % kStageRing;
    if (!S.done && hipEventCreateWithFlags(&S.done, hipEventDisableTiming) != hipSuccess) {
      S.done = nullptr;
      return LH_EHIP;
    }
    if (S.pending) {
      if (hipEventSynchronize(S.done) != hipSuccess) return LH_EHIP;
      S.pending = false;
    }
    if (S.host.size() < span) S.host.resize(span);
    done = &S.done;
    pending = &S.pending;
    h = S.host.data();
  } else {
    StageBuf& S = g_stage[dev][g_stage_next[dev]];
    g_stage_next[dev] = (g_stage_next[dev] + 1) % kStageRing;
    if (!S.done && hipEventCreateWithFlags(&S.done, hipEventDisableTiming) != hipSuccess) {
      S.done = nullptr;
      return LH_EHIP;
    }
    if (S.pending) {
      if (hipEventSynchronize(S.done) != hipSuccess) return LH_EHIP;
      S.pending = false;
    }
    if (S.bytes < span) {
      if (S.host) (void)hipHostFree(S.host);
      S.host = nullptr;
      S.bytes = 0;
      size_t sz = std::max<size_t>(span, 1 << 16);
      if (hipHostMalloc(&S.host, sz, hipHostMallocDefault) != hipSuccess) return LH_ENOMEM;
      S.bytes = sz;
    }
    done = &S.done;
    pending = &S.pending;
    h = static_cast<char*>(S.host);
  }
  std::memset(h, 0, span);
  std::memcpy(h + pl.lay.probs, pl.probs.data(), sizeof(Prob) * nprob);
  if (nit) std::memcpy(h + pl.lay.items, pl.items.data(), sizeof(Item) * nit);
  std::memcpy(h + pl.lay.aoff, pl.aoff.data(), 8 * nprob);
  std::memcpy(h + pl.lay.goff, pl.goff.data(), 8 * nprob);
  std::memcpy(h + pl.lay.ioff, pl.ioff.data(), 8 * nprob);
  const size_t off = pl.lay.probs;
  if (hipMemcpyAsync(base + off, h + off, span - off, hipMemcpyHostToDevice, st) != hipSuccess)
    return LH_EHIP;
  if (hipEventRecord(*done, st) != hipSuccess) return LH_EHIP;
  *pending = true;
  return LH_OK;
}

}  // namespace lh

using namespace lh;

namespace lh {

// ET sums over problems of tile > kEtSplitTile run as two launches over the
// same items: the terms whose reduced tile is at most kEtSplitTile in that
// tile's instance (more resident wavefronts), the others in the largest
// tile's instance.
constexpr int kEtSplitTile = 3;
#ifndef LH_ET_SPLIT
#define LH_ET_SPLIT 1
#endif

// Launch shape and plan tables of a persistent kernel over plan `pl`.
static PersistArgs persist_args(const Plan& pl, char* base, size_t lds, hipStream_t st) {
  PersistArgs a;
  a.probs = reinterpret_cast<const Prob*>(base + pl.lay.probs);
  a.items = reinterpret_cast<const Item*>(base + pl.lay.items);
  a.n_items = (int)pl.items.size();
  a.counter = reinterpret_cast<int*>(base + pl.lay.counter);
  a.nmax = std::max(pl.nmax, 1);
  a.grid = pl.grid;
  a.lds = lds;
  a.stream = st;
  return a;
}

// Copy the host plan (problem table, item list, offsets) into the workspace,
// stream-ordered (the host does not wait for the stream).
lh_status upload_plan(const Plan& pl, char* base, hipStream_t st, int dev, bool pageable = false);

lh_status run_forward(Plan& pl, const lh_c128* A, int64_t lda, const lh_c128* g,
                      const int32_t* idx, lh_c128* out, double* err, const lh_opts& o, void* ws,
                      hipStream_t st, int dev, bool pageable) {
  char* base = static_cast<char*>(ws);
  const int nprob = (int)pl.probs.size();
  lh_status us = upload_plan(pl, base, st, dev, pageable);
  if (us != LH_OK) return us;
  hipLaunchKernelGGL(pack_kernel, dim3(nprob), dim3(256), 0, st,
                     reinterpret_cast<const Prob*>(base + pl.lay.probs),
                     reinterpret_cast<const int64_t*>(base + pl.lay.aoff),
                     reinterpret_cast<const int64_t*>(base + pl.lay.goff),
                     reinterpret_cast<const int64_t*>(base + pl.lay.ioff), A, lda, g, idx,
                     reinterpret_cast<cd*>(base + pl.lay.cdata),
                     reinterpret_cast<int*>(base + pl.lay.counter));
  if (hipGetLastError() != hipSuccess) return LH_EHIP;
  // 0 plain FP64, 1 double-double accumulation (also with compensated recurrences)
  const int acc_dd = o.acc == LH_ACC_FP64 ? 0 : 1;
  const bool comp = o.acc == LH_ACC_DD_COMP;
  cd* sv = reinterpret_cast<cd*>(o.saved);
  const Partial* parts2 = nullptr;
  if (!pl.items.empty()) {
    const size_t lds = comp ? lds_bytes_comp(std::max(pl.nmax, 1))
                            : lds_bytes_for(std::max(pl.nmax, 1));
    PersistArgs pa = persist_args(pl, base, lds, st);
    const cd* wsc = reinterpret_cast<const cd*>(base + pl.lay.cdata);
    Partial* parts = reinterpret_cast<Partial*>(base + pl.lay.parts);
    const int et = o.sum == LH_SUM_ET;
    int tlo = 1;
    hipError_t e = hipSuccess;
    if (et && pl.bmax > kEtSplitTile && LH_ET_SPLIT) {
      // ET terms of reduced tile <= kEtSplitTile in that tile's instance (more
      // resident wavefronts), the rest below in the largest tile's
      PersistArgs pa1 = pa;
      pa1.grid = (int)std::min<int64_t>(
          (int64_t)g_dev[dev].cus *
              std::max(1, comp ? resident_forward_comp<kEtSplitTile>(lds, 1)
                               : resident_forward<kEtSplitTile>(lds, 1)),
          std::max<int64_t>(1, (int64_t)pl.items.size()));
      e = comp ? launch_forward_comp<kEtSplitTile>(pa1, wsc, parts, acc_dd, sv, 1, 1, kEtSplitTile)
               : launch_forward<kEtSplitTile>(pa1, wsc, parts, acc_dd, sv, 1, 1, kEtSplitTile);
      if (e != hipSuccess) return LH_EHIP;
      pa.counter += kSecondCounter;
      parts = reinterpret_cast<Partial*>(base + pl.lay.parts2);
      parts2 = parts;
      tlo = kEtSplitTile + 1;
    }
    switch (pl.bmax) {
#define LH_FCASE(BB) \
  case BB:                                                                   \
    e = comp ? launch_forward_comp<BB>(pa, wsc, parts, acc_dd, sv, et, tlo, 8) \
             : launch_forward<BB>(pa, wsc, parts, acc_dd, sv, et, tlo, 8);     \
    break;
      LH_FCASE(1) LH_FCASE(2) LH_FCASE(3) LH_FCASE(4) LH_FCASE(5) LH_FCASE(6) LH_FCASE(7)
      default: LH_FCASE(8)
#undef LH_FCASE
    }
    if (e != hipSuccess) return LH_EHIP;
  }
  hipLaunchKernelGGL(finalize_kernel, dim3((nprob + 127) / 128), dim3(128), 0, st,
                     reinterpret_cast<const Prob*>(base + pl.lay.probs), nprob,
                     reinterpret_cast<const Partial*>(base + pl.lay.parts), parts2, out, o.out_lo,
                     err, acc_dd, 0);
  if (hipGetLastError() != hipSuccess) return LH_EHIP;
  return LH_OK;
}

// ---------------------------------------------------------------------------
// Fixed device workspace of lhaf_batched_noalloc: one array per GPU, part of
// the library's code object, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): the device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and is kept in g_static.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
static void* g_static[64] = {nullptr};

lh_status static_scratch(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_static[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LH_EHIP;
    g_static[dev] = ptr;
  }
  *out = g_static[dev];
  return LH_OK;
}

}  // namespace lh

// ===========================================================================
// public ABI
extern "C" {

void lh_opts_default(lh_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sum = LH_SUM_FDS;
  o->acc = LH_ACC_DD;
  o->term_begin = 0;
  o->term_end = -1;
  o->scaled = 1;
  o->schedule = -1;
  o->workspace = nullptr;
  o->ws_bytes = 0;
  o->out_lo = nullptr;
}

const char* lh_status_string(lh_status s) {
  switch (s) {
    case LH_OK: return "ok";
    case LH_EINVAL: return "invalid argument";
    case LH_ESIZE: return "problem too large (N > 64)";
    case LH_EHIP: return "HIP runtime error";
    case LH_ENOMEM: return "workspace too small or allocation failed";
    case LH_EUNSUPPORTED: return "unsupported option combination";
    case LH_ESCRATCH: return "batch needs more than the fixed device scratch of lhaf_batched_noalloc";
    default: return "unknown status";
  }
}

int32_t lhaf_schedule_count(void) { return kNumSchedules; }

int64_t lhaf_term_count(int32_t N, const int32_t* r, int32_t sum) {
  if (N < 0) return -LH_EINVAL;
  PairPlan pp;
  if (r) {
    for (int i = 0; i < N; ++i)
      if (r[i] < 0) return -LH_EINVAL;
    pp = plan_repeated(r, N);
  } else {
    pp = plan_plain(N);
  }
  return term_count(pp, sum == LH_SUM_FDS ? 1 : 0, nullptr);
}

int32_t lhaf_plan_pairs(int32_t N, const int32_t* r, int32_t* pos, int32_t* eta) {
  if (N < 0 || !pos || !eta) return -LH_EINVAL;
  PairPlan pp;
  if (r) {
    int tot = 0;
    for (int i = 0; i < N; ++i) {
      if (r[i] < 0) return -LH_EINVAL;
      tot += r[i];
    }
    if (tot > kMaxN || N > kMaxRows) return -LH_ESIZE;
    pp = plan_repeated(r, N);
  } else {
    if (N > kMaxN) return -LH_ESIZE;
    pp = plan_plain(N);
  }
  for (int i = 0; i < 2 * pp.H; ++i) pos[i] = pp.pos[i];
  for (int p = 0; p < pp.H; ++p) eta[p] = pp.eta[p];
  return pp.H;
}

// Pair plans of the problems of a batch (index lists idx_off, optional
// multiplicities r packed like the index lists).
static lh_status parse_problems(int32_t B, const int64_t* idx_off, const int32_t* r,
                                int64_t stride_A, int64_t stride_g, std::vector<ProblemIn>& pin) {
  if (B < 0 || !idx_off) return LH_EINVAL;
  pin.assign(B, ProblemIn());
  for (int b = 0; b < B; ++b) {
    const int64_t s0 = idx_off[b], s1 = idx_off[b + 1];
    if (s1 < s0 || s0 < 0) return LH_EINVAL;
    const int64_t N = s1 - s0;
    if (r) {
      int64_t tot = 0;
      for (int64_t k = s0; k < s1; ++k) {
        if (r[k] < 0) return LH_EINVAL;
        tot += r[k];
      }
      if (N > kMaxRows || tot > kMaxN) return LH_ESIZE;
      pin[b].plan = plan_repeated(r + s0, (int)N);
    } else {
      if (N > kMaxN) return LH_ESIZE;
      pin[b].plan = plan_plain((int)N);
    }
    pin[b].a_off = (int64_t)b * stride_A;
    pin[b].g_off = (int64_t)b * stride_g;
    pin[b].i_off = s0;
  }
  return LH_OK;
}

// comp_ok: the entry point evaluates values through the forward kernels, the
// only ones with a compensated-recurrence instance
static lh_status validate_opts(const lh_opts* opts, lh_opts& o, bool comp_ok = false) {
  lh_opts_default(&o);
  if (opts) o = *opts;
  if (o.sum != LH_SUM_ET && o.sum != LH_SUM_FDS) return LH_EINVAL;
  if (o.acc != LH_ACC_FP64 && o.acc != LH_ACC_DD && o.acc != LH_ACC_DD_COMP) return LH_EINVAL;
  if (o.acc == LH_ACC_DD_COMP && (!comp_ok || o.saved || o.grads)) return LH_EUNSUPPORTED;
  if (o.saved && o.saved_count < 0) return LH_EINVAL;
  if (o.grads && o.grads_count < 0) return LH_EINVAL;
  return LH_OK;
}

static lh_status backward_impl(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                               const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                               const int64_t* idx_off, const int32_t* r, const lh_c128* grad_out,
                               lh_c128* dA, lh_c128* dgamma, int32_t base_dim, bool fused,
                               lh_c128* out, double* err_est, void* workspace, size_t ws_bytes,
                               const lh_opts& o, hipStream_t st, bool query_only,
                               size_t* need_bytes);

static lh_status batched_impl(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                              const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                              const int64_t* idx_off, const int32_t* r, lh_c128* out,
                              double* err_est, void* workspace, size_t ws_bytes,
                              const lh_opts& o, hipStream_t st, bool query_only,
                              size_t* need_bytes) {
  if (o.grads) {  // fused value + gradient pass
    if (!query_only && !out) return LH_EINVAL;
    void* ws = workspace;
    if (!ws && !query_only) {
      size_t need = 0;
      lh_status qs = backward_impl(B, nullptr, 1, 0, nullptr, 0, nullptr, idx_off, r, nullptr,
                                   nullptr, nullptr, 1, true, nullptr, nullptr, nullptr, 0, o, st,
                                   true, &need);
      if (qs != LH_OK) return qs;
      int dev = 0;
      qs = ensure_device(dev);
      if (qs != LH_OK) return qs;
      std::lock_guard<std::mutex> lk(g_mu);
      qs = get_scratch(dev, need, &ws);
      if (qs != LH_OK) return qs;
      return backward_impl(B, A_base, lda, stride_A, gamma_base, stride_g, idx, idx_off, r,
                           nullptr, nullptr, nullptr, 1, true, out, err_est, ws, need, o, st,
                           false, nullptr);
    }
    return backward_impl(B, A_base, lda, stride_A, gamma_base, stride_g, idx, idx_off, r, nullptr,
                         nullptr, nullptr, 1, true, out, err_est, ws, ws_bytes, o, st, query_only,
                         need_bytes);
  }
  std::vector<ProblemIn> pin;
  lh_status ps = parse_problems(B, idx_off, r, stride_A, stride_g, pin);
  if (ps != LH_OK) return ps;
  int dev = 0;
  if (!query_only || true) {
    lh_status s = ensure_device(dev);
    if (s != LH_OK) return s;
  }
  Plan pl;
  lh_status s = build_plan(pin, o, dev, pl, false);
  if (s != LH_OK) return s;
  if (query_only) {
    *need_bytes = pl.lay.total;
    return LH_OK;
  }
  if (o.saved && o.saved_count < pl.saved_need) return LH_ENOMEM;
  if (B == 0) return LH_OK;
  if (!A_base || !gamma_base || !out || lda < 1) return LH_EINVAL;
  void* ws = workspace;
  if (!ws) {
    std::lock_guard<std::mutex> lk(g_mu);
    s = get_scratch(dev, pl.lay.total, &ws);
    if (s != LH_OK) return s;
    return run_forward(pl, A_base, lda, gamma_base, idx, out, err_est, o, ws, st, dev);
  }
  if (ws_bytes < pl.lay.total) return LH_ENOMEM;
  return run_forward(pl, A_base, lda, gamma_base, idx, out, err_est, o, ws, st, dev);
}

size_t lhaf_batched_workspace(int32_t B, const int64_t* idx_off, const int32_t* r,
                              const lh_opts* opts) {
  lh_opts o;
  if (validate_opts(opts, o, true) != LH_OK) return 0;
  size_t need = 0;
  if (batched_impl(B, nullptr, 1, 0, nullptr, 0, nullptr, idx_off, r, nullptr, nullptr, nullptr,
                   0, o, nullptr, true, &need) != LH_OK)
    return 0;
  return need;
}

lh_status lhaf_batched(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                       const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                       const int64_t* idx_off, const int32_t* r, lh_c128* out, double* err_est,
                       void* workspace, size_t ws_bytes, const lh_opts* opts, void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o, true);
  if (s != LH_OK) return s;
  if (workspace == nullptr && o.workspace) {
    workspace = o.workspace;
    ws_bytes = o.ws_bytes;
  }
  return batched_impl(B, A_base, lda, stride_A, gamma_base, stride_g, idx, idx_off, r, out,
                      err_est, workspace, ws_bytes, o, (hipStream_t)stream, false, nullptr);
}

lh_status lhaf_batched_noalloc(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                               const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                               const int64_t* idx_off, const int32_t* r, lh_c128* out,
                               double* err_est, const lh_opts* opts, void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o, true);
  if (s != LH_OK) return s;
  if (o.grads) return LH_EUNSUPPORTED;
  std::vector<ProblemIn> pin;
  s = parse_problems(B, idx_off, r, stride_A, stride_g, pin);
  if (s != LH_OK) return s;
  int dev = 0;
  s = ensure_device(dev);
  if (s != LH_OK) return s;
  void* ptr = nullptr;
  s = static_scratch(dev, &ptr);
  if (s != LH_OK) return s;
  Plan pl;
  s = build_plan(pin, o, dev, pl, false);
  if (s != LH_OK) return s;
  if (pl.lay.total > kStaticScratchBytes) return LH_ESCRATCH;
  if (o.saved && o.saved_count < pl.saved_need) return LH_ENOMEM;
  if (B == 0) return LH_OK;
  if (!A_base || !gamma_base || !out || lda < 1) return LH_EINVAL;
  return run_forward(pl, A_base, lda, gamma_base, idx, out, err_est, o, ptr, (hipStream_t)stream,
                     dev, true);
}

size_t lhaf_noalloc_scratch_bytes(void) { return kStaticScratchBytes; }

lh_status lhaf(const lh_c128* A, int64_t lda, const lh_c128* gamma, int32_t N, lh_c128* out,
               double* err_est, const lh_opts* opts, void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o, true);
  if (s != LH_OK) return s;
  if (N < 0 || !out) return LH_EINVAL;
  if (N > kMaxN) return LH_ESIZE;
  if (N > 0 && (!A || !gamma || lda < N)) return LH_EINVAL;
  int64_t off[2] = {0, N};
  if (N == 0) {
    int dev;
    s = ensure_device(dev);
    if (s != LH_OK) return s;
    hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, out, o.out_lo,
                       err_est, 1);
    return hipGetLastError() == hipSuccess ? LH_OK : LH_EHIP;
  }
  return batched_impl(1, A, lda, 0, gamma, 0, nullptr, off, nullptr, out, err_est, o.workspace,
                      o.ws_bytes, o, (hipStream_t)stream, false, nullptr);
}

lh_status lhaf_repeated(const lh_c128* A, int64_t lda, const lh_c128* gamma, const int32_t* r,
                        int32_t M, lh_c128* out, double* err_est, const lh_opts* opts,
                        void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o, true);
  if (s != LH_OK) return s;
  if (M < 0 || !out || (M > 0 && !r)) return LH_EINVAL;
  int64_t tot = 0;
  for (int i = 0; i < M; ++i) {
    if (r[i] < 0) return LH_EINVAL;
    tot += r[i];
  }
  if (tot > kMaxN) return LH_ESIZE;
  if (M > 0 && (!A || !gamma || lda < M)) return LH_EINVAL;
  if (tot == 0) {
    int dev;
    s = ensure_device(dev);
    if (s != LH_OK) return s;
    hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, out, o.out_lo,
                       err_est, 1);
    return hipGetLastError() == hipSuccess ? LH_OK : LH_EHIP;
  }
  int64_t off[2] = {0, M};
  return batched_impl(1, A, lda, 0, gamma, 0, nullptr, off, r, out, err_est, o.workspace,
                      o.ws_bytes, o, (hipStream_t)stream, false, nullptr);
}

// One problem, several outputs (chain-rule step or loop-weight vectors).
static lh_status multi_impl(const PairPlan& plan, const lh_c128* A, int64_t lda,
                            const lh_c128* gamma, const lh_c128* gammas, int64_t ldg,
                            MultiArgs ma, lh_c128* out, double* err, const lh_opts& o,
                            hipStream_t st) {
  int dev = 0;
  lh_status s = ensure_device(dev);
  if (s != LH_OK) return s;
  std::vector<ProblemIn> pin(1);
  pin[0].plan = plan;
  pin[0].a_off = pin[0].g_off = pin[0].i_off = 0;
  Plan pl;
  s = build_plan(pin, o, dev, pl, false);
  if (s != LH_OK) return s;
  if (pl.probs[0].n > 32) return LH_ESIZE;
  const size_t parts_bytes = sizeof(Partial) * (size_t)std::max<size_t>(pl.items.size(), 1) * ma.nout;
  const size_t off_parts = pl.lay.total;
  const size_t off_vg = align_up(off_parts + parts_bytes);
  const size_t total = align_up(off_vg + sizeof(cd) * 64 * (size_t)(ma.mode == 1 ? ma.nout : 1));
  void* ws = o.workspace;
  std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);
  if (!ws) {
    lk.lock();
    s = get_scratch(dev, total, &ws);
    if (s != LH_OK) return s;
  } else if (o.ws_bytes < total) {
    return LH_ENOMEM;
  }
  char* base = static_cast<char*>(ws);
  s = upload_plan(pl, base, st, dev);
  if (s != LH_OK) return s;
  hipLaunchKernelGGL(pack_kernel, dim3(1), dim3(256), 0, st,
                     reinterpret_cast<const Prob*>(base + pl.lay.probs),
                     reinterpret_cast<const int64_t*>(base + pl.lay.aoff),
                     reinterpret_cast<const int64_t*>(base + pl.lay.goff),
                     reinterpret_cast<const int64_t*>(base + pl.lay.ioff), A, lda, gamma, nullptr,
                     reinterpret_cast<cd*>(base + pl.lay.cdata),
                     reinterpret_cast<int*>(base + pl.lay.counter));
  if (hipGetLastError() != hipSuccess) return LH_EHIP;
  cd* vg = reinterpret_cast<cd*>(base + off_vg);
  if (ma.mode == 1) {
    hipLaunchKernelGGL(pack_gammas_kernel, dim3((64 * ma.nout + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<const Prob*>(base + pl.lay.probs), gammas, ldg, ma.nout, vg);
    if (hipGetLastError() != hipSuccess) return LH_EHIP;
    ma.vg = vg;
  }
  Partial* parts = reinterpret_cast<Partial*>(base + off_parts);
  const int acc_dd = o.acc == LH_ACC_DD ? 1 : 0;
  if (!pl.items.empty()) {
    const int nmax = std::max(pl.nmax, 1);
    const size_t lds = multi_lds_bytes(nmax, ma.mode, ma.nout);
    const PersistArgs pa = persist_args(pl, base, lds, st);
    const cd* wsc = reinterpret_cast<const cd*>(base + pl.lay.cdata);
    hipError_t e;
#define LH_MLAUNCH(BB)                                            \
  e = ma.mode == 1 ? launch_multi<BB, 1>(pa, wsc, parts, acc_dd, ma) \
                   : launch_multi<BB, 0>(pa, wsc, parts, acc_dd, ma)
    switch (pl.bmax) {
      case 1: LH_MLAUNCH(1); break;
      case 2: LH_MLAUNCH(2); break;
      case 3: LH_MLAUNCH(3); break;
      case 4: LH_MLAUNCH(4); break;
      case 5: LH_MLAUNCH(5); break;
      case 6: LH_MLAUNCH(6); break;
      case 7: LH_MLAUNCH(7); break;
      default: LH_MLAUNCH(8); break;
    }
#undef LH_MLAUNCH
    if (e != hipSuccess) return LH_EHIP;
    if (hipGetLastError() != hipSuccess) return LH_EHIP;
  }
  hipLaunchKernelGGL(finalize_multi_kernel, dim3(1), dim3(64), 0, st,
                     reinterpret_cast<const Prob*>(base + pl.lay.probs), parts, ma, out, err,
                     acc_dd);
  if (hipGetLastError() != hipSuccess) return LH_EHIP;
  return LH_OK;
}

// Gradient pass over a batch.  Three uses:
//   lhaf_backward                : term pass -> per-problem gradients in the
//                                  workspace -> scatter with grad_out
//   lhaf_backward + opts->grads  : scatter from the gradients a fused pass
//                                  left in opts->grads (no term pass)
//   lhaf_batched + opts->grads   : fused pass: term pass that also sums the
//                                  values (out, err_est), gradients into
//                                  opts->grads (no scatter)
static lh_status backward_impl(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                               const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                               const int64_t* idx_off, const int32_t* r, const lh_c128* grad_out,
                               lh_c128* dA, lh_c128* dgamma, int32_t base_dim, bool fused,
                               lh_c128* out, double* err_est, void* workspace, size_t ws_bytes,
                               const lh_opts& o, hipStream_t st, bool query_only,
                               size_t* need_bytes) {
  std::vector<ProblemIn> pin;
  lh_status ps = parse_problems(B, idx_off, r, stride_A, stride_g, pin);
  if (ps != LH_OK) return ps;
  int dev = 0;
  lh_status s = ensure_device(dev);
  if (s != LH_OK) return s;
  const bool from_grads = !fused && o.grads != nullptr;
  // the gradient of a term range is that range's share of the full gradient
  // (FDS prefactor included), so slices add up
  lh_opts ob = o;
  ob.scaled = 1;
  Plan pl;
  s = build_plan(pin, ob, dev, pl, true);
  if (s != LH_OK) return s;
  size_t gtot = 0;
  for (auto& P : pl.probs) {
    P.g_off = (int64_t)gtot;
    gtot += (size_t)P.n_items * bwd_item_elems(P.B);
  }
  gtot = std::max<size_t>(gtot, 64);
  const size_t scr = (size_t)pl.grid * bwd_wave_scratch_elems(pl.bmax);
  size_t off_g = 0, off_r = 0, off_s = 0, total = pl.lay.total;
  if (!from_grads) {
    off_g = pl.lay.total;
    off_r = align_up(off_g + gtot * sizeof(cd));
    off_s = align_up(off_r + (fused ? 0 : (size_t)pl.grads_need * sizeof(cd)));
    total = align_up(off_s + scr * sizeof(cd));
  }
  if (query_only) {
    *need_bytes = total;
    return LH_OK;
  }
  if (o.grads && o.grads_count < pl.grads_need) return LH_ENOMEM;
  if (fused && o.saved) return LH_EUNSUPPORTED;
  if (B == 0) return LH_OK;
  if (!A_base || !gamma_base || lda < 1 || (fused && !out)) return LH_EINVAL;
  if (!fused) {
    if (!grad_out || !dA || !dgamma) return LH_EINVAL;
    if (base_dim < 1 || base_dim > kMaxRows || lda < base_dim) return LH_EINVAL;
    if (!idx) {  // without index lists, problem b's vertices are rows 0..N_b-1
      for (int b = 0; b < B; ++b)
        if (idx_off[b + 1] - idx_off[b] > base_dim) return LH_EINVAL;
    }
  }
  if (!workspace) return LH_EINVAL;
  if (ws_bytes < total) return LH_ENOMEM;
  if (o.saved && o.saved_count < pl.saved_need) return LH_ENOMEM;
  char* base = static_cast<char*>(workspace);
  s = upload_plan(pl, base, st, dev);
  if (s != LH_OK) return s;
  const int nprob = (int)pl.probs.size();
  const Prob* probs = reinterpret_cast<const Prob*>(base + pl.lay.probs);
  const int acc_dd = o.acc == LH_ACC_DD ? 1 : 0;
  cd* grads = from_grads || fused ? reinterpret_cast<cd*>(o.grads)
                                  : reinterpret_cast<cd*>(base + off_r);
  if (!from_grads) {
    hipLaunchKernelGGL(pack_kernel, dim3(nprob), dim3(256), 0, st, probs,
                       reinterpret_cast<const int64_t*>(base + pl.lay.aoff),
                       reinterpret_cast<const int64_t*>(base + pl.lay.goff),
                       reinterpret_cast<const int64_t*>(base + pl.lay.ioff), A_base, lda,
                       gamma_base, idx, reinterpret_cast<cd*>(base + pl.lay.cdata),
                       reinterpret_cast<int*>(base + pl.lay.counter));
    if (hipGetLastError() != hipSuccess) return LH_EHIP;
    cd* gsl = reinterpret_cast<cd*>(base + off_g);
    cd* scratch = reinterpret_cast<cd*>(base + off_s);
    Partial* parts = fused ? reinterpret_cast<Partial*>(base + pl.lay.parts) : nullptr;
    if (!pl.items.empty()) {
      const bool staged = bwd_staged(pl.bmax, o.saved != nullptr);
      const size_t lds = bwd_lds_bytes(pl.bmax, std::max(pl.nmax, 1), staged);
      const PersistArgs pa = persist_args(pl, base, lds, st);
      const cd* wsc = reinterpret_cast<const cd*>(base + pl.lay.cdata);
      const cd* sv = reinterpret_cast<const cd*>(o.saved);
      hipError_t e;
      switch (pl.bmax) {
#define LH_BCASE(BB) \
  case BB: e = launch_backward<BB>(pa, wsc, gsl, scratch, sv, parts, acc_dd, staged); break;
        LH_BCASE(1) LH_BCASE(2) LH_BCASE(3) LH_BCASE(4) LH_BCASE(5) LH_BCASE(6) LH_BCASE(7)
        default: LH_BCASE(8)
#undef LH_BCASE
      }
      if (e != hipSuccess) return LH_EHIP;
    }
    hipLaunchKernelGGL(greduce_kernel, dim3(nprob), dim3(256), 0, st, probs, gsl, grads);
    if (hipGetLastError() != hipSuccess) return LH_EHIP;
    if (fused) {
      hipLaunchKernelGGL(finalize_kernel, dim3((nprob + 127) / 128), dim3(128), 0, st, probs,
                         nprob, reinterpret_cast<const Partial*>(base + pl.lay.parts), nullptr,
                         out, o.out_lo, err_est, acc_dd, o.scaled ? 0 : 1);
      return hipGetLastError() == hipSuccess ? LH_OK : LH_EHIP;
    }
  }
  if (stride_A != 0) {
    hipLaunchKernelGGL(scatter_dense_kernel, dim3(nprob), dim3(256), 0, st, probs, grads,
                       reinterpret_cast<const int64_t*>(base + pl.lay.ioff), idx, grad_out, dA,
                       lda, stride_A, dgamma, stride_g, base_dim);
  } else {
    const int64_t E = (int64_t)base_dim * base_dim + base_dim;
    hipLaunchKernelGGL(scatter_shared_kernel, dim3((unsigned)((E + 127) / 128)), dim3(128), 0, st,
                       probs, nprob, reinterpret_cast<const int64_t*>(base + pl.lay.ioff), idx,
                       grads, grad_out, dA, lda, dgamma, base_dim);
  }
  if (hipGetLastError() != hipSuccess) return LH_EHIP;
  return LH_OK;
}

lh_status lhaf_mixed(const lh_c128* A, int64_t lda, const lh_c128* gamma, const int32_t* n,
                     int32_t M, lh_c128* out, double* err_est, const lh_opts* opts, void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o, true);
  if (s != LH_OK) return s;
  if (M < 0 || !out || (M > 0 && !n)) return LH_EINVAL;
  int64_t tot = 0;
  for (int i = 0; i < M; ++i) {
    if (n[i] < 0) return LH_EINVAL;
    tot += n[i];
  }
  if (2 * tot > kMaxN || 2 * (int64_t)M > kMaxRows) return LH_ESIZE;
  if (o.grads) return LH_EUNSUPPORTED;
  if (M > 0 && (!A || !gamma || lda < 2 * (int64_t)M)) return LH_EINVAL;
  int dev = 0;
  s = ensure_device(dev);
  if (s != LH_OK) return s;
  if (tot == 0) {
    hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, out, o.out_lo,
                       err_est, 1);
    return hipGetLastError() == hipSuccess ? LH_OK : LH_EHIP;
  }
  std::vector<ProblemIn> pin(1);
  pin[0].plan = plan_mixed(n, M);
  pin[0].a_off = pin[0].g_off = pin[0].i_off = 0;
  Plan pl;
  s = build_plan(pin, o, dev, pl, false);
  if (s != LH_OK) return s;
  if (o.saved && o.saved_count < pl.saved_need) return LH_ENOMEM;
  void* ws = o.workspace;
  std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);
  if (!ws) {
    lk.lock();
    s = get_scratch(dev, pl.lay.total, &ws);
    if (s != LH_OK) return s;
  } else if (o.ws_bytes < pl.lay.total) {
    return LH_ENOMEM;
  }
  return run_forward(pl, A, lda, gamma, nullptr, out, err_est, o, ws, (hipStream_t)stream, dev);
}

lh_status lhaf_real(const double* A, int64_t lda, const double* gamma, const int32_t* r,
                    int32_t M, double* out, double* err_est, const lh_opts* opts, void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o);
  if (s != LH_OK) return s;
  if (o.saved || o.out_lo || o.grads) return LH_EUNSUPPORTED;
  if (M < 0 || !out) return LH_EINVAL;
  PairPlan pp;
  if (r) {
    int64_t tot = 0;
    for (int i = 0; i < M; ++i) {
      if (r[i] < 0) return LH_EINVAL;
      tot += r[i];
    }
    if (tot > kMaxN || M > kMaxRows) return LH_ESIZE;
    pp = plan_repeated(r, M);
  } else {
    if (M > kMaxN) return LH_ESIZE;
    pp = plan_plain(M);
  }
  if (M > 0 && (!A || !gamma || lda < M)) return LH_EINVAL;
  int dev = 0;
  s = ensure_device(dev);
  if (s != LH_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  std::vector<ProblemIn> pin(1);
  pin[0].plan = pp;
  pin[0].a_off = pin[0].g_off = pin[0].i_off = 0;
  Plan pl;
  s = build_plan(pin, o, dev, pl, false);
  if (s != LH_OK) return s;
  void* ws = o.workspace;
  std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);
  if (!ws) {
    lk.lock();
    s = get_scratch(dev, pl.lay.total, &ws);
    if (s != LH_OK) return s;
  } else if (o.ws_bytes < pl.lay.total) {
    return LH_ENOMEM;
  }
  char* base = static_cast<char*>(ws);
  s = upload_plan(pl, base, st, dev);
  if (s != LH_OK) return s;
  hipLaunchKernelGGL(real::pack_kernel, dim3(1), dim3(256), 0, st,
                     reinterpret_cast<const Prob*>(base + pl.lay.probs), A, lda, gamma,
                     reinterpret_cast<double*>(base + pl.lay.cdata),
                     reinterpret_cast<int*>(base + pl.lay.counter));
  if (hipGetLastError() != hipSuccess) return LH_EHIP;
  const int acc_dd = o.acc == LH_ACC_DD ? 1 : 0;
  if (!pl.items.empty()) {
    const int nmax = std::max(pl.nmax, 1);
    const size_t lds = real::lds_bytes(nmax);
    const PersistArgs pa = persist_args(pl, base, lds, st);
    const double* wsr = reinterpret_cast<const double*>(base + pl.lay.cdata);
    Partial* parts = reinterpret_cast<Partial*>(base + pl.lay.parts);
    hipError_t e;
    switch (pl.bmax) {
#define LH_RCASE(BB) \
  case BB: e = launch_real<BB>(pa, wsr, parts, acc_dd); break;
      LH_RCASE(1) LH_RCASE(2) LH_RCASE(3) LH_RCASE(4) LH_RCASE(5) LH_RCASE(6) LH_RCASE(7)
      default: LH_RCASE(8)
#undef LH_RCASE
    }
    if (e != hipSuccess) return LH_EHIP;
    if (hipGetLastError() != hipSuccess) return LH_EHIP;
  }
  hipLaunchKernelGGL(real::finalize_kernel, dim3(1), dim3(64), 0, st,
                     reinterpret_cast<const Prob*>(base + pl.lay.probs),
                     reinterpret_cast<const Partial*>(base + pl.lay.parts), out, err_est, acc_dd);
  return hipGetLastError() == hipSuccess ? LH_OK : LH_EHIP;
}

lh_status lhaf_chain(const lh_c128* A, int64_t lda, const lh_c128* gamma, const int32_t* r,
                     int32_t M, int32_t mode_b, int32_t n_cut, lh_c128* out, double* err_est,
                     const lh_opts* opts, void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o);
  if (s != LH_OK) return s;
  if (o.sum != LH_SUM_ET) return LH_EUNSUPPORTED;
  if (o.saved || o.grads) return LH_EUNSUPPORTED;
  if (M < 1 || !r || !out || !A || !gamma || lda < M || mode_b < 0 || mode_b >= M || n_cut < 0)
    return LH_EINVAL;
  if (M > kMaxRows) return LH_ESIZE;
  int64_t tot = 0;
  for (int i = 0; i < M; ++i) {
    if (r[i] < 0) return LH_EINVAL;
    if (i != mode_b) tot += r[i];
  }
  if (r[mode_b] != 0) return LH_EINVAL;
  if (tot + n_cut > kMaxN || n_cut + 1 > 64) return LH_ESIZE;
  PairPlan pp = plan_repeated(r, M);
  const int nf = pp.n;
  MultiArgs ma{};
  ma.mode = 0;
  ma.nout = n_cut + 1;
  ma.nf = nf;
  ma.pbb = ma.pbp = -1;
  // append the batched mode: J self pairs, one pair with a padding vertex
  std::vector<int> u(pp.pos.begin(), pp.pos.begin() + pp.H), w(pp.pos.begin() + pp.H, pp.pos.end());
  const int J = n_cut / 2;
  if (J >= 1) {
    ma.pbb = (int)u.size();
    u.push_back(mode_b);
    w.push_back(mode_b);
    pp.eta.push_back(J);
  }
  if (n_cut >= 1) {
    ma.pbp = (int)u.size();
    u.push_back(mode_b);
    w.push_back(-1);
    pp.eta.push_back(1);
  }
  pp.H = (int)u.size();
  pp.n = 0;
  for (int e : pp.eta) pp.n += e;
  if (pp.H > kMaxPairs || 2 * pp.H > kMaxN || pp.n > 32) return LH_ESIZE;
  pp.pos.assign(2 * pp.H, -1);
  for (int p = 0; p < pp.H; ++p) {
    pp.pos[p] = u[p];
    pp.pos[pp.H + p] = w[p];
  }
  if (pp.H == 0) {  // nothing fixed, n_cut = 0: the empty pattern
    int dev;
    s = ensure_device(dev);
    if (s != LH_OK) return s;
    hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, out, nullptr,
                       err_est, 1);
    return hipGetLastError() == hipSuccess ? LH_OK : LH_EHIP;
  }
  return multi_impl(pp, A, lda, gamma, nullptr, 0, ma, out, err_est, o, (hipStream_t)stream);
}

lh_status lhaf_gammas(const lh_c128* A, int64_t lda, const lh_c128* gammas, int64_t ldg,
                      const int32_t* r, int32_t M, int32_t G, lh_c128* out, double* err_est,
                      const lh_opts* opts, void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o);
  if (s != LH_OK) return s;
  if (o.saved || o.grads) return LH_EUNSUPPORTED;
  if (M < 0 || G < 1 || !out || (M > 0 && (!A || !gammas || lda < M || ldg < M))) return LH_EINVAL;
  if (G > 64) return LH_ESIZE;
  PairPlan pp;
  if (r) {
    int64_t tot = 0;
    for (int i = 0; i < M; ++i) {
      if (r[i] < 0) return LH_EINVAL;
      tot += r[i];
    }
    if (tot > kMaxN || M > kMaxRows) return LH_ESIZE;
    pp = plan_repeated(r, M);
  } else {
    if (M > kMaxN) return LH_ESIZE;
    pp = plan_plain(M);
  }
  if (pp.n == 0) {
    int dev;
    s = ensure_device(dev);
    if (s != LH_OK) return s;
    hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, out, nullptr,
                       err_est, G);
    return hipGetLastError() == hipSuccess ? LH_OK : LH_EHIP;
  }
  MultiArgs ma{};
  ma.mode = 1;
  ma.nout = G;
  ma.pbb = ma.pbp = -1;
  return multi_impl(pp, A, lda, gammas, gammas, ldg, ma, out, err_est, o, (hipStream_t)stream);
}

int64_t lhaf_saved_count(int32_t B, const int64_t* idx_off, const int32_t* r, const lh_opts* opts) {
  lh_opts o;
  lh_status s = validate_opts(opts, o);
  if (s != LH_OK) return -s;
  std::vector<ProblemIn> pin;
  s = parse_problems(B, idx_off, r, 0, 0, pin);
  if (s != LH_OK) return -s;
  int64_t tot = 0;
  for (auto& pi : pin) {
    Prob P;
    if (!fill_prob(pi.plan, o.sum, o.term_begin, o.term_end, true, &P)) return -LH_ESIZE;
    if (P.n > 0) tot += (P.t1 - P.t0) * P.n;
  }
  return tot;
}

int64_t lhaf_grads_count(int32_t B, const int64_t* idx_off, const int32_t* r) {
  std::vector<ProblemIn> pin;
  lh_status s = parse_problems(B, idx_off, r, 0, 0, pin);
  if (s != LH_OK) return -s;
  int64_t tot = 0;
  for (auto& pi : pin) {
    Prob P;
    if (!fill_prob(pi.plan, LH_SUM_FDS, 0, -1, true, &P)) return -LH_ESIZE;
    tot += (int64_t)bwd_item_elems(P.B);
  }
  return tot;
}

size_t lhaf_backward_workspace(int32_t B, const int64_t* idx_off, const int32_t* r,
                               int32_t base_dim, const lh_opts* opts) {
  lh_opts o;
  if (validate_opts(opts, o) != LH_OK) return 0;
  size_t need = 0;
  if (backward_impl(B, nullptr, 1, 0, nullptr, 0, nullptr, idx_off, r, nullptr, nullptr, nullptr,
                    base_dim, false, nullptr, nullptr, nullptr, 0, o, nullptr, true, &need) != LH_OK)
    return 0;
  return need;
}

lh_status lhaf_backward(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                        const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                        const int64_t* idx_off, const int32_t* r, const lh_c128* grad_out,
                        lh_c128* dA, lh_c128* dgamma, int32_t base_dim, void* workspace,
                        size_t ws_bytes, const lh_opts* opts, void* stream) {
  lh_opts o;
  lh_status s = validate_opts(opts, o);
  if (s != LH_OK) return s;
  return backward_impl(B, A_base, lda, stride_A, gamma_base, stride_g, idx, idx_off, r, grad_out,
                       dA, dgamma, base_dim, false, nullptr, nullptr, workspace, ws_bytes, o,
                       (hipStream_t)stream, false, nullptr);
}

}  // extern "C"
