// Host-side launchers of the persistent (register-tile templated) kernels.
// Each instantiation lives in its own translation unit (lhaf_tile.hip built
// once per kernel family and tile), so the library compiles in parallel; the
// API layer only sees these declarations.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include "lhaf_device.h"
#include "lhaf_internal.h"

namespace lh {

struct MultiArgs;  // lhaf_multi.hip

// Arguments shared by every persistent launch: the plan tables in the
// workspace, the work counter, the packed problems and the launch shape.
struct PersistArgs {
  const Prob* probs;
  const Item* items;
  int n_items;
  int* counter;
  int nmax;
  int grid;
  size_t lds;
  hipStream_t stream;
};

// forward_kernel<B, et>: item partials (and the per-term coefficient store);
// et selects the ET instance (per-term tiles with pair deletion), which
// evaluates only the terms whose reduced tile lies in [tlo, thi]
template <int B>
hipError_t launch_forward(const PersistArgs& a, const cd* ws, Partial* parts, int acc_dd,
                          cd* saved, int et, int tlo, int thi);
// forward_comp_kernel<B, et>: the same with compensated recurrences
template <int B>
hipError_t launch_forward_comp(const PersistArgs& a, const cd* ws, Partial* parts, int acc_dd,
                               cd* saved, int et, int tlo, int thi);
// backward_kernel<B>: item gradient slots; per-wavefront scratch; with
// `parts` (fused pass) also the item partials of the value
template <int B, bool kStg>
hipError_t launch_backward_as(const PersistArgs& a, const cd* ws, cd* gslots, cd* scratch,
                              const cd* saved, Partial* parts, int acc_dd);
// multi_kernel<B, MODE>: MODE 0 chain-rule outputs, 1 loop-weight vectors
template <int B, int MODE>
hipError_t launch_multi(const PersistArgs& a, const cd* ws, Partial* parts, int acc_dd,
                        const MultiArgs& ma);
// real::real_kernel<B>
template <int B>
hipError_t launch_real(const PersistArgs& a, const double* ws, Partial* parts, int acc_dd);

// Resident workgroups per CU of one instance with `lds` bytes of dynamic LDS
// (occupancy query of the runtime; 0 if the query fails).
template <int B>
int resident_forward(size_t lds, int et);
template <int B>
int resident_forward_comp(size_t lds, int et);
template <int B, bool kStg>
int resident_backward_as(size_t lds);
#if defined(LH_STAGE_MAX_B) && defined(LH_STAGE_RECOMPUTE_MAX_B)
// the instance bwd_staged selected (only existing instances are referenced)
template <int B>
inline hipError_t launch_backward(const PersistArgs& a, const cd* ws, cd* gslots, cd* scratch,
                                  const cd* saved, Partial* parts, int acc_dd, int staged) {
  if constexpr (B <= LH_STAGE_MAX_B) {
    if (staged) return launch_backward_as<B, true>(a, ws, gslots, scratch, saved, parts, acc_dd);
  }
  if constexpr (B > LH_STAGE_RECOMPUTE_MAX_B) {
    if (!staged) return launch_backward_as<B, false>(a, ws, gslots, scratch, saved, parts, acc_dd);
  }
  return hipErrorInvalidValue;
}
template <int B>
inline int resident_backward(size_t lds, int staged) {
  if constexpr (B <= LH_STAGE_MAX_B) {
    if (staged) return resident_backward_as<B, true>(lds);
  }
  if constexpr (B > LH_STAGE_RECOMPUTE_MAX_B) {
    if (!staged) return resident_backward_as<B, false>(lds);
  }
  return 0;
}
#endif

}  // namespace lh
