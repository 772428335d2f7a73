// One register tile of one persistent-kernel family, as its own translation
// unit.  Built once per (LH_FAMILY, LH_TILE):
//   LH_FAMILY 0 forward_kernel<LH_TILE, ET and FDS> (+ occupancy query)
//   LH_FAMILY 1 backward_kernel<LH_TILE> (+ occupancy query)
//   LH_FAMILY 2 multi_kernel<LH_TILE, 0 and 1>
//   LH_FAMILY 3 real::real_kernel<LH_TILE>
//   LH_FAMILY 4 forward_comp_kernel<LH_TILE, ET and FDS> (+ occupancy query)
#include <hip/hip_runtime.h>

#ifndef LH_TILE
#error "LH_TILE (register tile 1..8) must be defined"
#endif
#ifndef LH_FAMILY
#error "LH_FAMILY (0 forward, 1 backward, 2 multi, 3 real, 4 compensated forward) must be defined"
#endif

// Code-generation choices of the wavefront reductions and the Hessenberg
// update, per tile (measured on MI355X, M terms/s, defaults vs the
// alternative): copy-free DPP moves and the paired complex column sum win up
// to tile 7 (forward N = 40: 15.4 vs 14.5 / 15.1, N = 52: 5.26 vs 4.97 /
// 5.14); at tile 8 the register file is full and the forward is fastest with
// neither and the two-step conjugate update (3.03 vs 2.24); the tile-7
// gradient pass is fastest with the in-place DPP moves (0.89 vs 0.69).
#ifndef LH_DPP_BOUND
#define LH_DPP_BOUND (LH_TILE <= 6 || (LH_TILE == 7 && LH_FAMILY != 1))
#endif
#ifndef LH_COL_PAIR
#define LH_COL_PAIR (LH_TILE <= 7)
#endif
#ifndef LH_FUSED_CONJ_UPDATE
#define LH_FUSED_CONJ_UPDATE (LH_TILE <= 7)
#endif

#include "lhaf.h"
#include "lhaf_device.h"
#include "lhaf_internal.h"
#include "lhaf_forward.hip"
#if LH_FAMILY == 1
#include "lhaf_backward.hip"
#elif LH_FAMILY == 2
#include "lhaf_multi.hip"
#elif LH_FAMILY == 3
#include "lhaf_real.hip"
#endif
#include "lhaf_launch.h"

namespace lh {

// Each unit defines the launcher templates of its family and instantiates
// them for its tile only; the API unit sees the declarations of
// lhaf_launch.h and links against these instantiations.
#if LH_FAMILY == 0
template <int B>
hipError_t launch_forward(const PersistArgs& a, const cd* ws, Partial* parts, int acc_dd,
                          cd* saved, int et, int tlo, int thi) {
  if (et)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(forward_kernel<B, true>), dim3(a.grid), dim3(64), a.lds,
                       a.stream, a.probs, a.items, a.n_items, a.counter, ws, parts, acc_dd, a.nmax,
                       saved, tlo, thi);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(forward_kernel<B, false>), dim3(a.grid), dim3(64), a.lds,
                       a.stream, a.probs, a.items, a.n_items, a.counter, ws, parts, acc_dd, a.nmax,
                       saved, 1, 8);
  return hipGetLastError();
}
template <int B>
int resident_forward(size_t lds, int et) {
  int blocks = 0;
  const void* fn = et ? reinterpret_cast<const void*>(&forward_kernel<B, true>)
                      : reinterpret_cast<const void*>(&forward_kernel<B, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, 64, lds) != hipSuccess) return 0;
  return blocks;
}
template hipError_t launch_forward<LH_TILE>(const PersistArgs&, const cd*, Partial*, int, cd*,
                                            int, int, int);
template int resident_forward<LH_TILE>(size_t, int);
#elif LH_FAMILY == 1
// LH_BWD_UNIT: 0 every instance of the tile, 1 the LDS-staged one only, 2 the
// unstaged one only (bwd_staged selects between them at launch)
#ifndef LH_BWD_UNIT
#define LH_BWD_UNIT 0
#endif
template <int B, bool kStg>
hipError_t launch_backward_as(const PersistArgs& a, const cd* ws, cd* gslots, cd* scratch,
                              const cd* saved, Partial* parts, int acc_dd) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(backward_kernel<B, kStg>), dim3(a.grid), dim3(64), a.lds,
                     a.stream, a.probs, a.items, a.n_items, a.counter, ws, gslots, scratch, a.nmax,
                     saved, parts, acc_dd);
  return hipGetLastError();
}
template <int B, bool kStg>
int resident_backward_as(size_t lds) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, reinterpret_cast<const void*>(&backward_kernel<B, kStg>), 64, lds) !=
      hipSuccess)
    return 0;
  return blocks;
}
#if LH_BWD_UNIT != 2 && LH_TILE <= LH_STAGE_MAX_B
template hipError_t launch_backward_as<LH_TILE, true>(const PersistArgs&, const cd*, cd*, cd*,
                                                      const cd*, Partial*, int);
template int resident_backward_as<LH_TILE, true>(size_t);
#endif
#if LH_BWD_UNIT != 1 && LH_TILE > LH_STAGE_RECOMPUTE_MAX_B
template hipError_t launch_backward_as<LH_TILE, false>(const PersistArgs&, const cd*, cd*, cd*,
                                                       const cd*, Partial*, int);
template int resident_backward_as<LH_TILE, false>(size_t);
#endif
#elif LH_FAMILY == 2
template <int B, int MODE>
hipError_t launch_multi(const PersistArgs& a, const cd* ws, Partial* parts, int acc_dd,
                        const MultiArgs& ma) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(multi_kernel<B, MODE>), dim3(a.grid), dim3(64), a.lds,
                     a.stream, a.probs, a.items, a.n_items, a.counter, ws, parts, acc_dd, a.nmax,
                     ma);
  return hipGetLastError();
}
template hipError_t launch_multi<LH_TILE, 0>(const PersistArgs&, const cd*, Partial*, int,
                                             const MultiArgs&);
template hipError_t launch_multi<LH_TILE, 1>(const PersistArgs&, const cd*, Partial*, int,
                                             const MultiArgs&);
#elif LH_FAMILY == 3
template <int B>
hipError_t launch_real(const PersistArgs& a, const double* ws, Partial* parts, int acc_dd) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(real::real_kernel<B>), dim3(a.grid), dim3(64), a.lds,
                     a.stream, a.probs, a.items, a.n_items, a.counter, ws, parts, acc_dd, a.nmax);
  return hipGetLastError();
}
template hipError_t launch_real<LH_TILE>(const PersistArgs&, const double*, Partial*, int);
#elif LH_FAMILY == 4
template <int B>
hipError_t launch_forward_comp(const PersistArgs& a, const cd* ws, Partial* parts, int acc_dd,
                               cd* saved, int et, int tlo, int thi) {
  if (et)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(forward_comp_kernel<B, true>), dim3(a.grid), dim3(64),
                       a.lds, a.stream, a.probs, a.items, a.n_items, a.counter, ws, parts, acc_dd,
                       a.nmax, saved, tlo, thi);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(forward_comp_kernel<B, false>), dim3(a.grid), dim3(64),
                       a.lds, a.stream, a.probs, a.items, a.n_items, a.counter, ws, parts, acc_dd,
                       a.nmax, saved, 1, 8);
  return hipGetLastError();
}
template <int B>
int resident_forward_comp(size_t lds, int et) {
  int blocks = 0;
  const void* fn = et ? reinterpret_cast<const void*>(&forward_comp_kernel<B, true>)
                      : reinterpret_cast<const void*>(&forward_comp_kernel<B, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, 64, lds) != hipSuccess) return 0;
  return blocks;
}
template hipError_t launch_forward_comp<LH_TILE>(const PersistArgs&, const cd*, Partial*, int,
                                                 cd*, int, int, int);
template int resident_forward_comp<LH_TILE>(size_t, int);
#endif

}  // namespace lh
