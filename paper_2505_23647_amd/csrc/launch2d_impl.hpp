// Body of the 2D step launcher; each k2d_*.hip instantiates it for one storage precision.
#pragma once
#include <type_traits>

#include "launch.hpp"
#include "step2d.hpp"
#include "tile2d.hpp"

namespace scl {

template <class S, class M, bool SHIFT>
hipError_t launch_step2d(const StepArgs& a, const void* fin, void* fout, MacroRec<M> rec, bool record) {
  // eight XCDs: the kernel maps workgroup id -> item so that each XCD takes a contiguous
  // eighth of the list; round the grid up to a multiple of 8
  const int per = (a.nitems + 7) / 8;
  const dim3 grid(8 * per);
#define SCL_2D_CASE(SETV, NOV, CPLV)                                                                  \
  if (a.set == SETV && a.strip == NOV && a.cpl == CPLV) {                                              \
    if constexpr (!std::is_same<S, _Float16>::value) {                                                 \
      if (record) {                                                                                    \
        hipLaunchKernelGGL((k_step2d<S, M, SETV, NOV, CPLV, SHIFT, true>), grid, dim3(NOV), 0, a.stream, \
                           (const S*)fin, (S*)fout, a.doms, a.items, a.nitems, rec);                   \
        return hipGetLastError();                                                                      \
      }                                                                                                \
    }                                                                                                  \
    hipLaunchKernelGGL((k_step2d<S, M, SETV, NOV, CPLV, SHIFT, false>), grid, dim3(NOV), 0, a.stream,  \
                       (const S*)fin, (S*)fout, a.doms, a.items, a.nitems, rec);                       \
    return hipGetLastError();                                                                          \
  }
  SCL_2D_CASE(0, 64, 1) SCL_2D_CASE(0, 128, 1) SCL_2D_CASE(0, 256, 1)
  SCL_2D_CASE(1, 64, 1) SCL_2D_CASE(1, 128, 1) SCL_2D_CASE(1, 256, 1)
  SCL_2D_CASE(0, 64, 2) SCL_2D_CASE(0, 128, 2) SCL_2D_CASE(0, 256, 2)
  SCL_2D_CASE(1, 64, 2) SCL_2D_CASE(1, 128, 2) SCL_2D_CASE(1, 256, 2)
  SCL_2D_CASE(2, 128, 1) SCL_2D_CASE(2, 256, 1)
  SCL_2D_CASE(0, 512, 1) SCL_2D_CASE(1, 512, 1)
#undef SCL_2D_CASE
  return hipErrorInvalidValue;
}

template <class S, class M, bool SHIFT>
hipError_t launch_tile2d(const StepArgs& a, const void* fin, void* fout) {
  const int per = (a.nitems + 7) / 8;
  const dim3 grid(8 * per);
#define SCL_T2_CASE(SETV, TXV, TYV, NWV)                                                              \
  if (a.set == SETV && a.tile_tx == TXV && a.tile_ty == TYV && a.tile2 == 64 * NWV) {                \
    hipLaunchKernelGGL((k_tile2d<S, M, SETV, TXV, TYV, NWV, SHIFT>), grid, dim3(64 * NWV), 0, a.stream, \
                       (const S*)fin, (S*)fout, a.doms, a.items, a.nitems);                          \
    return hipGetLastError();                                                                        \
  }
#define SCL_T2_SET(SETV)                                                                                  \
  SCL_T2_CASE(SETV, 64, 8, 4) SCL_T2_CASE(SETV, 64, 16, 4) SCL_T2_CASE(SETV, 64, 24, 4)                    \
  SCL_T2_CASE(SETV, 64, 32, 4) SCL_T2_CASE(SETV, 64, 16, 8) SCL_T2_CASE(SETV, 64, 24, 8)                   \
  SCL_T2_CASE(SETV, 64, 32, 8) SCL_T2_CASE(SETV, 128, 8, 4) SCL_T2_CASE(SETV, 128, 16, 4)                  \
  SCL_T2_CASE(SETV, 128, 24, 4) SCL_T2_CASE(SETV, 128, 32, 4) SCL_T2_CASE(SETV, 128, 16, 8)                \
  SCL_T2_CASE(SETV, 128, 24, 8) SCL_T2_CASE(SETV, 128, 32, 8)
  SCL_T2_SET(0) SCL_T2_SET(1) SCL_T2_SET(2)
#undef SCL_T2_SET
#undef SCL_T2_CASE
  return hipErrorInvalidValue;
}

}  // namespace scl
