// Body of the 3D step launcher; each k3d_*.hip instantiates it for one storage precision.
#pragma once
#include "launch.hpp"
#include "step3d.hpp"

namespace scl {

template <class S, class M, bool SHIFT>
hipError_t launch_step3d(const StepArgs& a, const void* fin, void* fout) {
  // pass 1: psi of every site, domain by domain
  for (int k = 0; k < a.ndom; ++k) {
    const DomDev& dd = a.hdoms[k];
    hipLaunchKernelGGL((k_psi3d<S, M, SHIFT>), dim3((dd.nx + 255) / 256, dd.ny, dd.nz), dim3(256), 0, a.stream,
                       (const S*)fin, (M*)a.psi, dd);
  }
  // pass 2: force, collision, streaming over the work items
  const int per = (a.nitems + 7) / 8;
  const dim3 grid(8 * per);
#define SCL_3D_CASE(SETV, TI, TXV, TYV)                                                          \
  if (a.set == SETV && a.tile3 == TI) {                                                            \
    hipLaunchKernelGGL((k_step3d<S, M, SETV, TXV, TYV, SHIFT>), grid, dim3(TXV * TYV), 0, a.stream, \
                       (const S*)fin, (S*)fout, (const M*)a.psi, a.doms, a.items, a.nitems);        \
    return hipGetLastError();                                                                     \
  }
  SCL_3D_CASE(0, 1, 64, 4) SCL_3D_CASE(0, 2, 64, 8) SCL_3D_CASE(0, 3, 32, 8) SCL_3D_CASE(0, 4, 128, 4)
  SCL_3D_CASE(1, 1, 64, 4) SCL_3D_CASE(1, 2, 64, 8) SCL_3D_CASE(1, 3, 32, 8) SCL_3D_CASE(1, 4, 128, 4)
  SCL_3D_CASE(2, 2, 64, 8) SCL_3D_CASE(2, 3, 32, 8)
#undef SCL_3D_CASE
  return hipErrorInvalidValue;
}

}  // namespace scl
