// Step launchers, one translation unit per storage precision (they compile in parallel).
// StepArgs carries what a launch needs from the lattice: the compile-time shell set, the
// tiling and the device work list.
#pragma once
#include <hip/hip_runtime.h>

#include "scl_common.hpp"

namespace scl {

struct StepArgs {
  int set;        // compile-time shell set index
  int strip;      // 2D: output lanes per workgroup in use
  int tile2;      // 2D: 0 = marching strips; 256 or 512 = one-shot 64 x tile_ty tiles, that many lanes
  int tile_ty;    // 2D tiles: rows per tile
  int tile_tx;    // 2D tiles: columns per tile (64 or 128)
  int cpl;        // 2D: sites per lane
  int tile3;      // 3D: tile index in use (1: 64x4, 2: 64x8, 3: 32x8)
  int nitems;
  const DomDev* doms;
  const WorkItem* items;
  hipStream_t stream;
  // 3D psi pass: one launch per domain over its sites
  int ndom;
  const DomDev* hdoms;  // host copies of the domain parameters
  void* psi;            // psi of every site (arithmetic precision)
};

// One 2D step from fin into fout; rec: record n, j, F of every site (adjoint recomputation).
template <class S, class M, bool SHIFT>
hipError_t launch_step2d(const StepArgs& a, const void* fin, void* fout, MacroRec<M> rec, bool record);
// One 2D step over one-shot tiles (no recording).
template <class S, class M, bool SHIFT>
hipError_t launch_tile2d(const StepArgs& a, const void* fin, void* fout);
// One 3D step (psi pass, then the fused pass) from fin into fout.
template <class S, class M, bool SHIFT>
hipError_t launch_step3d(const StepArgs& a, const void* fin, void* fout);

}  // namespace scl
