// libscl host side: the C ABI of include/scl.h, kernel dispatch, tiling, graphs, autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <sstream>
#include <string>
#include <array>
#include <vector>

#include "scl.h"
#include "scl_common.hpp"
#include "launch.hpp"
#include "step3d.hpp"
#include "readout.hpp"
#include "adjoint.hpp"

using namespace scl;

// row ranges of one strip handed out together in the 2D item order
#ifndef SCL_ITEM_BAND
#define SCL_ITEM_BAND 4
#endif

namespace {

thread_local std::string g_err;

scl_status fail(scl_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(SCL_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

size_t storage_bytes(scl_precision p) {
  switch (p) {
    case SCL_FP64: return 8;
    case SCL_FP32: case SCL_FP32_SHIFTED: return 4;
    case SCL_FP16S_FP32: return 2;
  }
  return 0;
}

// Shell codes of the compile-time sets (index = weight slot).
const int NSETS2 = 3, NSETS3 = 3, SETW = 12;  // sets per dimension, row width of the tables
const int SET2[NSETS2][SETW] = {{1, 2}, {1, 2, 4, 5, 8}, {1, 2, 4, 5, 8, 9, 16, 18}};
const int SET2N[NSETS2] = {2, 5, 8};
const int SET3[NSETS3][SETW] = {{1, 2, 3}, {1, 2, 3, 4, 5, 6, 8}, {1, 2, 3, 4, 5, 6, 8, 9, 1009, 16, 18}};
const int SET3N[NSETS3] = {3, 7, 11};

// Device memory: from the hook installed by scl_set_allocator when there is one, else from
// hipMalloc. A lattice keeps the hook that was installed when it was created.
struct AllocHook {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*free_)(void*, void*, void*) = nullptr;
  void* ctx = nullptr;
};
AllocHook g_hook;

// 3D tile shapes selectable through scl_set_tiling(strip = index).
struct Tile3 { int tx, ty; };
const Tile3 TILES3[5] = {{0, 0}, {64, 4}, {64, 8}, {32, 8}, {128, 4}};

}  // namespace

struct scl_lattice_s {
  scl_velset vs;
  scl_precision prec;
  int d, Q;
  int ndom;
  std::vector<int> nx, ny, nz;
  std::vector<long long> off;
  long long cells = 0;
  hipStream_t stream = nullptr;    // caller's stream (may be the null stream)
  hipStream_t launch = nullptr;    // stream the step kernels go to (the capture stream while capturing)
  hipStream_t cap = nullptr;       // private stream used only to capture graphs
  AllocHook hook;     // device memory source (scl_set_allocator at creation)
  void* A = nullptr;  // current state (post-collision values, pull layout)
  void* B = nullptr;  // scratch for the next state
  // physics
  bool have_physics = false, have_stencil = false, have_state = false;
  std::vector<double> tau, G, psi_param, rho0;
  std::vector<double> aF;          // A of the F^2 part of the Guo tensor (0: the paper's T = 2uF)
  int psi_kind = 0;
  int set = 1;                     // compile-time shell set
  std::vector<int> user_codes;     // as given
  std::vector<int> slot_of_user;   // user shell -> set slot
  std::vector<double> Wslot;       // ndom x MAX_SHELLS
  // device tables
  DomDev* d_doms = nullptr;
  WorkItem* d_items = nullptr;
  int nitems = 0;
  bool dirty_doms = true, dirty_items = true;
  // tiling
  int strip = 0, seg = 0;          // 2D: output lanes per workgroup, rows per item (0 = auto)
  int strip_eff = 256;             // 2D: output lanes per workgroup in use
  int tile2 = 0, tile_ty = 16;     // 2D: one-shot tiles requested (lanes, rows; 0 = none)
  int tile_tx = 64;                // 2D: tile width requested (64 or 128 columns)
  int tile2_eff = 0;               // 2D: tiles in use (lanes; 0 = marching strips)
  int tile_ty_eff = 16;            // 2D: rows per tile in use
  int tile_tx_eff = 64;            // 2D: tile width in use
  bool march_only = false;         // 2D: tiles switched off (the adjoint's recording pass)
  int cpl_req = 0;                 // 2D: sites per lane requested (0 = auto)
  int cpl = 1;                     // 2D: sites per lane in use
  int tile3 = 0, seg3 = 0;         // 3D: tile index, planes per item (0 = auto)
  int tile3_eff = 2;               // 3D: tile index in use
  // graphs
  int graph_k = 0;
  hipGraphExec_t gexec = nullptr;
  void* gexec_A = nullptr;         // buffer that was "A" when the graph was captured
  // readout scratch (double)
  double *d_n = nullptr, *d_psi = nullptr, *d_j = nullptr, *d_F = nullptr, *d_tmp = nullptr;
  double* d_part = nullptr;
  void* d_psi3 = nullptr;          // 3D: psi of every site (arithmetic precision), pass 1 -> pass 2
  std::vector<DomDev> h_doms;      // host copy of d_doms
  size_t part_cap = 0;
  int64_t steps = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // adjoint state
  AdjointState adj;
};

namespace {

hipError_t dmalloc(const scl_lattice_s* L, void** p, size_t bytes) {
  if (!L->hook.alloc) return hipMalloc(p, bytes);
  *p = bytes ? L->hook.alloc(bytes, L->hook.ctx, (void*)L->stream) : nullptr;
  return (*p || !bytes) ? hipSuccess : hipErrorOutOfMemory;
}
template <class T> hipError_t dmalloc(const scl_lattice_s* L, T** p, size_t bytes) {
  void* v = nullptr;
  const hipError_t e = dmalloc(L, &v, bytes);
  *p = static_cast<T*>(v);
  return e;
}
// Stream-ordered release: the memory may be handed out again for later work on the lattice's
// stream (every kernel and copy of the library runs on that stream or is synchronised first).
hipError_t dfree(const scl_lattice_s* L, void* p) {
  if (!p) return hipSuccess;
  if (!L->hook.alloc) return hipFree(p);
  L->hook.free_(p, L->hook.ctx, (void*)L->stream);
  return hipSuccess;
}

void adjoint_free(const scl_lattice_s* L, AdjointState& a) {
  void* ps[] = {a.pool, a.rec, a.lam[0], a.lam[1], a.gpart};
  for (void* p : ps) (void)dfree(L, p);
  a = AdjointState();
}

std::vector<DomDev> host_doms(const scl_lattice_s* L) {
  std::vector<DomDev> v(L->ndom);
  for (int k = 0; k < L->ndom; ++k) {
    DomDev& d = v[k];
    std::memset(&d, 0, sizeof(d));
    d.off = L->off[k];
    d.nx = L->nx[k]; d.ny = L->ny[k]; d.nz = L->nz[k];
    d.psi_kind = L->psi_kind;
    d.omega = 1.0 / L->tau[k];
    d.kappa = 1.0 - 0.5 / L->tau[k];
    d.gpre = -L->G[k] * CS2;
    d.eps = L->psi_param[k];
    d.inv_eps = L->psi_param[k] != 0.0 ? 1.0 / L->psi_param[k] : 0.0;
    d.rho0 = L->rho0[k];
    d.aff = L->aF[k] / L->tau[k];
    for (int s = 0; s < MAX_SHELLS; ++s) d.W[s] = L->Wslot[(size_t)k * MAX_SHELLS + s];
  }
  return v;
}

int stencil_reach(const scl_lattice_s* L) { return L->set == 0 ? 1 : (L->set == 1 ? 2 : 4); }

// All forcing vectors (both of every pair) of the lattice's compile-time set.
VecTable full_table(const scl_lattice_s* L) {
  VecTable t{};
  t.n = 0;
  if (L->d == 2) {
    auto add = [&](auto sh_tag) {
      using SH = decltype(sh_tag);
      for (int k = 0; k < SH::NH; ++k) {
        HalfVec h = SH::h(k);
        t.v[t.n++] = h;
        t.v[t.n++] = HalfVec{(int8_t)-h.x, (int8_t)-h.y, (int8_t)-h.z, h.slot};
      }
    };
    if (L->set == 0) add(Shells<2, 0>{});
    else if (L->set == 1) add(Shells<2, 1>{});
    else add(Shells<2, 2>{});
  } else {
    Half3Table h = make_half3(L->set);
    for (int k = 0; k < h.n; ++k) {
      t.v[t.n++] = h.v[k];
      t.v[t.n++] = HalfVec{(int8_t)-h.v[k].x, (int8_t)-h.v[k].y, (int8_t)-h.v[k].z, h.v[k].slot};
    }
  }
  return t;
}

bool planes_fit_tiles(const scl_lattice_s* L) {
  for (int k = 0; k < L->ndom; ++k)
    if ((long long)L->nx[k] * L->ny[k] * (long long)storage_bytes(L->prec) >= (1LL << 31)) return false;
  return true;
}

// Sites of 2D marching strips w lanes wide (cpl sites per lane) that lie past a domain's width.
long long strip_idle(const scl_lattice_s* L, int w, int cpl) {
  long long idle = 0;
  for (int k = 0; k < L->ndom; ++k) {
    const long long ow = (long long)w * cpl;
    idle += ((L->nx[k] + ow - 1) / ow * ow - L->nx[k]) * (long long)L->ny[k];
  }
  return idle;
}

// Automatic 2D strip: measured best on MI355X (4096^2, 24 vectors): 512 output lanes for 4-byte
// storage, 256 for FP64; 256 for the reach-4 set (larger ring and register sets). Narrow
// domains take narrower strips: the widest whose idle lanes (strip columns past a domain's
// width) stay under half the sites.
int auto_strip(const scl_lattice_s* L, int cpl) {
  int w = (storage_bytes(L->prec) == 4 && L->set != 2 && cpl == 1) ? 512 : 256;
  for (; w > 128; w /= 2)
    if (strip_idle(L, w, cpl) * 2 <= L->cells) break;
  return w;
}

scl_status build_items(scl_lattice_s* L) {
  std::vector<WorkItem> items;
  // 2D tiles: as requested, or automatically (no tiling asked for, shell sets of reach 1 and 2)
  //  * for FP64 storage: measured on MI355X, 4096^2, 24 vectors, 256-lane tiles of 128 x 8
  //    sites take 0.437 ms per step (64 x 16: 0.444) against 0.507 ms for the best marching
  //    strips;
  //  * for domains narrow enough that the automatic strips leave more than 1/8 of their lanes
  //    idle: the 64 droplet and bubble domains of sides 64..544 run 48.5 GLUPS on 512-lane
  //    tiles of 64 x 16 sites against 43.2 on 256-lane strips (30% idle lanes), FP32 shifted;
  //  * for FP16 storage: 256-lane tiles of 128 x 16 sites, 0.148 ms per step against 0.157 for
  //    the best marching strips (for FP32 storage the strips stay faster: 0.234 against 0.244
  //    for the best tiles).
  L->tile2_eff = 0;
  if (L->d == 2 && !L->march_only) {
    const bool asked = L->strip || L->seg || L->cpl_req;
    if (L->tile2) {
      L->tile2_eff = L->tile2;
      L->tile_ty_eff = L->tile_ty;
      L->tile_tx_eff = L->tile_tx;
    } else if (!asked && L->set != 2 && planes_fit_tiles(L)) {
      if (L->prec == SCL_FP64) {
        L->tile2_eff = 256;
        L->tile_ty_eff = 8;
        L->tile_tx_eff = 128;
      } else if (strip_idle(L, auto_strip(L, 1), 1) * 8 > L->cells) {
        L->tile2_eff = 512;
        L->tile_ty_eff = 16;
        L->tile_tx_eff = 64;
      } else if (L->prec == SCL_FP16S_FP32) {
        L->tile2_eff = 256;
        L->tile_ty_eff = 16;
        L->tile_tx_eff = 128;
      }
    }
  }
  if (L->tile2_eff) {
    L->cpl = 1;
    // one-shot tiles of tile_tx x tile_ty sites. Order: within each domain, column blocks of
    // 64 CB sites, each taken row by row. Each XCD takes a contiguous eighth of the list, and the
    // tile above a tile was loaded a block's width of tiles earlier, so the rim rows two tiles
    // share still sit in that XCD's L2. Row-major order over a 4096-wide domain (64 tiles per
    // row) let 256-lane FP32 tiles fetch 1.39x the populations they need. Measured on MI355X
    // (4096^2, 24 vectors, CB of 2, 4, 8, 16, 32, 64): FP64, 256-lane 64 x 16 tiles, 0.444 ms
    // per step at CB = 16 against 0.484 at 64 and 0.457 at 8; FP32, 512-lane 64 x 24 tiles,
    // 0.244 ms at CB = 8 against 0.252-0.253 at 16-64.
    const int CB = storage_bytes(L->prec) == 8 ? 16 : 8;
    for (int k = 0; k < L->ndom; ++k)
      for (int b0 = 0; b0 < L->nx[k]; b0 += 64 * CB)
        for (int y0 = 0; y0 < L->ny[k]; y0 += L->tile_ty_eff)
          for (int x0 = b0; x0 < std::min(b0 + 64 * CB, L->nx[k]); x0 += L->tile_tx_eff) {
            WorkItem w{};
            w.dom = k; w.x0 = x0; w.y0 = y0; w.y1 = std::min(y0 + L->tile_ty_eff, L->ny[k]);
            w.z0 = 0; w.z1 = 1; w.dir = 1;
            items.push_back(w);
          }
  } else if (L->d == 2) {
    // sites per lane (two need every domain width even)
    bool even = true;
    for (int k = 0; k < L->ndom; ++k) even = even && (L->nx[k] % 2 == 0);
    // automatic: one site per lane. Measured on MI355X (4096^2, 24-vector stencil) two sites
    // per lane lose to it: the shifted 8-byte pulls are unaligned and the extra registers
    // cut occupancy to 3 waves per SIMD.
    L->cpl = L->cpl_req ? L->cpl_req : 1;
    if (L->cpl == 2 && !even) return fail(SCL_E_INVALID, "two sites per lane need even domain widths");
    // output lanes per workgroup (64 domains 64..544 wide: 256-lane strips, 30% idle lanes,
    // run 7% faster than 128-lane strips with 18%; 512 lanes, 46% idle, lose)
    L->strip_eff = L->strip ? L->strip : auto_strip(L, L->cpl);
    const int outw = L->strip_eff * L->cpl;
    // rows per item: measured best on MI355X (4096^2, 24 vectors): 64 for 4- and 2-byte
    // storage, 32 for FP64. At 4096^2 with 512-lane strips, 64 rows make 512 items, exactly one
    // round of the 512 workgroups resident on the chip (0.236 ms per FP32 step, against 0.241
    // for 32 rows, two rounds); 24, 28, 36 or 40 rows leave a partial round and lose 7-14%.
    // Lattices too small to give 512 items at that height take lower ranges, down to 16 rows,
    // so that every CU still gets work.
    int seg = L->seg;
    if (seg <= 0) {
      seg = storage_bytes(L->prec) == 8 ? 32 : 64;
      auto nitems_at = [&](int sg) {
        long long n = 0;
        for (int k = 0; k < L->ndom; ++k)
          n += (long long)((L->nx[k] + outw - 1) / outw) * ((L->ny[k] + sg - 1) / sg);
        return n;
      };
      while (seg > 16 && nitems_at(seg) < 512) seg /= 2;
    }
    // Order: bands of BAND row ranges; within a band, strip by strip, the ranges of the band
    // in order. The device hands each XCD a contiguous eighth of this list, so an XCD works on
    // a compact block of neighbouring strips and ranges whose shared halos meet in its L2.
    // Consecutive ranges of a strip march in opposite directions. Bands of 4 ranges: at 4096^2
    // with 512-lane strips and 64 rows, 0.236 ms per FP32 step against 0.246 for bands of 8 and
    // 0.237 for whole strips (one strip per XCD).
    const int BAND = SCL_ITEM_BAND;
    for (int k = 0; k < L->ndom; ++k) {
      const int ns = (L->nx[k] + outw - 1) / outw;
      const int nseg = (L->ny[k] + seg - 1) / seg;
      for (int b0 = 0; b0 < nseg; b0 += BAND)
        for (int sx = 0; sx < ns; ++sx)
          for (int sg = b0; sg < std::min(b0 + BAND, nseg); ++sg) {
            WorkItem w{};
            w.dom = k; w.x0 = sx * outw; w.y0 = sg * seg; w.y1 = std::min((sg + 1) * seg, L->ny[k]);
            w.z0 = 0; w.z1 = 1;
            w.dir = (sg % 2 == 0) ? 1 : -1;
            items.push_back(w);
          }
    }
  } else {
    // automatic tile: measured best on MI355X (512^3, 92 vectors): 128x4 for 4-byte storage
    // (6.08 ms per step against 6.28 for 64x8: the x-shifted pulls of a wider tile touch
    // fewer extra cache lines), 64x8 for FP64, 64x4 for FP16 storage (4.13 ms against 4.36 for
    // 128x4); 64x8 for the reach-4 set
    L->tile3_eff = L->tile3 ? L->tile3
                            : (L->set == 2 ? 2 : (L->prec == SCL_FP16S_FP32 ? 1 : (storage_bytes(L->prec) == 4 ? 4 : 2)));
    const Tile3 t = TILES3[L->tile3_eff];
    const int ox = t.tx, oy = t.ty;
    int seg = L->seg3;
    if (seg <= 0) {
      long long work = 0;
      for (int k = 0; k < L->ndom; ++k)
        work += (long long)((L->nx[k] + ox - 1) / ox) * ((L->ny[k] + oy - 1) / oy) * L->nz[k];
      seg = (int)std::max<long long>(16, (work + 2047) / 2048);
    }
    // Order: tile by tile (x fastest), the z-ranges of a tile together, alternating their
    // marching direction, so that neighbouring tiles and ranges land on the same XCD.
    for (int k = 0; k < L->ndom; ++k) {
      const int nzr = (L->nz[k] + seg - 1) / seg;
      for (int y0 = 0; y0 < L->ny[k]; y0 += oy)
        for (int x0 = 0; x0 < L->nx[k]; x0 += ox)
          for (int zr = 0; zr < nzr; ++zr) {
            WorkItem w{};
            w.dom = k; w.x0 = x0; w.y0 = y0; w.y1 = std::min(y0 + oy, L->ny[k]);
            w.z0 = zr * seg; w.z1 = std::min(zr * seg + seg, L->nz[k]);
            w.dir = (zr % 2 == 0) ? 1 : -1;
            items.push_back(w);
          }
    }
  }
  if (L->d_items) { HIPCHK(dfree(L, L->d_items)); L->d_items = nullptr; }
  HIPCHK(dmalloc(L, &L->d_items, sizeof(WorkItem) * items.size()));
  HIPCHK(hipMemcpy(L->d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
  L->nitems = (int)items.size();
  L->dirty_items = false;
  return SCL_OK;
}

scl_status sync_params(scl_lattice_s* L) {
  if (L->dirty_doms) {
    std::vector<DomDev> v = host_doms(L);
    if (!L->d_doms) HIPCHK(dmalloc(L, &L->d_doms, sizeof(DomDev) * L->ndom));
    HIPCHK(hipMemcpyAsync(L->d_doms, v.data(), sizeof(DomDev) * L->ndom, hipMemcpyHostToDevice, L->stream));
    L->h_doms = v;
    HIPCHK(hipStreamSynchronize(L->stream));
    L->dirty_doms = false;
  }
  if (L->dirty_items) {
    scl_status s = build_items(L);
    if (s != SCL_OK) return s;
  }
  return SCL_OK;
}

void drop_graph(scl_lattice_s* L) {
  if (L->gexec) { (void)hipGraphExecDestroy(L->gexec); L->gexec = nullptr; }
}

// ------------------------------------------------------------------ step dispatch
// The launchers live in k2d_*.hip / k3d_*.hip, one translation unit per storage precision.
StepArgs step_args(const scl_lattice_s* L) {
  StepArgs a{};
  a.set = L->set;
  a.strip = L->strip_eff;
  a.tile2 = L->tile2_eff;
  a.tile_ty = L->tile_ty_eff;
  a.tile_tx = L->tile_tx_eff;
  a.cpl = L->cpl;
  a.tile3 = L->tile3_eff;
  a.nitems = L->nitems;
  a.doms = L->d_doms;
  a.items = L->d_items;
  a.stream = L->launch;
  a.ndom = L->ndom;
  a.hdoms = L->h_doms.data();
  a.psi = L->d_psi3;
  return a;
}

// One step from A into B (no swap).
hipError_t launch_step(scl_lattice_s* L, const void* fin, void* fout, const MacroRec<double>* rec64,
                       const MacroRec<float>* rec32) {
  const StepArgs a = step_args(L);
  if (L->d == 2 && L->tile2_eff && !rec64 && !rec32) {
    switch (L->prec) {
      case SCL_FP64: return launch_tile2d<double, double, false>(a, fin, fout);
      case SCL_FP32: return launch_tile2d<float, float, false>(a, fin, fout);
      case SCL_FP32_SHIFTED: return launch_tile2d<float, float, true>(a, fin, fout);
      case SCL_FP16S_FP32: return launch_tile2d<_Float16, float, true>(a, fin, fout);
    }
  }
  if (L->d == 2) {
    switch (L->prec) {
      case SCL_FP64:
        return launch_step2d<double, double, false>(a, fin, fout, rec64 ? *rec64 : MacroRec<double>{}, rec64 != nullptr);
      case SCL_FP32:
        return launch_step2d<float, float, false>(a, fin, fout, rec32 ? *rec32 : MacroRec<float>{}, rec32 != nullptr);
      case SCL_FP32_SHIFTED:
        return launch_step2d<float, float, true>(a, fin, fout, rec32 ? *rec32 : MacroRec<float>{}, rec32 != nullptr);
      case SCL_FP16S_FP32:
        return launch_step2d<_Float16, float, true>(a, fin, fout, MacroRec<float>{}, false);
    }
  } else {
    switch (L->prec) {
      case SCL_FP64: return launch_step3d<double, double, false>(a, fin, fout);
      case SCL_FP32: return launch_step3d<float, float, false>(a, fin, fout);
      case SCL_FP32_SHIFTED: return launch_step3d<float, float, true>(a, fin, fout);
      case SCL_FP16S_FP32: return launch_step3d<_Float16, float, true>(a, fin, fout);
    }
  }
  return hipErrorInvalidValue;
}

scl_status ready(scl_lattice_s* L) {
  if (!L->have_physics) return fail(SCL_E_STATE, "scl_set_physics has not been called");
  if (!L->have_stencil) return fail(SCL_E_STATE, "scl_set_stencil has not been called");
  if (!L->have_state) return fail(SCL_E_STATE, "scl_init_density has not been called");
  return sync_params(L);
}

scl_status plain_steps(scl_lattice_s* L, int64_t n) {
  for (int64_t s = 0; s < n; ++s) {
    hipError_t e = launch_step(L, L->A, L->B, nullptr, nullptr);
    if (e != hipSuccess) return fail(SCL_E_DEVICE, std::string("step launch: ") + hipGetErrorString(e));
    std::swap(L->A, L->B);
    L->steps++;
  }
  return SCL_OK;
}

scl_status do_steps(scl_lattice_s* L, int64_t n) {
  scl_status s = ready(L);
  if (s != SCL_OK) return s;
  if (L->graph_k <= 0 || n < L->graph_k) return plain_steps(L, n);
  const int k = L->graph_k;
  // the graph alternates A/B k times (k even), so it is valid whenever A is the buffer it
  // was captured with.
  if (L->gexec && L->gexec_A != L->A) drop_graph(L);
  if (!L->gexec) {
    // capture on a private stream (the caller's may be the null stream, which cannot be
    // captured); the instantiated graph is then launched on the caller's stream.
    if (!L->cap) HIPCHK(hipStreamCreateWithFlags(&L->cap, hipStreamNonBlocking));
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(L->cap, hipStreamCaptureModeThreadLocal));
    L->launch = L->cap;
    void* a = L->A;
    void* b = L->B;
    for (int q = 0; q < k; ++q) {
      hipError_t e = launch_step(L, a, b, nullptr, nullptr);
      if (e != hipSuccess) {
        hipGraph_t dummy;
        (void)hipStreamEndCapture(L->cap, &dummy);
        L->launch = L->stream;
        return fail(SCL_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
      }
      std::swap(a, b);
    }
    L->launch = L->stream;
    HIPCHK(hipStreamEndCapture(L->cap, &g));
    HIPCHK(hipGraphInstantiate(&L->gexec, g, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(g));
    L->gexec_A = L->A;
  }
  int64_t done = 0;
  while (n - done >= k) {
    HIPCHK(hipGraphLaunch(L->gexec, L->stream));
    done += k;
    L->steps += k;
  }
  return plain_steps(L, n - done);
}

scl_status ensure_scratch(scl_lattice_s* L) {
  if (!L->d_n) {
    const size_t c = (size_t)L->cells;
    HIPCHK(dmalloc(L, &L->d_n, c * sizeof(double)));
    HIPCHK(dmalloc(L, &L->d_psi, c * sizeof(double)));
    HIPCHK(dmalloc(L, &L->d_j, 3 * c * sizeof(double)));
    HIPCHK(dmalloc(L, &L->d_F, 3 * c * sizeof(double)));
    HIPCHK(dmalloc(L, &L->d_tmp, (L->d == 3 ? 6 : 3) * c * sizeof(double)));
  }
  return SCL_OK;
}

inline unsigned blocks_for(long long n, int nt) { return (unsigned)((n + nt - 1) / nt); }

// n, psi, j, F of the current state into the double scratch arrays.
scl_status compute_fields(scl_lattice_s* L, bool with_force) {
  scl_status s = ready(L);
  if (s != SCL_OK) return s;
  s = ensure_scratch(L);
  if (s != SCL_OK) return s;
  std::vector<DomDev> doms = host_doms(L);
  VecTable tab = full_table(L);
  for (int k = 0; k < L->ndom; ++k) {
    const long long c = (long long)L->nx[k] * L->ny[k] * L->nz[k];
    const unsigned nb = blocks_for(c, 256);
#define FIELDS(VS, S) hipLaunchKernelGGL((k_fields<VS, S>), dim3(nb), dim3(256), 0, L->stream, (const S*)L->A, L->d_n, L->d_psi, L->d_j, L->cells, doms[k])
    if (L->vs == SCL_D2Q9) {
      if (L->prec == SCL_FP64) FIELDS(0, double);
      else if (L->prec == SCL_FP16S_FP32) FIELDS(0, _Float16);
      else FIELDS(0, float);
    } else {
      if (L->prec == SCL_FP64) FIELDS(1, double);
      else if (L->prec == SCL_FP16S_FP32) FIELDS(1, _Float16);
      else FIELDS(1, float);
    }
#undef FIELDS
    HIPCHK(hipGetLastError());
  }
  if (with_force) {
    for (int k = 0; k < L->ndom; ++k) {
      const long long c = (long long)L->nx[k] * L->ny[k] * L->nz[k];
      if (L->d == 2) hipLaunchKernelGGL(k_force<2>, dim3(blocks_for(c, 256)), dim3(256), 0, L->stream, L->d_psi, L->d_F, L->cells, doms[k], tab);
      else hipLaunchKernelGGL(k_force<3>, dim3(blocks_for(c, 256)), dim3(256), 0, L->stream, L->d_psi, L->d_F, L->cells, doms[k], tab);
      HIPCHK(hipGetLastError());
    }
  }
  return SCL_OK;
}

scl_status copy_out(scl_lattice_s* L, double* out, const double* src, size_t count, int is_dev) {
  HIPCHK(hipMemcpyAsync(out, src, count * sizeof(double), is_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  return SCL_OK;
}

// ------------------------------------------------------------------ adjoint helpers
size_t state_bytes(const scl_lattice_s* L) { return (size_t)L->Q * L->cells * storage_bytes(L->prec); }

// Work items of the adjoint kernel: 128-lane strips, 32-row ranges, same order and
// alternating directions as the forward items.
std::vector<WorkItem> adjoint_items(const scl_lattice_s* L, int NO, int seg) {
  std::vector<WorkItem> items;
  const int BAND = 8;
  for (int k = 0; k < L->ndom; ++k) {
    const int ns = (L->nx[k] + NO - 1) / NO;
    const int nseg = (L->ny[k] + seg - 1) / seg;
    for (int b0 = 0; b0 < nseg; b0 += BAND)
      for (int sx = 0; sx < ns; ++sx)
        for (int sg = b0; sg < std::min(b0 + BAND, nseg); ++sg) {
          WorkItem w{};
          w.dom = k; w.x0 = sx * NO; w.y0 = sg * seg; w.y1 = std::min((sg + 1) * seg, L->ny[k]);
          w.z0 = 0; w.z1 = 1; w.dir = (sg % 2 == 0) ? 1 : -1;
          items.push_back(w);
        }
  }
  return items;
}

// Pair terms of the d = 2 lattice pressure tensor (same construction as k_ptensor2d):
// P^{mu nu}(x) = n c^2 delta + G c^2 sum_t coef W[slot] psi(x + a) psi(x + b) e^mu e^nu.
struct PTerm { double coef; int ax, ay, bx, by, ex, ey, slot; };

std::vector<PTerm> ptensor_terms(const scl_lattice_s* L) {
  std::vector<PTerm> t;
  VecTable tab = full_table(L);
  int slot5 = -1;
  for (int q = 0; q < SET2N[L->set]; ++q)
    if (SET2[L->set][q] == 5) slot5 = q;
  for (int k = 0; k < tab.n; ++k) {
    const int ex = tab.v[k].x, ey = tab.v[k].y, sl = tab.v[k].slot;
    const int ax = std::abs(ex), ay = std::abs(ey);
    if (ax * ax + ay * ay == 5) {
      t.push_back({0.25, 0, 0, ex, ey, ex, ey, sl});
    } else {
      const int kk = std::max(ax, ay), hx = ex / kk, hy = ey / kk;
      for (int m = 0; m < kk; ++m) t.push_back({1.0 / (2.0 * kk), -m * hx, -m * hy, -m * hx + ex, -m * hy + ey, ex, ey, sl});
    }
  }
  if (slot5 >= 0) {
    const int ev[4][2] = {{2, 1}, {1, 2}, {-1, 2}, {-2, 1}};
    const int pr[4][2][4] = {{{-1, 0, 1, 1}, {-1, -1, 1, 0}}, {{-1, -1, 0, 1}, {0, -1, 1, 1}},
                             {{0, -1, -1, 1}, {1, -1, 0, 1}}, {{1, -1, -1, 0}, {1, 0, -1, 1}}};
    for (int v = 0; v < 4; ++v)
      for (int p = 0; p < 2; ++p)
        t.push_back({0.25, pr[v][p][0], pr[v][p][1], pr[v][p][2], pr[v][p][3], ev[v][0], ev[v][1], slot5});
  }
  return t;
}

// Term list of k_ptensor_terms for the lattice's stencil (every vector of both signs).
std::vector<PTermDev> ptensor_link_terms(const scl_lattice_s* L) {
  std::vector<PTermDev> out;
  VecTable tab = full_table(L);
  for (int k = 0; k < tab.n; ++k) {
    const int e[3] = {tab.v[k].x, tab.v[k].y, tab.v[k].z};
    const int K = std::max(std::abs(e[0]), std::max(std::abs(e[1]), std::abs(e[2])));
    for (int m = 0; m < K; ++m) {
      int base[3], q = 0;
      bool off[3];
      for (int i = 0; i < 3; ++i) {
        const int num = m * e[i];
        off[i] = num % K != 0;
        base[i] = (int)std::floor((double)num / K);
        q += off[i];
      }
      const double share = 1.0 / (2.0 * K) / (double)(1 << q);
      for (int bits = 0; bits < 8; ++bits) {
        bool use = true;
        for (int i = 0; i < 3; ++i) use = use && (off[i] || !((bits >> i) & 1));
        if (!use) continue;
        PTermDev t{};
        t.coef = share;
        for (int i = 0; i < 3; ++i) {
          const int ci = base[i] + ((bits >> i) & 1);
          t.a[i] = (int8_t)(-ci);
          t.b[i] = (int8_t)(-ci + e[i]);
          t.e[i] = (int8_t)e[i];
        }
        t.slot = tab.v[k].slot;
        out.push_back(t);
      }
    }
  }
  return out;
}

double psi_host(double n, int kind, double eps) {
  if (kind == 0) return std::exp(-1.0 / n);
  if (kind == 1) return std::pow(n / (eps + n), 1.0 / eps);
  return 1.0 - std::exp(-n);
}
double dpsi_host(double n, double psi, int kind, double eps) {
  if (kind == 0) return psi / (n * n);
  if (kind == 1) return psi / (n * (eps + n));
  return 1.0 - psi;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int32_t scl_abi_version(void) { return SCL_ABI_VERSION; }

const char* scl_last_error(void) { return g_err.c_str(); }

int32_t scl_velocity_set(scl_velset vs, int32_t* xi, double* w) {
  if (vs == SCL_D2Q9) {
    for (int i = 0; i < 9; ++i) {
      if (xi) { xi[3 * i] = Vel<0>::cx(i); xi[3 * i + 1] = Vel<0>::cy(i); xi[3 * i + 2] = 0; }
      if (w) w[i] = Vel<0>::w(i);
    }
    return 9;
  }
  if (vs == SCL_D3Q19) {
    for (int i = 0; i < 19; ++i) {
      if (xi) { xi[3 * i] = Vel<1>::cx(i); xi[3 * i + 1] = Vel<1>::cy(i); xi[3 * i + 2] = Vel<1>::cz(i); }
      if (w) w[i] = Vel<1>::w(i);
    }
    return 19;
  }
  return -1;
}

scl_status scl_set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_)(void*, void*, void*), void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr)) return fail(SCL_E_INVALID, "give both allocator functions, or neither");
  g_hook.alloc = alloc;
  g_hook.free_ = free_;
  g_hook.ctx = alloc ? ctx : nullptr;
  return SCL_OK;
}

scl_status scl_create(scl_velset vs, scl_precision prec, int32_t ndom, const int32_t* dims, void* hip_stream,
                      scl_lattice* out) {
  if (!out) return fail(SCL_E_INVALID, "out is NULL");
  *out = nullptr;
  if (vs != SCL_D2Q9 && vs != SCL_D3Q19) return fail(SCL_E_INVALID, "unknown velocity set");
  if (storage_bytes(prec) == 0) return fail(SCL_E_INVALID, "unknown precision");
  if (ndom < 1 || !dims) return fail(SCL_E_INVALID, "need ndom >= 1 and dims");
  std::unique_ptr<scl_lattice_s> L(new scl_lattice_s());
  L->vs = vs;
  L->prec = prec;
  L->d = vs == SCL_D2Q9 ? 2 : 3;
  L->Q = vs == SCL_D2Q9 ? 9 : 19;
  L->ndom = ndom;
  long long tot = 0;
  for (int k = 0; k < ndom; ++k) {
    const int x = dims[3 * k], y = dims[3 * k + 1], z = dims[3 * k + 2];
    if (x < 1 || y < 1 || z < 1) return fail(SCL_E_INVALID, "every extent must be >= 1");
    if (L->d == 2 && z != 1) return fail(SCL_E_INVALID, "D2Q9 domains need nz = 1");
    // the 2D step addresses a row through a buffer descriptor with 31-bit byte offsets
    if (L->d == 2 && (long long)(x + 1) * 8 >= (1ll << 31)) return fail(SCL_E_INVALID, "D2Q9 domain width too large");
    // the 3D step addresses a z-plane the same way
    if (L->d == 3 && (long long)x * y * 8 >= (1ll << 31)) return fail(SCL_E_INVALID, "D3Q19 domain x-y plane too large");
    // the 3D psi pass launches a (x chunks, ny, nz) grid
    if (L->d == 3 && (y > 65535 || z > 65535)) return fail(SCL_E_INVALID, "D3Q19 domain ny and nz must be <= 65535");
    L->nx.push_back(x); L->ny.push_back(y); L->nz.push_back(z);
    L->off.push_back(tot);
    tot += (long long)x * y * z;
  }
  L->cells = tot;
  L->stream = (hipStream_t)hip_stream;
  L->launch = L->stream;
  L->hook = g_hook;
  L->tau.assign(ndom, 1.0);
  L->G.assign(ndom, 0.0);
  L->psi_param.assign(ndom, 0.0);
  L->rho0.assign(ndom, 0.0);
  L->aF.assign(ndom, 0.0);
  L->Wslot.assign((size_t)ndom * MAX_SHELLS, 0.0);
  const size_t bytes = (size_t)L->Q * tot * storage_bytes(prec);
  if (dmalloc(L.get(), &L->A, bytes) != hipSuccess || dmalloc(L.get(), &L->B, bytes) != hipSuccess) {
    if (L->A) (void)dfree(L.get(), L->A);
    (void)hipGetLastError();
    return fail(SCL_E_NOMEM, "population buffers do not fit in device memory");
  }
  if (L->d == 3 && dmalloc(L.get(), &L->d_psi3, (size_t)tot * (prec == SCL_FP64 ? 8 : 4)) != hipSuccess) {
    (void)dfree(L.get(), L->A);
    (void)dfree(L.get(), L->B);
    (void)hipGetLastError();
    return fail(SCL_E_NOMEM, "the psi array does not fit in device memory");
  }
  HIPCHK(hipEventCreate(&L->ev0));
  HIPCHK(hipEventCreate(&L->ev1));
  *out = L.release();
  return SCL_OK;
}

scl_status scl_destroy(scl_lattice L) {
  if (!L) return SCL_OK;
  drop_graph(L);
  adjoint_free(L, L->adj);
  void* ptrs[] = {L->A, L->B, L->d_doms, L->d_items, L->d_n, L->d_psi, L->d_j, L->d_F, L->d_tmp, L->d_part,
                  L->d_psi3};
  for (void* p : ptrs)
    if (p) (void)dfree(L, p);
  if (L->cap) (void)hipStreamDestroy(L->cap);
  if (L->ev0) (void)hipEventDestroy(L->ev0);
  if (L->ev1) (void)hipEventDestroy(L->ev1);
  delete L;
  return SCL_OK;
}

scl_status scl_set_physics(scl_lattice L, const double* tau, const double* G, scl_psi kind, const double* psi_param) {
  if (!L || !tau || !G) return fail(SCL_E_INVALID, "lattice, tau and G are required");
  if (kind != SCL_PSI_EXP && kind != SCL_PSI_EPS && kind != SCL_PSI_CLASSIC)
    return fail(SCL_E_INVALID, "unknown pseudopotential");
  if (kind == SCL_PSI_EPS && !psi_param) return fail(SCL_E_INVALID, "SCL_PSI_EPS needs psi_param");
  for (int k = 0; k < L->ndom; ++k) {
    if (!(tau[k] > 0.5) || !std::isfinite(tau[k])) return fail(SCL_E_INVALID, "tau must be finite and > 1/2");
    if (!std::isfinite(G[k])) return fail(SCL_E_INVALID, "G must be finite");
    if (kind == SCL_PSI_EPS && !(psi_param[k] > 0.0 && std::isfinite(psi_param[k])))
      return fail(SCL_E_INVALID, "eps must be finite and > 0");
  }
  for (int k = 0; k < L->ndom; ++k) {
    L->tau[k] = tau[k];
    L->G[k] = G[k];
    L->psi_param[k] = (kind == SCL_PSI_EPS) ? psi_param[k] : 0.0;
  }
  L->psi_kind = (int)kind;
  L->have_physics = true;
  L->dirty_doms = true;
  drop_graph(L);
  return SCL_OK;
}

scl_status scl_set_force_squared(scl_lattice L, const double* A) {
  if (!L || !A) return fail(SCL_E_INVALID, "bad arguments");
  for (int k = 0; k < L->ndom; ++k)
    if (!std::isfinite(A[k])) return fail(SCL_E_INVALID, "A must be finite");
  L->aF.assign(A, A + L->ndom);
  L->dirty_doms = true;
  drop_graph(L);
  return SCL_OK;
}

scl_status scl_set_stencil(scl_lattice L, int32_t nshells, const int32_t* codes, const double* W) {
  if (!L || !codes || !W || nshells < 1 || nshells > MAX_SHELLS) return fail(SCL_E_INVALID, "bad stencil arguments");
  const int* sets = L->d == 2 ? &SET2[0][0] : &SET3[0][0];
  const int nsets = L->d == 2 ? NSETS2 : NSETS3;
  const int* setn = L->d == 2 ? SET2N : SET3N;
  std::vector<int> slot(nshells, -1);
  for (int s = 0; s < nshells; ++s)
    for (int q = 0; q < s; ++q)
      if (codes[q] == codes[s]) return fail(SCL_E_INVALID, "repeated shell code");
  // the smallest compile-time set holding every requested shell
  int set = -1;
  for (int c = 0; c < nsets && set < 0; ++c) {
    bool all = true;
    for (int s = 0; s < nshells; ++s) {
      bool in = false;
      for (int q = 0; q < setn[c]; ++q) in |= sets[c * SETW + q] == codes[s];
      all &= in;
    }
    if (all) set = c;
  }
  if (set < 0)
    return fail(SCL_E_INVALID, std::string("unsupported shell codes") +
                                   (L->d == 2 ? " (2D supports 1,2,4,5,8,9,16,18)" : " (3D supports 1,2,3,4,5,6,8,9,1009,16,18)"));
  for (int k = 0; k < L->ndom; ++k)
    for (int s = 0; s < nshells; ++s)
      if (!std::isfinite(W[(size_t)k * nshells + s])) return fail(SCL_E_INVALID, "weights must be finite");
  for (int s = 0; s < nshells; ++s)
    for (int q = 0; q < setn[set]; ++q)
      if (sets[set * SETW + q] == codes[s]) slot[s] = q;
  L->set = set;
  if (L->d == 2 && set == 2) {
    // the reach-4 set is built for one site per lane and 128- or 256-lane strips
    if (L->strip == 64 || L->strip == 512) L->strip = 0;
    L->cpl_req = 0;
  }
  if (L->d == 3 && set == 2 && (L->tile3 == 1 || L->tile3 == 4)) L->tile3 = 2;  // reach 4: 64x8 and 32x8 tiles
  L->user_codes.assign(codes, codes + nshells);
  L->slot_of_user = slot;
  std::fill(L->Wslot.begin(), L->Wslot.end(), 0.0);
  for (int k = 0; k < L->ndom; ++k)
    for (int s = 0; s < nshells; ++s) L->Wslot[(size_t)k * MAX_SHELLS + slot[s]] = W[(size_t)k * nshells + s];
  L->have_stencil = true;
  L->dirty_doms = true;
  L->dirty_items = true;
  drop_graph(L);
  return SCL_OK;
}

scl_status scl_init_density(scl_lattice L, const double* n0, int32_t is_dev) {
  if (!L || !n0) return fail(SCL_E_INVALID, "lattice and n0 are required");
  std::vector<double> h((size_t)L->cells);
  if (is_dev) {
    HIPCHK(hipMemcpyAsync(h.data(), n0, h.size() * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
  } else {
    std::memcpy(h.data(), n0, h.size() * sizeof(double));
  }
  for (size_t c = 0; c < h.size(); ++c)
    if (!(h[c] > 0.0) || !std::isfinite(h[c])) return fail(SCL_E_INVALID, "initial density must be finite and > 0");
  const bool shifted = L->prec == SCL_FP32_SHIFTED || L->prec == SCL_FP16S_FP32;
  for (int k = 0; k < L->ndom; ++k) {
    const long long c = (long long)L->nx[k] * L->ny[k] * L->nz[k];
    double s = 0;
    for (long long q = 0; q < c; ++q) s += h[(size_t)(L->off[k] + q)];
    L->rho0[k] = shifted ? s / (double)c : 0.0;
  }
  L->dirty_doms = true;
  double* dn = nullptr;
  HIPCHK(dmalloc(L, &dn, h.size() * sizeof(double)));
  HIPCHK(hipMemcpyAsync(dn, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, L->stream));
  std::vector<DomDev> doms = host_doms(L);
  for (int k = 0; k < L->ndom; ++k) {
    const long long c = (long long)L->nx[k] * L->ny[k] * L->nz[k];
    const unsigned nb = blocks_for(c, 256);
#define INIT(VS, S) hipLaunchKernelGGL((k_init<VS, S>), dim3(nb), dim3(256), 0, L->stream, (S*)L->A, dn, doms[k])
    if (L->vs == SCL_D2Q9) {
      if (L->prec == SCL_FP64) INIT(0, double); else if (L->prec == SCL_FP16S_FP32) INIT(0, _Float16); else INIT(0, float);
    } else {
      if (L->prec == SCL_FP64) INIT(1, double); else if (L->prec == SCL_FP16S_FP32) INIT(1, _Float16); else INIT(1, float);
    }
#undef INIT
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(L->stream));
  HIPCHK(dfree(L, dn));
  L->have_state = true;
  L->steps = 0;
  L->adj.valid = false;
  drop_graph(L);
  return SCL_OK;
}

scl_status scl_step(scl_lattice L, int64_t nsteps) {
  if (!L || nsteps < 0) return fail(SCL_E_INVALID, "bad step arguments");
  return do_steps(L, nsteps);
}

scl_status scl_step_timed(scl_lattice L, int64_t nsteps, double* ms) {
  if (!L || nsteps < 0 || !ms) return fail(SCL_E_INVALID, "bad step arguments");
  scl_status s = ready(L);
  if (s != SCL_OK) return s;
  HIPCHK(hipEventRecord(L->ev0, L->stream));
  s = do_steps(L, nsteps);
  if (s != SCL_OK) return s;
  HIPCHK(hipEventRecord(L->ev1, L->stream));
  HIPCHK(hipEventSynchronize(L->ev1));
  float f = 0;
  HIPCHK(hipEventElapsedTime(&f, L->ev0, L->ev1));
  *ms = f;
  return SCL_OK;
}

scl_status scl_get_step_count(scl_lattice L, int64_t* steps) {
  if (!L || !steps) return fail(SCL_E_INVALID, "bad arguments");
  *steps = L->steps;
  return SCL_OK;
}

scl_status scl_get_density(scl_lattice L, double* out, int32_t is_dev) {
  if (!L || !out) return fail(SCL_E_INVALID, "bad arguments");
  scl_status s = compute_fields(L, false);
  if (s != SCL_OK) return s;
  return copy_out(L, out, L->d_n, (size_t)L->cells, is_dev);
}

scl_status scl_get_force(scl_lattice L, double* out, int32_t is_dev) {
  if (!L || !out) return fail(SCL_E_INVALID, "bad arguments");
  scl_status s = compute_fields(L, true);
  if (s != SCL_OK) return s;
  for (int q = 0; q < L->d; ++q) {
    s = copy_out(L, out + (size_t)q * L->cells, L->d_F + (size_t)q * L->cells, (size_t)L->cells, is_dev);
    if (s != SCL_OK) return s;
  }
  return SCL_OK;
}

scl_status scl_get_velocity(scl_lattice L, double* out, int32_t is_dev) {
  if (!L || !out) return fail(SCL_E_INVALID, "bad arguments");
  scl_status s = compute_fields(L, true);
  if (s != SCL_OK) return s;
  if (L->d == 2) hipLaunchKernelGGL(k_velocity<2>, dim3(blocks_for(L->cells, 256)), dim3(256), 0, L->stream, L->d_n, L->d_j, L->d_F, L->d_tmp, L->cells);
  else hipLaunchKernelGGL(k_velocity<3>, dim3(blocks_for(L->cells, 256)), dim3(256), 0, L->stream, L->d_n, L->d_j, L->d_F, L->d_tmp, L->cells);
  HIPCHK(hipGetLastError());
  return copy_out(L, out, L->d_tmp, (size_t)L->d * L->cells, is_dev);
}

scl_status scl_get_populations(scl_lattice L, double* out, int32_t is_dev) {
  if (!L || !out) return fail(SCL_E_INVALID, "bad arguments");
  scl_status s = ready(L);
  if (s != SCL_OK) return s;
  const size_t n = (size_t)L->Q * L->cells;
  double* dst = out;
  if (!is_dev) HIPCHK(dmalloc(L, &dst, n * sizeof(double)));
  std::vector<DomDev> doms = host_doms(L);
  for (int k = 0; k < L->ndom; ++k) {
    const long long c = (long long)L->nx[k] * L->ny[k] * L->nz[k];
    const unsigned nb = blocks_for(c, 256);
#define GETP(VS, S) hipLaunchKernelGGL((k_get_pops<VS, S>), dim3(nb), dim3(256), 0, L->stream, (const S*)L->A, dst, doms[k])
    if (L->vs == SCL_D2Q9) {
      if (L->prec == SCL_FP64) GETP(0, double); else if (L->prec == SCL_FP16S_FP32) GETP(0, _Float16); else GETP(0, float);
    } else {
      if (L->prec == SCL_FP64) GETP(1, double); else if (L->prec == SCL_FP16S_FP32) GETP(1, _Float16); else GETP(1, float);
    }
#undef GETP
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(L->stream));
  if (!is_dev) {
    HIPCHK(hipMemcpy(out, dst, n * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(dfree(L, dst));
  }
  return SCL_OK;
}

scl_status scl_set_populations(scl_lattice L, const double* in, int32_t is_dev) {
  if (!L || !in) return fail(SCL_E_INVALID, "bad arguments");
  if (!L->have_state) return fail(SCL_E_STATE, "scl_init_density has not been called");
  scl_status s = sync_params(L);
  if (s != SCL_OK) return s;
  const size_t n = (size_t)L->Q * L->cells;
  const double* src = in;
  double* tmp = nullptr;
  if (!is_dev) {
    HIPCHK(dmalloc(L, &tmp, n * sizeof(double)));
    HIPCHK(hipMemcpy(tmp, in, n * sizeof(double), hipMemcpyHostToDevice));
    src = tmp;
  }
  std::vector<DomDev> doms = host_doms(L);
  for (int k = 0; k < L->ndom; ++k) {
    const long long c = (long long)L->nx[k] * L->ny[k] * L->nz[k];
    const unsigned nb = blocks_for(c, 256);
#define SETP(VS, S) hipLaunchKernelGGL((k_set_pops<VS, S>), dim3(nb), dim3(256), 0, L->stream, (S*)L->A, src, doms[k])
    if (L->vs == SCL_D2Q9) {
      if (L->prec == SCL_FP64) SETP(0, double); else if (L->prec == SCL_FP16S_FP32) SETP(0, _Float16); else SETP(0, float);
    } else {
      if (L->prec == SCL_FP64) SETP(1, double); else if (L->prec == SCL_FP16S_FP32) SETP(1, _Float16); else SETP(1, float);
    }
#undef SETP
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(L->stream));
  if (tmp) HIPCHK(dfree(L, tmp));
  L->adj.valid = false;
  drop_graph(L);
  return SCL_OK;
}

scl_status scl_reduce_conserved(scl_lattice L, double* mass, double* momentum) {
  if (!L || !mass) return fail(SCL_E_INVALID, "bad arguments");
  scl_status s = compute_fields(L, true);
  if (s != SCL_OK) return s;
  const int nv = 1 + L->d;
  double* d_out = nullptr;
  HIPCHK(dmalloc(L, &d_out, sizeof(double) * nv * L->ndom));
  for (int k = 0; k < L->ndom; ++k) {
    const long long c = (long long)L->nx[k] * L->ny[k] * L->nz[k];
    const long long chunk = 4096;
    const int nb = (int)((c + chunk - 1) / chunk);
    if ((size_t)nb * nv > L->part_cap) {
      if (L->d_part) HIPCHK(dfree(L, L->d_part));
      L->part_cap = (size_t)nb * nv;
      HIPCHK(dmalloc(L, &L->d_part, sizeof(double) * L->part_cap));
    }
    if (L->d == 2)
      hipLaunchKernelGGL(k_reduce_partial<2>, dim3(nb), dim3(RED_NT), 0, L->stream, L->d_n, L->d_j, L->d_F, L->d_part, L->cells, L->off[k], c, chunk);
    else
      hipLaunchKernelGGL(k_reduce_partial<3>, dim3(nb), dim3(RED_NT), 0, L->stream, L->d_n, L->d_j, L->d_F, L->d_part, L->cells, L->off[k], c, chunk);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_NT), 0, L->stream, (const double*)L->d_part, nb, nv, d_out + (size_t)k * nv);
    HIPCHK(hipGetLastError());
  }
  std::vector<double> h((size_t)nv * L->ndom);
  HIPCHK(hipMemcpyAsync(h.data(), d_out, h.size() * sizeof(double), hipMemcpyDeviceToHost, L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  HIPCHK(dfree(L, d_out));
  bool finite = true;
  for (int k = 0; k < L->ndom; ++k) {
    mass[k] = h[(size_t)k * nv];
    finite = finite && std::isfinite(mass[k]);
    if (momentum)
      for (int q = 0; q < L->d; ++q) momentum[(size_t)k * L->d + q] = h[(size_t)k * nv + 1 + q];
  }
  if (!finite) return fail(SCL_E_NONFINITE, "mass is not finite: the run diverged");
  return SCL_OK;
}

scl_status scl_get_pressure_tensor(scl_lattice L, double* out, int32_t is_dev) {
  if (!L || !out) return fail(SCL_E_INVALID, "bad arguments");
  scl_status s = compute_fields(L, false);
  if (s != SCL_OK) return s;
  std::vector<DomDev> doms = host_doms(L);
  if (L->d == 3) {
    const std::vector<PTermDev> terms = ptensor_link_terms(L);
    PTermDev* d_terms = nullptr;
    HIPCHK(dmalloc(L, &d_terms, terms.size() * sizeof(PTermDev)));
    struct Guard {
      const scl_lattice_s* L;
      void* p;
      ~Guard() { (void)dfree(L, p); }
    } guard{L, d_terms};
    HIPCHK(hipMemcpyAsync(d_terms, terms.data(), terms.size() * sizeof(PTermDev), hipMemcpyHostToDevice, L->stream));
    for (int k = 0; k < L->ndom; ++k) {
      const long long c = (long long)L->nx[k] * L->ny[k] * L->nz[k];
      hipLaunchKernelGGL(k_ptensor_terms, dim3(blocks_for(c, 256)), dim3(256), 0, L->stream, (const double*)L->d_n,
                         (const double*)L->d_psi, L->d_tmp, L->cells, doms[k], d_terms, (int)terms.size());
      HIPCHK(hipGetLastError());
    }
    s = copy_out(L, out, L->d_tmp, (size_t)6 * L->cells, is_dev);
    HIPCHK(hipStreamSynchronize(L->stream));
    return s;
  }
  VecTable tab = full_table(L);
  int slot5 = -1;
  for (int q = 0; q < SET2N[L->set]; ++q)
    if (SET2[L->set][q] == 5) slot5 = q;
  for (int k = 0; k < L->ndom; ++k) {
    const long long c = (long long)L->nx[k] * L->ny[k];
    hipLaunchKernelGGL(k_ptensor2d, dim3(blocks_for(c, 256)), dim3(256), 0, L->stream, (const double*)L->d_n,
                       (const double*)L->d_psi, L->d_tmp, L->cells, doms[k], tab, slot5);
    HIPCHK(hipGetLastError());
  }
  return copy_out(L, out, L->d_tmp, (size_t)3 * L->cells, is_dev);
}

// d = 3: cubic domains, centre (x, y, z); Pbar = tr P / 3, C_d with weight r^2,
// R_s = (6 C_d / dP)^(1/3), sigma_s = dP R_s / 2, (4/3) pi R_e^3 n(centre) + (L^3 - (4/3) pi R_e^3) n(corner) = M.
static scl_status droplet_observables3d(scl_lattice L, const int32_t* center, const int8_t* is_bubble, double* out) {
  for (int k = 0; k < L->ndom; ++k) {
    if (L->nx[k] != L->ny[k] || L->nx[k] != L->nz[k]) return fail(SCL_E_INVALID, "3D droplet observables need cubic domains");
    for (int i = 0; i < 3; ++i)
      if (center[3 * k + i] < 0 || center[3 * k + i] >= L->nx[k]) return fail(SCL_E_INVALID, "centre outside the domain");
  }
  std::vector<double> P((size_t)6 * L->cells);
  scl_status s = scl_get_pressure_tensor(L, P.data(), 0);
  if (s != SCL_OK) return s;
  std::vector<double> n((size_t)L->cells);
  HIPCHK(hipMemcpy(n.data(), L->d_n, n.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> mass(L->ndom);
  s = scl_reduce_conserved(L, mass.data(), nullptr);
  if (s != SCL_OK) return s;
  const long long C = L->cells;
  for (int k = 0; k < L->ndom; ++k) {
    const int Ls = L->nx[k], cx = center[3 * k], cy = center[3 * k + 1], cz = center[3 * k + 2];
    const long long o = L->off[k];
    auto idx = [&](int x, int y, int z) {
      return (size_t)(o + ((long long)wrapi(z, Ls) * Ls + wrapi(y, Ls)) * Ls + wrapi(x, Ls));
    };
    auto pbar = [&](size_t c) { return (P[c] + P[(size_t)C + c] + P[(size_t)2 * C + c]) / 3.0; };
    const double Pc = pbar(idx(cx, cy, cz)), Po = pbar(idx(0, 0, 0));
    const double dP = Pc - Po;
    const int Rm = Ls / 2;
    double Cd = 0;
    for (int sg = -1; sg <= 1; sg += 2) {
      double sum = 0;
      for (int r = 0; r <= Rm; ++r) {
        double g = (double)r * r * (Po - P[(size_t)C + idx(cx + sg * r, cy, cz)]);
        if (r == 0 || r == Rm) g *= 0.5;
        sum += g;
      }
      Cd += 0.5 * sum;
    }
    const double Rs = std::cbrt(6.0 * Cd / dP);
    const double sgn = (is_bubble && is_bubble[k]) ? -1.0 : 1.0;
    const double nin = n[idx(cx, cy, cz)], nout = n[idx(0, 0, 0)];
    const double L3 = (double)Ls * Ls * Ls;
    const double Re = std::cbrt((mass[k] - L3 * nout) / (4.0 / 3.0 * M_PI * (nin - nout)));
    double* r6 = out + (size_t)6 * k;
    r6[0] = dP; r6[1] = Cd; r6[2] = Rs; r6[3] = 0.5 * dP * Rs; r6[4] = Re; r6[5] = sgn * (Re - Rs);
  }
  return SCL_OK;
}

scl_status scl_droplet_observables(scl_lattice L, const int32_t* center, const int8_t* is_bubble, double* out) {
  if (!L || !center || !out) return fail(SCL_E_INVALID, "bad arguments");
  if (L->d == 3) return droplet_observables3d(L, center, is_bubble, out);
  for (int k = 0; k < L->ndom; ++k) {
    if (L->nx[k] != L->ny[k]) return fail(SCL_E_INVALID, "droplet observables need square domains");
    if (center[2 * k] < 0 || center[2 * k] >= L->nx[k] || center[2 * k + 1] < 0 || center[2 * k + 1] >= L->ny[k])
      return fail(SCL_E_INVALID, "centre outside the domain");
  }
  std::vector<double> P((size_t)3 * L->cells);
  scl_status s = scl_get_pressure_tensor(L, P.data(), 0);
  if (s != SCL_OK) return s;
  std::vector<double> n((size_t)L->cells);
  HIPCHK(hipMemcpy(n.data(), L->d_n, n.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> mass(L->ndom);
  s = scl_reduce_conserved(L, mass.data(), nullptr);
  if (s != SCL_OK) return s;
  const long long C = L->cells;
  for (int k = 0; k < L->ndom; ++k) {
    const int Ls = L->nx[k], cx = center[2 * k], cy = center[2 * k + 1];
    const long long o = L->off[k];
    auto at = [&](int plane, int x, int y) { return P[(size_t)(plane * C + o + (long long)wrapi(y, Ls) * Ls + wrapi(x, Ls))]; };
    const double Pc = 0.5 * (at(0, cx, cy) + at(1, cx, cy));
    const double Po = 0.5 * (at(0, 0, 0) + at(1, 0, 0));
    const double dP = Pc - Po;
    const int Rm = Ls / 2;
    double Cd = 0;
    for (int sg = -1; sg <= 1; sg += 2) {
      double sum = 0;
      for (int r = 0; r <= Rm; ++r) {
        double g = r * (Po - at(1, cx + sg * r, cy));
        if (r == 0 || r == Rm) g *= 0.5;
        sum += g;
      }
      Cd += 0.5 * sum;
    }
    const double Rs = std::sqrt(2.0 * Cd / dP);
    const double sgn = (is_bubble && is_bubble[k]) ? -1.0 : 1.0;
    const double sig = dP * Rs;
    const double nin = n[(size_t)(o + (long long)cy * Ls + cx)];
    const double nout = n[(size_t)o];
    const double Re = std::sqrt((mass[k] - (double)Ls * Ls * nout) / (M_PI * (nin - nout)));
    double* r6 = out + (size_t)6 * k;
    r6[0] = dP; r6[1] = Cd; r6[2] = Rs; r6[3] = sig; r6[4] = Re; r6[5] = sgn * (Re - Rs);
  }
  return SCL_OK;
}

scl_status scl_flat_observables(scl_lattice L, const double* bulk, double* out) {
  if (!L || !out) return fail(SCL_E_INVALID, "bad arguments");
  for (int k = 0; k < L->ndom; ++k)
    if (L->nx[k] < 4 || L->nx[k] % 2) return fail(SCL_E_INVALID, "flat-interface observables need an even nx >= 4");
  const int planes = L->d == 2 ? 3 : 6;
  std::vector<double> P((size_t)planes * L->cells);
  scl_status s = scl_get_pressure_tensor(L, P.data(), 0);
  if (s != SCL_OK) return s;
  std::vector<double> n((size_t)L->cells);
  HIPCHK(hipMemcpy(n.data(), L->d_n, n.size() * sizeof(double), hipMemcpyDeviceToHost));
  const long long C = L->cells;
  for (int k = 0; k < L->ndom; ++k) {
    const int nx = L->nx[k], rows = L->ny[k] * L->nz[k];
    const long long o = L->off[k];
    // profiles along x: means over the rows (y, and z in 3D)
    std::vector<double> nb(nx, 0.0), pn(nx, 0.0), pt(nx, 0.0);
    for (int y = 0; y < rows; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t c = (size_t)(o + (long long)y * nx + x);
        nb[x] += n[c] / rows;
        pn[x] += P[c] / rows;
        pt[x] += P[(size_t)C + c] / rows;
      }
    double nl = bulk ? bulk[2 * k] : 0.0, ng = bulk ? bulk[2 * k + 1] : 0.0;
    if (!(nl > 0.0 && ng > 0.0)) {
      nl = *std::max_element(nb.begin(), nb.end());
      ng = *std::min_element(nb.begin(), nb.end());
    }
    for (int h = 0; h < 2; ++h) {
      const int lo = h * nx / 2, hi = (h + 1) * nx / 2;
      double sig = 0.0, mom = 0.0, mass = 0.0;
      for (int x = lo; x < hi; ++x) {
        sig += pn[x] - pt[x];
        mom += x * (pn[x] - pt[x]);
        mass += nb[x];
      }
      const double zs = mom / sig;
      // sharp step between the bulks holding the same mass; sites are cells [x - 1/2, x + 1/2)
      const bool liquid_low = nb[lo] > nb[hi - 1];
      const double nlo = liquid_low ? nl : ng, nhi = liquid_low ? ng : nl;
      const double a = lo - 0.5, b = hi - 0.5;
      const double ze = (mass + nlo * a - nhi * b) / (nlo - nhi);
      const double orient = liquid_low ? 1.0 : -1.0;
      const double delta = orient * (ze - zs);
      const double gam = mass - (nlo * (zs - a) + nhi * (b - zs));
      double* r = out + (size_t)10 * k + 5 * h;
      r[0] = sig; r[1] = zs; r[2] = ze; r[3] = delta; r[4] = gam / (nl - ng);
    }
  }
  return SCL_OK;
}

scl_status scl_set_tiling(scl_lattice L, int32_t strip, int32_t seg, int32_t cpl) {
  if (!L || seg < 0 || cpl < 0 || (strip < 0 && L->d != 2)) return fail(SCL_E_INVALID, "bad tiling");
  if (L->d == 2 && strip < 0) {
    // one-shot tiles: -strip lanes (256 or 512), seg rows per tile, cpl 64-column units of width
    const int nt = -strip, ty = seg ? seg : 16, tx = cpl == 2 ? 128 : 64;
    if (nt != 256 && nt != 512) return fail(SCL_E_INVALID, "2D tiles run 256 or 512 lanes (strip -256 or -512)");
    if (ty != 8 && ty != 16 && ty != 24 && ty != 32) return fail(SCL_E_INVALID, "2D tiles are 8, 16, 24 or 32 rows high");
    if (cpl > 2) return fail(SCL_E_INVALID, "2D tiles are 64 (cpl 0 or 1) or 128 (cpl 2) columns wide");
    if (nt == 512 && ty == 8) return fail(SCL_E_UNSUPPORTED, "512-lane tiles are 16, 24 or 32 rows high");
    if (!planes_fit_tiles(L)) return fail(SCL_E_UNSUPPORTED, "2D tiles need every domain's population plane under 2 GiB");
    L->tile2 = nt;
    L->tile_ty = ty;
    L->tile_tx = tx;
    L->dirty_items = true;
    drop_graph(L);
    return SCL_OK;
  }
  if (L->d == 2) {
    if (strip != 0 && strip != 64 && strip != 128 && strip != 256 && strip != 512)
      return fail(SCL_E_INVALID, "2D strip must be 64, 128, 256 or 512");
    if ((strip ? strip : L->strip) == 512 && cpl == 2)
      return fail(SCL_E_UNSUPPORTED, "512-lane strips run one site per lane");
    if (cpl > 2) return fail(SCL_E_INVALID, "sites per lane must be 1 or 2 (0 = automatic)");
    if (L->set == 2 && (strip == 64 || strip == 512 || cpl == 2))
      return fail(SCL_E_UNSUPPORTED, "the reach-4 shell set runs with 128- or 256-lane strips, one site per lane");
    if (cpl == 2)
      for (int k = 0; k < L->ndom; ++k)
        if (L->nx[k] % 2) return fail(SCL_E_INVALID, "two sites per lane need even domain widths");
    if (strip) L->strip = strip;
    if (strip) L->tile2 = 0;
    if (seg) L->seg = seg;
    L->cpl_req = cpl;
  } else {
    if (strip > 4) return fail(SCL_E_INVALID, "3D tile index must be 1 (64x4), 2 (64x8), 3 (32x8) or 4 (128x4)");
    if ((strip == 1 || strip == 4) && L->set == 2)
      return fail(SCL_E_UNSUPPORTED, "the reach-4 3D shell set runs with tiles 2 (64x8) and 3 (32x8)");
    if (strip) L->tile3 = strip;
    if (seg) L->seg3 = seg;
  }
  L->dirty_items = true;
  drop_graph(L);
  return SCL_OK;
}

scl_status scl_get_tiling(scl_lattice L, int32_t* strip, int32_t* seg, int32_t* cpl) {
  if (!L || !strip || !seg) return fail(SCL_E_INVALID, "bad arguments");
  if (L->dirty_items) {
    scl_status st = build_items(L);
    if (st != SCL_OK) return st;
  }
  *strip = L->d == 2 ? (L->tile2_eff ? -L->tile2_eff : L->strip_eff) : L->tile3_eff;
  *seg = L->d == 2 ? (L->tile2_eff ? L->tile_ty_eff : L->seg) : L->seg3;
  if (cpl) *cpl = L->d == 2 ? (L->tile2_eff ? L->tile_tx_eff / 64 : L->cpl) : 1;
  return SCL_OK;
}

scl_status scl_set_graph_steps(scl_lattice L, int32_t k) {
  if (!L || k < 0 || (k % 2) != 0) return fail(SCL_E_INVALID, "graph length must be even and >= 0");
  L->graph_k = k;
  drop_graph(L);
  return SCL_OK;
}

scl_status scl_tune(scl_lattice L, const char* cache_path) {
  if (!L) return fail(SCL_E_INVALID, "bad arguments");
  scl_status s = ready(L);
  if (s != SCL_OK) return s;
  hipDeviceProp_t prop;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  std::ostringstream key;
  key << prop.gcnArchName << " vs" << (int)L->vs << " reach" << stencil_reach(L) << " prec" << (int)L->prec;
  for (int k = 0; k < L->ndom; ++k) key << " " << L->nx[k] << "x" << L->ny[k] << "x" << L->nz[k];
  const std::string ks = key.str();
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t bar = line.rfind('|');
      if (bar == std::string::npos || line.substr(0, bar) != ks) continue;
      int a = 0, b = 0, c = 0;
      if (std::sscanf(line.c_str() + bar + 1, "%d %d %d", &a, &b, &c) >= 2) return scl_set_tiling(L, a, b, c);
    }
  }
  std::vector<std::array<int, 3>> cands;  // (strip, seg, cpl)
  if (L->d == 2) {
    for (int st : {64, 128, 256, 512}) {
      if ((st == 64 || st == 512) && L->set == 2) continue;
      for (int sg : {8, 16, 32, 64, 128}) cands.push_back({st, sg, 0});
    }
    if (planes_fit_tiles(L))
      for (int w : {1, 2}) {
        for (int ty : {8, 16, 24, 32}) cands.push_back({-256, ty, w});
        for (int ty : {16, 24, 32}) cands.push_back({-512, ty, w});
      }
  } else {
    for (int t : {1, 2, 3, 4}) {
      if ((t == 1 || t == 4) && L->set == 2) continue;
      for (int sg : {8, 16, 32, 64}) cands.push_back({t, sg, 0});
    }
  }
  const int saved_graph = L->graph_k;
  L->graph_k = 0;
  double best = 1e30;
  std::array<int, 3> bc = cands[0];
  const int reps = 4;
  for (auto c : cands) {
    s = scl_set_tiling(L, c[0], c[1], c[2]);
    if (s != SCL_OK) return s;
    double ms = 0;
    s = scl_step_timed(L, 2, &ms);  // warm-up (and item upload)
    if (s != SCL_OK) return s;
    s = scl_step_timed(L, reps, &ms);
    if (s != SCL_OK) return s;
    if (ms < best) { best = ms; bc = c; }
  }
  L->graph_k = saved_graph;
  s = scl_set_tiling(L, bc[0], bc[1], bc[2]);
  if (s != SCL_OK) return s;
  if (cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << ks << "|" << bc[0] << " " << bc[1] << " " << bc[2] << "\n";
  }
  return SCL_OK;
}

scl_status scl_checkpointed_forward(scl_lattice L, int64_t nsteps, int32_t every) {
  if (!L || nsteps < 1 || every < 1) return fail(SCL_E_INVALID, "need nsteps >= 1 and every >= 1");
  if (L->d != 2) return fail(SCL_E_UNSUPPORTED, "the adjoint is implemented for D2Q9");
  if (L->prec == SCL_FP16S_FP32) return fail(SCL_E_UNSUPPORTED, "the adjoint needs FP32 or FP64 populations");
  scl_status s = ready(L);
  if (s != SCL_OK) return s;
  AdjointState& a = L->adj;
  const size_t sb = state_bytes(L);
  const int nfull = (int)(nsteps / every);
  const int slots = nfull + 2;  // states at 0, every, ..., nfull*every, and the final one
  if (a.pool_bytes < (size_t)slots * sb) {
    if (a.pool) HIPCHK(dfree(L, a.pool));
    a.pool = nullptr;
    a.pool_bytes = 0;
    if (dmalloc(L, &a.pool, (size_t)slots * sb) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SCL_E_NOMEM, "checkpoint pool does not fit in device memory");
    }
    a.pool_bytes = (size_t)slots * sb;
  }
  char* pool = (char*)a.pool;
  HIPCHK(hipMemcpyAsync(pool, L->A, sb, hipMemcpyDeviceToDevice, L->stream));
  int64_t done = 0;
  for (int c = 1; c <= nfull; ++c) {
    s = do_steps(L, every);
    if (s != SCL_OK) return s;
    done += every;
    HIPCHK(hipMemcpyAsync(pool + (size_t)c * sb, L->A, sb, hipMemcpyDeviceToDevice, L->stream));
  }
  if (done < nsteps) {
    s = do_steps(L, nsteps - done);
    if (s != SCL_OK) return s;
  }
  HIPCHK(hipMemcpyAsync(pool + (size_t)(nfull + 1) * sb, L->A, sb, hipMemcpyDeviceToDevice, L->stream));
  a.nckpt = slots;
  a.every = every;
  a.nsteps = nsteps;
  a.valid = true;
  a.end_step = L->steps;
  return SCL_OK;
}

scl_status scl_adjoint(scl_lattice L, const double* seed_n, const double* seed_f, double* grad_W, double* grad_G) {
  if (!L || !grad_W || !grad_G) return fail(SCL_E_INVALID, "gradient outputs are required");
  AdjointState& a = L->adj;
  if (!a.valid || a.end_step != L->steps) return fail(SCL_E_STATE, "run scl_checkpointed_forward first (and leave the state unchanged)");
  // The recompute records n, j, F through the marching step: with one-shot tiles in use,
  // march for the duration of this call and return to the tiles afterwards.
  struct TileRestore {
    scl_lattice_s* L;
    bool on;
    ~TileRestore() {
      if (on) { L->march_only = false; L->dirty_items = true; drop_graph(L); }
    }
  } tile_restore{L, L->d == 2};
  if (L->d == 2) { L->march_only = true; L->dirty_items = true; drop_graph(L); }
  scl_status s = sync_params(L);
  if (s != SCL_OK) return s;
  const bool f64 = L->prec == SCL_FP64;
  const size_t ms = f64 ? 8 : 4;
  const size_t sb = state_bytes(L);
  const long long C = L->cells;
  const int every = a.every;
  // buffers
  const size_t rec_need = (size_t)every * 5 * C * ms;
  if (a.rec_bytes < rec_need) {
    if (a.rec) HIPCHK(dfree(L, a.rec));
    a.rec = nullptr;
    if (dmalloc(L, &a.rec, rec_need) != hipSuccess) { (void)hipGetLastError(); a.rec_bytes = 0; return fail(SCL_E_NOMEM, "recompute buffer does not fit"); }
    a.rec_bytes = rec_need;
  }
  const size_t lam_need = (size_t)L->Q * C * ms;
  if (a.lam_bytes < lam_need) {
    for (int b = 0; b < 2; ++b) {
      if (a.lam[b]) HIPCHK(dfree(L, a.lam[b]));
      a.lam[b] = nullptr;
      if (dmalloc(L, &a.lam[b], lam_need) != hipSuccess) { (void)hipGetLastError(); a.lam_bytes = 0; return fail(SCL_E_NOMEM, "adjoint buffers do not fit"); }
    }
    a.lam_bytes = lam_need;
  }
  constexpr int NO = 128;
  // rows per item: 32, halved down to 8 while the lattice gives fewer than 1024 items (one
  // 128-lane workgroup per item holds few waves, so small batches need many items to fill
  // the CUs: for 16 domains of 256^2 and 2000 steps the backward pass takes 0.152 s with 8
  // rows against 0.184 s with 32)
  int aseg = 32;
  while (aseg > 8 && adjoint_items(L, NO, aseg).size() < 1024) aseg /= 2;
  std::vector<WorkItem> items = adjoint_items(L, NO, aseg);
  WorkItem* d_items = nullptr;
  HIPCHK(dmalloc(L, &d_items, sizeof(WorkItem) * items.size()));
  HIPCHK(hipMemcpy(d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
  const int nitems = (int)items.size();
  const int NSG = 1 + ADJ_MAXS;
  if (a.gpart_cap < (size_t)nitems * NSG) {
    if (a.gpart) HIPCHK(dfree(L, a.gpart));
    HIPCHK(dmalloc(L, &a.gpart, sizeof(double) * nitems * NSG));
    a.gpart_cap = (size_t)nitems * NSG;
  }
  // seed
  std::vector<DomDev> doms = host_doms(L);
  for (int k = 0; k < L->ndom; ++k) {
    const long long c = (long long)L->nx[k] * L->ny[k];
    if (f64) hipLaunchKernelGGL(k_adj_seed<double>, dim3(blocks_for(c, 256)), dim3(256), 0, L->stream, (double*)a.lam[0], seed_n, seed_f, doms[k], L->Q);
    else hipLaunchKernelGGL(k_adj_seed<float>, dim3(blocks_for(c, 256)), dim3(256), 0, L->stream, (float*)a.lam[0], seed_n, seed_f, doms[k], L->Q);
    HIPCHK(hipGetLastError());
  }
  int cur = 0;
  bool first = true;
  const int per = (nitems + 7) / 8;
  char* pool = (char*)a.pool;
  const int nseg = (int)((a.nsteps + every - 1) / every);
  for (int sgi = nseg - 1; sgi >= 0; --sgi) {
    const long long t0 = (long long)sgi * every;
    const long long t1 = std::min<long long>(t0 + every, a.nsteps);
    HIPCHK(hipMemcpyAsync(L->A, pool + (size_t)sgi * sb, sb, hipMemcpyDeviceToDevice, L->stream));
    // recompute the segment, recording n, j, F of every step
    for (long long t = t0; t < t1; ++t) {
      char* base = (char*)a.rec + (size_t)(t - t0) * 5 * C * ms;
      hipError_t e;
      if (f64) {
        MacroRec<double> r{(double*)base, (double*)base + C, (double*)base + 3 * C, C};
        e = launch_step(L, L->A, L->B, &r, nullptr);
      } else {
        MacroRec<float> r{(float*)base, (float*)base + C, (float*)base + 3 * C, C};
        e = launch_step(L, L->A, L->B, nullptr, &r);
      }
      if (e != hipSuccess) { (void)dfree(L, d_items); return fail(SCL_E_DEVICE, std::string("recompute: ") + hipGetErrorString(e)); }
      std::swap(L->A, L->B);
    }
    // adjoint steps, last to first
    for (long long t = t1 - 1; t >= t0; --t) {
      char* base = (char*)a.rec + (size_t)(t - t0) * 5 * C * ms;
      const int acc = first ? 0 : 1;
#define ADJ_LAUNCH(M_, SETV)                                                                              \
  hipLaunchKernelGGL((k_adjoint2d<M_, SETV, NO>), dim3(8 * per), dim3(NO + 2 * Shells<2, SETV>::R), 0, L->stream, \
                     (const M_*)a.lam[cur], (M_*)a.lam[1 - cur], (const M_*)base, (const M_*)base + C,          \
                     (const M_*)base + 3 * C, C, L->d_doms, d_items, nitems, a.gpart, acc)
      if (f64) { if (L->set == 0) ADJ_LAUNCH(double, 0); else if (L->set == 1) ADJ_LAUNCH(double, 1); else ADJ_LAUNCH(double, 2); }
      else { if (L->set == 0) ADJ_LAUNCH(float, 0); else if (L->set == 1) ADJ_LAUNCH(float, 1); else ADJ_LAUNCH(float, 2); }
#undef ADJ_LAUNCH
      HIPCHK(hipGetLastError());
      cur = 1 - cur;
      first = false;
    }
  }
  // restore the final state
  HIPCHK(hipMemcpyAsync(L->A, pool + (size_t)(a.nckpt - 1) * sb, sb, hipMemcpyDeviceToDevice, L->stream));
  std::vector<double> part((size_t)nitems * NSG);
  HIPCHK(hipMemcpyAsync(part.data(), a.gpart, part.size() * sizeof(double), hipMemcpyDeviceToHost, L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  HIPCHK(dfree(L, d_items));
  a.lam_cur = cur;
  // per-domain sums in item order; slot order -> the caller's shells
  const int NS = SET2N[L->set];
  const int nsh = (int)L->user_codes.size();
  std::vector<double> gs((size_t)L->ndom * (NS + 1), 0.0);
  for (int i = 0; i < nitems; ++i)
    for (int q = 0; q <= NS; ++q)
      gs[(size_t)items[i].dom * (NS + 1) + q] += part[(size_t)i * NSG + (q < NS ? q : ADJ_MAXS)];
  for (int k = 0; k < L->ndom; ++k) {
    for (int u = 0; u < nsh; ++u) grad_W[(size_t)k * nsh + u] = gs[(size_t)k * (NS + 1) + L->slot_of_user[u]];
    grad_G[k] = gs[(size_t)k * (NS + 1) + NS];
  }
  return SCL_OK;
}

scl_status scl_get_adjoint_populations(scl_lattice L, double* out, int32_t is_dev) {
  if (!L || !out) return fail(SCL_E_INVALID, "bad arguments");
  AdjointState& a = L->adj;
  if (!a.lam[a.lam_cur]) return fail(SCL_E_STATE, "no adjoint has been computed");
  const size_t n = (size_t)L->Q * L->cells;
  double* dst = out;
  if (!is_dev) HIPCHK(dmalloc(L, &dst, n * sizeof(double)));
  if (L->prec == SCL_FP64) hipLaunchKernelGGL(k_adj_get<double>, dim3(blocks_for((long long)n, 256)), dim3(256), 0, L->stream, (const double*)a.lam[a.lam_cur], dst, (long long)n);
  else hipLaunchKernelGGL(k_adj_get<float>, dim3(blocks_for((long long)n, 256)), dim3(256), 0, L->stream, (const float*)a.lam[a.lam_cur], dst, (long long)n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(L->stream));
  if (!is_dev) {
    HIPCHK(hipMemcpy(out, dst, n * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(dfree(L, dst));
  }
  return SCL_OK;
}

scl_status scl_droplet_observables_vjp(scl_lattice L, const int32_t* center, const int8_t* is_bubble, const double* gobs,
                                       double* seed_n, int32_t is_dev, double* grad_W, double* grad_G) {
  if (!L || !center || !gobs || !seed_n || !grad_W || !grad_G) return fail(SCL_E_INVALID, "bad arguments");
  if (L->d != 2) return fail(SCL_E_UNSUPPORTED, "droplet observables are implemented for D2Q9 only");
  for (int k = 0; k < L->ndom; ++k) {
    if (L->nx[k] != L->ny[k]) return fail(SCL_E_INVALID, "droplet observables need square domains");
    if (center[2 * k] < 0 || center[2 * k] >= L->nx[k] || center[2 * k + 1] < 0 || center[2 * k + 1] >= L->ny[k])
      return fail(SCL_E_INVALID, "centre outside the domain");
  }
  scl_status s = compute_fields(L, false);
  if (s != SCL_OK) return s;
  std::vector<double> n((size_t)L->cells);
  HIPCHK(hipMemcpyAsync(n.data(), L->d_n, n.size() * sizeof(double), hipMemcpyDeviceToHost, L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  const std::vector<PTerm> terms = ptensor_terms(L);
  const int nsh = (int)L->user_codes.size();
  std::vector<double> gn((size_t)L->cells, 0.0);
  for (int k = 0; k < L->ndom; ++k) {
    const int Ls = L->nx[k], cx = center[2 * k], cy = center[2 * k + 1];
    const long long o = L->off[k];
    const double G = L->G[k];
    const double Gc2 = G * CS2;
    const double* W = &L->Wslot[(size_t)k * MAX_SHELLS];
    auto idx = [&](int x, int y) { return (size_t)(o + (long long)wrapi(y, Ls) * Ls + wrapi(x, Ls)); };
    auto psi = [&](int x, int y) { return psi_host(n[idx(x, y)], L->psi_kind, L->psi_param[k]); };
    auto P = [&](int x, int y, double& xx, double& yy) {
      double sxx = 0, syy = 0;
      for (const PTerm& t : terms) {
        const double v = t.coef * W[t.slot] * psi(x + t.ax, y + t.ay) * psi(x + t.bx, y + t.by);
        sxx += v * t.ex * t.ex;
        syy += v * t.ey * t.ey;
      }
      xx = n[idx(x, y)] * CS2 + Gc2 * sxx;
      yy = n[idx(x, y)] * CS2 + Gc2 * syy;
    };
    // forward quantities
    double pcx, pcy, pox, poy;
    P(cx, cy, pcx, pcy);
    P(0, 0, pox, poy);
    const double Pbc = 0.5 * (pcx + pcy), Pbo = 0.5 * (pox + poy), dP = Pbc - Pbo;
    const int Rm = Ls / 2;
    double Cd = 0, wsum = 0;
    for (int sg = -1; sg <= 1; sg += 2)
      for (int r = 0; r <= Rm; ++r) {
        double xx, yy;
        P(cx + sg * r, cy, xx, yy);
        const double tw = (r == 0 || r == Rm) ? 0.5 : 1.0;
        Cd += 0.5 * tw * r * (Pbo - yy);
        wsum += 0.5 * tw * r;
      }
    double M = 0;
    for (long long c = 0; c < (long long)Ls * Ls; ++c) M += n[(size_t)(o + c)];
    const double Rs = std::sqrt(2.0 * Cd / dP);
    const double sgn = (is_bubble && is_bubble[k]) ? -1.0 : 1.0;
    const double nin = n[idx(cx, cy)], nout = n[idx(0, 0)];
    const double Nn = M - (double)Ls * Ls * nout, Dd = M_PI * (nin - nout);
    const double Re = std::sqrt(Nn / Dd);
    // backward through the closed forms
    const double* g = gobs + (size_t)6 * k;
    const double gRs = g[2] + g[3] * dP - sgn * g[5];
    const double gRe = g[4] + sgn * g[5];
    const double gdP = g[0] + g[3] * Rs - gRs * Rs / (2.0 * dP);
    const double gCd = g[1] + gRs / (Rs * dP);
    const double gN = gRe / (2.0 * Re * Dd), gD = -gRe * Nn / (2.0 * Re * Dd * Dd);
    const double gM = gN, gno = -(double)Ls * Ls * gN - M_PI * gD, gnc = M_PI * gD;
    // gradients on P components at sites: (site, gPxx, gPyy)
    std::vector<std::tuple<int, int, double, double>> gp;
    const double gPbo = -gdP + gCd * wsum;
    gp.emplace_back(cx, cy, 0.5 * gdP, 0.5 * gdP);
    gp.emplace_back(0, 0, 0.5 * gPbo, 0.5 * gPbo);
    for (int sg = -1; sg <= 1; sg += 2)
      for (int r = 1; r <= Rm; ++r) {
        const double tw = (r == Rm) ? 0.5 : 1.0;
        gp.emplace_back(cx + sg * r, cy, 0.0, -gCd * 0.5 * tw * r);
      }
    std::vector<double> gWs(MAX_SHELLS, 0.0);
    double gG = 0.0;
    for (const auto& e : gp) {
      const int x = std::get<0>(e), y = std::get<1>(e);
      const double gxx = std::get<2>(e), gyy = std::get<3>(e);
      gn[idx(x, y)] += CS2 * (gxx + gyy);
      for (const PTerm& t : terms) {
        const double wgt = gxx * t.ex * t.ex + gyy * t.ey * t.ey;
        if (wgt == 0.0) continue;
        const double pa = psi(x + t.ax, y + t.ay), pb = psi(x + t.bx, y + t.by);
        const double c0 = wgt * t.coef;
        const size_t ia = idx(x + t.ax, y + t.ay), ib = idx(x + t.bx, y + t.by);
        gn[ia] += c0 * Gc2 * W[t.slot] * pb * dpsi_host(n[ia], pa, L->psi_kind, L->psi_param[k]);
        gn[ib] += c0 * Gc2 * W[t.slot] * pa * dpsi_host(n[ib], pb, L->psi_kind, L->psi_param[k]);
        gWs[t.slot] += c0 * Gc2 * pa * pb;
        gG += c0 * CS2 * W[t.slot] * pa * pb;
      }
    }
    for (long long c = 0; c < (long long)Ls * Ls; ++c) gn[(size_t)(o + c)] += gM;
    gn[idx(cx, cy)] += gnc;
    gn[idx(0, 0)] += gno;
    for (int u = 0; u < nsh; ++u) grad_W[(size_t)k * nsh + u] = gWs[L->slot_of_user[u]];
    grad_G[k] = gG;
  }
  HIPCHK(hipMemcpy(seed_n, gn.data(), gn.size() * sizeof(double), is_dev ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
  return SCL_OK;
}

}  // extern "C"
