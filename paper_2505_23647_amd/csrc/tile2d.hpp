// Fused D2Q9 Shan-Chen step over independent tiles: pull-stream, moments, psi, wide-stencil
// force, BGK + Guo collision, one workgroup per tile of TX x TY output sites, no march.
//
// A workgroup of NW waves owns the output sites [x0, x0 + TX) x [y0, y0 + TY) of one domain
// (TX = 64 or 128: one or two waves per tile row). Its lanes form RG = 64 NW / TX row groups;
// lane l of row group g holds the sites (x0 + l, y0 + g + RG k), k < TY / RG: it pulls their nine
// populations (f_i(x, t) = f*_i(x - xi_i, t - 1)) into registers. The psi of every site the
// stencil reaches, the tile plus a rim of R sites, goes to LDS: the tile's own sites from the
// populations just loaded, the rim's from a second set of pulls (2R rim rows of TX sites split
// over the row groups, and the (TY + 2R) x 2R side sites spread over all lanes). After one barrier
// each lane evaluates the force of eq. (sc_f) from LDS, collides (eqs. lbm, omega_i, f_eq,
// GuoForcing) and stores its sites. All of a tile's loads are issued at once, and the grid holds
// one workgroup per tile, so the chip keeps many independent loads in flight and consecutive
// workgroups touch neighbouring memory, as a plain copy does; the price is the rim's psi,
// computed again by each tile that reaches it (its populations mostly come from L2).
#pragma once
#include "scl_common.hpp"

namespace scl {

template <class S, class M, int SET, int TX, int TY, int NW, bool SHIFT>
__global__ void __launch_bounds__(64 * NW)
k_tile2d(const S* __restrict__ fin, S* __restrict__ fout, const DomDev* __restrict__ doms,
         const WorkItem* __restrict__ items, int nitems) {
  using V = Vel<0>;
  using SH = Shells<2, SET>;
  constexpr int Q = V::Q;
  constexpr int R = SH::R;
  constexpr int NT = 64 * NW;
  constexpr int LW = TX + 2 * R;            // LDS row: the tile's columns plus R on each side
  constexpr int LH = TY + 2 * R;            // LDS rows
  constexpr int RG = NT / TX;               // tile rows taken at once (TX lanes each)
  constexpr int KI = TY / RG;               // tile rows per lane
  constexpr int KH = (2 * R + RG - 1) / RG; // rim rows (main columns) per row group
  constexpr int NSIDE = LH * 2 * R;         // side sites: R columns on each side of every LDS row
  constexpr int KS = (NSIDE + NT - 1) / NT;
  static_assert(TX % 64 == 0 && NT % TX == 0 && TY % RG == 0, "tile rows must split evenly over the row groups");
  constexpr uint32_t OFF = 0x80000000u;     // byte offset past any buffer: access dropped

  __shared__ M psis[LH * LW];

  // XCD-aware mapping: consecutive workgroup ids go to different XCDs (round robin over 8);
  // XCD k takes the k-th contiguous eighth of the (row-major) tile list.
  const int per = (nitems + 7) >> 3;
  const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (item >= nitems) return;
  const WorkItem it = items[item];
  const DomDev& dm = doms[it.dom];
  const int nx = dm.nx, ny = dm.ny;
  const long long cells = (long long)nx * ny;
  const S* __restrict__ fb = fin + dm.off * Q;
  S* __restrict__ ob = fout + dm.off * Q;
  const M omega = M(dm.omega), kappa = M(dm.kappa), gpre = M(dm.gpre), aff = M(dm.aff);
  const M eps = M(dm.eps), inv_eps = M(dm.inv_eps), rho0 = M(dm.rho0);
  const int kind = dm.psi_kind;

  const int lane = (int)threadIdx.x % TX;                                 // column in the tile
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x / TX);   // row group (wave-uniform)
  const int x0 = it.x0, y0 = it.y0;
  const int xe = min(x0 + TX, nx), ye = it.y1;  // tile end (cut by the domain's edge)
  const int x = x0 + lane;
  const bool xin = x < xe;
  const uint32_t rowbytes = (uint32_t)nx * sizeof(S);
  // byte offsets of x - 1, x, x + 1 in a row (wrapped), or OFF for idle lanes
  uint32_t vo[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) vo[a] = xin ? (uint32_t)wrapi(x + a - 1, nx) * sizeof(S) : OFF;

  // the nine pulls of a site in row y of this lane's column (row-uniform descriptors)
  auto pull_row = [&](int y, bool on, M* f) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const Rsrc r = mkrsrc(fb + (long long)i * cells + (long long)wrapi(y - V::cy(i), ny) * nx, rowbytes);
      ldb<S, M, 1>(r, on ? vo[1 - V::cx(i)] : OFF, f + i);
    }
  };
  // sum of a site's stored values (the density, less rho0 for shifted storage)
  auto vsum = [&](const M* f) {
    M s = M(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) s += f[i];
    return s;
  };
  auto psi_of = [&](M s) { return psi_eval<M>(SHIFT ? rho0 + s : s, kind, eps, inv_eps); };

  // ---- 1. pulls: the lane's tile sites, its rim-row sites, its side sites
  M fi[KI][Q];
#pragma unroll
  for (int k = 0; k < KI; ++k) pull_row(y0 + w + RG * k, y0 + w + RG * k < ye, fi[k]);

  M fh[KH][Q];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int h = w + RG * k;  // rim row: 0 .. R-1 above the tile, R .. 2R-1 below it
    const int y = h < R ? y0 - R + h : ye + (h - R);
    pull_row(y, h < 2 * R, fh[k]);
  }

  M fs[KS][Q];
  int lds_side[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int idx = (int)threadIdx.x + NT * k;
    const int ly = idx / (2 * R), c = idx % (2 * R);
    // LDS row ly holds y0 - R + ly for the rim above and the tile's rows, and the rim below
    // right after the tile's last row (a tile cut by the domain's edge leaves a gap)
    const int ntile = ye - y0;
    int y;
    bool on = idx < NSIDE;
    int lrow = ly;
    if (ly < R + ntile) {
      y = y0 - R + ly;
    } else {
      y = ye + (ly - R - ntile);
      on = on && ly < 2 * R + ntile;
    }
    const int xs = c < R ? x0 - R + c : xe + (c - R);
    const int lcol = c < R ? c : (xe - x0) + R + (c - R);
    lds_side[k] = on ? lrow * LW + lcol : -1;
    const uint32_t ro[3] = {(uint32_t)wrapi(y + 1, ny) * rowbytes, (uint32_t)wrapi(y, ny) * rowbytes,
                            (uint32_t)wrapi(y - 1, ny) * rowbytes};
    constexpr uint32_t SB = sizeof(S);
    const uint32_t co[3] = {(uint32_t)wrapi(xs + 1, nx) * SB, (uint32_t)wrapi(xs, nx) * SB,
                            (uint32_t)wrapi(xs - 1, nx) * SB};
    const uint32_t pbytes = (uint32_t)(cells * sizeof(S));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const Rsrc r = mkrsrc(fb + (long long)i * cells, pbytes);
      // pull from (xs - cx, y - cy): index 1 - c selects -c
      ldb<S, M, 1>(r, on ? ro[1 + V::cy(i)] + co[1 + V::cx(i)] : OFF, fs[k] + i);
    }
  }

  // ---- 2. psi of every pulled site into LDS
  M ssum[KI];  // the tile sites' sums, reused by the collision
#pragma unroll
  for (int k = 0; k < KI; ++k) {
    const int ly = w + RG * k + R;
    ssum[k] = vsum(fi[k]);
    const M p = psi_of(ssum[k]);
    if (xin && y0 + w + RG * k < ye) psis[ly * LW + lane + R] = p;
  }
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int h = w + RG * k;
    const int ly = h < R ? h : (ye - y0) + R + (h - R);
    const M p = psi_of(vsum(fh[k]));
    if (xin && h < 2 * R) psis[ly * LW + lane + R] = p;
  }
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const M p = psi_of(vsum(fs[k]));
    if (lds_side[k] >= 0) psis[lds_side[k]] = p;
  }
  __syncthreads();

  // ---- 3. force, collision and store of the lane's tile sites
#pragma unroll
  for (int k = 0; k < KI; ++k) {
    const int y = y0 + w + RG * k;
    const int ly = w + RG * k + R;
    const M* c0 = psis + ly * LW + lane + R;
    const M psic = c0[0];
    M dxs[SH::NS], dys[SH::NS];
#pragma unroll
    for (int s = 0; s < SH::NS; ++s) { dxs[s] = M(0); dys[s] = M(0); }
#pragma unroll
    for (int h = 0; h < SH::NH; ++h) {
      const HalfVec hv = SH::h(h);
      const M d = c0[hv.y * LW + hv.x] - c0[-hv.y * LW - hv.x];
      if (hv.x != 0) dxs[hv.slot] += M(hv.x) * d;
      if (hv.y != 0) dys[hv.slot] += M(hv.y) * d;
    }
    M ax = M(0), ay = M(0);
#pragma unroll
    for (int s = 0; s < SH::NS; ++s) { ax += M(dm.W[s]) * dxs[s]; ay += M(dm.W[s]) * dys[s]; }
    const M Fx = gpre * psic * ax;
    const M Fy = gpre * psic * ay;
    const M sum = ssum[k];
    M jx = M(0), jy = M(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (V::cx(i) != 0) jx += M(V::cx(i)) * fi[k][i];
      if (V::cy(i) != 0) jy += M(V::cy(i)) * fi[k][i];
    }
    const M nn = SHIFT ? rho0 + sum : sum;
    const M inv_n = rcp<M>(nn);
    const M ux = (jx + M(0.5) * Fx) * inv_n;
    const M uy = (jy + M(0.5) * Fy) * inv_n;
    M fo[Q];
    collide<0, M>(fi[k], SHIFT ? sum : nn, nn, ux, uy, M(0), Fx, Fy, M(0), omega, kappa, aff, fo);
    const uint32_t so = (xin && y < ye) ? (uint32_t)x * sizeof(S) : OFF;
    const long long orow = (long long)(y < ye ? y : 0) * nx;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      stb<S, M, 1, SCL_STORE_AUX>(mkrsrc(ob + (long long)i * cells + orow, rowbytes), so, &fo[i]);
  }
}

}  // namespace scl
