// Fused D2Q9 Shan-Chen step: pull-stream, moments, psi, wide-stencil force, BGK + Guo
// collision, in one pass over the populations.
//
// Work decomposition. A workgroup owns a strip of CPL * NO output columns [x0, x0 + CPL*NO)
// (NO output lanes, CPL consecutive sites per lane) and marches along a range of rows. HL
// more lanes, placed after the output lanes, cover the HX = R (rounded up to CPL) halo
// columns on each side, which only supply psi. Output lanes therefore read and write whole,
// aligned cache lines. At every row r the workgroup
//   1. pulls the nine post-collision populations streaming into row r
//      (f_i(x, t) = f*_i(x - xi_i, t-1)) as CPL-wide vectors, adds them to n and stores psi(n)
//      in a ring of 2R + 2 rows in LDS, indexed by the row number;
//   2. collides row r - R (marching order): the force of eq. (sc_f) over the +-pairs of the
//      stencil reads psi from the ring; u = (j + F/2)/n, the equilibrium of eq. (f_eq), the
//      Guo term of eq. (GuoForcing) and the BGK update of eqs. (lbm), (omega_i) give the new
//      post-collision values, stored at x of the output buffer. The populations of a row stay
//      in registers for the R rows between their load and their collision (R + 1 register
//      sets rotated by unrolling).
// Row ranges of one strip alternate their marching direction (upward, downward, ...), so the
// halo rows two neighbouring ranges share are read by both at the same time: at the start of
// both or at the end of both. With the work items of one strip band handed to the same XCD
// (see the item order on the host), those re-reads hit that XCD's L2.
#pragma once
#include "scl_common.hpp"

namespace scl {

template <class S, int CPL> struct VecOf;
template <class S> struct VecOf<S, 1> { typedef S type; };
template <> struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<_Float16, 2> { typedef _Float16 type __attribute__((ext_vector_type(2))); };

// CPL consecutive stored values from p (element alignment suffices: 4-byte aligned global
// vector accesses are legal on gfx9).
template <class S, class M, int CPL> __device__ __forceinline__ void ldv(const S* p, M* out) {
  if constexpr (CPL == 1) {
    out[0] = static_cast<M>(*p);
  } else {
    typename VecOf<S, CPL>::type v;
    __builtin_memcpy(&v, p, sizeof(v));
#pragma unroll
    for (int c = 0; c < CPL; ++c) out[c] = static_cast<M>(v[c]);
  }
}

template <class S, class M, int CPL> __device__ __forceinline__ void stv(S* p, const M* in) {
  if constexpr (CPL == 1) {
    *p = static_cast<S>(in[0]);
  } else {
    typename VecOf<S, CPL>::type v;
#pragma unroll
    for (int c = 0; c < CPL; ++c) v[c] = static_cast<S>(in[c]);
    *reinterpret_cast<typename VecOf<S, CPL>::type*>(p) = v;
  }
}

// Values at row positions xw + dx .. xw + dx + CPL - 1 (dx in {-1, 0, 1}) of a periodic row of
// nx values; xw and nx are multiples of CPL, so only the first or last element can wrap.
// WRAP = false promises that xw + dx .. xw + dx + CPL - 1 lie inside the row: a plain load.
template <class S, class M, int CPL, bool WRAP>
__device__ __forceinline__ void ld_shift(const S* row, int xw, int nx, int dx, M* out) {
  if constexpr (!WRAP) {
    ldv<S, M, CPL>(row + xw + dx, out);
  } else if constexpr (CPL == 1) {
    out[0] = static_cast<M>(row[wrapi(xw + dx, nx)]);
  } else {
    if (dx == 0) {
      ldv<S, M, CPL>(row + xw, out);
    } else if (dx < 0) {
      M v[CPL];
      ldv<S, M, CPL>(row + (xw > 0 ? xw - 1 : 0), v);
      if (xw > 0) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) out[c] = v[c];
      } else {
        out[0] = static_cast<M>(row[nx - 1]);
#pragma unroll
        for (int c = 1; c < CPL; ++c) out[c] = v[c - 1];
      }
    } else {
      M v[CPL];
      const bool wrap = xw + CPL >= nx;
      ldv<S, M, CPL>(row + (wrap ? xw : xw + 1), v);
      if (!wrap) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) out[c] = v[c];
      } else {
#pragma unroll
        for (int c = 0; c < CPL - 1; ++c) out[c] = v[c + 1];
        out[CPL - 1] = static_cast<M>(row[0]);
      }
    }
  }
}

// NO output lanes (a multiple of 64) + 2 HL halo lanes.
template <int SET, int CPL> struct Halo2 {
  static constexpr int R = Shells<2, SET>::R;
  static constexpr int HX = ((R + CPL - 1) / CPL) * CPL;  // halo columns per side
  static constexpr int HL = HX / CPL;                     // halo lanes per side
};

template <class S, class M, int SET, int NO, int CPL, bool SHIFT, bool REC>
__global__ void __launch_bounds__((NO + 2 * Halo2<SET, CPL>::HL))
k_step2d(const S* __restrict__ fin, S* __restrict__ fout, const DomDev* __restrict__ doms,
         const WorkItem* __restrict__ items, int nitems, MacroRec<M> rec) {
  using V = Vel<0>;
  using SH = Shells<2, SET>;
  constexpr int Q = V::Q;
  constexpr int R = SH::R;
  constexpr int HX = Halo2<SET, CPL>::HX;
  constexpr int HL = Halo2<SET, CPL>::HL;
  constexpr int RING = 2 * R + 2;
  constexpr int NSLOT = R + 1;
  constexpr int WIDTH = CPL * NO + 2 * HX;  // ring row length (sites)

  __shared__ M psis[RING * WIDTH];

  // XCD-aware mapping: consecutive workgroup ids go to different XCDs (round robin over 8),
  // so give XCD k the k-th contiguous eighth of the item list.
  const int per = (nitems + 7) >> 3;
  const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (item >= nitems) return;
  const WorkItem it = items[item];
  const DomDev& dm = doms[it.dom];
  const int nx = dm.nx, ny = dm.ny;
  const long long cells = (long long)nx * ny;
  const S* __restrict__ fb = fin + dm.off * Q;
  S* __restrict__ ob = fout + dm.off * Q;
  const M omega = M(dm.omega), kappa = M(dm.kappa), gpre = M(dm.gpre);
  const M eps = M(dm.eps), inv_eps = M(dm.inv_eps), rho0 = M(dm.rho0);
  const int kind = dm.psi_kind;
  M Wv[SH::NS];
#pragma unroll
  for (int s = 0; s < SH::NS; ++s) Wv[s] = M(dm.W[s]);

  // lane -> first site X of the lane and its position q in a ring row
  const int lane = threadIdx.x;
  int X, q;
  if (lane < NO) {
    X = it.x0 + CPL * lane;
    q = HX + CPL * lane;
  } else if (lane < NO + HL) {
    X = it.x0 - HX + CPL * (lane - NO);
    q = CPL * (lane - NO);
  } else {
    X = it.x0 + CPL * NO + CPL * (lane - NO - HL);
    q = HX + CPL * NO + CPL * (lane - NO - HL);
  }
  const int xend = min(it.x0 + CPL * NO, nx);     // end of this strip's outputs
  const bool outl = lane < NO && X < xend;
  const bool need = X < xend + HX;                 // psi of this lane is read by an output
  const int xw = wrapi(X, nx);

  const int dir = it.dir;
  const int total = (it.y1 - it.y0) + 2 * R;
  const int rstart = dir > 0 ? it.y0 - R : it.y1 - 1 + R;
  const int rbase = it.y0 - R - RING;              // ring row of row r: (r - rbase) % RING
  // Strips whose pulls never cross the periodic seam in x (all but the first and last of a
  // domain) take a branch-free path; the others resolve the seam per lane.
  const bool seam = it.x0 - HX - 1 < 0 || it.x0 + CPL * NO + HX + 1 > nx;
  auto march = [&](auto SEAM) {
  constexpr bool WRAP = decltype(SEAM)::value;
  M fr[NSLOT][Q][CPL];

  for (int k0 = 0; k0 < total; k0 += NSLOT) {
    static_for<NSLOT>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int k = k0 + j;
      if (k < total) {
        const int r = rstart + dir * k;
        // ---------------- 1. pull row r, psi into the ring
        if (need) {
          const int rw = wrapi(r, ny), rm = wrapi(r - 1, ny), rp = wrapi(r + 1, ny);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const int cy = V::cy(i), cx = V::cx(i);
            const int srow = cy == 1 ? rm : (cy == -1 ? rp : rw);
            ld_shift<S, M, CPL, WRAP>(fb + (long long)i * cells + (long long)srow * nx, xw, nx, -cx, fr[j][i]);
          }
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            M sum = M(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) sum += fr[j][i][c];
            const M n = SHIFT ? rho0 + sum : sum;
            psis[((r - rbase) % RING) * WIDTH + q + c] = psi_eval<M>(n, kind, eps, inv_eps);
          }
        }
        __syncthreads();

        // ---------------- 2. collide row crow = r - R (marching order), output lanes only
        if (k >= 2 * R && outl) {
          constexpr int js = (j + NSLOT - R) % NSLOT;  // register set of that row
          const int crow = r - dir * R;
          int so[2 * R + 1];                           // ring row of crow + dy, dy = o - R
#pragma unroll
          for (int o = 0; o <= 2 * R; ++o) so[o] = ((crow - R + o - rbase) % RING) * WIDTH;
          const long long o_ = (long long)wrapi(crow, ny) * nx + xw;
          M out[Q][CPL];
          M recv[5][CPL];
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            const int qc = q + c;
            const M psic = psis[so[R] + qc];
            // force of eq. (sc_f) over +-pairs, summed shell by shell before the weight
            M dxs[SH::NS], dys[SH::NS];
#pragma unroll
            for (int s = 0; s < SH::NS; ++s) { dxs[s] = M(0); dys[s] = M(0); }
#pragma unroll
            for (int h = 0; h < SH::NH; ++h) {
              const HalfVec hv = SH::h(h);
              const M d = psis[so[R + hv.y] + qc + hv.x] - psis[so[R - hv.y] + qc - hv.x];
              if (hv.x != 0) dxs[hv.slot] += M(hv.x) * d;
              if (hv.y != 0) dys[hv.slot] += M(hv.y) * d;
            }
            M ax = M(0), ay = M(0);
#pragma unroll
            for (int s = 0; s < SH::NS; ++s) { ax += Wv[s] * dxs[s]; ay += Wv[s] * dys[s]; }
            const M Fx = gpre * psic * ax;
            const M Fy = gpre * psic * ay;
            M f[Q];
            M sum = M(0), jx = M(0), jy = M(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
              f[i] = fr[js][i][c];
              sum += f[i];
              if (V::cx(i) != 0) jx += M(V::cx(i)) * f[i];
              if (V::cy(i) != 0) jy += M(V::cy(i)) * f[i];
            }
            const M nn = SHIFT ? rho0 + sum : sum;
            const M inv_n = rcp<M>(nn);
            const M ux = (jx + M(0.5) * Fx) * inv_n;
            const M uy = (jy + M(0.5) * Fy) * inv_n;
            M fo[Q];
            collide<0, M>(f, SHIFT ? sum : nn, nn, ux, uy, M(0), Fx, Fy, M(0), omega, kappa, fo);
#pragma unroll
            for (int i = 0; i < Q; ++i) out[i][c] = fo[i];
            if (REC) {
              recv[0][c] = nn; recv[1][c] = jx; recv[2][c] = jy; recv[3][c] = Fx; recv[4][c] = Fy;
            }
          }
#pragma unroll
          for (int i = 0; i < Q; ++i) stv<S, M, CPL>(ob + (long long)i * cells + o_, out[i]);
          if (REC) {
            const long long g = dm.off + o_;
            stv<M, M, CPL>(rec.n + g, recv[0]);
            stv<M, M, CPL>(rec.j + g, recv[1]);
            stv<M, M, CPL>(rec.j + rec.cells + g, recv[2]);
            stv<M, M, CPL>(rec.F + g, recv[3]);
            stv<M, M, CPL>(rec.F + rec.cells + g, recv[4]);
          }
        }
      }
    });
  }
  };
  if (seam) march(std::true_type{});
  else march(std::false_type{});
}

}  // namespace scl
