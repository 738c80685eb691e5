// Fused D2Q9 Shan-Chen step: pull-stream, moments, psi, wide-stencil force, BGK + Guo
// collision, in one pass over the populations.
//
// Work decomposition. One workgroup of NT lanes owns a strip of NT - 2R output columns
// (R = stencil reach) and marches down a range of rows. Lane l sits on column
// x0 - R + l, so the outer R lanes on each side only supply psi to their neighbours. At
// every row r the workgroup
//   1. pulls the nine post-collision populations that stream into row r
//      (f_i(x, t) = f*_i(x - xi_i, t-1)), adds them to n and stores psi(n) in a ring of
//      2R + 2 rows held in LDS;
//   2. once the rows r - 2R .. r are in the ring, collides row r - R: the force of eq. (sc_f)
//      over the +-pairs of the stencil reads psi from the ring, then u = (j + F/2)/n, the
//      equilibrium of eq. (f_eq), the Guo term of eq. (GuoForcing) and the BGK update of
//      eqs. (lbm), (omega_i) give the new post-collision values, written in place (x) of the
//      output buffer. The populations of a row stay in registers for the R rows between
//      their load and their collision (a rotation of R + 1 register sets, unrolled).
// Each population is read once and written once per step; the only extra traffic is the
// 2R halo rows at the ends of a row range and the 2R halo columns of a strip, which the
// neighbouring workgroups also read (L2 / Infinity Cache hits).
#pragma once
#include "scl_common.hpp"

namespace scl {

template <class S, class M, int SET, int NT, bool SHIFT, bool REC>
__global__ void __launch_bounds__(NT)
k_step2d(const S* __restrict__ fin, S* __restrict__ fout, const DomDev* __restrict__ doms,
         const WorkItem* __restrict__ items, MacroRec<M> rec) {
  using V = Vel<0>;
  using SH = Shells<2, SET>;
  constexpr int Q = V::Q;
  constexpr int R = SH::R;
  constexpr int RING = 2 * R + 2;
  constexpr int NSLOT = R + 1;
  constexpr M inv_cs2 = M(3);
  constexpr M half_inv_cs4 = M(4.5);

  __shared__ M psis[RING][NT];

  const WorkItem it = items[blockIdx.x];
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

  const int lane = threadIdx.x;
  const int gx = it.x0 - R + lane;
  const int xw = wrapi(gx, nx), xm = wrapi(gx - 1, nx), xp = wrapi(gx + 1, nx);
  const bool outl = (lane >= R) && (lane < NT - R) && (gx < nx);

  const int total = (it.y1 - it.y0) + 2 * R;
  M fr[NSLOT][Q];

  for (int k0 = 0; k0 < total; k0 += NSLOT) {
    static_for<NSLOT>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int k = k0 + j;
      if (k < total) {
        // ---------------- 1. pull row r, psi into the ring
        const int r = it.y0 - R + k;
        const int rw = wrapi(r, ny), rm = wrapi(r - 1, ny), rp = wrapi(r + 1, ny);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int cy = V::cy(i), cx = V::cx(i);
          const int srow = cy == 1 ? rm : (cy == -1 ? rp : rw);
          const int scol = cx == 1 ? xm : (cx == -1 ? xp : xw);
          fr[j][i] = ld<S, M>(fb + (long long)i * cells + (long long)srow * nx + scol);
        }
        {
          M sum = M(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) sum += fr[j][i];
          const M n = SHIFT ? rho0 + sum : sum;
          psis[k % RING][lane] = psi_eval<M>(n, kind, eps, inv_eps);
        }
        __syncthreads();

        // ---------------- 2. collide row c = r - R (output lanes only)
        if (k >= 2 * R && outl) {
          constexpr int js = (j + 1) % NSLOT;  // slot loaded R iterations ago
          const int c = r - R;
          int so[2 * R + 1];                   // ring slot of row c + dy, dy = o - R
#pragma unroll
          for (int o = 0; o <= 2 * R; ++o) so[o] = (k - 2 * R + o) % RING;
          const M psic = psis[so[R]][lane];
          M ax = M(0), ay = M(0);
#pragma unroll
          for (int h = 0; h < SH::NH; ++h) {
            const HalfVec hv = SH::h(h);
            const M d = psis[so[R + hv.y]][lane + hv.x] - psis[so[R - hv.y]][lane - hv.x];
            const M wd = Wv[hv.slot] * d;
            if (hv.x != 0) ax += M(hv.x) * wd;
            if (hv.y != 0) ay += M(hv.y) * wd;
          }
          const M Fx = gpre * psic * ax;
          const M Fy = gpre * psic * ay;

          M sum = M(0), jx = M(0), jy = M(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const M f = fr[js][i];
            sum += f;
            if (V::cx(i) != 0) jx += M(V::cx(i)) * f;
            if (V::cy(i) != 0) jy += M(V::cy(i)) * f;
          }
          const M nn = SHIFT ? rho0 + sum : sum;
          const M inv_n = M(1) / nn;
          const M ux = (jx + M(0.5) * Fx) * inv_n;
          const M uy = (jy + M(0.5) * Fy) * inv_n;
          const M uu15 = M(1.5) * (ux * ux + uy * uy);  // u.u / (2 c^2)
          const M uF3 = M(3) * (ux * Fx + uy * Fy);     // c^2 u.F / c^4
          const long long o = (long long)wrapi(c, ny) * nx + xw;
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const int cx = V::cx(i), cy = V::cy(i);
            const M w = M(V::w(i));
            const M xu = M(cx) * ux + M(cy) * uy;
            const M xF = M(cx) * Fx + M(cy) * Fy;
            // f_eq = w n (1 + poly); with shifted storage the stored value is f - w rho0 and
            // its equilibrium w (n - rho0) + w n poly, formed without cancellation.
            const M poly = inv_cs2 * xu + half_inv_cs4 * xu * xu - uu15;
            const M feq = SHIFT ? w * (sum + nn * poly) : w * nn * (M(1) + poly);
            const M src = kappa * w * (inv_cs2 * xF + M(9) * xu * xF - uF3);
            const M f = fr[js][i];
            st<S, M>(ob + (long long)i * cells + o, f - omega * (f - feq) + src);
          }
          if (REC) {
            const long long g = dm.off + o;
            rec.n[g] = nn;
            rec.j[g] = jx; rec.j[rec.cells + g] = jy;
            rec.F[g] = Fx; rec.F[rec.cells + g] = Fy;
          }
        }
      }
    });
  }
}

}  // namespace scl
