// Adjoint (reverse-mode derivative) of the fused D2Q9 step, for gradients of a loss L of the
// final state with respect to the shell weights W and the coupling G.
//
// Forward step (per site y, time t):   f*_i(y) = (1-omega) f_i + omega f_i^eq(n, u) + S_i(u, F),
//   n = sum f, j = sum f xi, u = (j + F/2)/n, F(y) = -G c^2 psi(y) sum_a W_a psi(y + e_a) e_a,
//   f_i^{t+1}(y + xi_i) = f*_i(y).
// With lambda^t_i(y) = dL/df^t_i(y) and mu_i(y) = lambda^{t+1}_i(y + xi_i) = dL/df*_i(y):
//   moments of mu:  m0 = sum w_i mu_i, m1 = sum w_i mu_i xi, m2 = sum w_i mu_i xi xi
//   V    = 3 m1 + 9 m2.u - 3 m0 u                     (sum mu_i w_i dP_i/du, P_i = f^eq_i/(w_i n))
//   ubar = omega n V + kappa (9 m2.F - 3 m0 F)         dL/du
//   Fbar = kappa V + ubar / (2n) - kappa aff (9 m2.F - 3 m0 F)   dL/dF(y) (the last term: the F^2
//                                                                part of the Guo tensor, aff = A/tau)
//   nbar_loc = omega (m0 + 3 m1.u + 4.5 u.m2.u - 1.5 u.u m0) - ubar.u / n
//   jbar = ubar / n
//   psibar(y) = Fbar(y).F(y)/psi(y) + G c^2 sum_a W_a psi(y + e_a) Fbar(y + e_a).e_a
//             (the forward stencil applied to psi Fbar; W_{-a} = W_a, e_{-a} = -e_a)
//   lambda^t_k(y) = (1-omega) mu_k(y) + nbar_loc + psi'(n) psibar + xi_k.jbar
//   dL/dW_s += sum_y Fbar(y).(-G c^2 psi(y) sum_{a in s} psi(y + e_a) e_a)
//   dL/dG   += sum_y Fbar(y).F(y)/G = sum_y Fbar(y).(-c^2 psi(y) sum_a W_a psi(y + e_a) e_a)
// The step's fields n, j, F come from a recompute pass of the forward kernel (REC mode).
//
// The kernel marches rows like the forward kernel: row r computes Fbar and psi for every lane
// (outputs and R halo lanes on each side) into LDS rings; row r - R then gathers psibar and
// writes lambda^t. Gradient partials are accumulated per work item in double, in a fixed order,
// with no atomics.
#pragma once
#include "scl_common.hpp"

namespace scl {

struct AdjointState {
  void* pool = nullptr;        // checkpoints: states at steps 0, K, 2K, ... and the final one
  size_t pool_bytes = 0;
  int nckpt = 0;
  int every = 0;
  long long nsteps = 0;        // steps of the checkpointed forward
  bool valid = false;          // a checkpointed forward was run and the state is unchanged
  void* rec = nullptr;         // per-step n, j, F of one segment
  size_t rec_bytes = 0;
  void* lam[2] = {nullptr, nullptr};  // adjoint populations (A/B)
  size_t lam_bytes = 0;
  double* gpart = nullptr;     // per work item gradient partials
  size_t gpart_cap = 0;
  long long end_step = 0;      // step counter after the checkpointed forward
  int lam_cur = 0;             // buffer holding lambda after the last scl_adjoint
};


// lambda_i(x) = seed(x) for every i (a loss that depends on the final state through n only)
// or the given populations (natural layout, [Q][cells] per domain).
template <class M>
__global__ void k_adj_seed(M* __restrict__ lam, const double* __restrict__ seed_n, const double* __restrict__ seed_f,
                           DomDev dm, int Q) {
  const long long cells = (long long)dm.nx * dm.ny * dm.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  M* lb = lam + dm.off * Q;
  for (int i = 0; i < Q; ++i) {
    double v = 0.0;
    if (seed_n) v += seed_n[dm.off + c];
    if (seed_f) v += seed_f[dm.off * Q + (long long)i * cells + c];
    lb[(long long)i * cells + c] = static_cast<M>(v);
  }
}

template <class M>
__global__ void k_adj_get(const M* __restrict__ lam, double* __restrict__ out, long long n) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) out[c] = static_cast<double>(lam[c]);
}

constexpr int ADJ_MAXS = MAX_SHELLS;  // weight slots per domain

template <class M, int SET, int NO>
__global__ void __launch_bounds__((NO + 2 * Shells<2, SET>::R))
k_adjoint2d(const M* __restrict__ lin, M* __restrict__ lout, const M* __restrict__ rn, const M* __restrict__ rj,
            const M* __restrict__ rF, long long rcells, const DomDev* __restrict__ doms,
            const WorkItem* __restrict__ items, int nitems, double* __restrict__ gpart, int accumulate) {
  using V = Vel<0>;
  using SH = Shells<2, SET>;
  constexpr int Q = V::Q;
  constexpr int R = SH::R;
  constexpr int NS = SH::NS;
  constexpr int RING = 2 * R + 2;
  constexpr int NSLOT = R + 1;
  constexpr int WIDTH = NO + 2 * R;
  constexpr int NT = NO + 2 * R;

  __shared__ M rpsi[RING * WIDTH];
  __shared__ M rpx[RING * WIDTH];
  __shared__ M rpy[RING * WIDTH];
  __shared__ double red[NS + 1][NT];

  const int per = (nitems + 7) >> 3;
  const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (item >= nitems) return;
  const WorkItem it = items[item];
  const DomDev& dm = doms[it.dom];
  const int nx = dm.nx, ny = dm.ny;
  const long long cells = (long long)nx * ny;
  const M* __restrict__ lb = lin + dm.off * Q;
  M* __restrict__ ob = lout + dm.off * Q;
  const M omega = M(dm.omega), kappa = M(dm.kappa), gpre = M(dm.gpre), aff = M(dm.aff);
  const M eps = M(dm.eps), inv_eps = M(dm.inv_eps);
  const int kind = dm.psi_kind;
  M Wv[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) Wv[s] = M(dm.W[s]);

  const int lane = threadIdx.x;
  int X, q;
  if (lane < NO) { X = it.x0 + lane; q = R + lane; }
  else if (lane < NO + R) { X = it.x0 - R + (lane - NO); q = lane - NO; }
  else { X = it.x0 + NO + (lane - NO - R); q = R + NO + (lane - NO - R); }
  const int xend = min(it.x0 + NO, nx);
  const bool outl = lane < NO && X < xend;
  const bool need = X < xend + R;
  const int xw = wrapi(X, nx), xm = wrapi(X - 1, nx), xp = wrapi(X + 1, nx);

  double gW[NS], gG = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) gW[s] = 0.0;

  const int dir = it.dir;
  const int total = (it.y1 - it.y0) + 2 * R;
  const int rstart = dir > 0 ? it.y0 - R : it.y1 - 1 + R;
  const int rbase = it.y0 - R - RING;

  // per row kept until its gather: mu (Q), nbar_loc, jbar (2), Fbar (2), F (2), n, psi
  M mu[NSLOT][Q];
  M keep[NSLOT][9];

  for (int k0 = 0; k0 < total; k0 += NSLOT) {
    static_for<NSLOT>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int k = k0 + j;
      if (k < total) {
        const int r = rstart + dir * k;
        if (need) {
          const int rw = wrapi(r, ny), rm = wrapi(r - 1, ny), rp = wrapi(r + 1, ny);
          // mu_i(y) = lambda^{t+1}_i(y + xi_i)
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const int cx = V::cx(i), cy = V::cy(i);
            const int srow = cy == 1 ? rp : (cy == -1 ? rm : rw);
            const int scol = cx == 1 ? xp : (cx == -1 ? xm : xw);
            mu[j][i] = lb[(long long)i * cells + (long long)srow * nx + scol];
          }
          const long long g = dm.off + (long long)rw * nx + xw;
          const M n = rn[g], jx = rj[g], jy = rj[rcells + g], Fx = rF[g], Fy = rF[rcells + g];
          const M psi = psi_eval<M>(n, kind, eps, inv_eps);
          const M inv_n = M(1) / n;
          const M ux = (jx + M(0.5) * Fx) * inv_n, uy = (jy + M(0.5) * Fy) * inv_n;
          M m0 = M(0), m1x = M(0), m1y = M(0), mxx = M(0), mxy = M(0), myy = M(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const M wm = M(V::w(i)) * mu[j][i];
            const int cx = V::cx(i), cy = V::cy(i);
            m0 += wm;
            if (cx) { m1x += M(cx) * wm; mxx += wm; }
            if (cy) { m1y += M(cy) * wm; myy += wm; }
            if (cx && cy) mxy += M(cx * cy) * wm;
          }
          const M m2ux = mxx * ux + mxy * uy, m2uy = mxy * ux + myy * uy;
          const M Vx = M(3) * m1x + M(9) * m2ux - M(3) * m0 * ux;
          const M Vy = M(3) * m1y + M(9) * m2uy - M(3) * m0 * uy;
          const M Tx = M(9) * (mxx * Fx + mxy * Fy) - M(3) * m0 * Fx;
          const M Ty = M(9) * (mxy * Fx + myy * Fy) - M(3) * m0 * Fy;
          const M ubx = omega * n * Vx + kappa * Tx, uby = omega * n * Vy + kappa * Ty;
          const M Fbx = kappa * Vx + M(0.5) * ubx * inv_n - kappa * aff * Tx;
          const M Fby = kappa * Vy + M(0.5) * uby * inv_n - kappa * aff * Ty;
          const M uu = ux * ux + uy * uy;
          const M An = omega * (m0 + M(3) * (m1x * ux + m1y * uy) + M(4.5) * (ux * m2ux + uy * m2uy) -
                                M(1.5) * uu * m0);
          const M nbl = An - (ubx * ux + uby * uy) * inv_n;
          keep[j][0] = nbl;
          keep[j][1] = ubx * inv_n;
          keep[j][2] = uby * inv_n;
          keep[j][3] = Fbx;
          keep[j][4] = Fby;
          keep[j][5] = Fx;
          keep[j][6] = Fy;
          keep[j][7] = n;
          keep[j][8] = psi;
          const int sl = ((r - rbase) % RING) * WIDTH + q;
          rpsi[sl] = psi;
          rpx[sl] = psi * Fbx;
          rpy[sl] = psi * Fby;
        }
        __syncthreads();

        if (k >= 2 * R && outl) {
          constexpr int js = (j + NSLOT - R) % NSLOT;
          const int crow = r - dir * R;
          int so[2 * R + 1];
#pragma unroll
          for (int o = 0; o <= 2 * R; ++o) so[o] = ((crow - R + o - rbase) % RING) * WIDTH;
          M dxs[NS], dys[NS], gsum[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) { dxs[s] = M(0); dys[s] = M(0); gsum[s] = M(0); }
#pragma unroll
          for (int h = 0; h < SH::NH; ++h) {
            const HalfVec hv = SH::h(h);
            const int ip = so[R + hv.y] + q + hv.x, im = so[R - hv.y] + q - hv.x;
            const M d = rpsi[ip] - rpsi[im];
            if (hv.x != 0) { dxs[hv.slot] += M(hv.x) * d; gsum[hv.slot] += M(hv.x) * (rpx[ip] - rpx[im]); }
            if (hv.y != 0) { dys[hv.slot] += M(hv.y) * d; gsum[hv.slot] += M(hv.y) * (rpy[ip] - rpy[im]); }
          }
          const M nbl = keep[js][0], jbx = keep[js][1], jby = keep[js][2];
          const M Fbx = keep[js][3], Fby = keep[js][4], Fx = keep[js][5], Fy = keep[js][6];
          const M n = keep[js][7], psi = keep[js][8];
          M gath = M(0);
#pragma unroll
          for (int s = 0; s < NS; ++s) gath += Wv[s] * gsum[s];
          const M psibar = (Fbx * Fx + Fby * Fy) / psi - gpre * gath;
          const M nbar = nbl + dpsi_eval<M>(n, psi, kind, eps) * psibar;
          const long long o_ = (long long)wrapi(crow, ny) * nx + xw;
          const M om1 = M(1) - omega;
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            M v = om1 * mu[js][i] + nbar;
            if (V::cx(i)) v += M(V::cx(i)) * jbx;
            if (V::cy(i)) v += M(V::cy(i)) * jby;
            ob[(long long)i * cells + o_] = v;
          }
          M accG = M(0);
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const M a = dxs[s] * Fbx + dys[s] * Fby;
            gW[s] += (double)(gpre * psi * a);
            accG += Wv[s] * a;
          }
          gG += (double)(-M(1.0 / 3.0) * psi * accG);
        }
      }
    });
  }

  // fixed-order workgroup reduction of the gradient partials
#pragma unroll
  for (int s = 0; s < NS; ++s) red[s][lane] = gW[s];
  red[NS][lane] = gG;
  __syncthreads();
  if (lane < NS + 1) {
    double acc = 0.0;
    for (int l = 0; l < NT; ++l) acc += red[lane][l];
    // row of ADJ_MAXS + 1 values per item: weight slots, then dL/dG in the last column
    double* gp = gpart + (long long)item * (ADJ_MAXS + 1) + (lane < NS ? lane : ADJ_MAXS);
    *gp = accumulate ? *gp + acc : acc;
  }
}

}  // namespace scl
