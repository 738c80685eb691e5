// Fused D3Q19 Shan-Chen step (2.5-D blocking): one workgroup owns a TX x TY tile of lanes
// (its central (TX - 2R) x (TY - 2R) sites are outputs, the R-wide rim only supplies psi) and
// marches along z. At every plane it pulls the 19 populations streaming into the tile,
// stores psi(n) in a ring of 2R + 2 planes in LDS and collides the plane R behind, whose
// populations wait in registers (rotation of R + 1 register sets). Same arithmetic as the
// 2D kernel: force of eq. (sc_f) over +-pairs, eqs. (f_eq), (GuoForcing), (lbm), (omega_i).
#pragma once
#include "scl_common.hpp"

namespace scl {

// One vector of every +-pair of the 3D shell sets: the first non-zero component in the
// order (z, y, x) is positive.
struct Half3Table {
  HalfVec v[MAX_HALF_3D];
  int n;
};

__host__ __device__ constexpr int abs_i(int a) { return a < 0 ? -a : a; }

__host__ __device__ constexpr Half3Table make_half3(int set) {
  Half3Table t{};
  t.n = 0;
  constexpr int gens[7][3] = {{0, 0, 1}, {0, 1, 1}, {1, 1, 1}, {0, 0, 2}, {0, 1, 2}, {1, 1, 2}, {0, 2, 2}};
  const int ncodes = set == 0 ? 3 : 7;
  for (int s = 0; s < ncodes; ++s) {
    for (int z = -2; z <= 2; ++z)
      for (int y = -2; y <= 2; ++y)
        for (int x = -2; x <= 2; ++x) {
          int a = abs_i(x), b = abs_i(y), c = abs_i(z);
          // sort a <= b <= c
          if (a > b) { int q = a; a = b; b = q; }
          if (b > c) { int q = b; b = c; c = q; }
          if (a > b) { int q = a; a = b; b = q; }
          if (a != gens[s][0] || b != gens[s][1] || c != gens[s][2]) continue;
          const bool pos = z > 0 || (z == 0 && (y > 0 || (y == 0 && x > 0)));
          if (!pos) continue;
          t.v[t.n] = HalfVec{(int8_t)x, (int8_t)y, (int8_t)z, (int8_t)s};
          t.n++;
        }
  }
  return t;
}

template <> struct Shells<3, 0> {
  static constexpr int R = 1, NH = 13, NS = 3;
  __host__ __device__ static constexpr int code(int s) { constexpr int c[3] = {1, 2, 3}; return c[s]; }
  __host__ __device__ static constexpr HalfVec h(int k) {
    constexpr Half3Table t = make_half3(0);
    return t.v[k];
  }
};

template <> struct Shells<3, 1> {
  static constexpr int R = 2, NH = 46, NS = 7;
  __host__ __device__ static constexpr int code(int s) {
    constexpr int c[7] = {1, 2, 3, 4, 5, 6, 8};
    return c[s];
  }
  __host__ __device__ static constexpr HalfVec h(int k) {
    constexpr Half3Table t = make_half3(1);
    return t.v[k];
  }
};

static_assert(make_half3(0).n == 13, "3D reach-1 half list");
static_assert(make_half3(1).n == 46, "3D reach-2 half list");

template <class S, class M, int SET, int TX, int TY, bool SHIFT>
__global__ void __launch_bounds__(TX * TY)
k_step3d(const S* __restrict__ fin, S* __restrict__ fout, const DomDev* __restrict__ doms,
         const WorkItem* __restrict__ items) {
  using V = Vel<1>;
  using SH = Shells<3, SET>;
  constexpr int Q = V::Q;
  constexpr int R = SH::R;
  constexpr int RING = 2 * R + 2;
  constexpr int NSLOT = R + 1;
  constexpr int NT = TX * TY;

  __shared__ M psis[RING][NT];

  const WorkItem it = items[blockIdx.x];
  const DomDev& dm = doms[it.dom];
  const int nx = dm.nx, ny = dm.ny, nz = dm.nz;
  const long long plane = (long long)nx * ny;
  const long long cells = plane * nz;
  const S* __restrict__ fb = fin + dm.off * Q;
  S* __restrict__ ob = fout + dm.off * Q;
  const M omega = M(dm.omega), kappa = M(dm.kappa), gpre = M(dm.gpre);
  const M eps = M(dm.eps), inv_eps = M(dm.inv_eps), rho0 = M(dm.rho0);
  const int kind = dm.psi_kind;
  M Wv[SH::NS];
#pragma unroll
  for (int s = 0; s < SH::NS; ++s) Wv[s] = M(dm.W[s]);

  const int lane = threadIdx.x;
  const int tx = lane % TX, ty = lane / TX;
  const int gx = it.x0 - R + tx, gy = it.y0 - R + ty;
  const int xw = wrapi(gx, nx), xm = wrapi(gx - 1, nx), xp = wrapi(gx + 1, nx);
  const int yw = wrapi(gy, ny), ym = wrapi(gy - 1, ny), yp = wrapi(gy + 1, ny);
  const bool outl = tx >= R && tx < TX - R && ty >= R && ty < TY - R && gx < nx && gy < ny;

  const int total = (it.z1 - it.z0) + 2 * R;
  M fr[NSLOT][Q];

  for (int k0 = 0; k0 < total; k0 += NSLOT) {
    static_for<NSLOT>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int k = k0 + j;
      if (k < total) {
        const int zp_ = it.z0 - R + k;
        const long long zw = (long long)wrapi(zp_, nz) * plane;
        const long long zm = (long long)wrapi(zp_ - 1, nz) * plane;
        const long long zpp = (long long)wrapi(zp_ + 1, nz) * plane;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int cx = V::cx(i), cy = V::cy(i), cz = V::cz(i);
          const long long sz = cz == 1 ? zm : (cz == -1 ? zpp : zw);
          const int sy = cy == 1 ? ym : (cy == -1 ? yp : yw);
          const int sx = cx == 1 ? xm : (cx == -1 ? xp : xw);
          fr[j][i] = ld<S, M>(fb + (long long)i * cells + sz + (long long)sy * nx + sx);
        }
        {
          M sum = M(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) sum += fr[j][i];
          const M n = SHIFT ? rho0 + sum : sum;
          psis[k % RING][lane] = psi_eval<M>(n, kind, eps, inv_eps);
        }
        __syncthreads();

        if (k >= 2 * R && outl) {
          constexpr int js = (j + 1) % NSLOT;
          const int c = zp_ - R;
          int so[2 * R + 1];
#pragma unroll
          for (int o = 0; o <= 2 * R; ++o) so[o] = (k - 2 * R + o) % RING;
          const M psic = psis[so[R]][lane];
          M dxs[SH::NS], dys[SH::NS], dzs[SH::NS];
#pragma unroll
          for (int s = 0; s < SH::NS; ++s) { dxs[s] = M(0); dys[s] = M(0); dzs[s] = M(0); }
#pragma unroll
          for (int h = 0; h < SH::NH; ++h) {
            const HalfVec hv = SH::h(h);
            const int dl = hv.y * TX + hv.x;
            const M d = psis[so[R + hv.z]][lane + dl] - psis[so[R - hv.z]][lane - dl];
            if (hv.x != 0) dxs[hv.slot] += M(hv.x) * d;
            if (hv.y != 0) dys[hv.slot] += M(hv.y) * d;
            if (hv.z != 0) dzs[hv.slot] += M(hv.z) * d;
          }
          M ax = M(0), ay = M(0), az = M(0);
#pragma unroll
          for (int s = 0; s < SH::NS; ++s) { ax += Wv[s] * dxs[s]; ay += Wv[s] * dys[s]; az += Wv[s] * dzs[s]; }
          const M Fx = gpre * psic * ax, Fy = gpre * psic * ay, Fz = gpre * psic * az;

          M sum = M(0), jx = M(0), jy = M(0), jz = M(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const M f = fr[js][i];
            sum += f;
            if (V::cx(i) != 0) jx += M(V::cx(i)) * f;
            if (V::cy(i) != 0) jy += M(V::cy(i)) * f;
            if (V::cz(i) != 0) jz += M(V::cz(i)) * f;
          }
          const M nn = SHIFT ? rho0 + sum : sum;
          const M inv_n = rcp<M>(nn);
          const M ux = (jx + M(0.5) * Fx) * inv_n;
          const M uy = (jy + M(0.5) * Fy) * inv_n;
          const M uz = (jz + M(0.5) * Fz) * inv_n;
          const long long o = (long long)wrapi(c, nz) * plane + (long long)yw * nx + xw;
          M fo[Q];
          collide<1, M>(fr[js], SHIFT ? sum : nn, nn, ux, uy, uz, Fx, Fy, Fz, omega, kappa, fo);
#pragma unroll
          for (int i = 0; i < Q; ++i) st<S, M>(ob + (long long)i * cells + o, fo[i]);
        }
      }
    });
  }
}

}  // namespace scl
