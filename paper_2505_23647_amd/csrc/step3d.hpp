// D3Q19 Shan-Chen step in two passes: a density/psi pass over every site, then a fused
// force + collision + streaming pass that reads psi from LDS-staged tiles. (A single fused
// pass, as in 2D, would have to recompute psi on a rim around every tile and hold R + 1
// planes of 19 populations per lane in registers; in 3D that costs more than the 4 + 4 bytes
// per site of the psi array.)
#pragma once
#include "scl_common.hpp"



// minimum waves per SIMD the 3D step is compiled for (0: no bound beyond the block size)
#ifndef SCL_STEP3D_WPE
#define SCL_STEP3D_WPE 0
#endif
#if SCL_STEP3D_WPE > 0
#define SCL_STEP3D_ATTR __attribute__((amdgpu_waves_per_eu(SCL_STEP3D_WPE, SCL_STEP3D_WPE)))
#else
#define SCL_STEP3D_ATTR
#endif

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
  // generators (sorted absolute components) in slot order: 1, 2, 3, 4, 5, 6, 8, then the
  // reach-4 shells 9 = (2,2,1), 1009 = (3,0,0), 16 = (4,0,0), 18 = (3,3,0)
  constexpr int gens[11][3] = {{0, 0, 1}, {0, 1, 1}, {1, 1, 1}, {0, 0, 2}, {0, 1, 2}, {1, 1, 2},
                               {0, 2, 2}, {1, 2, 2}, {0, 0, 3}, {0, 0, 4}, {0, 3, 3}};
  const int ncodes = set == 0 ? 3 : (set == 1 ? 7 : 11);
  const int r = set == 2 ? 4 : 2;
  for (int s = 0; s < ncodes; ++s) {
    for (int z = -r; z <= r; ++z)
      for (int y = -r; y <= r; ++y)
        for (int x = -r; x <= r; ++x) {
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

// the shells of the 3D Tolman-length tuning table: R_F = 4, 140 vectors
template <> struct Shells<3, 2> {
  static constexpr int R = 4, NH = 70, NS = 11;
  __host__ __device__ static constexpr int code(int s) {
    constexpr int c[11] = {1, 2, 3, 4, 5, 6, 8, 9, 1009, 16, 18};
    return c[s];
  }
  __host__ __device__ static constexpr HalfVec h(int k) {
    constexpr Half3Table t = make_half3(2);
    return t.v[k];
  }
};

static_assert(make_half3(0).n == 13, "3D reach-1 half list");
static_assert(make_half3(1).n == 46, "3D reach-2 half list");
static_assert(make_half3(2).n == 70, "3D reach-4 half list");

// ------------------------------------------------------------------ pass 1: density and psi
// psi(x) = psi(n(x)) with n(x) = sum_i f_i(x) = sum_i A_i[x - xi_i] (the populations streaming
// into x). One lane per site of one x-row chunk of a domain; grid (x chunks, ny, nz).
template <class S, class M, bool SHIFT>
__global__ void __launch_bounds__(256)
k_psi3d(const S* __restrict__ fin, M* __restrict__ psi, DomDev dm) {
  using V = Vel<1>;
  constexpr int Q = V::Q;
  const int nx = dm.nx, ny = dm.ny, nz = dm.nz;
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= nx) return;
  const int y = blockIdx.y, z = blockIdx.z;
  const long long plane = (long long)nx * ny, cells = plane * nz;
  const S* __restrict__ fb = fin + dm.off * Q;
  const int xs[3] = {wrapi(x + 1, nx), x, wrapi(x - 1, nx)};  // [1 + cx]: x - cx
  const long long ys[3] = {(long long)wrapi(y + 1, ny) * nx, (long long)y * nx, (long long)wrapi(y - 1, ny) * nx};
  const long long zs[3] = {(long long)wrapi(z + 1, nz) * plane, (long long)z * plane, (long long)wrapi(z - 1, nz) * plane};
  M sum = M(0);
#pragma unroll
  for (int i = 0; i < Q; ++i)
    sum += static_cast<M>(fb[(long long)i * cells + zs[1 + V::cz(i)] + ys[1 + V::cy(i)] + xs[1 + V::cx(i)]]);
  const M n = SHIFT ? M(dm.rho0) + sum : sum;
  psi[dm.off + (long long)z * plane + (long long)y * nx + x] = psi_eval<M>(n, dm.psi_kind, M(dm.eps), M(dm.inv_eps));
}

// ------------------------------------------------------------------ pass 2: force, collide, stream
// One workgroup owns a TX x TY tile of output sites (one lane each; TX a multiple of 64 keeps
// every lane row of a wave on whole cache lines) and marches along a range of z. psi of the
// tile and an R-wide rim is staged plane by plane from the psi array into a ring of 2R + 2
// LDS planes; the force of eq. (sc_f) reads it there. The 19 populations of the plane being
// collided are pulled straight into registers, one plane ahead. Collision: eqs. (f_eq),
// (GuoForcing), (lbm), (omega_i), as in the 2D step. Every memory instruction is issued by
// every lane at every step (accesses with nothing to do carry an offset past the buffer's
// end), so that the compiler keeps the next plane's loads in flight.
template <class S, class M, int SET, int TX, int TY, bool SHIFT>
__global__ void __launch_bounds__(TX * TY) SCL_STEP3D_ATTR
k_step3d(const S* __restrict__ fin, S* __restrict__ fout, const M* __restrict__ psi,
         const DomDev* __restrict__ doms, const WorkItem* __restrict__ items, int nitems) {
  using V = Vel<1>;
  using SH = Shells<3, SET>;
  constexpr int Q = V::Q;
  constexpr int R = SH::R;
  constexpr int RING = 2 * R + 2;
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 2 * R, PY = TY + 2 * R;  // staged psi plane (tile + rim)
  constexpr int PN = PX * PY;
  constexpr int PL = (PN + NT - 1) / NT;            // psi values each lane stages per plane
  constexpr uint32_t OFF = 0x80000000u;

  __shared__ M ring[RING][PN];

  // XCD-aware mapping (as in the 2D step): XCD k takes the k-th contiguous eighth of the items.
  const int per = (nitems + 7) >> 3;
  const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (item >= nitems) return;
  const WorkItem it = items[item];
  const DomDev& dm = doms[it.dom];
  const int nx = dm.nx, ny = dm.ny, nz = dm.nz;
  const long long plane = (long long)nx * ny;
  const long long cells = plane * nz;
  const S* __restrict__ fb = fin + dm.off * Q;
  S* __restrict__ ob = fout + dm.off * Q;
  const M* __restrict__ pb = psi + dm.off;
  const M omega = M(dm.omega), kappa = M(dm.kappa), gpre = M(dm.gpre), rho0 = M(dm.rho0);
  const M aff = M(dm.aff);
  M Wv[SH::NS];
#pragma unroll
  for (int s = 0; s < SH::NS; ++s) Wv[s] = M(dm.W[s]);

  const int lane = threadIdx.x;
  const int tx = lane % TX, ty = lane / TX;
  const int gx = it.x0 + tx, gy = it.y0 + ty;
  const bool outl = gx < nx && gy < ny;
  const uint32_t pbytes = (uint32_t)(plane * (long long)sizeof(S));
  const uint32_t qbytes = (uint32_t)(plane * (long long)sizeof(M));
  // pull offsets within a z-plane: po[1 - cy][1 - cx] = offset of (gx - cx, gy - cy)
  uint32_t po[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      po[a][b] = outl ? (uint32_t)((long long)wrapi(gy + a - 1, ny) * nx + wrapi(gx + b - 1, nx)) * sizeof(S) : OFF;
  const uint32_t oo = outl ? (uint32_t)((long long)gy * nx + gx) * sizeof(S) : OFF;
  // psi staging: lane stages ring positions lane + NT * m of the (PX x PY) plane
  uint32_t so[PL];
#pragma unroll
  for (int m = 0; m < PL; ++m) {
    const int p = lane + NT * m;
    const int px = p % PX, py = p / PX;
    so[m] = p < PN ? (uint32_t)((long long)wrapi(it.y0 - R + py, ny) * nx + wrapi(it.x0 - R + px, nx)) * sizeof(M) : OFF;
  }

  const int dir = it.dir;
  const int total = it.z1 - it.z0;  // planes collided
  const int zstart = dir > 0 ? it.z0 : it.z1 - 1;
  const int zbase = it.z0 - R - RING - 2;  // ring slot of plane z: (z - zbase) % RING

  M fr[2][Q];   // populations of the plane being collided and of the next one
  M pv[2][PL];  // psi values being staged: plane z + R (in flight) and the next
  auto load_pops = [&](int z, bool ok, M* dst) {
    const long long zo[3] = {(long long)wrapi(z - 1, nz) * plane, (long long)wrapi(z, nz) * plane,
                             (long long)wrapi(z + 1, nz) * plane};
    const uint32_t sel = ok ? 0u : OFF;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      ldb<S, M, 1>(mkrsrc(fb + (long long)i * cells + zo[1 - V::cz(i)], pbytes), po[1 - V::cy(i)][1 - V::cx(i)] | sel, &dst[i]);
  };
  auto load_psi = [&](int z, M* dst) {
    const Rsrc rs = mkrsrc(pb + (long long)wrapi(z, nz) * plane, qbytes);
#pragma unroll
    for (int m = 0; m < PL; ++m) ldb<M, M, 1>(rs, so[m], &dst[m]);
  };
  auto put_psi = [&](int z, const M* v) {
    M* dst = ring[(z - zbase) % RING];
#pragma unroll
    for (int m = 0; m < PL; ++m)
      if (lane + NT * m < PN) dst[lane + NT * m] = v[m];
  };

  // prologue: psi planes zstart - dir R .. zstart + dir (R - 1) into the ring
  for (int d = -R; d < R; ++d) {
    load_psi(zstart + dir * d, pv[0]);
    put_psi(zstart + dir * d, pv[0]);
  }
  load_psi(zstart + dir * R, pv[0]);
  load_pops(zstart, true, fr[0]);

  for (int k0 = 0; k0 < total; k0 += 2) {
    static_for<2>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int k = k0 + j;
      const int z = zstart + dir * k;
      // start the next plane's loads, then stage psi of plane z + R
      load_psi(z + dir * (R + 1), pv[1 - j]);
      load_pops(z + dir, k + 1 < total, fr[1 - j]);
      put_psi(z + dir * R, pv[j]);
      __syncthreads();

      int sl[2 * R + 1];  // ring slots of planes z + dz, dz = o - R
#pragma unroll
      for (int o = 0; o <= 2 * R; ++o) sl[o] = (z - R + o - zbase) % RING;
      const int c0 = (ty + R) * PX + tx + R;  // this lane's site in a staged plane
      M fo[Q];
      const M psic = ring[sl[R]][c0];
      M ax = M(0), ay = M(0), az = M(0);
      // force of eq. (sc_f) over +-pairs, each difference weighted as it is read
#pragma unroll
      for (int h = 0; h < SH::NH; ++h) {
        const HalfVec hv = SH::h(h);
        const int dl = hv.y * PX + hv.x;
        const M wd = Wv[hv.slot] * (ring[sl[R + hv.z]][c0 + dl] - ring[sl[R - hv.z]][c0 - dl]);
        if (hv.x != 0) ax += M(hv.x) * wd;
        if (hv.y != 0) ay += M(hv.y) * wd;
        if (hv.z != 0) az += M(hv.z) * wd;
      }
      const M Fx = gpre * psic * ax, Fy = gpre * psic * ay, Fz = gpre * psic * az;
      M sum = M(0), jx = M(0), jy = M(0), jz = M(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const M f = fr[j][i];
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
      collide<1, M>(fr[j], SHIFT ? sum : nn, nn, ux, uy, uz, Fx, Fy, Fz, omega, kappa, aff, fo);
      const long long cz = (long long)wrapi(z, nz) * plane;
      const uint32_t sv = k < total ? oo : OFF;
#pragma unroll
      for (int i = 0; i < Q; ++i)
        stb<S, M, 1, SCL_STORE_AUX>(mkrsrc(ob + (long long)i * cells + cz, pbytes), sv, &fo[i]);
    });
  }
}

}  // namespace scl
