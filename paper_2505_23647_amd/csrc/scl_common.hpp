// Shared definitions of the libscl kernels: velocity sets, forcing-stencil half lists,
// per-domain parameters, work items and small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

// cache policy bits of the steps' population stores: non-temporal (the new state is not
// read again within the step, so it should not push out rows that neighbouring work items
// are about to re-read)
#ifndef SCL_STORE_AUX
#define SCL_STORE_AUX 2
#endif

namespace scl {

constexpr int MAX_SHELLS = 12;  // weight slots per domain
constexpr double CS2 = 1.0 / 3.0;

// ------------------------------------------------------------------ velocity sets
// D2Q9 order: rest, (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1).
// D3Q19 order: rest, +x, -x, +y, -y, +z, -z, then (+-1,+-1,0), (+-1,0,+-1), (0,+-1,+-1).
template <int VS> struct Vel;

template <> struct Vel<0> {
  static constexpr int Q = 9, D = 2;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int a[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    return a[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int a[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    return a[i];
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

template <> struct Vel<1> {
  static constexpr int Q = 19, D = 3;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int a[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return a[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int a[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    return a[i];
  }
  __host__ __device__ static constexpr int cz(int i) {
    constexpr int a[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
    return a[i];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

// ------------------------------------------------------------------ forcing-stencil half lists
// The force sums W_a psi(x + e_a) e_a over +-pairs; each list holds one vector of every pair
// (the other is its negative) and the weight slot of its shell. A shell set names a
// compile-time superset of shells; a domain's weights for absent shells are zero.
//   2D set 0: {1,2}             (8 vectors, reach 1)
//   2D set 1: {1,2,4,5,8}       (24 vectors, reach 2)
//   3D set 0: {1,2,3}           (26 vectors, reach 1)
//   3D set 1: {1,2,3,4,5,6,8}   (92 vectors, reach 2)
// (2D set 2 follows the two below.)
struct HalfVec { int8_t x, y, z, slot; };

template <int D, int SET> struct Shells;

template <> struct Shells<2, 0> {
  static constexpr int R = 1, NH = 4, NS = 2;
  __host__ __device__ static constexpr int code(int s) { constexpr int c[2] = {1, 2}; return c[s]; }
  __host__ __device__ static constexpr HalfVec h(int k) {
    constexpr HalfVec v[4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {1, 1, 0, 1}, {-1, 1, 0, 1}};
    return v[k];
  }
};

template <> struct Shells<2, 1> {
  static constexpr int R = 2, NH = 12, NS = 5;
  __host__ __device__ static constexpr int code(int s) { constexpr int c[5] = {1, 2, 4, 5, 8}; return c[s]; }
  __host__ __device__ static constexpr HalfVec h(int k) {
    constexpr HalfVec v[12] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {1, 1, 0, 1}, {-1, 1, 0, 1},
                               {2, 0, 0, 2}, {0, 2, 0, 2}, {2, 1, 0, 3}, {1, 2, 0, 3},
                               {-1, 2, 0, 3}, {-2, 1, 0, 3}, {2, 2, 0, 4}, {-2, 2, 0, 4}};
    return v[k];
  }
};

//   2D set 2: {1,2,4,5,8,9,16,18} (36 vectors, reach 4; the shells of the paper's
//             surface-tension and Tolman-length tuning stencils)
template <> struct Shells<2, 2> {
  static constexpr int R = 4, NH = 18, NS = 8;
  __host__ __device__ static constexpr int code(int s) {
    constexpr int c[8] = {1, 2, 4, 5, 8, 9, 16, 18};
    return c[s];
  }
  __host__ __device__ static constexpr HalfVec h(int k) {
    constexpr HalfVec v[18] = {{1, 0, 0, 0},  {0, 1, 0, 0},  {1, 1, 0, 1},  {-1, 1, 0, 1}, {2, 0, 0, 2},
                               {0, 2, 0, 2},  {2, 1, 0, 3},  {1, 2, 0, 3},  {-1, 2, 0, 3}, {-2, 1, 0, 3},
                               {2, 2, 0, 4},  {-2, 2, 0, 4}, {3, 0, 0, 5},  {0, 3, 0, 5},  {4, 0, 0, 6},
                               {0, 4, 0, 6},  {3, 3, 0, 7},  {-3, 3, 0, 7}};
    return v[k];
  }
};

// 3D half lists are generated on the host into constant tables of this size.
constexpr int MAX_HALF_3D = 70;

// ------------------------------------------------------------------ per-domain parameters
struct DomDev {
  long long off;        // first site of the domain in the concatenated site order
  int nx, ny, nz;
  int psi_kind;         // 0 exp(-1/n), 1 (n/(eps+n))^(1/eps), 2 1 - exp(-n)
  double omega;         // 1 / tau
  double kappa;         // 1 - 1/(2 tau)
  double gpre;          // -G c_s^2 (force prefactor)
  double eps;           // pseudopotential parameter
  double inv_eps;       // 1 / eps
  double rho0;          // storage shift (0 when not shifted)
  double aff;           // A / tau of the F^2 part of the Guo tensor, T = 2 u F - (A/tau) F F
  double W[MAX_SHELLS]; // weight of each shell slot of the compile-time set
};

// A workgroup's share of one step: a strip of output columns [x0, x0 + width) of domain dom
// (2D: rows [y0, y1); 3D: additionally output rows [y0, y0 + tile) and planes [z0, z1)).
struct WorkItem {
  int dom;
  int x0;
  int y0, y1;
  int z0, z1;
  int dir;  // marching direction along y (2D): +1 from y0 upward, -1 from y1 - 1 downward
  int pad_;
};

// Optional recording of the macroscopic fields of every site a step updates (used by the
// adjoint's recompute pass): n, j (d values), F (d values), each a [cells] plane.
template <class M> struct MacroRec {
  M* n;
  M* j;   // d planes
  M* F;   // d planes
  long long cells;
};

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1, so that register
// arrays indexed by I stay in registers.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F> __device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__host__ __device__ inline int wrapi(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// ------------------------------------------------------------------ pseudopotential
template <class M> __device__ inline M psi_eval(M n, int kind, M eps, M inv_eps);

// float, psi = exp(-1/n): exp2 of -log2(e)/n through the hardware reciprocal and the hardware
// base-2 exponential (three instructions; within 3 ulp for the densities of a Shan-Chen fluid,
// where -log2(e)/n stays far from the exponential's denormal range).
template <> __device__ inline float psi_eval<float>(float n, int kind, float eps, float inv_eps) {
  if (kind == 0) return __builtin_amdgcn_exp2f(-1.44269504088896341f * __builtin_amdgcn_rcpf(n));
  if (kind == 1) return powf(n / (eps + n), inv_eps);
  return 1.0f - expf(-n);
}
template <> __device__ inline double psi_eval<double>(double n, int kind, double eps, double inv_eps) {
  if (kind == 0) return exp(-1.0 / n);
  if (kind == 1) return pow(n / (eps + n), inv_eps);
  return 1.0 - exp(-n);
}

// dpsi/dn
template <class M> __device__ inline M dpsi_eval(M n, M psi, int kind, M eps) {
  if (kind == 0) return psi / (n * n);
  if (kind == 1) return psi / (n * (eps + n));
  return M(1) - psi;
}

// ------------------------------------------------------------------ fast reciprocal
// float: the hardware reciprocal (1 ulp); double: the correctly rounded quotient.
template <class M> __device__ inline M rcp(M x);
template <> __device__ inline float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double rcp<double>(double x) { return 1.0 / x; }

// ------------------------------------------------------------------ storage conversion
template <class S, class M> __device__ inline M ld(const S* p) { return static_cast<M>(*p); }
template <class S, class M> __device__ inline void st(S* p, M v) { *p = static_cast<S>(v); }
// Output store of the step: optionally non-temporal (the written state is not read again
// within the step, so it need not displace the halo rows other workgroups re-read).
template <class S, class M, bool NT> __device__ inline void st_out(S* p, M v) {
  if (NT) __builtin_nontemporal_store(static_cast<S>(v), p);
  else *p = static_cast<S>(v);
}

// ------------------------------------------------------------------ opposite velocities
template <int VS> __host__ __device__ constexpr int opp(int i) {
  using V = Vel<VS>;
  for (int j = 0; j < V::Q; ++j)
    if (V::cx(j) == -V::cx(i) && V::cy(j) == -V::cy(i) && V::cz(j) == -V::cz(i)) return j;
  return -1;
}

// ------------------------------------------------------------------ BGK + Guo collision
// f*_i = f_i - omega (f_i - f_i^eq) + S_i  (eqs. lbm, omega_i) with
//   f_i^eq = w_i n [1 + xi.u/c^2 + (xi.u)^2/(2c^4) - u.u/(2c^2)]          (eq. f_eq)
//   S_i    = kappa w_i [xi.F/c^2 + (xi xi - c^2 1) : T / (2 c^4)]           (eq. GuoForcing)
//            with T = 2 u F - aff F F: the paper's T = 2uF plus, for aff = A/tau != 0, the F^2
//            terms of the appendix on eps and e4; the contraction is
//            ((xi.u)(xi.F) - c^2 u.F)/c^4 - aff ((xi.F)^2 - c^2 F.F)/(2 c^4)
// written as f*_i = (1 - omega) f_i + A +- B for each pair (i, opposite of i): A collects the
// terms even in xi, B the odd ones. base = n for plain storage; for shifted storage (f holds
// f - w rho0) base = n - rho0 = sum of the stored values, which subtracts w rho0 from f^eq.
// emit(i, value) receives each post-collision value (pairs in turn), so a caller can store it
// at once instead of holding all Q.
template <int VS, class M, class Emit>
__device__ __forceinline__ void collide_emit(const M* f, M base, M nn, M ux, M uy, M uz, M Fx, M Fy, M Fz,
                                             M omega, M kappa, M aff, Emit&& emit) {
  using V = Vel<VS>;
  constexpr int Q = V::Q;
  const M uu15 = M(1.5) * (ux * ux + uy * uy + uz * uz);  // u.u / (2 c^2)
  const M uF3 = M(3) * (ux * Fx + uy * Fy + uz * Fz) - M(1.5) * aff * (Fx * Fx + Fy * Fy + Fz * Fz);
  const M aff45 = M(4.5) * aff;
  const M om1 = M(1) - omega;
  const M on = omega * nn;
  const M obase = omega * base;
  {
    constexpr M w = M(V::w(0));
    emit(0, om1 * f[0] + (w * (obase - on * uu15) - (kappa * w) * uF3));
  }
  static_for<Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int ib = opp<VS>(i);
    if constexpr (i > 0 && i < ib) {
      constexpr M w = M(V::w(i));
      constexpr int cx = V::cx(i), cy = V::cy(i), cz = V::cz(i);
      M xu = M(0), xF = M(0);
      if constexpr (cx != 0) { xu += M(cx) * ux; xF += M(cx) * Fx; }
      if constexpr (cy != 0) { xu += M(cy) * uy; xF += M(cy) * Fy; }
      if constexpr (cz != 0) { xu += M(cz) * uz; xF += M(cz) * Fz; }
      const M E = M(4.5) * xu * xu - uu15;
      const M Se = xF * (M(9) * xu - aff45 * xF) - uF3;
      const M A = w * (obase + on * E) + (kappa * w) * Se;
      const M B = (M(3) * w) * (on * xu + kappa * xF);
      emit(i, om1 * f[i] + (A + B));
      emit(ib, om1 * f[ib] + (A - B));
    }
  });
}

template <int VS, class M>
__device__ __forceinline__ void collide(const M* f, M base, M nn, M ux, M uy, M uz, M Fx, M Fy, M Fz, M omega,
                                        M kappa, M aff, M* fo) {
  collide_emit<VS, M>(f, base, nn, ux, uy, uz, Fx, Fy, Fz, omega, kappa, aff, [&](int i, M v) { fo[i] = v; });
}

// ------------------------------------------------------------------ buffer access
// The step reads and writes through buffer instructions: the row's base address lives in a
// (uniform) buffer descriptor, the lane supplies a 32-bit byte offset that stays fixed for the
// whole march, and the hardware range check bounds every access to the row.
typedef __amdgpu_buffer_rsrc_t Rsrc;

__device__ __forceinline__ Rsrc mkrsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// CPL stored values at byte offset voff + soff of the buffer r (soff: a uniform offset),
// converted to M. A voff at or past the buffer's size drops the access.
template <class S, class M, int CPL>
__device__ __forceinline__ void ldb(Rsrc r, uint32_t voff, M* out, uint32_t soff = 0) {
  constexpr int B = (int)sizeof(S) * CPL;
  S t[CPL];
  if constexpr (B == 2) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    __builtin_memcpy(t, &u, B);
  } else if constexpr (B == 4) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    __builtin_memcpy(t, &u, B);
  } else if constexpr (B == 8) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    __builtin_memcpy(t, &u, B);
  } else {
    static_assert(B == 16, "unsupported access width");
    const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    __builtin_memcpy(t, &u, B);
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c) out[c] = static_cast<M>(t[c]);
}

template <class S, class M, int CPL, int AUX = 0>
__device__ __forceinline__ void stb(Rsrc r, uint32_t voff, const M* in, uint32_t soff = 0) {
  constexpr int B = (int)sizeof(S) * CPL;
  S t[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) t[c] = static_cast<S>(in[c]);
  if constexpr (B == 2) {
    unsigned short u;
    __builtin_memcpy(&u, t, B);
    __builtin_amdgcn_raw_buffer_store_b16(u, r, voff, soff, AUX);
  } else if constexpr (B == 4) {
    uint32_t u;
    __builtin_memcpy(&u, t, B);
    __builtin_amdgcn_raw_buffer_store_b32(u, r, voff, soff, AUX);
  } else if constexpr (B == 8) {
    uint32_t u __attribute__((ext_vector_type(2)));
    __builtin_memcpy(&u, t, B);
    __builtin_amdgcn_raw_buffer_store_b64(u, r, voff, soff, AUX);
  } else {
    uint32_t u __attribute__((ext_vector_type(4)));
    __builtin_memcpy(&u, t, B);
    __builtin_amdgcn_raw_buffer_store_b128(u, r, voff, soff, AUX);
  }
}

}  // namespace scl
