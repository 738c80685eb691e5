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

// rows whose loads are kept in flight ahead of the row being reduced to psi (1 or 2)
#ifndef SCL_STEP2D_PF
#define SCL_STEP2D_PF 1
#endif
// minimum waves per SIMD the step is compiled for (0: no bound beyond the block size)
#ifndef SCL_STEP2D_WPE
#define SCL_STEP2D_WPE 0
#endif

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
// nx values. The descriptor r starts one value before the row (so every offset is
// non-negative) and spans nx + 1 values. Without WRAP the positions lie inside the row: the
// lane's byte offset xb = xw * sizeof(S) plus the constant (dx + 1) * sizeof(S). With WRAP
// (strips at the periodic seam) each value's position is wrapped on its own; the wrapped
// offsets wo[dx + 1][c] are fixed for the whole march and computed once. sel is 0, or an
// offset past the buffer's end for rows with nothing to load.
template <class S, class M, int CPL, bool WRAP>
__device__ __forceinline__ void ld_row(Rsrc r, uint32_t xb, const uint32_t (*wo)[CPL], int dx, uint32_t sel, M* out,
                                       uint32_t soff) {
  if constexpr (!WRAP) {
    ldb<S, M, CPL>(r, (xb | sel) + (uint32_t)((dx + 1) * (int)sizeof(S)), out, soff);
  } else {
#pragma unroll
    for (int c = 0; c < CPL; ++c) ldb<S, M, 1>(r, wo[dx + 1][c] | sel, out + c, soff);
  }
}

__host__ __device__ constexpr int ceil_pow2(int v) { return v <= 1 ? 1 : 2 * ceil_pow2((v + 1) / 2); }

// Halo geometry: HX = R rounded up to CPL halo columns on each side of a strip, covered by
// HL = HX / CPL halo lanes per side.
template <int SET, int CPL> struct Halo2 {
  static constexpr int R = Shells<2, SET>::R;
  static constexpr int HX = ((R + CPL - 1) / CPL) * CPL;
  static constexpr int HL = HX / CPL;
};

template <class S, class M, int SET, int NO, int CPL, bool SHIFT, bool REC>
__global__ void __launch_bounds__(NO, SCL_STEP2D_WPE)
k_step2d(const S* __restrict__ fin, S* __restrict__ fout, const DomDev* __restrict__ doms,
         const WorkItem* __restrict__ items, int nitems, MacroRec<M> rec) {
  using V = Vel<0>;
  using SH = Shells<2, SET>;
  constexpr int Q = V::Q;
  constexpr int R = SH::R;
  constexpr int HX = Halo2<SET, CPL>::HX;
  constexpr int HL = Halo2<SET, CPL>::HL;
  constexpr int RING = ceil_pow2(2 * R + 2);  // psi rows kept (at least 2R + 2; a power of two)
  // rows in registers: R + 1 waiting for their collision + PF whose loads are in flight; the
  // unrolled loop cycles through NSLOT register sets (a multiple of PF + 1, the halo's sets)
  constexpr int PF = SCL_STEP2D_PF;
  constexpr int NSLOT = (R + 1 + PF + PF) / (PF + 1) * (PF + 1);
  constexpr int WIDTH = CPL * NO + 2 * HX;      // ring row length (sites)
  static_assert(2 * HL <= 64, "halo lanes must fit in the first wave");

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
  const M omega = M(dm.omega), kappa = M(dm.kappa), gpre = M(dm.gpre), aff = M(dm.aff);
  const M eps = M(dm.eps), inv_eps = M(dm.inv_eps), rho0 = M(dm.rho0);
  const int kind = dm.psi_kind;
  M Wv[SH::NS];
#pragma unroll
  for (int s = 0; s < SH::NS; ++s) Wv[s] = M(dm.W[s]);

  // Every lane owns CPL output sites X .. X + CPL - 1 (ring position q). Lanes 0 .. 2 HL - 1
  // also load one halo group (position Xh, ring position qh): HL groups left of the strip and
  // HL right of it. For a strip cut short by the domain edge (xend < x0 + CPL NO), output lanes
  // past xend supply the right halo instead.
  const int lane = threadIdx.x;
  const int X = it.x0 + CPL * lane;
  const int q = HX + CPL * lane;
  const int xend = min(it.x0 + CPL * NO, nx);
  const bool outl = X < xend;
  const bool need = X < xend + HX;
  const int Xh = lane < HL ? it.x0 - HX + CPL * lane : it.x0 + CPL * NO + CPL * (lane - HL);
  const int qh = lane < HL ? CPL * lane : HX + CPL * NO + CPL * (lane - HL);
  const bool needh = lane < 2 * HL && Xh < xend + HX;
  const int xw = wrapi(X, nx), xwh = wrapi(Xh, nx);
  // Every memory instruction of the march is issued by every lane at every step, so that the
  // compiler can keep the next row's loads in flight (a load under a branch would force it to
  // wait for everything). A lane or row with nothing to move gets an offset past the end of
  // the buffer: the hardware range check then drops the access without touching memory.
  constexpr uint32_t OFF = 0x80000000u;
  const uint32_t xb = need ? (uint32_t)xw * sizeof(S) : OFF;
  const uint32_t xbh = needh ? (uint32_t)xwh * sizeof(S) : OFF;
  const uint32_t xbo = outl ? (uint32_t)xw * sizeof(S) : OFF;
  const uint32_t xbm = outl ? (uint32_t)xw * sizeof(M) : OFF;
  const uint32_t rowbytes = (uint32_t)(nx + 1) * sizeof(S);  // a row plus the value before it

  const int dir = it.dir;
  const int total = (it.y1 - it.y0) + 2 * R;  // marching steps: rows loaded
  const int steps = (total + NSLOT - 1) / NSLOT * NSLOT;
  const int rstart = dir > 0 ? it.y0 - R : it.y1 - 1 + R;
  const int rbase = it.y0 - R - RING - NSLOT;  // ring row of row r: (r - rbase) mod RING
  // Strips whose pulls never cross the periodic seam in x (all but the first and last of a
  // domain) take a branch-free path; the others resolve the seam per lane.
  const bool seam = it.x0 - HX - 1 < 0 || it.x0 + CPL * NO + HX + 1 > nx;
  // Addressing. WHOLE (a domain's state under 2 GiB): one buffer descriptor spans the whole
  // input state (from one value before it) and one the output; the plane and row of an access
  // go into the instruction's scalar offset, so a row costs a few scalar adds. Otherwise every
  // row of every plane gets a descriptor of its own.
  const uint32_t planeb = (uint32_t)(cells * (long long)sizeof(S));
  const uint32_t rowb = (uint32_t)nx * sizeof(S);
  const bool whole = (long long)Q * cells * (long long)sizeof(S) + (long long)sizeof(S) <= 0x7fffffffLL;
  const Rsrc rin = mkrsrc(fb - 1, (uint32_t)(Q * planeb + sizeof(S)));
  const Rsrc rout = mkrsrc(ob, (uint32_t)(Q * planeb));
  auto march = [&](auto SEAM, auto WH) {
    constexpr bool WRAP = decltype(SEAM)::value;
    constexpr bool WHOLE = decltype(WH)::value;
    // wrapped byte offsets of the lane's values (and its halo group's) at x + dx, dx = a - 1
    uint32_t wo[3][CPL], who[3][CPL];
    if constexpr (WRAP) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          wo[a][c] = need ? (uint32_t)(wrapi(xw + c + a - 1, nx) + 1) * sizeof(S) : OFF;
          who[a][c] = needh ? (uint32_t)(wrapi(xwh + c + a - 1, nx) + 1) * sizeof(S) : OFF;
        }
    }
    // fr: populations of the rows between their load and their collision (R + 1 rows) plus
    // the row whose loads are in flight; hr: the same for the halo group (current + next).
    M fr[NSLOT][Q][CPL];
    M nsum[NSLOT][CPL];  // sum of each row's stored values, formed for psi, reused by the collision
    S hr[PF + 1][Q][CPL];  // kept in the storage type: only the halo lanes convert them
#pragma unroll
    for (int a = 0; a < NSLOT; ++a)
#pragma unroll
      for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int c = 0; c < CPL; ++c) fr[a][i][c] = M(0);
#pragma unroll
    for (int a = 0; a < NSLOT; ++a)
#pragma unroll
      for (int c = 0; c < CPL; ++c) nsum[a][c] = M(0);

    // Wrapped row of the next load and of the next collision, advanced by one row per marching
    // step (no division in the loop).
    auto advance = [&](int a) {
      const int t = a + dir;
      return t == ny ? 0 : (t < 0 ? ny - 1 : t);
    };
    int rw_load = wrapi(rstart, ny);
    int rw_coll = wrapi(rstart - dir * R, ny);

    // Loads of marching step k (row r) into register set J: the nine populations streaming
    // into row r, f_i(x, t) = f*_i(x - xi_i, t - 1). Steps past the last row load nothing.
    // Called for k = 0, 1, 2, ... in order.
    auto issue = [&](int k, auto J) {
      constexpr int j = decltype(J)::value;
      const int rw = rw_load;
      rw_load = advance(rw);
      const int rwm = rw == 0 ? ny - 1 : rw - 1;  // rows r - 1 and r + 1, wrapped
      const int rwp = rw == ny - 1 ? 0 : rw + 1;
      const uint32_t rowoff = k < total ? 0u : OFF;
      if constexpr (WHOLE) {
        const uint32_t rb[3] = {(uint32_t)rwm * rowb, (uint32_t)rw * rowb, (uint32_t)rwp * rowb};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const uint32_t so = (uint32_t)i * planeb + rb[1 - V::cy(i)];
          ld_row<S, M, CPL, WRAP>(rin, xb, wo, -V::cx(i), rowoff, fr[j % NSLOT][i], so);
          ld_row<S, S, CPL, WRAP>(rin, xbh, who, -V::cx(i), rowoff, hr[j % (PF + 1)][i], so);
        }
      } else {
        const long long rowo[3] = {(long long)rwm * nx, (long long)rw * nx, (long long)rwp * nx};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const Rsrc rs = mkrsrc(fb + (long long)i * cells + rowo[1 - V::cy(i)] - 1, rowbytes);
          ld_row<S, M, CPL, WRAP>(rs, xb, wo, -V::cx(i), rowoff, fr[j % NSLOT][i], 0u);
          ld_row<S, S, CPL, WRAP>(rs, xbh, who, -V::cx(i), rowoff, hr[j % (PF + 1)][i], 0u);
        }
      }
    };

    static_for<PF>([&](auto J) { issue(decltype(J)::value, J); });
    for (int k0 = 0; k0 < steps; k0 += NSLOT) {
      static_for<NSLOT>([&](auto J) {
        constexpr int j = decltype(J)::value;
        const int k = k0 + j;
        // ---------------- 1. start the next row's loads, then psi of row r into the ring
        issue(k + PF, std::integral_constant<int, j + PF>{});
        const int r = rstart + dir * k;
        M* ringrow = psis + ((r - rbase) & (RING - 1)) * WIDTH;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          M sum = M(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) sum += fr[j][i][c];
          nsum[j][c] = sum;
          const M p = psi_eval<M>(SHIFT ? rho0 + sum : sum, kind, eps, inv_eps);
          if (need) ringrow[q + c] = p;
        }
        if (needh) {
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            M sum = M(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) sum += static_cast<M>(hr[j % (PF + 1)][i][c]);
            ringrow[qh + c] = psi_eval<M>(SHIFT ? rho0 + sum : sum, kind, eps, inv_eps);
          }
        }
        __syncthreads();

        // ---------------- 2. collide row crow = r - R (marching order); every lane computes,
        // only output lanes of rows of this item store.
        constexpr int js = (j + NSLOT - R) % NSLOT;  // register set of that row
        const int crow = r - dir * R;
        const bool rowok = k >= 2 * R && k < total;
        const M* so[2 * R + 1];                      // ring rows of crow + dy, dy = o - R
#pragma unroll
        for (int o = 0; o <= 2 * R; ++o) so[o] = psis + ((crow - R + o - rbase) & (RING - 1)) * WIDTH;
        const int cw = rw_coll;  // crow, wrapped
        rw_coll = advance(cw);
        const long long orow = (long long)cw * nx;
        M out[Q][CPL];
        M recv[5][CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const int qc = q + c;
          const M psic = so[R][qc];
          // force of eq. (sc_f) over +-pairs, summed shell by shell before the weight
          M dxs[SH::NS], dys[SH::NS];
#pragma unroll
          for (int s = 0; s < SH::NS; ++s) { dxs[s] = M(0); dys[s] = M(0); }
#pragma unroll
          for (int h = 0; h < SH::NH; ++h) {
            const HalfVec hv = SH::h(h);
            const M d = so[R + hv.y][qc + hv.x] - so[R - hv.y][qc - hv.x];
            if (hv.x != 0) dxs[hv.slot] += M(hv.x) * d;
            if (hv.y != 0) dys[hv.slot] += M(hv.y) * d;
          }
          M ax = M(0), ay = M(0);
#pragma unroll
          for (int s = 0; s < SH::NS; ++s) { ax += Wv[s] * dxs[s]; ay += Wv[s] * dys[s]; }
          const M Fx = gpre * psic * ax;
          const M Fy = gpre * psic * ay;
          M f[Q];
          const M sum = nsum[js][c];
          M jx = M(0), jy = M(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            f[i] = fr[js][i][c];
            if (V::cx(i) != 0) jx += M(V::cx(i)) * f[i];
            if (V::cy(i) != 0) jy += M(V::cy(i)) * f[i];
          }
          const M nn = SHIFT ? rho0 + sum : sum;
          const M inv_n = rcp<M>(nn);
          const M ux = (jx + M(0.5) * Fx) * inv_n;
          const M uy = (jy + M(0.5) * Fy) * inv_n;
          M fo[Q];
          collide<0, M>(f, SHIFT ? sum : nn, nn, ux, uy, M(0), Fx, Fy, M(0), omega, kappa, aff, fo);
#pragma unroll
          for (int i = 0; i < Q; ++i) out[i][c] = fo[i];
          if (REC) {
            recv[0][c] = nn; recv[1][c] = jx; recv[2][c] = jy; recv[3][c] = Fx; recv[4][c] = Fy;
          }
        }
        const uint32_t so_ = rowok ? xbo : OFF;
        if constexpr (WHOLE) {
          const uint32_t orb = (uint32_t)cw * rowb;
#pragma unroll
          for (int i = 0; i < Q; ++i) stb<S, M, CPL, SCL_STORE_AUX>(rout, so_, out[i], (uint32_t)i * planeb + orb);
        } else {
#pragma unroll
          for (int i = 0; i < Q; ++i)
            stb<S, M, CPL, SCL_STORE_AUX>(mkrsrc(ob + (long long)i * cells + orow, rowb), so_, out[i]);
        }
        if (REC) {
          const long long g = dm.off + orow;
          const uint32_t sm = rowok ? xbm : OFF;
          const uint32_t rb = (uint32_t)nx * sizeof(M);
          stb<M, M, CPL>(mkrsrc(rec.n + g, rb), sm, recv[0]);
          stb<M, M, CPL>(mkrsrc(rec.j + g, rb), sm, recv[1]);
          stb<M, M, CPL>(mkrsrc(rec.j + rec.cells + g, rb), sm, recv[2]);
          stb<M, M, CPL>(mkrsrc(rec.F + g, rb), sm, recv[3]);
          stb<M, M, CPL>(mkrsrc(rec.F + rec.cells + g, rb), sm, recv[4]);
        }
      });
    }
  };
  if (whole) {
    if (seam) march(std::true_type{}, std::true_type{});
    else march(std::false_type{}, std::true_type{});
  } else {
    if (seam) march(std::true_type{}, std::false_type{});
    else march(std::false_type{}, std::false_type{});
  }
}

}  // namespace scl
