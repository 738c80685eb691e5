// State conversion and double-precision readouts: initial populations, population
// get/set, macroscopic fields (n, j, psi, F, u), the d = 2 lattice pressure tensor and the
// fixed-order conservation reductions. These kernels run off the step loop; they favour
// plain per-site code over fusion.
#pragma once
#include "scl_common.hpp"

namespace scl {

// All forcing vectors of a stencil (both members of every pair), with their weight slot.
struct VecTable {
  HalfVec v[2 * MAX_HALF_3D];
  int n;
};

// ------------------------------------------------------------------ state conversion
// Stored value at site x of population i is the post-collision value that streams out of x:
// A_i[x] = f_i(x + xi_i, t) - w_i rho0.
template <int VS, class S>
__global__ void k_init(S* __restrict__ A, const double* __restrict__ n0, DomDev dm) {
  using V = Vel<VS>;
  const long long cells = (long long)dm.nx * dm.ny * dm.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const int x = (int)(c % dm.nx), y = (int)((c / dm.nx) % dm.ny), z = (int)(c / ((long long)dm.nx * dm.ny));
  S* Ab = A + dm.off * V::Q;
  const double* nb = n0 + dm.off;
#pragma unroll
  for (int i = 0; i < V::Q; ++i) {
    const long long src = wrapi(x + V::cx(i), dm.nx) + (long long)dm.nx *
                          (wrapi(y + V::cy(i), dm.ny) + (long long)dm.ny * wrapi(z + V::cz(i), dm.nz));
    Ab[(long long)i * cells + c] = static_cast<S>(V::w(i) * nb[src] - V::w(i) * dm.rho0);
  }
}

// out_i(x) = f_i(x, t) = A_i[x - xi_i] + w_i rho0, as doubles (population layout of the ABI).
template <int VS, class S>
__global__ void k_get_pops(const S* __restrict__ A, double* __restrict__ out, DomDev dm) {
  using V = Vel<VS>;
  const long long cells = (long long)dm.nx * dm.ny * dm.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const int x = (int)(c % dm.nx), y = (int)((c / dm.nx) % dm.ny), z = (int)(c / ((long long)dm.nx * dm.ny));
  const S* Ab = A + dm.off * V::Q;
  double* ob = out + dm.off * V::Q;
#pragma unroll
  for (int i = 0; i < V::Q; ++i) {
    const long long src = wrapi(x - V::cx(i), dm.nx) + (long long)dm.nx *
                          (wrapi(y - V::cy(i), dm.ny) + (long long)dm.ny * wrapi(z - V::cz(i), dm.nz));
    ob[(long long)i * cells + c] = static_cast<double>(Ab[(long long)i * cells + src]) + V::w(i) * dm.rho0;
  }
}

template <int VS, class S>
__global__ void k_set_pops(S* __restrict__ A, const double* __restrict__ in, DomDev dm) {
  using V = Vel<VS>;
  const long long cells = (long long)dm.nx * dm.ny * dm.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const int x = (int)(c % dm.nx), y = (int)((c / dm.nx) % dm.ny), z = (int)(c / ((long long)dm.nx * dm.ny));
  S* Ab = A + dm.off * V::Q;
  const double* ib = in + dm.off * V::Q;
#pragma unroll
  for (int i = 0; i < V::Q; ++i) {
    const long long src = wrapi(x + V::cx(i), dm.nx) + (long long)dm.nx *
                          (wrapi(y + V::cy(i), dm.ny) + (long long)dm.ny * wrapi(z + V::cz(i), dm.nz));
    Ab[(long long)i * cells + c] = static_cast<S>(ib[(long long)i * cells + src] - V::w(i) * dm.rho0);
  }
}

// ------------------------------------------------------------------ macroscopic fields (double)
// n = sum_i f_i, j = sum_i f_i xi_i (d planes), psi(n); arrays indexed by the global site.
template <int VS, class S>
__global__ void k_fields(const S* __restrict__ A, double* __restrict__ n, double* __restrict__ psi,
                         double* __restrict__ j, long long tot_cells, DomDev dm) {
  using V = Vel<VS>;
  const long long cells = (long long)dm.nx * dm.ny * dm.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const int x = (int)(c % dm.nx), y = (int)((c / dm.nx) % dm.ny), z = (int)(c / ((long long)dm.nx * dm.ny));
  const S* Ab = A + dm.off * V::Q;
  double sum = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < V::Q; ++i) {
    const long long src = wrapi(x - V::cx(i), dm.nx) + (long long)dm.nx *
                          (wrapi(y - V::cy(i), dm.ny) + (long long)dm.ny * wrapi(z - V::cz(i), dm.nz));
    const double f = static_cast<double>(Ab[(long long)i * cells + src]);
    sum += f;
    jx += V::cx(i) * f;
    jy += V::cy(i) * f;
    jz += V::cz(i) * f;
  }
  const long long g = dm.off + c;
  const double nn = sum + dm.rho0;
  n[g] = nn;
  psi[g] = psi_eval<double>(nn, dm.psi_kind, dm.eps, dm.inv_eps);
  j[g] = jx;
  j[tot_cells + g] = jy;
  if (V::D == 3) j[2 * tot_cells + g] = jz;
}

// F(x) = -G c_s^2 psi(x) sum_a W_a psi(x + e_a) e_a over every vector of the table.
template <int D>
__global__ void k_force(const double* __restrict__ psi, double* __restrict__ F, long long tot_cells,
                        DomDev dm, VecTable tab) {
  const long long cells = (long long)dm.nx * dm.ny * dm.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const int x = (int)(c % dm.nx), y = (int)((c / dm.nx) % dm.ny), z = (int)(c / ((long long)dm.nx * dm.ny));
  const double* pb = psi + dm.off;
  double a[3] = {0, 0, 0};
  for (int k = 0; k < tab.n; ++k) {
    const HalfVec e = tab.v[k];
    const long long nb = wrapi(x + e.x, dm.nx) + (long long)dm.nx *
                         (wrapi(y + e.y, dm.ny) + (long long)dm.ny * wrapi(z + e.z, dm.nz));
    const double t = dm.W[e.slot] * pb[nb];
    a[0] += t * e.x;
    a[1] += t * e.y;
    a[2] += t * e.z;
  }
  const double pre = dm.gpre * pb[c];
  for (int q = 0; q < D; ++q) F[q * tot_cells + dm.off + c] = pre * a[q];
}

// u = (j + F/2) / n
template <int D>
__global__ void k_velocity(const double* __restrict__ n, const double* __restrict__ j, const double* __restrict__ F,
                           double* __restrict__ u, long long tot_cells) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= tot_cells) return;
  const double inv = 1.0 / n[g];
  for (int q = 0; q < D; ++q) u[q * tot_cells + g] = (j[q * tot_cells + g] + 0.5 * F[q * tot_cells + g]) * inv;
}

// ------------------------------------------------------------------ lattice pressure tensor, d = 2
// Appendix "Lattice Pressure Tensor - d = 2", plus the ideal part n c_s^2 delta.
// A vector e = k e_hat along a line (e_hat primitive) contributes
//   (G c_s^2 / (2k)) W e e sum_{m=0}^{k-1} psi(x - m e_hat) psi(x - m e_hat + e),
// which is the appendix's psi(x)psi(x+e)/2 for k = 1 and psi(x)psi(x+e)/4 + psi(x+e/2)psi(x-e/2)/4
// for k = 2. The primitive |e|^2 = 5 group contributes psi(x)psi(x+e)/4 per vector plus its
// irregular pairs (the links of e13 = (2,1), e14 = (1,2), e15 = (-1,2), e16 = (-2,1) that cross
// the site), each with weight W(5)/4.
__global__ void k_ptensor2d(const double* __restrict__ n, const double* __restrict__ psi, double* __restrict__ P,
                            long long tot_cells, DomDev dm, VecTable tab, int slot5) {
  const long long cells = (long long)dm.nx * dm.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const int x = (int)(c % dm.nx), y = (int)(c / dm.nx);
  const double* pb = psi + dm.off;
  auto ps = [&](int a, int b) { return pb[wrapi(x + a, dm.nx) + (long long)dm.nx * wrapi(y + b, dm.ny)]; };
  double xx = 0, yy = 0, xy = 0;
  for (int k = 0; k < tab.n; ++k) {
    const HalfVec e = tab.v[k];
    const int ax = e.x < 0 ? -e.x : e.x, ay = e.y < 0 ? -e.y : e.y;
    double s;
    if (ax * ax + ay * ay == 5) {
      s = 0.25 * ps(0, 0) * ps(e.x, e.y);
    } else {
      const int kk = ax > ay ? ax : ay;           // lines: (k,0), (0,k), (k,k)
      const int hx = e.x / kk, hy = e.y / kk;
      double acc = 0;
      for (int m = 0; m < kk; ++m) acc += ps(-m * hx, -m * hy) * ps(-m * hx + e.x, -m * hy + e.y);
      s = acc / (2.0 * kk);
    }
    const double t = dm.W[e.slot] * s;
    xx += t * e.x * e.x;
    yy += t * e.y * e.y;
    xy += t * e.x * e.y;
  }
  if (slot5 >= 0) {
    const double q = 0.25 * dm.W[slot5];
    const int ev[4][2] = {{2, 1}, {1, 2}, {-1, 2}, {-2, 1}};
    const double pr[4] = {ps(-1, 0) * ps(1, 1) + ps(-1, -1) * ps(1, 0),
                          ps(-1, -1) * ps(0, 1) + ps(0, -1) * ps(1, 1),
                          ps(0, -1) * ps(-1, 1) + ps(1, -1) * ps(0, 1),
                          ps(1, -1) * ps(-1, 0) + ps(1, 0) * ps(-1, 1)};
    for (int v = 0; v < 4; ++v) {
      xx += q * pr[v] * ev[v][0] * ev[v][0];
      yy += q * pr[v] * ev[v][1] * ev[v][1];
      xy += q * pr[v] * ev[v][0] * ev[v][1];
    }
  }
  const double G_cs2 = -dm.gpre;
  const long long g = dm.off + c;
  const double id = n[g] * CS2;
  P[g] = id + G_cs2 * xx;
  P[tot_cells + g] = id + G_cs2 * yy;
  P[2 * tot_cells + g] = G_cs2 * xy;
}

// ------------------------------------------------------------------ lattice pressure tensor, any d
// P^{mu nu}(x) = n c^2 delta + G c^2 sum_terms coef W[slot] psi(x + a) psi(x + b) e^mu e^nu over a
// term list built on the host: every link y -> y + e of the stencil shares its interaction along
// the link, 1/(2K) at each of the points y + m e/K (K = max_i |e_i|, m = 0 .. K-1), a point off
// the lattice handing its share equally to the sites around it (the groups and irregular pairs
// of the appendices on the lattice pressure tensor). Out: 6 planes xx, yy, zz, xy, xz, yz.
struct PTermDev {
  double coef;
  int8_t a[3], b[3], e[3];
  int8_t slot;
};

__global__ void k_ptensor_terms(const double* __restrict__ n, const double* __restrict__ psi, double* __restrict__ P,
                                long long tot_cells, DomDev dm, const PTermDev* __restrict__ terms, int nterms) {
  const long long cells = (long long)dm.nx * dm.ny * dm.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const int x = (int)(c % dm.nx);
  const int y = (int)((c / dm.nx) % dm.ny);
  const int z = (int)(c / ((long long)dm.nx * dm.ny));
  const double* pb = psi + dm.off;
  auto ps = [&](const int8_t* o) {
    return pb[wrapi(x + o[0], dm.nx) + (long long)dm.nx * (wrapi(y + o[1], dm.ny) + (long long)dm.ny * wrapi(z + o[2], dm.nz))];
  };
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int t = 0; t < nterms; ++t) {
    const PTermDev& q = terms[t];
    const double v = q.coef * dm.W[q.slot] * ps(q.a) * ps(q.b);
    acc[0] += v * (q.e[0] * q.e[0]);
    acc[1] += v * (q.e[1] * q.e[1]);
    acc[2] += v * (q.e[2] * q.e[2]);
    acc[3] += v * (q.e[0] * q.e[1]);
    acc[4] += v * (q.e[0] * q.e[2]);
    acc[5] += v * (q.e[1] * q.e[2]);
  }
  const double G_cs2 = -dm.gpre;
  const long long g = dm.off + c;
  const double id = n[g] * CS2;
  for (int k = 0; k < 6; ++k) P[k * tot_cells + g] = G_cs2 * acc[k] + (k < 3 ? id : 0.0);
}

// ------------------------------------------------------------------ fixed-order reductions
// Each block reduces a contiguous chunk of one domain's sites into nv doubles: values[v] =
// sum over sites of field_v, field_0 = n, field_{1..d} = j + F/2. The chunking and the tree
// depend only on the domain size, so results are bitwise reproducible.
constexpr int RED_NT = 256;

template <int D>
__global__ void __launch_bounds__(RED_NT)
k_reduce_partial(const double* __restrict__ n, const double* __restrict__ j, const double* __restrict__ F,
                 double* __restrict__ part, long long tot_cells, long long off, long long cells, long long chunk) {
  constexpr int NV = 1 + D;
  __shared__ double sh[NV][RED_NT];
  const long long b0 = off + (long long)blockIdx.x * chunk;
  const long long b1 = min(b0 + chunk, off + cells);
  double acc[NV];
  for (int v = 0; v < NV; ++v) acc[v] = 0;
  for (long long g = b0 + threadIdx.x; g < b1; g += RED_NT) {
    acc[0] += n[g];
    for (int q = 0; q < D; ++q) acc[1 + q] += j[q * tot_cells + g] + 0.5 * F[q * tot_cells + g];
  }
  for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int s = RED_NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int v = 0; v < NV; ++v) part[(long long)blockIdx.x * NV + v] = sh[v][0];
}

// Sums nb partial rows (in order) into out[nv].
__global__ void k_reduce_final(const double* __restrict__ part, int nb, int nv, double* __restrict__ out) {
  __shared__ double sh[RED_NT];
  for (int v = 0; v < nv; ++v) {
    double a = 0;
    for (int b = threadIdx.x; b < nb; b += RED_NT) a += part[(long long)b * nv + v];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = RED_NT / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = sh[0];
    __syncthreads();
  }
}

}  // namespace scl
