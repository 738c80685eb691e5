// Oracle for the Shan-Chen lattice Boltzmann time step (Lulli & Ching, arXiv 2505.23647).
//
// TEST INFRASTRUCTURE ONLY. This file is a plain, slow, FP64 CPU reference used by the
// test suite, the smoke check and the CPU-baseline leg of the benchmark. Nothing in the
// product library may include, link or call it, and it shares no code with the GPU path.
//
// Every routine is written to read against the paper:
//   * lattice Boltzmann equation, BGK operator, Hermite equilibrium  -> Sec. "Lattice Boltzmann",
//     eqs. (lbm), (omega_i), (f_eq), velocity-set isotropy conditions that follow (f_eq);
//   * Guo forcing and the shifted equilibrium velocity               -> eq. (GuoForcing) and the
//     definition of u^(eq) right after it, with T = 2 u F;
//   * Shan-Chen force over the forcing stencil                       -> eq. (sc_f);
//   * pseudopotentials exp(-1/n) and (n/(eps+n))^(1/eps)             -> eq. (psieps) and Sec. on
//     the sigma_1 tuning (eps = 0 case);
//   * two-dimensional lattice pressure tensor                        -> Appendix "Lattice Pressure
//     Tensor - d = 2", with the ideal part n c_s^2 delta re-added (Sec. "Interface Physics");
//   * droplet observables (Delta P, generalised surface tension sigma[R], surface of tension
//     R_s, equimolar radius R_e)                                     -> Sec. "Interface Physics"
//     (sigma[R], P_J) and the Laplace-law paragraph of the sigma_1 tuning section.
//
// The arithmetic is templated on the scalar type so that the very same loops, run on
// forward-mode dual numbers, give exact tangent-linear derivatives with respect to the shell
// weights W and the coupling G. No blocking, fusion or reordering beyond the equations.
//
// Build: g++ -std=c++17 -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <array>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------- dual numbers (forward mode)
constexpr int ND = 8;  // up to 7 shell weights + G
struct Dual {
  double v;
  double d[ND];
  Dual() : v(0.0) { for (int k = 0; k < ND; ++k) d[k] = 0.0; }
  Dual(double x) : v(x) { for (int k = 0; k < ND; ++k) d[k] = 0.0; }
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, const Dual& b) { a = a - b; return a; }
inline Dual exp(const Dual& a) { double e = std::exp(a.v); Dual r(e); for (int k = 0; k < ND; ++k) r.d[k] = e * a.d[k]; return r; }
inline Dual log(const Dual& a) { Dual r(std::log(a.v)); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / a.v; return r; }
inline Dual pow(const Dual& a, double p) {
  double y = std::pow(a.v, p);
  Dual r(y);
  double dy = p * std::pow(a.v, p - 1.0);
  for (int k = 0; k < ND; ++k) r.d[k] = dy * a.d[k];
  return r;
}
inline Dual sqrt(const Dual& a) { return pow(a, 0.5); }
inline double val(const Dual& a) { return a.v; }
inline double val(double a) { return a; }
using std::exp;
using std::pow;
using std::sqrt;

// ---------------------------------------------------------------- velocity sets (Sec. Lattice Boltzmann)
// D2Q9: every vector with components in {-1,0,1}; D3Q19: those with |xi|^2 <= 2.
// Weights depend on |xi|^2 only: 2D 4/9, 1/9, 1/36; 3D 1/3, 1/18, 1/36.
struct VelSet {
  int d = 2, Q = 0;
  std::vector<std::array<int, 3>> xi;
  std::vector<double> w;
};

static VelSet make_velset(int d) {
  VelSet vs;
  vs.d = d;
  const int zr = (d == 3) ? 1 : 0;
  for (int len2 = 0; len2 <= 2; ++len2)
    for (int z = -zr; z <= zr; ++z)
      for (int y = -1; y <= 1; ++y)
        for (int x = -1; x <= 1; ++x) {
          if (x * x + y * y + z * z != len2) continue;
          vs.xi.push_back({x, y, z});
          double w;
          if (d == 2) w = (len2 == 0) ? 4.0 / 9.0 : (len2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
          else        w = (len2 == 0) ? 1.0 / 3.0 : (len2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
          vs.w.push_back(w);
        }
  vs.Q = (int)vs.xi.size();
  return vs;
}

// ---------------------------------------------------------------- forcing stencil (eq. sc_f, Fig. 1)
// A shell code names one symmetry group: all integer vectors obtained from a generator by
// permutations and sign flips. The code is |e|^2, except in 3D where |e|^2 = 9 holds two
// groups: code 9 is the (2,2,1) group and code 1009 the (3,0,0) group. Code 18 is (3,3,0).
static bool shell_generator(int d, int code, std::array<int, 3>& g) {
  switch (code) {
    case 1: g = {1, 0, 0}; return true;
    case 2: g = {1, 1, 0}; return true;
    case 3: g = {1, 1, 1}; return d == 3;
    case 4: g = {2, 0, 0}; return true;
    case 5: g = {2, 1, 0}; return true;
    case 6: g = {2, 1, 1}; return d == 3;
    case 8: g = {2, 2, 0}; return true;
    case 9: if (d == 2) { g = {3, 0, 0}; return true; } g = {2, 2, 1}; return true;
    case 1009: g = {3, 0, 0}; return d == 3;
    case 16: g = {4, 0, 0}; return true;
    case 18: g = {3, 3, 0}; return true;
    default: return false;
  }
}

struct Stencil {
  std::vector<std::array<int, 3>> e;
  std::vector<int> shell;  // index into the caller's shell list
  int reach = 0;           // largest |component|
};

static bool make_stencil(int d, int nshells, const int* codes, Stencil& st) {
  st = Stencil();
  for (int s = 0; s < nshells; ++s) {
    std::array<int, 3> g;
    if (!shell_generator(d, codes[s], g)) return false;
    std::array<int, 3> gs = g;
    std::sort(gs.begin(), gs.end());
    const int zr = (d == 3) ? 4 : 0;
    for (int z = -zr; z <= zr; ++z)
      for (int y = -4; y <= 4; ++y)
        for (int x = -4; x <= 4; ++x) {
          std::array<int, 3> a = {std::abs(x), std::abs(y), std::abs(z)};
          std::sort(a.begin(), a.end());
          if (a != gs) continue;
          st.e.push_back({x, y, z});
          st.shell.push_back(s);
          st.reach = std::max(st.reach, std::max(std::abs(x), std::max(std::abs(y), std::abs(z))));
        }
  }
  return true;
}

// ---------------------------------------------------------------- pseudopotentials
// kind 0: psi = exp(-1/n); kind 1: psi = (n/(eps+n))^(1/eps) (eq. psieps);
// kind 2: psi = 1 - exp(-n), the textbook form (not used by the paper).
template <class T>
static T psi_of(const T& n, int kind, double p) {
  if (kind == 0) return exp(-1.0 / n);
  if (kind == 1) return pow(n / (p + n), 1.0 / p);
  return 1.0 - exp(-1.0 * n);
}

// ---------------------------------------------------------------- geometry
struct Geom {
  int d, nx, ny, nz;
  long N() const { return (long)nx * ny * nz; }
  long idx(long x, long y, long z) const {
    x %= nx; if (x < 0) x += nx;
    y %= ny; if (y < 0) y += ny;
    z %= nz; if (z < 0) z += nz;
    return x + (long)nx * (y + (long)ny * z);
  }
  void coords(long c, long& x, long& y, long& z) const {
    x = c % nx; y = (c / nx) % ny; z = c / ((long)nx * ny);
  }
};

constexpr double CS2 = 1.0 / 3.0;

// ---------------------------------------------------------------- macroscopic fields
// n = sum_i f_i, j = sum_i f_i xi_i, psi = psi(n),
// F(x) = -G c_s^2 psi(x) sum_a W(|e_a|^2) psi(x + e_a) e_a      (eq. sc_f)
template <class T>
static void macro_fields(const Geom& g, const VelSet& vs, const Stencil& st, const T* W, const T& G,
                         int kind, double p, const T* f, std::vector<T>& n, std::vector<T>& j,
                         std::vector<T>& psi, std::vector<T>& F) {
  const long N = g.N();
  n.assign(N, T(0.0));
  j.assign(3 * N, T(0.0));
  psi.assign(N, T(0.0));
  F.assign(3 * N, T(0.0));
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    T nn(0.0), jx(0.0), jy(0.0), jz(0.0);
    for (int i = 0; i < vs.Q; ++i) {
      const T fi = f[(long)i * N + c];
      nn = nn + fi;
      jx = jx + fi * (double)vs.xi[i][0];
      jy = jy + fi * (double)vs.xi[i][1];
      jz = jz + fi * (double)vs.xi[i][2];
    }
    n[c] = nn;
    j[3 * c + 0] = jx; j[3 * c + 1] = jy; j[3 * c + 2] = jz;
    psi[c] = psi_of(nn, kind, p);
  }
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    long x, y, z;
    g.coords(c, x, y, z);
    T ax(0.0), ay(0.0), az(0.0);
    for (size_t a = 0; a < st.e.size(); ++a) {
      const auto& e = st.e[a];
      const T term = W[st.shell[a]] * psi[g.idx(x + e[0], y + e[1], z + e[2])];
      ax = ax + term * (double)e[0];
      ay = ay + term * (double)e[1];
      az = az + term * (double)e[2];
    }
    const T pre = -1.0 * G * CS2 * psi[c];
    F[3 * c + 0] = pre * ax; F[3 * c + 1] = pre * ay; F[3 * c + 2] = pre * az;
  }
}

// ---------------------------------------------------------------- one time step
// For every x, from time-t values only:
//   u = (j + F/2)/n                                                (shifted velocity)
//   feq_i = w_i n [1 + xi.u/c^2 + (xi.u)^2/(2c^4) - u.u/(2c^2)]   (eq. f_eq)
//   T_ab = 2 u_a F_b - (A/tau) F_a F_b                             (rank-two tensor of eq. GuoForcing;
//                                                                   A = 0: T = 2uF, the paper's
//                                                                   choice; A != 0: the F^2 terms of
//                                                                   the appendix on eps and e4)
//   S_i = (1 - 1/(2 tau)) w_i [xi.F/c^2 + (xi_a xi_b - c^2 delta_ab) T_ab / (2 c^4)]   (eq. GuoForcing)
//   f_i(x + xi_i, t+1) = f_i - (f_i - feq_i)/tau + S_i            (eqs. lbm, omega_i)
template <class T>
static void step(const Geom& g, const VelSet& vs, const Stencil& st, const T* W, const T& G, double tau,
                 double aF, int kind, double p, const T* f, T* fo) {
  std::vector<T> n, j, psi, F;
  macro_fields(g, vs, st, W, G, kind, p, f, n, j, psi, F);
  const long N = g.N();
  const double kappa = 1.0 - 1.0 / (2.0 * tau);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    long x, y, z;
    g.coords(c, x, y, z);
    T u[3], Fc[3];
    for (int k = 0; k < 3; ++k) {
      Fc[k] = F[3 * c + k];
      u[k] = (j[3 * c + k] + 0.5 * Fc[k]) / n[c];
    }
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T Tt[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Tt[a][b] = 2.0 * u[a] * Fc[b] - (aF / tau) * Fc[a] * Fc[b];
    for (int i = 0; i < vs.Q; ++i) {
      const double xi[3] = {(double)vs.xi[i][0], (double)vs.xi[i][1], (double)vs.xi[i][2]};
      const T xu = u[0] * xi[0] + u[1] * xi[1] + u[2] * xi[2];
      const T xF = Fc[0] * xi[0] + Fc[1] * xi[1] + Fc[2] * xi[2];
      const T feq = vs.w[i] * n[c] * (1.0 + xu / CS2 + xu * xu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
      T H(0.0);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) H = H + (xi[a] * xi[b] - (a == b ? CS2 : 0.0)) * Tt[a][b];
      const T S = kappa * vs.w[i] * (xF / CS2 + H / (2.0 * CS2 * CS2));
      const T fi = f[(long)i * N + c];
      const T fstar = fi - (fi - feq) / tau + S;
      fo[(long)i * N + g.idx(x + vs.xi[i][0], y + vs.xi[i][1], z + vs.xi[i][2])] = fstar;
    }
  }
}

// ---------------------------------------------------------------- lattice pressure tensor, d = 2
// Appendix "Lattice Pressure Tensor - d = 2". Returns (Pxx, Pyy, Pxy) at cell c.
// Groups along a line, e = k * e_hat with e_hat primitive (codes 1,2 with k=1; 4,8 with k=2;
// 9,18 with k=3; 16 with k=4), and the |e|^2 = 5 group with its regular and irregular parts.
// The |e|^2 = 16 group follows the d = 3 appendix formula, which involves only one direction.
template <class T>
static void ptensor2d_cell(const Geom& g, const Stencil& st, const int* codes, const T* W, const T& G,
                           const std::vector<T>& n, const std::vector<T>& psi, long c, T out[3]) {
  long x, y, z;
  g.coords(c, x, y, z);
  auto ps = [&](long a, long b) { return psi[g.idx(x + a, y + b, 0)]; };
  T xx(0.0), yy(0.0), xy(0.0);
  auto acc = [&](const T& s, long ex, long ey) {
    xx = xx + s * (double)(ex * ex);
    yy = yy + s * (double)(ey * ey);
    xy = xy + s * (double)(ex * ey);
  };
  const T psi0 = psi[c];
  for (size_t a = 0; a < st.e.size(); ++a) {
    const long ex = st.e[a][0], ey = st.e[a][1];
    const int code = codes[st.shell[a]];
    const T Wa = W[st.shell[a]];
    if (code == 1 || code == 2) {
      acc(0.5 * Wa * psi0 * ps(ex, ey), ex, ey);
    } else if (code == 4 || code == 8) {
      acc(0.25 * Wa * psi0 * ps(ex, ey), ex, ey);
      acc(0.25 * Wa * ps(ex / 2, ey / 2) * ps(-ex / 2, -ey / 2), ex, ey);
    } else if (code == 9 || code == 18) {
      acc((1.0 / 6.0) * Wa * psi0 * ps(ex, ey), ex, ey);
      acc((1.0 / 3.0) * Wa * ps(ex / 3, ey / 3) * ps(-2 * ex / 3, -2 * ey / 3), ex, ey);
    } else if (code == 16) {
      acc(0.125 * Wa * psi0 * ps(ex, ey), ex, ey);
      acc(0.25 * Wa * ps(ex / 4, ey / 4) * ps(-3 * ex / 4, -3 * ey / 4), ex, ey);
      acc(0.125 * Wa * ps(ex / 2, ey / 2) * ps(-ex / 2, -ey / 2), ex, ey);
    } else if (code == 5) {
      acc(0.25 * Wa * psi0 * ps(ex, ey), ex, ey);  // regular part
    }
  }
  // irregular part of the |e|^2 = 5 group: vectors (2,1), (1,2), (-1,2), (-2,1), each fed by
  // the two pairs of sites it links across the cell (psi_{a,b} = psi(x + a e_x + b e_y)).
  int s5 = -1;
  for (size_t a = 0; a < st.e.size(); ++a)
    if (codes[st.shell[a]] == 5) { s5 = st.shell[a]; break; }
  if (s5 >= 0) {
    const T W5 = W[s5];
    acc(0.25 * W5 * (ps(-1, 0) * ps(1, 1) + ps(-1, -1) * ps(1, 0)), 2, 1);
    acc(0.25 * W5 * (ps(-1, -1) * ps(0, 1) + ps(0, -1) * ps(1, 1)), 1, 2);
    acc(0.25 * W5 * (ps(0, -1) * ps(-1, 1) + ps(1, -1) * ps(0, 1)), -1, 2);
    acc(0.25 * W5 * (ps(1, -1) * ps(-1, 0) + ps(1, 0) * ps(-1, 1)), -2, 1);
  }
  const T pre = G * CS2;
  out[0] = n[c] * CS2 + pre * xx;
  out[1] = n[c] * CS2 + pre * yy;
  out[2] = pre * xy;
}

// ---------------------------------------------------------------- lattice pressure tensor, d = 2, 3
// One rule for every group of the appendices on the lattice pressure tensor: the interaction
// of a link from site y to y + e (weight W(|e|^2), ordered: the -e vector gives the reverse
// link) is shared along the link. With K = max_i |e_i|, the link contributes at the K points
// p_m = y + m e / K, m = 0 .. K-1, a share 1/(2K) each; a point that is not a lattice site
// (q non-integer coordinates) hands its share in equal parts to the 2^q sites around it:
//   P^{mu nu}(x) = n c^2 delta + G c^2 sum_e W e^mu e^nu sum_m (1/(2K)) sum_{corners c of p_m}
//                   2^{-q} psi(x - c) psi(x - c + e).
// For e along a line (e = K e_hat) this is the line rule of the symmetric groups (psi(x) psi(x+e)
// and psi(x + e/2) psi(x - e/2) for |e|^2 = 4, 8; the e/3 forms for 9, 18; the e/4 forms for 16,
// each after the +-e sum); for the groups (2,1,0), (2,1,1), (2,2,1) m = 0 is their regular part
// and m = 1 (the crossing of the plane midway) their irregular pairs: the two sites around
// (1, 1/2, 0) with share 1/8 per ordered vector (W/4 per pair), the four around (1, 1/2, 1/2)
// (W/8 per pair), the two around (1, 1, 1/2) (W/4 per pair). Out: xx, yy, zz, xy, xz, yz.
template <class T>
static void ptensor_cell(const Geom& g, const Stencil& st, const T* W, const T& G, const std::vector<T>& n,
                         const std::vector<T>& psi, long c, T out[6]) {
  long x, y, z;
  g.coords(c, x, y, z);
  T acc[6] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
  for (size_t a = 0; a < st.e.size(); ++a) {
    const long e[3] = {st.e[a][0], st.e[a][1], st.e[a][2]};
    const long K = std::max(std::labs(e[0]), std::max(std::labs(e[1]), std::labs(e[2])));
    T link(0.0);  // sum over m and corners of the weighted psi psi products
    for (long m = 0; m < K; ++m) {
      // p_m = m e / K: integer part and whether the coordinate is a half-integer or integer
      long base[3];
      bool frac[3];
      int q = 0;
      for (int i = 0; i < 3; ++i) {
        const long num = m * e[i];
        frac[i] = num % K != 0;
        base[i] = (long)std::floor((double)num / (double)K);
        q += frac[i] ? 1 : 0;
      }
      const double share = 1.0 / (2.0 * (double)K) / (double)(1 << q);
      for (int bits = 0; bits < 8; ++bits) {
        bool ok = true;
        long cc[3];
        for (int i = 0; i < 3; ++i) {
          const int b = (bits >> i) & 1;
          if (!frac[i] && b) { ok = false; break; }
          cc[i] = base[i] + b;
        }
        if (!ok) continue;
        const long y0[3] = {x - cc[0], y - cc[1], z - cc[2]};
        link = link + share * psi[g.idx(y0[0], y0[1], y0[2])] * psi[g.idx(y0[0] + e[0], y0[1] + e[1], y0[2] + e[2])];
      }
    }
    const T t = W[st.shell[a]] * link;
    acc[0] = acc[0] + t * (double)(e[0] * e[0]);
    acc[1] = acc[1] + t * (double)(e[1] * e[1]);
    acc[2] = acc[2] + t * (double)(e[2] * e[2]);
    acc[3] = acc[3] + t * (double)(e[0] * e[1]);
    acc[4] = acc[4] + t * (double)(e[0] * e[2]);
    acc[5] = acc[5] + t * (double)(e[1] * e[2]);
  }
  const T pre = G * CS2;
  for (int k = 0; k < 6; ++k) out[k] = pre * acc[k];
  for (int k = 0; k < 3; ++k) out[k] = out[k] + n[c] * CS2;
}

// ---------------------------------------------------------------- droplet observables, d = 3
// As in d = 2 with Pbar = tr P / 3, P_T = P^yy on the +-x half-lines through the centre,
// C_d = int_0^{L/2} r^2 (Pbar(corner) - P_T(r)) dr, R_s = (6 C_d / Delta P)^{1/3},
// sigma_s = Delta P R_s / 2 and (4/3) pi R_e^3 n_in + (L^3 - (4/3) pi R_e^3) n_out = M.
template <class T>
static void droplet_obs3d(const Geom& g, const Stencil& st, const T* W, const T& G, const std::vector<T>& n,
                          const std::vector<T>& psi, int cx, int cy, int cz, int bubble, T out[6]) {
  const int L = g.nx;
  T Pc[6], Po[6];
  ptensor_cell(g, st, W, G, n, psi, g.idx(cx, cy, cz), Pc);
  ptensor_cell(g, st, W, G, n, psi, g.idx(0, 0, 0), Po);
  const T Pbar_c = (Pc[0] + Pc[1] + Pc[2]) / 3.0;
  const T Pbar_o = (Po[0] + Po[1] + Po[2]) / 3.0;
  const T dP = Pbar_c - Pbar_o;
  const int R = L / 2;
  T Cd(0.0);
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    T sum(0.0);
    for (int r = 0; r <= R; ++r) {
      T P[6];
      ptensor_cell(g, st, W, G, n, psi, g.idx(cx + sgn * r, cy, cz), P);
      T gr = (double)r * (double)r * (Pbar_o - P[1]);
      if (r == 0 || r == R) gr = 0.5 * gr;
      sum = sum + gr;
    }
    Cd = Cd + 0.5 * sum;
  }
  const T Rs = cbrt(6.0 * Cd / dP);
  const T sig = 0.5 * dP * Rs;
  T M(0.0);
  for (long c = 0; c < g.N(); ++c) M = M + n[c];
  const T nin = n[g.idx(cx, cy, cz)];
  const T nout = n[0];
  const double PI = 3.14159265358979323846;
  const double L3 = (double)L * (double)L * (double)L;
  const T Re = cbrt((M - L3 * nout) / ((4.0 / 3.0) * PI * (nin - nout)));
  out[0] = dP; out[1] = Cd; out[2] = Rs; out[3] = sig; out[4] = Re; out[5] = (bubble ? -1.0 : 1.0) * (Re - Rs);
}

// ---------------------------------------------------------------- droplet observables, d = 2
// Inputs: square L x L domain, centre (cx, cy), b = 1 for a bubble.
//   Pbar = tr P / d; Delta P = Pbar(centre) - Pbar(corner (0,0)).
//   sigma[R] = R^{1-d} int_0^{L/2} r^{d-1} (P_J(r;R) - P_T(r)) dr with P_T(r) = P^yy on the
//   horizontal half-lines through the centre (trapezoid on sites, mean of +x and -x), i.e.
//   sigma[R] = C_d / R^{d-1} + Delta P R / d with C_d = int r^{d-1}(Pbar(corner) - P_T(r)) dr.
//   Its stationary point gives R_s = (d (d-1) C_d / Delta P)^{1/d}, sigma_s = Delta P R_s/(d-1).
//   The pressure inside is the higher one for droplets and bubbles alike, so Delta P, R_s and
//   sigma_s are positive for both; the bubble's sign (-1)^b belongs to its curvature (the
//   Tolman fits plot both branches against the signed curvature (-1)^b / R).
//   Equimolar radius: pi R_e^2 n_in + (L^2 - pi R_e^2) n_out = M.
//   Tolman length measured from the liquid side: delta = (-1)^b (R_e - R_s).
// out = (Delta P, C_d, R_s, sigma_s, R_e, delta).
template <class T>
static void droplet_obs2d(const Geom& g, const Stencil& st, const int* codes, const T* W, const T& G,
                          const std::vector<T>& n, const std::vector<T>& psi, int cx, int cy, int bubble,
                          T out[6]) {
  const int L = g.nx;
  T Pc[3], Po[3];
  ptensor2d_cell(g, st, codes, W, G, n, psi, g.idx(cx, cy, 0), Pc);
  ptensor2d_cell(g, st, codes, W, G, n, psi, g.idx(0, 0, 0), Po);
  const T Pbar_c = 0.5 * (Pc[0] + Pc[1]);
  const T Pbar_o = 0.5 * (Po[0] + Po[1]);
  const T dP = Pbar_c - Pbar_o;
  const int R = L / 2;
  T Cd(0.0);
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    T sum(0.0);
    for (int r = 0; r <= R; ++r) {
      T P[3];
      ptensor2d_cell(g, st, codes, W, G, n, psi, g.idx(cx + sgn * r, cy, 0), P);
      T gr = (double)r * (Pbar_o - P[1]);
      if (r == 0 || r == R) gr = 0.5 * gr;
      sum = sum + gr;
    }
    Cd = Cd + 0.5 * sum;
  }
  const T Rs = sqrt(2.0 * Cd / dP);
  const T sig = dP * Rs;
  T M(0.0);
  for (long c = 0; c < g.N(); ++c) M = M + n[c];
  const T nin = n[g.idx(cx, cy, 0)];
  const T nout = n[0];
  const double PI = 3.14159265358979323846;
  const T Re = sqrt((M - (double)L * (double)L * nout) / (PI * (nin - nout)));
  out[0] = dP; out[1] = Cd; out[2] = Rs; out[3] = sig; out[4] = Re; out[5] = (bubble ? -1.0 : 1.0) * (Re - Rs);
}

}  // namespace orc

// ======================================================================== C entry points
using namespace orc;

extern "C" {

// Threads the OpenMP loops use.
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Velocity set: writes Q vectors (3 ints each) and weights; returns Q.
int orc_velset(int d, int* xi, double* w) {
  VelSet vs = make_velset(d);
  for (int i = 0; i < vs.Q; ++i) {
    if (xi) for (int k = 0; k < 3; ++k) xi[3 * i + k] = vs.xi[i][k];
    if (w) w[i] = vs.w[i];
  }
  return vs.Q;
}

// Forcing vectors of the given shells: writes up to cap vectors and their shell index; returns
// the count, or -1 for an unknown shell code.
int orc_stencil(int d, int nshells, const int* codes, int cap, int* e, int* shell) {
  Stencil st;
  if (!make_stencil(d, nshells, codes, st)) return -1;
  for (size_t a = 0; a < st.e.size() && (int)a < cap; ++a) {
    for (int k = 0; k < 3; ++k) e[3 * a + k] = st.e[a][k];
    shell[a] = st.shell[a];
  }
  return (int)st.e.size();
}

// f_i(x, 0) = w_i n0(x): the fluid at rest (populations at equilibrium with u = 0).
int orc_init(int d, int nx, int ny, int nz, const double* n0, double* f) {
  VelSet vs = make_velset(d);
  Geom g{d, nx, ny, nz};
  const long N = g.N();
  for (int i = 0; i < vs.Q; ++i)
    for (long c = 0; c < N; ++c) f[(long)i * N + c] = vs.w[i] * n0[c];
  return 0;
}

// Advance f (Q x N, SoA, x fastest) by nsteps. Returns 0, -1 (bad shell), 5 (non-finite mass).
int orc_run(int d, int nx, int ny, int nz, double tau, double aF, double G, int kind, double p, int nshells,
            const int* codes, const double* W, double* f, long nsteps) {
  VelSet vs = make_velset(d);
  Stencil st;
  if (!make_stencil(d, nshells, codes, st)) return -1;
  Geom g{d, nx, ny, nz};
  const long N = g.N();
  std::vector<double> buf((size_t)vs.Q * N);
  for (long t = 0; t < nsteps; ++t) {
    step<double>(g, vs, st, W, G, tau, aF, kind, p, f, buf.data());
    std::memcpy(f, buf.data(), sizeof(double) * buf.size());
  }
  double M = 0.0;
  for (long c = 0; c < (long)vs.Q * N; ++c) M += f[c];
  return std::isfinite(M) ? 0 : 5;
}

// Macroscopic fields of a state: n (N), j (3N, interleaved xyz), psi (N), F (3N), u (3N).
int orc_fields(int d, int nx, int ny, int nz, double G, int kind, double p, int nshells, const int* codes,
               const double* W, const double* f, double* n_out, double* j_out, double* psi_out,
               double* F_out, double* u_out) {
  VelSet vs = make_velset(d);
  Stencil st;
  if (!make_stencil(d, nshells, codes, st)) return -1;
  Geom g{d, nx, ny, nz};
  std::vector<double> n, j, psi, F;
  macro_fields<double>(g, vs, st, W, G, kind, p, f, n, j, psi, F);
  const long N = g.N();
  for (long c = 0; c < N; ++c) {
    if (n_out) n_out[c] = n[c];
    if (psi_out) psi_out[c] = psi[c];
    for (int k = 0; k < 3; ++k) {
      if (j_out) j_out[3 * c + k] = j[3 * c + k];
      if (F_out) F_out[3 * c + k] = F[3 * c + k];
      if (u_out) u_out[3 * c + k] = (j[3 * c + k] + 0.5 * F[3 * c + k]) / n[c];
    }
  }
  return 0;
}

// Lattice pressure tensor (d = 2) of a state: out is 3 x N (xx, yy, xy planes).
int orc_ptensor2d(int nx, int ny, double G, int kind, double p, int nshells, const int* codes,
                  const double* W, const double* f, double* out) {
  VelSet vs = make_velset(2);
  Stencil st;
  if (!make_stencil(2, nshells, codes, st)) return -1;
  Geom g{2, nx, ny, 1};
  std::vector<double> n, j, psi, F;
  macro_fields<double>(g, vs, st, W, G, kind, p, f, n, j, psi, F);
  const long N = g.N();
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    double P[3];
    ptensor2d_cell<double>(g, st, codes, W, G, n, psi, c, P);
    out[c] = P[0]; out[N + c] = P[1]; out[2 * N + c] = P[2];
  }
  return 0;
}

// Lattice pressure tensor by the link-sharing rule (d = 2 or 3): out holds 6 planes of N
// values (xx, yy, zz, xy, xz, yz).
int orc_ptensor(int d, int nx, int ny, int nz, double G, int kind, double p, int nshells, const int* codes,
                const double* W, const double* f, double* out) {
  VelSet vs = make_velset(d);
  Stencil st;
  if (!make_stencil(d, nshells, codes, st)) return -1;
  Geom g{d, nx, ny, nz};
  std::vector<double> n, j, psi, F;
  macro_fields<double>(g, vs, st, W, G, kind, p, f, n, j, psi, F);
  const long N = g.N();
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    double P[6];
    ptensor_cell<double>(g, st, W, G, n, psi, c, P);
    for (int k = 0; k < 6; ++k) out[k * N + c] = P[k];
  }
  return 0;
}

// Droplet observables (d = 3, cubic domain) of a state f: out = (dP, C_d, R_s, sigma_s, R_e, delta).
int orc_droplet_obs3d(int n_, double G, int kind, double p, int nshells, const int* codes, const double* W,
                      const double* f, int cx, int cy, int cz, int bubble, double* out) {
  VelSet vs = make_velset(3);
  Stencil st;
  if (!make_stencil(3, nshells, codes, st)) return -1;
  Geom g{3, n_, n_, n_};
  std::vector<double> n, j, psi, F;
  macro_fields<double>(g, vs, st, W, G, kind, p, f, n, j, psi, F);
  double o[6];
  droplet_obs3d<double>(g, st, W, G, n, psi, cx, cy, cz, bubble, o);
  for (int k = 0; k < 6; ++k) out[k] = o[k];
  return 0;
}

// Droplet observables (d = 2) of a state f: out = (dP, C_d, R_s, sigma_s, R_e, R_e - R_s).
int orc_droplet_obs2d(int nx, int ny, double G, int kind, double p, int nshells, const int* codes,
                      const double* W, const double* f, int cx, int cy, int bubble, double* out) {
  if (nx != ny) return -2;
  VelSet vs = make_velset(2);
  Stencil st;
  if (!make_stencil(2, nshells, codes, st)) return -1;
  Geom g{2, nx, ny, 1};
  std::vector<double> n, j, psi, F;
  macro_fields<double>(g, vs, st, W, G, kind, p, f, n, j, psi, F);
  double o[6];
  droplet_obs2d<double>(g, st, codes, W, G, n, psi, cx, cy, bubble, o);
  for (int k = 0; k < 6; ++k) out[k] = o[k];
  return 0;
}

// Tangent-linear run (d = 2): starting from f_i = w_i n0, advance nsteps carrying derivatives
// with respect to (W_0 .. W_{nshells-1}, G); returns the six droplet observables and their
// Jacobian jac[6 x (nshells+1)], the FP64 reference gradient.
int orc_droplet_tl2d(int nx, int ny, double tau, double aF, double G, int kind, double p, int nshells,
                     const int* codes, const double* W, const double* n0, long nsteps, int cx, int cy,
                     int bubble, double* obs, double* jac) {
  if (nshells + 1 > ND) return -3;
  if (nx != ny) return -2;
  VelSet vs = make_velset(2);
  Stencil st;
  if (!make_stencil(2, nshells, codes, st)) return -1;
  Geom g{2, nx, ny, 1};
  const long N = g.N();
  std::vector<Dual> Wd(nshells);
  for (int s = 0; s < nshells; ++s) { Wd[s] = Dual(W[s]); Wd[s].d[s] = 1.0; }
  Dual Gd(G);
  Gd.d[nshells] = 1.0;
  std::vector<Dual> f((size_t)vs.Q * N), fo((size_t)vs.Q * N);
  for (int i = 0; i < vs.Q; ++i)
    for (long c = 0; c < N; ++c) f[(long)i * N + c] = Dual(vs.w[i] * n0[c]);
  for (long t = 0; t < nsteps; ++t) {
    step<Dual>(g, vs, st, Wd.data(), Gd, tau, aF, kind, p, f.data(), fo.data());
    std::swap(f, fo);
  }
  std::vector<Dual> n, j, psi, F;
  macro_fields<Dual>(g, vs, st, Wd.data(), Gd, kind, p, f.data(), n, j, psi, F);
  Dual o[6];
  droplet_obs2d<Dual>(g, st, codes, Wd.data(), Gd, n, psi, cx, cy, bubble, o);
  for (int k = 0; k < 6; ++k) {
    obs[k] = o[k].v;
    for (int q = 0; q <= nshells; ++q) jac[k * (nshells + 1) + q] = o[k].d[q];
  }
  return std::isfinite(obs[0]) ? 0 : 5;
}

}  // extern "C"
