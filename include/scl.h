/*
 * scl.h - C ABI of libscl, an MI355X (gfx950) implementation of the Shan-Chen multiphase
 * lattice Boltzmann time step with an extended, tunable forcing stencil
 * (Lulli & Ching, "Higher-order Tuning of Interface Physics in Multiphase Lattice
 * Boltzmann", arXiv 2505.23647).
 *
 * One time step, per lattice site x (Sec. "Lattice Boltzmann" and Sec. "Shan-Chen Model"):
 *   n = sum_i f_i, j = sum_i f_i xi_i, psi = psi(n)
 *   F(x) = -G c_s^2 psi(x) sum_a W(|e_a|^2) psi(x + e_a) e_a                     eq. (sc_f)
 *   u = (j + F/2) / n                                       (shifted velocity after eq. GuoForcing)
 *   f_i(x + xi_i, t+1) = f_i - (f_i - f_i^eq(n, u))/tau + F_i(u, F)       eqs. (lbm), (omega_i),
 *                                                                         (f_eq), (GuoForcing)
 * with c_s^2 = 1/3, the second-order Hermite equilibrium, Guo forcing with T = 2 u F, and
 * periodic boundaries in every direction.
 *
 * Conventions shared by every call
 *   - Every call returns scl_status; nothing throws across the ABI. scl_last_error() gives a
 *     thread-local text for the last failure on the calling thread.
 *   - Arguments are validated before any device work; a rejected call changes nothing.
 *   - The lattice owns its device buffers. The caller owns every array it passes (host or
 *     device) and keeps it alive for the duration of the call only.
 *   - Device work is ordered on the HIP stream given to scl_create (NULL = the default
 *     stream). Calls that return host data synchronise that stream before returning.
 *   - Site order: domains one after the other (in the order given to scl_create); inside a
 *     domain x fastest, then y, then z. "cells" below is the total over all domains.
 *   - Population layout: domain by domain, each domain a [Q][cells_of_domain] block.
 *   - Velocity order (see scl_velocity_set): D2Q9 rest, (1,0), (0,1), (-1,0), (0,-1),
 *     (1,1), (-1,1), (-1,-1), (1,-1); D3Q19 rest, +-x, +-y, +-z faces, then the 12 edges.
 *   - Shell codes name forcing-vector symmetry groups: the code is |e|^2, all vectors that a
 *     generator reaches by permutations and sign flips (Fig. 1 and Sec. on sigma_1 tuning).
 *     Supported: 2D {1,2,4,5,8,9,16,18}; 3D {1,2,3,4,5,6,8,9,1009,16,18} (see
 *     scl_set_stencil for the groups of 9, 1009, 16 and 18).
 *   - G follows eq. (sc_f): the force carries an explicit c_s^2, and the critical coupling of
 *     psi = exp(-1/n) with e_2 = 1 is G_c = -e^2.
 */
#ifndef SCL_H
#define SCL_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCL_ABI_VERSION 3

typedef struct scl_lattice_s* scl_lattice;

typedef enum {
  SCL_OK = 0,
  SCL_E_INVALID = 1,     /* bad argument (sizes, values, shell codes, missing pointer) */
  SCL_E_NOMEM = 2,       /* device allocation failed */
  SCL_E_DEVICE = 3,      /* a HIP call failed; scl_last_error() holds hipGetErrorString */
  SCL_E_STATE = 4,       /* call out of order (e.g. scl_step before scl_init_density) */
  SCL_E_NONFINITE = 5,   /* a checked readout found NaN or Inf (the run diverged) */
  SCL_E_UNSUPPORTED = 6  /* valid request the library does not implement */
} scl_status;

typedef enum { SCL_D2Q9 = 0, SCL_D3Q19 = 1 } scl_velset;

/* Storage / arithmetic of the populations.
 *   SCL_FP64          double storage, double arithmetic.
 *   SCL_FP32          float storage, float arithmetic.
 *   SCL_FP32_SHIFTED  float storage of g_i = f_i - w_i rho0 (rho0 = the domain's mean initial
 *                     density), float arithmetic on the deviations.
 *   SCL_FP16S_FP32    IEEE binary16 storage of g_i (round to nearest even), float arithmetic.
 * Readouts (mass, momentum, pressure tensor, observables) are always accumulated in double. */
typedef enum { SCL_FP64 = 0, SCL_FP32 = 1, SCL_FP32_SHIFTED = 2, SCL_FP16S_FP32 = 3 } scl_precision;

/* Pseudopotential psi(n).
 *   SCL_PSI_EXP      exp(-1/n)                      (eps = 0 case, Sec. on sigma_1 tuning)
 *   SCL_PSI_EPS      (n / (eps + n))^(1/eps)        eq. (psieps); eps > 0 from psi_param
 *   SCL_PSI_CLASSIC  1 - exp(-n)                    textbook form, not used by the paper */
typedef enum { SCL_PSI_EXP = 0, SCL_PSI_EPS = 1, SCL_PSI_CLASSIC = 2 } scl_psi;

/* ABI version of the loaded library (SCL_ABI_VERSION of the build). */
int32_t scl_abi_version(void);

/* Text of the last error on this thread ("" if none). Owned by the library. */
const char* scl_last_error(void);

/* Velocity set of vs: writes Q vectors (3 ints each, z = 0 in 2D) to xi and Q weights to w
 * (either may be NULL); returns Q, or -1 for an unknown vs. */
int32_t scl_velocity_set(scl_velset vs, int32_t* xi, double* w);

/* Device-memory source for lattices created afterwards (for callers that pool their device
 * memory, e.g. a framework's caching allocator). Every device buffer a lattice holds, and the
 * temporaries of its calls, come from alloc(bytes, ctx, stream) and go back through
 * free_(ptr, ctx, stream), where stream is the lattice's hipStream_t: a release is stream
 * ordered, and the memory may serve later work on that stream. alloc returns NULL when it
 * cannot allocate (the call then fails with SCL_E_NOMEM or SCL_E_DEVICE). Both functions NULL
 * (the default) means hipMalloc / hipFree. A lattice keeps the source it was created with until
 * scl_destroy, whatever is installed later. Process-wide setting; not synchronised with
 * concurrent scl_create calls on other threads. SCL_E_INVALID if exactly one function is NULL. */
scl_status scl_set_allocator(void* (*alloc)(size_t bytes, void* ctx, void* stream),
                             void (*free_)(void* ptr, void* ctx, void* stream), void* ctx);

/* Create a lattice of ndom independent periodic domains.
 *   dims: ndom x 3 ints (nx, ny, nz), nz = 1 for D2Q9. Each extent must be >= 1; the
 *         domain must hold at least one site. Batched domains may differ in size.
 *   hip_stream: hipStream_t on which all work is ordered (NULL = default stream).
 * Allocates two population buffers (A/B) of Q x cells x sizeof(storage), from the source
 * installed by scl_set_allocator (hipMalloc by default). */
scl_status scl_create(scl_velset vs, scl_precision prec, int32_t ndom, const int32_t* dims,
                      void* hip_stream, scl_lattice* out);

/* Free every device buffer of the lattice. NULL is accepted. */
scl_status scl_destroy(scl_lattice lat);

/* Physics per domain (arrays of ndom doubles): relaxation time tau > 1/2, coupling G
 * (eq. sc_f convention; any finite value), pseudopotential kind and its parameter
 * (eps > 0 for SCL_PSI_EPS; ignored otherwise; psi_param may be NULL then). */
scl_status scl_set_physics(scl_lattice lat, const double* tau, const double* G, scl_psi kind,
                           const double* psi_param);

/* Optional F^2 part of the Guo tensor (appendix on the role of eps and e4): with A != 0 the
 * rank-two tensor of eq. (GuoForcing) becomes T_ab = 2 u_a F_b - (A/tau) F_a F_b, which adds
 * a forcing contribution eps_F to the interface-profile exponent. A: ndom doubles (host),
 * finite; the default A = 0 is the paper's T = 2uF. Also used by the adjoint. */
scl_status scl_set_force_squared(scl_lattice lat, const double* A);

/* Forcing stencil (eq. sc_f): nshells distinct shell codes and the weights W(code) per
 * domain, W laid out ndom x nshells. Weights must be finite. A shell code is |e|^2 of its
 * vectors (App. "Defining the stencil"). D2Q9 accepts 1, 2, 4, 5, 8, 9, 16, 18 (9: (3,0),
 * 16: (4,0), 18: (3,3) groups; a stencil using 9, 16 or 18 reaches 4 sites and runs with
 * 128- or 256-lane strips, one site per lane); D3Q19 accepts 1, 2, 3, 4, 5, 6, 8 and, for
 * the 11-shell stencil of the 3D Tolman-length tuning table (tab. e4e6e8_tuning_6_3d), 9
 * (the (2,2,1) group), 1009 (the (3,0,0) group, also |e|^2 = 9), 16 ((4,0,0)) and 18
 * ((3,3,0)); a 3D stencil using any of these four reaches 4 sites and runs with tiles 2
 * and 3 (scl_set_tiling). At most 12 shells. */
scl_status scl_set_stencil(scl_lattice lat, int32_t nshells, const int32_t* shell_codes, const double* W);

/* Initial state f_i(x, 0) = w_i n0(x): the fluid at rest. n0 holds cells doubles (host, or
 * device when is_device_ptr != 0), every value finite and > 0. Resets the step counter and,
 * for shifted storage, sets rho0 per domain to the mean of n0 over that domain. */
scl_status scl_init_density(scl_lattice lat, const double* n0, int32_t is_device_ptr);

/* Advance every domain by nsteps >= 0 time steps (asynchronous on the lattice stream).
 * Needs scl_set_physics, scl_set_stencil and scl_init_density first (SCL_E_STATE). */
scl_status scl_step(scl_lattice lat, int64_t nsteps);

/* As scl_step, and returns the elapsed device time of the whole call in milliseconds,
 * measured with HIP events recorded on the lattice stream around the launches. */
scl_status scl_step_timed(scl_lattice lat, int64_t nsteps, double* ms);

/* Number of steps taken since scl_init_density. */
scl_status scl_get_step_count(scl_lattice lat, int64_t* steps);

/* Density n = sum_i f_i of the current state, cells doubles (host or device). */
scl_status scl_get_density(scl_lattice lat, double* out, int32_t is_device_ptr);

/* Velocity u = (j + F/2)/n of the current state, laid out d x cells (all x, then all y...). */
scl_status scl_get_velocity(scl_lattice lat, double* out, int32_t is_device_ptr);

/* Force F (eq. sc_f) of the current state, laid out d x cells. */
scl_status scl_get_force(scl_lattice lat, double* out, int32_t is_device_ptr);

/* Populations f_i(x, t) of the current state (the post-streaming values), in the population
 * layout above, as doubles. */
scl_status scl_get_populations(scl_lattice lat, double* out, int32_t is_device_ptr);

/* Replace the state by the given populations (same layout as scl_get_populations), rounded
 * to the storage precision. Keeps the step counter and rho0. */
scl_status scl_set_populations(scl_lattice lat, const double* in, int32_t is_device_ptr);

/* Per-domain mass M = sum_x n and total physical momentum sum_x (j + F/2), accumulated in
 * double with a fixed-order tree (bitwise reproducible). mass: ndom doubles; momentum:
 * ndom x d doubles (may be NULL). Returns SCL_E_NONFINITE if any mass is NaN or Inf. */
scl_status scl_reduce_conserved(scl_lattice lat, double* mass, double* momentum);

/* Lattice pressure tensor of the current state in double, with the ideal part n c_s^2 delta
 * added (Sec. "Interface Physics"). D2Q9: out holds 3 x cells values, the planes Pxx, Pyy, Pxy,
 * by the d = 2 appendix on the lattice pressure tensor (groups along a line plus the
 * irregular pairs of |e|^2 = 5). D3Q19: 6 x cells values, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz, by the
 * d = 3 appendix: every link y -> y + e shares its interaction along the link, 1/(2K) at each
 * point y + m e / K (K = max_i |e_i|, m = 0 .. K-1), a point between sites handing its share
 * equally to the sites around it; this gives the appendix's symmetric groups and the
 * irregular pairs of the (2,1,0), (2,1,1), (2,2,1) groups. */
scl_status scl_get_pressure_tensor(scl_lattice lat, double* out, int32_t is_device_ptr);

/* Droplet / bubble observables of each square D2Q9 domain or cubic D3Q19 domain (Sec.
 * "Interface Physics" and the Laplace-law paragraph of the sigma_1 tuning section), in double.
 * d = 3 uses Pbar = tr P / 3, the weight r^2 in C_d, R_s = (6 C_d / dP)^(1/3),
 * sigma_s = dP R_s / 2 and the sphere volume for R_e; center then holds ndom x 3 ints.
 * d = 2:
 *   Pbar = (Pxx + Pyy)/2, dP = Pbar(centre) - Pbar(corner (0,0));
 *   C_d = int_0^{L/2} r (Pbar(corner) - Pyy(centre + r e_x)) dr, trapezoid on sites, mean of
 *         the +x and -x half-lines;
 *   R_s = sqrt(2 C_d / dP), sigma_s = dP R_s (stationary point of sigma[R]);
 *   R_e from pi R_e^2 n(centre) + (L^2 - pi R_e^2) n(corner) = M;
 *   delta = (-1)^b (R_e - R_s), the Tolman length measured from the liquid side.
 * The inside pressure is the higher one for droplets and bubbles alike (dP, R_s, sigma_s > 0
 * for both); the sign (-1)^b of a bubble is that of its curvature.
 * R_s, sigma_s and delta are NaN while C_d / dP < 0 (an unrelaxed domain).
 * center: ndom x 2 ints (x, y); is_bubble: ndom bytes (b), may be NULL (droplets).
 * out: ndom x 6 doubles (dP, C_d, R_s, sigma_s, R_e, delta). Host arrays. */
scl_status scl_droplet_observables(scl_lattice lat, const int32_t* center, const int8_t* is_bubble,
                                   double* out);

/* Flat-interface observables of each domain holding a slab that varies along x (two
 * interfaces, one in each half [0, nx/2) and [nx/2, nx); profiles are means over the rows
 * along y, and z for D3Q19),
 * in double, from the lattice pressure tensor (Sec. "Interface Physics", Sec. "Tolman
 * Length"), per interface:
 *   sigma_0 = sum_x (P_N - P_T) (eq. sigma0pnpt), P_N = Pxx, P_T = Pyy;
 *   z_s = sum_x x (P_N - P_T) / sigma_0 (eq. ZSDef);
 *   z_e: position of the sharp step between the bulk densities that holds the half's mass
 *        (vanishing adsorbance), site x standing for the cell [x - 1/2, x + 1/2);
 *   delta = z_e - z_s measured from the liquid towards the vapour (eq. zemzs);
 *   delta_ads = Gamma(z_s) / (n_l - n_g) (eq. deltaads).
 * bulk: ndom x 2 doubles (n_l, n_g) or NULL (then the row-mean profile's max and min).
 * out: ndom x 2 x 5 doubles (sigma_0, z_s, z_e, delta, delta_ads) for the lower half, then
 * the upper. nx must be even and >= 4. Host arrays. */
scl_status scl_flat_observables(scl_lattice lat, const double* bulk, double* out);

/* Tiling of the fused step.
 *   2D marching strips: strip = output lanes per workgroup (64, 128, 256 or 512; 0 =
 *       automatic: 512 for FP32 storage, 256 otherwise and for the reach-4 shell set); seg =
 *       rows one workgroup marches (>= 1; 0 = automatic: 64 for 4- and 2-byte storage, 32
 *       for FP64, halved down to 16 while the lattice gives fewer than 512 work items);
 *       cpl = sites per lane (1, or 2 for vector accesses, which needs every domain width even
 *       and a strip of at most 256; 0 = automatic: one site per lane).
 *   2D one-shot tiles: strip = -256 or -512 (lanes per workgroup), seg = rows per tile (8, 16,
 *       24 or 32; 0 = 16; 512 lanes need at least 16), cpl = tile width in 64-column units (0 or
 *       1: 64, 2: 128): one workgroup per tile of 64 x seg or 128 x seg sites, no march. Needs every domain's population plane (sites x bytes per
 *       value) under 2 GiB (SCL_E_UNSUPPORTED otherwise). Results are bitwise those of the
 *       marching strips. With no tiling requested and the shell sets of reach 1 and 2, FP64
 *       storage runs 256-lane tiles of 128 x 8 sites; domains so narrow that the automatic
 *       strips would leave more than 1/8 of their lanes idle run 512-lane tiles of 64 x 16
 *       sites; FP16 storage otherwise runs 256-lane tiles of 128 x 16 sites; scl_adjoint's
 *       recording pass always marches.
 *   3D: strip = tile index (1: 64x4, 2: 64x8, 3: 32x8, 4: 128x4 output sites per workgroup;
 *       automatic until set: 128x4 for FP32 storage, 64x4 for FP16 storage, 64x8 for FP64
 *       and for the reach-4 set, which runs tiles 2 and 3 only); seg = planes one workgroup
 *       marches; cpl is ignored.
 * 0 keeps the current value (for cpl: automatic). */
scl_status scl_set_tiling(scl_lattice lat, int32_t strip, int32_t seg, int32_t cpl);
/* Current tiling (2D: the strip in use, or -lanes with seg = rows per tile and cpl = width in
 * 64-column units when one-shot tiles are in use; 3D: the tile in use); cpl may be NULL. seg 0
 * means the automatic choice. */
scl_status scl_get_tiling(scl_lattice lat, int32_t* strip, int32_t* seg, int32_t* cpl);

/* Autotuner: times the candidate tilings on this lattice (advancing it by the steps it
 * uses, see scl_get_step_count) and keeps the fastest. If cache_path is not NULL the choice
 * is read from / appended to that text file, keyed by device name, velocity set, stencil
 * reach, precision and domain sizes. */
scl_status scl_tune(scl_lattice lat, const char* cache_path);

/* Replay the step loop through HIP graphs of k launches (k even, 0 = plain launches).
 * The graph is captured on first use and re-captured after any change of tiling,
 * physics, stencil or state. */
scl_status scl_set_graph_steps(scl_lattice lat, int32_t k);

/* ---------------------------------------------------------------------------------------
 * Adjoint (reverse-mode gradients of a loss of the final state with respect to the shell
 * weights W and the coupling G). The transpose of the step is derived from eqs. (lbm),
 * (omega_i), (f_eq), (GuoForcing) and (sc_f); D2Q9 with FP64 or FP32 populations.
 * ------------------------------------------------------------------------------------- */

/* Advance nsteps >= 1 steps like scl_step, storing the state every `every` steps (and the
 * initial and final states) in a device checkpoint pool owned by the lattice. Required before
 * scl_adjoint; any later change of the state (step, init, set_populations) invalidates it. */
scl_status scl_checkpointed_forward(scl_lattice lat, int64_t nsteps, int32_t every);

/* Gradient of L through the last checkpointed forward. The seed is dL/df at the final time:
 * seed_n (cells doubles, device) gives dL/df_i(x) = seed_n(x) for every i (a loss of the
 * density), seed_f (Q x cells doubles, device, population layout) adds a general seed; either
 * may be NULL. Segment by segment (last to first) the forward is recomputed from its
 * checkpoint, recording n, j, F per step, and the adjoint step runs backwards.
 * grad_W (ndom x nshells, host, shells in the order of scl_set_stencil) and grad_G (ndom,
 * host) receive dL/dW and dL/dG through the time loop (the explicit dependence of a readout
 * on W and G is added by scl_droplet_observables_vjp). Restores the final state. */
scl_status scl_adjoint(scl_lattice lat, const double* seed_n, const double* seed_f, double* grad_W, double* grad_G);

/* dL/df at the initial time of the last scl_adjoint, as doubles in the population layout. */
scl_status scl_get_adjoint_populations(scl_lattice lat, double* out, int32_t is_device_ptr);

/* Vector-Jacobian product of scl_droplet_observables at the current state: given
 * g_obs = dL/d(observables) (ndom x 6, host) writes seed_n = dL/dn(x) (cells doubles, host or
 * device), and the explicit derivatives of the readout: grad_W (ndom x nshells, host) and
 * grad_G (ndom, host), which the caller adds to the scl_adjoint result. */
scl_status scl_droplet_observables_vjp(scl_lattice lat, const int32_t* center, const int8_t* is_bubble,
                                       const double* g_obs, double* seed_n, int32_t is_device_ptr,
                                       double* grad_W, double* grad_G);

#ifdef __cplusplus
}
#endif
#endif /* SCL_H */
