/*
 * mps_lbm.h - C ABI of the MI355X (gfx950) matrix-product-state lattice
 * Boltzmann library.
 *
 * The library advances a D3Q19 or D3Q15 BGK lattice Boltzmann simulation
 * whose Q = 19 or 15 particle distribution functions are each held as a
 * matrix product state
 * (MPS) over scale-ordered grid bits (paper: "Tensor Network Lattice
 * Boltzmann Method for Data-Compressed Fluid Simulations", Sections 2-3).
 * All state lives in device memory owned by the handle; every computation
 * of a step runs in the library's HIP kernels on the handle's stream.
 *
 * Conventions for every entry point:
 *  - Dense fields are C-order FP64 arrays indexed [x][y][z] (x slowest),
 *    side N = 2^n; vector fields are [3][N][N][N]; population arrays are
 *    [Q][N][N][N].  D3Q19 order: rest, +x,-x, +y,-y, +z,-z, then the
 *    twelve edges as opposite pairs (+x+y,-x-y), (+x-y,-x+y), (+x+z,-x-z),
 *    (+x-z,-x+z), (+y+z,-y-z), (+y-z,-y+z).  D3Q15 order: rest, +x,-x,
 *    +y,-y, +z,-z, then the eight corners as opposite pairs (+++,---),
 *    (++-,--+), (+-+,-+-), (-++,+--).
 *  - Host buffers are owned by the caller; the library copies inputs during
 *    the call and writes only into the output buffer it is given.
 *  - Return value 0 is success; negative values are the MPS_LBM_E* codes
 *    below.  On error nothing is written to outputs and
 *    mps_lbm_last_error() returns a message (thread-local).  No C++
 *    exception crosses this interface.
 *  - A handle must not be used from two threads at once.
 */
#ifndef MPS_LBM_H
#define MPS_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPS_LBM_OK 0
#define MPS_LBM_EINVAL (-1)       /* bad argument or configuration        */
#define MPS_LBM_ENOMEM (-2)       /* device allocation failed             */
#define MPS_LBM_EHIP (-3)         /* a HIP runtime call failed            */
#define MPS_LBM_ENUMERIC (-4)     /* NaN/Inf or SVD non-convergence       */
#define MPS_LBM_EUNSUPPORTED (-5) /* valid but not implemented            */

#define MPS_LBM_D3Q19 19 /* rest, 6 axis, 12 edge velocities (1/3, 1/18, 1/36) */
#define MPS_LBM_D3Q15 15 /* rest, 6 axis, 8 corner velocities (2/9, 1/9, 1/72): the
                            set of the paper's 3D runs (Section 4.1) */

/* arithmetic of the step (storage and contractions); the R-factor SVDs,
   rank selection and 1/rho coefficients are FP64 under every policy, and
   under FP32, BF16 and BF16X3 the inverse density (Section 3.2, Appendix B:
   the sums and variational products of the Taylor or Newton-Schulz form)
   runs in FP64 too, on a copy of rho converted to FP64, its result
   converted back to FP32.
   BF16: FP32 storage and factorisations as MPS_LBM_FP32, with the
   contractions of the variational products (Section 2.3) run on BF16 MFMA
   (operands rounded to BF16, FP32 accumulation).  BF16X3: as BF16, but each
   FP32 operand is split exactly into three BF16 terms and the six products
   of significant order are accumulated, which keeps the contractions at
   about FP32 accuracy on the BF16 matrix units. */
#define MPS_LBM_FP64 0
#define MPS_LBM_FP32 1
#define MPS_LBM_BF16 2
#define MPS_LBM_BF16X3 3

/* inverse density: second-order Taylor expansion about the mean density
   rho_0 (Section 3.2), or k Newton-Schulz steps from 1/rho_0 (k steps equal
   the Taylor expansion of order 2^k - 1) */
#define MPS_LBM_INV_TAYLOR2 0
#define MPS_LBM_INV_NEWTON 1

/* face boundary types for non-periodic axes (Section 3.2.1) */
#define MPS_LBM_BC_NONE 0
#define MPS_LBM_BC_VELOCITY 1 /* bounce-back with wall velocity u_b, rho_b = rho_0 */
#define MPS_LBM_BC_PRESSURE 2 /* anti-bounce-back with density rho_b, u_b = local u */

/* what mps_lbm_to_dense writes */
#define MPS_LBM_POPS 0 /* [Q][N][N][N] populations                        */
#define MPS_LBM_RHO 1  /* [N][N][N]     rho = sum_i f_i                     */
#define MPS_LBM_J 2    /* [3][N][N][N]  j = sum_i c_i f_i                   */
#define MPS_LBM_VEL 3  /* [3][N][N][N]  u = j / rho (0 where rho = 0)       */

#define MPS_LBM_MAX_SITES 10 /* n <= 10 (N <= 1024)                        */

typedef struct mps_lbm mps_lbm_t; /* opaque handle; owns all device state */

typedef struct {
  int n;            /* N = 2^n cells per axis, 2 <= n <= MPS_LBM_MAX_SITES */
  int lattice;      /* MPS_LBM_D3Q19 | MPS_LBM_D3Q15                      */
  int chi_max;      /* bond dimension cap of every population MPS, >= 1    */
  int chi_mask_max; /* rank cap of the obstacle-mask MPS; <= 0 means no cap:
                       the mask is then decomposed to tol_mask, i.e. to
                       machine precision (Section 5.2 sets the mask bond
                       dimension that way), with its own storage, and may
                       exceed chi_max                                     */
  double tol;       /* relative Frobenius truncation tolerance of a rounding */
  double tol_mask;  /* truncation tolerance of the mask decomposition      */
  double tau;       /* BGK relaxation time, > 1/2                          */
  double g[3];      /* body acceleration; force density F = rho g          */
  int inv_rho_mode; /* MPS_LBM_INV_TAYLOR2 | MPS_LBM_INV_NEWTON            */
  int inv_rho_iters;/* Newton-Schulz steps (>= 1) when mode is NEWTON      */
  int precision;    /* MPS_LBM_FP64 | MPS_LBM_FP32 | MPS_LBM_BF16 | ..X3   */
  int sweeps;       /* variational-product sweeps 1->n->1 (the paper: 2)   */
  int axis_open[3]; /* 0 = periodic (cyclic shift), 1 = open (non-cyclic)  */
  int face_bc[6];   /* faces x-lo, x-hi, y-lo, y-hi, z-lo, z-hi            */
  double face_val[6][3]; /* velocity faces: u_b; pressure faces: {rho_b,0,0} */
  unsigned long long seed; /* draws the Gaussian test matrix of the sketches */
  int rank_predictor;  /* 1: truncations are first tried on a randomized
                          sketch sized by the rank the same truncation chose
                          in the previous step, with exact-error acceptance
                          and full fallback (FP32/BF16 only); 2: as 1, with
                          the learned predictor below sizing the sketch once
                          trained; 0: off                                   */
  int rank_oversample; /* sketch width = predicted rank + this (>= 1)       */
} mps_lbm_config;

typedef struct {
  long long step;          /* steps taken since init                       */
  double mass;             /* <1, rho> = sum_i <1, f_i>                     */
  double momentum[3];      /* sum_i c_i <1, f_i>                            */
  double rho0;             /* mean fluid density used by the last step      */
  double n_fluid;          /* N^3 - <1, m_O>                                */
  int max_bond;            /* largest bond over the Q populations           */
  int bonds[19][MPS_LBM_MAX_SITES]; /* bond dims r_1..r_{n-1} per population
                                       (rows Q..18 zero under D3Q15)      */
  double nvps;             /* sum over populations of the core entries in use */
  double compression;      /* Q N^3 / nvps                                  */
  double max_discarded;    /* largest relative discarded weight of a rounding
                              in the last step                              */
  int mask_bond;           /* largest bond of the obstacle-mask MPS          */
  double mask_trunc_err;   /* ||m - m~|| / ||m|| of the mask decomposition   */
  long long roundings;     /* roundings in the last step                    */
  long long products;      /* variational products in the last step         */
  int svd_failures;        /* Jacobi SVDs that hit the sweep limit (total)   */
  int nonfinite;           /* 1 if a NaN/Inf was seen in the state           */
  double jacobi_sweeps;    /* mean Jacobi sweeps per truncation problem (total) */
  int lds_bytes;           /* LDS per workgroup the factorisation kernels use */
  long long rs_attempted;  /* truncations tried on a randomized sketch (total) */
  long long rs_accepted;   /* of those, accepted without fallback (total)    */
  double jacobi_sweeps_wide; /* the same for factors wider than 128 columns */
  double jacobi_cols_wide; /* their mean column count (numerical rank)      */
  double face_trunc_err;   /* largest ||m_B - m_B~|| / ||m_B|| of the open-face
                              masks (fluid cells of the face plane), which are
                              decomposed at tol_mask with rank cap chi_max */
  double dp_p0;            /* Delta p / p_0 over the region set by
                              mps_lbm_set_region (Section 4.2); 0 if none   */
  double region_cells;     /* |D|: fluid cells of that region               */
  double region_trunc_err; /* ||m_D - m_D~|| / ||m_D|| of its MPS            */
} mps_lbm_obs;

/*
 * Register the source of every device buffer of handles created from now on
 * (process-wide; each handle keeps the allocator it was created with).
 * alloc(bytes, stream, ctx) returns device memory usable on `stream` (the
 * handle's hip_stream, NULL for handle-less calls) or NULL when it has none
 * left, which the calling entry point reports as MPS_LBM_ENOMEM; free_(ptr,
 * stream, ctx) takes back what alloc returned.  Meant for a framework's
 * caching allocator (the Python binding registers PyTorch's), so that the
 * library's state, workspaces and read-back staging share its memory pool.
 * Both NULL restore hipMalloc / hipFree.  The library calls free_ only after
 * the stream has finished with the buffer.  (Section 3.2 describes the
 * step; this call only concerns where its memory lives.)
 * Errors: EINVAL (exactly one of alloc, free_ is NULL).
 */
int mps_lbm_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                          void (*free_)(void* ptr, void* stream, void* ctx), void* ctx);

/* Fill *cfg with defaults: D3Q19, FP64, TAYLOR2, 2 sweeps, tol 1e-10,
   tol_mask 1e-12, tau 0.8, periodic, no force, chi_max 16, no rank
   predictor (oversampling 16). */
void mps_lbm_default_config(mps_lbm_config* cfg);

/*
 * Create a simulation.  Initial populations are the equilibrium
 * f_i = (1 - m_O) w_i rho (1 + 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u.u)
 * of the given rho [N][N][N] and u [3][N][N][N] (equilibrium equation),
 * or, when f is non-NULL, the given populations [Q][N][N][N] (rho and u
 * are then ignored and may be NULL).  solid [N][N][N] (1 = solid) defines
 * the obstacle mask m_O (Section 3.2.1, objects equation); NULL = none.
 * Each field is decomposed into an MPS by successive truncated SVDs
 * (Section 2.1, svd-comp equation) on the device.  hip_stream is the
 * hipStream_t every later call of this handle runs on (NULL = default).
 * Errors: EINVAL (n out of range, chi_max < 1, tau <= 1/2, unknown lattice,
 * precision, BC or inverse mode, missing fields), ENOMEM, EHIP.
 */
int mps_lbm_init_from_field(const mps_lbm_config* cfg, const double* rho,
                            const double* u, const double* f,
                            const uint8_t* solid, void* hip_stream,
                            mps_lbm_t** out);

/*
 * Create a simulation whose obstacle geometry repeats a unit geometry on a
 * coarse grid (Appendix D): solid_outer [L][L][L] (L = 2^l) marks the
 * coarse cells that hold the unit geometry solid_inner [K][K][K]
 * (K = 2^(n-l)), both C-order uint8 host arrays with 1 = solid, so that
 * solid(x) = solid_outer(x >> (n-l)) * solid_inner(x mod K) per axis.  The
 * obstacle mask m_O is the tensor product of the two parts: each part is
 * decomposed on its own grid by successive truncated SVDs at tol_mask (rank
 * cap chi_mask_max when > 0) and the two MPS are chained, the l coarse
 * sites first, with bond 1 between them, so that the mask's largest bond is
 * the larger of the parts' (no N^3 decomposition of the mask is made).  The
 * dense composite solid is formed on the device for the initial
 * populations, N_fluid and the face masks.  rho, u, f and hip_stream are
 * as in mps_lbm_init_from_field.  The mask decomposition error reported in
 * the observables is that of the chained mask against the composite.
 * Errors: as mps_lbm_init_from_field; EINVAL also for NULL parts or
 * l outside [2, n - 2].
 */
int mps_lbm_init_tensor_mask(const mps_lbm_config* cfg, const double* rho, const double* u,
                             const double* f, const uint8_t* solid_outer, int l,
                             const uint8_t* solid_inner, void* hip_stream, mps_lbm_t** out);

/*
 * Numerical failures.  The factorisation kernels flag non-finite values and
 * Jacobi sweeps that stop at their iteration limit (Section 2.1 truncations)
 * in device memory.  Every call that synchronises with the device to read
 * the state (mps_lbm_to_dense*, mps_lbm_get_mps) first checks these flags:
 * a non-finite value makes it, and every later such call and mps_lbm_step,
 * return MPS_LBM_ENUMERIC without writing outputs or stepping (the handle
 * remains destroyable and mps_lbm_observables still reports the counts); new
 * sweep-limit hits are returned once as MPS_LBM_ENUMERIC, after which the
 * state can be read again.
 */

/*
 * Advance nsteps lattice Boltzmann steps (Section 3.2): moments,
 * 1/rho approximation, equilibrium by variational Hadamard products
 * (Section 2.3), BGK relaxation, streaming by shift MPOs (Section 2.5),
 * open-face boundary terms and masked bounce-back, every sum followed by
 * rounding to chi_max.  Runs asynchronously on the handle's stream with
 * no host synchronisation.  Errors: EINVAL (NULL handle, nsteps < 0), EHIP.
 */
int mps_lbm_step(mps_lbm_t* h, int nsteps);

/*
 * Time-dependent inflow (Section 4.1: the aneurysm's pulse, the pin-fin
 * ramp).  From the next step on, velocity face `face` (0..5 as in
 * face_bc) of domain `domain` uses u_b(t) = face_val[face] * phi(t) with
 *   phi(t) = c0 + c1 (1 - exp(-c2 t)) + c3 t^c4 exp(-c5 t),
 * coef = {c0, ..., c5}, and t = k dt for the step that starts after k
 * steps since init (k counted on the device, so captured graphs follow the
 * profile too).  Examples: the ramp u_0 (1 - e^{-1.5 t}) is {0, 1, 1.5, 0,
 * 0, 0} with dt = 1 / (steps per flow-through time L / u_0); the pulse
 * 0.1 + 18 t^1.5 e^{-10 t} is {0.1, 0, 0, 18, 1.5, 10} with dt in seconds per
 * step and face_val the lattice velocity of 1 m/s.  coef = NULL restores
 * the constant face (phi = 1).  Synchronises the handle's stream.
 * Errors: EINVAL (NULL handle, domain or face out of range, the face is not
 * a velocity face, a non-finite coefficient, c4 < 0, dt < 0), EHIP.
 */
int mps_lbm_set_face_profile(mps_lbm_t* h, int domain, int face, const double* coef,
                             double dt);

/*
 * Region of interest of the pressure metric (Section 4.2):
 *   Delta p / p_0 = (1 / (p_0 |D|)) sum_{x in D} (p_x - p_0),
 * p = c_s^2 rho, p_0 = c_s^2 rho_ref (the density prescribed at the
 * outflow), D = the fluid cells of the box lo[a] <= x_a < hi[a].  The
 * indicator of D is decomposed into an MPS m_D at tol_mask without a rank
 * cap (like the obstacle mask; the solid cells are read from it), |D| is
 * counted exactly, and mps_lbm_observables then reports dp_p0 =
 * sum_i <m_D, f_i> / (rho_ref |D|) - 1, an exact contraction of the state.
 * A later call replaces the region.  Synchronises the handle's stream.
 * Errors: EINVAL (NULL handle or box, domain out of range, empty box or box
 * outside the grid, no fluid cell in it, rho_ref <= 0), ENOMEM, EHIP.
 */
int mps_lbm_set_region(mps_lbm_t* h, int domain, const int* lo, const int* hi, double rho_ref);

/* Testing hook for the numerical-failure path: adds nonfinite to the
   device's non-finite count and sweep_limit to its sweep-limit count, as a
   kernel that met them would (enqueued on the handle's stream; no kernel
   computes on invalid data).  Errors: EINVAL (NULL handle, negative
   counts), EHIP. */
int mps_lbm_debug_raise_flags(mps_lbm_t* h, int nonfinite, int sweep_limit);

/*
 * Contract the state to a dense host array (synchronises the stream).
 * what = MPS_LBM_POPS | RHO | J | VEL; out_len is the number of doubles
 * available at out.  Errors: EINVAL (bad what, out_len too small), EHIP.
 */
int mps_lbm_to_dense(mps_lbm_t* h, int what, double* out, size_t out_len);

/*
 * Total kinetic energy of domain `domain` (Section 4.2, with the density
 * normalised so that the total mass is 1 and V_c = (L/N)^3):
 *   e_kin = (1 / (2 N^3)) sum_x |u_x|^2,  u = j / rho (0 where rho = 0),
 * in lattice units (multiply by the squared velocity conversion factor for
 * physical units), from a dense contraction of the state on the device
 * (Q N^3 elements of the working type, twice, for the call).  The paper's
 * dissipation -dE_kin/dt is the caller's second-order finite difference of
 * successive values.  Synchronises the stream.
 * Errors: EINVAL (NULL handle or e_kin, domain out of range), ENUMERIC,
 * ENOMEM, EHIP.
 */
int mps_lbm_kinetic_energy(mps_lbm_t* h, int domain, double* e_kin);

/* Scalar observables (synchronises the stream). */
int mps_lbm_observables(mps_lbm_t* h, mps_lbm_obs* out);

/*
 * Batched domains: count independent simulations (each the problem of
 * Section 3.2 with its own configuration, geometry and initial fields) held
 * by one handle and advanced together by mps_lbm_step.  Domains that share
 * n, the velocity set, chi_max, chi_mask_max, precision, tol, sweeps, the
 * inverse-density mode and the rank-predictor settings form a group: every
 * operation of the step is issued once for the MPS of all domains of the
 * group.  Domains of different sizes or policies form several groups, which
 * run one after another on the handle's stream (and are recorded into one
 * graph by mps_lbm_capture_step).  rho[d], u[d] and solid[d] are as in
 * mps_lbm_init_from_field (solid, or an entry of it, may be NULL for no
 * obstacles).  The handle's plain entry points address domain 0; the
 * per-domain forms below address any.  The rank-predictor entry points and
 * mps_lbm_debug_raise_flags address the group of domain 0;
 * mps_lbm_kernel_stats and mps_lbm_autotune cover every group.
 * Errors: EINVAL (count < 1, an invalid configuration, NULL fields),
 * ENOMEM, EHIP.
 */
int mps_lbm_init_batch(const mps_lbm_config* cfgs, int count, const double* const* rho,
                       const double* const* u, const uint8_t* const* solid, void* hip_stream,
                       mps_lbm_t** out);

/*
 * Record the step as a HIP graph: one eager step is taken (it brings the
 * handle's MPS pool to its peak size and counts as a step), then the next
 * step is captured together with copies that return the new populations to
 * the slots the step reads, and every later mps_lbm_step replays the graph
 * (one launch per step, identical arithmetic).  The handle's stream must not
 * be the default stream.  Kernel timing is not recorded inside the graph.
 * Errors: EINVAL (NULL handle, default stream), EHIP.
 */
int mps_lbm_capture_step(mps_lbm_t* h);

/* Number of domains of the handle (1 after mps_lbm_init_from_field), or
   EINVAL for a NULL handle. */
int mps_lbm_domains(const mps_lbm_t* h);

/* mps_lbm_to_dense and mps_lbm_observables for domain 0 <= domain <
   mps_lbm_domains(h); the roundings and products of the observables count
   all domains of the handle.  Errors: as the plain forms, and EINVAL for a
   domain out of range. */
int mps_lbm_to_dense_domain(mps_lbm_t* h, int domain, int what, double* out, size_t out_len);
int mps_lbm_observables_domain(mps_lbm_t* h, int domain, mps_lbm_obs* out);

/* mps_lbm_get_mps: index of the obstacle-mask MPS (0..Q-1 are populations) */
#define MPS_LBM_MPS_MASK 19

/*
 * Copy one MPS of the state to the host (synchronises the stream).
 * which = 0..Q-1 selects population i (order above), MPS_LBM_MPS_MASK
 * the obstacle mask m_O (Section 3.2.1, objects equation).  bonds receives
 * n + 1 ints: r_0 = 1, r_1, ..., r_n = 1.  When out is non-NULL it receives
 * the cores one after another, core k (k = 0..n-1) as a C-order FP64 array
 * [r_k][8][r_{k+1}] (MPS equation, Section 2.1), its middle index being
 * sigma = 4 x_k + 2 y_k + z_k with x_k the k-th most significant bit of x
 * (scale ordering, Section 2.4); out_len is the number of doubles at out
 * and must be at least sum_k r_k 8 r_{k+1}.  Pass out = NULL to read the
 * bonds only.  Errors: EINVAL (NULL handle or bonds, which out of range, no
 * obstacle mask, out_len too small), EHIP.
 */
int mps_lbm_get_mps(mps_lbm_t* h, int which, double* out, size_t out_len, int* bonds);

/* Kernel classes that can be timed for roofline reporting. */
#define MPS_LBM_K_NONE 0
#define MPS_LBM_K_JACOBI 1      /* one-sided Jacobi SVD of the bond matrices   */
#define MPS_LBM_K_HOUSEHOLDER 2 /* Householder QR of core unfoldings          */
#define MPS_LBM_K_PRODGEMM 3    /* contraction GEMMs of the variational product */
#define MPS_LBM_K_CHOLESKY 4    /* pivoted Cholesky of the FP32-policy Gram matrices */

typedef struct {
  long long launches; /* launches of the class since timing was enabled       */
  double total_ms;    /* sum of their durations (HIP events around each launch) */
  double flops;       /* algorithmic floating-point operations they performed,
                         counted on the device from the actual shapes          */
} mps_lbm_kstats;

/*
 * Time every launch of one kernel class with HIP events recorded on the
 * handle's stream around that launch, and count its algorithmic work.
 * kind = MPS_LBM_K_* (MPS_LBM_K_NONE switches timing off); enabling resets
 * the statistics.  Timing adds two event records per launch of the class
 * and nothing to other kernels.  Errors: EINVAL (NULL handle, bad kind).
 */
int mps_lbm_kernel_timing(mps_lbm_t* h, int kind);

/* Statistics of the timed class since it was enabled (synchronises the
   stream).  Errors: EINVAL (NULL handle or out), EHIP. */
int mps_lbm_kernel_stats(mps_lbm_t* h, mps_lbm_kstats* out);

/* Autotune the contractions: the split of K of the long ones (K capacity
   above 512) and, for the product contractions on BF16 matrix cores, the
   tile edge (64 or 128).  Every contraction class met in the steps taken
   so far (arithmetic, capacities M, N, K, problem and batch counts) is
   timed on scratch operands of its capacity shape for 1, 2, 4 and 8 shares
   of K (and both tile edges where they apply), and later steps use the
   fastest (untuned classes use one share per 256 columns of K and tiles of
   64).  The tile edge keeps each output's summation order; the share
   count changes it.  Allocates and frees scratch memory; synchronises the
   stream.
   *classes_tuned (may be NULL) receives the number of classes tuned.
   Errors: EINVAL (NULL handle, no step taken), EUNSUPPORTED (after graph
   capture), ENOMEM, EHIP. */
int mps_lbm_autotune(mps_lbm_t* h, int* classes_tuned);

/* ---- learned rank predictor (rank_predictor = 2) --------------------------
   The rounding's truncations (FP32/BF16 policies) record, per truncation,
   the spectrum around the cut: sigma_{r-16} .. sigma_{r+15} as
   log10(sigma / sigma_1) / 8 (absent: -2) and the step index / 1000; each
   later step adds a training sample (that record, the rank change / 16).
   A multilayer perceptron 33 -> 128 -> 128 -> 128 -> 1 (ReLU, FP32) trained
   on these samples then predicts the rank that sizes the randomised sketch
   of the truncation (rank_predictor = 1 uses the previous rank); the
   acceptance test and the full-path fallback are the same. */
typedef struct {
  long long samples;      /* training samples recorded (total)             */
  int trained;            /* 1 once mps_lbm_train_rank_predictor ran        */
  double first_loss;      /* mean squared error of the first epoch          */
  double last_loss;       /* of the last epoch                              */
  long long predictions;  /* predictions scored since the last training     */
  double mlp_abs_err;     /* mean |predicted rank - chosen rank|, network   */
  double prev_abs_err;    /* the same for the previous rank as prediction   */
} mps_lbm_predictor_info;

/* Train the network on the samples recorded so far: `epochs` passes of
   Adam (beta 0.9, 0.999) with learning rate lr over batches of up to 1024,
   on the handle's stream with the library's kernels; *loss_out (may be
   NULL) receives the last epoch's mean squared error.  Synchronises the
   stream.  Errors: EINVAL (NULL handle, epochs < 1, lr outside (0, 1), fewer
   than 16 samples), EUNSUPPORTED (predictor not in mode 2, or after graph
   capture). */
int mps_lbm_train_rank_predictor(mps_lbm_t* h, int epochs, double lr, double* loss_out);

/* Trained weights of the predictor network (37505 FP32 values in the
   layout of mps_lbm_mlp_gradient's params): load copies them into the
   handle and marks the network trained, so that a model trained once can
   size the sketches of later runs; get copies the handle's weights out.
   Both synchronise the stream.  Errors: EINVAL (NULL handle or weights,
   n != 37505 for load, n < 37505 for get), EUNSUPPORTED (predictor not in
   mode 2; load after graph capture), EHIP. */
int mps_lbm_load_rank_model(mps_lbm_t* h, const float* weights, size_t n);
int mps_lbm_get_rank_model(mps_lbm_t* h, float* weights, size_t n);

/* Predictor statistics (all zero when the predictor is not in mode 2).
   Errors: EINVAL (NULL handle or out), EHIP. */
int mps_lbm_rank_predictor_info(mps_lbm_t* h, mps_lbm_predictor_info* out);

/* One forward and backward pass of the predictor network on the current
   device, for checking its gradients: params (host, 37505 floats in the
   layout W1 (33 x 128, row i = input i), b1, W2 (128 x 128), b2, W3, b3,
   W4 (128 x 1), b4), x (host, batch x 33), t (host, batch targets);
   *loss receives mean (f(x) - t)^2 and grad (host, 37505 floats) its
   gradient.  Allocates and frees its own device buffers.  Errors: EINVAL
   (NULL pointer, batch outside [1, 1024]), ENOMEM, EHIP. */
int mps_lbm_mlp_gradient(const float* params, const float* x, const float* t, int batch,
                         float* loss, float* grad);

/*
 * mps_lbm_mlp_gradient without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  params (37505 floats), x (batch x 33),
 * t (batch), loss (1 float) and grad (37505 floats) are DEVICE pointers
 * owned by the caller; the activations live in a fixed device array of the
 * library (4.7 MB per GPU, held until the process ends), so batch is at
 * most 1024.  Enqueued on hip_stream (NULL = default stream) without
 * synchronising; the results are those of mps_lbm_mlp_gradient.  Calls
 * that overlap on one GPU (any streams) share that array and race.
 * Errors: EINVAL (NULL pointer, batch outside [1, 1024]), EHIP.
 */
int mps_lbm_mlp_gradient_device(const float* params, const float* x, const float* t, int batch,
                                float* loss, float* grad, void* hip_stream);

/* Release every device buffer of the handle; NULL is ignored. */
void mps_lbm_destroy(mps_lbm_t* h);

/* Message of the last error on this thread ("" if none). */
const char* mps_lbm_last_error(void);

/* Library version string. */
const char* mps_lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPS_LBM_H */
