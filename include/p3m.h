/*
 * p3m.h -- C ABI of libp3m.so, the MI355X (gfx950) P3M periodic-gravity force.
 *
 * The library computes the gravitational force of the P3M method of the
 * CONCEPT N-body code (CONCEPT User's Guide, arXiv:1510.07621): a
 * particle-mesh long-range part and a short-range pair sum, split at a scale
 * r_s and cut off at r_c, in a periodic cubic comoving box, for one particle
 * group with Plummer softening; plus the kick and drift particle updates.
 * Guide references: Ch. 1 (PP, PM and P3M gravity); Ch. 5 "Parameters"
 * (boxsize, PM_gridsize, PM_scale, P3M_cutoff, softeningfactors,
 * kick_algorithms); Ch. 6 (particle data: one mass per group, comoving
 * positions posx/posy/posz and momenta momx/momy/momz in
 * length*mass/time); Ch. 8 (drift and kick tests).
 *
 * Mathematics (the guide names the method but gives no formulas; these are
 * the definitions this library implements):
 *   h = box / grid_n, r_s = rs_cells * h, r_c = cutoff_rs * r_s.
 *   PP:  a_i = -G sum_{j != i, r < r_c} m_j r_ij f(r) / (r^2 + eps^2)^(3/2),
 *        r_ij the minimum-image separation, r = |r_ij|,
 *        f(r) = erfc(r/(2 r_s)) + r/(r_s sqrt(pi)) exp(-r^2/(4 r_s^2)).
 *   PM:  cloud-in-cell deposit to nodes c*h; FFT; multiply by
 *        G(k) = -4 pi G exp(-k^2 r_s^2) / (k^2 W(k)^deconv_power), G(0) = 0,
 *        W(k) = prod_d sinc^2(pi n_d / grid_n); inverse FFT; central
 *        difference gradient (fd_order 4 or 2); CIC interpolation; a = -grad.
 *   F_i = m_i (a_PP + a_PM).
 *
 * Conventions for every call:
 *   - Device arrays are plain HIP device pointers on the current device.
 *     Vector arrays are structure-of-arrays: x[0..n), then y, then z.
 *   - pos components must lie in [0, box). Positions outside are clamped to
 *     the nearest cell for binning (memory-safe) but give undefined forces.
 *   - Work is enqueued on a HIP stream and the call returns without
 *     synchronising. Asynchronous device errors surface at the caller's
 *     next synchronisation. Outputs are overwritten, never accumulated.
 *   - Argument errors are detected before any work is enqueued; nothing is
 *     written then. The library never aborts and never throws across the ABI.
 *   - The caller owns all particle arrays; a plan owns its workspace,
 *     allocated once by p3m_plan_create. Force calls allocate nothing.
 *   - A plan is not thread-safe: use one plan from one host thread and one
 *     stream at a time.
 */
#ifndef P3M_H
#define P3M_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define P3M_OK       0
#define P3M_EINVAL  -1  /* null pointer, n < 0, n > n_max, bad parameter     */
#define P3M_ENOMEM  -2  /* device allocation failed in p3m_plan_create        */
#define P3M_EHIP    -3  /* a HIP runtime call or kernel launch failed          */
#define P3M_ERANGE  -4  /* r_c >= box/2 (minimum image insufficient)           */
#define P3M_ESIZE   -5  /* sizes beyond the fixed workspace of pp_force_noalloc */

/* Arithmetic of the force path (particle storage, kick and drift stay FP64). */
#define P3M_FP64     0  /* pair loop, FFT and grids in double precision        */
#define P3M_FP32     1  /* pair loop, FFT and grids in single precision, pair
                           separations from cell-relative FP32 offsets        */

typedef struct p3m_params {
  int32_t grid_n;       /* PM_gridsize: power of two, 16..512                        */
  int32_t precision;    /* P3M_FP64 or P3M_FP32                                      */
  int32_t fd_order;     /* 4 (default) or 2: central-difference gradient order       */
  int32_t deconv_power; /* 2 (default) or 0: powers of the CIC window divided out    */
  double  box;          /* boxsize L > 0 (comoving side of the periodic cube)        */
  double  rs_cells;     /* PM_scale: r_s in PM cells, > 0 (1.25 typical)             */
  double  cutoff_rs;    /* P3M_cutoff: r_c in units of r_s, > 0 (4.5 typical)        */
  double  softening;    /* Plummer radius eps as a length, >= 0                      */
  double  G;            /* gravitational constant                                    */
  int32_t adjoint;      /* 1: also allocate the workspace of the *_force_vjp calls   */
  int32_t ewald_gridsize; /* ewald_gridsize: 0, or even in 8..512 to tabulate the
                             Ewald correction of pp_ewald_force                    */
  int32_t pair_partials;  /* short-range sum: 0 evaluates every pair from both
                             sides; > 0 evaluates a pair of particles in two
                             dense groups (more than 32 particles each) once
                             (the force on one is minus that on the other) and
                             keeps the reactions as partials, of which the plan
                             holds pair_partials per particle (80 suits strongly
                             clustered sets); a call that needs more falls back
                             to both sides. Pays on clustered sets (256^3
                             Plummer mix: -11 %), not on smooth ones            */
} p3m_params;

/* Opaque plan: derived geometry, device workspace, and optional stage timers. */
typedef struct p3m_plan p3m_plan;

/* Fill *out with the documented defaults for a grid of grid_n^3 cells in a
 * box of side box: FP32, fd_order 4, deconv_power 2, rs_cells 1.25,
 * cutoff_rs 4.5, softening 0, G 1, adjoint 0, ewald_gridsize 0,
 * pair_partials 0. Returns
 * P3M_EINVAL for a null out. */
int p3m_params_default(p3m_params* out, int32_t grid_n, double box);

/* Create a plan for up to n_max particles whose work runs on hip_stream
 * (a hipStream_t; NULL = the null stream). Validates the parameters
 * (EINVAL for a non-power-of-two or out-of-range grid, box <= 0,
 * rs_cells <= 0, cutoff_rs <= 0, softening < 0, adjoint not 0 or 1,
 * ewald_gridsize not 0 or even in 8..512,
 * n_max < 0 or n_max >= 2^31; ERANGE when r_c >= box/2), then allocates the
 * workspace (with adjoint = 1 also that of the VJP calls: one more real grid,
 * three cotangent grids and a sorted cotangent array; with pair_partials > 0
 * the reaction partials, pair_partials n_max + 65536 of 3 reals each (at 80:
 * 0.96 KB (FP32) or 1.9 KB (FP64) per particle), plus per-group offsets; if
 * that allocation fails the plan evaluates every pair from both sides)
 * (ENOMEM on failure; nothing is leaked). *out is set only on success.
 * CONCEPT User's Guide Ch. 5 (PM_gridsize, PM_scale, P3M_cutoff,
 * softeningfactors, boxsize) for the parameters. */
int p3m_plan_create(const p3m_params* params, int64_t n_max, void* hip_stream,
                    p3m_plan** out);

/* Release the plan and its workspace (the counterpart of p3m_plan_create).
 * Synchronises the plan's stream first. A null plan is a no-op returning
 * P3M_OK. */
int p3m_plan_destroy(p3m_plan* plan);

/* Change the stream later calls on this plan enqueue on. */
int p3m_plan_set_stream(p3m_plan* plan, void* hip_stream);

/* Full P3M force (PP + PM) on n particles. After binning on the plan's
 * stream, the mesh part (deposit, Poisson solve) runs on a second stream of
 * the plan (default priority) beside the pair sum, which writes its sorted
 * acceleration; the plan's stream then waits for it and the interpolation
 * adds the mesh force and writes the force. With the one-sided pair sum
 * (pair_partials > 0) the interpolation runs on the second stream too and
 * the gather of the reactions, after the pair sum, adds it and writes the
 * force. To the caller all of it is ordered on the plan's stream, as one
 * call. Stage timers of deposit, FFT and (one-sided) interpolation are
 * recorded on the second stream, so they include the time those kernels
 * wait for compute units held by the pair sum.
 *   pos         device, double [3][n], components in [0, box)
 *   mass        device, double [n], or NULL to give every particle mass_scalar
 *               (one mass per particle group, guide Ch. 6)
 *   force       device output [3][n]: double if force_fp32 == 0, float otherwise;
 *               must not overlap pos or mass
 * n == 0 is a successful no-op. */
int p3m_force(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
              double mass_scalar, void* force, int32_t force_fp32);

/* The force of p3m_force written in the cell order of this call's binning
 * rather than the input order, together with that order: force[.][s] is the
 * force on input particle order_out[s]. The order sorts the particles by PM
 * cell (cell index (cx ng + cy) ng + cz); inside a cell it can differ from
 * call to call. A caller that keeps its particles in this order (see
 * p3m_kick_reorder) hands the next call input that is nearly sorted already
 * (particles move little between steps), so the binning and the force's
 * stores touch memory in order instead of scattering. Same computation and
 * arguments as p3m_force; order_out: device int32 [n], overwritten, not
 * overlapping pos, mass or force (EINVAL). Guide Ch. 1 and Ch. 5 as for
 * p3m_force. */
int p3m_force_cell_order(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
                         double mass_scalar, void* force, int32_t force_fp32,
                         int32_t* order_out);

/* Long-range (PM) part only: F_i = m_i a_PM(x_i). Same arguments. */
int pm_force(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
             double mass_scalar, void* force, int32_t force_fp32);

/* Short-range (PP) part only: F_i = m_i a_PP(x_i). Same arguments. */
int pp_force(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
             double mass_scalar, void* force, int32_t force_fp32);

/* Adjoint of the force (vector-Jacobian product), for gradients through
 * trajectories. The guide gives no derivatives; these are the exact
 * transposes of the definitions above (away from the measure-zero sets where
 * a pair crosses r_c or a particle crosses a node plane, where the force is
 * not differentiable). For a cotangent lam on the force F:
 *   pos_bar_k = sum_i lam_i . dF_i/dx_k.
 * PP:  pos_bar_k = -G m_k sum_{j: 0 < r < r_c} m_j J(r_kj) (lam_k - lam_j),
 *      J = g I + (g'(r)/r) r r^T, g = f / (r^2 + eps^2)^(3/2).
 * PM:  pos_bar_k = m_k sum_c grad W(x_k - c) [h^-3 psi(c) - lam_k . E(c)],
 *      E = D phi the node gradient of the forward potential,
 *      psi = P (sum_d D_d Lam_d), Lam_d(c) = sum_i m_i lam_{i,d} W(x_i - c),
 *      P the Green's function operator of the forward solve.
 *   pos, mass, mass_scalar  as for p3m_force
 *   force_bar   device, double [3][n] (input order)
 *   pos_bar     device output, double [3][n], overwritten; must not overlap
 *               pos, mass or force_bar
 * The plan must have been created with params.adjoint = 1 (else EINVAL).
 * The arithmetic is the plan's precision. In J, g'(r) comes from the
 * derivative of the split-factor pieces the forward pair sum evaluates (the
 * exact derivative of that piecewise f; within 1e-5 (FP32) / 1e-11 (FP64)
 * of the closed form for r_c <= 4.5 r_s), except for tables over r (wide
 * softening) and the FP64 pieces next to r = 0, which use the closed form.
 * As in p3m_force, the mesh part runs on the plan's second stream beside
 * the pair part, joined before the call's last kernel on the plan's
 * stream. n == 0 is a successful no-op. */
int p3m_force_vjp(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
                  double mass_scalar, const double* force_bar, double* pos_bar);

/* Adjoint of the long-range (PM) part only. Same arguments. */
int pm_force_vjp(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
                 double mass_scalar, const double* force_bar, double* pos_bar);

/* Adjoint of the short-range (PP) part only. Same arguments. */
int pp_force_vjp(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
                 double mass_scalar, const double* force_bar, double* pos_bar);

/* Power spectrum of the particle density on the plan's PM grid (guide Ch. 5:
 * PM_gridsize is also the power-spectrum grid, R_tophat the radius of the
 * top-hat for sigma; Ch. 8 powerspec test). The guide gives no estimator;
 * this one: the CIC deposit rho of the force path, delta = rho / rho_bar - 1,
 * P(k) = box^3 |FFT(delta)_k|^2 / grid_n^6 for k != 0, divided by W(k)^2 (the
 * CIC window, W = prod_d sinc^2(pi n_d / grid_n)) unless the plan's
 * deconv_power is 0. Shells of unit width in |n| (k = 2 pi n / box): shell b
 * holds the modes with b + 1/2 <= |n| < b + 3/2, b = 0 .. nbins - 1, counted
 * over the full k-space. sigma^2(R) = box^-3 sum_{k != 0} P(k) W_TH(k R)^2
 * over all grid modes, W_TH(x) = 3 (sin x - x cos x) / x^3 (R = 0: the grid
 * variance of delta).
 *   pos, mass, mass_scalar  as for p3m_force (n >= 1, positive total mass)
 *   nbins       1 .. 512
 *   r_tophat    R >= 0, a length
 *   k_out, power_out, modes_out   device double [nbins]: the shell's mean |k|,
 *               mean P and number of modes (0, 0, 0 for an empty shell)
 *   sigma_out   device double [1] or NULL
 * The FFT runs in the plan's precision; the sums in double. EINVAL for
 * n < 1, a bad nbins or r_tophat, null outputs or a non-positive scalar mass. */
int p3m_power_spectrum(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
                       double mass_scalar, int32_t nbins, double r_tophat, double* k_out,
                       double* power_out, double* modes_out, double* sigma_out);

/* PP gravity with a tabulated Ewald correction (guide Ch. 5: use_Ewald,
 * ewald_gridsize; Ch. 8 kick_PP_with_Ewald test), all pairs, FP64, for
 * small-N validation (cost O(n^2)):
 *   F_i = -G m_i sum_{j != i} m_j [ r / (r^2 + eps^2)^(3/2) + c(r) ],
 * r the minimum-image separation, c(r) = e(r) - r / |r|^3 the correction of
 * the periodic field e of a unit mass with its images in a neutralising
 * background (Ewald sum, as a multiple of -G), tabulated by the plan on the
 * ewald_gridsize^3 node grid (spacing box / ewald_gridsize; c is odd in each
 * coordinate, so the octant [0, box/2]^3 is stored) and interpolated
 * trilinearly. Softening acts on the minimum-image term only. Arguments as
 * for p3m_force; the plan must have ewald_gridsize > 0 (else EINVAL). The
 * call bins the particles into the plan's cells first, as the force calls
 * do, and sums over the i's in cell order. */
int pp_ewald_force(p3m_plan* plan, int64_t n, const double* pos, const double* mass,
                   double mass_scalar, void* force, int32_t force_fp32);

/* The tabulated correction c(r) of pp_ewald_force at npts separations
 * r (device double [3][npts], reduced to the minimum image), written to
 * c_out (device double [3][npts], not overlapping r). For testing the table;
 * EINVAL without a table. */
int p3m_ewald_correction(p3m_plan* plan, int64_t npts, const double* r, double* c_out);

/* Count the ordered pairs (i, j != i) with minimum-image separation in
 * (0, r_c), the pairs the short-range sum evaluates (a diagnostic for
 * interaction rates). count_out: device int64 [1], overwritten. Separations
 * are tested in the plan's precision. */
int p3m_pair_count(p3m_plan* plan, int64_t n, const double* pos,
                   int64_t* count_out);

/* Kick (guide Ch. 5 kick_algorithms, Ch. 8 kick tests): p <- p + c_kick * F,
 * each product and sum one IEEE double operation (no fused multiply-add).
 * mom: device double [3][n] in place; force: device [3][n], float if
 * force_fp32 != 0 else double. */
int p3m_kick(int64_t n, double* mom, const void* force, int32_t force_fp32,
             double c_kick, void* hip_stream);

/* Kick and reorder (guide Ch. 5 kick_algorithms): the second half-kick of
 * a kick-drift-kick step for a caller that keeps its particles in the cell
 * order of the last force call. With i = order[s]:
 *   mom_out[.][s] = mom[.][i] + c_kick * force[.][s]   (force in cell order,
 *                                                      as p3m_force_cell_order
 *                                                      writes it)
 *   pos_out[.][s] = pos[.][i], ids_out[s] = ids[i], mass_out[s] = mass[i]
 * Each sum and product is one IEEE double operation, as in p3m_kick, so the
 * momenta equal p3m_kick's followed by the permutation bit for bit.
 *   order       device int32 [n], a permutation of 0 .. n-1 (entries out of
 *               range are clamped into it: wrong values, no fault)
 *   pos, mom    device double [3][n]; force device [3][n], float if
 *               force_fp32 != 0 else double
 *   ids, mass   device int64 [n] / double [n] carried along, or NULL (then
 *               ids_out / mass_out NULL too, else EINVAL)
 *   outputs     device, the shapes of the inputs; no output may overlap an
 *               input or another output (EINVAL) */
int p3m_kick_reorder(int64_t n, const int32_t* order, const double* pos, const double* mom,
                     const void* force, int32_t force_fp32, const int64_t* ids,
                     const double* mass, double c_kick, double* pos_out, double* mom_out,
                     int64_t* ids_out, double* mass_out, void* hip_stream);

/* Drift (guide Ch. 8 drift test: comoving motion, crossing box faces):
 * x <- wrap(x + c_drift * (p / m)), wrap(y) = y - box*floor(y/box) and a
 * result equal to box becomes 0; one IEEE double operation per step, no
 * fused multiply-add. pos: device double [3][n] in place; mom: device double
 * [3][n]; mass: device double [n] or NULL for mass_scalar. box > 0. */
int p3m_drift(int64_t n, double* pos, const double* mom, const double* mass,
              double mass_scalar, double c_drift, double box, void* hip_stream);

/* Kick then drift in one pass (the first half of a kick-drift-kick step):
 * p <- p + c_kick * F, then x <- wrap(x + c_drift * (p / m)) with the new p;
 * the same operations in the same order as p3m_kick followed by p3m_drift,
 * so the results are bitwise the same, with the momenta read and written
 * once. Arguments as for those two calls; pos and mom must not overlap. */
int p3m_kick_drift(int64_t n, double* pos, double* mom, const void* force, int32_t force_fp32,
                   const double* mass, double mass_scalar, double c_kick, double c_drift,
                   double box, void* hip_stream);

/* Transpose of the drift: x1 = wrap(x + c_drift p / m) has slope 1 in x and
 * c_drift / m in p, so mom_bar <- mom_bar + (c_drift / m) * pos_bar (the
 * quotient first, then one product and one sum per component, no fused
 * multiply-add). mom_bar: device double [3][n] in place; pos_bar: device
 * double [3][n], not overlapping mom_bar; mass: device double [n] or NULL for
 * mass_scalar. (The kick's transpose needs no call: its force cotangent is
 * c_kick * p_bar, passed to p3m_force_vjp by scaling its result.) */
int p3m_drift_vjp(int64_t n, double* mom_bar, const double* pos_bar, const double* mass,
                  double mass_scalar, double c_drift, void* hip_stream);

/* Stage timers. p3m_set_timing(plan, capacity) with capacity > 0 records HIP
 * events around the stages of the next `capacity` force calls, on the plan's
 * stream and without synchronising (pm_force and pp_force record the stages
 * they run); capacity 0 stops recording. Either call first synchronises the
 * plan's stream and drops any earlier record. capacity <= 2^20, else EINVAL.
 * p3m_stage_times synchronises the plan's stream, writes to ms_out[s], for
 * s < n_stages, the total duration in milliseconds of stage s over the
 * recorded calls (0 for a stage that never ran), and returns the number of
 * recorded calls (>= 0) or a negative status. Stage indices: */
#define P3M_STAGE_BIN      0  /* cell keys, counts, scan, scatter, work list
                                 (+ reaction offsets of the one-sided sum)     */
#define P3M_STAGE_DEPOSIT  1  /* CIC mass deposit                              */
#define P3M_STAGE_FFT      2  /* forward FFT, Green's function, inverse FFT   */
#define P3M_STAGE_INTERP   3  /* finite-difference gradient + interpolation   */
#define P3M_STAGE_PP       4  /* short-range pair loop (+ combine, unpermute) */
#define P3M_STAGE_REACT    5  /* one-sided sum: gather of the reactions       */
#define P3M_NUM_STAGES     6
int p3m_set_timing(p3m_plan* plan, int32_t capacity);
int p3m_stage_times(p3m_plan* plan, double* ms_out, int32_t n_stages);

/* Short-range (PP) force without a plan, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc). The same force as pp_force on a plan made from
 * `params` for n particles, computed by the same kernels, with every pair
 * evaluated from both sides. The call allocates nothing: its workspace is
 * one fixed device array of 12 MiB per GPU, held from the library's first
 * such call on that GPU until the process ends; the stencil rows and
 * split-factor tables are computed on the host and copied into it on
 * hip_stream (from host memory the call owns) before the kernels run.
 *   params      as for p3m_plan_create (all of it validated the same way;
 *               fd_order, deconv_power, adjoint and ewald_gridsize unused)
 *   n           0 <= n <= P3M_NOALLOC_MAX_N
 *   pos, mass, mass_scalar, force, force_fp32   as for pp_force
 *   hip_stream  the stream the work runs on (NULL = the null stream)
 * Limits: n <= P3M_NOALLOC_MAX_N, params->grid_n <= P3M_NOALLOC_MAX_GRID and
 * at most 4096 stencil rows (r_c up to about 30 cells); beyond them
 * P3M_ESIZE before anything is enqueued. Every call on a GPU shares that
 * GPU's array, which keeps the last call's contents (the call clears what
 * must start at zero): calls that overlap on one GPU (other streams, other
 * host threads between enqueue and completion) race. Host threads are
 * serialised while they enqueue. n == 0 is a successful no-op. */
#define P3M_NOALLOC_MAX_N    65536
#define P3M_NOALLOC_MAX_GRID 64
int pp_force_noalloc(const p3m_params* params, int64_t n, const double* pos,
                     const double* mass, double mass_scalar, void* force,
                     int32_t force_fp32, void* hip_stream);

/* Static text for a status code ("unknown status" for others). */
const char* p3m_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* P3M_H */
