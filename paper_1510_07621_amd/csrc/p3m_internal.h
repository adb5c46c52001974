// Internal declarations shared by the translation units of libp3m.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "p3m.h"
#include "p3m_host.h"

namespace p3m {

// Vector types for the two arithmetic precisions of the force path.
template <typename T> struct Vec;
template <> struct Vec<float> {
  using v2 = float2;
  using v4 = float4;
};
template <> struct Vec<double> {
  using v2 = double2;
  using v4 = double4;
};

constexpr int kPairCap = 128;     // j-particles staged in LDS per pass of the pair loop
constexpr int kBrick = 8;         // cells per brick edge (deposit, interpolation)
constexpr int kChunk = 64;        // i-particles per pair-loop work item (one wavefront)
constexpr int kXcds = 8;          // accelerator complex dies of an MI355X (one L2 each)
constexpr int kSplitBins = 64;    // pieces of the split-factor tables
constexpr int kSplitCoef64 = 7;   // coefficients per piece of the FP64 table (degree 6)
constexpr double kGroupTarget = 64.0;  // mean particles per i-group the plan aims for
constexpr int kMaxPowerBins = 512;     // shells of the power spectrum
// Row stride of the half-complex spectrum along kz: the ng/2 + 1 values of a
// row padded to a multiple of 16, so that every row, and every 8- or
// 16-column chunk of one, starts on a 64- (FP32) or 128-byte (FP64) boundary.
// (With the odd ng/2 + 1 as stride each chunk of a row read by the y and x
// passes straddled two cache lines.)
__host__ __device__ inline int spec_stride(int ng) { return ((ng >> 1) + 1 + 15) & ~15; }
// Reaction partials a plan holds for the one-sided pair sum by default, per
// particle and in all (the 256^3 Plummer mix writes 56 per particle).
constexpr int64_t kPartialsPerParticle = 80;
// A group is dense (pairs with other dense groups evaluated once) above
// this many particles. Measured on the clustered 256^3 set (FP32 pair
// kernel + gather per force call, partials stored by record): above 48
// particles 33.1 + 5.0 ms, above 40 32.8 + 5.2, above 32 32.5 + 5.6, above
// 24 32.4 + 6.2 ms: fewer evaluations, more partials to gather; the sum is
// flat from 48 down to 32, which has the faster pair kernel. On a displaced
// lattice at one particle per cell (64 per group) most groups are then
// dense and the one-sided sum does not pay there, which is why it is a plan
// option for clustered input.
#ifndef P3M_DENSE_MIN
#define P3M_DENSE_MIN 32
#endif
constexpr int kDenseMin = P3M_DENSE_MIN;
constexpr int64_t kPartialsSlack = 65536;

// One particle in cell order: offsets from its cell's lower corner and mass.
// (x, y, z, m) as float4 (FP32 path) or double4 (FP64 path).

struct Workspace {
  int32_t* key = nullptr;       // [n_max]   cell index per particle (input order)
  int32_t* rank = nullptr;      // [n_max]   rank inside its cell
  int32_t* count = nullptr;     // [ncell+1] particles per cell
  int32_t* start = nullptr;     // [ncell+1] first sorted slot of each cell; start[ncell] = n
  int32_t* perm = nullptr;      // [n_max]   sorted slot -> input index
  int32_t* skey = nullptr;      // [n_max]   cell index per sorted slot
  int32_t* scan_tmp = nullptr;  // block sums of the scans
  int32_t* gchunk = nullptr;    // [ngroup+1] 64-particle chunks per i-group
  int32_t* goff = nullptr;      // [ngroup+1] exclusive scan of gchunk; goff[ngroup] = items
  int2* items = nullptr;        // [max_items] (group, chunk) work items of the pair loop
  int4* rows = nullptr;         // [nrows]   neighbour stencil of an i-group
  void* rec = nullptr;          // [n_max]   sorted particle records (T4)
  void* acc_pm = nullptr;       // [n_max]   PM acceleration in sorted order (T4)
  void* grid = nullptr;         // [ng^3]    real grid (density, then potential)
  void* spec = nullptr;         // [ng*ng*spec_stride(ng)] half-complex spectrum (T2), kz fastest
  void* twiddle = nullptr;      // [ng/2]    exp(-2 pi i k / ng) (T2)
  void* gtab = nullptr;         // [2*ng]    Green's function factor tables (T)
  unsigned long long* counter = nullptr;  // [1] pair-count scratch
  float* split_tab = nullptr;   // [4][kSplitBins + 1] cubic pieces of f on [0, r_c)
  double* split_tab64 = nullptr;  // [kSplitCoef64][kSplitBins + 1] FP64 pieces of f(r)
  double* power_acc = nullptr;  // [3 * kMaxPowerBins + 2] power-spectrum sums
  void* ewald_tab = nullptr;    // [(E/2+1)^3] double4 Ewald correction octant (E > 0)
  void* ewald_zpair = nullptr;  // [(E/2+1)^2 (E/2)][3] double2: z-adjacent node pairs of it
  // one-sided pair sum between dense groups (Newton's third law; plans
  // with rcap > 0)
  int4* segrows = nullptr;      // [nseg]    stencil cut into group segments, staging order:
                                //           (dx & 0xffff | dy << 16, dz_lo, dz_hi, sign)
  int4* prows = nullptr;        // [npos]    the positive segments (sign > 0), in that order
  int4* pbrows = nullptr;       // [npos]    the same bucketed by (dx mod G, dy mod G), w = index
  int32_t* pboff = nullptr;     // [G*G+1]   first bucketed segment of each bucket
  int32_t* rowoff = nullptr;    // [ngroup][npos+1] reaction entries of a dense group before
                                //           each positive segment; [npos] = total
  int32_t* gipre = nullptr;     // [ngroup][G*G] particles of a group before each of its z-runs
  int32_t* gntot = nullptr;     // [ngroup]  particles per i-group
  long long* gtot = nullptr;    // [ngroup]  reaction partials per i-group
  long long* gbase = nullptr;   // [ngroup+1] exclusive scan of gtot; [ngroup] = total
  long long* gscan_tmp = nullptr;  // tile sums of that scan
  void* rpart = nullptr;        // [rcap][3] reaction partials (T), components together
  void* acc_mesh = nullptr;     // [n_max]   sorted mesh acceleration of a one-sided force (T4)
  // adjoint workspace (plans created with params.adjoint != 0)
  void* lam = nullptr;          // [n_max]   force cotangent in sorted order (T4)
  void* grid2 = nullptr;        // [ng^3]    second real grid (divergence, then psi)
  void* lam_grid = nullptr;     // [3][ng^3] CIC deposit of m * cotangent
};

}  // namespace p3m

struct p3m_plan {
  p3m_params prm{};
  int64_t n_max = 0;
  hipStream_t stream = nullptr;
  // second stream of the P3M force: the mesh part (deposit, Poisson solve)
  // runs on it while the pair sum runs on `stream`; events fork and join
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int device = 0;
  // set for the duration of a p3m_force_cell_order call: the force is
  // written at the particle's sorted slot instead of its input index
  bool cell_order = false;
  // geometry
  int ng = 0, lg = 0;           // grid cells per side and its log2
  int64_t ncell = 0;
  double h = 0, r_s = 0, r_c = 0, eps = 0;
  int G = 2, lgG = 1;           // i-group edge in cells and its log2
  int ngd = 0;                  // i-groups per side
  int64_t ngroup = 0;
  int nrows = 0;
  int nseg = 0, npos = 0;       // stencil segments, and the positive ones
  int64_t rcap = 0;             // reaction partials the plan holds (0: two-sided sum only)
  int64_t max_items = 0;
  int tab_var = 0;              // FP32 split table: variable (0: r, 1: softened r)
  double tab_v0 = 0, tab_v1 = 0;  // and its range, as lengths
  int tab64_var = 0;            // FP64 split table: the same, and the number of
  double tab64_v0 = 0, tab64_v1 = 0;  // leading pieces evaluated exactly
  int tab64_exact = 0;
  int scan_tmp_len = 0;
  int count_dirty = 1;          // cell counts not known to be zero (set until a binning's scan)
  p3m::Workspace ws;
  // stage timers: events [call][2 * stage + {0: start, 1: end}]
  int timing_cap = 0;           // force calls that can be recorded
  int timing_calls = 0;         // calls recorded so far
  int timing_slot = -1;         // slot of the call in progress (-1: not recording)
  hipEvent_t* ev = nullptr;     // [timing_cap * 2 * P3M_NUM_STAGES]
  unsigned char* ran = nullptr; // [timing_cap * P3M_NUM_STAGES]
};

namespace p3m {

// Launchers (each enqueues on plan->stream; returns hipSuccess or the error).
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_scan(int32_t* in, int32_t* out, int64_t len, int32_t* tmp, hipStream_t s,
                       bool zero_in = false);
int scan_tmp_size(int64_t len);
int items_tmp_size(int64_t ngroup);   // block sums of the work-list scan

hipError_t launch_bin(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                      double mass_scalar);
hipError_t launch_items(p3m_plan* P);

template <typename T>
hipError_t launch_deposit(p3m_plan* P);
template <typename T>
hipError_t launch_deposit3(p3m_plan* P, const void* lam, void* grids);   // m * lam, 3 grids
template <typename T>
hipError_t launch_fft_poisson(p3m_plan* P);
template <typename T>
hipError_t launch_interp(p3m_plan* P, int64_t n, void* force_out, int force_fp32,
                         const void* acc_pp = nullptr, void* sorted_out = nullptr);
template <typename T>
hipError_t launch_pairs(p3m_plan* P, int64_t n, bool add_pm, void* force_out, int force_fp32,
                        bool uniform_mass, void* acc_out = nullptr);
template <typename T>
hipError_t launch_pair_count(p3m_plan* P, int64_t n, int64_t* count_out);
// One-sided pair sum (plans with rcap > 0): per-group reaction offsets and
// partial bases (after the work list, before the pair kernel, which then
// writes the sorted action to ws.acc_pm), and the gather of the reaction
// partials onto that action (after it): the result goes to acc_out (sorted,
// T4) if not null, else to out in input order as m * a (float if out_fp32).
hipError_t launch_react_prepass(p3m_plan* P);
template <typename T>
hipError_t launch_pair_gather(p3m_plan* P, int64_t n, bool vjp, bool uniform_mass,
                              void* acc_out, void* out, int out_fp32,
                              const void* acc_add = nullptr);
int64_t react_scan_tmp_size(int64_t ngroup);
template <typename T>
hipError_t launch_react_gather(p3m_plan* P, int64_t n, double rscale, bool uniform_mass,
                               void* acc_out, void* out, int out_fp32,
                               const void* acc_add = nullptr);
template <typename T>
hipError_t launch_tables(p3m_plan* P);

hipError_t launch_ewald_table(p3m_plan* P);
hipError_t launch_pp_ewald(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                           double ms, const int32_t* order, void* force, int force_fp32);
hipError_t launch_ewald_eval(p3m_plan* P, int64_t npts, const double* r, double* out);
template <typename T>
hipError_t launch_power_spectrum(p3m_plan* P, int nbins, double r_tophat, double* k_out,
                                 double* p_out, double* m_out, double* sigma_out);

// Adjoint stages (workspace of plans created with params.adjoint != 0).
template <typename T>
hipError_t launch_lambda_sort(p3m_plan* P, int64_t n, const double* force_bar);
template <typename T>
hipError_t launch_deposit_lambda(p3m_plan* P);   // divergence of the deposit -> grid2
template <typename T>
hipError_t launch_interp_vjp(p3m_plan* P, int64_t n, double* pos_bar,
                             const void* acc_pp = nullptr);
template <typename T>
hipError_t launch_pairs_vjp(p3m_plan* P, int64_t n, bool add_pm, double* pos_bar,
                            bool uniform_mass, void* acc_out = nullptr);
hipError_t launch_drift_vjp(int64_t n, double* mom_bar, const double* pos_bar,
                            const double* mass, double ms, double c, hipStream_t s);
hipError_t launch_kick_drift(int64_t n, double* pos, double* mom, const void* force, int fp32,
                             const double* mass, double ms, double ck, double cd, double box,
                             hipStream_t s);
hipError_t launch_kick(int64_t n, double* mom, const void* force, int fp32, double c,
                       hipStream_t s);
hipError_t launch_kick_reorder(int64_t n, const int32_t* order, const double* pos,
                               const double* mom, const void* force, int fp32,
                               const int64_t* ids, const double* mass, double c,
                               double* pos_out, double* mom_out, int64_t* ids_out,
                               double* mass_out, hipStream_t s);
hipError_t launch_drift(int64_t n, double* pos, const double* mom, const double* mass,
                        double ms, double c, double box, hipStream_t s);

// Host geometry helpers.
int stencil_rows(int g, double radius_cells, int32_t* out, int cap);
// The stencil rows cut where their z range crosses a group boundary: each
// segment lies in one group at offset (ox, oy, oz) = floor((dx, dy, dz) / g),
// with the sign of that offset in lexicographic order (0: the group itself).
// Entries (dx & 0xffff | dy << 16, dz_lo, dz_hi, sign); returns the count
// (and the positive count in *npos).
int segment_rows(int g, double radius_cells, int32_t* out, int cap, int* npos);
// Validation of the parameters (the checks and status codes of
// p3m_plan_create) and the plan's geometry: grid, split and cutoff lengths,
// i-group edge, stencil row count, work-list bound. Allocates nothing.
int plan_geometry(const p3m_params& q, int64_t n_max, p3m_plan* P);
// The stencil rows (computed into rows_host, P->nrows entries of 4 int32)
// and the split-factor tables copied into the plan's workspace on its
// stream (pageable host sources: each copy has read its source on return);
// sets the plan's table maps.
hipError_t plan_upload_tables(p3m_plan* P, int32_t* rows_host);
// Split-factor table: out[c * (bins + 1) + k] is coefficient c of bin k of
// the cubic pieces over v in [v0, v1] (units of r_s); var 0: v = r / r_s,
// var 1: v = sqrt(r^2 + eps^2) / r_s.
struct SplitMap {
  int var;
  double v0, v1;
  int exact;    // FP64: leading pieces the kernel replaces by the exact formula
};
SplitMap split_table(double cutoff_rs, double soft_rs, int bins, float* out);
// FP64 table: out[l * (kSplitBins + 1) + k] is the coefficient of t^l
// (t in [0, 1) across the bin) of piece k of the same variable choice; entry kSplitBins is
// the constant value at v1.
SplitMap split_table64(double cutoff_rs, double soft_rs, double* out);

}  // namespace p3m
