// Short-range pair sum of P3M over the sorted cell list.
//
//   a_i = -G sum_{j != i, 0 < r < r_c} m_j r_ij f(r) / (r^2 + eps^2)^(3/2)
//   f(r) = erfc(u) + (2u / sqrt(pi)) exp(-u^2),  u = r / (2 r_s)
//
// Work decomposition. The grid's cells are grouped into i-groups of G^3
// cells; a work item is (group, chunk) with up to kChunk (64) of the
// group's particles, one wavefront per item. The j-candidates of a group are the
// particles of every cell whose box comes closer than r_c to the group's box
// (the stencil rows: z-runs of cells, precomputed per plan).
//
// Lanes. Each lane holds U i-particles ("slots"), so every j it reads from
// LDS is tested against U particles: the LDS read, not the arithmetic, is the
// scarce resource of a cutoff test. With n_i particles the wave has
// n_u = ceil(n_i / U) slot-sets and s = 64 / n_u streams: lane (set, stream)
// takes every s-th staged j, so small groups still fill the wave, and the s
// partial sums of each i are added at the end. FP32: U = 8 above 32
// particles, else 4; FP64: U = 2; U = 1 for an item with a single particle.
//
// Staging. Per batch of 64 stencil rows each lane resolves one row into at
// most three contiguous sorted runs (the z-run split where it crosses the
// periodic box face), a wave scan flattens them, and the wave stages the
// runs' particles into LDS (kPairCap at a time) as positions relative to the
// group's first cell, carrying the periodic shift of the run. Positions are
// rebuilt from cell-relative offsets and small integer cell differences, so
// the FP32 path never subtracts two large coordinates. Over the
// softened-distance table they are kept in the table's units (times s), so
// the squared separation is the table's argument as it stands.
//
// Arithmetic. FP32: rsq(r^2 + eps^2) and f from a table of 64 cubic pieces
// held in LDS, fitted in FP64 by the plan at the Chebyshev points of each
// piece (error below 1e-7). The table's variable is the softened distance
// sqrt(r^2 + eps^2), which rsq already yields, so a pair costs a single
// transcendental; when eps is too large against a piece for the cubic to
// follow the kink at r = 0, the plan tabulates over r and a square root is
// added. FP64: the hardware rsqrt refined by one third-order step, and f
// from 64 pieces of degree 6 (fitted in extended precision at the Chebyshev
// points of each piece; error at FP64 rounding) over the softened distance
// as well, with the few pieces next to the kink evaluated exactly; or over r,
// with a square root.
#include <algorithm>

#include "p3m_internal.h"

namespace p3m {
namespace {

constexpr int kDesc = 3 * 64;          // runs per batch of 64 rows
// j-particles staged in LDS per pass: kPairCap for the FP32 force, half that
// for FP64 and for the adjoint (which stages the cotangents too), so that the
// workgroup's LDS leaves room for the waves per SIMD that kPairWaves asks the
// compiler to fit in registers (FP32 force 5, FP64 force 4, FP32 adjoint 4,
// FP64 adjoint 3; measured best).
template <typename T, bool VJP> struct Stage {
  static constexpr int kCap = sizeof(T) == 4 && !VJP ? kPairCap : kPairCap / 2;
  static constexpr int kPer = kCap / 64;   // consecutive staged entries per lane
};
// At most kStreams streams, so kStreams far sentinels after the staged
// entries cover every read past the end (an item with fewer than 64 / kStreams
// slot sets leaves lanes idle; only items of a handful of particles).
constexpr int kStreams = 16;
// Waves per SIMD the compiler must leave room for (caps the registers).
template <typename T, bool VJP>
constexpr int kPairWaves = sizeof(T) == 4 ? (VJP ? 4 : 5) : (VJP ? 3 : 4);
// A coordinate far outside any box: its squared separation from any real
// particle is ~1e37, finite in FP32 and far beyond every cutoff.
constexpr float kFar = 1e18f;

template <typename T>
struct PairArgs {
  const typename Vec<T>::v4* __restrict__ rec;
  const int32_t* __restrict__ skey;
  const int32_t* __restrict__ start;
  const int2* __restrict__ items;
  const int32_t* __restrict__ n_items;
  const int4* __restrict__ rows;
  int nrows;
  int ng, lg, G, lgG;
  T h, rc2;
  T eps2, inv2rs;                       // FP64 weight
  // FP32 weight from the split table: with s = kSplitBins / (v1 - v0) per
  // length, q = s^2 (r^2 + eps^2), the bin coordinate is x = q rsq(q) - s v0
  // (softened variable) or x = s r (plain r), and the returned weight is
  // f rsq(q)^3 = f / (s^3 (r^2 + eps^2)^(3/2)).
  const T* __restrict__ split_tab;      // FP32 [4][kSplitBins + 1], FP64 [7][kSplitBins + 1]
  float tab_s, tab_s2, tab_e2, tab_off;
  // Force over the softened-distance table: positions scaled by s, so
  // rho^2 starts from e2 = (s eps)^2 (floored: FP32 at tab_e2's 1e-12, FP64
  // at 1e-100) and is tested against s^2 r_c^2 + e2.
  float rho_e2, rho_cut2;               // FP32
  double rho_e2d, rho_cut2d;            // FP64
  double rho_inv2rs;                    // FP64: 1 / (2 r_s s), for the series
  double tab_s64, tab_off64;            // FP64 table: x = s v - s v0 (v = r or rho)
  int tab_exact;                        // FP64: leading pieces evaluated exactly
  double wscale;                        // -G, times s^3 on the FP32 path
  double wscale_rho;                    // -G s^2: force on scaled positions
  double wscale_vjp;                    // -G s^3: adjoint on scaled positions
  T rc2s;                               // s^2 r_c^2: cutoff on scaled positions
  // adjoint mode: sorted cotangent (x, y, z, -) and the constants of the
  // pair Hessian (see pair_vjp_weights)
  const typename Vec<T>::v4* __restrict__ lam;
  T vjp_ce, vjp_k5, vjp_e2, vjp_ce_s;   // vjp_ce_s = vjp_ce / s^3
  const typename Vec<T>::v4* __restrict__ acc_pm;  // sorted PM acceleration or null
  typename Vec<T>::v4* __restrict__ acc_out;       // sorted output acceleration or null
  const int32_t* __restrict__ perm;
  int64_t n;
  void* __restrict__ force;
  int force_fp32;
  unsigned long long* __restrict__ counter;      // pair count mode
  // one-sided sum between dense groups: the stencil's group segments,
  // particles per group, per-group reaction offsets and partial bases, the
  // partials [rcap][3] and their total this call (gbase[ngroup])
  const int4* __restrict__ segrows;
  int nseg, npos;
  const int32_t* __restrict__ gntot;
  const int32_t* __restrict__ rowoff;
  const long long* __restrict__ gbase;
  const long long* __restrict__ gtotal;
  void* __restrict__ rpart;
  long long rcap;
};

// The split-factor table in LDS, one array per coefficient so that the
// random per-lane bin lookups spread over the banks. FP32: cubic pieces in
// t in [0, 1); FP64: degree-6 pieces in t as well.
constexpr int kTabStride = kSplitBins + 1;
template <typename T> struct SplitTable;
template <> struct SplitTable<float> {
  static constexpr int kCoef = 4;
  float c[kCoef][kTabStride];
};
template <> struct SplitTable<double> {
  static constexpr int kCoef = kSplitCoef64;
  double c[kCoef][kTabStride];
};

// f near r = 0 from its series: df/du = -(4/sqrt(pi)) u^2 e^{-u^2}, so
// f = 1 - (4/sqrt(pi)) u^3 sum_n (-1)^n u^{2n} / (n! (2n + 3)), alternating with
// falling terms for u < 1: 16 terms leave less than 4e-17 for u <= 0.9.
constexpr int kSeriesTerms = 16;
constexpr double series_coef(int n) {
  double fact = 1.0;
  for (int i = 2; i <= n; ++i) fact *= i;
  return (n % 2 ? -1.0 : 1.0) / (fact * (2 * n + 3));
}

// Out of line: its sixteen constants would otherwise stay in registers
// across the whole pair loop for a branch that is rarely taken (FP64 loop
// 128 -> 108 VGPRs, no spills, 2.5 % faster).
__device__ __attribute__((noinline)) double split_f64_series(double r2, double inv2rs) {
  const double s = r2 * inv2rs * inv2rs;              // u^2
  double p = series_coef(kSeriesTerms - 1);
#pragma unroll
  for (int n = kSeriesTerms - 2; n >= 0; --n) p = fma(p, s, series_coef(n));
  return 1.0 - 2.2567583341910251 * (sqrt(r2) * inv2rs) * s * p;
}

// 1 / sqrt(q) to FP64 rounding for q > 0: the hardware estimate refined by
// one third-order step, y (1 + e/2 + 3e^2/8) with e = 1 - q y^2 (cubic
// convergence from its roughly 23 correct bits). No fix-ups for zero,
// infinite or negative q: the only such case, q = 0 (a self pair without
// softening), has its weight discarded by the caller.
__device__ __forceinline__ double rsqrt_pos(double q) {
  const double y = __builtin_amdgcn_rsq(q);
  const double e = fma(-q * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// FP64 split factor f from the table. TAB 1: the variable is the softened
// distance rho = q rsqrt(q), q = r^2 + eps^2 (no square root); the few
// leading pieces next to the kink at r = 0 that a polynomial cannot follow to
// FP64 rounding take the series above instead (pairs closer than a few bins,
// u <= 0.9 by the plan's choice: rare, so the divergent branch is cheap).
// TAB 0: the variable is r.
template <int TAB>
__device__ __forceinline__ double split_f64(double r2, double q, double inv,
                                            const PairArgs<double>& A,
                                            const SplitTable<double>& tab) {
  const double x = TAB ? fma(q * inv, A.tab_s64, -A.tab_off64) : sqrt(r2) * A.tab_s64;
  const int k = min(max((int)x, 0), kSplitBins);   // x >= 0 and k <= kSplitBins for r < r_c
  if (TAB && k < A.tab_exact) return split_f64_series(r2, A.inv2rs);
  const double t = __builtin_amdgcn_fract(x);     // x >= 0 (k = 64: constant piece)
  double f = tab.c[kSplitCoef64 - 1][k];
#pragma unroll
  for (int l = kSplitCoef64 - 2; l >= 0; --l) f = f * t + tab.c[l][k];
  return f;
}

// f(r) / (r^2 + eps^2)^(3/2) for 0 <= r < r_c, up to the factor folded into
// wscale. Self pairs (r = 0) give a finite weight times a zero separation.
// FP32: f from the table, TAB selecting the variable (1: softened distance).
// The squared scaled radius is floored at 1e-12 bins^2 (a radius a million
// times below a bin, beneath FP32 position resolution), which keeps the
// weight finite at r = 0 when eps = 0.
template <int TAB>
__device__ __forceinline__ float pair_weight(float r2, const PairArgs<float>& A,
                                             const SplitTable<float>& tab) {
  const float q = __builtin_fmaf(r2, A.tab_s2, A.tab_e2);
  const float inv = __builtin_amdgcn_rsqf(q);
  const float x = TAB ? __builtin_fmaf(q, inv, -A.tab_off)
                      : __builtin_amdgcn_sqrtf(r2) * A.tab_s;   // >= 0
  const int k = (int)x;                 // <= kSplitBins since r < r_c
  const float t = __builtin_amdgcn_fractf(x);
  const float f = tab.c[0][k] + t * (tab.c[1][k] + t * (tab.c[2][k] + t * tab.c[3][k]));
  return f * (inv * inv * inv);
}

// The same weight from q = s^2 (r^2 + eps^2) (floored as above), formed from
// positions already scaled by s.
__device__ __forceinline__ float pair_weight_rho(float q, const PairArgs<float>& A,
                                                 const SplitTable<float>& tab) {
  const float inv = __builtin_amdgcn_rsqf(q);
  const float x = __builtin_fmaf(q, inv, -A.tab_off);
  const int k = (int)x;
  const float t = __builtin_amdgcn_fractf(x);
  const float f = tab.c[0][k] + t * (tab.c[1][k] + t * (tab.c[2][k] + t * tab.c[3][k]));
  return f * (inv * inv * inv);
}

template <int TAB>
__device__ __forceinline__ double pair_weight(double r2, const PairArgs<double>& A,
                                              const SplitTable<double>& tab) {
  const double q = r2 + A.eps2;
  const double inv = rsqrt_pos(q);
  const double f = split_f64<TAB>(r2, q, inv, A, tab);
  return r2 > 0.0 ? f * (inv * inv * inv) : 0.0;   // eps may be 0
}

// The same weight (softened-distance table) from q = s^2 (r^2 + eps^2),
// formed from positions already scaled by s, so the bin coordinate is
// q rsqrt(q) - s v0 and the weight f / (s rho)^3; r^2 itself is formed only
// for the series pieces. q starts from (s eps)^2 floored at 1e-100, so the
// weight is finite for every pair (at most 1e150, leaving room for a
// per-particle mass factor up to 1e150) and a self or coincident pair
// contributes it times a zero separation. The bin coordinate lies in
// [0, kSplitBins] without clamping: the table starts a hair below s eps and
// the cutoff test bounds q by s^2 (r_c^2 + eps^2), its end.
__device__ __forceinline__ double pair_weight_rho(double q, const PairArgs<double>& A,
                                                  const SplitTable<double>& tab) {
  const double inv = rsqrt_pos(q);
  const double x = fma(q, inv, -A.tab_off64);
  const int k = (int)x;
  double f;
  if (k < A.tab_exact) {
    f = split_f64_series(fmax(q - A.rho_e2d, 0.0), A.rho_inv2rs);
  } else {
    const double t = __builtin_amdgcn_fract(x);
    f = tab.c[kSplitCoef64 - 1][k];
#pragma unroll
    for (int l = kSplitCoef64 - 2; l >= 0; --l) f = f * t + tab.c[l][k];
  }
  return f * (inv * inv * inv);
}

// Adjoint weights of a pair: with g = f / rho^3 and the pair Jacobian
// J = g I + (g'(r)/r) r r^T, J dl = w1 dl + w2 (r . dl) r, where
// w1 = g and w2 = g'(r)/r = d / rho^3 - 3 f / rho^5, d = f'(r) / r.
// Over the softened-distance table (TAB 1), d = (df/drho) / rho, and df/drho
// is s times the derivative of the piece in its position t (the piece's
// derivative misses f' by at most a few 1e-6 of w2 in FP32, 4e-11 in FP64,
// both at the cutoff); the FP64 leading pieces evaluated exactly take
// d = -r e^{-u^2} / (2 sqrt(pi) r_s^3) with e^{-u^2} from its series. Over r
// (TAB 0, wide softening) d comes from that formula with the library
// exponential.
// Units. TAB 1 works on positions scaled by s (r2 = s^2 r^2): with
// inv = 1 / (s rho) the returned w1 = f inv^3 and w2 = inv^3 (ft inv - 3 f
// inv^2) (ft the piece's t-derivative) are g / s^3 and (g'(r)/r) / s^5, so
// J dl = s^3 (w1 dl + w2 (r_s . dl) r_s) with r_s the scaled separation; the
// s^3 sits in wscale_vjp. TAB 0 works on physical positions: FP32 in the
// scaled units of pair_weight (rsq(q) = 1 / (s rho), s^3 folded into wscale,
// vjp_k5 = 3 s^2); FP64 in physical units (vjp_k5 = 3).
// Called only for 0 < r2 < r_c^2: the pair loop's test excludes coincident
// particles (their pairs contribute nothing), so the weights need no guard.
template <int TAB>
__device__ __forceinline__ void pair_vjp_weights(float r2, const PairArgs<float>& A,
                                                 const SplitTable<float>& tab, float& w1,
                                                 float& w2) {
  const float q = TAB ? r2 + A.tab_e2 : __builtin_fmaf(r2, A.tab_s2, A.tab_e2);
  const float inv = __builtin_amdgcn_rsqf(q);
  const float x = TAB ? __builtin_fmaf(q, inv, -A.tab_off)
                      : __builtin_amdgcn_sqrtf(r2) * A.tab_s;
  const int k = (int)x;
  const float t = __builtin_amdgcn_fractf(x);
  const float inv2 = inv * inv, inv3 = inv2 * inv;
  if constexpr (TAB == 1) {
    // the cubic and its t-derivative together (Horner on both)
    float f = tab.c[3][k], ft = f;
    f = __builtin_fmaf(f, t, tab.c[2][k]);
    ft = __builtin_fmaf(ft, t, f);
    f = __builtin_fmaf(f, t, tab.c[1][k]);
    ft = __builtin_fmaf(ft, t, f);
    f = __builtin_fmaf(f, t, tab.c[0][k]);
    w1 = f * inv3;
    w2 = inv3 * (ft * inv - 3.f * f * inv2);
  } else {
    const float f = tab.c[0][k] + t * (tab.c[1][k] + t * (tab.c[2][k] + t * tab.c[3][k]));
    const float d = -A.vjp_ce * __builtin_amdgcn_sqrtf(r2) * __builtin_amdgcn_exp2f(r2 * A.vjp_e2);
    w1 = f * inv3;
    w2 = inv3 * (d - A.vjp_k5 * f * inv2);
  }
}

// e^{-s}, 0 <= s <= 0.81 (u <= 0.9), from its series: 19 terms leave less
// than 1e-17.
__device__ __forceinline__ double exp_neg_series(double s) {
  double p = 1.0;
#pragma unroll
  for (int n = 18; n >= 1; --n) p = fma(p, -s * (1.0 / n), 1.0);
  return p;
}

template <int TAB>
__device__ __forceinline__ void pair_vjp_weights(double r2, const PairArgs<double>& A,
                                                 const SplitTable<double>& tab, double& w1,
                                                 double& w2) {
  const double q = r2 + (TAB ? A.rho_e2d : A.eps2);
  const double inv = rsqrt_pos(q);
  const double inv2 = inv * inv, inv3 = inv2 * inv;
  double f, d;
  if constexpr (TAB == 1) {             // scaled positions; x in [0, kSplitBins]
    const double x = fma(q, inv, -A.tab_off64);
    const int k = (int)x;
    if (k < A.tab_exact) {              // next to the kink at r = 0: rare
      const double u2 = r2 * A.rho_inv2rs * A.rho_inv2rs;
      f = split_f64_series(r2, A.rho_inv2rs);
      d = -A.vjp_ce_s * (r2 * rsqrt_pos(r2)) * exp_neg_series(u2);
    } else {
      const double t = __builtin_amdgcn_fract(x);
      f = tab.c[kSplitCoef64 - 1][k];
      double ft = f;                    // the piece and its t-derivative by Horner
      f = fma(f, t, tab.c[kSplitCoef64 - 2][k]);
#pragma unroll
      for (int l = kSplitCoef64 - 3; l >= 0; --l) {
        ft = fma(ft, t, f);
        f = fma(f, t, tab.c[l][k]);
      }
      d = ft * inv;
    }
  } else {
    const double r = sqrt(r2);
    const double u = r * A.inv2rs;
    f = split_f64<TAB>(r2, q, inv, A, tab);
    d = -A.vjp_ce * r * exp(-u * u);
  }
  w1 = f * inv3;
  w2 = inv3 * (d - A.vjp_k5 * f * inv2);
}

__device__ __forceinline__ int wave_inclusive(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// The bounding box of an item's i-particles (relative to the group's first
// cell, in the kernel's position units) and the reach r_c (with a 1e-4
// margin, far above rounding): a stencil cell whose box stays farther than
// r_c from the item's box holds no partner of any of its particles, so the
// rows are clipped to the cells within reach.
template <typename T>
struct ItemBox {
  T lo[3], hi[3];
  T hs;       // cell size
  T reach2;   // (r_c (1 + 1e-4))^2
};
template <>
struct ItemBox<double> {};     // the FP64 pair loop stages whole rows

template <typename T, bool VJP, bool HALF>
struct PairShared {
  SplitTable<T> tab;                       // first, so one address register reaches
                                           // all coefficient arrays
  typename Vec<T>::v4 jb[Stage<T, VJP>::kCap + kStreams];   // staged j (+ far sentinels); reused for
                                                // the reduction
  typename Vec<T>::v4 jl[VJP ? Stage<T, VJP>::kCap + kStreams : 1];   // adjoint mode: staged j cotangents
  int d_lo[kDesc], d_pre[kDesc + 1], d_zs[kDesc];
  int d_rp[HALF ? kDesc : 1];              // one-sided sum: partial offset of each run's
                                           // first entry in the item's reactions, or -1
  int owner[Stage<T, VJP>::kCap];               // run of each staged entry of a chunk
  int d_rx[64], d_ry[64];                  // x, y cell offsets of each row
  int i_lo[16], i_pre[17];
  ItemBox<T> box;                          // the item's i-particles' bounding box
};

// Sum of v over each aligned group of nu lanes (nu a power of two <= 32),
// left in the group's top lane (lane % nu == nu - 1): pairwise sums inside
// quads, then right shifts within rows of 16, then the row broadcast. The
// other lanes hold partial sums.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_take(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_take(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int NU, typename T>
__device__ __forceinline__ T group_sum_top(T v) {
  if constexpr (NU >= 2) v += dpp_take<0xB1>(v);          // quad_perm [1, 0, 3, 2]
  if constexpr (NU >= 4) v += dpp_take<0x4E>(v);          // quad_perm [2, 3, 0, 1]
  if constexpr (NU >= 8) v += dpp_take<0x114>(v);         // row_shr:4
  if constexpr (NU >= 16) v += dpp_take<0x118>(v);        // row_shr:8
  if constexpr (NU >= 32) v += dpp_take<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  return v;
}

// Cells [z0, z1] of the column at (dx, dy) clipped to those within reach of
// the item's box; false if none.
template <typename T>
__device__ __forceinline__ bool clip_to_box(const ItemBox<T>& B, int dx, int dy, int& z0,
                                            int& z1) {
  if constexpr (sizeof(T) == 8) {
    return true;     // FP64: whole rows
  } else {
  const T gx = fmax(T(0), fmax(T(dx) * B.hs - B.hi[0], B.lo[0] - T(dx + 1) * B.hs));
  const T gy = fmax(T(0), fmax(T(dy) * B.hs - B.hi[1], B.lo[1] - T(dy + 1) * B.hs));
  const T rem = B.reach2 - gx * gx - gy * gy;
  if (!(rem > T(0))) return false;
  const T zr = sqrt(rem);
  z0 = max(z0, (int)floor((B.lo[2] - zr) / B.hs));
  z1 = min(z1, (int)floor((B.hi[2] + zr) / B.hs));
  return z0 <= z1;
  }
}

// One stencil row (per lane) resolved into at most three contiguous sorted
// runs (the z-run split where it crosses the periodic box face): first slot,
// count and the unwrapped z-cell shift of each run relative to the group.
template <typename T>
struct RowRuns {
  int cnt[3], lo[3], zs[3];
  int rx, ry;                               // x, y cell offset of the row's column
  int rf;                                   // one-sided sum: run 0 takes reactions
};

template <typename T>
__device__ __forceinline__ RowRuns<T> resolve_rows(const PairArgs<T>& A, const int4* rows,
                                                   int nrows, int rb, int lane, int gx0,
                                                   int gy0, int gz0, const ItemBox<T>& B) {
  RowRuns<T> R;
  const int lg = A.lg, ng = A.ng, mask = ng - 1;
#pragma unroll
  for (int k = 0; k < 3; ++k) R.cnt[k] = R.lo[k] = R.zs[k] = 0;
  R.rx = R.ry = R.rf = 0;
  int z0 = 0, z1 = -1;
  int4 row = make_int4(0, 0, 0, -1);
  if (rb + lane < nrows) {
    row = rows[rb + lane];
    z0 = row.z;
    z1 = row.w;
  }
  if (z0 <= z1 && clip_to_box(B, row.x, row.y, z0, z1)) {
    const int jx = (gx0 + row.x) & mask, jy = (gy0 + row.y) & mask;
    R.rx = row.x;
    R.ry = row.y;
    const int zhi = gz0 + z1;
    int z = gz0 + z0;
    const int cbase = ((jx << lg) | jy) << lg;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (z <= zhi) {
        int zw = z & mask;
        int len = min(zhi - z + 1, ng - zw);
        int l0 = A.start[cbase + zw];
        R.lo[k] = l0;
        R.cnt[k] = A.start[cbase + zw + len] - l0;
        R.zs[k] = (z - zw) - gz0;
        z += len;
      }
    }
  }
  return R;
}

// The item's own group as runs (one z-run of G cells per lane < G^2, in the
// group's flattened order), from flattened index `from` on.
template <typename T, typename SH>
__device__ __forceinline__ RowRuns<T> own_group_runs(const SH& S, int lane,
                                                     int lgG, int G, int gz0, int from) {
  RowRuns<T> R;
#pragma unroll
  for (int k = 0; k < 3; ++k) R.cnt[k] = R.lo[k] = R.zs[k] = 0;
  R.rx = R.ry = R.rf = 0;
  if (lane < G * G) {
    const int c = S.i_pre[lane + 1] - S.i_pre[lane];
    const int skip = min(max(from - S.i_pre[lane], 0), c);
    R.rx = lane >> lgG;
    R.ry = lane & (G - 1);
    R.lo[0] = S.i_lo[lane] + skip;
    R.cnt[0] = c - skip;
    R.zs[0] = -gz0;
  }
  return R;
}

// One group segment of the stencil (per lane) for an item of a dense group:
// a segment in another dense group at a positive offset is staged with its
// reactions, one in a sparse group (either sign) without, others not at
// all (the group's own segments: staged from the group itself; a dense
// group at a negative offset: that group evaluates the pairs). A segment
// lies inside one group, so it is one contiguous run.
template <typename T>
__device__ __forceinline__ RowRuns<T> resolve_segments(const PairArgs<T>& A, int rb, int lane,
                                                       int gx0, int gy0, int gz0,
                                                       const ItemBox<T>& B) {
  RowRuns<T> R;
  const int lg = A.lg, ng = A.ng, mask = ng - 1, lgG = A.lgG;
#pragma unroll
  for (int k = 0; k < 3; ++k) R.cnt[k] = R.lo[k] = R.zs[k] = 0;
  R.rx = R.ry = R.rf = 0;
  if (rb + lane < A.nseg) {
    const int4 sg = A.segrows[rb + lane];
    const int dx = (int)(short)(sg.x & 0xffff), dy = sg.x >> 16;
    const int lgd = lg - lgG, md = (1 << lgd) - 1;
    const int64_t g2 = ((int64_t)(((gx0 >> lgG) + (dx >> lgG)) & md) << (2 * lgd)) |
                       ((int64_t)(((gy0 >> lgG) + (dy >> lgG)) & md) << lgd) |
                       (((gz0 >> lgG) + (sg.y >> lgG)) & md);
    const bool dense = sg.w != 0 && A.gntot[g2] > kDenseMin;
    const bool react = sg.w > 0 && dense;
    // a segment without reactions is clipped to the cells within reach of
    // the item's box; one with reactions is staged whole (the partial
    // offsets of all the group's items follow its full particle count)
    int z0 = sg.y, z1 = sg.z;
    if ((sg.w > 0 || (sg.w < 0 && !dense)) && (react || clip_to_box(B, dx, dy, z0, z1))) {
      const int jx = (gx0 + dx) & mask, jy = (gy0 + dy) & mask;
      const int cbase = ((jx << lg) | jy) << lg;
      const int z = gz0 + z0, zw = z & mask;
      const int l0 = A.start[cbase + zw];
      R.lo[0] = l0;
      R.cnt[0] = A.start[cbase + zw + (z1 - z0 + 1)] - l0;
      R.zs[0] = (z - zw) - gz0;
      R.rx = dx;
      R.ry = dy;
      R.rf = react;
    }
  }
  return R;
}

// One work item with U i-slots per lane. UM: every particle has the same mass
// (mass applied once at the end instead of per pair). VJP: the adjoint sum
// J(r_ij) (lam_i - lam_j) in place of the force r_ij g(r_ij). HALF: the
// one-sided sum (each pair of distinct items' particles once, the reaction
// on every staged entry past the item's own chunk written as a partial);
// else every pair from both sides over the full stencil. NU: the number of
// slot sets of the one-sided sum (a power of two, fixed per instantiation so
// that the sums over them are straight-line code).
template <typename T, int U, bool COUNT, bool UM, int TAB, bool VJP, bool HALF, int NU,
          typename SH>
__device__ __forceinline__ void pair_item(const PairArgs<T>& A, SH& S, int gx0,
                                          int gy0, int gz0, int ibeg, int ni, int64_t g) {
  using T4 = typename Vec<T>::v4;
  constexpr int kCap = Stage<T, VJP>::kCap, kStage = Stage<T, VJP>::kPer;
  const int lane = threadIdx.x;
  const int ng = A.ng, mask = ng - 1, lgG = A.lgG, G = A.G, GG = G * G;
  // The force over the softened-distance table runs on positions scaled by
  // the table's s (the bin coordinate then needs no extra multiply). An i
  // and its own staged copy must come out bit-identical (the self pair's
  // separation is exactly zero), so both are formed by the same fma and then
  // the same multiply.
  constexpr bool SC = TAB == 1 && !COUNT;
  const T h = A.h;
  const T ps = sizeof(T) == 4 ? T(A.tab_s) : T(A.tab_s64);
  auto coord = [&](int cell, T off) {
    const T v = fma(T(cell), h, off);
    return SC ? v * ps : v;
  };
  // slot sets; the one-sided sum sums each staged entry's reaction over the
  // sets, so their number is rounded up to a power of two (empty sets idle)
  const int nu = HALF ? NU : (ni + U - 1) / U;
  const int ns = min(64 / nu, kStreams);  // streams
  const int il = lane % nu, st = lane / nu;
  const bool active = st < ns;

  T xi[U], yi[U], zi[U], ax[U], ay[U], az[U];
  T lxi[VJP ? U : 1], lyi[VJP ? U : 1], lzi[VJP ? U : 1];
  T mi[HALF && !UM ? U : 1];
  int si[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = il + u * nu;            // particle of this slot within the chunk
    const bool has = active && q < ni;
    const int fi = ibeg + min(q, ni - 1);
    int run = 0;
    while (run + 1 < GG && S.i_pre[run + 1] <= fi) ++run;
    si[u] = S.i_lo[run] + (fi - S.i_pre[run]);
    const T4 pi = A.rec[si[u]];
    const int czi = A.skey[si[u]] & mask;
    xi[u] = has ? coord(run >> lgG, pi.x) : T(kFar);
    yi[u] = has ? coord(run & (G - 1), pi.y) : T(kFar);
    zi[u] = has ? coord(czi - gz0, pi.z) : T(kFar);
    ax[u] = ay[u] = az[u] = T(0);
    if constexpr (HALF && !UM) mi[u] = pi.w;
    if constexpr (VJP) {
      const T4 li = A.lam[si[u]];
      lxi[u] = li.x;
      lyi[u] = li.y;
      lzi[u] = li.z;
    }
  }
  // the item's bounding box (empty slots excluded), for clipping the rows;
  // kept in LDS (read once per batch of rows) to spare registers. FP32
  // only: the FP64 pair loop measured slower with it (117 -> 125 ms on the
  // 256^3 clustered set; FP32 44.3 -> 41.8 ms).
  if constexpr (sizeof(T) == 4) {
    T lo0 = T(kFar), lo1 = T(kFar), lo2 = T(kFar), hi0 = T(-kFar), hi1 = T(-kFar), hi2 = T(-kFar);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (xi[u] < T(0.5 * kFar)) {        // a particle, not an empty slot
        lo0 = fmin(lo0, xi[u]); hi0 = fmax(hi0, xi[u]);
        lo1 = fmin(lo1, yi[u]); hi1 = fmax(hi1, yi[u]);
        lo2 = fmin(lo2, zi[u]); hi2 = fmax(hi2, zi[u]);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo0 = fmin(lo0, __shfl_xor(lo0, o, 64)); hi0 = fmax(hi0, __shfl_xor(hi0, o, 64));
      lo1 = fmin(lo1, __shfl_xor(lo1, o, 64)); hi1 = fmax(hi1, __shfl_xor(hi1, o, 64));
      lo2 = fmin(lo2, __shfl_xor(lo2, o, 64)); hi2 = fmax(hi2, __shfl_xor(hi2, o, 64));
    }
    if (lane == 0) {
      S.box.lo[0] = lo0; S.box.lo[1] = lo1; S.box.lo[2] = lo2;
      S.box.hi[0] = hi0; S.box.hi[1] = hi1; S.box.hi[2] = hi2;
      S.box.hs = SC ? h * ps : h;
      S.box.reach2 = (SC ? A.rc2s : A.rc2) * T(1.0002);

    }
    __syncthreads();
  }
  const ItemBox<T>& B = S.box;
  int npairs = 0;
  // one-sided sum: the item's partials start at ibase; staged entry P (in
  // staging order over the item's own group, then the half stencil) past its
  // own chunk (P >= ni) goes to ibase + P - ni
  long long ibase = 0, ptotal = 0;
  int staged = 0;     // entries staged so far (phase 1: the item's own group)
  int rstaged = 0;    // reaction entries staged so far (phase 2: the segments)
  if constexpr (HALF) {
    ptotal = *A.gtotal;
    const int ntot = S.i_pre[GG];
    const int L = A.rowoff[g * (A.npos + 1) + A.npos];
    const int a = ibeg / kChunk;
    ibase = A.gbase[g] + (long long)a * (ntot + L) - 32LL * a * (a + 1);
  }

  // The staged entries of one batch of rows (descriptors per lane), kCap at
  // a time.
  // phase 1: the item's own group (reactions for entries past its own
  // chunk, by position); phase 2: group segments (reactions for flagged runs).
  auto run_batch = [&](const RowRuns<T>& cur, int phase) {
    __syncthreads();       // previous batch is done with the descriptors and jb
    const int tot_l = cur.cnt[0] + cur.cnt[1] + cur.cnt[2];
    const int inc = wave_inclusive(tot_l);
    int rtotal = 0;
    if (HALF && phase == 2) {
      const int rc = cur.rf ? cur.cnt[0] : 0;
      const int rinc = wave_inclusive(rc);
      const int intra = S.i_pre[GG] - ibeg - ni;
      S.d_rp[3 * lane] = cur.rf ? intra + rstaged + rinc - rc : -1;
      S.d_rp[3 * lane + 1] = S.d_rp[3 * lane + 2] = -1;
      rtotal = __builtin_amdgcn_readfirstlane(__shfl(rinc, 63, 64));
    }
    int pre[3];
    {
      int base = inc - tot_l;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        pre[k] = base;
        S.d_lo[3 * lane + k] = cur.lo[k];
        S.d_pre[3 * lane + k] = base;
        S.d_zs[3 * lane + k] = cur.zs[k];
        base += cur.cnt[k];
      }
    }
    S.d_rx[lane] = cur.rx;
    S.d_ry[lane] = cur.ry;
    const int total = __builtin_amdgcn_readfirstlane(__shfl(inc, 63, 64));
    if (lane == 63) S.d_pre[kDesc] = total;

    for (int c0 = 0; c0 < total; c0 += kCap) {
      const int cn = min(kCap, total - c0);
      __syncthreads();     // descriptors visible; previous chunk done with jb
      // owner[q] = run of chunk entry q: each run marks its first entry in the
      // chunk, then a prefix maximum over the chunk fills the rest
      const int q0 = kStage * lane;
#pragma unroll
      for (int e = 0; e < kStage; ++e) S.owner[q0 + e] = -1;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int s = pre[k] - c0;
        if (cur.cnt[k] > 0 && s + cur.cnt[k] > 0 && s < cn) S.owner[max(s, 0)] = 3 * lane + k;
      }
      __syncthreads();
      int dd[kStage];
      {
        int run = -1;
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
          run = max(run, S.owner[q0 + e]);
          dd[e] = run;
        }
        // exclusive prefix maximum of the lanes' last values
        int carry = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          int t = __shfl_up(carry, o, 64);
          if (lane >= o) carry = max(carry, t);
        }
        int before = __shfl_up(carry, 1, 64);
        if (lane == 0) before = -1;
#pragma unroll
        for (int e = 0; e < kStage; ++e) dd[e] = max(dd[e], before);
      }
      // stage entries [kStage*lane, kStage*lane + kStage) of this chunk, all
      // loads in flight together
      {
        int src[kStage];
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
          const int f = c0 + q0 + e;
          src[e] = q0 + e < cn ? S.d_lo[dd[e]] + (f - S.d_pre[dd[e]]) : -1;
        }
        T4 pj[kStage], lj[VJP ? kStage : 1];
        int cz[kStage];
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
          if (src[e] >= 0) {
            pj[e] = A.rec[src[e]];
            cz[e] = A.skey[src[e]] & mask;
            if constexpr (VJP) lj[e] = A.lam[src[e]];
          }
        }
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
          if (src[e] >= 0) {
            const int d = dd[e];
            T4 o;
            o.x = coord(S.d_rx[d / 3], pj[e].x);
            o.y = coord(S.d_ry[d / 3], pj[e].y);
            o.z = coord(cz[e] + S.d_zs[d], pj[e].z);
            o.w = pj[e].w;
            S.jb[q0 + e] = o;
            if constexpr (VJP) S.jl[q0 + e] = lj[e];
          }
        }
      }
      {                                // far-away sentinels after the last entry
        T4 far;
        far.x = far.y = far.z = T(-kFar);
        far.w = T(0);
        if (lane < kStreams) S.jb[cn + lane] = far;
      }
      __syncthreads();
      // lane (set, stream) takes staged entries st, st + ns, ...; the trip
      // count is wave-uniform; reads past the end (at most ns - 1) hit the
      // sentinels, and empty slots sit at +kFar, so both fail the cutoff test.
      // Lanes beyond the streams (st >= ns, all slots empty) read stream 0's
      // entries, so no read passes the sentinels. In the one-sided sum the
      // top lane of each stream's slot sets writes the step's reaction on its
      // entry over that entry in jb once every lane has read it (each entry
      // is read in one step only, by its own stream).
      const int iters = (cn + ns - 1) / ns;
      const int st_r = active ? st : 0;
      T4* jp = S.jb + st_r;
      const bool top = active && il == nu - 1;
      if constexpr (VJP) {
        // sentinel slots carry no cotangent; their separations fail the test
        const T4* lp = S.jl + st_r;
#pragma unroll 2
        for (int t = 0; t < iters; ++t) {
          const T4 pj = jp[t * ns];
          const T4 lj = t * ns + st_r < cn ? lp[t * ns] : T4{};
          T rx = 0, ry = 0, rz = 0;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const T dx = xi[u] - pj.x, dy = yi[u] - pj.y, dz = zi[u] - pj.z;
            const T r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < (SC ? A.rc2s : A.rc2) && r2 > T(0)) {   // coincident: nothing
              T w1, w2;
              pair_vjp_weights<TAB>(r2, A, S.tab, w1, w2);
              const T lx = lxi[u] - lj.x, ly = lyi[u] - lj.y, lz = lzi[u] - lj.z;
              const T c = w2 * (dx * lx + dy * ly + dz * lz);
              const T tx = w1 * lx + c * dx, ty = w1 * ly + c * dy, tz = w1 * lz + c * dz;
              if constexpr (UM) {
                ax[u] += tx;
                ay[u] += ty;
                az[u] += tz;
                if constexpr (HALF) {
                  rx += tx;
                  ry += ty;
                  rz += tz;
                }
              } else {
                ax[u] += pj.w * tx;
                ay[u] += pj.w * ty;
                az[u] += pj.w * tz;
                if constexpr (HALF) {
                  rx += mi[u] * tx;
                  ry += mi[u] * ty;
                  rz += mi[u] * tz;
                }
              }
            }
          }
          if constexpr (HALF) {
            rx = group_sum_top<NU>(rx);
            ry = group_sum_top<NU>(ry);
            rz = group_sum_top<NU>(rz);
            if (top) {
              T4 o;
              o.x = rx; o.y = ry; o.z = rz; o.w = T(0);
              jp[t * ns] = o;
            }
          }
        }
      } else {
        // RHO (force over the softened-distance table): the squared separation
        // is accumulated on top of eps^2, so the test compares
        // rho^2 = r^2 + eps^2 with r_c^2 + eps^2 and the weight starts from rho^2
        // (FP32: all of it in the scaled units)
        constexpr bool RHO = TAB == 1 && !COUNT;
        const T e2r = sizeof(T) == 4 ? T(A.rho_e2) : T(A.rho_e2d);
        const T cut2 = RHO ? (sizeof(T) == 4 ? T(A.rho_cut2) : T(A.rho_cut2d)) : A.rc2;
        // FP64 reads the next staged j while the current one is tested
        // (measured 3 % faster; FP32 gains nothing and spills more)
        constexpr bool PF = sizeof(T) == 8;
        T4 pn = jp[0];
#pragma unroll 2
        for (int t = 0; t < iters; ++t) {
          T4 pj;
          if constexpr (PF) {
            pj = pn;
            pn = jp[min(t + 1, iters - 1) * ns];
          } else {
            pj = jp[t * ns];
          }
          const T jx = pj.x, jy = pj.y, jz = pj.z;
          T rx = 0, ry = 0, rz = 0;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const T dx = xi[u] - jx, dy = yi[u] - jy, dz = zi[u] - jz;
            T r2;
            if constexpr (RHO) {
              r2 = fma(dx, dx, e2r);
              r2 = fma(dy, dy, r2);
              r2 = fma(dz, dz, r2);
            } else {
              r2 = dx * dx + dy * dy + dz * dz;
            }
            if (r2 < cut2) {
              if (COUNT) {
                npairs += r2 > T(0) ? 1 : 0;
              } else {
                T w;
                if constexpr (RHO)
                  w = pair_weight_rho(r2, A, S.tab);
                else
                  w = pair_weight<TAB>(r2, A, S.tab);
                const T wa = UM ? w : w * pj.w;
                ax[u] += wa * dx;
                ay[u] += wa * dy;
                az[u] += wa * dz;
                if constexpr (HALF) {
                  const T wr = UM ? w : w * mi[u];
                  rx += wr * dx;
                  ry += wr * dy;
                  rz += wr * dz;
                }
              }
            }
          }
          if constexpr (HALF) {
            rx = group_sum_top<NU>(rx);
            ry = group_sum_top<NU>(ry);
            rz = group_sum_top<NU>(rz);
            if (top) {
              T4 o;
              o.x = rx; o.y = ry; o.z = rz; o.w = T(0);
              jp[t * ns] = o;
            }
          }
        }
      }
      if constexpr (HALF) {
        // the chunk's reactions to their partials: each lane its own staged
        // entries (phase 1: those past the item's own chunk, at their
        // position; phase 2: those of runs that take reactions)
        __syncthreads();
        T* px = (T*)A.rpart;
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
          const int q = q0 + e;
          if (q >= cn) continue;
          long long idx = -1;
          if (phase == 1) {
            const int P = staged + c0 + q;
            if (P >= ni) idx = ibase + (P - ni);
          } else {
            const int rp = S.d_rp[dd[e]];
            if (rp >= 0) idx = ibase + rp + (c0 + q - S.d_pre[dd[e]]);
          }
          if (idx >= 0 && idx < ptotal) {    // (always below: a guard only)
            const T4 r = S.jb[q];            // partial idx: 3 components together
            px[3 * idx] = r.x;
            px[3 * idx + 1] = r.y;
            px[3 * idx + 2] = r.z;
          }
        }
      }
    }
    staged += total;
    rstaged += rtotal;
  };

  if constexpr (HALF) {
    run_batch(own_group_runs<T>(S, lane, lgG, G, gz0, ibeg), 1);
    for (int rb = 0; rb < A.nseg; rb += 64)
      run_batch(resolve_segments<T>(A, rb, lane, gx0, gy0, gz0, B), 2);
  } else {
    for (int rb = 0; rb < A.nrows; rb += 64)
      run_batch(resolve_rows<T>(A, A.rows, A.nrows, rb, lane, gx0, gy0, gz0, B), 0);
  }

  if (COUNT) {
    int v = active ? npairs : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0 && v) atomicAdd(A.counter, (unsigned long long)v);
    return;
  }

  // add the stream partials of each i, one slot at a time: red[c][lane]
  // (aliasing the j stage); particle u * nu + q is the sum over streams k of
  // lane k * nu + q's slot u
  T* red = reinterpret_cast<T*>(S.jb);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    __syncthreads();
    red[0 * 64 + lane] = ax[u];
    red[1 * 64 + lane] = ay[u];
    red[2 * 64 + lane] = az[u];
    __syncthreads();
    const int q = u * nu + lane;
    if (lane >= nu || q >= ni) continue;
    T sx = 0, sy = 0, sz = 0;
#pragma unroll 2
    for (int k = 0; k < ns; ++k) {
      sx += red[0 * 64 + k * nu + lane];
      sy += red[1 * 64 + k * nu + lane];
      sz += red[2 * 64 + k * nu + lane];
    }
    const int fi = ibeg + q;
    int run = 0;
    while (run + 1 < GG && S.i_pre[run + 1] <= fi) ++run;
    const int s = S.i_lo[run] + (fi - S.i_pre[run]);
    const double m = (double)A.rec[s].w;
    const double ws = !SC ? A.wscale : (VJP ? A.wscale_vjp : A.wscale_rho);
    double gx = ws * (double)sx, gy = ws * (double)sy, gz = ws * (double)sz;
    if (UM) {
      gx *= m; gy *= m; gz *= m;
    }
    if (A.acc_pm) {
      const T4 pm = A.acc_pm[s];
      gx += (double)pm.x; gy += (double)pm.y; gz += (double)pm.z;
    }
    if (A.acc_out) {            // sorted acceleration, for the mesh part to add to
      T4 o;
      o.x = (T)gx; o.y = (T)gy; o.z = (T)gz; o.w = T(0);
      A.acc_out[s] = o;
      continue;
    }
    const int64_t i = A.perm[s];
    if (A.force_fp32) {
      float* F = (float*)A.force;
      F[i] = (float)(m * gx);
      F[A.n + i] = (float)(m * gy);
      F[2 * A.n + i] = (float)(m * gz);
    } else {
      double* F = (double*)A.force;
      F[i] = m * gx;
      F[A.n + i] = m * gy;
      F[2 * A.n + i] = m * gz;
    }
  }
}

// i-slots per lane: enough that ceil(ni / U) slot sets fit in the wave. The
// one-sided sum rounds the slot sets up to a power of two NU.
template <typename T, bool COUNT, bool UM, int TAB, bool VJP, bool HALF, typename SH>
__device__ __forceinline__ void pair_dispatch(const PairArgs<T>& A, SH& S,
                                              int gx0, int gy0, int gz0, int ibeg, int ni,
                                              int64_t g) {
#define P3M_ITEM(U_, NU_) \
  pair_item<T, U_, COUNT, UM, TAB, VJP, HALF, NU_>(A, S, gx0, gy0, gz0, ibeg, ni, g)
  if constexpr (!HALF) {
    if (ni == 1)
      P3M_ITEM(1, 0);
    else if (sizeof(T) == 8)
      P3M_ITEM(2, 0);
    else if (ni <= 32 || VJP)
      P3M_ITEM(4, 0);
    else
      P3M_ITEM(8, 0);
  } else if constexpr (sizeof(T) == 8) {
    if (ni == 1)
      P3M_ITEM(1, 1);
    else if (ni <= 4)
      P3M_ITEM(2, 2);
    else if (ni <= 8)
      P3M_ITEM(2, 4);
    else if (ni <= 16)
      P3M_ITEM(2, 8);
    else if (ni <= 32)
      P3M_ITEM(2, 16);
    else
      P3M_ITEM(2, 32);
  } else {
    if (ni == 1)
      P3M_ITEM(1, 1);
    else if (ni <= 8)
      P3M_ITEM(4, 2);
    else if (ni <= 16)
      P3M_ITEM(4, 4);
    else if (ni <= 32)
      P3M_ITEM(4, 8);
    else if constexpr (!VJP)
      P3M_ITEM(8, 8);
    else
      P3M_ITEM(4, 16);
  }
#undef P3M_ITEM
}

template <typename T, bool COUNT, bool UM, int TAB, bool VJP = false, bool HALF = false>
__global__ void __launch_bounds__(64, (kPairWaves<T, VJP>))
k_pairs(PairArgs<T> A) {
  __shared__ PairShared<T, VJP, HALF> S;
  const int lane = threadIdx.x;
  // Items in group order, dealt round-robin over the XCDs by the hardware:
  // the eight XCDs then work on neighbouring groups at the same time, which
  // measured faster than giving each XCD its own slab of the box.
  const int item = (int)blockIdx.x;
  if (item >= *A.n_items) return;
  const int2 it = A.items[item];
  const int lg = A.lg, lgG = A.lgG, G = A.G, GG = G * G;
  const int lgd = lg - lgG, md = (1 << lgd) - 1;
  const int gx0 = (it.x >> (2 * lgd)) << lgG;
  const int gy0 = ((it.x >> lgd) & md) << lgG;
  const int gz0 = (it.x & md) << lgG;

  if (!COUNT) {                        // split-factor table into LDS
    T* tab = &S.tab.c[0][0];
    for (int e = lane; e < SplitTable<T>::kCoef * kTabStride; e += 64) tab[e] = A.split_tab[e];
  }
  // i side: the group's G*G z-runs
  {
    int cnt = 0;
    if (lane < GG) {
      int a = lane >> lgG, b = lane & (G - 1);
      int c0 = ((((gx0 + a) << lg) | (gy0 + b)) << lg) | gz0;
      int lo = A.start[c0];
      S.i_lo[lane] = lo;
      cnt = A.start[c0 + G] - lo;
    }
    int inc = wave_inclusive(cnt);
    if (lane < GG) S.i_pre[lane + 1] = inc;
    if (lane == 0) S.i_pre[0] = 0;
  }
  __syncthreads();
  // wave-uniform counts (scalar registers, so the loops are scalar)
  const int ntot = __builtin_amdgcn_readfirstlane(S.i_pre[GG]);
  const int ibeg = it.y * kChunk;
  const int ni = min(kChunk, ntot - ibeg);
  // the one-sided sum for an item of a dense group, unless the partials
  // exceed the plan's capacity this call (then every pair from both sides,
  // as in a plan without partials); items of sparse groups from both sides
  if (HALF && ntot > kDenseMin && *A.gtotal <= A.rcap)
    pair_dispatch<T, COUNT, UM, TAB, VJP, true>(A, S, gx0, gy0, gz0, ibeg, ni, it.x);
  else
    pair_dispatch<T, COUNT, UM, TAB, VJP, false>(A, S, gx0, gy0, gz0, ibeg, ni, it.x);
}

// Grid of the pair kernel: the item bound rounded up to a multiple of kXcds.
unsigned pair_grid(const p3m_plan* P) {
  return (unsigned)((P->max_items + kXcds - 1) / kXcds * kXcds);
}

template <typename T>
PairArgs<T> make_args(p3m_plan* P, int64_t n) {
  Workspace& W = P->ws;
  PairArgs<T> A{};
  A.rec = (const typename Vec<T>::v4*)W.rec;
  A.skey = W.skey;
  A.start = W.start;
  A.items = W.items;
  A.n_items = W.goff + P->ngroup;
  A.rows = W.rows;
  A.nrows = P->nrows;
  A.ng = P->ng;
  A.lg = P->lg;
  A.G = P->G;
  A.lgG = P->lgG;
  A.h = (T)P->h;
  A.rc2 = (T)(P->r_c * P->r_c);
  A.eps2 = (T)(P->eps * P->eps);
  A.inv2rs = (T)(1.0 / (2.0 * P->r_s));
  A.wscale = -P->prm.G;
  if constexpr (sizeof(T) == 8) {
    const double s = kSplitBins / (P->tab64_v1 - P->tab64_v0);
    A.split_tab = W.split_tab64;
    A.tab_s64 = s;
    A.tab_off64 = s * P->tab64_v0;
    A.rho_e2d = std::max(s * s * P->eps * P->eps, 1e-100);
    A.rho_cut2d = s * s * P->r_c * P->r_c + A.rho_e2d;
    A.rho_inv2rs = 1.0 / (2.0 * P->r_s * s);
    A.wscale_rho = -P->prm.G * s * s;
    A.wscale_vjp = -P->prm.G * s * s * s;
    A.rc2s = s * s * P->r_c * P->r_c;
    A.tab_exact = P->tab64_exact;
  }
  if constexpr (sizeof(T) == 4) {
    const double s = kSplitBins / (P->tab_v1 - P->tab_v0);
    A.split_tab = W.split_tab;
    A.tab_s = (float)s;
    A.tab_s2 = (float)(s * s);
    A.tab_e2 = (float)std::max(s * s * P->eps * P->eps, 1e-12);
    A.tab_off = (float)(s * P->tab_v0);
    A.rho_e2 = A.tab_e2;
    A.rho_cut2 = (float)(s * s * P->r_c * P->r_c + (double)A.tab_e2);
    A.wscale_rho = A.wscale * s * s;
    A.wscale_vjp = A.wscale * s * s * s;
    A.rc2s = (float)(s * s * P->r_c * P->r_c);
    A.wscale *= s * s * s;
    A.vjp_k5 = (T)(3.0 * s * s);
    A.vjp_e2 = (T)(-1.4426950408889634 / (4.0 * P->r_s * P->r_s));
  } else {
    A.vjp_k5 = T(3);
  }
  const double ce = 1.0 / (2.0 * 1.7724538509055160 * P->r_s * P->r_s * P->r_s);
  const double s_tab = sizeof(T) == 4 ? kSplitBins / (P->tab_v1 - P->tab_v0)
                                      : kSplitBins / (P->tab64_v1 - P->tab64_v0);
  A.vjp_ce = (T)ce;
  A.vjp_ce_s = (T)(ce / (s_tab * s_tab * s_tab));
  A.perm = W.perm;
  A.n = n;
  A.segrows = W.segrows;
  A.nseg = P->nseg;
  A.npos = P->npos;
  A.gntot = W.gntot;
  A.rowoff = W.rowoff;
  A.gbase = W.gbase;
  A.gtotal = W.gbase ? W.gbase + P->ngroup : nullptr;
  A.rpart = W.rpart;
  A.rcap = P->rcap;
  return A;
}

// Scale of the pair kernel's sorted output (times the mass when all masses
// are equal): the reaction partials enter the gather with its negative.
template <typename T>
double out_scale(const PairArgs<T>& A, int tab, bool vjp) {
  return tab != 1 ? A.wscale : (vjp ? A.wscale_vjp : A.wscale_rho);
}

}  // namespace

template <typename T, bool VJP>
hipError_t launch_pair_kernel(p3m_plan* P, const PairArgs<T>& A, bool uniform_mass, bool half) {
  const unsigned grid = pair_grid(P);
  const bool tab = (sizeof(T) == 4 ? P->tab_var : P->tab64_var) == 1;
  // table over the softened distance (1) or over r (0)
  if (half) {
    if (tab) {
      if (uniform_mass)
        k_pairs<T, false, true, 1, VJP, true><<<grid, 64, 0, P->stream>>>(A);
      else
        k_pairs<T, false, false, 1, VJP, true><<<grid, 64, 0, P->stream>>>(A);
    } else {
      if (uniform_mass)
        k_pairs<T, false, true, 0, VJP, true><<<grid, 64, 0, P->stream>>>(A);
      else
        k_pairs<T, false, false, 0, VJP, true><<<grid, 64, 0, P->stream>>>(A);
    }
    return hipGetLastError();
  }
  if (tab) {
    if (uniform_mass)
      k_pairs<T, false, true, 1, VJP><<<grid, 64, 0, P->stream>>>(A);
    else
      k_pairs<T, false, false, 1, VJP><<<grid, 64, 0, P->stream>>>(A);
  } else {
    if (uniform_mass)
      k_pairs<T, false, true, 0, VJP><<<grid, 64, 0, P->stream>>>(A);
    else
      k_pairs<T, false, false, 0, VJP><<<grid, 64, 0, P->stream>>>(A);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pairs(p3m_plan* P, int64_t n, bool add_pm, void* force_out, int force_fp32,
                        bool uniform_mass, void* acc_out) {
  PairArgs<T> A = make_args<T>(P, n);
  if (P->rcap > 0 && !add_pm) {
    // one-sided sum: the sorted action into ws.acc_pm; launch_pair_gather
    // then adds the reactions and writes the result
    A.acc_out = (typename Vec<T>::v4*)P->ws.acc_pm;
    return launch_pair_kernel<T, false>(P, A, uniform_mass, true);
  }
  A.acc_pm = add_pm ? (const typename Vec<T>::v4*)P->ws.acc_pm : nullptr;
  A.acc_out = (typename Vec<T>::v4*)acc_out;
  A.force = force_out;
  A.force_fp32 = force_fp32;
  return launch_pair_kernel<T, false>(P, A, uniform_mass, false);
}

template <typename T>
hipError_t launch_pairs_vjp(p3m_plan* P, int64_t n, bool add_pm, double* pos_bar,
                            bool uniform_mass, void* acc_out) {
  PairArgs<T> A = make_args<T>(P, n);
  A.lam = (const typename Vec<T>::v4*)P->ws.lam;
  if (P->rcap > 0 && !add_pm) {
    A.acc_out = (typename Vec<T>::v4*)P->ws.acc_pm;
    return launch_pair_kernel<T, true>(P, A, uniform_mass, true);
  }
  A.acc_pm = add_pm ? (const typename Vec<T>::v4*)P->ws.acc_pm : nullptr;
  A.acc_out = (typename Vec<T>::v4*)acc_out;
  A.force = pos_bar;
  A.force_fp32 = 0;
  return launch_pair_kernel<T, true>(P, A, uniform_mass, false);
}

template <typename T>
hipError_t launch_pair_gather(p3m_plan* P, int64_t n, bool vjp, bool uniform_mass,
                              void* acc_out, void* out, int out_fp32, const void* acc_add) {
  const PairArgs<T> A = make_args<T>(P, n);
  const int tab = sizeof(T) == 4 ? P->tab_var : P->tab64_var;
  return launch_react_gather<T>(P, n, -out_scale(A, tab, vjp), uniform_mass, acc_out, out,
                                out_fp32, acc_add);
}

template <typename T>
hipError_t launch_pair_count(p3m_plan* P, int64_t n, int64_t* count_out) {
  PairArgs<T> A = make_args<T>(P, n);
  A.counter = (unsigned long long*)count_out;
  hipError_t e = launch_fill_i32((int32_t*)count_out, 2, 0, P->stream);
  if (e != hipSuccess) return e;
  k_pairs<T, true, true, 0><<<pair_grid(P), 64, 0, P->stream>>>(A);
  return hipGetLastError();
}

template hipError_t launch_pairs<float>(p3m_plan*, int64_t, bool, void*, int, bool, void*);
template hipError_t launch_pairs<double>(p3m_plan*, int64_t, bool, void*, int, bool, void*);
template hipError_t launch_pairs_vjp<float>(p3m_plan*, int64_t, bool, double*, bool, void*);
template hipError_t launch_pairs_vjp<double>(p3m_plan*, int64_t, bool, double*, bool, void*);
template hipError_t launch_pair_gather<float>(p3m_plan*, int64_t, bool, bool, void*, void*,
                                               int, const void*);
template hipError_t launch_pair_gather<double>(p3m_plan*, int64_t, bool, bool, void*, void*,
                                                int, const void*);
template hipError_t launch_pair_count<float>(p3m_plan*, int64_t, int64_t*);
template hipError_t launch_pair_count<double>(p3m_plan*, int64_t, int64_t*);

}  // namespace p3m
