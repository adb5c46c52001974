// Short-range pair sum of P3M over the sorted cell list.
//
//   a_i = -G sum_{j != i, 0 < r < r_c} m_j r_ij f(r) / (r^2 + eps^2)^(3/2)
//   f(r) = erfc(u) + (2u / sqrt(pi)) exp(-u^2),  u = r / (2 r_s)
//
// Work decomposition. The grid's cells are grouped into i-groups of G^3
// cells; a work item is (group, chunk) with up to 64 of the group's
// particles, one wavefront per item. The j-candidates of a group are the
// particles of every cell whose box comes closer than r_c to the group's box
// (the stencil rows: z-runs of cells, precomputed per plan). With n_i
// i-particles the 64 lanes form n_i x s lanes (s = 64 / n_i "streams"): lane
// (i, stream) takes every s-th staged j, so small groups still fill the wave,
// and the s partial sums of each i are added at the end.
//
// Per batch of 64 stencil rows: each lane resolves one row into at most three
// contiguous sorted runs (the z-run split where it crosses the periodic box
// face), a wave scan flattens them, and the wave stages the runs' particles
// into LDS (kPairCap at a time) as positions relative to the group's first
// cell, carrying the periodic shift of the run. Positions are rebuilt from the
// cell-relative offsets and small integer cell differences, so the FP32 path
// never subtracts two large coordinates.
//
// FP32 evaluation: rsq(r^2 + eps^2), sqrt(r^2), exp(-u^2), and erfc(u) from
// the Abramowitz & Stegun 7.1.26 rational form t P(t) exp(-u^2),
// t = 1/(1 + p u) (absolute error <= 1.5e-7), sharing the exponential.
// FP64 evaluation: the device library's erfc, exp, sqrt and rsqrt.
#include "p3m_internal.h"

namespace p3m {
namespace {

constexpr int kDesc = 3 * 64;       // runs per batch of 64 rows
constexpr int kStage = kPairCap / 64;  // consecutive staged entries per lane
template <typename T>
constexpr int kUnroll = sizeof(T) == 4 ? 4 : 2;  // staged j read ahead per lane
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
  T h, rc2, eps2, inv2rs, negG;
  const typename Vec<T>::v4* __restrict__ acc_pm;  // sorted PM acceleration or null
  const int32_t* __restrict__ perm;
  int64_t n;
  void* __restrict__ force;
  int force_fp32;
  unsigned long long* __restrict__ counter;      // pair count mode
};

// f(r) / (r^2 + eps^2)^(3/2) for 0 < r2.
__device__ __forceinline__ float pair_weight(float r2, float eps2, float inv2rs) {
  const float kP = 0.3275911f;
  const float kA1 = 0.254829592f, kA2 = -0.284496736f, kA3 = 1.421413741f,
              kA4 = -1.453152027f, kA5 = 1.061405429f;
  const float kTwoOverSqrtPi = 1.1283791670955126f;
  const float kNegLog2e = -1.4426950408889634f;
  float inv = __builtin_amdgcn_rsqf(r2 + eps2);
  float inv3 = inv * inv * inv;
  float r = __builtin_amdgcn_sqrtf(r2);
  float u = r * inv2rs;
  float e = __builtin_amdgcn_exp2f(u * u * kNegLog2e);
  float t = __builtin_amdgcn_rcpf(1.0f + kP * u);
  float poly = t * (kA1 + t * (kA2 + t * (kA3 + t * (kA4 + t * kA5))));
  float f = e * (poly + kTwoOverSqrtPi * u);
  return f * inv3;
}

__device__ __forceinline__ double pair_weight(double r2, double eps2, double inv2rs) {
  const double kTwoOverSqrtPi = 1.1283791670955126;
  double inv = rsqrt(r2 + eps2);
  double r = sqrt(r2);
  double u = r * inv2rs;
  double f = erfc(u) + kTwoOverSqrtPi * u * exp(-u * u);
  return f * (inv * inv * inv);
}

// Largest d with pre[d] <= f (pre non-decreasing, pre[0] = 0 <= f < pre[kDesc]).
__device__ __forceinline__ int find_desc(const int* __restrict__ pre, int f) {
  int lo = 0, hi = kDesc;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pre[mid] <= f) lo = mid; else hi = mid;
  }
  return lo;
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

template <typename T, bool COUNT>
__global__ void __launch_bounds__(64) k_pairs(PairArgs<T> A) {
  using T4 = typename Vec<T>::v4;
  __shared__ T4 jb[kPairCap + 1];     // + the far sentinel
  __shared__ int d_lo[kDesc], d_pre[kDesc + 1], d_zs[kDesc];
  __shared__ T d_sx[64], d_sy[64];
  __shared__ int i_lo[16], i_pre[17];
  __shared__ T red[3][64];

  const int lane = threadIdx.x;
  if ((int)blockIdx.x >= *A.n_items) return;
  const int2 it = A.items[blockIdx.x];
  const int lg = A.lg, ng = A.ng, mask = ng - 1, lgG = A.lgG, G = A.G, GG = G * G;
  const int lgd = lg - lgG, md = (1 << lgd) - 1;
  const int gx0 = (it.x >> (2 * lgd)) << lgG;
  const int gy0 = ((it.x >> lgd) & md) << lgG;
  const int gz0 = (it.x & md) << lgG;
  const T h = A.h;

  // i side: the group's G*G z-runs
  {
    int cnt = 0;
    if (lane < GG) {
      int a = lane >> lgG, b = lane & (G - 1);
      int c0 = ((((gx0 + a) << lg) | (gy0 + b)) << lg) | gz0;
      int lo = A.start[c0];
      i_lo[lane] = lo;
      cnt = A.start[c0 + G] - lo;
    }
    int inc = wave_inclusive(cnt);
    if (lane < GG) i_pre[lane + 1] = inc;
    if (lane == 0) i_pre[0] = 0;
  }
  __syncthreads();
  // wave-uniform counts (scalar registers, so the loops below are scalar)
  const int ntot = __builtin_amdgcn_readfirstlane(i_pre[GG]);
  const int ibeg = it.y * 64;
  const int ni = min(64, ntot - ibeg);
  const int ns = 64 / ni;
  const int il = lane % ni, st = lane / ni;
  const bool active = st < ns;
  int run = 0;
  const int fi = ibeg + il;
  while (run + 1 < GG && i_pre[run + 1] <= fi) ++run;
  const int si = i_lo[run] + (fi - i_pre[run]);
  const T4 pi = A.rec[si];
  const int czi = A.skey[si] & mask;
  const T xi = active ? T(run >> lgG) * h + pi.x : kFar;
  const T yi = active ? T(run & (G - 1)) * h + pi.y : kFar;
  const T zi = active ? T(czi - gz0) * h + pi.z : kFar;

  T ax = 0, ay = 0, az = 0;
  int npairs = 0;

  for (int rb = 0; rb < A.nrows; rb += 64) {
    // resolve one stencil row per lane into up to three sorted runs
    int cnt[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, zs[3] = {0, 0, 0};
    T sx = 0, sy = 0;
    if (rb + lane < A.nrows) {
      const int4 row = A.rows[rb + lane];
      const int jx = (gx0 + row.x) & mask, jy = (gy0 + row.y) & mask;
      sx = T(row.x) * h;
      sy = T(row.y) * h;
      const int zhi = gz0 + row.w;
      int z = gz0 + row.z;
      const int cbase = ((jx << lg) | jy) << lg;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (z <= zhi) {
          int zw = z & mask;
          int len = min(zhi - z + 1, ng - zw);
          int l0 = A.start[cbase + zw];
          lo[k] = l0;
          cnt[k] = A.start[cbase + zw + len] - l0;
          zs[k] = (z - zw) - gz0;
          z += len;
        }
      }
    }
    __syncthreads();       // previous batch is done with the descriptors and jb
    const int tot_l = cnt[0] + cnt[1] + cnt[2];
    const int inc = wave_inclusive(tot_l);
    int base = inc - tot_l;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d_lo[3 * lane + k] = lo[k];
      d_pre[3 * lane + k] = base;
      d_zs[3 * lane + k] = zs[k];
      base += cnt[k];
    }
    d_sx[lane] = sx;
    d_sy[lane] = sy;
    const int total = __builtin_amdgcn_readfirstlane(__shfl(inc, 63, 64));
    if (lane == 63) d_pre[kDesc] = total;
    __syncthreads();

    for (int c0 = 0; c0 < total; c0 += kPairCap) {
      const int cn = min(kPairCap, total - c0);
      if (c0 > 0) __syncthreads();
      // stage entries [kStage*lane, kStage*lane + kStage) of this chunk: one
      // search for the first, a short forward walk for the rest, then all
      // loads in flight together
      {
        const int q0 = kStage * lane;
        int src[kStage], dd[kStage];
        int d = q0 < cn ? find_desc(d_pre, c0 + q0) : 0;
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
          const int f = c0 + q0 + e;
          if (q0 + e < cn)
            while (d_pre[d + 1] <= f) ++d;
          dd[e] = d;
          src[e] = q0 + e < cn ? d_lo[d] + (f - d_pre[d]) : -1;
        }
        T4 pj[kStage];
        int cz[kStage];
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
          if (src[e] >= 0) {
            pj[e] = A.rec[src[e]];
            cz[e] = A.skey[src[e]] & mask;
          }
        }
#pragma unroll
        for (int e = 0; e < kStage; ++e) {
          if (src[e] >= 0) {
            const int d = dd[e];
            T4 o;
            o.x = d_sx[d / 3] + pj[e].x;
            o.y = d_sy[d / 3] + pj[e].y;
            o.z = T(cz[e] + d_zs[d]) * h + pj[e].z;
            o.w = pj[e].w;
            jb[q0 + e] = o;
          }
        }
      }
      if (lane == 0) {                 // a far-away sentinel after the last entry
        T4 far;
        far.x = far.y = far.z = -kFar;
        far.w = T(0);
        jb[cn] = far;
      }
      __syncthreads();
      // lane (il, st) takes staged entries st, st + ns, ...; the trip count is
      // wave-uniform; reads past the end hit the sentinel, and lanes without
      // an i sit at +kFar, so both fail the cutoff test
      const int iters = (cn + ns - 1) / ns;
      for (int t0 = 0; t0 < iters; t0 += kUnroll<T>) {
        T4 pj[kUnroll<T>];
#pragma unroll
        for (int u = 0; u < kUnroll<T>; ++u) pj[u] = jb[min(st + (t0 + u) * ns, cn)];
#pragma unroll
        for (int u = 0; u < kUnroll<T>; ++u) {
          const T dx = xi - pj[u].x, dy = yi - pj[u].y, dz = zi - pj[u].z;
          const T r2 = dx * dx + dy * dy + dz * dz;
          if (r2 < A.rc2) {
            if (COUNT) {
              npairs += r2 > T(0) ? 1 : 0;
            } else {
              T w = pj[u].w * pair_weight(r2, A.eps2, A.inv2rs);
              w = r2 > T(0) ? w : T(0);      // zero separation: no contribution
              ax += w * dx;
              ay += w * dy;
              az += w * dz;
            }
          }
        }
      }
    }
  }

  if (COUNT) {
    int v = active ? npairs : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0 && v) atomicAdd(A.counter, (unsigned long long)v);
    return;
  }

  // add the stream partials of each i
  red[0][lane] = ax;
  red[1][lane] = ay;
  red[2][lane] = az;
  __syncthreads();
  if (lane < ni) {
    T sx = 0, sy = 0, sz = 0;
    for (int k = 0; k < ns; ++k) {
      sx += red[0][lane + k * ni];
      sy += red[1][lane + k * ni];
      sz += red[2][lane + k * ni];
    }
    T gx = A.negG * sx, gy = A.negG * sy, gz = A.negG * sz;
    if (A.acc_pm) {
      const T4 pm = A.acc_pm[si];
      gx += pm.x; gy += pm.y; gz += pm.z;
    }
    const int64_t i = A.perm[si];
    const double m = (double)pi.w;
    if (A.force_fp32) {
      float* F = (float*)A.force;
      F[i] = (float)(m * (double)gx);
      F[A.n + i] = (float)(m * (double)gy);
      F[2 * A.n + i] = (float)(m * (double)gz);
    } else {
      double* F = (double*)A.force;
      F[i] = m * (double)gx;
      F[A.n + i] = m * (double)gy;
      F[2 * A.n + i] = m * (double)gz;
    }
  }
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
  A.negG = (T)(-P->prm.G);
  A.perm = W.perm;
  A.n = n;
  return A;
}

}  // namespace

template <typename T>
hipError_t launch_pairs(p3m_plan* P, int64_t n, bool add_pm, void* force_out, int force_fp32) {
  PairArgs<T> A = make_args<T>(P, n);
  A.acc_pm = add_pm ? (const typename Vec<T>::v4*)P->ws.acc_pm : nullptr;
  A.force = force_out;
  A.force_fp32 = force_fp32;
  k_pairs<T, false><<<(unsigned)P->max_items, 64, 0, P->stream>>>(A);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pair_count(p3m_plan* P, int64_t n, int64_t* count_out) {
  PairArgs<T> A = make_args<T>(P, n);
  A.counter = (unsigned long long*)count_out;
  hipError_t e = launch_fill_i32((int32_t*)count_out, 2, 0, P->stream);
  if (e != hipSuccess) return e;
  k_pairs<T, true><<<(unsigned)P->max_items, 64, 0, P->stream>>>(A);
  return hipGetLastError();
}

template hipError_t launch_pairs<float>(p3m_plan*, int64_t, bool, void*, int);
template hipError_t launch_pairs<double>(p3m_plan*, int64_t, bool, void*, int);
template hipError_t launch_pair_count<float>(p3m_plan*, int64_t, int64_t*);
template hipError_t launch_pair_count<double>(p3m_plan*, int64_t, int64_t*);

}  // namespace p3m
