// Brick decomposition shared by the mesh kernels (deposit, interpolation and
// their adjoints): a workgroup owns a brick of kBrick^3 cells, finds its
// particles as kBrick^2 z-runs of the sorted cell list, and touches
// (kBrick + 1)^3 nodes (plus a two-node halo for the gradient).
#pragma once

#include "p3m_internal.h"

namespace p3m {
namespace brick {

constexpr int kThreads = 256;
constexpr int kRows = kBrick * kBrick;      // (cx, cy) columns of a brick
constexpr int kN1 = kBrick + 1;             // nodes per axis touched by a brick
constexpr int kN5 = kBrick + 5;             // nodes per axis with the gradient halo

// Column table of a brick: first slot and exclusive prefix of the particle
// counts of its kRows z-runs (each run = kBrick cells of one column).
struct BrickRuns {
  int lo[kRows];
  int pre[kRows + 1];
};

__device__ inline void load_runs(BrickRuns& R, const int32_t* __restrict__ start, int lg, int bx0,
                          int by0, int bz0) {
  const int t = threadIdx.x;
  if (t < kRows) {
    int cx = bx0 + t / kBrick, cy = by0 + t % kBrick;
    int c0 = (((cx << lg) | cy) << lg) | bz0;
    int lo = start[c0];
    R.lo[t] = lo;
    R.pre[t + 1] = start[c0 + kBrick] - lo;      // count, prefix-summed below
  }
  __syncthreads();
  if (t < 64) {                                   // one wave scans the kRows counts
    int v = (t < kRows) ? R.pre[t + 1] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int u = __shfl_up(v, o, 64);
      if (t >= o) v += u;
    }
    if (t < kRows) R.pre[t + 1] = v;
    if (t == 0) R.pre[0] = 0;
  }
  __syncthreads();
}

// Run index r with R.pre[r] <= f < R.pre[r+1].
__device__ __forceinline__ int find_run(const BrickRuns& R, int f) {
  int lo = 0, hi = kRows;                         // invariant: pre[lo] <= f < pre[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (R.pre[mid] <= f) lo = mid; else hi = mid;
  }
  return lo;
}

// Interpolation bricks of BX x BX x BZ cells: BX^2 z-runs of BZ cells each.
// A deeper brick along z makes a wave's particles longer runs of consecutive
// cells, so that for inputs stored in cell-like order (a lattice) the
// per-particle stores in input order fill longer pieces of cache lines.
template <int BX, int BZ>
struct InterpRuns {
  static constexpr int kR = BX * BX;
  int lo[kR];
  int pre[kR + 1];
};

template <int BX, int BZ>
__device__ inline void load_interp_runs(InterpRuns<BX, BZ>& R, const int32_t* __restrict__ start,
                                        int lg, int bx0, int by0, int bz0) {
  constexpr int kR = InterpRuns<BX, BZ>::kR;
  static_assert(kR <= 64, "one wave scans the run counts");
  const int t = threadIdx.x;
  if (t < kR) {
    int cx = bx0 + t / BX, cy = by0 + t % BX;
    int c0 = (((cx << lg) | cy) << lg) | bz0;
    int lo = start[c0];
    R.lo[t] = lo;
    R.pre[t + 1] = start[c0 + BZ] - lo;           // c0 + BZ <= ng^3: start has ng^3 + 1
  }
  __syncthreads();
  if (t < 64) {
    int v = (t < kR) ? R.pre[t + 1] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int u = __shfl_up(v, o, 64);
      if (t >= o) v += u;
    }
    if (t < kR) R.pre[t + 1] = v;
    if (t == 0) R.pre[0] = 0;
  }
  __syncthreads();
}

template <int BX, int BZ>
__device__ __forceinline__ int find_interp_run(const InterpRuns<BX, BZ>& R, int f) {
  int lo = 0, hi = InterpRuns<BX, BZ>::kR;        // invariant: pre[lo] <= f < pre[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (R.pre[mid] <= f) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace brick
}  // namespace p3m
