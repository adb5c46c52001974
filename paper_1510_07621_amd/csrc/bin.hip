// Counting-sort binning of particles into the cells of the PM grid, and the
// work list of the pair loop.
//
// Cells are the grid's own cells (side h = box / grid_n), indexed
// c = (cx * ng + cy) * ng + cz (z fastest), so each (cx, cy) column of cells is
// one contiguous run of particles after sorting. Steps:
//   1. keys + histogram: cell of each particle; atomic count per cell, whose
//      return value is the particle's rank inside the cell;
//   2. exclusive scan of the counts -> first slot of every cell;
//   3. scatter + pack: each particle goes to slot start[c] + rank as a record
//      of its offset from the cell's lower corner (in the path's precision)
//      and its mass, with its input index (perm) and cell (skey).
// The order inside a cell follows the atomic ranks, so it can differ between
// runs; every later step is a sum, so only rounding depends on it.
#include "p3m_internal.h"

namespace p3m {
namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 8;                       // per thread
constexpr int kScanTile = kThreads * kScanItems;    // per block
static_assert(kScanItems == 8, "k_scan_tiles moves a thread's values as two int4");

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// Cell coordinate of t = x / h, clamped into [0, ng) (NaN -> 0).
__device__ __forceinline__ int cell_coord(double t, int ng) {
  t = fmax(floor(t), 0.0);
  t = fmin(t, (double)(ng - 1));
  return (int)t;
}

// Consecutive lanes of a wave in the same cell (input already in cell order,
// as a caller that keeps its particles in the order of the last binning
// hands it) share one atomic: the run's first lane adds the run's length
// and each lane's rank is the old count plus its place in the run. With
// input in random order every lane is a run of one.
__global__ void __launch_bounds__(256)
k_bin_count(int64_t n, const double* __restrict__ pos, int ng, int lg, double inv_h,
            int32_t* __restrict__ key, int32_t* __restrict__ rank,
            int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  int c = -1;
  if (valid) {
    int cx = cell_coord(pos[i] * inv_h, ng);
    int cy = cell_coord(pos[n + i] * inv_h, ng);
    int cz = cell_coord(pos[2 * n + i] * inv_h, ng);
    c = (((cx << lg) | cy) << lg) | cz;
    key[i] = c;
  }
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(c, 1, 64);
  const bool head = valid && (lane == 0 || prev != c);
  const unsigned long long heads = __ballot(head);
  // runs end at the next head or at the first lane past n
  const unsigned long long bounds = heads | ~__ballot(valid);
  const unsigned long long upto = lane == 63 ? ~0ull : (2ull << lane) - 1;
  const int start = valid ? 63 - __builtin_clzll(heads & upto) : lane;
  int base = 0;
  if (head) {
    const unsigned long long above = lane == 63 ? 0ull : bounds >> (lane + 1);
    const int len = above ? __builtin_ctzll(above) + 1 : 64 - lane;
    base = atomicAdd(&count[c], len);
  }
  base = __shfl(base, start, 64);
  if (valid) rank[i] = base + (lane - start);
}

template <typename T>
__global__ void k_scatter(int64_t n, const double* __restrict__ pos,
                          const double* __restrict__ mass, double mass_scalar, int ng,
                          int lg, double h, const int32_t* __restrict__ key,
                          const int32_t* __restrict__ rank,
                          const int32_t* __restrict__ start, int32_t* __restrict__ perm,
                          int32_t* __restrict__ skey, typename Vec<T>::v4* __restrict__ rec) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = key[i];
  int dst = start[c] + rank[i];
  int mask = ng - 1;
  int cz = c & mask, cy = (c >> lg) & mask, cx = c >> (2 * lg);
  typename Vec<T>::v4 r;
  r.x = (T)(pos[i] - cx * h);
  r.y = (T)(pos[n + i] - cy * h);
  r.z = (T)(pos[2 * n + i] - cz * h);
  r.w = (T)(mass ? mass[i] : mass_scalar);
  rec[dst] = r;
  perm[dst] = (int32_t)i;
  skey[dst] = c;
}

// ---- exclusive scan of int32 (three kernels: tiles, tile sums, add) ----

__device__ __forceinline__ int wave_inclusive(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan of one value per thread over the block; returns the block total.
__device__ __forceinline__ int block_exclusive(int v, int* __restrict__ wsum, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int inc = wave_inclusive(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int base = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    int s = wsum[k];
    if (k < w) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

// ZERO: the input is cleared as it is read (the cell counts, so that the
// next binning starts from zero without a fill pass).
template <bool ZERO>
__global__ void __launch_bounds__(kThreads)
k_scan_tiles(int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t len,
             int32_t* __restrict__ tile_sum) {
  __shared__ int wsum[kThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  // a thread's kScanItems values are 32-byte aligned (in and out are device
  // allocations): whole slices move as two int4, the ragged end one by one
  const bool whole = base + kScanItems <= len;
  int v[kScanItems];
  if (whole) {
    const int4 a = reinterpret_cast<const int4*>(in + base)[0];
    const int4 b = reinterpret_cast<const int4*>(in + base)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    if (ZERO) {
      reinterpret_cast<int4*>(in + base)[0] = int4{0, 0, 0, 0};
      reinterpret_cast<int4*>(in + base)[1] = int4{0, 0, 0, 0};
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < len) ? in[base + k] : 0;
    if (ZERO) {
#pragma unroll
      for (int k = 0; k < kScanItems; ++k)
        if (base + k < len) in[base + k] = 0;
    }
  }
  int local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) local += v[k];
  int total;
  int run = block_exclusive(local, wsum, total);
  int e[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    e[k] = run;
    run += v[k];
  }
  if (whole) {
    reinterpret_cast<int4*>(out + base)[0] = int4{e[0], e[1], e[2], e[3]};
    reinterpret_cast<int4*>(out + base)[1] = int4{e[4], e[5], e[6], e[7]};
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
      if (base + k < len) out[base + k] = e[k];
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Single block: exclusive scan of the tile sums in place; writes the grand
// total to *grand.
__global__ void __launch_bounds__(1024)
k_scan_sums(int32_t* __restrict__ sums, int nt, int32_t* __restrict__ grand) {
  __shared__ int wsum[1024 / 64];
  int carry = 0;
  for (int b = 0; b < nt; b += blockDim.x) {
    int i = b + threadIdx.x;
    int v = i < nt ? sums[i] : 0;
    int total;
    int ex = block_exclusive(v, wsum, total);
    if (i < nt) sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *grand = carry;
}

// Whole tiles as int4 (consecutive threads, consecutive 16 bytes), the
// ragged last tile one value at a time.
__global__ void __launch_bounds__(kThreads)
k_scan_add(int32_t* __restrict__ out, int64_t len, const int32_t* __restrict__ tile_off) {
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int add = tile_off[blockIdx.x];
  if (base + kScanTile <= len) {
    int4* o = reinterpret_cast<int4*>(out + base);
    for (int k = threadIdx.x; k < kScanTile / 4; k += kThreads) {
      int4 q = o[k];
      q.x += add; q.y += add; q.z += add; q.w += add;
      o[k] = q;
    }
    return;
  }
  for (int k = threadIdx.x; k < kScanTile; k += kThreads) {
    int64_t i = base + k;
    if (i < len) out[i] += add;
  }
}

// ---- pair-loop work list ----

// Chunks of one i-group: its particles (G x G z-runs of G cells) over kChunk.
__device__ __forceinline__ int group_chunks(const int32_t* __restrict__ start, int lg, int G,
                                            int lgG, int64_t g) {
  const int lgd = lg - lgG, md = (1 << lgd) - 1;
  int gz = (int)(g & md), gy = (int)((g >> lgd) & md), gx = (int)(g >> (2 * lgd));
  int cnt = 0;
  for (int a = 0; a < G; ++a)
    for (int b = 0; b < G; ++b) {
      int c0 = ((((gx * G + a) << lg) | (gy * G + b)) << lg) | (gz * G);
      cnt += start[c0 + G] - start[c0];
    }
  return (cnt + kChunk - 1) / kChunk;
}

// Work list, pass 1: chunk counts of a tile of kThreads groups (one per
// thread), their exclusive scan within the tile (goff) and the tile total.
__global__ void __launch_bounds__(kThreads)
k_items_tiles(const int32_t* __restrict__ start, int lg, int G, int lgG, int64_t ngroup,
              int32_t* __restrict__ gchunk, int32_t* __restrict__ goff,
              int32_t* __restrict__ tile_sum) {
  __shared__ int wsum[kThreads / 64];
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int v = g < ngroup ? group_chunks(start, lg, G, lgG, g) : 0;
  int total;
  const int ex = block_exclusive(v, wsum, total);
  if (g < ngroup) {
    gchunk[g] = v;
    goff[g] = ex;
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Pass 3 (after the tile sums are scanned): each group's items at its offset.
__global__ void __launch_bounds__(kThreads)
k_emit_items(const int32_t* __restrict__ gchunk, const int32_t* __restrict__ goff,
             const int32_t* __restrict__ tile_off, int64_t ngroup, int2* __restrict__ items) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroup) return;
  int nc = gchunk[g], o = goff[g] + tile_off[g / kThreads];
  for (int c = 0; c < nc; ++c) items[o + c] = make_int2((int)g, c);
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int scan_tmp_size(int64_t len) { return (int)((len + kScanTile - 1) / kScanTile) + 1; }
int items_tmp_size(int64_t ngroup) { return (int)((ngroup + kThreads - 1) / kThreads) + 1; }

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + kThreads - 1) / kThreads;
  unsigned blocks = (unsigned)(b < 65536 ? b : 65536);
  k_fill_i32<<<blocks, kThreads, 0, s>>>(p, n, v);
  return hipGetLastError();
}

// out[0..len) = exclusive scan of in[0..len); out[len] = total; with
// zero_in, in[0..len) is cleared as it is read. tmp needs scan_tmp_size(len)
// entries; in and out must be 16-byte aligned (device allocations are).
hipError_t launch_scan(int32_t* in, int32_t* out, int64_t len, int32_t* tmp, hipStream_t s,
                       bool zero_in) {
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15)
    return hipErrorInvalidValue;
  int nt = (int)((len + kScanTile - 1) / kScanTile);
  if (nt == 0) return launch_fill_i32(out, 1, 0, s);
  if (zero_in)
    k_scan_tiles<true><<<nt, kThreads, 0, s>>>(in, out, len, tmp);
  else
    k_scan_tiles<false><<<nt, kThreads, 0, s>>>(in, out, len, tmp);
  k_scan_sums<<<1, 1024, 0, s>>>(tmp, nt, out + len);
  k_scan_add<<<nt, kThreads, 0, s>>>(out, len, tmp);
  return hipGetLastError();
}

hipError_t launch_bin(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                      double mass_scalar) {
  Workspace& W = P->ws;
  hipStream_t s = P->stream;
  hipError_t e;
  // The counts start at zero: cleared by the previous binning's scan, or
  // here when that binning did not get as far (a failed launch)
  if (P->count_dirty && (e = launch_fill_i32(W.count, P->ncell, 0, s)) != hipSuccess) return e;
  P->count_dirty = 1;
  k_bin_count<<<blocks_for(n, kThreads), kThreads, 0, s>>>(n, pos, P->ng, P->lg, 1.0 / P->h,
                                                           W.key, W.rank, W.count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_scan(W.count, W.start, P->ncell, W.scan_tmp, s, true)) != hipSuccess) return e;
  P->count_dirty = 0;
  if (P->prm.precision == P3M_FP32)
    k_scatter<float><<<blocks_for(n, kThreads), kThreads, 0, s>>>(
        n, pos, mass, mass_scalar, P->ng, P->lg, P->h, W.key, W.rank, W.start, W.perm,
        W.skey, (float4*)W.rec);
  else
    k_scatter<double><<<blocks_for(n, kThreads), kThreads, 0, s>>>(
        n, pos, mass, mass_scalar, P->ng, P->lg, P->h, W.key, W.rank, W.start, W.perm,
        W.skey, (double4*)W.rec);
  return hipGetLastError();
}

hipError_t launch_items(p3m_plan* P) {
  Workspace& W = P->ws;
  hipStream_t s = P->stream;
  // chunk counts + tile scans, scan of the tile sums (total to goff[ngroup]),
  // then the items at tile offset + offset within the tile
  const int nt = (int)((P->ngroup + kThreads - 1) / kThreads);
  k_items_tiles<<<nt, kThreads, 0, s>>>(W.start, P->lg, P->G, P->lgG, P->ngroup, W.gchunk,
                                        W.goff, W.scan_tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan_sums<<<1, 1024, 0, s>>>(W.scan_tmp, nt, W.goff + P->ngroup);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_emit_items<<<blocks_for(P->ngroup, kThreads), kThreads, 0, s>>>(W.gchunk, W.goff,
                                                                    W.scan_tmp, P->ngroup,
                                                                    W.items);
  return hipGetLastError();
}

}  // namespace p3m
