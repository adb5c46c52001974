// Newton's third law in the short-range pair sum.
//
// The pair force of i on j is minus that of j on i (the Plummer-softened,
// erfc-split pair law depends on the separation only, and it is odd in it),
// and so is the pair term of the force adjoint. Where particles are dense,
// the pair sum evaluates each such pair once and keeps the other particle's
// share as a partial. A group is dense when it holds more than kDenseMin
// particles; a work item (group g, chunk a of kChunk particles) of a dense
// group stages
//   1. its own group's particles from its chunk on (flattened index >= 64 a):
//      its own chunk first (both sides of each pair evaluated, the item's own
//      action only), then the later chunks, with their reactions;
//   2. the stencil cut into group segments: a segment in another dense group
//      at a lexicographically positive offset with the reactions, one in a
//      sparse group on either side without (that group evaluates its own
//      side), and none in a dense group at a negative offset (that group
//      evaluates the pair);
// and for every staged entry that takes a reaction it writes the reaction
// the item's particles exert on that entry as one partial (its 3 components
// together) at a fixed place. Sparse groups evaluate every pair from both sides. This
// file holds the steps around the pair kernel:
//   - per group: its particle count and the particles before each of its
//     z-runs; per dense group the reaction entries before each positive
//     segment and its number of partials T(g) = K L + (K - 1) n - 32 K (K - 1),
//     K = ceil(n / 64) chunks, n particles, L reaction entries of the
//     stencil (item (g, a) writes (n - 64 (a + 1))^+ + L of them);
//   - an exclusive scan of T over the groups (64-bit);
//   - the gather: every particle of a dense group sums the partials that
//     name it, in a fixed order (no atomics), and adds them to its action.
// When the partials of a call exceed the plan's capacity, every pair is
// evaluated from both sides for that call (decided on the device).
#include "p3m_internal.h"

namespace p3m {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int wave_inclusive(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Particles in the cells [A, B) (unwrapped z) of one column of the sorted
// cell list, colbase the column's first cell: whole turns around the
// periodic box, then at most two runs split at the face.
__device__ __forceinline__ int column_count(const int32_t* __restrict__ start, int colbase,
                                            int A, int B, int ng) {
  int len = B - A;
  if (len <= 0) return 0;
  int total = 0;
  const int whole = start[colbase + ng] - start[colbase];
  while (len >= ng) {
    total += whole;
    len -= ng;
  }
  const int a = A & (ng - 1), b = a + len;
  if (b <= ng) return total + start[colbase + b] - start[colbase + a];
  return total + (start[colbase + ng] - start[colbase + a]) + (start[colbase + b - ng] - start[colbase]);
}

// Per group: its particle count and the particles before each of its
// G * G z-runs (flattened order: run (a, b) at a * G + b).
__global__ void __launch_bounds__(kThreads)
k_group_runs(const int32_t* __restrict__ start, int lg, int G, int lgG, int64_t ngroup,
             int32_t* __restrict__ gipre, int32_t* __restrict__ gntot) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= ngroup) return;
  const int lgd = lg - lgG, md = (1 << lgd) - 1;
  const int gx0 = (int)(g >> (2 * lgd)) << lgG;
  const int gy0 = (int)((g >> lgd) & md) << lgG;
  const int gz0 = (int)(g & md) << lgG;
  int acc = 0;
  for (int run = 0; run < G * G; ++run) {
    const int c0 = ((((gx0 + (run >> lgG)) << lg) | (gy0 + (run & (G - 1)))) << lg) | gz0;
    gipre[g * G * G + run] = acc;
    acc += start[c0 + G] - start[c0];
  }
  gntot[g] = acc;
}

// Group index of the group at offset (ox, oy, oz) from the group at (gx, gy,
// gz) (group units, periodic).
__device__ __forceinline__ int64_t group_at(int gx, int gy, int gz, int ox, int oy, int oz,
                                            int lgd) {
  const int md = (1 << lgd) - 1;
  return ((int64_t)((gx + ox) & md) << (2 * lgd)) | ((int64_t)((gy + oy) & md) << lgd) |
         ((gz + oz) & md);
}

// One wavefront per dense group: the reaction entries (particles of the
// segment when its group is dense) before each positive segment, their
// total L, and the group's number of partials T(g); 0 for a sparse group.
__global__ void __launch_bounds__(64)
k_react_rows(const int32_t* __restrict__ start, const int32_t* __restrict__ gntot,
             const int4* __restrict__ prows, int npos, int lg, int lgG, int64_t ngroup,
             int32_t* __restrict__ rowoff, long long* __restrict__ gtot) {
  const int64_t g = blockIdx.x;
  if (g >= ngroup) return;
  const int lane = threadIdx.x;
  const int ntot = gntot[g];
  if (ntot <= kDenseMin) {
    if (lane == 0) gtot[g] = 0;
    return;
  }
  const int ng = 1 << lg, mask = ng - 1, lgd = lg - lgG, md = (1 << lgd) - 1;
  const int gx = (int)(g >> (2 * lgd)), gy = (int)((g >> lgd) & md), gz = (int)(g & md);
  const int gx0 = gx << lgG, gy0 = gy << lgG, gz0 = gz << lgG;
  int32_t* ro = rowoff + g * (npos + 1);
  int carry = 0;
  for (int rb = 0; rb < npos; rb += 64) {
    const int k = rb + lane;
    int c = 0;
    if (k < npos) {
      const int4 p = prows[k];
      const int dx = (int)(short)(p.x & 0xffff), dy = p.x >> 16;
      const int64_t g2 = group_at(gx, gy, gz, dx >> lgG, dy >> lgG, p.y >> lgG, lgd);
      if (gntot[g2] > kDenseMin) {
        const int colbase = ((((gx0 + dx) & mask) << lg) | ((gy0 + dy) & mask)) << lg;
        const int zw = (gz0 + p.y) & mask;
        c = start[colbase + zw + (p.z - p.y + 1)] - start[colbase + zw];
      }
    }
    const int inc = wave_inclusive(c);
    if (k < npos) ro[k] = carry + inc - c;
    carry += __shfl(inc, 63, 64);
  }
  if (lane == 0) {
    ro[npos] = carry;
    const long long K = (ntot + kChunk - 1) / kChunk;
    gtot[g] = K * carry + (K - 1) * ntot - 32 * K * (K - 1);
  }
}

// ---- exclusive scan of int64 (tiles of 1024, tile sums, add) ----

constexpr int kScan64Items = 4;
constexpr int kScan64Tile = kThreads * kScan64Items;

__device__ __forceinline__ long long wave_inclusive64(long long v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ long long block_exclusive64(long long v, long long* wsum,
                                                       long long& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  long long inc = wave_inclusive64(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  long long base = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    long long s = wsum[k];
    if (k < w) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

__global__ void __launch_bounds__(kThreads)
k_scan64_tiles(const long long* __restrict__ in, long long* __restrict__ out, int64_t len,
               long long* __restrict__ tile_sum) {
  __shared__ long long wsum[kThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScan64Tile + (int64_t)threadIdx.x * kScan64Items;
  long long v[kScan64Items], local = 0;
#pragma unroll
  for (int k = 0; k < kScan64Items; ++k) {
    v[k] = base + k < len ? in[base + k] : 0;
    local += v[k];
  }
  long long total;
  long long run = block_exclusive64(local, wsum, total);
#pragma unroll
  for (int k = 0; k < kScan64Items; ++k) {
    if (base + k < len) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024)
k_scan64_sums(long long* __restrict__ sums, int64_t nt, long long* __restrict__ grand) {
  __shared__ long long wsum[1024 / 64];
  long long carry = 0;
  for (int64_t b = 0; b < nt; b += blockDim.x) {
    const int64_t i = b + threadIdx.x;
    long long v = i < nt ? sums[i] : 0;
    long long total;
    long long ex = block_exclusive64(v, wsum, total);
    if (i < nt) sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *grand = carry;
}

__global__ void __launch_bounds__(kThreads)
k_scan64_add(long long* __restrict__ out, int64_t len, const long long* __restrict__ tile_off) {
  const int64_t base = (int64_t)blockIdx.x * kScan64Tile;
  const long long add = tile_off[blockIdx.x];
  for (int k = threadIdx.x; k < kScan64Tile; k += kThreads) {
    const int64_t i = base + k;
    if (i < len) out[i] += add;
  }
}

// ---- the gather ----

template <typename T>
struct GatherArgs {
  const typename Vec<T>::v4* __restrict__ rec;   // sorted records (mass in w)
  const int32_t* __restrict__ skey;
  const int32_t* __restrict__ start;
  const int4* __restrict__ pbrows;
  const int32_t* __restrict__ pboff;
  const int32_t* __restrict__ rowoff;
  const int32_t* __restrict__ gipre;
  const int32_t* __restrict__ gntot;
  const long long* __restrict__ gbase;           // [ngroup + 1]
  const T* __restrict__ rpart;                   // [rcap][3]
  long long rcap;
  int npos, lg, G, lgG;
  int64_t ngroup;
  int64_t n;
  double rscale;                                 // -(the pair kernel's output scale)
  const typename Vec<T>::v4* __restrict__ acc;   // sorted action (acceleration)
  const typename Vec<T>::v4* __restrict__ add;   // sorted acceleration added at the end, or null
  typename Vec<T>::v4* __restrict__ acc_out;     // sorted result, or null
  const int32_t* __restrict__ perm;
  void* __restrict__ out;                        // input-order result m * a, or null
  int out_fp32;
};

// Partial index of item (g, a)'s entry at staged offset q past its own
// chunk: the group's base, the items before it, then q.
__device__ __forceinline__ long long item_base(long long gb, int ntot, int L, int a) {
  return gb + (long long)a * (ntot + L) - 32LL * a * (a + 1);
}

// One thread per particle in sorted order. UM: one mass for all particles
// (the partials then carry no mass factor). A particle of a dense group
// gathers the partials of the earlier chunks of its own group and those of
// the dense groups that see its cell in a positive segment; the wavefront's
// consecutive particles mostly share their cell, so they read consecutive
// partials.
template <typename T, bool UM>
__global__ void __launch_bounds__(kThreads)
k_react_gather(GatherArgs<T> A) {
  using T4 = typename Vec<T>::v4;
  const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (s >= A.n) return;
  const int ng = 1 << A.lg, mask = ng - 1, G = A.G, lgG = A.lgG;
  const int lgd = A.lg - lgG;
  const T4 rs = A.rec[s];
  const T4 a = A.acc[s];
  double ax = (double)a.x, ay = (double)a.y, az = (double)a.z;   // the result
  const long long total = A.gbase[A.ngroup];
  const int c = A.skey[s];
  const int cz = c & mask, cy = (c >> A.lg) & mask, cx = c >> (2 * A.lg);
  const int gx = cx >> lgG, gy = cy >> lgG, gz = cz >> lgG;
  const int64_t gs = ((int64_t)gx << (2 * lgd)) | ((int64_t)gy << lgd) | gz;
  const int ntot_s = A.gntot[gs];
  if (total <= A.rcap && ntot_s > kDenseMin) {   // one-sided sum, dense group: reactions
    const T* pr = A.rpart;                   // partial idx at pr[3 idx .. 3 idx + 2]
    const long long last = total > 0 ? total - 1 : 0;
    const int colbase = ((cx << A.lg) | cy) << A.lg;
    const int np1 = A.npos + 1;
    T sx = 0, sy = 0, sz = 0;
    // 1. the earlier chunks of its own group (its flattened index fi: the
    //    particles of the group's z-runs before its own, then its place in
    //    its run, which starts at the group's first z-cell)
    {
      const int run = ((cx & (G - 1)) << lgG) | (cy & (G - 1));
      const int fi = A.gipre[gs * G * G + run] + (int)(s - A.start[colbase + (gz << lgG)]);
      if (fi >= kChunk) {
        const int L = A.rowoff[gs * np1 + A.npos];
        const long long gb = A.gbase[gs];
#pragma unroll 4
        for (int ch = 0; ch < fi / kChunk; ++ch) {
          // (the clamp never acts: a guard that keeps the loads in flight together)
          const long long idx =
              min(item_base(gb, ntot_s, L, ch) + (fi - kChunk * (ch + 1)), last);
          sx += pr[3 * idx];
          sy += pr[3 * idx + 1];
          sz += pr[3 * idx + 2];
        }
      }
    }
    // 2. the dense groups that see the particle's cell in a positive segment:
    //    segments of the class of its column; the one at group offset
    //    (ox, oy, oz) belongs to the group at minus that offset, and holds
    //    the cell when the cell's z offset from that group lies in it
    const int key = ((cx & (G - 1)) << lgG) | (cy & (G - 1));
    const int kb = A.pboff[key], ke = A.pboff[key + 1];
    for (int k = kb; k < ke; ++k) {
      const int4 p = A.pbrows[k];
      const int oz = p.y >> lgG;
      const int zoff = (oz << lgG) + (cz & (G - 1));
      if (zoff < p.y || zoff > p.z) continue;
      const int dx = (int)(short)(p.x & 0xffff), dy = p.x >> 16;
      const int64_t g = group_at(gx, gy, gz, -(dx >> lgG), -(dy >> lgG), -oz, lgd);
      const int ntot = A.gntot[g];
      if (ntot <= kDenseMin) continue;         // sparse: wrote no partials
      const int K = (ntot + kChunk - 1) / kChunk;
      const int32_t* ro = A.rowoff + g * np1;
      const int L = ro[A.npos];
      // the segment's cells below the particle's (same column, same group
      // of cells along z), then the particle's place in its cell
      const long long q = ro[p.w] + (s - A.start[colbase + cz - (zoff - p.y)]);
      const long long gb = A.gbase[g];
#pragma unroll 4
      for (int ch = 0; ch < K; ++ch) {
        const long long idx =
            min(item_base(gb, ntot, L, ch) + max(ntot - kChunk * (ch + 1), 0) + q, last);
        sx += pr[3 * idx];
        sy += pr[3 * idx + 1];
        sz += pr[3 * idx + 2];
      }
    }
    const double f = UM ? A.rscale * (double)rs.w : A.rscale;
    ax += f * (double)sx;
    ay += f * (double)sy;
    az += f * (double)sz;
  }
  if (A.add) {                         // the mesh part (P3M force)
    const T4 b = A.add[s];
    ax += (double)b.x;
    ay += (double)b.y;
    az += (double)b.z;
  }
  if (A.acc_out) {
    T4 o;
    o.x = (T)ax; o.y = (T)ay; o.z = (T)az; o.w = T(0);
    A.acc_out[s] = o;
    return;
  }
  const int64_t i = A.perm ? A.perm[s] : s;   // (no permutation: cell order)
  const double m = (double)rs.w;
  if (A.out_fp32) {
    float* F = (float*)A.out;
    F[i] = (float)(m * ax);
    F[A.n + i] = (float)(m * ay);
    F[2 * A.n + i] = (float)(m * az);
  } else {
    double* F = (double*)A.out;
    F[i] = m * ax;
    F[A.n + i] = m * ay;
    F[2 * A.n + i] = m * az;
  }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_react_prepass(p3m_plan* P) {
  Workspace& W = P->ws;
  hipStream_t s = P->stream;
  k_group_runs<<<blocks_for(P->ngroup, kThreads), kThreads, 0, s>>>(
      W.start, P->lg, P->G, P->lgG, P->ngroup, W.gipre, W.gntot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_react_rows<<<(unsigned)P->ngroup, 64, 0, s>>>(W.start, W.gntot, W.prows, P->npos, P->lg,
                                                  P->lgG, P->ngroup, W.rowoff, W.gtot);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t nt = (P->ngroup + kScan64Tile - 1) / kScan64Tile;
  k_scan64_tiles<<<(unsigned)nt, kThreads, 0, s>>>(W.gtot, W.gbase, P->ngroup, W.gscan_tmp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_scan64_sums<<<1, 1024, 0, s>>>(W.gscan_tmp, nt, W.gbase + P->ngroup);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_scan64_add<<<(unsigned)nt, kThreads, 0, s>>>(W.gbase, P->ngroup, W.gscan_tmp);
  return hipGetLastError();
}

int64_t react_scan_tmp_size(int64_t ngroup) { return (ngroup + kScan64Tile - 1) / kScan64Tile + 1; }

template <typename T>
hipError_t launch_react_gather(p3m_plan* P, int64_t n, double rscale, bool uniform_mass,
                               void* acc_out, void* out, int out_fp32, const void* acc_add) {
  Workspace& W = P->ws;
  GatherArgs<T> A{};
  A.rec = (const typename Vec<T>::v4*)W.rec;
  A.skey = W.skey;
  A.start = W.start;
  A.pbrows = W.pbrows;
  A.pboff = W.pboff;
  A.rowoff = W.rowoff;
  A.gipre = W.gipre;
  A.gntot = W.gntot;
  A.gbase = W.gbase;
  A.rpart = (const T*)W.rpart;
  A.rcap = P->rcap;
  A.npos = P->npos;
  A.lg = P->lg;
  A.G = P->G;
  A.lgG = P->lgG;
  A.ngroup = P->ngroup;
  A.n = n;
  A.rscale = rscale;
  A.acc = (const typename Vec<T>::v4*)W.acc_pm;
  A.add = (const typename Vec<T>::v4*)acc_add;
  A.acc_out = (typename Vec<T>::v4*)acc_out;
  A.perm = P->cell_order ? nullptr : W.perm;
  A.out = out;
  A.out_fp32 = out_fp32;
  if (uniform_mass)
    k_react_gather<T, true><<<blocks_for(n, kThreads), kThreads, 0, P->stream>>>(A);
  else
    k_react_gather<T, false><<<blocks_for(n, kThreads), kThreads, 0, P->stream>>>(A);
  return hipGetLastError();
}

template hipError_t launch_react_gather<float>(p3m_plan*, int64_t, double, bool, void*, void*,
                                               int, const void*);
template hipError_t launch_react_gather<double>(p3m_plan*, int64_t, double, bool, void*, void*,
                                                int, const void*);

}  // namespace p3m
