// Cloud-in-cell mass deposit and the fused finite-difference gradient +
// cloud-in-cell interpolation of the long-range (PM) force.
//
// Both kernels work on bricks of grid cells. A particle in cell c
// (offset t = (x - c h)/h in [0,1) per axis) touches the nodes c and c + 1 of
// each axis with weights 1 - t and t (nodes at c h, periodic), so a brick's
// particles touch one node more per axis than it has cells.
//
// Deposit: each brick's 8^3 nodes gather the particles of the cells around
// them (no atomics; see k_deposit_gather). The density is rho = sum m W / h^3.
//
// Interpolation (bricks of BX x BX x BZ cells, 4 x 4 x 16): the brick's
// potential plus a two-node halo, (BX + 5)^2 (BZ + 5) values, is staged in
// LDS; the central-difference gradient (order 4:
// [8(phi(c+1) - phi(c-1)) - (phi(c+2) - phi(c-2))] / 12h, or order 2) is formed
// on the (BX + 1)^2 (BZ + 1) nodes in LDS, and each particle takes
// a = -sum_nodes W * grad. The result goes to the sorted-order PM buffer (to be
// combined with the pair sum) or, for the PM-only call, straight to the
// force array in input order as m * a.
#include "brick.h"

namespace p3m {
namespace {

using namespace brick;

// Deposit by gathering: the workgroup owns the 8^3 nodes of its brick (every
// grid node belongs to exactly one brick, so each is written once, with no
// atomics and in a fixed order). Node n takes, per axis, weight t from the
// particles of cell n - 1 (n is that cell's upper node) and 1 - t from those
// of cell n, so the 8^3 nodes need the cells [-1, 8)^3 around the brick,
// whose sorted ranges are staged in LDS first. NC = 1: mass, scaled by
// 1 / h^3 (the density); NC = 3: mass times each component of a cotangent
// (the adjoint's deposit), unscaled, to out[c * ng^3 + node].
//
// Heavy cells (NC = 1): a node thread that loops over the particles of its
// eight cells takes as long as the most crowded of them, so on clustered
// input a few threads would hold their brick for thousands of iterations.
// A cell with more than kHeavy particles is instead reduced once, by one
// wave (the lanes split its particles), into its eight corner sums
// sum m (1 - t or t)_x (1 - t or t)_y (1 - t or t)_z, kept in LDS for up to
// kHeavySlots such cells per brick; its nodes add the one sum each needs.
// (Further heavy cells of a brick are looped over as before.)
constexpr int kHeavy = 16;
constexpr int kHeavySlots = 96;

template <typename T, int NC>
__global__ void __launch_bounds__(kThreads)
k_deposit_gather(const typename Vec<T>::v4* __restrict__ rec,
                 const typename Vec<T>::v4* __restrict__ lam, const int32_t* __restrict__ start,
                 int ng, int lg, T inv_h, T scale, T* __restrict__ out) {
  constexpr int kC = kN1 * kN1 * kN1;             // cells [-1, kBrick)^3
  constexpr bool HV = NC == 1;                    // heavy cells reduced once
  __shared__ int cs[kC], cn[kC];
  __shared__ short hidx[HV ? kC : 1];             // slot of a heavy cell, or -1
  __shared__ short hcell[HV ? kHeavySlots : 1];
  __shared__ T mom[HV ? kHeavySlots : 1][8];
  __shared__ int hcount;
  const int lb = lg - 3, mb = (1 << lb) - 1, mask = ng - 1;
  const int b = blockIdx.x;
  const int bz0 = (b & mb) * kBrick, by0 = ((b >> lb) & mb) * kBrick, bx0 = (b >> (2 * lb)) * kBrick;
  if (HV && threadIdx.x == 0) hcount = 0;
  for (int e = threadIdx.x; e < kC; e += kThreads) {
    const int gx = (bx0 - 1 + e / (kN1 * kN1)) & mask, gy = (by0 - 1 + (e / kN1) % kN1) & mask,
              gz = (bz0 - 1 + e % kN1) & mask;
    const int64_t c = (((int64_t)gx << lg | gy) << lg) | gz;
    const int lo = start[c];
    cs[e] = lo;
    cn[e] = start[c + 1] - lo;
  }
  __syncthreads();
  if constexpr (HV) {
    for (int e = threadIdx.x; e < kC; e += kThreads) {
      short slot = -1;
      if (cn[e] > kHeavy) {
        const int k = atomicAdd(&hcount, 1);
        if (k < kHeavySlots) {
          slot = (short)k;
          hcell[k] = (short)e;
        }
      }
      hidx[e] = slot;
    }
    __syncthreads();
    const int nh = min(hcount, kHeavySlots);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = wave; k < nh; k += kThreads / 64) {
      const int e = hcell[k];
      const int s0 = cs[e], s1 = s0 + cn[e];
      T m8[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) m8[q] = T(0);
      for (int s = s0 + lane; s < s1; s += 64) {
        const typename Vec<T>::v4 p = rec[s];
        const T tx = p.x * inv_h, ty = p.y * inv_h, tz = p.z * inv_h;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int a = q >> 2, bb = (q >> 1) & 1, c = q & 1;
          m8[q] += p.w * ((a ? T(1) - tx : tx) * (bb ? T(1) - ty : ty) * (c ? T(1) - tz : tz));
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m8[q] += __shfl_xor(m8[q], o, 64);
      }
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) mom[k][q] = m8[q];
      }
    }
    __syncthreads();
  }
  const int64_t ncell = (int64_t)1 << (3 * lg);
  for (int node = threadIdx.x; node < kBrick * kBrick * kBrick; node += kThreads) {
    const int i = node >> 6, j = (node >> 3) & 7, k = node & 7;
    T acc[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int e = ((i + a) * kN1 + (j + bb)) * kN1 + (k + c);
          if constexpr (HV) {
            const int h = hidx[e];
            if (h >= 0) {
              acc[0] += mom[h][(a << 2) | (bb << 1) | c];
              continue;
            }
          }
          const int s0 = cs[e], s1 = s0 + cn[e];
          for (int s = s0; s < s1; ++s) {
            const typename Vec<T>::v4 p = rec[s];
            const T tx = p.x * inv_h, ty = p.y * inv_h, tz = p.z * inv_h;
            const T w = (a ? T(1) - tx : tx) * (bb ? T(1) - ty : ty) * (c ? T(1) - tz : tz);
            if constexpr (NC == 1) {
              acc[0] += p.w * w;
            } else {
              const typename Vec<T>::v4 l = lam[s];
              const T mw = p.w * w;
              acc[0] += mw * l.x;
              acc[1] += mw * l.y;
              acc[2] += mw * l.z;
            }
          }
        }
    const int64_t g = (((int64_t)(bx0 + i) << lg | (by0 + j)) << lg) | (bz0 + k);
#pragma unroll
    for (int q = 0; q < NC; ++q) out[q * ncell + g] = acc[q] * scale;
  }
}

template <typename T, int BX, int BZ>
__global__ void __launch_bounds__(kThreads)
k_interp(const typename Vec<T>::v4* __restrict__ rec, const int32_t* __restrict__ skey,
         const int32_t* __restrict__ start, int ng, int lg, T inv_h, const T* __restrict__ phi,
         T c1, T c2, typename Vec<T>::v4* __restrict__ acc_out, const int32_t* __restrict__ perm,
         int64_t n, void* __restrict__ force, int force_fp32,
         const typename Vec<T>::v4* __restrict__ acc_pp) {
  constexpr int X1 = BX + 1, Z1 = BZ + 1;        // nodes touched per axis
  constexpr int X5 = BX + 5, Z5 = BZ + 5;        // with the two-node gradient halo
  __shared__ T ph[X5 * X5 * Z5];
  __shared__ T gr[3][X1 * X1 * Z1];
  __shared__ InterpRuns<BX, BZ> R;
  const int mask = ng - 1, nbz = ng / BZ, nbx = ng / BX;
  const int b = blockIdx.x;
  const int bz0 = (b % nbz) * BZ, by0 = ((b / nbz) % nbx) * BX, bx0 = (b / (nbz * nbx)) * BX;
  for (int i = threadIdx.x; i < X5 * X5 * Z5; i += kThreads) {
    int nx = i / (X5 * Z5), ny = (i / Z5) % X5, nz = i % Z5;
    int gx = (bx0 - 2 + nx) & mask, gy = (by0 - 2 + ny) & mask, gz = (bz0 - 2 + nz) & mask;
    ph[i] = phi[(((int64_t)gx << lg | gy) << lg) | gz];
  }
  load_interp_runs(R, start, lg, bx0, by0, bz0);  // contains __syncthreads
  for (int i = threadIdx.x; i < X1 * X1 * Z1; i += kThreads) {
    int nx = i / (X1 * Z1), ny = (i / Z1) % X1, nz = i % Z1;
    int q = ((nx + 2) * X5 + (ny + 2)) * Z5 + (nz + 2);
    const int sx = X5 * Z5, sy = Z5, sz = 1;
    gr[0][i] = c1 * (ph[q + sx] - ph[q - sx]) + c2 * (ph[q + 2 * sx] - ph[q - 2 * sx]);
    gr[1][i] = c1 * (ph[q + sy] - ph[q - sy]) + c2 * (ph[q + 2 * sy] - ph[q - 2 * sy]);
    gr[2][i] = c1 * (ph[q + sz] - ph[q - sz]) + c2 * (ph[q + 2 * sz] - ph[q - 2 * sz]);
  }
  __syncthreads();
  const int total = R.pre[InterpRuns<BX, BZ>::kR];
  for (int f = threadIdx.x; f < total; f += kThreads) {
    int r = find_interp_run(R, f);
    int s = R.lo[r] + (f - R.pre[r]);
    typename Vec<T>::v4 p = rec[s];
    int lx = r / BX, ly = r % BX, lz = (skey[s] & mask) - bz0;
    T tx = p.x * inv_h, ty = p.y * inv_h, tz = p.z * inv_h;
    T wx[2] = {T(1) - tx, tx}, wy[2] = {T(1) - ty, ty}, wz[2] = {T(1) - tz, tz};
    T ax = 0, ay = 0, az = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          T w = wx[a] * wy[c] * wz[d];
          int q = ((lx + a) * X1 + (ly + c)) * Z1 + (lz + d);
          ax += w * gr[0][q];
          ay += w * gr[1][q];
          az += w * gr[2][q];
        }
    if (acc_out) {
      typename Vec<T>::v4 o;
      o.x = -ax; o.y = -ay; o.z = -az; o.w = T(0);
      acc_out[s] = o;
    } else {
      int64_t i = perm ? perm[s] : s;      // (no permutation: cell order)
      double m = (double)p.w;
      // acc_pp: the pair sum's sorted acceleration, added here (the P3M call
      // whose mesh part ran beside the pair sum)
      double gx = -(double)ax, gy = -(double)ay, gz = -(double)az;
      if (acc_pp) {
        const typename Vec<T>::v4 a = acc_pp[s];
        gx += (double)a.x; gy += (double)a.y; gz += (double)a.z;
      }
      if (force_fp32) {
        float* F = (float*)force;
        F[i] = (float)(m * gx);
        F[n + i] = (float)(m * gy);
        F[2 * n + i] = (float)(m * gz);
      } else {
        double* F = (double*)force;
        F[i] = m * gx;
        F[n + i] = m * gy;
        F[2 * n + i] = m * gz;
      }
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_deposit(p3m_plan* P) {
  Workspace& W = P->ws;
  const int nb = (int)(P->ncell / (kBrick * kBrick * kBrick));
  k_deposit_gather<T, 1><<<nb, kThreads, 0, P->stream>>>(
      (const typename Vec<T>::v4*)W.rec, nullptr, W.start, P->ng, P->lg, T(1.0 / P->h),
      T(1.0 / (P->h * P->h * P->h)), (T*)W.grid);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_deposit3(p3m_plan* P, const void* lam, void* grids) {
  Workspace& W = P->ws;
  const int nb = (int)(P->ncell / (kBrick * kBrick * kBrick));
  k_deposit_gather<T, 3><<<nb, kThreads, 0, P->stream>>>(
      (const typename Vec<T>::v4*)W.rec, (const typename Vec<T>::v4*)lam, W.start, P->ng, P->lg,
      T(1.0 / P->h), T(1), (T*)grids);
  return hipGetLastError();
}

// One interpolation launch over bricks of BX x BX x BZ cells (one workgroup
// per brick); the grid's edge must be a multiple of BX and BZ.
template <typename T, int BX, int BZ>
hipError_t launch_interp_bricks(p3m_plan* P, int64_t n, void* force_out, int force_fp32,
                                const void* acc_pp, T c1, T c2, void* sorted_out) {
  Workspace& W = P->ws;
  const int nb = (int)(P->ncell / (BX * BX * BZ));
  typename Vec<T>::v4* acc = (typename Vec<T>::v4*)sorted_out;
  k_interp<T, BX, BZ><<<nb, kThreads, 0, P->stream>>>(
      (const typename Vec<T>::v4*)W.rec, W.skey, W.start, P->ng, P->lg, T(1.0 / P->h),
      (const T*)W.grid, c1, c2, acc, P->cell_order ? nullptr : W.perm, n, force_out, force_fp32,
      (const typename Vec<T>::v4*)acc_pp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp(p3m_plan* P, int64_t n, void* force_out, int force_fp32,
                         const void* acc_pp, void* sorted_out) {
  double h = P->h;
  T c1, c2;
  if (P->prm.fd_order == 2) {
    c1 = T(1.0 / (2.0 * h));
    c2 = T(0);
  } else {
    c1 = T(8.0 / (12.0 * h));
    c2 = T(-1.0 / (12.0 * h));
  }
  // Bricks of 4 x 4 x 16 cells (grids are at least 16 cells on a side): a
  // wave's particles are 4 runs of 16 cells. Measured at 128^3 against 8^3
  // bricks: FP32 65 -> 47 us (4 x 4 x 32: the same; 2 x 2 x 64: 55), FP64
  // 77 -> 62 us (4 x 4 x 32: 72, its LDS costing occupancy; 2 x 2 x 32: 72).
  // no force: the sorted mesh acceleration, to sorted_out (default: ws.acc_pm)
  if (!force_out && !sorted_out) sorted_out = P->ws.acc_pm;
  return launch_interp_bricks<T, 4, 16>(P, n, force_out, force_fp32, acc_pp, c1, c2,
                                        force_out ? nullptr : sorted_out);
}

template hipError_t launch_deposit<float>(p3m_plan*);
template hipError_t launch_deposit<double>(p3m_plan*);
template hipError_t launch_deposit3<float>(p3m_plan*, const void*, void*);
template hipError_t launch_deposit3<double>(p3m_plan*, const void*, void*);
template hipError_t launch_interp<float>(p3m_plan*, int64_t, void*, int, const void*, void*);
template hipError_t launch_interp<double>(p3m_plan*, int64_t, void*, int, const void*, void*);

}  // namespace p3m
