// Cloud-in-cell mass deposit and the fused finite-difference gradient +
// cloud-in-cell interpolation of the long-range (PM) force.
//
// Both kernels work on bricks of kBrick^3 grid cells. A particle in cell c
// (offset t = (x - c h)/h in [0,1) per axis) touches the nodes c and c + 1 of
// each axis with weights 1 - t and t (nodes at c h, periodic), so a brick's
// particles touch (kBrick + 1)^3 nodes.
//
// Deposit: the brick's particles are accumulated into an LDS copy of those
// nodes with LDS atomics, then each non-zero node is added to the global grid
// with one global atomic (only the brick faces overlap other bricks). The
// density is rho = sum m W / h^3.
//
// Interpolation: the brick's potential plus a two-node halo, (kBrick + 5)^3
// values, is staged in LDS; the central-difference gradient (order 4:
// [8(phi(c+1) - phi(c-1)) - (phi(c+2) - phi(c-2))] / 12h, or order 2) is formed
// on the (kBrick + 1)^3 nodes in LDS, and each particle takes
// a = -sum_nodes W * grad. The result goes to the sorted-order PM buffer (to be
// combined with the pair sum) or, for the PM-only call, straight to the
// force array in input order as m * a.
#include "brick.h"

namespace p3m {
namespace {

using namespace brick;

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_deposit(const typename Vec<T>::v4* __restrict__ rec, const int32_t* __restrict__ skey,
          const int32_t* __restrict__ start, int ng, int lg, T inv_h, T inv_h3,
          T* __restrict__ grid) {
  __shared__ T acc[kN1 * kN1 * kN1];
  __shared__ BrickRuns R;
  const int lb = lg - 3;                          // log2(ng / kBrick)
  const int b = blockIdx.x, mb = (1 << lb) - 1;
  const int bz0 = (b & mb) * kBrick, by0 = ((b >> lb) & mb) * kBrick, bx0 = (b >> (2 * lb)) * kBrick;
  for (int i = threadIdx.x; i < kN1 * kN1 * kN1; i += kThreads) acc[i] = T(0);
  load_runs(R, start, lg, bx0, by0, bz0);
  const int total = R.pre[kRows];
  for (int f = threadIdx.x; f < total; f += kThreads) {
    int r = find_run(R, f);
    int s = R.lo[r] + (f - R.pre[r]);
    typename Vec<T>::v4 p = rec[s];
    int lx = r / kBrick, ly = r % kBrick, lz = (skey[s] & (ng - 1)) - bz0;
    T tx = p.x * inv_h, ty = p.y * inv_h, tz = p.z * inv_h;
    T wx[2] = {T(1) - tx, tx}, wy[2] = {T(1) - ty, ty}, wz[2] = {T(1) - tz, tz};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T mxy = p.w * wx[a] * wy[c];
        int base = ((lx + a) * kN1 + (ly + c)) * kN1 + lz;
        atomicAdd(&acc[base], mxy * wz[0]);
        atomicAdd(&acc[base + 1], mxy * wz[1]);
      }
  }
  __syncthreads();
  const int mask = ng - 1;
  for (int i = threadIdx.x; i < kN1 * kN1 * kN1; i += kThreads) {
    T v = acc[i];
    if (v != T(0)) {
      int nx = i / (kN1 * kN1), ny = (i / kN1) % kN1, nz = i % kN1;
      int gx = (bx0 + nx) & mask, gy = (by0 + ny) & mask, gz = (bz0 + nz) & mask;
      atomicAdd(&grid[(((int64_t)gx << lg | gy) << lg) | gz], v * inv_h3);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_interp(const typename Vec<T>::v4* __restrict__ rec, const int32_t* __restrict__ skey,
         const int32_t* __restrict__ start, int ng, int lg, T inv_h, const T* __restrict__ phi,
         T c1, T c2, typename Vec<T>::v4* __restrict__ acc_out, const int32_t* __restrict__ perm,
         int64_t n, void* __restrict__ force, int force_fp32) {
  __shared__ T ph[kN5 * kN5 * kN5];
  __shared__ T gr[3][kN1 * kN1 * kN1];
  __shared__ BrickRuns R;
  const int lb = lg - 3, mb = (1 << lb) - 1, mask = ng - 1;
  const int b = blockIdx.x;
  const int bz0 = (b & mb) * kBrick, by0 = ((b >> lb) & mb) * kBrick, bx0 = (b >> (2 * lb)) * kBrick;
  for (int i = threadIdx.x; i < kN5 * kN5 * kN5; i += kThreads) {
    int nx = i / (kN5 * kN5), ny = (i / kN5) % kN5, nz = i % kN5;
    int gx = (bx0 - 2 + nx) & mask, gy = (by0 - 2 + ny) & mask, gz = (bz0 - 2 + nz) & mask;
    ph[i] = phi[(((int64_t)gx << lg | gy) << lg) | gz];
  }
  load_runs(R, start, lg, bx0, by0, bz0);       // contains __syncthreads
  for (int i = threadIdx.x; i < kN1 * kN1 * kN1; i += kThreads) {
    int nx = i / (kN1 * kN1), ny = (i / kN1) % kN1, nz = i % kN1;
    int q = ((nx + 2) * kN5 + (ny + 2)) * kN5 + (nz + 2);
    const int sx = kN5 * kN5, sy = kN5, sz = 1;
    gr[0][i] = c1 * (ph[q + sx] - ph[q - sx]) + c2 * (ph[q + 2 * sx] - ph[q - 2 * sx]);
    gr[1][i] = c1 * (ph[q + sy] - ph[q - sy]) + c2 * (ph[q + 2 * sy] - ph[q - 2 * sy]);
    gr[2][i] = c1 * (ph[q + sz] - ph[q - sz]) + c2 * (ph[q + 2 * sz] - ph[q - 2 * sz]);
  }
  __syncthreads();
  const int total = R.pre[kRows];
  for (int f = threadIdx.x; f < total; f += kThreads) {
    int r = find_run(R, f);
    int s = R.lo[r] + (f - R.pre[r]);
    typename Vec<T>::v4 p = rec[s];
    int lx = r / kBrick, ly = r % kBrick, lz = (skey[s] & mask) - bz0;
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
          int q = ((lx + a) * kN1 + (ly + c)) * kN1 + (lz + d);
          ax += w * gr[0][q];
          ay += w * gr[1][q];
          az += w * gr[2][q];
        }
    if (acc_out) {
      typename Vec<T>::v4 o;
      o.x = -ax; o.y = -ay; o.z = -az; o.w = T(0);
      acc_out[s] = o;
    } else {
      int64_t i = perm[s];
      double m = (double)p.w;
      if (force_fp32) {
        float* F = (float*)force;
        F[i] = (float)(-m * (double)ax);
        F[n + i] = (float)(-m * (double)ay);
        F[2 * n + i] = (float)(-m * (double)az);
      } else {
        double* F = (double*)force;
        F[i] = -m * (double)ax;
        F[n + i] = -m * (double)ay;
        F[2 * n + i] = -m * (double)az;
      }
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_deposit(p3m_plan* P) {
  Workspace& W = P->ws;
  hipError_t e = launch_fill_i32((int32_t*)W.grid, P->ncell * (int64_t)(sizeof(T) / 4), 0,
                                 P->stream);
  if (e != hipSuccess) return e;
  int nb = (int)(P->ncell / (kBrick * kBrick * kBrick));
  T inv_h = T(1.0 / P->h);
  T inv_h3 = T(1.0 / (P->h * P->h * P->h));
  k_deposit<T><<<nb, kThreads, 0, P->stream>>>((const typename Vec<T>::v4*)W.rec, W.skey,
                                               W.start, P->ng, P->lg, inv_h, inv_h3,
                                               (T*)W.grid);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp(p3m_plan* P, int64_t n, void* force_out, int force_fp32) {
  Workspace& W = P->ws;
  int nb = (int)(P->ncell / (kBrick * kBrick * kBrick));
  double h = P->h;
  T c1, c2;
  if (P->prm.fd_order == 2) {
    c1 = T(1.0 / (2.0 * h));
    c2 = T(0);
  } else {
    c1 = T(8.0 / (12.0 * h));
    c2 = T(-1.0 / (12.0 * h));
  }
  typename Vec<T>::v4* acc = force_out ? nullptr : (typename Vec<T>::v4*)W.acc_pm;
  k_interp<T><<<nb, kThreads, 0, P->stream>>>((const typename Vec<T>::v4*)W.rec, W.skey,
                                              W.start, P->ng, P->lg, T(1.0 / h),
                                              (const T*)W.grid, c1, c2, acc, W.perm, n,
                                              force_out, force_fp32);
  return hipGetLastError();
}

template hipError_t launch_deposit<float>(p3m_plan*);
template hipError_t launch_deposit<double>(p3m_plan*);
template hipError_t launch_interp<float>(p3m_plan*, int64_t, void*, int);
template hipError_t launch_interp<double>(p3m_plan*, int64_t, void*, int);

}  // namespace p3m
