// Mesh part of the force adjoint, and the transpose of the drift.
//
// For a cotangent lam on the force F_i = m_i a_PM(x_i), with
// a_PM(x) = -sum_c W(x - c) E(c), E = D phi, phi = P rho and
// rho(c) = h^-3 sum_j m_j W(x_j - c) (P: the Green's function operator, real
// and even in k, so P^T = P; D: central differences, D^T = -D), the position
// cotangent is
//
//   pos_bar_k = m_k sum_c grad W(x_k - c) [h^-3 psi(c) - lam_k . E(c)],
//   psi = P S,  S = sum_d D_d Lam_d,  Lam_d(c) = sum_i m_i lam_{i,d} W(x_i - c):
//
// the particle's effect on the density it deposits, and on its own
// interpolation weights. The stages: sort lam into the particle order of the
// sorted cell list; deposit Lam (three components, gathered per node like
// the mass deposit) and take its divergence S on the nodes; solve psi = P S with the same FFT Poisson solve as the forward
// potential; then, per brick, stage phi (with the gradient halo) and psi in
// LDS and gather the weight gradients of each particle.
//
// The drift transpose: x1 = wrap(x + c p / m) gives p_bar += (c / m) x1_bar.
#include "brick.h"

namespace p3m {
namespace {

using namespace brick;

// In input order (coalesced reads of the three cotangent rows); each particle
// goes to its sorted slot start[key] + rank, as in the binning's scatter.
template <typename T>
__global__ void __launch_bounds__(256)
k_lambda_sort(int64_t n, const int32_t* __restrict__ key, const int32_t* __restrict__ rank,
              const int32_t* __restrict__ start, const double* __restrict__ fbar,
              typename Vec<T>::v4* __restrict__ lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = start[key[i]] + rank[i];
  typename Vec<T>::v4 o;
  o.x = (T)fbar[i];
  o.y = (T)fbar[n + i];
  o.z = (T)fbar[2 * n + i];
  o.w = T(0);
  lam[s] = o;
}

// S(c) = sum_d (D_d Lam_d)(c), D_d the central difference of the forward path.
template <typename T>
__global__ void __launch_bounds__(256)
k_divergence(const T* __restrict__ grids, int lg, T c1, T c2, T* __restrict__ out) {
  const int64_t ncell = (int64_t)1 << (3 * lg);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncell) return;
  const int mask = (1 << lg) - 1;
  const int x = (int)(g >> (2 * lg)), y = (int)(g >> lg) & mask, z = (int)g & mask;
  auto at = [&](int k, int xx, int yy, int zz) {
    return grids[k * ncell + ((((int64_t)(xx & mask) << lg) | (yy & mask)) << lg | (zz & mask))];
  };
  T s = c1 * (at(0, x + 1, y, z) - at(0, x - 1, y, z)) +
        c2 * (at(0, x + 2, y, z) - at(0, x - 2, y, z));
  s += c1 * (at(1, x, y + 1, z) - at(1, x, y - 1, z)) +
       c2 * (at(1, x, y + 2, z) - at(1, x, y - 2, z));
  s += c1 * (at(2, x, y, z + 1) - at(2, x, y, z - 1)) +
       c2 * (at(2, x, y, z + 2) - at(2, x, y, z - 2));
  out[g] = s;
}

// pos_bar_k / m_k = sum_c grad W(x_k - c) [h^-3 psi(c) - lam_k . (D phi)(c)],
// to the sorted buffer (added by the pair adjoint) or, for the mesh-only
// call, times m_k straight to pos_bar in input order. Bricks of BX x BX x BZ
// cells, as the forward interpolation.
template <typename T, int BX, int BZ>
__global__ void __launch_bounds__(kThreads)
k_interp_vjp(const typename Vec<T>::v4* __restrict__ rec,
             const typename Vec<T>::v4* __restrict__ lam, const int32_t* __restrict__ skey,
             const int32_t* __restrict__ start, int ng, int lg, T inv_h, T inv_h3,
             const T* __restrict__ phi, const T* __restrict__ psi, T c1, T c2,
             typename Vec<T>::v4* __restrict__ acc_out, const int32_t* __restrict__ perm,
             int64_t n, double* __restrict__ pos_bar,
             const typename Vec<T>::v4* __restrict__ acc_pp) {
  constexpr int X1 = BX + 1, Z1 = BZ + 1;        // nodes touched per axis
  constexpr int X5 = BX + 5, Z5 = BZ + 5;        // with the two-node gradient halo
  __shared__ T ph[X5 * X5 * Z5];
  __shared__ T gr[3][X1 * X1 * Z1];
  __shared__ T ps[X1 * X1 * Z1];
  __shared__ InterpRuns<BX, BZ> R;
  const int mask = ng - 1, nbz = ng / BZ, nbx = ng / BX;
  const int b = blockIdx.x;
  const int bz0 = (b % nbz) * BZ, by0 = ((b / nbz) % nbx) * BX, bx0 = (b / (nbz * nbx)) * BX;
  for (int i = threadIdx.x; i < X5 * X5 * Z5; i += kThreads) {
    int nx = i / (X5 * Z5), ny = (i / Z5) % X5, nz = i % Z5;
    int gx = (bx0 - 2 + nx) & mask, gy = (by0 - 2 + ny) & mask, gz = (bz0 - 2 + nz) & mask;
    ph[i] = phi[(((int64_t)gx << lg | gy) << lg) | gz];
  }
  for (int i = threadIdx.x; i < X1 * X1 * Z1; i += kThreads) {
    int nx = i / (X1 * Z1), ny = (i / Z1) % X1, nz = i % Z1;
    int gx = (bx0 + nx) & mask, gy = (by0 + ny) & mask, gz = (bz0 + nz) & mask;
    ps[i] = inv_h3 * psi[(((int64_t)gx << lg | gy) << lg) | gz];
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
    const typename Vec<T>::v4 p = rec[s];
    const typename Vec<T>::v4 l = lam[s];
    int lx = r / BX, ly = r % BX, lz = (skey[s] & mask) - bz0;
    T tx = p.x * inv_h, ty = p.y * inv_h, tz = p.z * inv_h;
    T wx[2] = {T(1) - tx, tx}, wy[2] = {T(1) - ty, ty}, wz[2] = {T(1) - tz, tz};
    const T dw[2] = {-inv_h, inv_h};               // d/dx of (1 - t, t)
    T bx = 0, by = 0, bz = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const int q = ((lx + a) * X1 + (ly + c)) * Z1 + (lz + d);
          const T sv = ps[q] - (l.x * gr[0][q] + l.y * gr[1][q] + l.z * gr[2][q]);
          bx += dw[a] * wy[c] * wz[d] * sv;
          by += wx[a] * dw[c] * wz[d] * sv;
          bz += wx[a] * wy[c] * dw[d] * sv;
        }
    if (acc_out) {
      typename Vec<T>::v4 o;
      o.x = bx; o.y = by; o.z = bz; o.w = T(0);
      acc_out[s] = o;
    } else {
      // acc_pp: the pair adjoint's sorted cotangent, added here (the P3M
      // call whose mesh part ran beside the pair adjoint)
      double gx = (double)bx, gy = (double)by, gz = (double)bz;
      if (acc_pp) {
        const typename Vec<T>::v4 a = acc_pp[s];
        gx += (double)a.x; gy += (double)a.y; gz += (double)a.z;
      }
      const int64_t i = perm[s];
      const double m = (double)p.w;
      pos_bar[i] = m * gx;
      pos_bar[n + i] = m * gy;
      pos_bar[2 * n + i] = m * gz;
    }
  }
}

__global__ void __launch_bounds__(256)
k_drift_vjp(int64_t n, double* __restrict__ mom_bar, const double* __restrict__ pos_bar,
            const double* __restrict__ mass, double ms, double c) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double q = c / (mass ? mass[i] : ms);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double t = q * pos_bar[d * n + i];
    mom_bar[d * n + i] = mom_bar[d * n + i] + t;
  }
}

template <typename T>
void fd_coefficients(const p3m_plan* P, T& c1, T& c2) {
  const double h = P->h;
  if (P->prm.fd_order == 2) {
    c1 = T(1.0 / (2.0 * h));
    c2 = T(0);
  } else {
    c1 = T(8.0 / (12.0 * h));
    c2 = T(-1.0 / (12.0 * h));
  }
}

unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

template <typename T>
hipError_t launch_lambda_sort(p3m_plan* P, int64_t n, const double* force_bar) {
  k_lambda_sort<T><<<blocks_of(n, 256), 256, 0, P->stream>>>(
      n, P->ws.key, P->ws.rank, P->ws.start, force_bar, (typename Vec<T>::v4*)P->ws.lam);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_deposit_lambda(p3m_plan* P) {
  Workspace& W = P->ws;
  hipError_t e = launch_deposit3<T>(P, W.lam, W.lam_grid);
  if (e != hipSuccess) return e;
  T c1, c2;
  fd_coefficients(P, c1, c2);
  k_divergence<T><<<blocks_of(P->ncell, 256), 256, 0, P->stream>>>(
      (const T*)W.lam_grid, P->lg, c1, c2, (T*)W.grid2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp_vjp(p3m_plan* P, int64_t n, double* pos_bar, const void* acc_pp) {
  Workspace& W = P->ws;
  // bricks of 4 x 4 x 16 cells, as the forward interpolation (grids are at
  // least 16 cells on a side)
  constexpr int BX = 4, BZ = 16;
  const int nb = (int)(P->ncell / (BX * BX * BZ));
  T c1, c2;
  fd_coefficients(P, c1, c2);
  const double h = P->h;
  typename Vec<T>::v4* acc = pos_bar ? nullptr : (typename Vec<T>::v4*)W.acc_pm;
  k_interp_vjp<T, BX, BZ><<<nb, kThreads, 0, P->stream>>>(
      (const typename Vec<T>::v4*)W.rec, (const typename Vec<T>::v4*)W.lam, W.skey, W.start,
      P->ng, P->lg, T(1.0 / h), T(1.0 / (h * h * h)), (const T*)W.grid, (const T*)W.grid2, c1,
      c2, acc, W.perm, n, pos_bar, (const typename Vec<T>::v4*)acc_pp);
  return hipGetLastError();
}

hipError_t launch_drift_vjp(int64_t n, double* mom_bar, const double* pos_bar,
                            const double* mass, double ms, double c, hipStream_t s) {
  k_drift_vjp<<<blocks_of(n, 256), 256, 0, s>>>(n, mom_bar, pos_bar, mass, ms, c);
  return hipGetLastError();
}

template hipError_t launch_lambda_sort<float>(p3m_plan*, int64_t, const double*);
template hipError_t launch_lambda_sort<double>(p3m_plan*, int64_t, const double*);
template hipError_t launch_deposit_lambda<float>(p3m_plan*);
template hipError_t launch_deposit_lambda<double>(p3m_plan*);
template hipError_t launch_interp_vjp<float>(p3m_plan*, int64_t, double*, const void*);
template hipError_t launch_interp_vjp<double>(p3m_plan*, int64_t, double*, const void*);

}  // namespace p3m
