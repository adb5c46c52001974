// PP gravity with a tabulated Ewald correction (the guide's PP-with-Ewald
// kick: CONCEPT User's Guide, Ch. 5 entries use_Ewald and ewald_gridsize;
// Ch. 8 test kick_PP_with_Ewald), for small-N validation of the P3M path.
//
// Periodic field of a unit point mass at the origin with its images in a
// neutralising background, as a multiple of -G:
//   e(r) = sum_n r_n g(|r_n|) + (4 pi / L^3) sum_{k != 0} (k / k^2) e^{-k^2/(4 a^2)} sin(k . r),
//   g(s) = (erfc(a s) + (2 a s / sqrt(pi)) e^{-a^2 s^2}) / s^3,  r_n = r + n L,
// independent of the splitting a (here a = 2 / L, real images to erfc(7),
// Fourier terms to e^{-40}). The correction c(r) = e(r) - r / |r|^3 (the
// periodic images and the background, without the minimum-image Newtonian
// term) is smooth over the minimum-image cell and odd in each coordinate,
// so one octant [0, L/2]^3 of the ewald_gridsize^3 node grid (spacing
// L / ewald_gridsize) holds it: node (i, j, k), 0 <= i, j, k <= E/2. Between
// nodes it is trilinear in |r_d|, with the sign of r_d per component.
//
// The pair sum: F_i = -G m_i sum_{j != i} m_j [ r / (|r|^2 + eps^2)^(3/2) + c(r) ],
// r the minimum-image separation, all pairs, in FP64. A pair at zero
// separation contributes nothing.
#include "p3m_internal.h"

namespace p3m {
namespace {

constexpr int kEwI = 64;                       // i-particles per block of the pair sum
constexpr int kEwWaves = 16;                   // waves per block, each on a share of the j's
constexpr int kEwThreads = kEwI * kEwWaves;

// c(r) at one octant node, in FP64.
__global__ void __launch_bounds__(256)
k_ewald_table(int E, double box, double4* __restrict__ tab) {
  const int H = E / 2 + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= H * H * H) return;
  const int i = idx / (H * H), j = (idx / H) % H, k = idx % H;
  const double h = box / E;
  const double rx = i * h, ry = j * h, rz = k * h;
  const double a = 2.0 / box;
  const double kTwoOverSqrtPi = 1.1283791670955126;
  double cx = 0, cy = 0, cz = 0;
  if (i | j | k) {
    // real space: every image within erfc(7); the minimum image (n = 0) with
    // its Newtonian part removed, written so that small |r| does not cancel
    const double span = 7.0 / a;
    const int nmax = (int)ceil(span / box) + 1;
    for (int nx = -nmax; nx <= nmax; ++nx)
      for (int ny = -nmax; ny <= nmax; ++ny)
        for (int nz = -nmax; nz <= nmax; ++nz) {
          const double px = rx + nx * box, py = ry + ny * box, pz = rz + nz * box;
          const double s2 = px * px + py * py + pz * pz;
          const double s = sqrt(s2);
          if (s > span) continue;
          const double as = a * s;
          const double gauss = kTwoOverSqrtPi * as * exp(-as * as);
          double f;
          if (nx == 0 && ny == 0 && nz == 0)
            f = (gauss - erf(as)) / (s2 * s);     // erfc - 1 = -erf
          else
            f = (erfc(as) + gauss) / (s2 * s);
          cx += px * f;
          cy += py * f;
          cz += pz * f;
        }
    // Fourier space: (4 pi / L^3) sum (k / k^2) e^{-k^2/(4 a^2)} sin(k . r)
    const double kf = 2.0 * M_PI / box;
    const int mmax = (int)ceil(sqrt(40.0) * 2.0 * a / kf);
    const double pref = 4.0 * M_PI / (box * box * box);
    for (int mx = -mmax; mx <= mmax; ++mx)
      for (int my = -mmax; my <= mmax; ++my)
        for (int mz = -mmax; mz <= mmax; ++mz) {
          const int m2 = mx * mx + my * my + mz * mz;
          if (m2 == 0) continue;
          const double k2 = kf * kf * m2;
          const double w = exp(-k2 / (4.0 * a * a));
          if (w < 4e-18) continue;
          const double sn = sin(kf * (mx * rx + my * ry + mz * rz));
          const double c = pref * w / k2 * sn;
          cx += c * kf * mx;
          cy += c * kf * my;
          cz += c * kf * mz;
        }
  }
  tab[idx] = make_double4(cx, cy, cz, 0.0);
}

// The node table regrouped for the interpolation: entry (i, j, k), k < E/2,
// holds c at nodes (i, j, k) and (i, j, k + 1) as three double2 (48 bytes,
// 16-byte aligned), so the two z-corners of a trilinear cell come in three
// aligned 16-byte loads instead of the four that two padded double4 nodes
// take.
__global__ void __launch_bounds__(256)
k_ewald_zpairs(int E, const double4* __restrict__ tab, double2* __restrict__ zp) {
  const int H = E / 2 + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= H * H * (H - 1)) return;
  const int col = idx / (H - 1), k = idx % (H - 1);
  const double4 a = tab[col * H + k], b = tab[col * H + k + 1];
  zp[3 * idx + 0] = make_double2(a.x, a.y);
  zp[3 * idx + 1] = make_double2(a.z, b.x);
  zp[3 * idx + 2] = make_double2(b.y, b.z);
}

// Trilinear c(r) from the octant table (z-pair layout), r a minimum-image
// separation.
__device__ __forceinline__ double3 ewald_corr(const double2* __restrict__ zp, int E,
                                              double inv_h, double dx, double dy, double dz) {
  const int H = E / 2 + 1;
  // clamped to the octant (also keeps a non-finite input inside the table)
  const double top = H - 1.0;
  const double ux = fmin(fabs(dx) * inv_h, top), uy = fmin(fabs(dy) * inv_h, top),
               uz = fmin(fabs(dz) * inv_h, top);
  const int ix = min((int)ux, H - 2), iy = min((int)uy, H - 2), iz = min((int)uz, H - 2);
  const double tx = ux - ix, ty = uy - iy, tz = uz - iz;
  double3 c = make_double3(0.0, 0.0, 0.0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double wxy = (a ? tx : 1.0 - tx) * (b ? ty : 1.0 - ty);
      const double2* e = zp + 3 * (((ix + a) * H + (iy + b)) * (H - 1) + iz);
      const double2 v0 = e[0], v1 = e[1], v2 = e[2];
      const double w0 = wxy * (1.0 - tz), w1 = wxy * tz;
      c.x += w0 * v0.x + w1 * v1.y;
      c.y += w0 * v0.y + w1 * v2.x;
      c.z += w0 * v1.x + w1 * v2.y;
    }
  c.x = dx < 0 ? -c.x : c.x;
  c.y = dy < 0 ? -c.y : c.y;
  c.z = dz < 0 ? -c.z : c.z;
  return c;
}

__device__ __forceinline__ double min_image(double d, double box, double inv_box) {
  return d - box * rint(d * inv_box);
}

// All pairs, j tiles in LDS. A block holds kEwI i-particles, one per lane,
// and kEwWaves waves that each take their own contiguous share of every j
// tile, so a small n still spreads over every CU with several waves per SIMD
// to cover the latency of the table's gathers. The i- and j-particles are
// both taken in cell order (order[s] is the input index of sorted slot s): a
// block's i's sit in a few neighbouring cells, so for one broadcast j its
// lanes' separations fall on nearby table nodes that share cache lines, and
// consecutive j's are neighbours, so consecutive steps revisit those lines.
// The waves' partial sums are added in wave order at the end (no atomics),
// so the summation order is the sorted order. Within a cell that order is
// the binning's atomic rank, which may differ between calls: the result can
// change at rounding level from call to call, like the P3M force.
__global__ void __launch_bounds__(kEwThreads)
k_pp_ewald(int64_t n, const double* __restrict__ pos, const double* __restrict__ mass,
           double ms, double box, double eps2, double negG, const double2* __restrict__ tab,
           int E, const int32_t* __restrict__ order, void* __restrict__ force,
           int force_fp32) {
  __shared__ double4 tile[kEwThreads];
  __shared__ double red[3][kEwWaves][kEwI];
  const int lane = threadIdx.x % kEwI, wave = threadIdx.x / kEwI;
  const int64_t slot = (int64_t)blockIdx.x * kEwI + lane;
  const bool live = slot < n;
  const int64_t i = live ? (int64_t)order[slot] : -1;
  const double xi = live ? pos[i] : 0.0, yi = live ? pos[n + i] : 0.0,
               zi = live ? pos[2 * n + i] : 0.0;
  const double inv_box = 1.0 / box, inv_h = E / box;
  double ax = 0, ay = 0, az = 0;
  for (int64_t j0 = 0; j0 < n; j0 += kEwThreads) {
    const int64_t jl = j0 + threadIdx.x;
    __syncthreads();
    if (jl < n) {
      const int64_t j = order[jl];
      tile[threadIdx.x] = make_double4(pos[j], pos[n + j], pos[2 * n + j], mass ? mass[j] : ms);
    }
    __syncthreads();
    // this wave's entries [tb, tb + cnt) of the tile (cnt <= 0 past the end)
    const int tb = wave * kEwI;
    const int64_t jb = j0 + tb;
    const int cnt = (int)min<int64_t>(kEwI, n - jb);
    for (int t = 0; t < cnt; ++t) {
      const double4 pj = tile[tb + t];
      const double dx = min_image(xi - pj.x, box, inv_box);
      const double dy = min_image(yi - pj.y, box, inv_box);
      const double dz = min_image(zi - pj.z, box, inv_box);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (!live || jb + t == slot || r2 == 0.0) continue;
      const double inv = rsqrt(r2 + eps2);
      const double w = inv * inv * inv;
      const double3 c = ewald_corr(tab, E, inv_h, dx, dy, dz);
      ax += pj.w * (dx * w + c.x);
      ay += pj.w * (dy * w + c.y);
      az += pj.w * (dz * w + c.z);
    }
  }
  red[0][wave][lane] = ax;
  red[1][wave][lane] = ay;
  red[2][wave][lane] = az;
  __syncthreads();
  if (wave != 0 || !live) return;
  ax = ay = az = 0;
#pragma unroll
  for (int w = 0; w < kEwWaves; ++w) {
    ax += red[0][w][lane];
    ay += red[1][w][lane];
    az += red[2][w][lane];
  }
  const double m = mass ? mass[i] : ms;
  const double fx = negG * m * ax, fy = negG * m * ay, fz = negG * m * az;
  if (force_fp32) {
    float* F = (float*)force;
    F[i] = (float)fx;
    F[n + i] = (float)fy;
    F[2 * n + i] = (float)fz;
  } else {
    double* F = (double*)force;
    F[i] = fx;
    F[n + i] = fy;
    F[2 * n + i] = fz;
  }
}

// The interpolated correction at given minimum-image separations.
__global__ void __launch_bounds__(256)
k_ewald_eval(int64_t npts, const double* __restrict__ r, double box,
             const double2* __restrict__ tab, int E, double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double inv_box = 1.0 / box;
  const double dx = min_image(r[p], box, inv_box), dy = min_image(r[npts + p], box, inv_box),
               dz = min_image(r[2 * npts + p], box, inv_box);
  const double3 c = ewald_corr(tab, E, E / box, dx, dy, dz);
  out[p] = c.x;
  out[npts + p] = c.y;
  out[2 * npts + p] = c.z;
}

}  // namespace

hipError_t launch_ewald_table(p3m_plan* P) {
  const int E = P->prm.ewald_gridsize, H = E / 2 + 1;
  const int total = H * H * H;
  k_ewald_table<<<(total + 255) / 256, 256, 0, P->stream>>>(E, P->prm.box,
                                                           (double4*)P->ws.ewald_tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int pairs = H * H * (H - 1);
  k_ewald_zpairs<<<(pairs + 255) / 256, 256, 0, P->stream>>>(
      E, (const double4*)P->ws.ewald_tab, (double2*)P->ws.ewald_zpair);
  return hipGetLastError();
}

hipError_t launch_pp_ewald(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                           double ms, const int32_t* order, void* force, int force_fp32) {
  const unsigned blocks = (unsigned)((n + kEwI - 1) / kEwI);
  k_pp_ewald<<<blocks, kEwThreads, 0, P->stream>>>(
      n, pos, mass, ms, P->prm.box, P->eps * P->eps, -P->prm.G,
      (const double2*)P->ws.ewald_zpair, P->prm.ewald_gridsize, order, force, force_fp32);
  return hipGetLastError();
}

hipError_t launch_ewald_eval(p3m_plan* P, int64_t npts, const double* r, double* out) {
  k_ewald_eval<<<(unsigned)((npts + 255) / 256), 256, 0, P->stream>>>(
      npts, r, P->prm.box, (const double2*)P->ws.ewald_zpair, P->prm.ewald_gridsize, out);
  return hipGetLastError();
}

}  // namespace p3m
