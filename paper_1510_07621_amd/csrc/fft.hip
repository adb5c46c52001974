// Hand-written 3-D real-to-complex FFT Poisson solve on the PM grid.
//
// Layout: the real grid is [x][y][z] (z fastest, ng^3 values); the spectrum
// is [kx][ky][kz] with kz = 0..ng/2, each (kx, ky) row of ng/2 + 1 values
// padded to spec_stride(ng) so that rows start on cache-line boundaries.
// Five passes, each reading and writing the grid once, each 1-D transform
// held by one workgroup:
//   1. z, real -> complex: each z-line of ng reals is transformed as ng/2
//      complex values (even samples real, odd samples imaginary) and the
//      ng/2 + 1 outputs are separated with the usual split step;
//   2. y, complex forward;
//   3. x, complex forward, multiply by the Green's function, x inverse (fused);
//   4. y, complex inverse;
//   5. z, complex -> real (the split step in reverse, then ng/2 complex inverse).
// Transforms are radix-2: decimation in time (bit-reversed input, natural
// output) forward and decimation in frequency (natural input, bit-reversed
// output) inverse, so no pass needs a separate reordering step; three levels
// at a time run in registers between LDS exchanges, the first level group of
// a transform loading straight from global memory and the last storing
// straight to it. All
// transforms are unnormalised; the 1/ng^3 of the inverse is folded into the
// Green's function
//     G(k) = -4 pi G exp(-k^2 r_s^2) / (k^2 W(k)^p) / ng^3,  G(0) = 0,
//     W(k) = prod_d sinc^2(pi n_d / ng),  k = 2 pi n / box,
// which is separable apart from 1/k^2: G = c * e(nx) e(ny) e(nz) / (k2(nx) +
// k2(ny) + k2(nz)) with per-axis tables e(n) = exp(-k_n^2 r_s^2) / W1(n)^p and
// k2(n) = k_n^2, built once per plan.
#include "p3m_internal.h"

namespace p3m {
namespace {

constexpr int kThreads = 256;
constexpr int kLdsElems = 2048;   // complex values staged per block
// LDS index of staged element i: one complex of padding after every
// 2^kPadShift, so that the bit-reversed and the column-strided accesses of
// neighbouring threads fall in different banks.
constexpr int kPadShift = 4;      // (3 and 5 measured the same; none 2-4 % slower at 256^3)
__device__ __forceinline__ int pd(int i) { return i + (i >> kPadShift); }
__host__ __device__ inline int padded(int elems) { return elems + (elems >> kPadShift) + 1; }

// The twiddle table (ng/2 values) is staged in LDS after a block's values,
// so the butterflies read it there rather than through the vector cache.
template <typename T2>
__device__ __forceinline__ T2* stage_twiddles(T2* buf, int staged, const T2* __restrict__ tw,
                                              int ng) {
  T2* t = buf + padded(staged);
  for (int i = threadIdx.x; i < (ng >> 1); i += blockDim.x) t[i] = tw[i];
  return t;
}

template <typename T2>
__device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  T2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

__device__ __forceinline__ int brev(int v, int bits) {
  return bits ? (int)(__brev((unsigned)v) >> (32 - bits)) : 0;
}

// The radix-2 levels run kGroup at a time: a task holds in registers the 2^g
// elements that g consecutive levels l0 .. l0 + g - 1 combine among
// themselves (positions p0 + m 2^l0, m < 2^g, p0 = base + j with j < 2^l0),
// does the g levels' butterflies and stores them back, so a transform of
// length 2^L takes ceil(L / kGroup) exchanges instead of L. Every element
// sees the same butterflies with the same twiddles, in the same level
// order, as one level at a time. Twiddles: tw[k] = exp(-2 pi i k / twn),
// k < twn/2; the inverse uses their conjugates.
constexpr int kGroup = 3;    // measured: 2 and 4 levels per group were slower (256^3: 0.35, 0.55 ms)

// Decimation in time (bit-reversed input, natural output): levels ascending.
template <typename T, bool INV>
__device__ __forceinline__ void dit_levels(typename Vec<T>::v2 (&x)[1 << kGroup], int g, int j,
                                           int l0, const typename Vec<T>::v2* tw, int twn) {
  using T2 = typename Vec<T>::v2;
#pragma unroll
  for (int t = 0; t < kGroup; ++t) {
    if (t >= g) break;
    const int tstride = twn >> (l0 + t + 1);
#pragma unroll
    for (int m = 0; m < (1 << kGroup); ++m) {
      if (m >= (1 << g) || (m & (1 << t))) continue;
      const int m1 = m | (1 << t);
      const int r = j + ((m & ((1 << t) - 1)) << l0);
      T2 w = tw[r * tstride];
      if (INV) w.y = -w.y;
      const T2 a = x[m], c = cmul(x[m1], w);
      x[m].x = a.x + c.x; x[m].y = a.y + c.y;
      x[m1].x = a.x - c.x; x[m1].y = a.y - c.y;
    }
  }
}

// Decimation in frequency (natural input, bit-reversed output): levels
// descending.
template <typename T, bool INV>
__device__ __forceinline__ void dif_levels(typename Vec<T>::v2 (&x)[1 << kGroup], int g, int j,
                                           int l0, const typename Vec<T>::v2* tw, int twn) {
  using T2 = typename Vec<T>::v2;
#pragma unroll
  for (int t = kGroup - 1; t >= 0; --t) {
    if (t >= g) continue;
    const int tstride = twn >> (l0 + t + 1);
#pragma unroll
    for (int m = 0; m < (1 << kGroup); ++m) {
      if (m >= (1 << g) || (m & (1 << t))) continue;
      const int m1 = m | (1 << t);
      const int r = j + ((m & ((1 << t) - 1)) << l0);
      T2 w = tw[r * tstride];
      if (INV) w.y = -w.y;
      const T2 a = x[m], c = x[m1];
      T2 d;
      x[m].x = a.x + c.x; x[m].y = a.y + c.y;
      d.x = a.x - c.x; d.y = a.y - c.y;
      x[m1] = cmul(d, w);
    }
  }
}

// One level group (levels l0 .. l0 + g - 1) of nb transforms of length
// len = 2^lglen held line by line (element i of line b at p = b len + i):
// LD(p) gives element p, ST(p, v) takes it back. The z passes.
template <typename T, bool DIT, bool INV, typename LD, typename ST>
__device__ __forceinline__ void line_group(int nb, int len, int lglen, int l0, int g,
                                           const typename Vec<T>::v2* tw, int twn, LD ld,
                                           ST st) {
  using T2 = typename Vec<T>::v2;
  const int tasks = len >> g;                 // per transform
  const int lgt = lglen - g;
  for (int q = threadIdx.x; q < nb * tasks; q += blockDim.x) {
    const int bi = q >> lgt, rem = q & (tasks - 1);
    const int j = rem & ((1 << l0) - 1), base = (rem >> l0) << (l0 + g);
    const int p0 = bi * len + base + j;
    T2 x[1 << kGroup];
#pragma unroll
    for (int m = 0; m < (1 << kGroup); ++m)
      if (m < (1 << g)) x[m] = ld(p0 + (m << l0));
    if (DIT) dit_levels<T, INV>(x, g, j, l0, tw, twn);
    else dif_levels<T, INV>(x, g, j, l0, tw, twn);
#pragma unroll
    for (int m = 0; m < (1 << kGroup); ++m)
      if (m < (1 << g)) st(p0 + (m << l0), x[m]);
  }
}

template <typename T2>
struct LineLds {
  T2* buf;
  __device__ T2 operator()(int p) const { return buf[pd(p)]; }
  __device__ void operator()(int p, T2 v) const { buf[pd(p)] = v; }
};

// Pass 1: real z-lines -> half spectra. lines per block = nl.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fft_z_r2c(const T* __restrict__ grid, typename Vec<T>::v2* __restrict__ spec, int ng, int lg,
            int nl, const typename Vec<T>::v2* __restrict__ tw) {
  using T2 = typename Vec<T>::v2;
  extern __shared__ unsigned char smem_raw[];
  T2* buf = reinterpret_cast<T2*>(smem_raw);
  const int M = ng >> 1, lgM = lg - 1;
  const int64_t line0 = (int64_t)blockIdx.x * nl;
  const int Ms = spec_stride(ng);
  const T2* in = reinterpret_cast<const T2*>(grid);
  const T2* twl = stage_twiddles(buf, nl * M, tw, ng);
  const LineLds<T2> lds{buf};
  // DIT, levels from the bottom up; the first group reads its (bit-reversed)
  // inputs straight from global memory, with the twiddles from there too
  auto gin = [&](int p) {
    const int b = p >> lgM, i = p & (M - 1);
    return in[(line0 + b) * M + brev(i, lgM)];
  };
  line_group<T, true, false>(nl, M, lgM, 0, min(kGroup, lgM), tw, ng, gin, lds);
  __syncthreads();
  for (int l0 = kGroup; l0 < lgM; l0 += kGroup) {
    line_group<T, true, false>(nl, M, lgM, l0, min(kGroup, lgM - l0), twl, ng, lds, lds);
    __syncthreads();
  }
  const int M1 = M + 1;
  for (int idx = threadIdx.x; idx < nl * M1; idx += kThreads) {
    int b = idx / M1, k = idx - b * M1;
    T2 zk = buf[pd(b * M + (k & (M - 1)))];
    T2 zc = buf[pd(b * M + ((M - k) & (M - 1)))];
    zc.y = -zc.y;
    // E = (Z_k + conj Z_{M-k}) / 2,  O = (Z_k - conj Z_{M-k}) / 2i
    T2 E, O;
    E.x = T(0.5) * (zk.x + zc.x); E.y = T(0.5) * (zk.y + zc.y);
    O.x = T(0.5) * (zk.y - zc.y); O.y = -T(0.5) * (zk.x - zc.x);
    T2 w;
    if (k < M) w = twl[k]; else { w.x = T(-1); w.y = T(0); }
    T2 wo = cmul(w, O);
    T2 X;
    X.x = E.x + wo.x; X.y = E.y + wo.y;
    spec[(line0 + b) * Ms + k] = X;
  }
}

// Pass 5: half spectra -> real z-lines (unnormalised inverse).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fft_z_c2r(const typename Vec<T>::v2* __restrict__ spec, T* __restrict__ grid, int ng, int lg,
            int nl, const typename Vec<T>::v2* __restrict__ tw) {
  using T2 = typename Vec<T>::v2;
  extern __shared__ unsigned char smem_raw[];
  T2* buf = reinterpret_cast<T2*>(smem_raw);
  const int M = ng >> 1, lgM = lg - 1, Ms = spec_stride(ng);
  const int64_t line0 = (int64_t)blockIdx.x * nl;
  for (int idx = threadIdx.x; idx < nl * M; idx += kThreads) {
    int b = idx >> lgM, k = idx & (M - 1);
    const T2* row = spec + (line0 + b) * Ms;
    T2 xk = row[k], xc = row[M - k];
    xc.y = -xc.y;
    // E = X_k + conj X_{M-k},  O = (X_k - conj X_{M-k}) * conj(W^k),  Z = E + i O
    T2 E, D, w = tw[k];
    E.x = xk.x + xc.x; E.y = xk.y + xc.y;
    D.x = xk.x - xc.x; D.y = xk.y - xc.y;
    w.y = -w.y;
    T2 O = cmul(D, w);
    T2 Z;
    Z.x = E.x - O.y; Z.y = E.y + O.x;
    buf[pd(b * M + k)] = Z;
  }
  const T2* twl = stage_twiddles(buf, nl * M, tw, ng);
  __syncthreads();
  // DIF, levels from the top down; the last group stores its (bit-reversed)
  // outputs straight to global memory
  T2* out = reinterpret_cast<T2*>(grid);
  auto gout = [&](int p, T2 v) {
    const int b = p >> lgM, i = p & (M - 1);
    out[(line0 + b) * M + brev(i, lgM)] = v;
  };
  const LineLds<T2> lds{buf};
  for (int k = 0; k < lgM; k += kGroup) {
    const int g = min(kGroup, lgM - k), l0 = lgM - k - g;
    if (l0 > 0) {
      line_group<T, false, true>(nl, M, lgM, l0, g, twl, ng, lds, lds);
      __syncthreads();
    } else {
      line_group<T, false, true>(nl, M, lgM, l0, g, twl, ng, lds, gout);
    }
  }
}


// ---- Column passes (y and x): kc columns of one plane per block ----
// A block transforms kc columns (adjacent kz values) of length ng = 2^lg
// along y or x. In LDS element i of column c sits at pd(i kc + c), so the kc
// columns of one row are adjacent. The levels go in groups: the lowest
// lg mod 3 (3 if none) first, then three at a time. A task is one column
// and the 2^g elements of one level group; consecutive threads take
// consecutive columns, so the kc columns of a row move as one contiguous
// run of global memory. The first group of a transform loads its elements
// from global memory and the last stores them there: only the groups
// between pass through LDS (at 256 points, one exchange per transform; the
// x pass's forward top group, the Green's function and the inverse top
// group share one task).
__device__ __forceinline__ int low_group(int lg) {
  const int r = lg % kGroup;
  return r ? r : kGroup;
}

// Work item of a column-pass block. Workgroups go to the 8 XCDs in turn
// (block b to XCD b mod 8), each XCD with its own L2, and two neighbouring
// chunks of a row share cache lines (an FP32 chunk of 8 columns is half a
// 128-byte line); so items 2i and 2i + 1 run as blocks 16s + r and
// 16s + r + 8, on one XCD one after the other. The block count is a multiple
// of 16 (ng is).
__device__ __forceinline__ int col_item() {
  const int b = blockIdx.x, r = b & 15;
  return (b & ~15) + 2 * (r & 7) + (r >> 3);
}

struct ColGroup {
  int l0, g;
};
// Level group k (ascending from the bottom) of a length-2^lg transform.
__device__ __forceinline__ ColGroup col_group_levels(int lg, int k) {
  const int low = low_group(lg);
  return k == 0 ? ColGroup{0, low} : ColGroup{low + kGroup * (k - 1), kGroup};
}
__device__ __forceinline__ int col_groups(int lg) { return 1 + (lg - low_group(lg)) / kGroup; }

// One level group over the block's columns: LD(p, c) gives element p of
// column c, MID(x, p0, l0, g, c, j) acts on the task's values after the
// butterflies, ST(p, c, v) takes them back.
template <typename T, bool DIT, bool INV, typename LD, typename MID, typename ST>
__device__ __forceinline__ void col_group(int kc, int lgkc, int lg, ColGroup lv,
                                          const typename Vec<T>::v2* tw, int twn, LD ld, MID mid,
                                          ST st) {
  using T2 = typename Vec<T>::v2;
  const int l0 = lv.l0, g = lv.g;
  const int tasks = kc << (lg - g);
  for (int q = threadIdx.x; q < tasks; q += blockDim.x) {
    const int c = q & (kc - 1), rem = q >> lgkc;
    const int j = rem & ((1 << l0) - 1), base = (rem >> l0) << (l0 + g);
    const int p0 = base + j;
    T2 x[1 << kGroup];
#pragma unroll
    for (int m = 0; m < (1 << kGroup); ++m)
      if (m < (1 << g)) x[m] = ld(p0 + (m << l0), c);
    if (DIT) dit_levels<T, INV>(x, g, j, l0, tw, twn);
    else dif_levels<T, INV>(x, g, j, l0, tw, twn);
    mid(x, p0, l0, g, c, j);
#pragma unroll
    for (int m = 0; m < (1 << kGroup); ++m)
      if (m < (1 << g)) st(p0 + (m << l0), c, x[m]);
  }
}

struct NoMid {
  template <typename X>
  __device__ void operator()(X&, int, int, int, int, int) const {}
};

// LDS access of the column passes.
template <typename T2>
struct ColLds {
  T2* buf;
  int kc;
  __device__ T2 operator()(int p, int c) const { return buf[pd(p * kc + c)]; }
  __device__ void operator()(int p, int c, T2 v) const { buf[pd(p * kc + c)] = v; }
};

// Global access of the column passes: element p of column c is row
// (BREV ? bit-reverse of p : p) of the plane, at row stride rs; columns at
// or past kn (the spectrum's last, narrower chunk) read as zero and are not
// written.
template <typename T2, bool BREV>
struct ColGlobal {
  T2* base;
  int64_t rs;
  int kn, lg;
  __device__ T2 operator()(int p, int c) const {
    T2 v;
    if (c < kn) {
      v = base[(int64_t)(BREV ? brev(p, lg) : p) * rs + c];
    } else {
      v.x = 0; v.y = 0;
    }
    return v;
  }
  __device__ void operator()(int p, int c, T2 v) const {
    if (c < kn) base[(int64_t)(BREV ? brev(p, lg) : p) * rs + c] = v;
  }
};

// Forward (DIT: bit-reversed rows in, natural rows out) or inverse (DIF:
// natural rows in, bit-reversed rows out) column transforms, with the top
// group's values passed through MID before they are stored (the x pass's
// Green's function and inverse, the power spectrum's shell sums).
template <typename T, bool INV, typename MID, typename TOPST>
__device__ __forceinline__ void col_transform(typename Vec<T>::v2* buf, typename Vec<T>::v2* gbase,
                                              int64_t rs, int kn, int kc, int lg,
                                              const typename Vec<T>::v2* tw,
                                              const typename Vec<T>::v2* twl, MID mid,
                                              TOPST topst) {
  using T2 = typename Vec<T>::v2;
  const int ng = 1 << lg, lgkc = __builtin_ctz(kc), ngr = col_groups(lg);
  const ColLds<T2> lds{buf, kc};
  if (!INV) {
    const ColGlobal<T2, true> in{gbase, rs, kn, lg};
    // the bottom group reads the twiddles from global memory: the barrier
    // after it is the one that makes the staged copy visible
    col_group<T, true, false>(kc, lgkc, lg, col_group_levels(lg, 0), tw, ng, in, NoMid{}, lds);
    __syncthreads();
    for (int k = 1; k < ngr - 1; ++k) {
      col_group<T, true, false>(kc, lgkc, lg, col_group_levels(lg, k), twl, ng, lds, NoMid{},
                                lds);
      __syncthreads();
    }
    col_group<T, true, false>(kc, lgkc, lg, col_group_levels(lg, ngr - 1), twl, ng, lds, mid,
                              topst);
  } else {
    const ColGlobal<T2, false> in{gbase, rs, kn, lg};
    col_group<T, false, true>(kc, lgkc, lg, col_group_levels(lg, ngr - 1), tw, ng, in, mid,
                              lds);
    __syncthreads();
    for (int k = ngr - 2; k > 0; --k) {
      col_group<T, false, true>(kc, lgkc, lg, col_group_levels(lg, k), twl, ng, lds, NoMid{},
                                lds);
      __syncthreads();
    }
    const ColGlobal<T2, true> out{gbase, rs, kn, lg};
    col_group<T, false, true>(kc, lgkc, lg, col_group_levels(lg, 0), twl, ng, lds, NoMid{}, out);
  }
}

// Pass 2 / 4: complex transform along y for one x-plane and a chunk of kc
// kz-columns.
template <typename T, bool INV>
__global__ void __launch_bounds__(kThreads)
k_fft_y(typename Vec<T>::v2* __restrict__ spec, int ng, int lg, int kc,
        const typename Vec<T>::v2* __restrict__ tw) {
  using T2 = typename Vec<T>::v2;
  extern __shared__ unsigned char smem_raw[];
  T2* buf = reinterpret_cast<T2*>(smem_raw);
  const int M1 = (ng >> 1) + 1, Ms = spec_stride(ng);
  const int nchunk = (M1 + kc - 1) / kc;
  const int item = col_item();
  const int x = item / nchunk, kz0 = (item % nchunk) * kc;
  const int kn = min(kc, M1 - kz0);
  T2* plane = spec + (int64_t)x * ng * Ms + kz0;
  const T2* twl = stage_twiddles(buf, kc * ng, tw, ng);
  if (INV)
    col_transform<T, true>(buf, plane, Ms, kn, kc, lg, tw, twl, NoMid{}, ColLds<T2>{buf, kc});
  else
    col_transform<T, false>(buf, plane, Ms, kn, kc, lg, tw, twl, NoMid{},
                            ColGlobal<T2, false>{plane, Ms, kn, lg});
}

// Pass 3: forward x transform, Green's function, inverse x transform, for one
// y-row and a chunk of kc kz-columns. The forward transform's top level group
// ends with the modes in natural order, so the same task multiplies them by
// G and runs the inverse's top group before they go back to LDS.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fft_x_green(typename Vec<T>::v2* __restrict__ spec, int ng, int lg, int kc,
              const typename Vec<T>::v2* __restrict__ tw, const T* __restrict__ etab,
              const T* __restrict__ k2tab, T gconst) {
  using T2 = typename Vec<T>::v2;
  extern __shared__ unsigned char smem_raw[];
  T2* buf = reinterpret_cast<T2*>(smem_raw);
  const int M1 = (ng >> 1) + 1, Ms = spec_stride(ng);
  const int nchunk = (M1 + kc - 1) / kc;
  const int item = col_item();
  const int y = item / nchunk, kz0 = (item % nchunk) * kc;
  const int kn = min(kc, M1 - kz0);
  const int64_t xs = (int64_t)ng * Ms;
  T2* col = spec + (int64_t)y * Ms + kz0;
  const T2* twl = stage_twiddles(buf, kc * ng, tw, ng);
  const T ey = etab[y], k2y = k2tab[y];
  auto green = [&](T2 (&x)[1 << kGroup], int p0, int l0, int g, int c, int j) {
    const int kz = kz0 + c;
#pragma unroll
    for (int m = 0; m < (1 << kGroup); ++m) {
      if (m >= (1 << g)) continue;
      const int kx = p0 + (m << l0);
      T gk = T(0);
      if (c < kn) {
        T k2 = k2tab[kx] + k2y + k2tab[kz];
        if (k2 > T(0)) gk = gconst * etab[kx] * ey * etab[kz] / k2;
      }
      x[m].x *= gk; x[m].y *= gk;
    }
    dif_levels<T, true>(x, g, j, l0, twl, ng);
  };
  const ColLds<T2> lds{buf, kc};
  col_transform<T, false>(buf, col, xs, kn, kc, lg, tw, twl, green, lds);
  __syncthreads();
  // the inverse below its top group
  const int lgkc = __builtin_ctz(kc), ngr = col_groups(lg);
  for (int k = ngr - 2; k > 0; --k) {
    col_group<T, false, true>(kc, lgkc, lg, col_group_levels(lg, k), twl, ng, lds, NoMid{}, lds);
    __syncthreads();
  }
  const ColGlobal<T2, true> out{col, xs, kn, lg};
  col_group<T, false, true>(kc, lgkc, lg, col_group_levels(lg, 0), twl, ng, lds, NoMid{}, out);
}

// Power spectrum: forward x transform of one y-row and a chunk of kc
// kz-columns (after the z and y forward passes), then each mode's |rho_k|^2,
// divided by W(k)^2 when deconvolving, is added with its full-space
// multiplicity (1 on the kz = 0 and Nyquist planes, else 2) into its shell
// b = floor(|n| - 1/2): acc = [power sums | |n| sums | mode counts][nbins],
// then the top-hat-weighted sum for sigma and rho_0 (the k = 0 value).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fft_x_power(const typename Vec<T>::v2* __restrict__ spec, int ng, int lg, int kc,
              const typename Vec<T>::v2* __restrict__ tw, int deconv, int nbins, double kr_unit,
              double* __restrict__ acc) {
  using T2 = typename Vec<T>::v2;
  extern __shared__ unsigned char smem_raw[];
  T2* buf = reinterpret_cast<T2*>(smem_raw);
  __shared__ double hist[3 * kMaxPowerBins + 1];
  const int M1 = (ng >> 1) + 1, Ms = spec_stride(ng);
  const int nchunk = (M1 + kc - 1) / kc;
  const int item = col_item();
  const int y = item / nchunk, kz0 = (item % nchunk) * kc;
  const int kn = min(kc, M1 - kz0);
  const int64_t xs = (int64_t)ng * Ms;
  // (read only: the transform's global stores go to LDS or to the sums)
  T2* col = const_cast<T2*>(spec) + (int64_t)y * Ms + kz0;
  for (int i = threadIdx.x; i < 3 * nbins + 1; i += kThreads) hist[i] = 0.0;
  const T2* twl = stage_twiddles(buf, kc * ng, tw, ng);
  const int half = ng >> 1;
  const int ny = y < half ? y : y - ng;
  auto shells = [&](int kx, int c, T2 v) {
    const int kz = kz0 + c;
    if (c >= kn) return;
    const int nx = kx < half ? kx : kx - ng;
    const int n2 = nx * nx + ny * ny + kz * kz;
    if (n2 == 0) {
      acc[3 * nbins + 1] = (double)v.x;             // rho_0: one thread of one block
      return;
    }
    double pw = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    if (deconv) {
      double w = 1.0;
      const int nn[3] = {nx, ny, kz};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (nn[d] != 0) {
          const double a = (double)nn[d] / ng;
          const double sc = sinpi(a) / (M_PI * a);
          w *= sc * sc;
        }
      pw /= w * w;
    }
    const double mult = (kz == 0 || kz == half) ? 1.0 : 2.0;
    const double nabs = sqrt((double)n2);
    const int b = (int)floor(nabs - 0.5);
    if (b >= 0 && b < nbins) {
      atomicAdd(&hist[b], mult * pw);
      atomicAdd(&hist[nbins + b], mult * nabs);
      atomicAdd(&hist[2 * nbins + b], mult);
    }
    const double x = kr_unit * nabs;
    double wt;
    if (x < 1e-3) {
      wt = 1.0 - x * x / 10.0;
    } else {
      double sx, cx;
      sincos(x, &sx, &cx);
      wt = 3.0 * (sx - x * cx) / (x * x * x);
    }
    atomicAdd(&hist[3 * nbins], mult * pw * wt * wt);
  };
  // The transform's top level group stores the modes to LDS; the shell sums
  // (double precision, kept out of the transform's registers) then read them,
  // consecutive threads on consecutive columns. (The histogram's clearing is
  // ordered before the sums by the transform's barriers.)
  col_transform<T, false>(buf, col, xs, kn, kc, lg, tw, twl, NoMid{}, ColLds<T2>{buf, kc});
  __syncthreads();
  for (int idx = threadIdx.x; idx < ng * kc; idx += kThreads) {
    const int kx = idx / kc, c = idx - kx * kc;
    shells(kx, c, buf[pd(idx)]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * nbins + 1; i += kThreads)
    if (hist[i] != 0.0) atomicAdd(&acc[i], hist[i]);
}


// Shell averages and sigma from the accumulated sums.
__global__ void __launch_bounds__(256)
k_power_finish(const double* __restrict__ acc, int nbins, double box, double* __restrict__ k_out,
               double* __restrict__ p_out, double* __restrict__ m_out,
               double* __restrict__ sigma_out) {
  const double rho0 = acc[3 * nbins + 1];
  const double inv2 = 1.0 / (rho0 * rho0);
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    const double m = acc[2 * nbins + b];
    m_out[b] = m;
    p_out[b] = m > 0 ? box * box * box * acc[b] * inv2 / m : 0.0;
    k_out[b] = m > 0 ? 2.0 * M_PI / box * acc[nbins + b] / m : 0.0;
  }
  if (threadIdx.x == 0 && sigma_out) sigma_out[0] = sqrt(acc[3 * nbins] * inv2);
}

template <typename T>
__global__ void k_tables(int ng, double box, double r_s, int deconv_power,
                         typename Vec<T>::v2* __restrict__ tw, T* __restrict__ etab,
                         T* __restrict__ k2tab) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  if (i < ng / 2) {
    double s, c;
    sincospi(2.0 * i / ng, &s, &c);
    typename Vec<T>::v2 w;
    w.x = (T)c; w.y = (T)(-s);
    tw[i] = w;
  }
  int n = i < ng / 2 ? i : i - ng;
  double k = 2.0 * M_PI * n / box;
  double sinc = n == 0 ? 1.0 : sinpi((double)n / ng) / (M_PI * (double)n / ng);
  double w1 = sinc * sinc;
  double e = exp(-k * k * r_s * r_s);
  for (int p = 0; p < deconv_power; ++p) e /= w1;
  etab[i] = (T)e;
  k2tab[i] = (T)(k * k);
}

// Largest power of two <= v (v >= 1).
inline int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}

}  // namespace

template <typename T>
hipError_t launch_tables(p3m_plan* P) {
  Workspace& W = P->ws;
  int ng = P->ng;
  T* etab = (T*)W.gtab;
  k_tables<T><<<(ng + 255) / 256, 256, 0, P->stream>>>(ng, P->prm.box, P->r_s,
                                                        P->prm.deconv_power,
                                                        (typename Vec<T>::v2*)W.twiddle, etab,
                                                        etab + ng);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_poisson(p3m_plan* P) {
  using T2 = typename Vec<T>::v2;
  Workspace& W = P->ws;
  const int ng = P->ng, lg = P->lg, M = ng / 2, M1 = M + 1;
  const T2* tw = (const T2*)W.twiddle;
  T2* spec = (T2*)W.spec;
  T* grid = (T*)W.grid;
  hipStream_t s = P->stream;
  // z passes: nl lines per block
  int nl = pow2_floor(kLdsElems / M);
  if (nl > ng * ng) nl = ng * ng;
  size_t lds_z = (size_t)(padded(nl * M) + M) * sizeof(T2);
  unsigned blocks_z = (unsigned)((int64_t)ng * ng / nl);
  // y / x passes: kc kz-columns per block
  int kc = kLdsElems / ng;
  if (kc > 8) kc = 8;      // 8 columns per block: twice the blocks of 16 (measured 6 % faster at 128^3)
  if (kc < 1) kc = 1;
  size_t lds_c = (size_t)(padded(kc * ng) + M) * sizeof(T2);
  unsigned nchunk = (unsigned)((M1 + kc - 1) / kc);
  const T* etab = (const T*)W.gtab;
  T gconst = (T)(-4.0 * M_PI * P->prm.G / ((double)ng * ng * ng));

  k_fft_z_r2c<T><<<blocks_z, kThreads, lds_z, s>>>(grid, spec, ng, lg, nl, tw);
  k_fft_y<T, false><<<ng * nchunk, kThreads, lds_c, s>>>(spec, ng, lg, kc, tw);
  k_fft_x_green<T><<<ng * nchunk, kThreads, lds_c, s>>>(spec, ng, lg, kc, tw, etab,
                                                        etab + ng, gconst);
  k_fft_y<T, true><<<ng * nchunk, kThreads, lds_c, s>>>(spec, ng, lg, kc, tw);
  k_fft_z_c2r<T><<<blocks_z, kThreads, lds_z, s>>>(spec, grid, ng, lg, nl, tw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_power_spectrum(p3m_plan* P, int nbins, double r_tophat, double* k_out,
                                 double* p_out, double* m_out, double* sigma_out) {
  using T2 = typename Vec<T>::v2;
  Workspace& W = P->ws;
  const int ng = P->ng, lg = P->lg, M = ng / 2, M1 = M + 1;
  const T2* tw = (const T2*)W.twiddle;
  T2* spec = (T2*)W.spec;
  hipStream_t s = P->stream;
  hipError_t e = launch_fill_i32((int32_t*)W.power_acc, 2 * (3 * nbins + 2), 0, s);
  if (e != hipSuccess) return e;
  int nl = pow2_floor(kLdsElems / M);
  if (nl > ng * ng) nl = ng * ng;
  size_t lds_z = (size_t)(padded(nl * M) + M) * sizeof(T2);
  unsigned blocks_z = (unsigned)((int64_t)ng * ng / nl);
  int kc = kLdsElems / ng;
  if (kc > 8) kc = 8;      // 8 columns per block: twice the blocks of 16 (measured 6 % faster at 128^3)
  if (kc < 1) kc = 1;
  size_t lds_c = (size_t)(padded(kc * ng) + M) * sizeof(T2);
  unsigned nchunk = (unsigned)((M1 + kc - 1) / kc);
  k_fft_z_r2c<T><<<blocks_z, kThreads, lds_z, s>>>((const T*)W.grid, spec, ng, lg, nl, tw);
  k_fft_y<T, false><<<ng * nchunk, kThreads, lds_c, s>>>(spec, ng, lg, kc, tw);
  k_fft_x_power<T><<<ng * nchunk, kThreads, lds_c, s>>>(
      spec, ng, lg, kc, tw, P->prm.deconv_power != 0 ? 1 : 0, nbins,
      2.0 * M_PI / P->prm.box * r_tophat, W.power_acc);
  k_power_finish<<<1, 256, 0, s>>>(W.power_acc, nbins, P->prm.box, k_out, p_out, m_out,
                                   sigma_out);
  return hipGetLastError();
}

template hipError_t launch_tables<float>(p3m_plan*);
template hipError_t launch_tables<double>(p3m_plan*);
template hipError_t launch_fft_poisson<float>(p3m_plan*);
template hipError_t launch_fft_poisson<double>(p3m_plan*);
template hipError_t launch_power_spectrum<float>(p3m_plan*, int, double, double*, double*,
                                                 double*, double*);
template hipError_t launch_power_spectrum<double>(p3m_plan*, int, double, double*, double*,
                                                  double*, double*);

}  // namespace p3m
