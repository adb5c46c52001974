// The C ABI of libp3m.so: argument checking, plan geometry and workspace,
// and the order of the force stages. Declared in include/p3m.h and
// include/p3m_host.h.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "p3m_internal.h"

using namespace p3m;

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t{1} << (l + 1)) <= v) ++l;
  return l;
}

// Minimum gap, in whole cells, between an i-group spanning cells [0, g) of
// one axis and the cell at offset d.
int axis_gap(int d, int g) {
  if (d < 0) return -d - 1;
  if (d >= g) return d - g;
  return 0;
}

template <typename T>
T* dev_alloc(size_t count, hipError_t& err) {
  void* p = nullptr;
  if (err != hipSuccess) return nullptr;
  size_t bytes = count * sizeof(T);
  if (bytes == 0) bytes = 256;
  err = hipMalloc(&p, bytes);
  return err == hipSuccess ? (T*)p : nullptr;
}

void free_workspace(p3m_plan* P) {
  Workspace& W = P->ws;
  void* ptrs[] = {W.key,  W.rank,   W.count,  W.start, W.perm,  W.skey,    W.scan_tmp,
                  W.gchunk, W.goff, W.items,  W.rows,  W.rec,   W.acc_pm,  W.grid,
                  W.spec, W.twiddle, W.gtab,  W.counter, W.split_tab, W.split_tab64, W.lam,
                  W.grid2, W.lam_grid, W.power_acc, W.ewald_tab, W.ewald_zpair,
                  W.segrows, W.prows, W.pbrows, W.pboff, W.rowoff, W.gipre, W.gntot,
                  W.gtot, W.gbase, W.gscan_tmp, W.rpart, W.acc_mesh};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  W = Workspace{};
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  if (P->stream2) (void)hipStreamDestroy(P->stream2);
  P->ev_fork = P->ev_join = nullptr;
  P->stream2 = nullptr;
}

void free_timers(p3m_plan* P) {
  if (P->ev)
    for (int i = 0; i < P->timing_cap * 2 * P3M_NUM_STAGES; ++i)
      if (P->ev[i]) (void)hipEventDestroy(P->ev[i]);
  delete[] P->ev;
  delete[] P->ran;
  P->ev = nullptr;
  P->ran = nullptr;
  P->timing_cap = P->timing_calls = 0;
  P->timing_slot = -1;
}

int status_of(hipError_t e) {
  if (e == hipSuccess) return P3M_OK;
  if (e == hipErrorOutOfMemory) return P3M_ENOMEM;
  return P3M_EHIP;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!a || !b) return false;
  auto pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + bbytes && pb < pa + abytes;
}

struct StageTimer {
  p3m_plan* P;
  int stage;
  StageTimer(p3m_plan* p, int s) : P(p), stage(s) {
    if (P->timing_slot >= 0)
      (void)hipEventRecord(P->ev[(P->timing_slot * P3M_NUM_STAGES + stage) * 2], P->stream);
  }
  ~StageTimer() {
    if (P->timing_slot >= 0) {
      int k = P->timing_slot * P3M_NUM_STAGES + stage;
      (void)hipEventRecord(P->ev[2 * k + 1], P->stream);
      P->ran[k] = 1;
    }
  }
};

// Claim a timer slot for the force call about to run (if recording).
void begin_call(p3m_plan* P) {
  P->timing_slot = -1;
  if (P->timing_cap > 0 && P->timing_calls < P->timing_cap) P->timing_slot = P->timing_calls++;
}

enum class Part { kP3M, kPM, kPP };

// Launches that take the plan's stream enqueue on `s` while this is alive.
struct OnStream {
  p3m_plan* P;
  hipStream_t saved;
  OnStream(p3m_plan* p, hipStream_t s) : P(p), saved(p->stream) { P->stream = s; }
  ~OnStream() { P->stream = saved; }
};

template <typename T>
hipError_t run_force(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                     double ms, void* force, int f32, Part part) {
  hipError_t e;
  const bool half = P->rcap > 0 && part != Part::kPM;
  {
    StageTimer t(P, P3M_STAGE_BIN);
    if ((e = launch_bin(P, n, pos, mass, ms)) != hipSuccess) return e;
    if (part != Part::kPM && (e = launch_items(P)) != hipSuccess) return e;
    if (half && (e = launch_react_prepass(P)) != hipSuccess) return e;
  }
  if (part == Part::kP3M) {
    // The mesh part (deposit, Poisson solve) on the second stream beside the
    // pair sum, which writes its sorted acceleration; the interpolation then
    // adds the mesh acceleration and writes the force once both are done.
    // Both read the binned particles only. One-sided sum: the interpolation
    // also runs on the second stream (to the sorted mesh acceleration), and
    // the gather of the reactions, after the pair sum, adds it and writes
    // the force.
    const hipStream_t main = P->stream;
    if ((e = hipEventRecord(P->ev_fork, main)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(P->stream2, P->ev_fork, 0)) != hipSuccess) return e;
    {
      OnStream on(P, P->stream2);
      {
        StageTimer t(P, P3M_STAGE_DEPOSIT);
        if ((e = launch_deposit<T>(P)) != hipSuccess) return e;
      }
      {
        StageTimer t(P, P3M_STAGE_FFT);
        if ((e = launch_fft_poisson<T>(P)) != hipSuccess) return e;
      }
      if (half) {
        StageTimer t(P, P3M_STAGE_INTERP);
        if ((e = launch_interp<T>(P, n, nullptr, f32, nullptr, P->ws.acc_mesh)) != hipSuccess)
          return e;
      }
      if ((e = hipEventRecord(P->ev_join, P->stream2)) != hipSuccess) return e;
    }
    {
      StageTimer t(P, P3M_STAGE_PP);
      if ((e = launch_pairs<T>(P, n, false, nullptr, f32, mass == nullptr, P->ws.acc_pm)) !=
          hipSuccess)
        return e;
    }
    if ((e = hipStreamWaitEvent(main, P->ev_join, 0)) != hipSuccess) return e;
    if (half) {
      StageTimer t(P, P3M_STAGE_REACT);
      return launch_pair_gather<T>(P, n, false, mass == nullptr, nullptr, force, f32,
                                   P->ws.acc_mesh);
    }
    StageTimer t(P, P3M_STAGE_INTERP);
    return launch_interp<T>(P, n, force, f32, P->ws.acc_pm);
  }
  if (part != Part::kPP) {
    {
      StageTimer t(P, P3M_STAGE_DEPOSIT);
      if ((e = launch_deposit<T>(P)) != hipSuccess) return e;
    }
    {
      StageTimer t(P, P3M_STAGE_FFT);
      if ((e = launch_fft_poisson<T>(P)) != hipSuccess) return e;
    }
    {
      StageTimer t(P, P3M_STAGE_INTERP);
      if ((e = launch_interp<T>(P, n, part == Part::kPM ? force : nullptr, f32)) != hipSuccess)
        return e;
    }
  }
  if (part != Part::kPM) {
    {
      StageTimer t(P, P3M_STAGE_PP);
      if ((e = launch_pairs<T>(P, n, false, force, f32, mass == nullptr)) != hipSuccess) return e;
    }
    if (half) {
      StageTimer t(P, P3M_STAGE_REACT);
      if ((e = launch_pair_gather<T>(P, n, false, mass == nullptr, nullptr, force, f32)) !=
          hipSuccess)
        return e;
    }
  }
  return hipSuccess;
}

int force_entry(p3m_plan* P, int64_t n, const double* pos, const double* mass, double ms,
                void* force, int32_t f32, Part part) {
  if (!P || n < 0 || n > P->n_max) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!pos || !force) return P3M_EINVAL;
  if (!mass && !std::isfinite(ms)) return P3M_EINVAL;
  size_t fbytes = (size_t)(3 * n) * (f32 ? sizeof(float) : sizeof(double));
  if (overlaps(force, fbytes, pos, (size_t)(3 * n) * sizeof(double)) ||
      overlaps(force, fbytes, mass, (size_t)n * sizeof(double)))
    return P3M_EINVAL;
  begin_call(P);
  hipError_t e = P->prm.precision == P3M_FP32
                     ? run_force<float>(P, n, pos, mass, ms, force, f32 ? 1 : 0, part)
                     : run_force<double>(P, n, pos, mass, ms, force, f32 ? 1 : 0, part);
  return status_of(e);
}

// The adjoint stages. The two Poisson solves run on the same in-place FFT:
// the forward potential phi in `grid`, then psi in `grid2` (buffers swapped
// around the second solve).
template <typename T>
hipError_t run_vjp(p3m_plan* P, int64_t n, const double* pos, const double* mass, double ms,
                   const double* fbar, double* pbar, Part part) {
  hipError_t e;
  Workspace& W = P->ws;
  const bool half = P->rcap > 0 && part != Part::kPM;
  {
    StageTimer t(P, P3M_STAGE_BIN);
    if ((e = launch_bin(P, n, pos, mass, ms)) != hipSuccess) return e;
    if (part != Part::kPM && (e = launch_items(P)) != hipSuccess) return e;
    if (half && (e = launch_react_prepass(P)) != hipSuccess) return e;
    if ((e = launch_lambda_sort<T>(P, n, fbar)) != hipSuccess) return e;
  }
  if (part == Part::kP3M) {
    // As in the force: the mesh adjoint's deposits and Poisson solves on the
    // second stream beside the pair adjoint, which writes its sorted
    // cotangent; the gather then adds the mesh part and writes pos_bar.
    const hipStream_t main = P->stream;
    if ((e = hipEventRecord(P->ev_fork, main)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(P->stream2, P->ev_fork, 0)) != hipSuccess) return e;
    {
      OnStream on(P, P->stream2);
      {
        StageTimer t(P, P3M_STAGE_DEPOSIT);
        if ((e = launch_deposit<T>(P)) != hipSuccess) return e;
        if ((e = launch_deposit_lambda<T>(P)) != hipSuccess) return e;
      }
      {
        StageTimer t(P, P3M_STAGE_FFT);
        if ((e = launch_fft_poisson<T>(P)) != hipSuccess) return e;
        std::swap(W.grid, W.grid2);
        e = launch_fft_poisson<T>(P);
        std::swap(W.grid, W.grid2);
        if (e != hipSuccess) return e;
      }
      if ((e = hipEventRecord(P->ev_join, P->stream2)) != hipSuccess) return e;
    }
    {
      StageTimer t(P, P3M_STAGE_PP);
      if ((e = launch_pairs_vjp<T>(P, n, false, pbar, mass == nullptr, W.acc_pm)) !=
          hipSuccess)
        return e;
    }
    if (half) {
      StageTimer t(P, P3M_STAGE_REACT);
      if ((e = launch_pair_gather<T>(P, n, true, mass == nullptr, W.acc_pm, nullptr, 0)) !=
          hipSuccess)
        return e;
    }
    if ((e = hipStreamWaitEvent(main, P->ev_join, 0)) != hipSuccess) return e;
    StageTimer t(P, P3M_STAGE_INTERP);
    return launch_interp_vjp<T>(P, n, pbar, W.acc_pm);
  }
  if (part != Part::kPP) {
    {
      StageTimer t(P, P3M_STAGE_DEPOSIT);
      if ((e = launch_deposit<T>(P)) != hipSuccess) return e;
      if ((e = launch_deposit_lambda<T>(P)) != hipSuccess) return e;
    }
    {
      StageTimer t(P, P3M_STAGE_FFT);
      if ((e = launch_fft_poisson<T>(P)) != hipSuccess) return e;
      std::swap(W.grid, W.grid2);
      e = launch_fft_poisson<T>(P);
      std::swap(W.grid, W.grid2);
      if (e != hipSuccess) return e;
    }
    {
      StageTimer t(P, P3M_STAGE_INTERP);
      if ((e = launch_interp_vjp<T>(P, n, part == Part::kPM ? pbar : nullptr)) != hipSuccess)
        return e;
    }
  }
  if (part != Part::kPM) {
    {
      StageTimer t(P, P3M_STAGE_PP);
      if ((e = launch_pairs_vjp<T>(P, n, false, pbar, mass == nullptr)) != hipSuccess) return e;
    }
    if (half) {
      StageTimer t(P, P3M_STAGE_REACT);
      if ((e = launch_pair_gather<T>(P, n, true, mass == nullptr, nullptr, pbar, 0)) !=
          hipSuccess)
        return e;
    }
  }
  return hipSuccess;
}

int vjp_entry(p3m_plan* P, int64_t n, const double* pos, const double* mass, double ms,
              const double* fbar, double* pbar, Part part) {
  if (!P || n < 0 || n > P->n_max) return P3M_EINVAL;
  if (!P->prm.adjoint) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!pos || !fbar || !pbar) return P3M_EINVAL;
  if (!mass && !std::isfinite(ms)) return P3M_EINVAL;
  const size_t vbytes = (size_t)(3 * n) * sizeof(double);
  if (overlaps(pbar, vbytes, pos, vbytes) || overlaps(pbar, vbytes, fbar, vbytes) ||
      overlaps(pbar, vbytes, mass, (size_t)n * sizeof(double)))
    return P3M_EINVAL;
  begin_call(P);
  hipError_t e = P->prm.precision == P3M_FP32
                     ? run_vjp<float>(P, n, pos, mass, ms, fbar, pbar, part)
                     : run_vjp<double>(P, n, pos, mass, ms, fbar, pbar, part);
  return status_of(e);
}

}  // namespace

namespace p3m {

// Split factor f(u) = erfc(u) + (2u/sqrt(pi)) exp(-u^2), u = r / (2 r_s).
static double split_f(double u) {
  return std::erfc(u) + 1.1283791670955126 * u * std::exp(-u * u);
}

// f as a function of the table variable v (in units of r_s): v = r / r_s, or
// v = sqrt(r^2 + eps^2) / r_s (e = eps / r_s; values below e never occur and
// take f(0)).
static double split_g(int var, double e, double v) {
  if (var == 0) return split_f(0.5 * v);
  return split_f(0.5 * std::sqrt(std::max(v * v - e * e, 0.0)));
}

// Cubic pieces of g over [v0, v1] (FP64 coefficients) and their largest
// deviation from g on a dense sample.
static double fit_table(int var, double e, double v0, double v1, int bins, double* c) {
  const double kPi = 3.14159265358979323846;
  const double w = (v1 - v0) / bins;
  double worst = 0;
  for (int k = 0; k < bins; ++k) {
    // the cubic in t through g at the four Chebyshev points of [0, 1]
    double V[4][5];
    for (int j = 0; j < 4; ++j) {
      double t = 0.5 - 0.5 * std::cos((2 * j + 1) * kPi / 8.0);
      double p = 1.0;
      for (int l = 0; l < 4; ++l, p *= t) V[j][l] = p;
      V[j][4] = split_g(var, e, v0 + (k + t) * w);
    }
    for (int col = 0; col < 4; ++col) {     // Gauss-Jordan, partial pivoting
      int piv = col;
      for (int r = col + 1; r < 4; ++r)
        if (std::fabs(V[r][col]) > std::fabs(V[piv][col])) piv = r;
      for (int l = 0; l < 5; ++l) std::swap(V[col][l], V[piv][l]);
      for (int r = 0; r < 4; ++r) {
        if (r == col) continue;
        double m = V[r][col] / V[col][col];
        for (int l = col; l < 5; ++l) V[r][l] -= m * V[col][l];
      }
    }
    for (int l = 0; l < 4; ++l) c[4 * k + l] = V[l][4] / V[l][l];
    for (int j = 0; j <= 64; ++j) {
      double t = j / 64.0;
      double f = c[4 * k] + t * (c[4 * k + 1] + t * (c[4 * k + 2] + t * c[4 * k + 3]));
      worst = std::max(worst, std::fabs(f - split_g(var, e, v0 + (k + t) * w)));
    }
  }
  return worst;
}

SplitMap split_table(double cutoff_rs, double soft_rs, int bins, float* out) {
  // Prefer the softened distance as the variable (no square root in the pair
  // loop); it has a kink at v = e, which a cubic piece follows only while e
  // is small against the bin width, so fall back to r when the fit misses
  // the bound. The start sits a hair below e so that rounding never takes
  // the kernel's bin coordinate below zero.
  const double kFitBound = 1e-7;
  double c[4 * kSplitBins];
  bins = std::min(bins, kSplitBins);
  SplitMap m{1, soft_rs * (1.0 - 1e-6), std::sqrt(cutoff_rs * cutoff_rs + soft_rs * soft_rs), 0};
  if (fit_table(m.var, soft_rs, m.v0, m.v1, bins, c) > kFitBound) {
    m = SplitMap{0, 0.0, cutoff_rs, 0};
    fit_table(m.var, soft_rs, m.v0, m.v1, bins, c);
  }
  const int stride = bins + 1;
  for (int k = 0; k < bins; ++k)
    for (int l = 0; l < 4; ++l) out[l * stride + k] = (float)c[4 * k + l];
  // entry `bins`: the constant g(v1), for arguments rounded up onto the cutoff
  out[0 * stride + bins] = (float)split_g(m.var, soft_rs, m.v1);
  out[1 * stride + bins] = out[2 * stride + bins] = out[3 * stride + bins] = 0.0f;
  return m;
}

// One set of degree-6 pieces of g over [v0, v1] in extended precision:
// piece k covers v = v0 + (k + t)(v1 - v0)/B, t in [0, 1]; in powers of t,
// the polynomial through g at the seven Chebyshev points of [0, 1] (the
// pieces are narrow, so the coefficients fall off fast and only the final
// rounding to double remains). err[k]: the largest deviation from g of the
// rounded piece on a dense sample.
static void fit_table64(int var, long double e, long double v0, long double v1, double* out,
                        long double* err) {
  typedef long double LD;
  const int B = kSplitBins, C = kSplitCoef64, stride = B + 1;
  const LD kPi = 3.14159265358979323846264338327950288L;
  auto f = [](LD u) { return std::erfc(u) + 1.12837916709551257389615890312154517L * u *
                                                std::exp(-u * u); };
  auto g = [&](LD v) {
    if (var == 0) return f(0.5L * v);
    LD r2 = v * v - e * e;
    return f(0.5L * std::sqrt(r2 > 0 ? r2 : 0.0L));
  };
  const LD w = (v1 - v0) / B;
  for (int k = 0; k < B; ++k) {
    LD V[kSplitCoef64][kSplitCoef64 + 1];
    for (int j = 0; j < C; ++j) {
      LD t = 0.5L - 0.5L * std::cos((2 * j + 1) * kPi / (2 * C));
      LD p = 1.0L;
      for (int l = 0; l < C; ++l, p *= t) V[j][l] = p;
      V[j][C] = g(v0 + w * ((LD)k + t));
    }
    for (int col = 0; col < C; ++col) {     // Gauss-Jordan, partial pivoting
      int piv = col;
      for (int r = col + 1; r < C; ++r)
        if (std::fabs(V[r][col]) > std::fabs(V[piv][col])) piv = r;
      for (int l = 0; l <= C; ++l) std::swap(V[col][l], V[piv][l]);
      for (int r = 0; r < C; ++r) {
        if (r == col) continue;
        LD m = V[r][col] / V[col][col];
        for (int l = col; l <= C; ++l) V[r][l] -= m * V[col][l];
      }
    }
    for (int l = 0; l < C; ++l) out[l * stride + k] = (double)(V[l][C] / V[l][l]);
    err[k] = 0;
    for (int j = 0; j <= 32; ++j) {
      LD t = j / 32.0L, p = 0;
      for (int l = C - 1; l >= 0; --l) p = p * t + (LD)out[l * stride + k];
      err[k] = std::max(err[k], std::fabs(p - g(v0 + w * ((LD)k + t))));
    }
  }
  out[B] = (double)g(v1);
  for (int l = 1; l < C; ++l) out[l * stride + B] = 0.0;
}

SplitMap split_table64(double cutoff_rs, double soft_rs, double* out) {
  // Softened distance as the variable when the pieces that miss the accuracy
  // of the r table (twice its worst piece, at least 4e-16) are only a few
  // leading ones next to the kink at r = 0: those pairs, closer than a few
  // bins, take a series of f in the kernel. Else r.
  const int kMaxExact = 8;
  long double err[kSplitBins];
  const long double e = soft_rs;
  fit_table64(0, e, 0.0L, cutoff_rs, out, err);
  long double bound = 4e-16L;
  for (int k = 0; k < kSplitBins; ++k) bound = std::max(bound, 2.0L * err[k]);
  SplitMap m{1, soft_rs * (1.0 - 1e-9), std::sqrt(cutoff_rs * cutoff_rs + soft_rs * soft_rs), 0};
  fit_table64(1, e, m.v0, m.v1, out, err);
  for (int k = 0; k < kSplitBins; ++k)
    if (err[k] > bound) m.exact = k + 1;
  // the kernel's series for the exact pieces holds for u = r / (2 r_s) <= 0.9
  const double u_top = 0.5 * (m.v0 + m.exact * (m.v1 - m.v0) / kSplitBins);
  if (m.exact > kMaxExact || u_top > 0.9) {
    m = SplitMap{0, 0.0, cutoff_rs, 0};
    fit_table64(0, e, m.v0, m.v1, out, err);
  }
  return m;
}

// The stencil rows of a g^3-cell group, all of them (half = false) or the
// half of them with a lexicographically positive group offset.
static int stencil_rows_of(int g, double radius_cells, bool half, int32_t* out, int cap) {
  if (g < 1 || !(radius_cells > 0) || !std::isfinite(radius_cells)) return P3M_EINVAL;
  // A cell can hold a partner closer than r_c iff its gap to the group box is
  // below r_c; the small margin keeps rounding in the pair test harmless.
  const double R = radius_cells + 1e-9;
  const double R2 = R * R;
  const int reach = (int)std::ceil(R) + 1;
  // group offset of a cell offset d (floor division by g)
  auto gof = [g](int d) { return d >= 0 ? d / g : -((-d + g - 1) / g); };
  int count = 0;
  for (int dx = -reach; dx < g + reach; ++dx) {
    int gx = axis_gap(dx, g);
    for (int dy = -reach; dy < g + reach; ++dy) {
      int gy = axis_gap(dy, g);
      double gxy = double(gx) * gx + double(gy) * gy;
      if (!(gxy < R2)) continue;
      int lo = 0, hi = -1;
      for (int dz = -reach; dz < g + reach; ++dz) {
        int gz = axis_gap(dz, g);
        if (gxy + double(gz) * gz < R2) {
          if (hi < lo) lo = dz;
          hi = dz;
        }
      }
      if (half) {
        const int ox = gof(dx), oy = gof(dy);
        if (ox < 0 || (ox == 0 && oy < 0)) continue;   // lexicographically negative columns
        if (ox == 0 && oy == 0) lo = std::max(lo, g);  // own column: the groups above only
        if (lo > hi) continue;
      }
      if (count < cap && out) {
        out[4 * count + 0] = dx;
        out[4 * count + 1] = dy;
        out[4 * count + 2] = lo;
        out[4 * count + 3] = hi;
      }
      ++count;
    }
  }
  return count;
}

int stencil_rows(int g, double radius_cells, int32_t* out, int cap) {
  return stencil_rows_of(g, radius_cells, false, out, cap);
}

int segment_rows(int g, double radius_cells, int32_t* out, int cap, int* npos) {
  const int nfull = stencil_rows_of(g, radius_cells, false, nullptr, 0);
  if (nfull < 0) return nfull;
  const double R = radius_cells + 1e-9;
  const double R2 = R * R;
  const int reach = (int)std::ceil(R) + 1;
  auto gof = [g](int d) { return d >= 0 ? d / g : -((-d + g - 1) / g); };
  int count = 0, pos = 0;
  // the full stencil's rows in their order (as stencil_rows_of walks them),
  // each cut where its z range crosses a group boundary
  for (int dx = -reach; dx < g + reach; ++dx) {
    int gx = axis_gap(dx, g);
    for (int dy = -reach; dy < g + reach; ++dy) {
      int gy = axis_gap(dy, g);
      double gxy = double(gx) * gx + double(gy) * gy;
      if (!(gxy < R2)) continue;
      int lo = 0, hi = -1;
      for (int dz = -reach; dz < g + reach; ++dz) {
        int gz = axis_gap(dz, g);
        if (gxy + double(gz) * gz < R2) {
          if (hi < lo) lo = dz;
          hi = dz;
        }
      }
      const int ox = gof(dx), oy = gof(dy);
      for (int oz = gof(lo); oz <= gof(hi); ++oz) {
        const int zlo = std::max(lo, oz * g), zhi = std::min(hi, oz * g + g - 1);
        const int sign = ox != 0 ? (ox > 0 ? 1 : -1)
                       : oy != 0 ? (oy > 0 ? 1 : -1)
                       : oz != 0 ? (oz > 0 ? 1 : -1) : 0;
        if (count < cap && out) {
          out[4 * count + 0] = (dx & 0xffff) | (int32_t)((uint32_t)dy << 16);
          out[4 * count + 1] = zlo;
          out[4 * count + 2] = zhi;
          out[4 * count + 3] = sign;
        }
        ++count;
        pos += sign > 0;
      }
    }
  }
  if (npos) *npos = pos;
  return count;
}

int plan_geometry(const p3m_params& q, int64_t n_max, p3m_plan* P) {
  if (!is_pow2(q.grid_n) || q.grid_n < 16 || q.grid_n > 512) return P3M_EINVAL;
  if (q.precision != P3M_FP64 && q.precision != P3M_FP32) return P3M_EINVAL;
  if (q.fd_order != 2 && q.fd_order != 4) return P3M_EINVAL;
  if (q.deconv_power != 0 && q.deconv_power != 2) return P3M_EINVAL;
  if (!(q.box > 0) || !std::isfinite(q.box)) return P3M_EINVAL;
  if (!(q.rs_cells > 0) || !std::isfinite(q.rs_cells)) return P3M_EINVAL;
  if (!(q.cutoff_rs > 0) || !std::isfinite(q.cutoff_rs)) return P3M_EINVAL;
  if (!(q.softening >= 0) || !std::isfinite(q.softening)) return P3M_EINVAL;
  if (!std::isfinite(q.G)) return P3M_EINVAL;
  if (n_max < 0 || n_max >= (int64_t{1} << 31)) return P3M_EINVAL;
  if (q.adjoint != 0 && q.adjoint != 1) return P3M_EINVAL;
  if (q.pair_partials < 0) return P3M_EINVAL;
  if (q.ewald_gridsize != 0 &&
      (q.ewald_gridsize < 8 || q.ewald_gridsize > 512 || (q.ewald_gridsize & 1)))
    return P3M_EINVAL;
  const double h = q.box / q.grid_n;
  const double r_s = q.rs_cells * h;
  const double r_c = q.cutoff_rs * r_s;
  if (!(r_c < 0.5 * q.box)) return P3M_ERANGE;
  P->prm = q;
  P->n_max = n_max;
  P->ng = q.grid_n;
  P->lg = ilog2(q.grid_n);
  P->ncell = (int64_t)q.grid_n * q.grid_n * q.grid_n;
  P->h = h;
  P->r_s = r_s;
  P->r_c = r_c;
  P->eps = q.softening;
  P->G = p3m_group_edge(n_max, q.grid_n);
  P->lgG = ilog2(P->G);
  P->ngd = q.grid_n / P->G;
  P->ngroup = (int64_t)P->ngd * P->ngd * P->ngd;
  P->nrows = stencil_rows(P->G, r_c / h, nullptr, 0);
  P->nseg = segment_rows(P->G, r_c / h, nullptr, 0, &P->npos);
  if (P->nseg < 0) return P->nseg;
  P->max_items = P->ngroup + (n_max + kChunk - 1) / kChunk;
  P->scan_tmp_len = std::max(scan_tmp_size(P->ncell), items_tmp_size(P->ngroup));
  return P3M_OK;
}

hipError_t plan_upload_tables(p3m_plan* P, int32_t* rows_host) {
  const p3m_params& q = P->prm;
  stencil_rows(P->G, P->r_c / P->h, rows_host, P->nrows);
  hipError_t err = hipMemcpyAsync(P->ws.rows, rows_host, sizeof(int4) * P->nrows,
                                  hipMemcpyHostToDevice, P->stream);
  if (err == hipSuccess && P->ws.segrows) {
    // the stencil cut into group segments (staging order), its positive
    // segments in the same order, and those bucketed by the class
    // (dx mod G, dy mod G) of their column offset with their index among
    // the positive ones (for the gather of the reactions: a particle in a
    // column of class (a, b) lies in segments of that class only)
    int32_t* seg = rows_host + 4 * (size_t)P->nrows;
    int32_t* pos = seg + 4 * (size_t)P->nseg;
    int32_t* pb = pos + 4 * (size_t)P->npos;
    int32_t* off = pb + 4 * (size_t)P->npos;
    segment_rows(P->G, P->r_c / P->h, seg, P->nseg, nullptr);
    int k = 0;
    for (int r = 0; r < P->nseg; ++r)
      if (seg[4 * r + 3] > 0) {
        for (int c = 0; c < 4; ++c) pos[4 * k + c] = seg[4 * r + c];
        pos[4 * k + 3] = k;
        ++k;
      }
    const int G = P->G, nb = G * G;
    int m = 0;
    for (int b = 0; b < nb; ++b) {
      off[b] = m;
      for (int r = 0; r < P->npos; ++r) {
        const int dx = (int)(int16_t)(pos[4 * r] & 0xffff), dy = pos[4 * r] >> 16;
        if ((((dx & (G - 1)) * G) | (dy & (G - 1))) != b) continue;
        for (int c = 0; c < 4; ++c) pb[4 * m + c] = pos[4 * r + c];
        ++m;
      }
    }
    off[nb] = m;
    err = hipMemcpyAsync(P->ws.segrows, seg, sizeof(int4) * P->nseg, hipMemcpyHostToDevice,
                         P->stream);
    if (err == hipSuccess)
      err = hipMemcpyAsync(P->ws.prows, pos, sizeof(int4) * P->npos, hipMemcpyHostToDevice,
                           P->stream);
    if (err == hipSuccess)
      err = hipMemcpyAsync(P->ws.pbrows, pb, sizeof(int4) * P->npos, hipMemcpyHostToDevice,
                           P->stream);
    if (err == hipSuccess)
      err = hipMemcpyAsync(P->ws.pboff, off, sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice,
                           P->stream);
  }
  if (err == hipSuccess) {
    float tab[4 * (kSplitBins + 1)];
    SplitMap m = split_table(q.cutoff_rs, q.softening / P->r_s, kSplitBins, tab);
    P->tab_var = m.var;
    P->tab_v0 = m.v0 * P->r_s;
    P->tab_v1 = m.v1 * P->r_s;
    err = hipMemcpyAsync(P->ws.split_tab, tab, sizeof(tab), hipMemcpyHostToDevice, P->stream);
  }
  if (err == hipSuccess) {
    double tab64[kSplitCoef64 * (kSplitBins + 1)];
    SplitMap m = split_table64(q.cutoff_rs, q.softening / P->r_s, tab64);
    P->tab64_var = m.var;
    P->tab64_v0 = m.v0 * P->r_s;
    P->tab64_v1 = m.v1 * P->r_s;
    P->tab64_exact = m.exact;
    err = hipMemcpyAsync(P->ws.split_tab64, tab64, sizeof(tab64), hipMemcpyHostToDevice,
                         P->stream);
  }
  return err;
}

}  // namespace p3m

extern "C" {

int32_t p3m_stencil_rows(int32_t g, double radius_cells, int32_t* rows_out, int32_t cap) {
  if (cap < 0 || (cap > 0 && !rows_out)) return P3M_EINVAL;
  return p3m::stencil_rows(g, radius_cells, rows_out, cap);
}

int32_t p3m_segment_rows(int32_t g, double radius_cells, int32_t* rows_out, int32_t cap) {
  if (cap < 0 || (cap > 0 && !rows_out)) return P3M_EINVAL;
  return p3m::segment_rows(g, radius_cells, rows_out, cap, nullptr);
}

int32_t p3m_split_table(double cutoff_rs, double softening_rs, float* out, int32_t cap,
                        double* map_out) {
  if (!(cutoff_rs > 0) || !std::isfinite(cutoff_rs) || !(softening_rs >= 0) ||
      !std::isfinite(softening_rs) || cap < 0 || (cap > 0 && !out))
    return P3M_EINVAL;
  if (cap >= 4 * (kSplitBins + 1)) {
    p3m::SplitMap m = p3m::split_table(cutoff_rs, softening_rs, kSplitBins, out);
    if (map_out) {
      map_out[0] = m.var;
      map_out[1] = m.v0;
      map_out[2] = m.v1;
    }
  }
  return kSplitBins;
}

int32_t p3m_split_table64(double cutoff_rs, double softening_rs, double* out, int32_t cap,
                          double* map_out) {
  if (!(cutoff_rs > 0) || !std::isfinite(cutoff_rs) || !(softening_rs >= 0) ||
      !std::isfinite(softening_rs) || cap < 0 || (cap > 0 && !out))
    return P3M_EINVAL;
  if (cap >= kSplitCoef64 * (kSplitBins + 1)) {
    p3m::SplitMap m = p3m::split_table64(cutoff_rs, softening_rs, out);
    if (map_out) {
      map_out[0] = m.var;
      map_out[1] = m.v0;
      map_out[2] = m.v1;
      map_out[3] = m.exact;
    }
  }
  return kSplitBins;
}

int32_t p3m_group_edge(int64_t n, int32_t grid_n) {
  if (n <= 0 || grid_n < 2) return 1;
  double cells_per_particle = std::pow((double)grid_n, 3) / (double)n;
  int best = 1;
  double best_err = 1e300;
  for (int g = 1; g <= 4 && g <= grid_n / 2; g *= 2) {
    double mean = (double)g * g * g / cells_per_particle;
    double err = std::fabs(std::log(mean / kGroupTarget));
    if (err < best_err) {
      best_err = err;
      best = g;
    }
  }
  return best;
}

int p3m_params_default(p3m_params* out, int32_t grid_n, double box) {
  if (!out) return P3M_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->grid_n = grid_n;
  out->precision = P3M_FP32;
  out->fd_order = 4;
  out->deconv_power = 2;
  out->box = box;
  out->rs_cells = 1.25;
  out->cutoff_rs = 4.5;
  out->softening = 0.0;
  out->G = 1.0;
  out->pair_partials = 0;
  return P3M_OK;
}

int p3m_plan_create(const p3m_params* prm, int64_t n_max, void* hip_stream, p3m_plan** out) {
  if (!prm || !out) return P3M_EINVAL;
  const p3m_params& q = *prm;
  p3m_plan* P = new (std::nothrow) p3m_plan;
  if (!P) return P3M_ENOMEM;
  const int st = p3m::plan_geometry(q, n_max, P);
  if (st != P3M_OK) {
    delete P;
    return st;
  }
  P->stream = (hipStream_t)hip_stream;
  const int64_t nspec = (int64_t)q.grid_n * q.grid_n * p3m::spec_stride(q.grid_n);
  const size_t real = q.precision == P3M_FP32 ? sizeof(float) : sizeof(double);
  const int64_t nn = n_max > 0 ? n_max : 1;

  hipError_t err = hipGetDevice(&P->device);
  Workspace& W = P->ws;
  W.key = dev_alloc<int32_t>(nn, err);
  W.rank = dev_alloc<int32_t>(nn, err);
  W.count = dev_alloc<int32_t>(P->ncell + 1, err);
  W.start = dev_alloc<int32_t>(P->ncell + 1, err);
  W.perm = dev_alloc<int32_t>(nn, err);
  W.skey = dev_alloc<int32_t>(nn, err);
  W.scan_tmp = dev_alloc<int32_t>(P->scan_tmp_len, err);
  W.gchunk = dev_alloc<int32_t>(P->ngroup + 1, err);
  W.goff = dev_alloc<int32_t>(P->ngroup + 1, err);
  W.items = dev_alloc<int2>(P->max_items, err);
  W.rows = dev_alloc<int4>(P->nrows, err);
  W.rec = dev_alloc<unsigned char>(nn * 4 * real, err);
  W.acc_pm = dev_alloc<unsigned char>(nn * 4 * real, err);
  W.grid = dev_alloc<unsigned char>(P->ncell * real, err);
  W.spec = dev_alloc<unsigned char>(nspec * 2 * real, err);
  W.twiddle = dev_alloc<unsigned char>((q.grid_n / 2) * 2 * real, err);
  W.gtab = dev_alloc<unsigned char>(2 * q.grid_n * real, err);
  W.counter = dev_alloc<unsigned long long>(1, err);
  W.split_tab = dev_alloc<float>(4 * (kSplitBins + 1), err);
  W.split_tab64 = dev_alloc<double>(kSplitCoef64 * (kSplitBins + 1), err);
  W.power_acc = dev_alloc<double>(3 * kMaxPowerBins + 2, err);
  if (q.ewald_gridsize) {
    const int64_t H = q.ewald_gridsize / 2 + 1;
    W.ewald_tab = dev_alloc<double4>(H * H * H, err);
    W.ewald_zpair = dev_alloc<double2>(H * H * (H - 1) * 3, err);
  }
  if (q.adjoint) {
    W.lam = dev_alloc<unsigned char>(nn * 4 * real, err);
    W.grid2 = dev_alloc<unsigned char>(P->ncell * real, err);
    W.lam_grid = dev_alloc<unsigned char>(3 * P->ncell * real, err);
  }
  // the one-sided pair sum: half stencil, per-group offsets, partials; if the
  // partials do not fit, the plan sums every pair from both sides
  if (err == hipSuccess && q.pair_partials > 0 && P->npos > 0) {
    W.segrows = dev_alloc<int4>(P->nseg, err);
    W.prows = dev_alloc<int4>(P->npos, err);
    W.pbrows = dev_alloc<int4>(P->npos, err);
    W.pboff = dev_alloc<int32_t>(P->G * P->G + 1, err);
    W.gipre = dev_alloc<int32_t>(P->ngroup * P->G * P->G, err);
    W.rowoff = dev_alloc<int32_t>(P->ngroup * (P->npos + 1), err);
    W.gntot = dev_alloc<int32_t>(P->ngroup, err);
    W.gtot = dev_alloc<long long>(P->ngroup, err);
    W.gbase = dev_alloc<long long>(P->ngroup + 1, err);
    W.gscan_tmp = dev_alloc<long long>(react_scan_tmp_size(P->ngroup), err);
    const int64_t cap = (int64_t)q.pair_partials * nn + kPartialsSlack;
    if (err == hipSuccess) {
      void* p = nullptr;
      if (hipMalloc(&p, (size_t)cap * 3 * real) == hipSuccess) {
        W.rpart = p;
        P->rcap = cap;
        W.acc_mesh = dev_alloc<unsigned char>(nn * 4 * real, err);
      } else {
        (void)hipGetLastError();          // clear the failed allocation's error
      }
    }
  }
  // the P3M force's second stream (default priority) and its fork / join events
  if (err == hipSuccess) err = hipStreamCreateWithFlags(&P->stream2, hipStreamNonBlocking);
  if (err == hipSuccess) err = hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming);
  if (err == hipSuccess) err = hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming);
  if (err == hipSuccess) {
    int32_t* rows =
        new (std::nothrow) int32_t[4 * (size_t)(P->nrows + P->nseg + 2 * P->npos) + 17];
    if (!rows) {
      free_workspace(P);
      delete P;
      return P3M_ENOMEM;
    }
    err = p3m::plan_upload_tables(P, rows);
    delete[] rows;
  }
  if (err == hipSuccess)
    err = q.precision == P3M_FP32 ? launch_tables<float>(P) : launch_tables<double>(P);
  if (err == hipSuccess && q.ewald_gridsize) err = launch_ewald_table(P);
  if (err == hipSuccess) err = hipStreamSynchronize(P->stream);
  if (err != hipSuccess) {
    free_workspace(P);
    delete P;
    return status_of(err);
  }
  *out = P;
  return P3M_OK;
}

int p3m_plan_destroy(p3m_plan* P) {
  if (!P) return P3M_OK;
  hipError_t e = hipStreamSynchronize(P->stream);
  free_workspace(P);
  free_timers(P);
  delete P;
  return status_of(e);
}

int p3m_plan_set_stream(p3m_plan* P, void* hip_stream) {
  if (!P) return P3M_EINVAL;
  P->stream = (hipStream_t)hip_stream;
  return P3M_OK;
}

int p3m_force(p3m_plan* P, int64_t n, const double* pos, const double* mass,
              double mass_scalar, void* force, int32_t force_fp32) {
  return force_entry(P, n, pos, mass, mass_scalar, force, force_fp32, Part::kP3M);
}

int p3m_force_cell_order(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                         double mass_scalar, void* force, int32_t force_fp32,
                         int32_t* order_out) {
  if (!P || n < 0 || n > P->n_max) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!order_out) return P3M_EINVAL;
  const size_t obytes = (size_t)n * sizeof(int32_t);
  const size_t fbytes = (size_t)(3 * n) * (force_fp32 ? sizeof(float) : sizeof(double));
  if (overlaps(order_out, obytes, pos, (size_t)(3 * n) * sizeof(double)) ||
      overlaps(order_out, obytes, mass, (size_t)n * sizeof(double)) ||
      overlaps(order_out, obytes, force, fbytes))
    return P3M_EINVAL;
  struct CellOrder {   // the force's final stores skip the permutation for this call
    p3m_plan* P;
    explicit CellOrder(p3m_plan* p) : P(p) { P->cell_order = true; }
    ~CellOrder() { P->cell_order = false; }
  } on(P);
  const int st = force_entry(P, n, pos, mass, mass_scalar, force, force_fp32, Part::kP3M);
  if (st != P3M_OK) return st;
  return status_of(hipMemcpyAsync(order_out, P->ws.perm, obytes, hipMemcpyDeviceToDevice,
                                  P->stream));
}

int pm_force(p3m_plan* P, int64_t n, const double* pos, const double* mass,
             double mass_scalar, void* force, int32_t force_fp32) {
  return force_entry(P, n, pos, mass, mass_scalar, force, force_fp32, Part::kPM);
}

int pp_force(p3m_plan* P, int64_t n, const double* pos, const double* mass,
             double mass_scalar, void* force, int32_t force_fp32) {
  return force_entry(P, n, pos, mass, mass_scalar, force, force_fp32, Part::kPP);
}

int p3m_force_vjp(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                  double mass_scalar, const double* force_bar, double* pos_bar) {
  return vjp_entry(P, n, pos, mass, mass_scalar, force_bar, pos_bar, Part::kP3M);
}

int pm_force_vjp(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                 double mass_scalar, const double* force_bar, double* pos_bar) {
  return vjp_entry(P, n, pos, mass, mass_scalar, force_bar, pos_bar, Part::kPM);
}

int pp_force_vjp(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                 double mass_scalar, const double* force_bar, double* pos_bar) {
  return vjp_entry(P, n, pos, mass, mass_scalar, force_bar, pos_bar, Part::kPP);
}

int p3m_power_spectrum(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                       double mass_scalar, int32_t nbins, double r_tophat, double* k_out,
                       double* power_out, double* modes_out, double* sigma_out) {
  if (!P || n <= 0 || n > P->n_max || !pos) return P3M_EINVAL;
  if (nbins < 1 || nbins > kMaxPowerBins) return P3M_EINVAL;
  if (!(r_tophat >= 0) || !std::isfinite(r_tophat)) return P3M_EINVAL;
  if (!k_out || !power_out || !modes_out) return P3M_EINVAL;
  if (!mass && !(mass_scalar > 0 && std::isfinite(mass_scalar))) return P3M_EINVAL;
  begin_call(P);
  hipError_t e;
  {
    StageTimer t(P, P3M_STAGE_BIN);
    if ((e = launch_bin(P, n, pos, mass, mass_scalar)) != hipSuccess) return status_of(e);
  }
  const bool f32 = P->prm.precision == P3M_FP32;
  {
    StageTimer t(P, P3M_STAGE_DEPOSIT);
    e = f32 ? launch_deposit<float>(P) : launch_deposit<double>(P);
    if (e != hipSuccess) return status_of(e);
  }
  StageTimer t(P, P3M_STAGE_FFT);
  e = f32 ? launch_power_spectrum<float>(P, nbins, r_tophat, k_out, power_out, modes_out,
                                         sigma_out)
          : launch_power_spectrum<double>(P, nbins, r_tophat, k_out, power_out, modes_out,
                                          sigma_out);
  return status_of(e);
}

int pp_ewald_force(p3m_plan* P, int64_t n, const double* pos, const double* mass,
                   double mass_scalar, void* force, int32_t force_fp32) {
  if (!P || n < 0 || n > P->n_max || !P->prm.ewald_gridsize) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!pos || !force) return P3M_EINVAL;
  if (!mass && !std::isfinite(mass_scalar)) return P3M_EINVAL;
  size_t fbytes = (size_t)(3 * n) * (force_fp32 ? sizeof(float) : sizeof(double));
  if (overlaps(force, fbytes, pos, (size_t)(3 * n) * sizeof(double)) ||
      overlaps(force, fbytes, mass, (size_t)n * sizeof(double)))
    return P3M_EINVAL;
  P->timing_slot = -1;
  // the binning's permutation orders the i-particles by cell (table locality)
  hipError_t e = launch_bin(P, n, pos, mass, mass_scalar);
  if (e != hipSuccess) return status_of(e);
  return status_of(launch_pp_ewald(P, n, pos, mass, mass_scalar, P->ws.perm, force,
                                   force_fp32 ? 1 : 0));
}

int p3m_ewald_correction(p3m_plan* P, int64_t npts, const double* r, double* c_out) {
  if (!P || npts < 0 || !P->prm.ewald_gridsize) return P3M_EINVAL;
  if (npts == 0) return P3M_OK;
  if (!r || !c_out ||
      overlaps(r, (size_t)(3 * npts) * sizeof(double), c_out,
               (size_t)(3 * npts) * sizeof(double)))
    return P3M_EINVAL;
  return status_of(launch_ewald_eval(P, npts, r, c_out));
}

int p3m_pair_count(p3m_plan* P, int64_t n, const double* pos, int64_t* count_out) {
  if (!P || n < 0 || n > P->n_max || !count_out) return P3M_EINVAL;
  if (n > 0 && !pos) return P3M_EINVAL;
  hipError_t e;
  if (n == 0) return status_of(launch_fill_i32((int32_t*)count_out, 2, 0, P->stream));
  P->timing_slot = -1;
  if ((e = launch_bin(P, n, pos, nullptr, 1.0)) != hipSuccess) return status_of(e);
  if ((e = launch_items(P)) != hipSuccess) return status_of(e);
  e = P->prm.precision == P3M_FP32 ? launch_pair_count<float>(P, n, count_out)
                                   : launch_pair_count<double>(P, n, count_out);
  return status_of(e);
}

int p3m_kick(int64_t n, double* mom, const void* force, int32_t force_fp32, double c_kick,
             void* hip_stream) {
  if (n < 0) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!mom || !force || !std::isfinite(c_kick)) return P3M_EINVAL;
  return status_of(launch_kick(n, mom, force, force_fp32 ? 1 : 0, c_kick,
                               (hipStream_t)hip_stream));
}

int p3m_kick_reorder(int64_t n, const int32_t* order, const double* pos, const double* mom,
                     const void* force, int32_t force_fp32, const int64_t* ids,
                     const double* mass, double c_kick, double* pos_out, double* mom_out,
                     int64_t* ids_out, double* mass_out, void* hip_stream) {
  if (n < 0) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!order || !pos || !mom || !force || !pos_out || !mom_out || !std::isfinite(c_kick))
    return P3M_EINVAL;
  if ((ids == nullptr) != (ids_out == nullptr) || (mass == nullptr) != (mass_out == nullptr))
    return P3M_EINVAL;
  const size_t vb = (size_t)(3 * n) * sizeof(double), sb8 = (size_t)n * 8;
  const size_t fb = (size_t)(3 * n) * (force_fp32 ? sizeof(float) : sizeof(double));
  const void* in[] = {order, pos, mom, force, ids, mass};
  const size_t inb[] = {(size_t)n * sizeof(int32_t), vb, vb, fb, sb8, sb8};
  void* out[] = {pos_out, mom_out, ids_out, mass_out};
  const size_t outb[] = {vb, vb, sb8, sb8};
  for (int a = 0; a < 4; ++a) {
    for (int b = 0; b < 6; ++b)
      if (overlaps(out[a], outb[a], in[b], inb[b])) return P3M_EINVAL;
    for (int b = a + 1; b < 4; ++b)
      if (overlaps(out[a], outb[a], out[b], outb[b])) return P3M_EINVAL;
  }
  return status_of(launch_kick_reorder(n, order, pos, mom, force, force_fp32 ? 1 : 0, ids, mass,
                                       c_kick, pos_out, mom_out, ids_out, mass_out,
                                       (hipStream_t)hip_stream));
}

int p3m_drift(int64_t n, double* pos, const double* mom, const double* mass,
              double mass_scalar, double c_drift, double box, void* hip_stream) {
  if (n < 0) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!pos || !mom || !(box > 0) || !std::isfinite(box) || !std::isfinite(c_drift))
    return P3M_EINVAL;
  if (!mass && !(mass_scalar != 0 && std::isfinite(mass_scalar))) return P3M_EINVAL;
  return status_of(launch_drift(n, pos, mom, mass, mass_scalar, c_drift, box,
                                (hipStream_t)hip_stream));
}

int p3m_kick_drift(int64_t n, double* pos, double* mom, const void* force, int32_t force_fp32,
                   const double* mass, double mass_scalar, double c_kick, double c_drift,
                   double box, void* hip_stream) {
  if (n < 0) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!pos || !mom || !force || !(box > 0) || !std::isfinite(box) || !std::isfinite(c_kick) ||
      !std::isfinite(c_drift))
    return P3M_EINVAL;
  if (!mass && !(mass_scalar != 0 && std::isfinite(mass_scalar))) return P3M_EINVAL;
  const size_t vbytes = (size_t)(3 * n) * sizeof(double);
  if (overlaps(pos, vbytes, mom, vbytes)) return P3M_EINVAL;
  return status_of(launch_kick_drift(n, pos, mom, force, force_fp32 ? 1 : 0, mass, mass_scalar,
                                     c_kick, c_drift, box, (hipStream_t)hip_stream));
}

int p3m_drift_vjp(int64_t n, double* mom_bar, const double* pos_bar, const double* mass,
                  double mass_scalar, double c_drift, void* hip_stream) {
  if (n < 0) return P3M_EINVAL;
  if (n == 0) return P3M_OK;
  if (!mom_bar || !pos_bar || !std::isfinite(c_drift)) return P3M_EINVAL;
  if (!mass && !(mass_scalar != 0 && std::isfinite(mass_scalar))) return P3M_EINVAL;
  if (overlaps(mom_bar, (size_t)(3 * n) * sizeof(double), pos_bar,
               (size_t)(3 * n) * sizeof(double)))
    return P3M_EINVAL;
  return status_of(launch_drift_vjp(n, mom_bar, pos_bar, mass, mass_scalar, c_drift,
                                    (hipStream_t)hip_stream));
}

int p3m_set_timing(p3m_plan* P, int32_t capacity) {
  if (!P || capacity < 0 || capacity > (1 << 20)) return P3M_EINVAL;
  hipError_t e = hipStreamSynchronize(P->stream);
  free_timers(P);
  if (e != hipSuccess) return status_of(e);
  if (capacity == 0) return P3M_OK;
  const int nev = capacity * 2 * P3M_NUM_STAGES;
  P->ev = new (std::nothrow) hipEvent_t[nev]();
  P->ran = new (std::nothrow) unsigned char[(size_t)capacity * P3M_NUM_STAGES]();
  if (!P->ev || !P->ran) {
    delete[] P->ev;
    delete[] P->ran;
    P->ev = nullptr;
    P->ran = nullptr;
    return P3M_ENOMEM;
  }
  P->timing_cap = capacity;
  for (int i = 0; i < nev; ++i) {
    if ((e = hipEventCreate(&P->ev[i])) != hipSuccess) {
      free_timers(P);
      return status_of(e);
    }
  }
  return P3M_OK;
}

int p3m_stage_times(p3m_plan* P, double* ms_out, int32_t n_stages) {
  if (!P || (n_stages > 0 && !ms_out) || n_stages < 0) return P3M_EINVAL;
  hipError_t e = hipStreamSynchronize(P->stream);
  if (e != hipSuccess) return status_of(e);
  for (int s = 0; s < n_stages; ++s) ms_out[s] = 0.0;
  for (int c = 0; c < P->timing_calls; ++c)
    for (int s = 0; s < n_stages && s < P3M_NUM_STAGES; ++s) {
      int k = c * P3M_NUM_STAGES + s;
      if (!P->ran[k]) continue;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, P->ev[2 * k], P->ev[2 * k + 1])) != hipSuccess)
        return status_of(e);
      ms_out[s] += ms;
    }
  return P->timing_calls;
}

const char* p3m_strerror(int status) {
  switch (status) {
    case P3M_OK: return "success";
    case P3M_EINVAL: return "invalid argument";
    case P3M_ENOMEM: return "out of device memory";
    case P3M_EHIP: return "HIP runtime error";
    case P3M_ERANGE: return "cutoff must be below half the box (minimum image)";
    case P3M_ESIZE: return "sizes beyond the fixed workspace of the allocation-free call";
    default: return "unknown status";
  }
}

}  // extern "C"
