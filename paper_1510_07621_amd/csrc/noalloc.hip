// Short-range force without a plan: pp_force_noalloc, for callers that
// cannot allocate device memory. Its workspace (binning arrays, work list,
// stencil rows, split tables, sorted records) is carved from one file-scope
// device array of fixed size; the stencil and the split tables are computed
// on the host per call and copied in on the caller's stream. The arithmetic
// is that of pp_force (the same kernels), with every pair evaluated from
// both sides.
#include <cmath>
#include <cstdint>
#include <mutex>

#include "p3m_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t{12} << 20;
constexpr int kMaxDevices = 64;
constexpr int kMaxRows = 4096;

// The workspace of every pp_force_noalloc call on a device. In host code the
// name stands for the host-side shadow of the symbol; device addresses come
// from hipGetSymbolAddress, one per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;                       // the address table and the host row buffer
void* g_scratch[kMaxDevices] = {};
int32_t g_rows[8 * kMaxRows];

// Device address of this device's scratch array (looked up once per device,
// with that device current).
hipError_t scratch_address(int dev, unsigned char** out) {
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = ptr;
  }
  *out = (unsigned char*)g_scratch[dev];
  return hipSuccess;
}

// Carves the plan's workspace from the scratch array at base; returns the
// bytes used (the caller checks them against kScratchBytes first with
// base == nullptr).
size_t carve(p3m_plan* P, unsigned char* base, int64_t n) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  const size_t real = P->prm.precision == P3M_FP32 ? sizeof(float) : sizeof(double);
  const int64_t nn = n > 0 ? n : 1;
  p3m::Workspace& W = P->ws;
  W.key = (int32_t*)take(sizeof(int32_t) * nn);
  W.rank = (int32_t*)take(sizeof(int32_t) * nn);
  W.perm = (int32_t*)take(sizeof(int32_t) * nn);
  W.skey = (int32_t*)take(sizeof(int32_t) * nn);
  W.count = (int32_t*)take(sizeof(int32_t) * (P->ncell + 1));
  W.start = (int32_t*)take(sizeof(int32_t) * (P->ncell + 1));
  W.scan_tmp = (int32_t*)take(sizeof(int32_t) * P->scan_tmp_len);
  W.gchunk = (int32_t*)take(sizeof(int32_t) * (P->ngroup + 1));
  W.goff = (int32_t*)take(sizeof(int32_t) * (P->ngroup + 1));
  W.items = (int2*)take(sizeof(int2) * P->max_items);
  W.rows = (int4*)take(sizeof(int4) * P->nrows);
  W.rec = take(4 * real * nn);
  W.split_tab = (float*)take(sizeof(float) * 4 * (p3m::kSplitBins + 1));
  W.split_tab64 = (double*)take(sizeof(double) * p3m::kSplitCoef64 * (p3m::kSplitBins + 1));
  return off;
}

int status_of(hipError_t e) {
  if (e == hipSuccess) return P3M_OK;
  if (e == hipErrorOutOfMemory) return P3M_ENOMEM;
  return P3M_EHIP;
}

}  // namespace

extern "C" int pp_force_noalloc(const p3m_params* params, int64_t n, const double* pos,
                                const double* mass, double mass_scalar, void* force,
                                int32_t force_fp32, void* hip_stream) {
  if (!params || n < 0) return P3M_EINVAL;
  if (n > P3M_NOALLOC_MAX_N || params->grid_n > P3M_NOALLOC_MAX_GRID) return P3M_ESIZE;
  p3m_plan P;
  int st = p3m::plan_geometry(*params, n, &P);
  if (st != P3M_OK) return st;
  if (n == 0) return P3M_OK;
  if (!pos || !force) return P3M_EINVAL;
  if (!mass && !std::isfinite(mass_scalar)) return P3M_EINVAL;
  const size_t fbytes = (size_t)(3 * n) * (force_fp32 ? sizeof(float) : sizeof(double));
  const auto lo = [](const void* p) { return (uintptr_t)p; };
  if ((lo(force) < lo(pos) + 3 * n * sizeof(double) && lo(pos) < lo(force) + fbytes) ||
      (mass && lo(force) < lo(mass) + n * sizeof(double) && lo(mass) < lo(force) + fbytes))
    return P3M_EINVAL;
  if (P.nrows > kMaxRows || carve(&P, nullptr, n) > kScratchBytes) return P3M_ESIZE;
  P.stream = (hipStream_t)hip_stream;
  P.count_dirty = 1;             // the array keeps the last call's counts: clear them
  P.timing_slot = -1;

  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return status_of(e);
  if (dev < 0 || dev >= kMaxDevices) return P3M_EINVAL;
  unsigned char* base = nullptr;
  if ((e = scratch_address(dev, &base)) != hipSuccess) return status_of(e);
  P.device = dev;
  carve(&P, base, n);
  if ((e = p3m::plan_upload_tables(&P, g_rows)) != hipSuccess) return status_of(e);
  if ((e = p3m::launch_bin(&P, n, pos, mass, mass_scalar)) != hipSuccess) return status_of(e);
  if ((e = p3m::launch_items(&P)) != hipSuccess) return status_of(e);
  e = params->precision == P3M_FP32
          ? p3m::launch_pairs<float>(&P, n, false, force, force_fp32 ? 1 : 0, mass == nullptr)
          : p3m::launch_pairs<double>(&P, n, false, force, force_fp32 ? 1 : 0, mass == nullptr);
  return status_of(e);
}
