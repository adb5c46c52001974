// Kick and drift: the two particle updates of a leapfrog step, in FP64.
//
//   kick:  p <- p + c_kick F
//   drift: x <- wrap(x + c_drift (p / m)),  wrap(y) = y - box floor(y / box),
//          a result equal to box becomes 0
//
// Every product, quotient, sum and difference is a single correctly rounded
// IEEE double operation in this order (floating-point contraction is switched
// off in these kernels, so no multiply-add is fused), which makes the updates
// reproducible bit for bit on any IEEE implementation that performs the same
// operations.
#include "p3m_internal.h"

namespace p3m {
namespace {

constexpr int kThreads = 256;

template <typename F>
__global__ void k_kick(int64_t n, double* __restrict__ mom, const F* __restrict__ force,
                       double c) {
#pragma clang fp contract(off)
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  double f = (double)force[i];
  mom[i] = mom[i] + c * f;
}

__global__ void k_drift(int64_t n, double* __restrict__ pos, const double* __restrict__ mom,
                        const double* __restrict__ mass, double mass_scalar, double c,
                        double box) {
#pragma clang fp contract(off)
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  int64_t i = k % n;
  double m = mass ? mass[i] : mass_scalar;
  double v = mom[k] / m;
  double y = pos[k] + c * v;
  double w = y - box * floor(y / box);
  pos[k] = (w >= box) ? 0.0 : w;
}

// Kick then drift in one pass over the particles (the first half of a
// kick-drift-kick step): the same operations in the same order as k_kick
// followed by k_drift, so the result is bitwise the same, without writing and
// re-reading the momenta.
template <typename F>
__global__ void k_kick_drift(int64_t n, double* __restrict__ pos, double* __restrict__ mom,
                             const F* __restrict__ force, const double* __restrict__ mass,
                             double mass_scalar, double ck, double cd, double box) {
#pragma clang fp contract(off)
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  int64_t i = k % n;
  double f = (double)force[k];
  double p = mom[k] + ck * f;
  mom[k] = p;
  double m = mass ? mass[i] : mass_scalar;
  double v = p / m;
  double y = pos[k] + cd * v;
  double w = y - box * floor(y / box);
  pos[k] = (w >= box) ? 0.0 : w;
}

// Kick and reorder: component k = d n + s of the outputs takes particle
// i = order[s] of the inputs; the momentum's sum is k_kick's operation.
template <typename F>
__global__ void k_kick_reorder(int64_t n, const int32_t* __restrict__ order,
                               const double* __restrict__ pos, const double* __restrict__ mom,
                               const F* __restrict__ force, const int64_t* __restrict__ ids,
                               const double* __restrict__ mass, double c,
                               double* __restrict__ pos_out, double* __restrict__ mom_out,
                               int64_t* __restrict__ ids_out, double* __restrict__ mass_out) {
#pragma clang fp contract(off)
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  const int64_t d = k / n, s = k - d * n;
  // (clamped: an order that is not a permutation gives wrong values, never
  // an access outside the arrays)
  const int64_t o = min(max((int64_t)order[s], (int64_t)0), n - 1);
  const int64_t i = d * n + o;
  double f = (double)force[k];
  mom_out[k] = mom[i] + c * f;
  pos_out[k] = pos[i];
  if (d == 0) {
    if (ids) ids_out[s] = ids[o];
    if (mass) mass_out[s] = mass[o];
  }
}

}  // namespace

hipError_t launch_kick_reorder(int64_t n, const int32_t* order, const double* pos,
                               const double* mom, const void* force, int fp32,
                               const int64_t* ids, const double* mass, double c,
                               double* pos_out, double* mom_out, int64_t* ids_out,
                               double* mass_out, hipStream_t s) {
  unsigned blocks = (unsigned)((3 * n + kThreads - 1) / kThreads);
  if (fp32)
    k_kick_reorder<float><<<blocks, kThreads, 0, s>>>(n, order, pos, mom, (const float*)force,
                                                      ids, mass, c, pos_out, mom_out, ids_out,
                                                      mass_out);
  else
    k_kick_reorder<double><<<blocks, kThreads, 0, s>>>(n, order, pos, mom,
                                                       (const double*)force, ids, mass, c,
                                                       pos_out, mom_out, ids_out, mass_out);
  return hipGetLastError();
}

hipError_t launch_kick_drift(int64_t n, double* pos, double* mom, const void* force, int fp32,
                             const double* mass, double ms, double ck, double cd, double box,
                             hipStream_t s) {
  unsigned blocks = (unsigned)((3 * n + kThreads - 1) / kThreads);
  if (fp32)
    k_kick_drift<float><<<blocks, kThreads, 0, s>>>(n, pos, mom, (const float*)force, mass, ms,
                                                    ck, cd, box);
  else
    k_kick_drift<double><<<blocks, kThreads, 0, s>>>(n, pos, mom, (const double*)force, mass,
                                                     ms, ck, cd, box);
  return hipGetLastError();
}

hipError_t launch_kick(int64_t n, double* mom, const void* force, int fp32, double c,
                       hipStream_t s) {
  unsigned blocks = (unsigned)((3 * n + kThreads - 1) / kThreads);
  if (fp32)
    k_kick<float><<<blocks, kThreads, 0, s>>>(n, mom, (const float*)force, c);
  else
    k_kick<double><<<blocks, kThreads, 0, s>>>(n, mom, (const double*)force, c);
  return hipGetLastError();
}

hipError_t launch_drift(int64_t n, double* pos, const double* mom, const double* mass,
                        double ms, double c, double box, hipStream_t s) {
  unsigned blocks = (unsigned)((3 * n + kThreads - 1) / kThreads);
  k_drift<<<blocks, kThreads, 0, s>>>(n, pos, mom, mass, ms, c, box);
  return hipGetLastError();
}

}  // namespace p3m
