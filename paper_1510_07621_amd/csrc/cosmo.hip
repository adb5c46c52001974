// Background cosmology for comoving kick and drift coefficients (host code).
//
// The guide evolves comoving positions and momenta (Ch. 6) over a global
// time step set as a fraction of the current age of the universe
// (Ch. 5, Delta t_factor), with the background set by H0, Omega_m,
// Omega_Lambda and a_begin (Ch. 5, cosmological parameters). With canonical
// momenta p = a^2 m dx/dt and the force F = -m grad(phi) of the comoving
// density, the leapfrog coefficients of one kick or drift from a0 to a1 are
//     c_kick  = int dt / a   = int_{a0}^{a1} da / (a^2 H(a)),
//     c_drift = int dt / a^2 = int_{a0}^{a1} da / (a^3 H(a)),
//     H(a) = H0 sqrt(Omega_m a^-3 + Omega_k a^-2 + Omega_Lambda),
//     Omega_k = 1 - Omega_m - Omega_Lambda,
// and the age is t(a) = int_0^a da / (a H(a)). The integrals are evaluated
// by adaptive Simpson quadrature in s = sqrt(a) (which removes the a^(1/2)
// behaviour of the age integrand at a = 0) to a relative tolerance of 1e-13.
#include <cmath>

#include "p3m_internal.h"

namespace {

struct Bg {
  double H0, Om, Ok, OL;
  double H(double a) const {
    return H0 * std::sqrt(Om / (a * a * a) + Ok / (a * a) + OL);
  }
};

// f(s) for the integrals in s = sqrt(a), da = 2 s ds.
enum class Kind { kAge, kKick, kDrift };

double integrand(const Bg& b, Kind k, double s) {
  double a = s * s;
  if (a <= 0) return 0.0;             // all three integrands vanish or are integrable at 0
  double h = b.H(a);
  switch (k) {
    case Kind::kAge: return 2.0 * s / (a * h);
    case Kind::kKick: return 2.0 * s / (a * a * h);
    case Kind::kDrift: return 2.0 * s / (a * a * a * h);
  }
  return 0.0;
}

double simpson(const Bg& b, Kind k, double lo, double hi, double flo, double fmid, double fhi,
               double whole, double tol, int depth) {
  double mid = 0.5 * (lo + hi);
  double lm = 0.5 * (lo + mid), rm = 0.5 * (mid + hi);
  double flm = integrand(b, k, lm), frm = integrand(b, k, rm);
  double left = (mid - lo) / 6.0 * (flo + 4.0 * flm + fmid);
  double right = (hi - mid) / 6.0 * (fmid + 4.0 * frm + fhi);
  double sum = left + right;
  if (depth <= 0 || std::fabs(sum - whole) <= 15.0 * tol)
    return sum + (sum - whole) / 15.0;
  return simpson(b, k, lo, mid, flo, flm, fmid, left, 0.5 * tol, depth - 1) +
         simpson(b, k, mid, hi, fmid, frm, fhi, right, 0.5 * tol, depth - 1);
}

double integrate(const Bg& b, Kind k, double a0, double a1) {
  double s0 = std::sqrt(a0), s1 = std::sqrt(a1);
  // split into pieces so the recursion tolerance is meaningful per piece
  const int pieces = 16;
  double total = 0.0;
  for (int p = 0; p < pieces; ++p) {
    double lo = s0 + (s1 - s0) * p / pieces, hi = s0 + (s1 - s0) * (p + 1) / pieces;
    double flo = integrand(b, k, lo), fhi = integrand(b, k, hi);
    double fmid = integrand(b, k, 0.5 * (lo + hi));
    double whole = (hi - lo) / 6.0 * (flo + 4.0 * fmid + fhi);
    double scale = std::fabs(whole) + 1e-300;
    total += simpson(b, k, lo, hi, flo, fmid, fhi, whole, 1e-14 * scale, 40);
  }
  return total;
}

bool valid(const p3m_cosmology* c) {
  if (!c || !(c->H0 > 0) || !std::isfinite(c->H0) || !(c->Omega_m > 0) ||
      !std::isfinite(c->Omega_m) || !std::isfinite(c->Omega_L))
    return false;
  return true;
}

Bg background(const p3m_cosmology* c) {
  return Bg{c->H0, c->Omega_m, 1.0 - c->Omega_m - c->Omega_L, c->Omega_L};
}

// H^2 must stay positive on [a0, a1] (no turnaround inside the step).
bool expanding(const Bg& b, double a0, double a1) {
  const int n = 64;
  for (int i = 0; i <= n; ++i) {
    double a = a0 + (a1 - a0) * i / n;
    double h2 = b.Om / (a * a * a) + b.Ok / (a * a) + b.OL;
    if (!(h2 > 0)) return false;
  }
  return true;
}

}  // namespace

extern "C" {

int p3m_cosmo_age(const p3m_cosmology* c, double a, double* t_out) {
  if (!valid(c) || !t_out || !(a > 0) || !std::isfinite(a)) return P3M_EINVAL;
  Bg b = background(c);
  if (!expanding(b, a * 1e-6, a)) return P3M_ERANGE;
  *t_out = integrate(b, Kind::kAge, 0.0, a);
  return P3M_OK;
}

int p3m_cosmo_scale_factor(const p3m_cosmology* c, double t, double* a_out) {
  if (!valid(c) || !a_out || !(t > 0) || !std::isfinite(t)) return P3M_EINVAL;
  Bg b = background(c);
  // bracket a with t(a_hi) >= t, then bisect on the monotone age
  double lo = 0.0, hi = 1.0, th = 0.0;
  for (int it = 0; it < 200; ++it) {
    if (!expanding(b, hi * 1e-6, hi)) return P3M_ERANGE;
    th = integrate(b, Kind::kAge, 0.0, hi);
    if (th >= t) break;
    lo = hi;
    hi *= 2.0;
  }
  if (th < t) return P3M_ERANGE;
  for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
    double mid = 0.5 * (lo + hi);
    if (integrate(b, Kind::kAge, 0.0, mid) < t) lo = mid; else hi = mid;
  }
  *a_out = 0.5 * (lo + hi);
  return P3M_OK;
}

int p3m_cosmo_kick_drift(const p3m_cosmology* c, double a0, double a1, double* c_kick,
                         double* c_drift) {
  if (!valid(c) || !c_kick || !c_drift || !(a0 > 0) || !(a1 >= a0) || !std::isfinite(a1))
    return P3M_EINVAL;
  Bg b = background(c);
  if (!expanding(b, a0, a1)) return P3M_ERANGE;
  *c_kick = integrate(b, Kind::kKick, a0, a1);
  *c_drift = integrate(b, Kind::kDrift, a0, a1);
  return P3M_OK;
}

int p3m_cosmo_kdk_step(const p3m_cosmology* c, double a, double dt_factor, double* a_next,
                       double* c_kick1, double* c_drift, double* c_kick2) {
  if (!valid(c) || !a_next || !c_kick1 || !c_drift || !c_kick2 || !(a > 0) ||
      !std::isfinite(a) || !(dt_factor > 0) || !std::isfinite(dt_factor))
    return P3M_EINVAL;
  // the step's length: dt_factor times the age at its start; the middle and
  // the end of the step in time, then their scale factors
  double t0 = 0, ah = 0, a1 = 0;
  int st = p3m_cosmo_age(c, a, &t0);
  if (st != P3M_OK) return st;
  const double dt = dt_factor * t0;
  if ((st = p3m_cosmo_scale_factor(c, t0 + 0.5 * dt, &ah)) != P3M_OK) return st;
  if ((st = p3m_cosmo_scale_factor(c, t0 + dt, &a1)) != P3M_OK) return st;
  double k1 = 0, k2 = 0, d = 0, unused = 0;
  if ((st = p3m_cosmo_kick_drift(c, a, ah, &k1, &unused)) != P3M_OK) return st;
  if ((st = p3m_cosmo_kick_drift(c, ah, a1, &k2, &unused)) != P3M_OK) return st;
  if ((st = p3m_cosmo_kick_drift(c, a, a1, &unused, &d)) != P3M_OK) return st;
  *a_next = a1;
  *c_kick1 = k1;
  *c_drift = d;
  *c_kick2 = k2;
  return P3M_OK;
}

}  // extern "C"
