/*
 * p3m_host.h -- host-only helpers of libp3m.so (no GPU needed).
 *
 * These expose the plan's geometry decisions so they can be checked on a
 * machine without a GPU. They allocate nothing and launch nothing.
 */
#ifndef P3M_HOST_H
#define P3M_HOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Short-range neighbour stencil of an i-group of g x g x g cells.
 *
 * The pair sum visits, for each i-group, every cell whose box comes closer
 * than r_c to the group's box (cells of side h, radius_cells = r_c / h).
 * Cells are visited as z-runs: row k is (dx, dy, dz_lo, dz_hi), the cells at
 * offsets (dx, dy, dz) from the group's first cell for dz_lo <= dz <= dz_hi.
 * Writes min(count, cap) rows as 4 int32 each into rows_out (may be NULL when
 * cap == 0) and returns the total count, or P3M_EINVAL (-1) for g < 1 or
 * radius_cells <= 0 or non-finite. */
int32_t p3m_stencil_rows(int32_t g, double radius_cells, int32_t* rows_out,
                         int32_t cap);

/* The same stencil cut into group segments, for the pair sum that evaluates
 * a pair of particles in two dense groups once (the force on one is minus
 * that on the other; Newton's third law). A cell at offset d from the
 * group's first cell lies in the group offset o = floor(d / g) (per axis);
 * every row is cut where its z range crosses a multiple of g, and each piece
 * carries the lexicographic sign of its (ox, oy, oz): +1, -1, or 0 for the
 * group itself. Of two distinct groups, exactly one sees the other at a
 * positive offset. Entries of 4 int32: (dx & 0xffff) | (dy << 16), dz_lo,
 * dz_hi, sign; in the order of p3m_stencil_rows, pieces by increasing z.
 * Writes min(count, cap) entries, returns the count or P3M_EINVAL as
 * p3m_stencil_rows. */
int32_t p3m_segment_rows(int32_t g, double radius_cells, int32_t* rows_out, int32_t cap);

/* Table of the split factor f = erfc(u) + (2u/sqrt(pi)) exp(-u^2),
 * u = r / (2 r_s), that the FP32 pair sum evaluates (P3M short-range force,
 * CONCEPT User's Guide, Ch. 5: P3M_scale, P3M_cutoff, softening). Arguments:
 * cutoff_rs = r_c / r_s, softening_rs = eps / r_s.
 *
 * The table variable v (in units of r_s) is the softened distance
 * sqrt(r^2 + eps^2) / r_s when cubic pieces of f over it stay within 1e-7 of
 * f (f has a kink at r = 0, which only pieces that are wide against eps
 * follow), else r / r_s. [v0, v1] is cut into B equal bins; with
 * x = (v - v0) B / (v1 - v0), k = floor(x), t = x - k, the table gives
 * f = c0[k] + t (c1[k] + t (c2[k] + t c3[k])), the cubic through f at the four
 * Chebyshev points of bin k; entry B is the constant f at v1 (for arguments
 * rounded up onto the cutoff).
 *
 * Layout: out[c * (B + 1) + k] for c = 0..3, k = 0..B; map_out (may be NULL)
 * receives {variable (0: r, 1: softened distance), v0, v1}. Returns B and
 * writes the 4 (B + 1) floats and the map when cap >= 4 (B + 1) (out may be
 * NULL with cap == 0). P3M_EINVAL (-1) for cutoff_rs <= 0, softening_rs < 0,
 * a non-finite argument, or cap > 0 with NULL out. */
int32_t p3m_split_table(double cutoff_rs, double softening_rs, float* out, int32_t cap,
                        double* map_out);

/* FP64 table of the same split factor f: the variable v is chosen as for the
 * FP32 table, but the softened distance is kept whenever only up to 8
 * leading bins (next to the kink at r = 0, with r / (2 r_s) <= 0.9) miss
 * twice the accuracy of the table over r (at least 4e-16); the pair sum
 * evaluates those bins with a power series of f. [v0, v1] is cut into B equal
 * bins; with x = (v - v0) B / (v1 - v0), k = floor(x), t = x - k,
 * f = sum_{l=0..6} c_l[k] t^l, the degree-6 polynomial through f at the
 * seven Chebyshev points of bin k (fitted in extended precision); entry B is
 * the constant f at v1. Layout: out[l * (B + 1) + k], l = 0..6, k = 0..B;
 * map_out (may be NULL) receives {variable (0: r, 1: softened distance), v0,
 * v1, exact bins}. Returns B and writes the 7 (B + 1) doubles and the map
 * when cap >= 7 (B + 1) (out may be NULL with cap == 0). P3M_EINVAL (-1) for
 * cutoff_rs <= 0, softening_rs < 0, a non-finite argument, or cap > 0 with
 * NULL out. */
int32_t p3m_split_table64(double cutoff_rs, double softening_rs, double* out, int32_t cap,
                          double* map_out);

/* Edge, in cells, of the i-groups the pair sum uses for n particles on a
 * grid of grid_n^3 cells: the power of two (1, 2 or 4) closest to a mean of
 * 64 particles per group, never larger than grid_n / 2. */
int32_t p3m_group_edge(int64_t n, int32_t grid_n);

/* Background cosmology for comoving kick and drift coefficients (CONCEPT
 * User's Guide, Ch. 5: H0, Omega_m, Omega_Lambda, a_begin, and a time step
 * given as a fraction of the age of the universe; Ch. 6: comoving positions
 * and momenta). H(a) = H0 sqrt(Omega_m a^-3 + Omega_k a^-2 + Omega_Lambda)
 * with Omega_k = 1 - Omega_m - Omega_Lambda; H0 in inverse time units of the
 * simulation. Errors: P3M_EINVAL for a null pointer, H0 <= 0, Omega_m <= 0,
 * non-finite values or a <= 0; P3M_ERANGE if H^2 <= 0 somewhere on the
 * range (a turnaround). */
typedef struct p3m_cosmology {
  double H0;
  double Omega_m;
  double Omega_L;
} p3m_cosmology;

/* Age t(a) = int_0^a da' / (a' H(a')). */
int p3m_cosmo_age(const p3m_cosmology* c, double a, double* t_out);

/* Inverse of the age: the scale factor a with t(a) = t (t > 0). */
int p3m_cosmo_scale_factor(const p3m_cosmology* c, double t, double* a_out);

/* Leapfrog coefficients between scale factors a0 <= a1, for canonical
 * momenta p = a^2 m dx/dt and a force F = -m grad(phi) computed from the
 * comoving density: c_kick = int dt / a (use p += c_kick F) and
 * c_drift = int dt / a^2 (use x += c_drift p / m), both integrated over
 * a in [a0, a1] with dt = da / (a H(a)). */
int p3m_cosmo_kick_drift(const p3m_cosmology* c, double a0, double a1, double* c_kick,
                         double* c_drift);

/* One kick-drift-kick step in comoving coordinates whose length is a
 * fraction dt_factor of the age of the universe at its start (guide Ch. 5:
 * Delta_t_factor; H0, Omega_m, Omega_Lambda and a_begin set the background):
 * with t0 = t(a) and dt = dt_factor t0, the step ends at a_next = a(t0 + dt);
 * the first kick covers the first half in time, [a, a(t0 + dt/2)], the
 * second kick the second half, and the drift the whole step, so a step is
 *   p += c_kick1 F(x);  x = wrap(x + c_drift p / m);  p += c_kick2 F(x)
 * with the canonical momenta of p3m_cosmo_kick_drift. Errors as for those
 * calls; P3M_EINVAL also for dt_factor <= 0 or non-finite, or a null output. */
int p3m_cosmo_kdk_step(const p3m_cosmology* c, double a, double dt_factor, double* a_next,
                       double* c_kick1, double* c_drift, double* c_kick2);

#ifdef __cplusplus
}
#endif

#endif /* P3M_HOST_H */
