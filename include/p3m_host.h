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

/* Edge, in cells, of the i-groups the pair sum uses for n particles on a
 * grid of grid_n^3 cells: the power of two (1, 2 or 4) closest to a mean of
 * 8 particles per group, never larger than grid_n / 2. */
int32_t p3m_group_edge(int64_t n, int32_t grid_n);

#ifdef __cplusplus
}
#endif

#endif /* P3M_HOST_H */
