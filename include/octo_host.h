/*
 * octo_host.h -- host-only introspection of liboctofmm (no GPU needed).
 *
 * These calls expose the library's host logic -- tree validation and layout,
 * adaptive refinement, interaction stencils -- so that it can be checked on a
 * machine without a GPU.  They allocate only host memory and never touch a
 * device.  Return values and errors follow include/octo.h (octo_status, with
 * octo_last_error() describing failures).
 */
#ifndef OCTO_HOST_H
#define OCTO_HOST_H

#include "octo.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Stencil sizes for opening angle theta (levels >= 1), per parity class p of
 * the target cell (p = (ix&1)<<2 | (iy&1)<<1 | (iz&1)):
 * out[p] = multipole partners (well separated, parents not; Sec. 2.2),
 * out[8+p] = near partners (neither, excluding the cell itself),
 * out[16+p] = maximum |offset| component over both lists.
 * Errors: OCTO_E_UNSUPPORTED for theta outside [0.34, 1). */
octo_status octo_host_stencil_sizes(double theta, int32_t *out);

/* The near-field walk of the leaf kernel for opening angle theta (levels >= 1):
 * the entries of target class p and sign octant o (o = (dx<0)<<2 | (dy<0)<<1 |
 * (dz<0) for the nonzero components of d; a zero component may sit in either
 * octant of its axis) are d[beg[9*p+o] .. beg[9*p+o+1]), each packed as
 * (dx & 255) | (dy & 255) << 8 | (dz & 255) << 16, with 0 for the padding
 * that fills every octant list to whole blocks of 8.  beg holds 73 entries
 * (beg[72] = total).  If d is NULL or cap is too small only beg and *n are set.
 * Errors: OCTO_E_UNSUPPORTED for theta outside [0.34, 1). */
octo_status octo_host_near_lists(double theta, int32_t *beg, int32_t *d, int64_t cap, int64_t *n);

/* The staging table of the near-field kernel's leaf-mass halo (the 18^3 cells
 * within 5 cells of a sub-grid, Sec. 2.2's near partners of its cells): entry
 * e = u * 512 + t (thread t, step u < 12) names halo cell c = e (local
 * coordinate (c / 324 - 5, (c / 18) % 18 - 5, c % 18 - 5)) as
 * slot | store << 5 | dest << 14, where slot is the neighbour sub-grid
 * ((sx >> 3) + 1) * 9 + ((sy >> 3) + 1) * 3 + (sz >> 3) + 1, store the cell's
 * parity-major storage index there, and dest its index in the parity-split
 * halo; -1 for e >= 18^3.  out must hold cap >= 6144 entries; *n = 6144.
 * Errors: OCTO_E_INVALID for NULL pointers. */
octo_status octo_host_near_stage(int32_t *out, int64_t cap, int64_t *n);

/* Validate a leaf list exactly as octo_tree_build does and report its layout:
 * out[3*l+0] = nodes at level l, out[3*l+1] = interior nodes, out[3*l+2] =
 * leaf nodes that touch an interior node of their level; *n_levels = deepest
 * level + 1.  out must hold 3 * 10 entries. */
octo_status octo_host_layout(const octo_leaf *leaves, int64_t n_leaves, int32_t *n_levels, int64_t *out);

/* The layout octo_tree_build gives a leaf list (leaf-list density layout):
 * sizes of level `level` (as octo_tree_level_tables) and, if out is not
 * NULL, its node tables in the format of octo_level_tables.
 * Errors: as octo_tree_build for the list; OCTO_E_INVALID for a level
 * outside [0, deepest level]. */
octo_status octo_host_level_tables(const octo_leaf *leaves, int64_t n_leaves, int32_t level, int64_t *sizes,
                                   const octo_level_tables *out);

/* Leaf list of octo_tree_build_adaptive (same refinement and nesting rule,
 * same order).  If out is NULL or cap is too small only *n is set. */
octo_status octo_host_adaptive_leaves(octo_boxmax_fn boxmax, void *user, int max_level, double threshold,
                                      octo_leaf *out, int64_t cap, int64_t *n);

#ifdef __cplusplus
}
#endif

#endif /* OCTO_HOST_H */
