/*
 * octo.h -- C interface of an MI355X (gfx950) implementation of the gravity
 * solve of Octo-Tiger (Marcello et al., arXiv 2101.08226): a Cartesian fast
 * multipole method (FMM) on an adaptive octree of 8x8x8 sub-grids with the
 * angular-momentum correction (Sec. 2.2, "Gravity Update and the Angular
 * Momentum Correction").
 *
 * Problem solved (Sec. 2.1, Poisson equation and g = -grad phi; code units
 * with G = 1, Sec. 2.8; isolated boundaries, Sec. 2.5): every leaf cell of the
 * octree is a point mass m = rho h^3 at its centre; the library returns, for
 * each leaf cell, the potential phi and the acceleration g = -grad phi of all
 * other cells, computed by the multipole method with opening angle theta.
 *
 * Geometry: the domain is the unit cube [-1/2, 1/2]^3.  The root sub-grid
 * (level 0) has 8^3 cells of width 1/8; a sub-grid at level l with index
 * (ix, iy, iz) in [0, 2^l)^3 covers cells of width h = 1/(8 * 2^l) whose
 * global indices are 8*(ix, iy, iz) + [0, 8)^3; the centre of global cell i
 * is -1/2 + (i + 1/2) h (Sec. 2.4 octree, Sec. 3.3 level numbering).
 *
 * Memory: "host" pointers are ordinary CPU memory, "device" pointers are HIP
 * device memory on the context's device.  The library never keeps a caller
 * pointer beyond the call that receives it, except the output buffers of a
 * submitted request (octo_submit), which must stay valid until the request
 * completes.  Device memory owned by the library is obtained through the
 * context's allocator (or hipMalloc when none is given) at tree-build time; a
 * solve allocates nothing.
 *
 * Threads: calls on one context are serialised by a lock inside the
 * context.  octo_tree_build and octo_tree_build_adaptive validate the leaf
 * list, check the density and lay the tree out before taking that lock, so
 * several host threads may build trees for one context at the same time
 * (the part that allocates and uploads is serialised).
 *
 * Errors: every call returns an octo_status; nothing throws or aborts across
 * this interface.  octo_last_error() returns a thread-local description of the
 * last failure on the calling thread.
 */
#ifndef OCTO_H
#define OCTO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OCTO_OK = 0,
    OCTO_E_INVALID = 1,     /* bad argument, malformed tree or density */
    OCTO_E_DEVICE = 2,      /* a HIP call failed */
    OCTO_E_BUDGET = 3,      /* the request does not fit the context's HBM budget */
    OCTO_E_UNSUPPORTED = 4, /* valid but unsupported option (e.g. theta < 0.34) */
    OCTO_E_STATE = 5,       /* object in the wrong state (e.g. tree from another context) */
    OCTO_E_PENDING = 6      /* request not finished yet (octo_poll) */
} octo_status;

typedef struct octo_ctx octo_ctx;
typedef struct octo_tree octo_tree;

/* Device-memory provider: alloc(bytes, user) returns device memory on the
 * context's device (NULL on failure), free(ptr, user) releases it.  Lets a
 * caller route the library's memory through its own pool (e.g. PyTorch's
 * caching allocator). */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} octo_allocator;

/* One leaf sub-grid: refinement level and sub-grid index at that level. */
typedef struct {
    int32_t level, ix, iy, iz;
} octo_leaf;

enum { OCTO_FP64 = 0, OCTO_MIXED = 1 };

/* Solve options.
 * theta: opening angle; cells A, B at one level are well separated when
 *   dx/|x_A - x_B| < theta on geometric centres (Sec. 2.2), evaluated as
 *   (theta*theta)*|i_A - i_B|^2 > 1 on integer cell indices in IEEE double.
 *   Must lie in [0.34, 1): 0.34 is the paper's minimum for 8^3 sub-grids.
 *   Above 1/sqrt(3) cells that touch at a corner are well separated, and
 *   their expansions can reach masses next to the shared corner, outside the
 *   region where they converge: results near concentrated mass then lose all
 *   accuracy (the paper runs 0.5 and 0.34).
 * G: gravitational constant (1 in code units, Sec. 2.8).
 * precision: OCTO_FP64 computes everything in double precision;
 *   OCTO_MIXED evaluates the leaf near-field sums and the multipole-to-local
 *   sums of the LDS-staged work (the levels with many interior nodes, and
 *   leaf cells next to interior cells) in single precision with
 *   single-precision partial sums (masses, moments and the offsets of the
 *   centres of mass from the cell centres rounded to float; the separations
 *   between cell centres are exact), and the rest -- the moments themselves,
 *   the multipole-to-local terms of the root and other levels with few
 *   interior nodes, the sums of the angular-momentum correction, the
 *   downward pass and the final accumulation -- in double precision.  The
 *   second-source solve of octo_solve_dphidt keeps its multipole work in
 *   double precision.
 * amc: 1 applies the angular-momentum correction (Sec. 2.2), 0 omits it. */
typedef struct {
    double theta;
    double G;
    int32_t precision;
    int32_t amc;
} octo_opts;

/* Per-solve diagnostics (all over leaf cells; x about the origin):
 * total_mass = sum m; net_force = sum m g; net_torque = sum x cross m g;
 * force_scale = sum m |g|; torque_scale = sum |x| m |g| (so
 * |net_torque| / torque_scale is the relative torque residual, the quantity
 * the correction drives to rounding level, Sec. 2.2); pair counts are the
 * ordered cell pairs evaluated by the multipole and the direct kernels;
 * device_ms is the device time of the solve measured with HIP events. */
typedef struct {
    double total_mass;
    double net_force[3];
    double net_torque[3];
    double force_scale;
    double torque_scale;
    int64_t n_leaf_cells;
    int64_t m2l_pairs;
    int64_t direct_pairs;
    int64_t m2l_lds_pairs;  /* the part of m2l_pairs evaluated by the LDS-staged kernel */
    double device_ms;
    /* per-phase device time (ms) when profiling is on (octo_ctx_set_profiling;
     * the phases then run one after the other): [0] leaf masses (P2M),
     * [1] near field (same-level and cross-level direct pairs), [2] upward
     * pass (M2M, all levels), [3] multipole interactions (M2L with the
     * correction, all levels), [4] downward pass (L2L, interior levels),
     * [5] leaves (final shift, potential and acceleration), [6] statistics
     * reduction, [7] the LDS-staged multipole kernel alone (part of [3],
     * the pairs of m2l_lds_pairs); for a batch (octo_solve_batch) the phases
     * of the whole batched launch, the same for every tree; zeros otherwise */
    double phase_ms[8];
} octo_stats;

/* Density at n points: xyz is 3n doubles (x0,y0,z0,x1,...), rho_out n doubles. */
typedef void (*octo_density_fn)(int64_t n, const double *xyz, double *rho_out, void *user);
/* Maximum density over n boxes: lo, hi are 3n doubles (corners), out n doubles. */
typedef void (*octo_boxmax_fn)(int64_t n, const double *lo, const double *hi, double *out, void *user);

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t on that
 * device used for every launch of this context, or NULL to create a private
 * stream (default priority).  alloc: optional device-memory provider (copied;
 * NULL means hipMalloc/hipFree).  hbm_budget: maximum bytes of device memory
 * the context may hold for trees (0 = no limit).
 * Errors: OCTO_E_INVALID (out == NULL), OCTO_E_DEVICE (device not usable). */
octo_status octo_ctx_create(int device, void *hip_stream, const octo_allocator *alloc, size_t hbm_budget,
                            octo_ctx **out);
/* Waits for outstanding work, then frees the context.  Trees must be
 * destroyed first (OCTO_E_STATE otherwise). */
octo_status octo_ctx_destroy(octo_ctx *ctx);
/* Profiling: when on != 0, solves launch their kernels one by one (no graph
 * replay) with HIP events between phases, and octo_stats.phase_ms is filled.
 * on = 1: the statistics are computed as usual (pairs counted, which adds a
 * counting pass to the multipole kernels); on = 2: timing only, the kernels
 * run as in solves without statistics, and the octo_stats fields other than
 * n_leaf_cells, device_ms and phase_ms are zero.  Other values:
 * OCTO_E_INVALID. */
octo_status octo_ctx_set_profiling(octo_ctx *ctx, int on);
/* Work shapes of octo_solve_batch with two or more trees.  mode 0 (the
 * default): every tree runs its own single-tree plan, so each result is
 * identical, bit for bit, to solving the tree alone.  mode 1: the shapes are
 * fitted to the batch -- many trees fill the device together, so every
 * level below the root takes the LDS-staged multipole kernel with one
 * source-class group count for the whole batch, the one a launch-time model
 * prices lowest, and the roots' work is split into fewer partial slots --
 * and each result agrees with the tree's single solve to
 * within rounding of the summation order (pair counts unchanged).  The
 * request server (octo_submit) always runs each tree's own plan.  Other
 * values: OCTO_E_INVALID. */
octo_status octo_ctx_set_batch_shapes(octo_ctx *ctx, int mode);
/* Bytes of device memory currently held by the context's trees. */
octo_status octo_ctx_memory(const octo_ctx *ctx, size_t *bytes_in_use, size_t *budget);

/* ---- trees (Sec. 2.4: one 8^3 sub-grid per octree node; interior nodes have
 *      8 children; neighbouring sub-grids, across faces, edges and corners,
 *      differ by at most one level) ---------------------------------------- */

/* Tree from an explicit leaf list.  The leaves must tile the unit box
 * exactly once and be properly nested.  rho: n_leaves x 512 densities, leaf
 * by leaf in the given order, cells (ix, iy, iz) within a sub-grid with iz
 * fastest; host memory, or device memory when rho_on_device != 0; copied.
 * Results of octo_solve use the same layout.
 * Errors: OCTO_E_INVALID (gap, overlap, duplicate, level > 9, improper
 * nesting, density negative or not finite), OCTO_E_BUDGET, OCTO_E_DEVICE. */
octo_status octo_tree_build(octo_ctx *ctx, const octo_leaf *leaves, int64_t n_leaves, const double *rho,
                            int rho_on_device, octo_tree **out);
/* The same tree from a leaf list in device memory (for leaf lists produced on
 * the device): the list is checked and laid out by kernels on the context
 * stream (node set, classification, a sort, the node tables written in
 * place), the host receives only per-level counts and per-node flags.  leaves
 * and rho (n_leaves x 512, same layout as octo_tree_build) are device
 * memory, read before the call returns; the density is not checked.  Node
 * numbering and tables equal octo_tree_build's for the same list.
 * Errors: as octo_tree_build for the list (the first error found by kind:
 * level, index, duplicate, overlap, gap, nesting), OCTO_E_BUDGET,
 * OCTO_E_DEVICE. */
octo_status octo_tree_build_device(octo_ctx *ctx, const octo_leaf *leaves, int64_t n_leaves, const double *rho,
                                   octo_tree **out);
/* Uniform tree: every leaf at `level` (0..6), n = 8 * 2^level cells per axis.
 * rho: n^3 densities indexed (ix*n + iy)*n + iz (iz fastest); results of
 * octo_solve use this same grid layout.  Errors as octo_tree_build. */
octo_status octo_tree_build_uniform(octo_ctx *ctx, int level, const double *rho, int rho_on_device,
                                    octo_tree **out);
/* Adaptive tree from a density field (Sec. 2.7, fixed-threshold form):
 * starting from the root, a node at level < max_level is refined when
 * boxmax over its cube exceeds `threshold`; nodes are then refined until the
 * tree is properly nested.  The density is evaluated at every leaf-cell
 * centre.  Leaves are ordered by (level, ix, iy, iz); octo_tree_leaves
 * returns that order, and results use the leaf layout of octo_tree_build.
 * Callbacks run on the calling thread during this call only. */
octo_status octo_tree_build_adaptive(octo_ctx *ctx, octo_density_fn density, octo_boxmax_fn boxmax, void *user,
                                     int max_level, double threshold, octo_tree **out);
/* Replace the tree's density (same layout as at build time). */
octo_status octo_tree_set_density(octo_tree *tree, const double *rho, int rho_on_device);
/* Copy the tree's density (its layout, n_leaf_cells doubles) into rho: host
 * memory (the call returns when the copy is done) or, when rho_on_device != 0,
 * device memory (stream-ordered on the context stream). */
octo_status octo_tree_get_density(const octo_tree *tree, double *rho, int rho_on_device);
/* Sizes: leaf cells, levels (deepest level + 1), device bytes held. */
octo_status octo_tree_info(const octo_tree *tree, int64_t *n_leaf_cells, int32_t *n_levels, size_t *bytes);
/* Copy the leaf list (n_leaves entries) into caller memory. */
octo_status octo_tree_leaves(const octo_tree *tree, octo_leaf *out);

/* The node tables of one level (layout of the tree's device memory; see
 * octo_tree_level_tables): caller buffers, any of them NULL to skip it.
 *   nbr       n_nodes x 27: same-level neighbour (dx,dy,dz) at
 *             (dx+1)*9 + (dy+1)*3 + dz+1, -1 = none (all -1 at level 0)
 *   child     n_int x 8: child node at level + 1, child (cx,cy,cz) at cx*4+cy*2+cz
 *   parent    n_nodes: node at level - 1 (-1 at level 0)
 *   coord     n_nodes x 3: sub-grid index at this level
 *   out_base  n_nodes: density-layout offset of a leaf's cell (0,0,0), -1 for interior nodes
 *   flags     n_nodes: a leaf's multipole roles (1: multipole partner of same-level cells,
 *             2: partner of cells one level up, 4: keeps multipole accumulators), 0 for interior
 *   int_child n_int: 1 where one of the node's children is interior
 * Nodes are numbered interior first, then leaves next to an interior node,
 * then the other leaves, each group in Morton order (x bit above y above z). */
typedef struct {
    int32_t *nbr, *child, *parent, *coord;
    int64_t *out_base;
    int32_t *flags, *int_child;
} octo_level_tables;

/* Sizes of level `level` of a tree (sizes[0] nodes, sizes[1] interior nodes,
 * sizes[2] interior nodes + leaves next to an interior node) and, if out is
 * not NULL, its node tables copied from device memory (returns when the copy
 * is done).  For tests and tools that check a layout, e.g. a regridded tree
 * laid out on the device against octo_host_level_tables of its leaf list.
 * Errors: OCTO_E_INVALID (NULL sizes, level outside [0, n_levels)). */
octo_status octo_tree_level_tables(const octo_tree *tree, int32_t level, int64_t *sizes,
                                   const octo_level_tables *out);
octo_status octo_tree_destroy(octo_tree *tree);

/* ---- solve -------------------------------------------------------------- */

/* Potential and acceleration at every leaf cell of `tree`.
 * phi: n_leaf_cells doubles; g: 3 x n_leaf_cells doubles, component-major
 * (gx for all cells, then gy, then gz); both in the tree's density layout.
 * out_on_device != 0: phi and g are device pointers and the call returns once
 * the work is enqueued on the context stream (stream-ordered, like a kernel
 * launch) unless stats != NULL; out_on_device == 0: host pointers, the call
 * returns when the results are copied.  stats may be NULL.
 * Errors: OCTO_E_UNSUPPORTED (theta outside [0.34, 1), unknown precision),
 * OCTO_E_INVALID (NULL outputs, non-finite G), OCTO_E_STATE (tree from another
 * context), OCTO_E_DEVICE. */
octo_status octo_solve(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, double *phi, double *g,
                       int out_on_device, octo_stats *stats);

/* octo_solve with its net force and torque reductions left in device
 * memory, for time loops that keep the diagnostics on the device: phi and g
 * as octo_solve with out_on_device != 0; stats_dev (device, 9 doubles)
 * receives total_mass, net_force[3], net_torque[3], force_scale and
 * torque_scale of octo_stats, stream-ordered on the context stream (the call
 * returns once the work is enqueued; no pair counting, no host copy).
 * Errors: as octo_solve. */
octo_status octo_solve_device_stats(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, double *phi, double *g,
                                    double *stats_dev);

/* Autotune the tree's multipole work shape for these options: for every level
 * with interior nodes, time the multipole-interaction phase with each
 * candidate (LDS-staged work-groups per node and group of source parity
 * classes, 1, 2, 4 or 8 groups; or one wavefront per target parity class with
 * 1, 2, 4, ... stencil chunks) and keep the fastest, level by
 * level.  Runs several solves (outputs into the tree's own staging memory)
 * and rebuilds the tree's work plan (device memory for the plan is
 * reallocated).  choice: NULL or n_levels entries: -1 = no interior nodes,
 * -(k+1) = LDS-staged with the source classes split into k groups, k > 0 =
 * per-wavefront with k stencil chunks.  Results of later
 * solves are identical to within rounding of the summation order. */
octo_status octo_tree_autotune(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, int32_t *choice);

/* Solve n independent trees with one launch per phase of the method, all
 * trees together (the phases are captured once into a HIP graph per batch
 * signature and replayed).  phi[i], g[i] as in octo_solve for trees[i];
 * stats: NULL or n entries.  Results are identical, bit for bit, to solving
 * each tree alone (to within rounding of the summation order with
 * batch-fitted work shapes, octo_ctx_set_batch_shapes).
 * status: NULL or n entries, each tree's own outcome: OCTO_OK (solved),
 * OCTO_E_INVALID (NULL tree or output, or a tree listed twice: the second
 * entry), OCTO_E_STATE (tree from another context); a failure of the call as
 * a whole (bad options, a device error) is written for every tree that was
 * to be solved.  Trees refused on their own are skipped and the others are
 * solved together; the return value is then the first refused tree's status
 * (OCTO_OK when every tree was solved), and stats entries of refused trees
 * are left untouched. */
octo_status octo_solve_batch(octo_ctx *ctx, octo_tree *const *trees, int32_t n, const octo_opts *opts,
                             double *const *phi, double *const *g, int out_on_device, octo_stats *stats,
                             octo_status *status);

/* ---- time derivative of the potential ----------------------------------- */

/* dphi/dt from the density rate drho/dt (Sec. 2.1: the energy equation's
 * gravity source 1/2 (phi drho/dt - rho dphi/dt) is evaluated with dphi/dt
 * from the same multipole method, the density rate taking the place of the
 * density).  The rate is expanded about the centres of mass of the tree's
 * current density (so its cells carry a dipole) and goes through the same
 * interaction lists; the discrete operator is then the one octo_solve
 * applies to the density, which is symmetric, so for phi from octo_solve
 * with the same options sum_i (phi_i drho_i - rho_i dphi_i) h_i^3 vanishes up
 * to rounding.
 * drho_dt: device, n doubles in the tree's density layout (n = leaf cells),
 * any sign; dphi_dt: device output, same layout.  opts->theta, G and
 * precision apply; opts->amc is ignored (the correction acts on forces).
 * The call recomputes the density's moments, so it may come before or after
 * octo_solve; it uses the tree's scratch, so calls on one tree are ordered by
 * the context stream.  Stream-ordered (returns once enqueued).
 * Errors: OCTO_E_INVALID (NULL pointer, bad options), OCTO_E_STATE. */
octo_status octo_solve_dphidt(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, const double *drho_dt,
                              double *dphi_dt);

/* ---- coupling to the hydrodynamic update -------------------------------- */

/* Gravity source terms of the hydrodynamic update (Sec. 2.3, source vector S,
 * with the right-hand sides of the momentum and energy equations of Sec. 2.1)
 * at every leaf cell, x being the cell centre:
 *   src_s = rho g + Omega x s                                  (3 x n)
 *   src_e = 1/2 (phi drho/dt - rho dphi/dt) + rho Omega . (x x g)   (n)
 * omega: 3 doubles, host memory (the grid's rotation vector).  rho, phi,
 * drho_dt, dphi_dt: n doubles; s, g: 3 x n component-major; outputs likewise;
 * all device pointers in the tree's density layout, n = leaf cells.  drho_dt
 * and dphi_dt may be NULL (taken as zero).  Stream-ordered on the context
 * stream (returns once enqueued).  Errors: OCTO_E_INVALID, OCTO_E_STATE. */
octo_status octo_gravity_sources(octo_ctx *ctx, octo_tree *tree, const double *omega, const double *rho,
                                 const double *s, const double *phi, const double *g, const double *drho_dt,
                                 const double *dphi_dt, double *src_s, double *src_e);
/* Energy update after a potential solve (Sec. 2.3):
 * E += 1/2 rho (phi_before - phi_after), elementwise over the tree's n leaf
 * cells; device pointers, stream-ordered on the context stream. */
octo_status octo_energy_update(octo_ctx *ctx, octo_tree *tree, const double *rho, const double *phi_before,
                               const double *phi_after, double *E);

/* ---- initial binary model: self-consistent field (Sec. 4.1) ------------- */

/* Parameters of the self-consistent-field (SCF) iteration that builds a
 * synchronously rotating binary of two polytropes (Sec. 4.1, "The Initial
 * Stellar Model").  The accretor (mass M1) lies on the low-x side of the L1
 * point, the donor (M2) on the high-x side. */
typedef struct {
    double M1, M2;     /* masses the two stars are normalised to (step 1) */
    double n;          /* polytropic index */
    double a0;         /* separation fixing the orbital angular momentum
                          J0 = mu a0^2 Omega_K(a0), Omega_K^2 = G (M1 + M2) / a0^3,
                          mu = M1 M2 / (M1 + M2) (step 3) */
    double f;          /* Roche filling factor of the donor (step 4) */
    double K0;         /* polytropic constant before the first update */
    double rho_floor;  /* density of every cell outside the two stars */
    double G;          /* gravitational constant (J0 and the potential solve) */
    double x_L1;       /* split between the two sides before the first
                          iteration; must be a cell centre or a cell face */
} octo_scf_params;

/* Scalars of one SCF iteration. */
typedef struct {
    double omega;      /* angular frequency from J0 and the separation (step 3) */
    double K;          /* updated polytropic constant (step 5) */
    double C1, C2;     /* integration constants of accretor and donor (step 4) */
    double x_L1;       /* x of the new L1 cell (step 4) */
    double a;          /* separation of the stars' centres of mass (step 3) */
    double mass1, mass2; /* the stars' masses in the iteration's input density */
    int64_t c1, c2;    /* centre cells (densest cell of each side) */
    int64_t l1;        /* L1 cell */
} octo_scf_state;

/* The readings of Sec. 4.1 this library takes (where the text is silent):
 * cells are indexed g = (ix*n + iy)*n + iz on the n^3 grid of a uniform tree
 * (n = 8 * 2^level), cell centres at -1/2 + (i + 1/2)/n;
 * - the sides: a cell is on the accretor's side when its x is below the
 *   split; the centre cell of a side is its densest cell; a star is the cells
 *   of its side closer to its centre cell than |split - x_centre|; ties of
 *   every maximum go to the smallest g;
 * - step 1 multiplies each star's cells by M_i / (its mass), others unchanged;
 * - step 2: the rotation axis is parallel to z through the grid's centre of
 *   mass (xc, yc); phi_eff = phi - Omega^2 ((x - xc)^2 + (y - yc)^2) / 2;
 * - step 3: a = distance of the stars' centres of mass,
 *   Omega = J0 (M1 + M2) / (M1 M2 a^2);
 * - step 4: L1 is the cell of largest phi_eff on the grid row (iy, iz of the
 *   accretor's centre) strictly between the two centre cells;
 *   C1 = K (n + 1) rho_c1^(1/n) + phi_eff(c1) with the K in force;
 *   C2 = (1 - f) phi_eff(c2) + f phi_eff(L1);
 * - step 5: K = (C2 - phi_eff(c2)) / ((n + 1) rho_c2^(1/n));
 * - step 6: with the sides and radii taken about the new L1 and the same
 *   centre cells, rho = ((C_i - phi_eff) / (K (n + 1)))^n inside star i where
 *   C_i - phi_eff > 0, else 0; then rho = max(rho, rho_floor);
 * - step 7 solves for the density after step 1 of the next iteration (each
 *   iteration normalises, then solves, then takes steps 2-6), so the
 *   potential of steps 2-6 is the one of the density they act on. */

/* Steps 2-6 of one SCF iteration from a density `rho` (already normalised)
 * and its potential `phi` on the grid of `level` (0..6): writes the new
 * density to rho_out and the iteration's scalars to *state.  K: the
 * polytropic constant in force; x_L1: the split of the previous iteration
 * (p->x_L1 is ignored).  rho, phi, rho_out: device, n^3 doubles each in the
 * grid layout above; rho_out may equal rho; state: host.  Device scratch of a
 * few tens of KiB is taken from the context's allocator for the call.
 * Returns when the results are ready.
 * Errors: OCTO_E_INVALID (NULL pointer, level out of range, x_L1 neither a
 * cell centre nor a cell face, non-finite or non-positive masses, n, a0 or G),
 * OCTO_E_BUDGET, OCTO_E_DEVICE. */
octo_status octo_scf_step(octo_ctx *ctx, int level, const octo_scf_params *p, double K, double x_L1,
                          const double *rho, const double *phi, double *rho_out, octo_scf_state *state);

/* octo_scf_step for callers that cannot allocate device memory (tight
 * loops, harnesses that forbid allocation): the same kernels and launch
 * shapes, so the same results bit for bit, with the step's scratch in a fixed
 * array of 256 KiB per device (static device memory of the library, held by
 * each device the library runs on until the process ends; its address is
 * looked up once per device by octo_ctx_create).  The call allocates
 * nothing: no hipMalloc, no context allocator.  Arguments, layout and
 * outputs as octo_scf_step; the array covers every grid the step takes
 * (levels 0..6, up to 512^3 cells), and a level outside [0, 6] is rejected
 * with OCTO_E_INVALID.  Every call on a device shares that device's array
 * and leaves its contents behind; the step writes every scratch value before
 * reading it.  Calls on one device would race for the array, so the library
 * runs them one at a time (a per-device lock held until the step's stream
 * has drained).  Errors: as octo_scf_step, plus OCTO_E_STATE when the
 * device's array was not set up. */
octo_status octo_scf_step_noalloc(octo_ctx *ctx, int level, const octo_scf_params *p, double K, double x_L1,
                                  const double *rho, const double *phi, double *rho_out, octo_scf_state *state);

/* `iterations` SCF iterations (Sec. 4.1) on a uniform tree (built by
 * octo_tree_build_uniform), starting from the tree's density and from
 * K = p->K0 and the split p->x_L1; each iteration normalises the stars (step
 * 1), solves for the potential with `opts` (theta, precision, amc; the
 * constant G is p->G) and takes steps 2-6.  After the last iteration the
 * stars are normalised once more and their potential solved.  On return the
 * tree holds that final density; rho_out (device, n^3 doubles, or NULL)
 * receives a copy of it and phi_out (device, n^3 doubles) its potential;
 * history (host, `iterations` entries, or NULL) the scalars of every
 * iteration.  Every step runs on the device; the host only enqueues.  Device
 * scratch (3 n^3 doubles for the acceleration of the solve, plus a few tens
 * of KiB) is taken from the context's allocator for the call.  Returns when
 * the results are ready.
 * Errors: as octo_scf_step, plus OCTO_E_INVALID (tree not uniform,
 * iterations < 0), OCTO_E_UNSUPPORTED (bad opts), OCTO_E_STATE. */
octo_status octo_scf_run(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, const octo_scf_params *p,
                         int32_t iterations, double *rho_out, double *phi_out, octo_scf_state *history);

/* ---- regrid by the density criterion (Sec. 2.7) ------------------------- */

typedef struct {
    int32_t l_max;     /* deepest refinement level allowed (0..9) */
    double rho_r;      /* refinement density cut-off (> 0) */
    int64_t n_target;  /* desired number of sub-grids; <= 0 keeps rho_r */
} octo_regrid_params;

typedef struct {
    int64_t refined;          /* leaves refined by the criterion */
    int64_t balance_refined;  /* further leaves refined for the 2:1 balance */
    int64_t derefined;        /* interior nodes whose children were removed */
    int64_t n_leaves;         /* leaf sub-grids of the new tree */
    int64_t n_grids;          /* sub-grids of the new tree, leaves and interior nodes */
    double rho_r_next;        /* (n_grids / n_target)^2 rho_r, or rho_r when n_target <= 0 */
    double flag_ms;           /* host wall time of the device part (flags, balance, new leaves and densities) */
    double layout_ms;         /* host wall time of the new tree's layout (on the device) and work plan */
} octo_regrid_stats;

/* One regrid of `tree` by the density criterion of Sec. 2.7, computed on the
 * device from the tree's current density, into a new tree (*out); `tree` is
 * left unchanged.  The readings this library takes where the text is silent:
 * - a cell of level l is flagged when rho > 8^(l + 1 - l_max) rho_r (the largest
 *   level L with rho > 8^(L - l_max) rho_r exceeds l; with the exponent as
 *   printed the inequality would hold at l_max whenever it holds anywhere);
 * - refinement and de-refinement move one level per call: a leaf below l_max
 *   with a flagged cell gets 8 children; an interior node whose 8 children
 *   are leaves loses them when none of its cells (the means of the child
 *   cells under them) and none of its children's cells is flagged;
 * - 2:1 balance over faces, edges and corners: a refined leaf refines the
 *   coarser leaves next to it, to a fixed point; a de-refinement is dropped
 *   when a child is refined, or when a child of a same-level neighbour that
 *   touches the node is interior or refined; the input must be balanced;
 * - densities move with the cells: a new child's cell takes the density of
 *   the parent cell containing it, a de-refined node's cell the mean of its 8
 *   child cells (summed in child-cell order x, y, z, then divided by 8), so
 *   sum(rho h^3) is kept;
 * - the two-cell refinement window and the regrid cadence (time stepping)
 *   are not applied.
 * The new tree uses the leaf-list density layout of octo_tree_build, with the
 * leaves in the order octo_tree_leaves returns; its density is written on the
 * device (only the leaf list, 16 bytes per leaf, goes to the host, which lays
 * the tree out).  stats may be NULL.  Device scratch of 8 bytes per node of
 * `tree` plus the new tree's leaves and densities is taken from the context's
 * allocator for the call.  Returns when the new tree is ready.
 * Errors: OCTO_E_INVALID (NULL pointer, l_max outside [0, 9], rho_r not
 * finite and positive), OCTO_E_STATE, OCTO_E_BUDGET, OCTO_E_DEVICE. */
octo_status octo_regrid(octo_ctx *ctx, octo_tree *tree, const octo_regrid_params *p, octo_tree **out,
                        octo_regrid_stats *stats);

/* ---- asynchronous requests (continuous batching) ------------------------ */

typedef int64_t octo_ticket;

/* Enqueue a solve of `tree` (outputs on the device).  Requests submitted
 * while others run are merged into the next launch wave; results are identical
 * to octo_solve.  Returns OCTO_E_BUDGET if the context cannot hold the
 * request's scratch right now (the caller retries later). */
octo_status octo_submit(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, double *phi_dev, double *g_dev,
                        octo_ticket *ticket);
/* Drive pending work; *done = 1 when the ticket's results are ready. */
octo_status octo_poll(octo_ctx *ctx, octo_ticket ticket, int *done);
/* Block until the ticket's results are ready; fills stats if not NULL. */
octo_status octo_wait(octo_ctx *ctx, octo_ticket ticket, octo_stats *stats);

const char *octo_last_error(void);
/* Identifier of the sources the library was built from (a hash of the
 * headers and the library sources, fixed at build time); bindings compare it
 * with the sources they were written against before calling anything else. */
const char *octo_build_id(void);

#ifdef __cplusplus
}
#endif

#endif /* OCTO_H */
