// Host runtime: tree layout, interaction stencils, solve plans and launches.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "octo.h"
#include "octo_internal.h"

namespace octo {

// error carrying an octo_status across the C++ side of the library
struct Error {
    octo_status code;
    std::string msg;
};

[[noreturn]] void fail(octo_status code, const std::string &msg);
void check_hip(hipError_t e, const char *what);

// ---------------------------------------------------------------- layout

struct HostLevel {
    int n_nodes = 0, n_int = 0, n_rec = 0;
    std::vector<int32_t> nbr, child, parent, coord;
    std::vector<int64_t> out_base;
    std::vector<int32_t> flags;  // kLeaf* flags per node (leaf nodes)
    std::vector<char> int_child;  // per interior node: 1 if one of its children is interior
};

struct Layout {
    int n_levels = 0;
    int64_t n_leaf_cells = 0;
    int64_t sx = 64, sy = 8, sz = 1;
    std::vector<HostLevel> lv;
    std::vector<octo_leaf> leaves;  // caller order
};

// Validate a leaf list (tiling, nesting) and lay the tree out level by level.
// grid_level >= 0: uniform grid layout of 8 * 2^grid_level cells per axis for
// the caller's arrays; otherwise leaf-list layout.
Layout build_layout(const octo_leaf *leaves, int64_t n, int grid_level);

// Leaves of the adaptive tree of a density field (refinement + nesting).
std::vector<octo_leaf> adaptive_leaves(octo_boxmax_fn boxmax, void *user, int max_level, double threshold);

// ---------------------------------------------------------------- stencils

struct Stencil {
    double theta = 0;
    std::vector<int32_t> m2l, nearo, leaf, m2l_src, leaf_off, leaf_widx, m2l_touch, near_touch, m2l_src_touch;
    std::vector<int32_t> m2l_src_d;  // per m2l_src entry: its offset d, packed
    std::vector<int32_t> near_stage;  // the near-field kernel's halo staging table (kNearStage entries)
    std::vector<double> leaf_tab;
    // cross-level near partners: offsets, class masks, per-class touch masks
    // (8 per entry), weights (64 per entry), largest component of an offset
    std::vector<int32_t> xl_off, xl_cls, xl_touch;
    std::vector<double> xl_w;
    int xl_reach = 0;
    int m2l_beg[9], near_beg[9], leaf_beg[9];
    int leaf_oct_beg[73];
    int m2l_src_beg[73];
    int m2l_src_any[64];  // per (target class, source class): the union of its entries' touch masks
};

Stencil make_stencil(double theta);

// ---------------------------------------------------------------- plans

// Host description of the work of one or more trees (concatenated), uploaded
// into one device buffer.
struct PlanHost {
    std::vector<LevelDesc> levels;
    std::vector<TreeDesc> trees;
    std::vector<M2LItem> m2l;
    std::vector<LeafItem> leaf;
    std::vector<NodeItem> p2m;
    std::vector<M2LItem> m2l_nodes;  // (node, source-class group) items of the LDS-staged kernel
    std::vector<M2LItem> m2l_leaf;   // record leaves (leaf targets next to interior nodes), LDS-staged
    // interior nodes by level index (level l of every tree)
    std::vector<std::vector<NodeItem>> interior;
    // the interior nodes with an interior child, by level index: the L2L pass
    // (the other interior nodes are finished by their leaves, kLeafDefer)
    std::vector<std::vector<NodeItem>> l2l;
    std::vector<int32_t> tree_leaf_beg, tree_m2l_beg, tree_m2ln_beg, tree_m2lf_beg;  // per tree, +1 sentinel
};

struct DeviceBlock {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Plan {
    int n_trees = 0, n_levels_max = 0;
    int n_m2l = 0, n_leaf = 0, n_p2m = 0, n_m2l_nodes = 0, n_m2l_leaf = 0;
    std::vector<int> n_interior;        // per level index
    std::vector<size_t> interior_off;   // element offset into d_interior per level index
    std::vector<int> n_l2l;             // per level index: nodes of the L2L pass
    std::vector<size_t> l2l_off;        // element offset into d_l2l per level index
    LevelDesc *d_levels = nullptr;
    TreeDesc *d_trees = nullptr;
    M2LItem *d_m2l = nullptr;
    LeafItem *d_leaf = nullptr;
    NodeItem *d_p2m = nullptr;
    M2LItem *d_m2l_nodes = nullptr;
    M2LItem *d_m2l_leaf = nullptr;
    std::vector<char> sum_parts_level;  // per level index: partial slots summed in a separate wide pass
    int lds_min_level = 0;  // shallowest level with LDS-staged multipole items (n_levels_max if none)
    NodeItem *d_interior = nullptr;
    NodeItem *d_l2l = nullptr;
    int32_t *d_tree_leaf_beg = nullptr, *d_tree_m2l_beg = nullptr, *d_tree_m2ln_beg = nullptr,
            *d_tree_m2lf_beg = nullptr;
    double *d_stat = nullptr;      // n_leaf * kStat (per leaf node)
    int64_t *d_leaf_cnt = nullptr;  // n_leaf
    int64_t *d_m2l_cnt = nullptr;   // n_m2l + n_m2l_nodes
    double *d_out = nullptr;        // n_trees * 12: stats per tree
    double *d_stat_part = nullptr;  // n_trees * kStatBlocks * 12: the stats reduction's per-work-group slots
    int32_t *d_stat_done = nullptr; // n_trees: work-groups of the stats reduction finished (zero between solves)
    DeviceBlock block;
    std::vector<TreeDesc> trees_host;  // current tree descriptors (outputs, G, amc)
};

size_t plan_bytes(const PlanHost &ph);
size_t plan_layout(const PlanHost &ph, void *dev, Plan &plan, std::vector<char> &image);
void plan_upload(const PlanHost &ph, void *dev, Plan &plan, hipStream_t s);

struct StencilDevHolder {
    Stencil host;
    StencilDev dev;
    DeviceBlock block;
};

// ---------------------------------------------------------------- launches

struct LaunchOpts {
    int precision = OCTO_FP64;
    bool count = true;                   // count evaluated pairs (statistics; implies reduce)
    bool reduce = false;                 // net force / torque reductions without pair counts
    bool source = false;                 // second-source solve (potential of the density rate)
    bool amc = true;                     // angular-momentum correction (a kernel variant of the LDS-staged M2L)
    hipEvent_t *phase_events = nullptr;  // 8 events around the 7 phases + 1 before the LDS M2L kernel, or NULL
    hipStream_t aux = nullptr;           // second stream for concurrent multipole work, or NULL
    hipEvent_t fork = nullptr, join = nullptr;
    hipStream_t aux_near = nullptr;      // third stream for the near field, or NULL
    hipEvent_t fork_near = nullptr, join_near = nullptr;
};

// enqueue one full solve of a plan on stream s
void launch_solve(const Plan &plan, const StencilDev &st, const LaunchOpts &o, hipStream_t s);
// the record leaves' constant multipole records of a tree (once, with its plan)
void launch_leaf_records(const Plan &plan, hipStream_t s);
// coupling of the solve to the hydrodynamic update (single-tree plans)
void launch_sources(const Plan &p, const double omega[3], const double *rho, const double *s, const double *phi,
                    const double *g, const double *drho, const double *dphi, double *src_s, double *src_e,
                    hipStream_t st);
void launch_energy_update(int64_t n, const double *rho, const double *before, const double *after, double *E,
                          hipStream_t st);

}  // namespace octo

// ---------------------------------------------------------------- objects

namespace octo {
// a concatenated plan of several trees with its device block and graphs
struct BatchPlan {
    std::vector<octo_tree *> sig;
    PlanHost ph;
    Plan plan;
    void *mem = nullptr;
    size_t bytes = 0;
    std::map<std::pair<uint64_t, int>, hipGraphExec_t> graphs;  // (theta bits, precision)
    void *staging = nullptr;  // pinned upload image (asynchronous waves), from the context's pool
    size_t staging_bytes = 0;
    std::vector<double> stats;  // per tree, 12 values, after completion
    bool fitted = false;        // work shapes fitted to the batch (not each tree's own)
};

// an asynchronous request
struct Request {
    octo_ticket ticket;
    octo_tree *tree;
    octo_opts opts;
    double *phi, *g;
    int wave = -1;
    bool done = false;
    int index = 0;  // position in its wave
    double stats[12] = {0};
    octo_status status = OCTO_OK;  // OCTO_E_BUDGET: its plan does not fit even alone
    std::string err;
};

struct Wave {
    std::vector<octo_ticket> tickets;
    std::unique_ptr<BatchPlan> bp;
    hipEvent_t done = nullptr;
    bool finished = false;
    int lane = -1;
};

// The streams one launch wave of the request server runs on: waves in flight
// together run on different lanes, so their work overlaps on the device.
struct Lane {
    hipStream_t s = nullptr, aux = nullptr, aux_near = nullptr;
    hipEvent_t start = nullptr, fork = nullptr, join = nullptr, fork_near = nullptr, join_near = nullptr;
};
}  // namespace octo

namespace octo {
// the device layout's buffers, kept by the context: the dense cells of
// `levels` levels (all clear between uses) and the work arrays of `cap` nodes
struct LayBuf {
    void *cell = nullptr, *work = nullptr;
    size_t cell_bytes = 0, work_bytes = 0, sort_bytes = 0;
    int levels = 0;
    int64_t cap = 0;
    LayK pending{};  // the passes of the layout in progress (between layout_device and its tables)
    int *deepest = nullptr;  // one int: the deepest level of a leaf list (layout_device_levels)
};
}  // namespace octo

namespace octo {
// An event recorded after the last work enqueued on a tree's memory; the
// trees of one batched launch share one (a single record for all of them:
// each record is a packet the device processes in order, about 4 us apiece).
struct UseMark {
    hipEvent_t ev = nullptr;
    UseMark() {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) throw Error{OCTO_E_DEVICE, "event"};
    }
    ~UseMark() { (void)hipEventDestroy(ev); }
    UseMark(const UseMark &) = delete;
    UseMark &operator=(const UseMark &) = delete;
};
}  // namespace octo

struct octo_ctx {
    // serialises every call that touches the context (several threads may
    // build trees at once: validation and layout happen before the lock)
    mutable std::recursive_mutex mu;
    int device = 0;
    int n_cu = 256;  // compute units of the device (sizes the multipole work shape)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool has_alloc = false;
    octo_allocator alloc{};
    size_t budget = 0, in_use = 0;
    int n_trees = 0;
    std::map<uint64_t, std::unique_ptr<octo::StencilDevHolder>> stencils;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t capture = nullptr;  // private stream for graph capture
    hipStream_t aux = nullptr, capture_aux = nullptr;  // second streams (direct launches, capture)
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    hipStream_t aux_near = nullptr, capture_near = nullptr;  // near-field streams
    hipEvent_t fork_near_ev = nullptr, join_near_ev = nullptr;
    bool use_graphs = true;
    int profiling = 0;  // 0 off, 1 phase timings with statistics, 2 phase timings only
    int batch_shapes = 0;  // 1: octo_solve_batch fits the work shapes to the whole batch
    hipEvent_t phase_ev[9] = {};
    double *h_stats = nullptr;  // pinned host staging for stats
    // pinned upload buffers, reused (freeing pinned memory can wait for the
    // device); each is free once its event (the upload that read it) is done
    struct Pinned {
        void *p;
        size_t bytes;
        hipEvent_t ready;  // NULL: free now
    };
    std::vector<Pinned> pinned_free;
    void *pinned_get(size_t bytes, size_t *got);
    void pinned_put(void *p, size_t bytes, hipEvent_t ready = nullptr);
    size_t h_stats_cap = 0;
    // last batch signature (octo_solve_batch)
    std::unique_ptr<octo::BatchPlan> batch;
    void *batch_mem = nullptr;
    size_t batch_bytes = 0;
    // asynchronous requests
    octo_ticket next_ticket = 1;
    std::map<octo_ticket, octo::Request> requests;
    std::deque<octo_ticket> pending;
    std::map<int, octo::Wave> waves;
    int next_wave = 0;
    int max_inflight_waves = 2;
    std::vector<octo::Lane> lanes;  // max_inflight_waves lanes, created with the first wave

    octo::LayBuf lay;  // device layout (regridded trees)

    void *dev_alloc(size_t bytes);
    void dev_free(void *p, size_t bytes);
    const octo::StencilDevHolder &stencil(double theta);
    void invalidate_batches();
    void release_batch(octo::BatchPlan *bp);
};

struct octo_tree {
    octo_ctx *ctx = nullptr;
    octo::Layout layout;
    octo::PlanHost ph;    // single-tree plan (host copy)
    octo::Plan plan;      // single-tree plan (device)
    octo::DeviceBlock data;        // tables + fields
    octo::DeviceBlock plan_block;  // work plan
    std::vector<int> parts_alloc, parts, m2l_lds;  // per level: multipole work choices
    // work lists for batched solves by source-class group count (every level
    // below the root LDS-staged), built on first use
    std::map<int, octo::PlanHost> ph_batch;
    bool leaf_lds = true;  // leaf targets of multipole work in the LDS-staged kernel
    double *rho = nullptr;
    double *stage = nullptr;  // device staging of phi, g for host outputs
    std::shared_ptr<octo::UseMark> last_use;  // recorded after the last work enqueued on the tree's memory
    hipStream_t last_stream = nullptr;  // the stream last_use was recorded on
    size_t bytes = 0;
    std::map<std::pair<uint64_t, int>, hipGraphExec_t> graphs;  // (theta bits, precision)
};

namespace octo {
// Order work on the context stream after the tree's last use on another
// stream (a launch wave of the request server); a no-op wait is skipped.
inline void tree_acquire(octo_ctx *ctx, octo_tree *t) {
    if (t->last_stream && t->last_stream != ctx->stream) {
        if (hipStreamWaitEvent(ctx->stream, t->last_use->ev, 0) != hipSuccess)
            throw Error{OCTO_E_DEVICE, "stream wait on a tree's last use"};
    }
}
// record the last use of trees[0, n) on stream s: one event for all of them
// (a fresh one: an event another tree still holds is not moved)
inline void trees_release(octo_tree *const *trees, int n, hipStream_t s) {
    if (n <= 0) return;
    auto m = std::make_shared<UseMark>();
    if (hipEventRecord(m->ev, s) != hipSuccess) throw Error{OCTO_E_DEVICE, "event record"};
    for (int i = 0; i < n; ++i) {
        trees[i]->last_use = m;
        trees[i]->last_stream = s;
    }
}
inline void tree_release(octo_tree *t, hipStream_t s) { trees_release(&t, 1, s); }
// launch a plan through a cached graph (captured on first use) or directly
void run_plan(octo_ctx *ctx, Plan &plan, std::map<std::pair<uint64_t, int>, hipGraphExec_t> &graphs,
              const std::vector<TreeDesc> &want, const octo_opts *o, bool count = true, bool source = false,
              bool reduce = false);
void drop_graphs(std::map<std::pair<uint64_t, int>, hipGraphExec_t> &graphs);
// self-consistent-field iteration (Sec. 4.1) on the n^3 grid of `level`; s2:
// split between the two sides in half-cell units, x = s2 h/2 - 1/2
void scf_step(octo_ctx *ctx, int level, const octo_scf_params &p, double K, int64_t s2, const double *rho,
              const double *phi, double *rho_out, octo_scf_state *state);
// the same step with its scratch in a fixed per-device array (no allocation);
// scf_fixed_scratch_init(device) must have run with `device` current
void scf_step_noalloc(octo_ctx *ctx, int level, const octo_scf_params &p, double K, int64_t s2, const double *rho,
                      const double *phi, double *rho_out, octo_scf_state *state);
void scf_fixed_scratch_init(int device);
size_t scf_fixed_scratch_bytes();
void scf_run(octo_ctx *ctx, octo_tree *t, int level, const octo_opts &o, const octo_scf_params &p, int64_t s2,
             int iterations, double *rho_out, double *phi_out, octo_scf_state *history);
// one regrid by the density criterion (Sec. 2.7) on the device: the new leaf
// list and its densities (device, leaf layout), owned until destruction
struct RegridOut {
    octo_ctx *ctx = nullptr;
    void *scratch = nullptr, *out = nullptr;
    size_t scratch_bytes = 0, out_bytes = 0;
    double *rho = nullptr;
    const octo_leaf *leaves = nullptr;
    int64_t n_leaves = 0;
    int levels = 0;  // the new leaves lie in levels [0, levels)
    int64_t refined = 0, balance_refined = 0, derefined = 0;
    RegridOut() = default;
    RegridOut(const RegridOut &) = delete;
    RegridOut &operator=(const RegridOut &) = delete;
    ~RegridOut();
};
void regrid_device(octo_ctx *ctx, octo_tree *t, int l_max, double rho_r, RegridOut &r);
// Device layout of a leaf list in device memory (leaf-list layout, levels
// [0, levels) at most), on the context stream under the context lock:
// layout_device fills L's counts, leaf flags, parents, interior-child bits and
// leaf list (one synchronisation; OCTO_E_INVALID for a list that is not a
// tree); layout_device_tables then writes the node tables of the same list
// and clears the cells, or layout_device_abort only clears them.
void layout_device(octo_ctx *ctx, const octo_leaf *leaf, int64_t n, int levels, Layout &L);
// the level count a device leaf list needs (deepest level + 1, at most
// kMaxLevel + 1; one synchronisation)
int layout_device_levels(octo_ctx *ctx, const octo_leaf *leaf, int64_t n);
void layout_device_tables(octo_ctx *ctx, const LayTables &t);
void layout_device_abort(octo_ctx *ctx);
void layout_device_release(octo_ctx *ctx);
void build_tree_plan(octo_tree *t);
void phase_times(const octo_ctx *ctx, double *phase_ms);
void plan_items(const octo_tree *t, const std::vector<int> &parts, const std::vector<int> &m2l_lds, PlanHost &ph);
double lds_launch_cost(const std::vector<int64_t> &n_int, const std::vector<int> &g, int n_cu);
}  // namespace octo
