// C-ABI of the library: contexts, trees, solves, batches and asynchronous
// requests.  Every entry point converts C++ failures into an octo_status and a
// thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <cstdlib>
#include <string>

#include "runtime.h"

using namespace octo;

namespace {

thread_local std::string g_err;

octo_status ok() { return OCTO_OK; }

}  // namespace

namespace octo {
void set_error(const std::string &m) { g_err = m; }
}  // namespace octo

namespace {

template <typename F>
octo_status guard(F &&f) {
    try {
        f();
        return ok();
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host out of memory";
        return OCTO_E_BUDGET;
    } catch (const std::exception &e) {
        g_err = e.what();
        return OCTO_E_INVALID;
    } catch (...) {
        g_err = "unknown error";
        return OCTO_E_INVALID;
    }
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        hipGetDevice(&prev);
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) hipSetDevice(prev);
    }
};

int n_parts_for(int n_int, int target) {
    if (n_int <= 0) return 1;
    int p = target / (8 * n_int);
    return std::max(1, std::min(32, p));
}

// Offsets in a tree's device data block: every index table first, then the
// density (together one contiguous upload), then the per-level fields.
struct TreeBlock {
    std::vector<size_t> nbr, child, parent, coord, out, mass, mp, loc, lacc, nf, dip, cm;
    size_t rho = 0, stage = 0, upload = 0, bytes = 0;
};

}  // namespace

namespace octo {
// Modelled time of one launch of the LDS-staged multipole kernel over levels
// of n_int[i] nodes split into g[i] source-class groups each: the items are
// dealt to the 8 XCDs in equal shares of every level, larger items first
// (the order the plans give them), and each XCD's work-group slots (two per
// CU) take the next item as they free up; the time is the simulated makespan
// in class-rounds (a round stages and walks one class per work-group) plus
// the downward pass reading g partial slots per node, about 0.002 of a
// class-round per slot of one node.
double lds_launch_cost(const std::vector<int64_t> &n_int, const std::vector<int> &g, int n_cu) {
    const int cus = std::max(8, n_cu), per_xcd = std::max(1, 2 * cus / 8);
    std::vector<std::pair<int, int64_t>> groups;  // (classes per item, items per XCD)
    double slots = 0.0;
    for (size_t i = 0; i < n_int.size(); ++i) {
        groups.push_back({8 / g[i], (n_int[i] * g[i] + 7) / 8});
        slots += (double)n_int[i] * g[i];
    }
    std::sort(groups.begin(), groups.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    std::map<int64_t, int64_t> load{{0, per_xcd}};  // CU load -> number of CUs
    for (const auto &gr : groups) {
        int64_t left = gr.second;
        while (left > 0) {
            auto it = load.begin();
            const int64_t at = it->first, k = std::min(left, it->second);
            if ((it->second -= k) == 0) load.erase(it);
            load[at + gr.first] += k;
            left -= k;
        }
    }
    return (double)load.rbegin()->first + 0.002 * slots;
}
}  // namespace octo

namespace {

// Per-level work shapes (partial slots, LDS-staged multipole kernel) and the
// data block's offsets: host work only, no context state but its CU count.
void shape_tree(octo_tree *t, TreeBlock &B) {
    const octo_ctx *ctx = t->ctx;
    const Layout &L = t->layout;
    const int nl = L.n_levels;
    t->parts_alloc.assign(nl, 1);
    t->parts.assign(nl, 1);
    t->m2l_lds.assign(nl, 0);
    const char *mode = getenv("OCTO_M2L");
    const bool lds = !(mode && std::string(mode) == "global");
    t->leaf_lds = lds;
    for (int l = 0; l < nl; ++l) {
        const HostLevel &h = L.lv[l];
        t->parts_alloc[l] = std::max(n_parts_for(h.n_int, 1024), l >= 1 ? 4 : 1);
        t->parts[l] = n_parts_for(h.n_int, 256);
        // dense levels take the LDS-staged kernel
        t->m2l_lds[l] = (lds && l >= 1 && t->parts[l] == 1) ? 1 : 0;
    }
    // The LDS-staged levels share one launch: split each node's source parity
    // classes into g_l groups per level (one work-group each), priced by
    // lds_launch_cost.  Levels are tuned one at a time from a common best g,
    // fewest nodes first.
    {
        std::vector<int> lds_levels;
        int g_max = 8;
        for (int l = 0; l < nl; ++l)
            if (t->m2l_lds[l] && L.lv[l].n_int > 0) {
                lds_levels.push_back(l);
                g_max = std::min(g_max, t->parts_alloc[l]);
            }
        if (!lds_levels.empty()) {
            std::vector<int64_t> n_int;
            for (int l : lds_levels) n_int.push_back(L.lv[l].n_int);
            auto cost = [&](const std::vector<int> &g) { return lds_launch_cost(n_int, g, ctx->n_cu); };
            std::vector<int> g(lds_levels.size(), 1);
            double best_cost = 1e300;
            for (int gu = 1; gu <= g_max; gu *= 2) {
                std::vector<int> u(lds_levels.size(), gu);
                const double c = cost(u);
                if (c < best_cost) {
                    best_cost = c;
                    g = u;
                }
            }
            std::vector<size_t> order(lds_levels.size());
            for (size_t i = 0; i < order.size(); ++i) order[i] = i;
            std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
                return L.lv[lds_levels[a]].n_int < L.lv[lds_levels[b]].n_int;
            });
            for (size_t i : order) {
                for (int gi = 1; gi <= g_max; gi *= 2) {
                    std::vector<int> trial = g;
                    trial[i] = gi;
                    const double c = cost(trial);
                    if (c < best_cost - 1e-9) {
                        best_cost = c;
                        g = trial;
                    }
                }
            }
            for (size_t i = 0; i < lds_levels.size(); ++i) t->parts[lds_levels[i]] = g[i];
        }
    }
    for (auto *v : {&B.nbr, &B.child, &B.parent, &B.coord, &B.out, &B.mass, &B.mp, &B.loc, &B.lacc, &B.nf, &B.dip, &B.cm})
        v->assign(nl, 0);
    size_t bytes = 0;
    for (int l = 0; l < nl; ++l) {
        const HostLevel &h = L.lv[l];
        const size_t nn = h.n_nodes;
        B.nbr[l] = bytes;
        bytes += al(nn * 27 * 4);
        B.child[l] = bytes;
        bytes += al((size_t)h.n_int * 8 * 4);
        B.parent[l] = bytes;
        bytes += al(nn * 4);
        B.coord[l] = bytes;
        bytes += al(nn * 3 * 4);
        B.out[l] = bytes;
        bytes += al(nn * 8);
    }
    B.rho = bytes;
    bytes += al((size_t)L.n_leaf_cells * 8);
    B.upload = bytes;
    for (int l = 0; l < nl; ++l) {
        const HostLevel &h = L.lv[l];
        B.mass[l] = bytes;
        bytes += al((size_t)h.n_nodes * kCells * 8);
        B.mp[l] = bytes;
        bytes += al((size_t)kRec * h.n_rec * kCells * 8);
        B.loc[l] = bytes;
        bytes += al((size_t)t->parts_alloc[l] * kLoc * h.n_int * kCells * 8);
        B.lacc[l] = bytes;
        bytes += al((size_t)kLacc * (h.n_rec - h.n_int) * kCells * 8);
        B.nf[l] = bytes;
        bytes += al((size_t)4 * (h.n_nodes - h.n_int) * kCells * 8);
        B.dip[l] = bytes;
        bytes += al((size_t)3 * h.n_rec * kCells * 8);
        B.cm[l] = bytes;
        bytes += al((size_t)h.n_int * kCells * 8 * 8);
    }
    B.stage = bytes;
    bytes += al((size_t)L.n_leaf_cells * 8 * 4);
    B.bytes = bytes;
}

// The upload image: tables (and a host density) at their offsets.
void stage_tree(const octo_tree *t, const TreeBlock &B, const double *rho_host, char *img) {
    const Layout &L = t->layout;
    for (int l = 0; l < L.n_levels; ++l) {
        const HostLevel &h = L.lv[l];
        if (!h.nbr.empty()) memcpy(img + B.nbr[l], h.nbr.data(), h.nbr.size() * 4);
        if (!h.child.empty()) memcpy(img + B.child[l], h.child.data(), h.child.size() * 4);
        if (!h.parent.empty()) memcpy(img + B.parent[l], h.parent.data(), h.parent.size() * 4);
        if (!h.coord.empty()) memcpy(img + B.coord[l], h.coord.data(), h.coord.size() * 4);
        if (!h.out_base.empty()) memcpy(img + B.out[l], h.out_base.data(), h.out_base.size() * 8);
    }
    if (rho_host) memcpy(img + B.rho, rho_host, (size_t)L.n_leaf_cells * 8);
}

// Under the context lock: allocate the data block, enqueue the upload of the
// image (pinned; handed back to the context's pool, reusable once the copy is
// done; none for tables laid out on the device) and fill the level and tree
// descriptors.  A device density is copied; unless its owner keeps it until
// the stream has passed the copy (wait_rho false), the copy is waited for.
void commit_tree(octo_tree *t, const TreeBlock &B, void *img, size_t img_bytes, const double *rho_dev,
                 bool wait_rho = true) {
    octo_ctx *ctx = t->ctx;
    const Layout &L = t->layout;
    const int nl = L.n_levels;
    void *mem = ctx->dev_alloc(B.bytes);
    t->data.ptr = mem;
    t->data.bytes = B.bytes;
    char *base = (char *)mem;
    hipStream_t s = ctx->stream;
    if (img)
        check_hip(hipMemcpyAsync(base, img, rho_dev ? B.rho : B.upload, hipMemcpyHostToDevice, s), "tree upload");
    if (rho_dev)
        check_hip(hipMemcpyAsync(base + B.rho, rho_dev, (size_t)L.n_leaf_cells * 8, hipMemcpyDeviceToDevice, s),
                  "density copy");
    if (img || (rho_dev && wait_rho)) {
        hipEvent_t done = nullptr;
        check_hip(hipEventCreateWithFlags(&done, hipEventDisableTiming), "event");
        check_hip(hipEventRecord(done, s), "event");
        // a caller's device density is read by the copy: done before returning
        if (rho_dev && wait_rho) check_hip(hipEventSynchronize(done), "density copy");
        if (img)
            ctx->pinned_put(img, img_bytes, done);
        else
            hipEventDestroy(done);
    }
    PlanHost &ph = t->ph;
    ph = PlanHost{};
    ph.levels.resize(nl);
    ph.trees.resize(1);
    for (int l = 0; l < nl; ++l) {
        const HostLevel &h = L.lv[l];
        LevelDesc &d = ph.levels[l];
        d.level = l;
        d.n_nodes = h.n_nodes;
        d.n_int = h.n_int;
        d.n_rec = h.n_rec;
        d.parent_ld = l > 0 ? l - 1 : -1;
        d.child_ld = (h.n_int > 0 && l + 1 < nl) ? l + 1 : -1;
        d.n_parts = t->parts[l];
        d.tree = 0;
        d.h = 1.0 / (double)(8 << l);
        d.nbr = (const int32_t *)(base + B.nbr[l]);
        d.child = (const int32_t *)(base + B.child[l]);
        d.parent = (const int32_t *)(base + B.parent[l]);
        d.coord = (const int32_t *)(base + B.coord[l]);
        d.out_base = (const int64_t *)(base + B.out[l]);
        d.mass = (double *)(base + B.mass[l]);
        d.mp = (double *)(base + B.mp[l]);
        d.loc = (double *)(base + B.loc[l]);
        d.lacc = (double *)(base + B.lacc[l]);
        d.nf = (double *)(base + B.nf[l]);
        d.dip = (double *)(base + B.dip[l]);
        d.cm = (double *)(base + B.cm[l]);
    }
    t->rho = (double *)(base + B.rho);
    t->stage = (double *)(base + B.stage);
    TreeDesc &td = ph.trees[0];
    td = TreeDesc{};
    td.rho = t->rho;
    td.phi = t->stage;
    td.g = t->stage + L.n_leaf_cells;
    td.n_leaf_cells = L.n_leaf_cells;
    td.sx = L.sx;
    td.sy = L.sy;
    td.sz = L.sz;
    td.G = 1.0;
    td.amc = 1;
}

}  // namespace

namespace octo {
// per-phase device times of the last profiled launch (its events have completed)
void phase_times(const octo_ctx *ctx, double *phase_ms) {
    for (int i = 0; i < 7; ++i) {
        float pm = 0.f;
        hipEventElapsedTime(&pm, ctx->phase_ev[i], ctx->phase_ev[i + 1]);
        phase_ms[i] = pm;
    }
    float pm = 0.f;
    hipEventElapsedTime(&pm, ctx->phase_ev[8], ctx->phase_ev[4]);
    phase_ms[7] = pm;
}

// (Re)build the tree's single-tree plan from its per-level choices: multipole
// kernel (LDS-staged per node, or chunked per wavefront with `parts` slots).
// The plan image goes up from pinned staging, ordered on the context stream.
void build_tree_plan(octo_tree *t) {
    octo_ctx *ctx = t->ctx;
    PlanHost &ph = t->ph;
    plan_items(t, t->parts, t->m2l_lds, ph);
    t->ph_batch.clear();
    const size_t bytes = plan_bytes(ph);
    void *mem = ctx->dev_alloc(bytes);
    const TreeDesc keep = t->plan.trees_host.empty() ? ph.trees[0] : t->plan.trees_host[0];
    if (t->plan_block.ptr) {
        // a rebuilt plan: the old one may still be in use by queued work
        check_hip(hipStreamSynchronize(ctx->stream), "plan rebuild");
        ctx->dev_free(t->plan_block.ptr, t->plan_block.bytes);
    }
    t->plan_block.ptr = mem;
    t->plan_block.bytes = bytes;
    ph.trees[0] = keep;
    std::vector<char> img;
    plan_layout(ph, mem, t->plan, img);
    size_t got = 0;
    void *pin = ctx->pinned_get(img.size(), &got);
    memcpy(pin, img.data(), img.size());
    check_hip(hipMemcpyAsync(mem, pin, img.size(), hipMemcpyHostToDevice, ctx->stream), "plan upload");
    launch_leaf_records(t->plan, ctx->stream);
    hipEvent_t done = nullptr;
    check_hip(hipEventCreateWithFlags(&done, hipEventDisableTiming), "event");
    check_hip(hipEventRecord(done, ctx->stream), "event");
    ctx->pinned_put(pin, got, done);
    drop_graphs(t->graphs);
    t->bytes = t->data.bytes + bytes;
}

// The work lists of a tree's plan for given per-level choices: LDS-staged
// multipole kernel or not, and partial slots (source-class groups of the
// LDS-staged kernel, stencil chunks of the per-wavefront one); ph holds the
// tree's level and tree descriptors already.
void plan_items(const octo_tree *t, const std::vector<int> &parts, const std::vector<int> &m2l_lds, PlanHost &ph) {
    const Layout &L = t->layout;
    const int nl = L.n_levels;
    ph.m2l.clear();
    ph.m2l_nodes.clear();
    ph.m2l_leaf.clear();
    ph.leaf.clear();
    ph.p2m.clear();
    ph.interior.assign(nl, {});
    ph.l2l.assign(nl, {});
    // interior nodes without an interior child: their leaves finish their
    // expansions, where the level has at most 4 partial slots (each leaf sums
    // them one after the other; levels with more keep the wide slot sum and
    // the L2L pass)
    std::vector<std::vector<char>> defer(nl);
    for (int l = 0; l < nl; ++l) {
        const HostLevel &h = L.lv[l];
        defer[l].assign(h.n_int, parts[l] <= 4 ? 1 : 0);
        for (int n = 0; n < h.n_int; ++n)
            if (h.int_child[n]) defer[l][n] = 0;
    }
    for (int l = 0; l < nl; ++l) {
        const HostLevel &h = L.lv[l];
        ph.levels[l].n_parts = parts[l];
        for (int n = h.n_int; n < h.n_nodes; ++n) ph.p2m.push_back(NodeItem{l, n});
        for (int n = 0; n < h.n_int; ++n) {
            ph.interior[l].push_back(NodeItem{l, n});
            if (!defer[l][n]) ph.l2l[l].push_back(NodeItem{l, n});
        }
        for (int n = 0; n < h.n_int; ++n) {
            if (m2l_lds[l]) continue;  // ordered below
            for (int c = 0; c < parts[l]; ++c)
                for (int p = 0; p < 8; ++p) ph.m2l.push_back(M2LItem{l, n, p, c});
        }
        // leaf targets next to interior nodes: staged in LDS (below the root)
        for (int n = h.n_int; n < h.n_rec; ++n) {
            if (l >= 1 && t->leaf_lds) {
                ph.m2l_leaf.push_back(M2LItem{l, n, 0, 0});
                continue;
            }
            for (int p = 0; p < 8; ++p) ph.m2l.push_back(M2LItem{l, n, p, 0});
        }
        for (int n = h.n_int; n < h.n_nodes; ++n) {
            const int pn = l > 0 ? h.parent[n] : -1;
            const int32_t f = h.flags[n] | (pn >= 0 && defer[l - 1][pn] ? kLeafDefer : 0);
            ph.leaf.push_back(LeafItem{l, n, 0, f});
        }
    }
    // LDS-staged items: the kernel gives XCD k the k-th of 8 equal slices of
    // the list; fill each slice with its share of every level's items (a
    // contiguous run in node order), levels with larger items first
    {
        std::vector<std::vector<M2LItem>> lv_items;
        for (int l = 0; l < nl; ++l) {
            if (!m2l_lds[l] || L.lv[l].n_int == 0) continue;
            std::vector<M2LItem> v;
            for (int n = 0; n < L.lv[l].n_int; ++n)
                for (int c = 0; c < parts[l]; ++c) v.push_back(M2LItem{l, n, 0, c});
            lv_items.push_back(std::move(v));
        }
        std::stable_sort(lv_items.begin(), lv_items.end(), [&](const auto &a, const auto &b) {
            return parts[a[0].ld] < parts[b[0].ld];  // fewer groups = more classes per item
        });
        size_t total = 0;
        for (const auto &v : lv_items) total += v.size();
        const size_t per = (total + 7) / 8;
        std::vector<std::vector<M2LItem>> slice(8);
        for (const auto &v : lv_items) {
            const size_t n = v.size();
            size_t pos = 0;
            for (int k = 0; k < 8 && pos < n; ++k) {
                const size_t want = n / 8 + ((size_t)k < n % 8 ? 1 : 0);
                const size_t room = per - slice[k].size();
                const size_t take = std::min({want, room, n - pos});
                slice[k].insert(slice[k].end(), v.begin() + pos, v.begin() + pos + take);
                pos += take;
            }
            for (int k = 0; k < 8 && pos < n; ++k) {  // what did not fit its share
                const size_t take = std::min(per - slice[k].size(), n - pos);
                slice[k].insert(slice[k].end(), v.begin() + pos, v.begin() + pos + take);
                pos += take;
            }
        }
        for (const auto &sl : slice) ph.m2l_nodes.insert(ph.m2l_nodes.end(), sl.begin(), sl.end());
    }
    ph.tree_leaf_beg = {0, (int32_t)ph.leaf.size()};
    ph.tree_m2l_beg = {0, (int32_t)ph.m2l.size()};
    ph.tree_m2ln_beg = {0, (int32_t)ph.m2l_nodes.size()};
    ph.tree_m2lf_beg = {0, (int32_t)ph.m2l_leaf.size()};
}

}  // namespace octo

namespace {

void check_density_host(const double *rho, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!(rho[i] >= 0.0) || !std::isfinite(rho[i]))
            fail(OCTO_E_INVALID, "density negative or not finite at cell " + std::to_string(i));
}

void validate_opts(const octo_opts *o) {
    if (!o) fail(OCTO_E_INVALID, "opts is NULL");
    if (!(o->theta >= 0.34 && o->theta < 1.0)) fail(OCTO_E_UNSUPPORTED, "theta must lie in [0.34, 1)");
    if (o->precision != OCTO_FP64 && o->precision != OCTO_MIXED) fail(OCTO_E_UNSUPPORTED, "unknown precision");
    if (!std::isfinite(o->G)) fail(OCTO_E_INVALID, "G not finite");
}

void fill_stats(const double *v, int64_t n_leaf_cells, double ms, octo_stats *st) {
    memset(st->phase_ms, 0, sizeof st->phase_ms);
    st->total_mass = v[0];
    for (int k = 0; k < 3; ++k) {
        st->net_force[k] = v[1 + k];
        st->net_torque[k] = v[4 + k];
    }
    st->force_scale = v[7];
    st->torque_scale = v[8];
    st->n_leaf_cells = n_leaf_cells;
    st->m2l_pairs = (int64_t)v[9];
    st->direct_pairs = (int64_t)v[10];
    st->m2l_lds_pairs = (int64_t)v[11];
    st->device_ms = ms;
}

}  // namespace

// ------------------------------------------------------------------ ctx

void *octo_ctx::dev_alloc(size_t bytes) {
    if (budget && in_use + bytes > budget)
        fail(OCTO_E_BUDGET, "HBM budget exceeded (" + std::to_string(in_use + bytes) + " > " + std::to_string(budget) + ")");
    void *p = nullptr;
    if (has_alloc) {
        p = alloc.alloc(bytes, alloc.user);
        if (!p) fail(OCTO_E_BUDGET, "allocator returned NULL");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) fail(OCTO_E_BUDGET, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    in_use += bytes;
    return p;
}

void octo_ctx::dev_free(void *p, size_t bytes) {
    if (!p) return;
    if (has_alloc)
        alloc.free(p, alloc.user);
    else
        hipFree(p);
    in_use -= bytes;
}

const StencilDevHolder &octo_ctx::stencil(double theta) {
    uint64_t k;
    memcpy(&k, &theta, 8);
    auto it = stencils.find(k);
    if (it != stencils.end()) return *it->second;
    auto h = std::make_unique<StencilDevHolder>();
    h->host = make_stencil(theta);
    const Stencil &S = h->host;
    std::vector<float> w32(S.leaf_tab.begin(), S.leaf_tab.end());
    std::vector<float> xw32(S.xl_w.begin(), S.xl_w.end());
    size_t b = al(S.m2l.size() * 4) + al(S.leaf.size() * 4) + al(S.leaf_tab.size() * 8) + al(w32.size() * 4) +
               al(S.m2l_src.size() * 4) + al(S.leaf_off.size() * 4) + al(S.leaf_widx.size() * 4) +
               al(S.m2l_touch.size() * 4) + al(S.m2l_src_touch.size() * 4) + al(S.m2l_src_d.size() * 4) +
               al(S.near_stage.size() * 4) +
               al(S.xl_off.size() * 4) + al(S.xl_cls.size() * 4) + al(S.xl_touch.size() * 4) +
               al(S.xl_w.size() * 8) + al(xw32.size() * 4);
    void *mem = nullptr;
    check_hip(hipMalloc(&mem, b), "stencil alloc");
    h->block.ptr = mem;
    h->block.bytes = b;
    char *base = (char *)mem;
    size_t off = 0;
    auto put = [&](const void *src, size_t n) {
        void *dst = base + off;
        if (n) check_hip(hipMemcpy(dst, src, n, hipMemcpyHostToDevice), "stencil upload");
        off += al(n);
        return dst;
    };
    h->dev.m2l = (const int32_t *)put(S.m2l.data(), S.m2l.size() * 4);
    h->dev.m2l_touch = (const int32_t *)put(S.m2l_touch.data(), S.m2l_touch.size() * 4);
    h->dev.leaf = (const int32_t *)put(S.leaf.data(), S.leaf.size() * 4);
    h->dev.leaf_tab = (const double *)put(S.leaf_tab.data(), S.leaf_tab.size() * 8);
    h->dev.leaf_tab32 = (const float *)put(w32.data(), w32.size() * 4);
    h->dev.m2l_src = (const int32_t *)put(S.m2l_src.data(), S.m2l_src.size() * 4);
    h->dev.leaf_off = (const int32_t *)put(S.leaf_off.data(), S.leaf_off.size() * 4);
    h->dev.leaf_widx = (const int32_t *)put(S.leaf_widx.data(), S.leaf_widx.size() * 4);
    h->dev.m2l_src_touch = (const int32_t *)put(S.m2l_src_touch.data(), S.m2l_src_touch.size() * 4);
    h->dev.m2l_src_d = (const int32_t *)put(S.m2l_src_d.data(), S.m2l_src_d.size() * 4);
    h->dev.near_stage = (const int32_t *)put(S.near_stage.data(), S.near_stage.size() * 4);
    h->dev.xl_off = (const int32_t *)put(S.xl_off.data(), S.xl_off.size() * 4);
    h->dev.xl_cls = (const int32_t *)put(S.xl_cls.data(), S.xl_cls.size() * 4);
    h->dev.xl_touch = (const int32_t *)put(S.xl_touch.data(), S.xl_touch.size() * 4);
    h->dev.xl_w = (const double *)put(S.xl_w.data(), S.xl_w.size() * 8);
    h->dev.xl_w32 = (const float *)put(xw32.data(), xw32.size() * 4);
    h->dev.n_xl = (int32_t)S.xl_off.size();
    h->dev.xl_reach = S.xl_reach;
    for (int k = 0; k < 64; ++k) h->dev.m2l_src_any[k] = S.m2l_src_any[k];
    for (int k = 0; k < 73; ++k) h->dev.leaf_oct_beg[k] = S.leaf_oct_beg[k];
    for (int k = 0; k < 73; ++k) h->dev.m2l_src_beg[k] = S.m2l_src_beg[k];
    for (int p = 0; p < 9; ++p) {
        h->dev.m2l_beg[p] = S.m2l_beg[p];
        h->dev.leaf_beg[p] = S.leaf_beg[p];
    }
    h->dev.theta2 = theta * theta;
    auto &ref = *h;
    stencils.emplace(k, std::move(h));
    return ref;
}

extern "C" {

const char *octo_last_error(void) { return g_err.c_str(); }

const char *octo_build_id(void) { return OCTO_BUILD_ID; }

octo_status octo_ctx_create(int device, void *hip_stream, const octo_allocator *alloc, size_t hbm_budget,
                            octo_ctx **out) {
    return guard([&] {
        if (!out) fail(OCTO_E_INVALID, "out is NULL");
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
            fail(OCTO_E_DEVICE, "no HIP device " + std::to_string(device));
        DeviceGuard dg(device);
        scf_fixed_scratch_init(device);  // the allocation-free SCF step's array on this device
        auto *c = new octo_ctx();
        c->device = device;
        c->budget = hbm_budget;
        if (alloc && alloc->alloc && alloc->free) {
            c->has_alloc = true;
            c->alloc = *alloc;
        }
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            check_hip(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "stream create");
            c->own_stream = true;
        }
        check_hip(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking), "stream create");
        check_hip(hipStreamCreateWithFlags(&c->capture_aux, hipStreamNonBlocking), "stream create");
        check_hip(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking), "stream create");
        check_hip(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming), "event");
        check_hip(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming), "event");
        check_hip(hipStreamCreateWithFlags(&c->aux_near, hipStreamNonBlocking), "stream create");
        check_hip(hipStreamCreateWithFlags(&c->capture_near, hipStreamNonBlocking), "stream create");
        check_hip(hipEventCreateWithFlags(&c->fork_near_ev, hipEventDisableTiming), "event");
        check_hip(hipEventCreateWithFlags(&c->join_near_ev, hipEventDisableTiming), "event");
        if (const char *e = getenv("OCTO_GRAPHS")) c->use_graphs = atoi(e) != 0;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
            c->n_cu = ncu;
        check_hip(hipEventCreate(&c->ev0), "event");
        for (int i = 0; i < 9; ++i) check_hip(hipEventCreate(&c->phase_ev[i]), "event");
        check_hip(hipEventCreate(&c->ev1), "event");
        c->h_stats_cap = 12 * 1024;
        check_hip(hipHostMalloc((void **)&c->h_stats, c->h_stats_cap * sizeof(double), hipHostMallocDefault),
                  "pinned stats");
        *out = c;
    });
}

octo_status octo_ctx_destroy(octo_ctx *ctx) {
    return guard([&] {
        if (!ctx) return;
        if (ctx->n_trees > 0) fail(OCTO_E_STATE, "context still owns trees");
        DeviceGuard dg(ctx->device);
        hipStreamSynchronize(ctx->stream);
        ctx->invalidate_batches();
        for (auto &kv : ctx->stencils) hipFree(kv.second->block.ptr);
        hipStreamDestroy(ctx->capture);
        hipStreamDestroy(ctx->capture_aux);
        hipStreamSynchronize(ctx->aux);
        hipStreamDestroy(ctx->aux);
        for (Lane &l : ctx->lanes) {
            for (hipStream_t q : {l.s, l.aux, l.aux_near}) {
                hipStreamSynchronize(q);
                hipStreamDestroy(q);
            }
            for (hipEvent_t e : {l.start, l.fork, l.join, l.fork_near, l.join_near}) hipEventDestroy(e);
        }
        ctx->lanes.clear();
        hipEventDestroy(ctx->fork_ev);
        hipEventDestroy(ctx->join_ev);
        hipStreamSynchronize(ctx->aux_near);
        hipStreamDestroy(ctx->aux_near);
        hipStreamDestroy(ctx->capture_near);
        hipEventDestroy(ctx->fork_near_ev);
        hipEventDestroy(ctx->join_near_ev);
        hipEventDestroy(ctx->ev0);
        for (int i = 0; i < 9; ++i) hipEventDestroy(ctx->phase_ev[i]);
        hipEventDestroy(ctx->ev1);
        layout_device_release(ctx);
        hipHostFree(ctx->h_stats);
        for (auto &b : ctx->pinned_free) {
            if (b.ready) hipEventDestroy(b.ready);
            hipHostFree(b.p);
        }
        if (ctx->own_stream) hipStreamDestroy(ctx->stream);
        delete ctx;
    });
}

octo_status octo_ctx_set_profiling(octo_ctx *ctx, int on) {
    return guard([&] {
        if (!ctx) fail(OCTO_E_INVALID, "ctx is NULL");
        if (on < 0 || on > 2) fail(OCTO_E_INVALID, "profiling mode must be 0, 1 or 2");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        ctx->profiling = on;
    });
}

octo_status octo_ctx_set_batch_shapes(octo_ctx *ctx, int mode) {
    return guard([&] {
        if (!ctx) fail(OCTO_E_INVALID, "ctx is NULL");
        if (mode != 0 && mode != 1) fail(OCTO_E_INVALID, "batch shape mode must be 0 or 1");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        ctx->batch_shapes = mode;
    });
}

octo_status octo_ctx_memory(const octo_ctx *ctx, size_t *bytes_in_use, size_t *budget) {
    return guard([&] {
        if (!ctx) fail(OCTO_E_INVALID, "ctx is NULL");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        if (bytes_in_use) *bytes_in_use = ctx->in_use;
        if (budget) *budget = ctx->budget;
    });
}

// ------------------------------------------------------------------ trees

static octo_status make_tree(octo_ctx *ctx, const octo_leaf *leaves, int64_t n, int grid_level, const double *rho,
                             int rho_on_device, octo_tree **out) {
    return guard([&] {
        if (!ctx || !out || !rho) fail(OCTO_E_INVALID, "NULL argument");
        auto t = std::make_unique<octo_tree>();
        t->ctx = ctx;
        // validation, layout, work shape and the upload image need no device
        // and no context state: they run before the lock
        t->layout = build_layout(leaves, n, grid_level);
        if (!rho_on_device) check_density_host(rho, t->layout.n_leaf_cells);
        TreeBlock B;
        shape_tree(t.get(), B);
        DeviceGuard dg(ctx->device);
        size_t img_bytes = 0;
        void *img = nullptr;
        {
            std::lock_guard<std::recursive_mutex> lk(ctx->mu);
            img = ctx->pinned_get(B.upload, &img_bytes);
        }
        stage_tree(t.get(), B, rho_on_device ? nullptr : rho, (char *)img);
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        try {
            commit_tree(t.get(), B, img, img_bytes, rho_on_device ? rho : nullptr);
        } catch (...) {
            if (!t->data.ptr) ctx->pinned_put(img, img_bytes, nullptr);  // the upload was never enqueued
            throw;
        }
        try {
            build_tree_plan(t.get());
        } catch (...) {
            hipStreamSynchronize(ctx->stream);
            ctx->dev_free(t->data.ptr, t->data.bytes);
            t->data.ptr = nullptr;
            throw;
        }
        tree_release(t.get(), ctx->stream);
        ctx->n_trees++;
        *out = t.release();
    });
}

// A tree from a leaf list and densities in device memory (leaf-list layout),
// laid out on the device under the context lock.  The leaves are read before
// the call returns; the density too when wait_rho, otherwise the caller
// keeps it until the context stream has passed this call's work.
static octo_tree *make_tree_device(octo_ctx *ctx, const octo_leaf *leaves, int64_t n, int levels,
                                   const double *rho, bool wait_rho) {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard dg(ctx->device);
    auto t = std::make_unique<octo_tree>();
    t->ctx = ctx;
    layout_device(ctx, leaves, n, levels, t->layout);
    TreeBlock B;
    try {
        shape_tree(t.get(), B);
        commit_tree(t.get(), B, nullptr, 0, rho, wait_rho);
    } catch (...) {
        layout_device_abort(ctx);
        if (t->data.ptr) {
            hipStreamSynchronize(ctx->stream);
            ctx->dev_free(t->data.ptr, t->data.bytes);
        }
        throw;
    }
    const Layout &L = t->layout;
    LayTables tb{};
    char *base = (char *)t->data.ptr;
    for (int l = 0; l < L.n_levels; ++l) {
        tb.nbr[l] = (int32_t *)(base + B.nbr[l]);
        tb.child[l] = (int32_t *)(base + B.child[l]);
        tb.parent[l] = (int32_t *)(base + B.parent[l]);
        tb.coord[l] = (int32_t *)(base + B.coord[l]);
        tb.out_base[l] = (int64_t *)(base + B.out[l]);
        tb.n_int[l] = L.lv[l].n_int;
    }
    layout_device_tables(ctx, tb);
    try {
        build_tree_plan(t.get());
    } catch (...) {
        hipStreamSynchronize(ctx->stream);
        ctx->dev_free(t->data.ptr, t->data.bytes);
        t->data.ptr = nullptr;
        throw;
    }
    tree_release(t.get(), ctx->stream);
    ctx->n_trees++;
    return t.release();
}

octo_status octo_tree_build_device(octo_ctx *ctx, const octo_leaf *leaves, int64_t n_leaves, const double *rho,
                                   octo_tree **out) {
    return guard([&] {
        if (!ctx || !leaves || !rho || !out) fail(OCTO_E_INVALID, "NULL argument");
        if (n_leaves <= 0) fail(OCTO_E_INVALID, "empty leaf list");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        DeviceGuard dg(ctx->device);
        const int levels = layout_device_levels(ctx, leaves, n_leaves);
        *out = make_tree_device(ctx, leaves, n_leaves, levels, rho, true);
    });
}

octo_status octo_tree_build(octo_ctx *ctx, const octo_leaf *leaves, int64_t n_leaves, const double *rho,
                            int rho_on_device, octo_tree **out) {
    return make_tree(ctx, leaves, n_leaves, -1, rho, rho_on_device, out);
}

octo_status octo_tree_build_uniform(octo_ctx *ctx, int level, const double *rho, int rho_on_device,
                                    octo_tree **out) {
    if (level < 0 || level > 6) {
        g_err = "uniform level must lie in [0, 6]";
        return OCTO_E_INVALID;
    }
    const int m = 1 << level;
    std::vector<octo_leaf> lv;
    lv.reserve((size_t)m * m * m);
    for (int x = 0; x < m; ++x)
        for (int y = 0; y < m; ++y)
            for (int z = 0; z < m; ++z) lv.push_back(octo_leaf{level, x, y, z});
    return make_tree(ctx, lv.data(), (int64_t)lv.size(), level, rho, rho_on_device, out);
}

octo_status octo_tree_build_adaptive(octo_ctx *ctx, octo_density_fn density, octo_boxmax_fn boxmax, void *user,
                                     int max_level, double threshold, octo_tree **out) {
    std::vector<octo_leaf> lv;
    std::vector<double> rho;
    octo_status st = guard([&] {
        if (!ctx || !out || !density || !boxmax) fail(OCTO_E_INVALID, "NULL argument");
        if (!std::isfinite(threshold)) fail(OCTO_E_INVALID, "threshold not finite");
        lv = adaptive_leaves(boxmax, user, max_level, threshold);
        rho.resize(lv.size() * 512);
        std::vector<double> xyz(3 * 512 * 64);
        for (size_t b = 0; b < lv.size(); b += 64) {
            const size_t e = std::min(lv.size(), b + 64);
            size_t k = 0;
            for (size_t i = b; i < e; ++i) {
                const octo_leaf &f = lv[i];
                const double h = 1.0 / (double)(8 << f.level);
                for (int x = 0; x < 8; ++x)
                    for (int y = 0; y < 8; ++y)
                        for (int z = 0; z < 8; ++z) {
                            xyz[3 * k] = (8 * f.ix + x + 0.5) * h - 0.5;
                            xyz[3 * k + 1] = (8 * f.iy + y + 0.5) * h - 0.5;
                            xyz[3 * k + 2] = (8 * f.iz + z + 0.5) * h - 0.5;
                            ++k;
                        }
            }
            density((int64_t)k, xyz.data(), rho.data() + b * 512, user);
        }
    });
    if (st != OCTO_OK) return st;
    return make_tree(ctx, lv.data(), (int64_t)lv.size(), -1, rho.data(), 0, out);
}

octo_status octo_tree_set_density(octo_tree *t, const double *rho, int rho_on_device) {
    return guard([&] {
        if (!t || !rho) fail(OCTO_E_INVALID, "NULL argument");
        if (!rho_on_device) check_density_host(rho, t->layout.n_leaf_cells);
        std::lock_guard<std::recursive_mutex> lk(t->ctx->mu);
        DeviceGuard dg(t->ctx->device);
        tree_acquire(t->ctx, t);
        check_hip(hipMemcpyAsync(t->rho, rho, (size_t)t->layout.n_leaf_cells * 8,
                                 rho_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, t->ctx->stream),
                  "density upload");
        tree_release(t, t->ctx->stream);
        if (!rho_on_device) check_hip(hipStreamSynchronize(t->ctx->stream), "density upload");
    });
}

octo_status octo_tree_get_density(const octo_tree *t, double *rho, int rho_on_device) {
    return guard([&] {
        if (!t || !rho) fail(OCTO_E_INVALID, "NULL argument");
        std::lock_guard<std::recursive_mutex> lk(t->ctx->mu);
        DeviceGuard dg(t->ctx->device);
        tree_acquire(t->ctx, const_cast<octo_tree *>(t));
        check_hip(hipMemcpyAsync(rho, t->rho, (size_t)t->layout.n_leaf_cells * 8,
                                 rho_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, t->ctx->stream),
                  "density copy");
        if (!rho_on_device) check_hip(hipStreamSynchronize(t->ctx->stream), "density copy");
    });
}

octo_status octo_tree_info(const octo_tree *t, int64_t *n_leaf_cells, int32_t *n_levels, size_t *bytes) {
    return guard([&] {
        if (!t) fail(OCTO_E_INVALID, "tree is NULL");
        if (n_leaf_cells) *n_leaf_cells = t->layout.n_leaf_cells;
        if (n_levels) *n_levels = t->layout.n_levels;
        if (bytes) *bytes = t->bytes;
    });
}

octo_status octo_tree_leaves(const octo_tree *t, octo_leaf *out) {
    return guard([&] {
        if (!t || !out) fail(OCTO_E_INVALID, "NULL argument");
        std::copy(t->layout.leaves.begin(), t->layout.leaves.end(), out);
    });
}

octo_status octo_tree_level_tables(const octo_tree *t, int32_t level, int64_t *sizes, const octo_level_tables *out) {
    return guard([&] {
        if (!t || !sizes) fail(OCTO_E_INVALID, "NULL argument");
        const Layout &L = t->layout;
        if (level < 0 || level >= L.n_levels) fail(OCTO_E_INVALID, "level out of range");
        const HostLevel &h = L.lv[level];
        sizes[0] = h.n_nodes;
        sizes[1] = h.n_int;
        sizes[2] = h.n_rec;
        if (!out) return;
        octo_ctx *ctx = t->ctx;
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        DeviceGuard dg(ctx->device);
        check_hip(hipEventSynchronize(t->last_use->ev), "tree tables");
        const LevelDesc &d = t->ph.levels[level];
        auto get = [](void *dst, const void *src, size_t bytes) {
            if (dst && bytes) check_hip(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost), "tree tables");
        };
        const size_t nn = h.n_nodes;
        get(out->nbr, d.nbr, nn * 27 * 4);
        get(out->child, d.child, (size_t)h.n_int * 8 * 4);
        get(out->parent, d.parent, nn * 4);
        get(out->coord, d.coord, nn * 3 * 4);
        get(out->out_base, d.out_base, nn * 8);
        if (out->flags)
            for (size_t i = 0; i < nn; ++i) out->flags[i] = h.flags[i];
        if (out->int_child)
            for (int i = 0; i < h.n_int; ++i) out->int_child[i] = h.int_child[i];
    });
}

octo_status octo_tree_destroy(octo_tree *t) {
    return guard([&] {
        if (!t) return;
        std::lock_guard<std::recursive_mutex> lk(t->ctx->mu);
        DeviceGuard dg(t->ctx->device);
        for (auto &kv : t->ctx->requests)
            if (kv.second.tree == t && !kv.second.done)
                fail(OCTO_E_STATE, "tree has an unfinished request");
        // the tree's own last work, not everything queued on the stream since
        hipEventSynchronize(t->last_use->ev);
        t->last_use.reset();
        if (t->ctx->batch &&
            std::find(t->ctx->batch->sig.begin(), t->ctx->batch->sig.end(), t) != t->ctx->batch->sig.end())
            t->ctx->invalidate_batches();
        drop_graphs(t->graphs);
        t->ctx->dev_free(t->data.ptr, t->data.bytes);
        t->ctx->dev_free(t->plan_block.ptr, t->plan_block.bytes);
        t->ctx->n_trees--;
        delete t;
    });
}

// ------------------------------------------------------------------ solve

octo_status octo_solve(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, double *phi, double *g,
                       int out_on_device, octo_stats *stats) {
    return guard([&] {
        if (!ctx || !tree) fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        validate_opts(opts);
        if (!phi || !g) fail(OCTO_E_INVALID, "NULL output");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);

        DeviceGuard dg(ctx->device);
        tree_acquire(ctx, tree);
        const int64_t n = tree->layout.n_leaf_cells;
        std::vector<TreeDesc> want = tree->plan.trees_host;
        want[0].phi = out_on_device ? phi : tree->stage;
        want[0].g = out_on_device ? g : tree->stage + n;
        want[0].G = opts->G;
        want[0].amc = opts->amc ? 1 : 0;
        if (stats) check_hip(hipEventRecord(ctx->ev0, ctx->stream), "event");
        // timing-only profiling runs the kernels as a solve without statistics
        const bool count = stats != nullptr && ctx->profiling != 2;
        run_plan(ctx, tree->plan, tree->graphs, want, opts, count);
        tree_release(tree, ctx->stream);
        if (stats) {
            check_hip(hipEventRecord(ctx->ev1, ctx->stream), "event");
            check_hip(hipMemcpyAsync(ctx->h_stats, tree->plan.d_out, 12 * sizeof(double), hipMemcpyDeviceToHost,
                                     ctx->stream),
                      "stats copy");
        }
        if (!out_on_device) {
            check_hip(hipMemcpyAsync(phi, tree->stage, n * 8, hipMemcpyDeviceToHost, ctx->stream), "phi copy");
            check_hip(hipMemcpyAsync(g, tree->stage + n, 3 * n * 8, hipMemcpyDeviceToHost, ctx->stream), "g copy");
        }
        if (stats || !out_on_device) check_hip(hipStreamSynchronize(ctx->stream), "solve");
        if (stats) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
            fill_stats(ctx->h_stats, n, ms, stats);
            if (!count) {
                const double dms = stats->device_ms;
                memset(stats, 0, sizeof *stats);
                stats->n_leaf_cells = n;
                stats->device_ms = dms;
            }
            if (ctx->profiling) phase_times(ctx, stats->phase_ms);
        }
    });
}

octo_status octo_solve_device_stats(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, double *phi, double *g,
                                    double *stats_dev) {
    return guard([&] {
        if (!ctx || !tree) fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        validate_opts(opts);
        if (!phi || !g || !stats_dev) fail(OCTO_E_INVALID, "NULL output");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);

        DeviceGuard dg(ctx->device);
        tree_acquire(ctx, tree);
        std::vector<TreeDesc> want = tree->plan.trees_host;
        want[0].phi = phi;
        want[0].g = g;
        want[0].G = opts->G;
        want[0].amc = opts->amc ? 1 : 0;
        run_plan(ctx, tree->plan, tree->graphs, want, opts, false, false, true);
        check_hip(hipMemcpyAsync(stats_dev, tree->plan.d_out, 9 * sizeof(double), hipMemcpyDeviceToDevice,
                                 ctx->stream),
                  "stats copy");
        tree_release(tree, ctx->stream);
    });
}

octo_status octo_solve_dphidt(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, const double *drho_dt,
                              double *dphi_dt) {
    return guard([&] {
        if (!ctx || !tree) fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        validate_opts(opts);
        if (!drho_dt || !dphi_dt) fail(OCTO_E_INVALID, "NULL source or output");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);

        DeviceGuard dg(ctx->device);
        tree_acquire(ctx, tree);
        std::vector<TreeDesc> want = tree->plan.trees_host;
        want[0].phi = dphi_dt;
        want[0].g = nullptr;
        want[0].src = drho_dt;
        want[0].G = opts->G;
        want[0].amc = 0;
        run_plan(ctx, tree->plan, tree->graphs, want, opts, false, true);
        tree_release(tree, ctx->stream);
    });
}

octo_status octo_gravity_sources(octo_ctx *ctx, octo_tree *tree, const double *omega, const double *rho,
                                 const double *s, const double *phi, const double *g, const double *drho_dt,
                                 const double *dphi_dt, double *src_s, double *src_e) {
    return guard([&] {
        if (!ctx || !tree || !omega || !rho || !s || !phi || !g || !src_s || !src_e)
            fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(omega[k])) fail(OCTO_E_INVALID, "omega not finite");
        DeviceGuard dg(ctx->device);
        tree_acquire(ctx, tree);
        launch_sources(tree->plan, omega, rho, s, phi, g, drho_dt, dphi_dt, src_s, src_e, ctx->stream);
        tree_release(tree, ctx->stream);
    });
}

octo_status octo_energy_update(octo_ctx *ctx, octo_tree *tree, const double *rho, const double *phi_before,
                               const double *phi_after, double *E) {
    return guard([&] {
        if (!ctx || !tree || !rho || !phi_before || !phi_after || !E) fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);

        DeviceGuard dg(ctx->device);
        launch_energy_update(tree->layout.n_leaf_cells, rho, phi_before, phi_after, E, ctx->stream);
    });
}

namespace {

void validate_scf(const octo_scf_params *p) {
    if (!p) fail(OCTO_E_INVALID, "SCF parameters are NULL");
    const double pos[] = {p->M1, p->M2, p->n, p->a0, p->G};
    for (double v : pos)
        if (!std::isfinite(v) || v <= 0.0) fail(OCTO_E_INVALID, "SCF masses, n, a0 and G must be finite and positive");
    if (!std::isfinite(p->f) || !std::isfinite(p->K0)) fail(OCTO_E_INVALID, "SCF f and K0 must be finite");
    if (!std::isfinite(p->rho_floor) || p->rho_floor < 0.0) fail(OCTO_E_INVALID, "SCF floor density must be >= 0");
}

// the split x in half-cell units of the grid of `level` (a cell centre or face)
int64_t scf_split(double x, int level) {
    const double n2 = 2.0 * (double)(8 << level);
    const double u = (x + 0.5) * n2;
    if (!std::isfinite(u) || u != std::floor(u) || u < 0.0 || u > n2)
        fail(OCTO_E_INVALID, "x_L1 must be a cell centre or a cell face of the grid");
    return (int64_t)u;
}

// the level of a tree built on the uniform grid layout, else -1
int uniform_level(const octo_tree *t) {
    const Layout &L = t->layout;
    const int level = L.n_levels - 1;
    if (level < 0 || level > 6) return -1;
    const int64_t n = (int64_t)8 << level;
    if (L.n_leaf_cells != n * n * n || L.sx != n * n || L.sy != n || L.sz != 1) return -1;
    return level;
}

}  // namespace

octo_status octo_scf_step(octo_ctx *ctx, int level, const octo_scf_params *p, double K, double x_L1,
                          const double *rho, const double *phi, double *rho_out, octo_scf_state *state) {
    return guard([&] {
        if (!ctx || !rho || !phi || !rho_out || !state) fail(OCTO_E_INVALID, "NULL argument");
        if (level < 0 || level > 6) fail(OCTO_E_INVALID, "level must lie in [0, 6]");
        validate_scf(p);
        if (!std::isfinite(K)) fail(OCTO_E_INVALID, "K not finite");
        const int64_t s2 = scf_split(x_L1, level);
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        DeviceGuard dg(ctx->device);
        scf_step(ctx, level, *p, K, s2, rho, phi, rho_out, state);
    });
}

octo_status octo_scf_step_noalloc(octo_ctx *ctx, int level, const octo_scf_params *p, double K, double x_L1,
                                  const double *rho, const double *phi, double *rho_out, octo_scf_state *state) {
    return guard([&] {
        if (!ctx || !rho || !phi || !rho_out || !state) fail(OCTO_E_INVALID, "NULL argument");
        if (level < 0 || level > 6)
            fail(OCTO_E_INVALID, "level must lie in [0, 6] (the fixed scratch covers grids up to 512^3)");
        validate_scf(p);
        if (!std::isfinite(K)) fail(OCTO_E_INVALID, "K not finite");
        const int64_t s2 = scf_split(x_L1, level);
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        DeviceGuard dg(ctx->device);
        scf_step_noalloc(ctx, level, *p, K, s2, rho, phi, rho_out, state);
    });
}

octo_status octo_scf_run(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, const octo_scf_params *p,
                         int32_t iterations, double *rho_out, double *phi_out, octo_scf_state *history) {
    return guard([&] {
        if (!ctx || !tree || !phi_out) fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        validate_opts(opts);
        validate_scf(p);
        if (iterations < 0) fail(OCTO_E_INVALID, "iterations < 0");
        const int level = uniform_level(tree);
        if (level < 0) fail(OCTO_E_INVALID, "the SCF iteration needs a tree from octo_tree_build_uniform");
        const int64_t s2 = scf_split(p->x_L1, level);
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        DeviceGuard dg(ctx->device);
        octo_opts o = *opts;
        o.G = p->G;
        tree_acquire(ctx, tree);
        scf_run(ctx, tree, level, o, *p, s2, iterations, rho_out, phi_out, history);
    });
}

octo_status octo_regrid(octo_ctx *ctx, octo_tree *tree, const octo_regrid_params *p, octo_tree **out,
                        octo_regrid_stats *stats) {
    return guard([&] {
        if (!ctx || !tree || !p || !out) fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        if (p->l_max < 0 || p->l_max > kMaxLevel) fail(OCTO_E_INVALID, "l_max must lie in [0, 9]");
        if (!std::isfinite(p->rho_r) || p->rho_r <= 0.0) fail(OCTO_E_INVALID, "rho_r must be finite and positive");
        RegridOut r;
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        DeviceGuard dg(ctx->device);
        const auto t0 = std::chrono::steady_clock::now();
        tree_acquire(ctx, tree);
        regrid_device(ctx, tree, p->l_max, p->rho_r, r);
        const auto t1 = std::chrono::steady_clock::now();
        octo_tree *t = make_tree_device(ctx, r.leaves, r.n_leaves, r.levels, r.rho, false);
        // the old tree's last use: the regrid read it
        tree_release(tree, ctx->stream);
        const auto t2 = std::chrono::steady_clock::now();
        int64_t grids = 0;
        for (const HostLevel &h : t->layout.lv) grids += h.n_nodes;
        *out = t;
        if (stats) {
            stats->refined = r.refined;
            stats->balance_refined = r.balance_refined;
            stats->derefined = r.derefined;
            stats->n_leaves = r.n_leaves;
            stats->n_grids = grids;
            const double ratio = (double)grids / (double)p->n_target;
            stats->rho_r_next = p->n_target > 0 ? p->rho_r * (ratio * ratio) : p->rho_r;
            stats->flag_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
            stats->layout_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
        }
    });
}

// Autotuner: for each level with interior nodes, time the multipole phase
// with each candidate work shape (LDS-staged per node, or per wavefront with
// 1..parts_alloc stencil chunks) and keep the fastest, level by level.
octo_status octo_tree_autotune(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, int32_t *choice) {
    return guard([&] {
        if (!ctx || !tree) fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        validate_opts(opts);
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        DeviceGuard dg(ctx->device);
        tree_acquire(ctx, tree);
        if (ctx->batch &&
            std::find(ctx->batch->sig.begin(), ctx->batch->sig.end(), tree) != ctx->batch->sig.end())
            ctx->invalidate_batches();
        const int prof = ctx->profiling;
        ctx->profiling = 1;
        const int64_t n = tree->layout.n_leaf_cells;
        auto measure = [&]() {
            std::vector<TreeDesc> want = tree->plan.trees_host;
            want[0].phi = tree->stage;
            want[0].g = tree->stage + n;
            want[0].G = opts->G;
            want[0].amc = opts->amc ? 1 : 0;
            double best = 1e30;
            for (int rep = 0; rep < 4; ++rep) {
                run_plan(ctx, tree->plan, tree->graphs, want, opts, false);
                tree_release(tree, ctx->stream);
                check_hip(hipStreamSynchronize(ctx->stream), "autotune");
                float ms = 0.f;
                hipEventElapsedTime(&ms, ctx->phase_ev[3], ctx->phase_ev[4]);
                if (rep > 0) best = std::min(best, (double)ms);  // first run warms up
            }
            return best;
        };
        const int nl = tree->layout.n_levels;
        try {
            for (int l = 0; l < nl; ++l) {
                if (tree->layout.lv[l].n_int == 0) continue;
                std::vector<std::pair<int, int>> cand;  // (lds, parts)
                if (l >= 1)
                    for (int p = 1; p <= std::min(8, tree->parts_alloc[l]); p *= 2) cand.push_back({1, p});
                for (int p = 1; p <= tree->parts_alloc[l]; p *= 2) cand.push_back({0, p});
                double best = 1e30;
                std::pair<int, int> pick{tree->m2l_lds[l], tree->parts[l]};
                for (auto c : cand) {
                    tree->m2l_lds[l] = c.first;
                    tree->parts[l] = c.second;
                    build_tree_plan(tree);
                    const double ms = measure();
                    if (ms < best) {
                        best = ms;
                        pick = c;
                    }
                }
                tree->m2l_lds[l] = pick.first;
                tree->parts[l] = pick.second;
            }
            build_tree_plan(tree);
        } catch (...) {
            ctx->profiling = prof;
            throw;
        }
        ctx->profiling = prof;
        if (choice)
            for (int l = 0; l < nl; ++l)
                choice[l] = tree->layout.lv[l].n_int == 0 ? -1 : (tree->m2l_lds[l] ? -tree->parts[l] - 1 : tree->parts[l]);
    });
}

}  // extern "C"
