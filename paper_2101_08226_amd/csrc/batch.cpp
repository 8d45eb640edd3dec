// Batched solves (many trees per launch), graph replay and asynchronous
// requests merged into launch waves (continuous batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>

#include "runtime.h"

using namespace octo;

namespace octo {

namespace {
__global__ void k_set_tree(TreeDesc *dst, TreeDesc v) { *dst = v; }

uint64_t theta_bits(double t) {
    uint64_t k;
    memcpy(&k, &t, 8);
    return k;
}
}  // namespace

void drop_graphs(std::map<std::pair<uint64_t, int>, hipGraphExec_t> &graphs) {
    for (auto &kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
}

void run_plan(octo_ctx *ctx, Plan &plan, std::map<std::pair<uint64_t, int>, hipGraphExec_t> &graphs,
              const std::vector<TreeDesc> &want, const octo_opts *o, bool count, bool source, bool reduce) {
    // tree descriptors (outputs, G, correction switch) live in device memory
    // and are refreshed only when they change
    for (int i = 0; i < plan.n_trees; ++i) {
        TreeDesc &cur = plan.trees_host[i];
        if (memcmp(&cur, &want[i], sizeof(TreeDesc)) != 0) {
            cur = want[i];
            hipLaunchKernelGGL(k_set_tree, dim3(1), dim3(1), 0, ctx->stream, plan.d_trees + i, cur);
        }
    }
    const StencilDevHolder &st = ctx->stencil(o->theta);
    LaunchOpts lo;
    lo.precision = o->precision;
    lo.count = count;
    lo.reduce = reduce;
    lo.source = source;
    lo.amc = o->amc != 0;
    lo.fork = ctx->fork_ev;
    lo.join = ctx->join_ev;
    lo.fork_near = ctx->fork_near_ev;
    lo.join_near = ctx->join_near_ev;
    if (ctx->profiling) {
        // phases are timed one after the other: no concurrent streams
        lo.phase_events = ctx->phase_ev;
        launch_solve(plan, st.dev, lo, ctx->stream);
        return;
    }
    if (!ctx->use_graphs) {
        lo.aux = ctx->aux;
        lo.aux_near = ctx->aux_near;
        launch_solve(plan, st.dev, lo, ctx->stream);
        return;
    }
    lo.aux = ctx->capture_aux;
    lo.aux_near = ctx->capture_near;
    const auto key = std::make_pair(theta_bits(o->theta), (int)o->precision * 16 + (o->amc ? 8 : 0) +
                                                               (reduce ? 4 : 0) + (source ? 2 : 0) + (count ? 1 : 0));
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        hipGraph_t g = nullptr;
        check_hip(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal), "graph capture");
        try {
            launch_solve(plan, st.dev, lo, ctx->capture);
        } catch (...) {
            hipStreamEndCapture(ctx->capture, &g);
            if (g) hipGraphDestroy(g);
            throw;
        }
        check_hip(hipStreamEndCapture(ctx->capture, &g), "graph capture");
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        check_hip(e, "graph instantiate");
        it = graphs.emplace(key, ex).first;
    }
    check_hip(hipGraphLaunch(it->second, ctx->stream), "graph launch");
}

// A tree's work lists inside a batch: every level below the root with
// interior nodes takes the LDS-staged multipole kernel with g source-class
// groups (at most the tree's partial slots); the root's per-wavefront work
// is split into root_parts stencil chunks (at most its partial slots).
static const PlanHost &batch_lists(octo_tree *t, int g, int root_parts) {
    const int key = g * 64 + root_parts;
    auto it = t->ph_batch.find(key);
    if (it != t->ph_batch.end()) return it->second;
    const int nl = t->layout.n_levels;
    std::vector<int> parts = t->parts, lds = t->m2l_lds;
    if (t->layout.lv[0].n_int > 0 && !lds[0]) parts[0] = std::min(root_parts, t->parts_alloc[0]);
    for (int l = 1; l < nl; ++l)
        if (t->layout.lv[l].n_int > 0) {
            lds[l] = 1;
            parts[l] = std::min(g, t->parts_alloc[l]);
        }
    PlanHost ph;
    ph.levels = t->ph.levels;
    ph.trees = t->ph.trees;
    plan_items(t, parts, lds, ph);
    return t->ph_batch.emplace(key, std::move(ph)).first->second;
}

// Concatenate the plans of several trees: each tree's own plan, or with
// `fitted` (and several trees), shapes fitted to the batch.  Several trees
// share each launch, so a level's few nodes no longer leave the device idle:
// all levels below the root go to the LDS-staged kernel, with the
// source-class group count (the same for every tree) that the launch model
// prices lowest over the whole batch, and the roots' per-wavefront work is
// split only as far as it takes to give every CU four wavefronts (a single
// tree splits its root 32 ways, each part writing a partial slot of every
// root cell that the downward pass then reads).
static std::unique_ptr<BatchPlan> make_batch(octo_tree *const *trees, int n, const std::vector<TreeDesc> &descs,
                                             bool fitted) {
    auto bp = std::make_unique<BatchPlan>();
    bp->sig.assign(trees, trees + n);
    PlanHost &ph = bp->ph;
    bool shared = fitted && n > 1;
    for (int i = 0; i < n; ++i) shared = shared && trees[i]->leaf_lds;
    int g_best = 0;
    if (shared) {
        double best = 1e300;
        for (int g = 1; g <= 4; g *= 2) {
            std::vector<int64_t> n_int;
            std::vector<int> gs;
            for (int i = 0; i < n; ++i)
                for (int l = 1; l < trees[i]->layout.n_levels; ++l)
                    if (trees[i]->layout.lv[l].n_int > 0) {
                        n_int.push_back(trees[i]->layout.lv[l].n_int);
                        gs.push_back(std::min(g, trees[i]->parts_alloc[l]));
                    }
            if (n_int.empty()) break;
            const double c = lds_launch_cost(n_int, gs, trees[0]->ctx->n_cu);
            if (c < best - 1e-9) {
                best = c;
                g_best = g;
            }
        }
    }
    int roots = 0;
    for (int i = 0; i < n; ++i) roots += trees[i]->layout.lv[0].n_int > 0 ? 1 : 0;
    const int n_cu = std::max(8, trees[0]->ctx->n_cu);
    const int root_parts = std::max(1, std::min(32, (4 * n_cu + 8 * std::max(1, roots) - 1) / (8 * std::max(1, roots))));
    std::vector<const PlanHost *> src(n);
    for (int i = 0; i < n; ++i) src[i] = g_best ? &batch_lists(trees[i], g_best, root_parts) : &trees[i]->ph;
    size_t max_lv = 0;
    for (int i = 0; i < n; ++i) max_lv = std::max(max_lv, src[i]->interior.size());
    ph.interior.resize(max_lv);
    ph.l2l.resize(max_lv);
    for (int i = 0; i < n; ++i) {
        const PlanHost &t = *src[i];
        const int base = (int)ph.levels.size();
        for (LevelDesc d : t.levels) {
            if (d.parent_ld >= 0) d.parent_ld += base;
            if (d.child_ld >= 0) d.child_ld += base;
            d.tree = i;
            ph.levels.push_back(d);
        }
        ph.trees.push_back(descs[i]);
        ph.tree_leaf_beg.push_back((int32_t)ph.leaf.size());
        ph.tree_m2l_beg.push_back((int32_t)ph.m2l.size());
        ph.tree_m2ln_beg.push_back((int32_t)ph.m2l_nodes.size());
        ph.tree_m2lf_beg.push_back((int32_t)ph.m2l_leaf.size());
        for (M2LItem q : t.m2l_nodes) {
            q.ld += base;
            ph.m2l_nodes.push_back(q);
        }
        for (M2LItem q : t.m2l_leaf) {
            q.ld += base;
            ph.m2l_leaf.push_back(q);
        }
        for (M2LItem m : t.m2l) {
            m.ld += base;
            ph.m2l.push_back(m);
        }
        for (LeafItem f : t.leaf) {
            f.ld += base;
            ph.leaf.push_back(f);
        }
        for (NodeItem q : t.p2m) {
            q.ld += base;
            ph.p2m.push_back(q);
        }
        for (size_t l = 0; l < t.interior.size(); ++l) {
            for (NodeItem q : t.interior[l]) {
                q.ld += base;
                ph.interior[l].push_back(q);
            }
            for (NodeItem q : t.l2l[l]) {
                q.ld += base;
                ph.l2l[l].push_back(q);
            }
        }
    }
    ph.tree_leaf_beg.push_back((int32_t)ph.leaf.size());
    ph.tree_m2l_beg.push_back((int32_t)ph.m2l.size());
    ph.tree_m2ln_beg.push_back((int32_t)ph.m2l_nodes.size());
    ph.tree_m2lf_beg.push_back((int32_t)ph.m2l_leaf.size());
    return bp;
}

static TreeDesc desc_for(octo_tree *t, double *phi, double *g, const octo_opts *o) {
    TreeDesc d = t->ph.trees[0];
    d.phi = phi;
    d.g = g;
    d.G = o->G;
    d.amc = o->amc ? 1 : 0;
    return d;
}

static void validate(const octo_opts *o) {
    if (!o) fail(OCTO_E_INVALID, "opts is NULL");
    if (!(o->theta >= 0.34 && o->theta < 1.0)) fail(OCTO_E_UNSUPPORTED, "theta must lie in [0.34, 1)");
    if (o->precision != OCTO_FP64 && o->precision != OCTO_MIXED) fail(OCTO_E_UNSUPPORTED, "unknown precision");
    if (!std::isfinite(o->G)) fail(OCTO_E_INVALID, "G not finite");
}

static void fill(const double *v, int64_t n_leaf_cells, double ms, octo_stats *st) {
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

}  // namespace octo

void octo_ctx::release_batch(BatchPlan *bp) {
    if (!bp) return;
    drop_graphs(bp->graphs);
    if (bp->mem) dev_free(bp->mem, bp->bytes);
    if (bp->staging) pinned_put(bp->staging, bp->staging_bytes);
    bp->mem = nullptr;
    bp->staging = nullptr;
}

void *octo_ctx::pinned_get(size_t bytes, size_t *got) {
    size_t best = pinned_free.size();
    for (size_t i = 0; i < pinned_free.size(); ++i) {
        Pinned &b = pinned_free[i];
        if (b.bytes < bytes || (best < pinned_free.size() && b.bytes >= pinned_free[best].bytes)) continue;
        if (b.ready) {
            if (hipEventQuery(b.ready) != hipSuccess) continue;  // its upload is still queued
            hipEventDestroy(b.ready);
            b.ready = nullptr;
        }
        best = i;
    }
    if (best < pinned_free.size()) {
        Pinned b = pinned_free[best];
        pinned_free.erase(pinned_free.begin() + best);
        *got = b.bytes;
        return b.p;
    }
    const size_t n = std::max(bytes, (size_t)1 << 20);
    void *p = nullptr;
    check_hip(hipHostMalloc(&p, n, hipHostMallocDefault), "pinned staging");
    *got = n;
    return p;
}

void octo_ctx::pinned_put(void *p, size_t bytes, hipEvent_t ready) { pinned_free.push_back(Pinned{p, bytes, ready}); }

void octo_ctx::invalidate_batches() {
    if (batch) {
        hipStreamSynchronize(stream);
        release_batch(batch.get());
        batch.reset();
    }
}

namespace octo {
void set_error(const std::string &m);
}

template <typename F>
static octo_status guard_b(F &&f) {
    try {
        f();
        return OCTO_OK;
    } catch (const Error &e) {
        octo::set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        octo::set_error(e.what());
        return OCTO_E_INVALID;
    }
}

// ------------------------------------------------------------------ waves

static void retire_waves(octo_ctx *ctx) {
    for (auto it = ctx->waves.begin(); it != ctx->waves.end();) {
        Wave &w = it->second;
        if (hipEventQuery(w.done) != hipSuccess) {
            ++it;
            continue;
        }
        const int nt = (int)w.tickets.size();
        w.bp->stats.resize((size_t)nt * 12);
        check_hip(hipMemcpy(w.bp->stats.data(), w.bp->plan.d_out, (size_t)nt * 12 * sizeof(double),
                            hipMemcpyDeviceToHost),
                  "wave stats");
        for (int i = 0; i < nt; ++i) {
            auto r = ctx->requests.find(w.tickets[i]);
            if (r != ctx->requests.end()) r->second.done = true;
        }
        hipEventDestroy(w.done);
        // keep the stats with the requests, release the device block
        for (int i = 0; i < nt; ++i) {
            auto r = ctx->requests.find(w.tickets[i]);
            if (r != ctx->requests.end()) {
                r->second.wave = -1;
                memcpy(r->second.stats, w.bp->stats.data() + 12 * i, 12 * sizeof(double));
            }
        }
        ctx->release_batch(w.bp.get());
        it = ctx->waves.erase(it);
    }
}

static void make_lanes(octo_ctx *ctx) {
    if (!ctx->lanes.empty()) return;
    ctx->lanes.resize(ctx->max_inflight_waves);
    for (Lane &l : ctx->lanes) {
        for (hipStream_t *q : {&l.s, &l.aux, &l.aux_near})
            check_hip(hipStreamCreateWithFlags(q, hipStreamNonBlocking), "lane stream");
        for (hipEvent_t *e : {&l.start, &l.fork, &l.join, &l.fork_near, &l.join_near})
            check_hip(hipEventCreateWithFlags(e, hipEventDisableTiming), "lane event");
    }
}

// Launch waves while fewer than max_inflight_waves are on the device: each
// wave takes the pending requests with the first request's (theta,
// precision, correction switch), at most one request per tree, as many as
// its work plan fits the context's HBM budget (halving the wave until it
// does); a request whose plan does not fit even alone, with no wave in
// flight to free memory, fails on its own ticket (OCTO_E_BUDGET).  Each wave
// runs on a lane of its own: after the work already on the context stream
// and the last use of each of its trees (a tree may still be in the other
// lane's wave).
static void pump(octo_ctx *ctx) {
    retire_waves(ctx);
    while (!ctx->pending.empty() && (int)ctx->waves.size() < ctx->max_inflight_waves) {
        const Request &first = ctx->requests.at(ctx->pending.front());
        const double theta = first.opts.theta;
        const int prec = first.opts.precision;
        const bool amc = first.opts.amc != 0;
        std::vector<octo_ticket> take;
        std::set<octo_tree *> used;
        for (octo_ticket t : ctx->pending) {
            Request &r = ctx->requests.at(t);
            if (r.opts.theta == theta && r.opts.precision == prec && (r.opts.amc != 0) == amc &&
                !used.count(r.tree)) {
                used.insert(r.tree);
                take.push_back(t);
            }
        }
        std::unique_ptr<BatchPlan> bp;
        std::vector<octo_tree *> trees;
        std::vector<char> img;
        void *mem = nullptr;
        size_t bytes = 0;
        while (!mem) {
            trees.clear();
            std::vector<TreeDesc> descs;
            for (octo_ticket t : take) {
                Request &r = ctx->requests.at(t);
                trees.push_back(r.tree);
                descs.push_back(desc_for(r.tree, r.phi, r.g, &r.opts));
            }
            bp = make_batch(trees.data(), (int)trees.size(), descs, false);
            bytes = plan_layout(bp->ph, nullptr, bp->plan, img);
            try {
                mem = ctx->dev_alloc(bytes);
            } catch (const Error &e) {
                if (e.code != OCTO_E_BUDGET) throw;
                if (!ctx->waves.empty()) return;  // retry when a wave retires
                if (take.size() > 1) {
                    take.resize(take.size() / 2);
                    continue;
                }
                Request &r = ctx->requests.at(take[0]);
                r.status = OCTO_E_BUDGET;
                r.err = "the request's work plan (" + std::to_string(bytes) +
                        " bytes) does not fit the HBM budget with nothing else in flight";
                r.done = true;
                ctx->pending.erase(std::find(ctx->pending.begin(), ctx->pending.end(), take[0]));
                break;
            }
        }
        if (!mem) continue;  // the head request failed; try the next
        std::set<octo_ticket> taken(take.begin(), take.end());
        std::deque<octo_ticket> rest;
        for (octo_ticket t : ctx->pending)
            if (!taken.count(t)) rest.push_back(t);
        make_lanes(ctx);
        int lane = 0;
        for (; lane < (int)ctx->lanes.size(); ++lane) {
            bool busy = false;
            for (auto &kv : ctx->waves) busy = busy || kv.second.lane == lane;
            if (!busy) break;
        }
        Lane &L = ctx->lanes.at(lane);
        bp->mem = mem;
        bp->bytes = bytes;
        plan_layout(bp->ph, mem, bp->plan, img);
        const StencilDevHolder &st = ctx->stencil(theta);
        check_hip(hipEventRecord(L.start, ctx->stream), "event");
        check_hip(hipStreamWaitEvent(L.s, L.start, 0), "lane wait");
        {
            // one wait per distinct event (the trees of a batch share one)
            std::vector<UseMark *> seen;
            for (octo_tree *t : trees)
                if (t->last_stream != L.s && std::find(seen.begin(), seen.end(), t->last_use.get()) == seen.end()) {
                    seen.push_back(t->last_use.get());
                    check_hip(hipStreamWaitEvent(L.s, t->last_use->ev, 0), "lane wait");
                }
        }
        bp->staging = ctx->pinned_get(img.size(), &bp->staging_bytes);
        memcpy(bp->staging, img.data(), img.size());
        check_hip(hipMemcpyAsync(mem, bp->staging, img.size(), hipMemcpyHostToDevice, L.s), "wave upload");
        LaunchOpts lo;
        lo.precision = prec;
        lo.amc = amc;
        lo.aux = L.aux;
        lo.fork = L.fork;
        lo.join = L.join;
        lo.aux_near = L.aux_near;
        lo.fork_near = L.fork_near;
        lo.join_near = L.join_near;
        launch_solve(bp->plan, st.dev, lo, L.s);
        Wave w;
        w.lane = lane;
        check_hip(hipEventCreateWithFlags(&w.done, hipEventDisableTiming), "event");
        check_hip(hipEventRecord(w.done, L.s), "event");
        trees_release(trees.data(), (int)trees.size(), L.s);
        w.tickets = take;
        w.bp = std::move(bp);
        const int id = ctx->next_wave++;
        for (size_t i = 0; i < take.size(); ++i) {
            Request &r = ctx->requests.at(take[i]);
            r.wave = id;
            r.index = (int)i;
        }
        ctx->waves.emplace(id, std::move(w));
        ctx->pending.swap(rest);
    }
}

// The trees of a batch that pass the per-tree checks are solved together;
// the others get their own status and are left alone.
static octo_status solve_batch_impl(octo_ctx *ctx, octo_tree *const *trees_in, int32_t n_in, const octo_opts *opts,
                                    double *const *phi_in, double *const *g_in, int out_on_device,
                                    octo_stats *stats_in, octo_status *status) {
    std::vector<int> idx;  // positions of the trees that are solved
    std::string first_msg;
    octo_status first = OCTO_OK;
    bool decided = false;  // per-tree statuses written
    const octo_status s = guard_b([&] {
        if (!ctx || !trees_in || n_in <= 0 || !phi_in || !g_in) fail(OCTO_E_INVALID, "bad batch arguments");
        validate(opts);
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);

        std::set<octo_tree *> seen;
        for (int i = 0; i < n_in; ++i) {
            octo_status si = OCTO_OK;
            const char *why = nullptr;
            if (!trees_in[i] || !phi_in[i] || !g_in[i]) {
                si = OCTO_E_INVALID;
                why = "NULL tree or output in batch";
            } else if (trees_in[i]->ctx != ctx) {
                si = OCTO_E_STATE;
                why = "tree belongs to another context";
            } else if (!seen.insert(trees_in[i]).second) {
                si = OCTO_E_INVALID;
                why = "a tree appears twice in one batch";
            }
            if (status) status[i] = si;
            if (si == OCTO_OK) {
                idx.push_back(i);
            } else if (first == OCTO_OK) {
                first = si;
                first_msg = std::string(why) + " (batch entry " + std::to_string(i) + ")";
            }
        }
        decided = true;
        if (idx.empty()) fail(first, first_msg);
        const int n = (int)idx.size();
        std::vector<octo_tree *> trees_v(n);
        std::vector<double *> phi_v(n), g_v(n);
        std::vector<octo_stats> st_v(stats_in ? n : 0);
        for (int k = 0; k < n; ++k) {
            trees_v[k] = trees_in[idx[k]];
            phi_v[k] = phi_in[idx[k]];
            g_v[k] = g_in[idx[k]];
        }
        octo_tree *const *trees = trees_v.data();
        double *const *phi = phi_v.data();
        double *const *g = g_v.data();
        octo_stats *stats = stats_in ? st_v.data() : nullptr;
        hipSetDevice(ctx->device);
        std::vector<octo_tree *> sig(trees, trees + n);
        if (!ctx->batch || ctx->batch->sig != sig || ctx->batch->fitted != (ctx->batch_shapes == 1)) {
            ctx->invalidate_batches();
            std::vector<TreeDesc> descs;
            for (int i = 0; i < n; ++i) descs.push_back(trees[i]->ph.trees[0]);
            auto bp = make_batch(trees, n, descs, ctx->batch_shapes == 1);
            bp->fitted = ctx->batch_shapes == 1;
            const size_t bytes = plan_bytes(bp->ph);
            bp->mem = ctx->dev_alloc(bytes);
            bp->bytes = bytes;
            plan_upload(bp->ph, bp->mem, bp->plan, ctx->stream);
            ctx->batch = std::move(bp);
        }
        BatchPlan &bp = *ctx->batch;
        {
            // one wait per distinct event (the trees of a batch share one)
            std::vector<UseMark *> seen;
            for (int i = 0; i < n; ++i)
                if (std::find(seen.begin(), seen.end(), trees[i]->last_use.get()) == seen.end()) {
                    seen.push_back(trees[i]->last_use.get());
                    tree_acquire(ctx, trees[i]);
                }
        }
        std::vector<TreeDesc> want;
        for (int i = 0; i < n; ++i) {
            octo_tree *t = trees[i];
            const int64_t m = t->layout.n_leaf_cells;
            want.push_back(desc_for(t, out_on_device ? phi[i] : t->stage, out_on_device ? g[i] : t->stage + m, opts));
        }
        if (stats) check_hip(hipEventRecord(ctx->ev0, ctx->stream), "event");
        const bool count = stats != nullptr && ctx->profiling != 2;  // timing-only profiling: no counts
        run_plan(ctx, bp.plan, bp.graphs, want, opts, count);
        trees_release(trees, n, ctx->stream);
        if (stats) {
            check_hip(hipEventRecord(ctx->ev1, ctx->stream), "event");
            if ((size_t)n * 12 > ctx->h_stats_cap) fail(OCTO_E_INVALID, "batch too large for statistics");
            check_hip(hipMemcpyAsync(ctx->h_stats, bp.plan.d_out, (size_t)n * 12 * sizeof(double),
                                     hipMemcpyDeviceToHost, ctx->stream),
                      "stats copy");
        }
        if (!out_on_device)
            for (int i = 0; i < n; ++i) {
                octo_tree *t = trees[i];
                const int64_t m = t->layout.n_leaf_cells;
                check_hip(hipMemcpyAsync(phi[i], t->stage, m * 8, hipMemcpyDeviceToHost, ctx->stream), "phi copy");
                check_hip(hipMemcpyAsync(g[i], t->stage + m, 3 * m * 8, hipMemcpyDeviceToHost, ctx->stream),
                          "g copy");
            }
        if (stats || !out_on_device) check_hip(hipStreamSynchronize(ctx->stream), "batch");
        if (stats) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
            for (int i = 0; i < n; ++i) {
                fill(ctx->h_stats + 12 * i, trees[i]->layout.n_leaf_cells, ms, &stats[i]);
                if (!count) {
                    memset(&stats[i], 0, sizeof stats[i]);
                    stats[i].n_leaf_cells = trees[i]->layout.n_leaf_cells;
                    stats[i].device_ms = ms;
                }
                if (ctx->profiling) phase_times(ctx, stats[i].phase_ms);  // the whole batch's phases
            }
            for (int k = 0; k < n; ++k) stats_in[idx[k]] = stats[k];
        }
    });
    if (s != OCTO_OK) {
        // a failure of the whole call (arguments, options, device) is every
        // tree's that was to be solved; trees refused on their own keep
        // their status
        if (status && n_in > 0) {
            if (!decided)
                for (int i = 0; i < n_in; ++i) status[i] = s;
            else
                for (int k : idx) status[k] = s;
        }
        return s;
    }
    if (first != OCTO_OK) octo::set_error(first_msg);
    return first;
}

extern "C" {

octo_status octo_solve_batch(octo_ctx *ctx, octo_tree *const *trees, int32_t n, const octo_opts *opts,
                             double *const *phi, double *const *g, int out_on_device, octo_stats *stats,
                             octo_status *status) {
    return solve_batch_impl(ctx, trees, n, opts, phi, g, out_on_device, stats, status);
}

octo_status octo_submit(octo_ctx *ctx, octo_tree *tree, const octo_opts *opts, double *phi_dev, double *g_dev,
                        octo_ticket *ticket) {
    return guard_b([&] {
        if (!ctx || !tree || !phi_dev || !g_dev || !ticket) fail(OCTO_E_INVALID, "NULL argument");
        if (tree->ctx != ctx) fail(OCTO_E_STATE, "tree belongs to another context");
        validate(opts);
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);

        hipSetDevice(ctx->device);
        Request r{};
        r.ticket = ctx->next_ticket++;
        r.tree = tree;
        r.opts = *opts;
        r.phi = phi_dev;
        r.g = g_dev;
        ctx->requests.emplace(r.ticket, r);
        ctx->pending.push_back(r.ticket);
        try {
            pump(ctx);
        } catch (...) {
            ctx->pending.erase(std::remove(ctx->pending.begin(), ctx->pending.end(), r.ticket), ctx->pending.end());
            ctx->requests.erase(r.ticket);
            throw;
        }
        *ticket = r.ticket;
    });
}

octo_status octo_poll(octo_ctx *ctx, octo_ticket ticket, int *done) {
    return guard_b([&] {
        if (!ctx || !done) fail(OCTO_E_INVALID, "NULL argument");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        auto it = ctx->requests.find(ticket);
        if (it == ctx->requests.end()) fail(OCTO_E_INVALID, "unknown ticket");
        hipSetDevice(ctx->device);
        pump(ctx);
        const Request &r = ctx->requests.at(ticket);
        *done = r.done ? 1 : 0;
        if (!*done) fail(OCTO_E_PENDING, "pending");
        if (r.status != OCTO_OK) fail(r.status, r.err);
    });
}

octo_status octo_wait(octo_ctx *ctx, octo_ticket ticket, octo_stats *stats) {
    return guard_b([&] {
        if (!ctx) fail(OCTO_E_INVALID, "NULL argument");
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        auto it = ctx->requests.find(ticket);
        if (it == ctx->requests.end()) fail(OCTO_E_INVALID, "unknown ticket");
        hipSetDevice(ctx->device);
        while (!ctx->requests.at(ticket).done) {
            pump(ctx);
            Request &r = ctx->requests.at(ticket);
            if (r.done) break;
            if (r.wave >= 0) {
                check_hip(hipEventSynchronize(ctx->waves.at(r.wave).done), "wait");
            } else if (ctx->waves.empty() && !ctx->pending.empty()) {
                pump(ctx);  // nothing in flight: the pending wave launches now
            } else if (!ctx->waves.empty()) {
                check_hip(hipEventSynchronize(ctx->waves.begin()->second.done), "wait");
            }
        }
        Request &r = ctx->requests.at(ticket);
        if (r.status != OCTO_OK) {
            const octo_status code = r.status;
            const std::string msg = r.err;
            ctx->requests.erase(ticket);
            fail(code, msg);
        }
        if (stats) fill(r.stats, r.tree->layout.n_leaf_cells, 0.0, stats);
        ctx->requests.erase(ticket);
    });
}

}  // extern "C"
