// Device tree layout: a leaf list in device memory (the output of a regrid)
// becomes a laid-out tree without the host walking its nodes.  The passes
// run on the context stream:
//   mark leaves, mark ancestors  -- the node set in dense per-level cells
//   classify                     -- interior / record leaf / other leaf, the
//                                   leaf flags, the checks, a sort key
//   radix sort by (level, class, Morton index)
//   bounds, index, parent        -- node numbers written into the cells
// then one download (per-level counts, per-node flags and parents, the leaf
// list: what the host's work lists need) and, once the tree's block is
// allocated, the tables pass and the clearing of the cells.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <string>
#include <vector>

#include "runtime.h"

#define LAY_CAS32(p, c, v) atomicCAS((p), (c), (v))
#define LAY_ADD64(p, v) atomicAdd((p), (v))
#define LAY_MIN64(p, v) atomicMin((p), (v))
#include "layout_ops.h"

namespace octo {
namespace {

constexpr int kLayT = 256;

__global__ __launch_bounds__(64) void k_lay_init(unsigned long long *ctl) {
    for (int i = threadIdx.x; i < kCtlWords; i += 64) ctl[i] = i == 0 ? 0ull : ~0ull;
}

// the deepest level of a leaf list (clamped to [-1, kMaxLevel + 1])
__global__ __launch_bounds__(kLayT) void k_lay_deepest(const octo_leaf *leaf, int64_t n, int *out) {
    const int64_t i = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (i < n) atomicMax(out, std::min(std::max(leaf[i].level, -1), kMaxLevel + 1));
}

__global__ __launch_bounds__(64) void k_lay_set(int *p, int v) {
    if (threadIdx.x == 0) *p = v;
}

__global__ __launch_bounds__(kLayT) void k_lay_leaf(LayK k) {
    const int64_t i = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (i < k.n_leaf) lay_mark_leaf(k, i);
}

__global__ __launch_bounds__(kLayT) void k_lay_anc(LayK k) {
    const int64_t i = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (i < k.n_leaf) lay_mark_ancestors(k, i);
}

__global__ __launch_bounds__(kLayT) void k_lay_class(LayK k) {
    const int64_t s = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (s < k.cap) lay_classify(k, s);
}

__global__ __launch_bounds__(kLayT) void k_lay_bounds(LayK k) {
    const int64_t i = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (i < k.cap) lay_bounds(k, i);
}

__global__ __launch_bounds__(kLayT) void k_lay_index(LayK k) {
    const int64_t i = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (i < k.cap) lay_index(k, i);
}

__global__ __launch_bounds__(kLayT) void k_lay_parent(LayK k) {
    const int64_t i = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (i < k.cap) lay_parent(k, i);
}

__global__ __launch_bounds__(kLayT) void k_lay_tables(LayK k, LayTables t) {
    const int64_t i = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (i < k.cap) lay_tables(k, t, i);
}

__global__ __launch_bounds__(kLayT) void k_lay_clear(LayK k) {
    const int64_t s = (int64_t)blockIdx.x * kLayT + threadIdx.x;
    if (s < k.cap) lay_clear(k, s);
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t cells_below(int levels) {
    int64_t c = 0;
    for (int l = 0; l < levels; ++l) c += (int64_t)1 << (3 * l);
    return c;
}

// the context's cells (levels [0, levels)) and work arrays (cap nodes)
LayK lay_buffers(octo_ctx *ctx, const octo_leaf *leaf, int64_t n, int levels) {
    LayBuf &b = ctx->lay;
    hipStream_t s = ctx->stream;
    const int64_t cap = n + (n + 6) / 7 + 16;  // a complete octree of n leaves has (n - 1) / 7 interior nodes
    if (levels > b.levels) {
        check_hip(hipStreamSynchronize(s), "layout cells");
        ctx->dev_free(b.cell, b.cell_bytes);
        b.cell = nullptr;
        b.levels = 0;
        const size_t bytes = (size_t)cells_below(levels) * 4;
        b.cell = ctx->dev_alloc(bytes);
        b.cell_bytes = bytes;
        b.levels = levels;
        // cleared once; every use clears the cells it set
        check_hip(hipMemsetAsync(b.cell, 0, bytes, s), "layout cells");
    }
    if (cap > b.cap) {
        size_t sort_bytes = 0;
        check_hip(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const uint64_t *)nullptr,
                                                      (uint64_t *)nullptr, (const int32_t *)nullptr,
                                                      (int32_t *)nullptr, (int)cap, 0, kKeyBits, s),
                  "layout sort size");
        const size_t c = (size_t)cap;
        size_t bytes = al(kCtlWords * 8);
        for (size_t per : {8, 4, 8, 4, 8, 4, 4, 8}) bytes += al(per * c);
        bytes += al(sort_bytes);
        check_hip(hipStreamSynchronize(s), "layout work");
        ctx->dev_free(b.work, b.work_bytes);
        b.work = nullptr;
        b.cap = 0;
        b.work = ctx->dev_alloc(bytes);
        b.work_bytes = bytes;
        b.sort_bytes = sort_bytes;
        b.cap = cap;
    }
    LayK k{};
    k.leaf = leaf;
    k.n_leaf = n;
    k.cell = (int32_t *)b.cell;
    for (int l = 0; l <= kMaxLevel + 1; ++l) k.goff[l] = cells_below(std::min(l, b.levels));
    k.levels = b.levels;
    k.cap = cap;
    char *p = (char *)b.work;
    k.ctl = (unsigned long long *)p;
    p += al(kCtlWords * 8);
    const size_t c = (size_t)b.cap;
    k.node_lm = (uint64_t *)p;
    p += al(8 * c);
    k.node_leaf = (int32_t *)p;
    p += al(4 * c);
    k.key = (uint64_t *)p;
    p += al(8 * c);
    k.val = (int32_t *)p;
    p += al(4 * c);
    k.skey = (const uint64_t *)p;
    p += al(8 * c);
    k.sval = (const int32_t *)p;
    p += al(4 * c);
    k.info = (int32_t *)p;
    p += al(4 * c);
    k.host = (int32_t *)p;
    return k;
}

void *sort_temp(const octo_ctx *ctx) {
    const LayBuf &b = ctx->lay;
    return (char *)b.work + b.work_bytes - al(b.sort_bytes);
}

dim3 blocks(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, (n + kLayT - 1) / kLayT)); }

[[noreturn]] void lay_fail(uint64_t e) {
    const uint64_t code = e >> 32;
    const int64_t item = (int64_t)(e & 0xffffffff);
    switch (code) {
        case kLayLevel: fail(OCTO_E_INVALID, "leaf " + std::to_string(item) + ": level out of range");
        case kLayIndex: fail(OCTO_E_INVALID, "leaf " + std::to_string(item) + ": index out of range");
        case kLayDup: fail(OCTO_E_INVALID, "leaf " + std::to_string(item) + ": duplicate");
        case kLayInside: fail(OCTO_E_INVALID, "leaf " + std::to_string(item) + " lies inside another leaf");
        case kLayGap: {
            int x, y, z;
            lay_unmorton((uint32_t)(item & ((1 << 27) - 1)), x, y, z);
            fail(OCTO_E_INVALID, "the leaves leave a gap below node (" + std::to_string(item >> 27) + "," +
                                     std::to_string(x) + "," + std::to_string(y) + "," + std::to_string(z) + ")");
        }
        case kLayNest: fail(OCTO_E_INVALID, "leaves are not properly nested (2:1 balance)");
        default: fail(OCTO_E_INVALID, "leaf list does not form a tree (node capacity exceeded)");
    }
}

}  // namespace

void layout_device(octo_ctx *ctx, const octo_leaf *leaf, int64_t n, int levels, Layout &L) {
    if (n <= 0) fail(OCTO_E_INVALID, "empty leaf list");
    if (levels < 1 || levels > kMaxLevel + 1) fail(OCTO_E_INVALID, "level bound out of range");
    hipStream_t s = ctx->stream;
    const LayK k = lay_buffers(ctx, leaf, n, levels);
    LayBuf &b = ctx->lay;
    hipLaunchKernelGGL(k_lay_init, dim3(1), dim3(64), 0, s, k.ctl);
    hipLaunchKernelGGL(k_lay_leaf, blocks(n), dim3(kLayT), 0, s, k);
    hipLaunchKernelGGL(k_lay_anc, blocks(n), dim3(kLayT), 0, s, k);
    hipLaunchKernelGGL(k_lay_class, blocks(k.cap), dim3(kLayT), 0, s, k);
    size_t sort_bytes = b.sort_bytes;
    check_hip(hipcub::DeviceRadixSort::SortPairs(sort_temp(ctx), sort_bytes, k.key, (uint64_t *)k.skey, k.val,
                                                  (int32_t *)k.sval, (int)k.cap, 0, kKeyBits, s),
              "layout sort");
    hipLaunchKernelGGL(k_lay_bounds, blocks(k.cap), dim3(kLayT), 0, s, k);
    hipLaunchKernelGGL(k_lay_index, blocks(k.cap), dim3(kLayT), 0, s, k);
    hipLaunchKernelGGL(k_lay_parent, blocks(k.cap), dim3(kLayT), 0, s, k);
    check_hip(hipGetLastError(), "layout launch");
    b.pending = k;
    unsigned long long ctl[kCtlWords];
    std::vector<int32_t> host((size_t)2 * k.cap);
    L = Layout{};
    L.leaves.resize(n);
    check_hip(hipMemcpyAsync(ctl, k.ctl, sizeof ctl, hipMemcpyDeviceToHost, s), "layout counts");
    check_hip(hipMemcpyAsync(host.data(), k.host, host.size() * 4, hipMemcpyDeviceToHost, s), "layout nodes");
    check_hip(hipMemcpyAsync(L.leaves.data(), leaf, (size_t)n * sizeof(octo_leaf), hipMemcpyDeviceToHost, s),
              "layout leaves");
    check_hip(hipStreamSynchronize(s), "layout");
    if (ctl[1] != ~0ull) {
        // leave the cells clear for the next use
        if ((ctl[1] >> 32) == kLayFull)
            check_hip(hipMemsetAsync(b.cell, 0, b.cell_bytes, s), "layout cells");
        else
            layout_device_abort(ctx);
        check_hip(hipStreamSynchronize(s), "layout");
        lay_fail(ctl[1]);
    }
    const int64_t count = (int64_t)ctl[0];
    // per level: first sorted position of each class (none: past every node)
    const int64_t none = INT64_MAX;
    auto at = [&](int l, int c) { return ctl[2 + 3 * l + c] == ~0ull ? none : (int64_t)ctl[2 + 3 * l + c]; };
    auto start = [&](int l) { return std::min({at(l, 0), at(l, 1), at(l, 2)}); };
    int nl = 0;
    while (nl < k.levels && start(nl) != none) ++nl;
    L.n_levels = nl;
    L.n_leaf_cells = n * kCells;
    L.lv.resize(nl);
    int64_t beg = 0;
    for (int l = 0; l < nl && beg >= 0; ++l) {
        if (start(l) != beg) {
            beg = -1;
            break;
        }
        const int64_t end = l + 1 < nl ? start(l + 1) : count;
        const int64_t c1 = std::min({at(l, 1), at(l, 2), end}), c2 = std::min(at(l, 2), end);
        HostLevel &h = L.lv[l];
        h.n_nodes = (int)(end - beg);
        h.n_int = (int)(c1 - beg);
        h.n_rec = (int)(c2 - beg);
        h.flags.assign(h.n_nodes, 0);
        h.parent.resize(h.n_nodes);
        h.int_child.resize(h.n_int);
        for (int64_t i = beg; i < end; ++i) {
            const int j = (int)(i - beg);
            if (j < h.n_int)
                h.int_child[j] = (char)host[2 * i];
            else
                h.flags[j] = host[2 * i];
            h.parent[j] = host[2 * i + 1];
        }
        beg = end;
    }
    if (beg != count) {
        layout_device_abort(ctx);
        check_hip(hipStreamSynchronize(s), "layout");
        fail(OCTO_E_INVALID, "leaf list does not form a tree (levels not contiguous)");
    }
}

int layout_device_levels(octo_ctx *ctx, const octo_leaf *leaf, int64_t n) {
    if (n <= 0) fail(OCTO_E_INVALID, "empty leaf list");
    LayBuf &b = ctx->lay;
    hipStream_t s = ctx->stream;
    if (!b.deepest) b.deepest = (int *)ctx->dev_alloc(256);
    hipLaunchKernelGGL(k_lay_set, dim3(1), dim3(64), 0, s, b.deepest, -1);
    hipLaunchKernelGGL(k_lay_deepest, blocks(n), dim3(kLayT), 0, s, leaf, n, b.deepest);
    check_hip(hipGetLastError(), "layout levels");
    int d = -1;
    check_hip(hipMemcpyAsync(&d, b.deepest, 4, hipMemcpyDeviceToHost, s), "layout levels");
    check_hip(hipStreamSynchronize(s), "layout levels");
    // a leaf deeper than kMaxLevel (or above the root) fails the layout's range check
    return std::min(std::max(d, 0), kMaxLevel) + 1;
}

void layout_device_tables(octo_ctx *ctx, const LayTables &t) {
    LayBuf &b = ctx->lay;
    hipStream_t s = ctx->stream;
    const LayK &k = b.pending;
    hipLaunchKernelGGL(k_lay_tables, blocks(k.cap), dim3(kLayT), 0, s, k, t);
    hipLaunchKernelGGL(k_lay_clear, blocks(k.cap), dim3(kLayT), 0, s, k);
    check_hip(hipGetLastError(), "layout tables");
}

void layout_device_abort(octo_ctx *ctx) {
    LayBuf &b = ctx->lay;
    hipLaunchKernelGGL(k_lay_clear, blocks(b.pending.cap), dim3(kLayT), 0, ctx->stream, b.pending);
}

void layout_device_release(octo_ctx *ctx) {
    LayBuf &b = ctx->lay;
    ctx->dev_free(b.cell, b.cell_bytes);
    ctx->dev_free(b.work, b.work_bytes);
    ctx->dev_free(b.deepest, 256);
    b = LayBuf{};
}

}  // namespace octo
