// One regrid of a tree by the density criterion of Sec. 2.7 ("Refinement
// Criteria") on the device: flags, 2:1 balance, the new leaf list and the
// densities moved onto it.  The leaf list and the densities stay on the
// device, where the new tree is laid out (csrc/layout.hip).
//
// Criterion: a cell of level l is flagged when rho > 8^(l + 1 - l_max) rho_r
// (the largest level L with rho > 8^(L - l_max) rho_r exceeds l).  A leaf
// below l_max with a flagged cell is refined; an interior node whose children
// are all leaves is de-refined when none of its cells (means of the child
// cells) and none of its children's cells is flagged.  Balance over the 26
// neighbours: a refined leaf refines the coarser leaves next to it, to a fixed
// point; a de-refinement is dropped when a child is refined or when a child of
// a same-level neighbour touching the node is interior or refined.  New
// children take the density of the parent cell containing them; a de-refined
// node's cell is the mean of its 8 child cells, summed in child-cell order.
//
// Per-node marks: bit 0 refined by the criterion, bit 1 refined for balance,
// bit 2 de-refinement candidate, bit 3 de-refinement dropped.
#include <algorithm>
#include <vector>

#include "runtime.h"

namespace octo {
namespace {

constexpr int kRgT = 256;

struct RgConst {
    int n_levels, l_max, n_total;
    int32_t nodeoff[kMaxLevel + 2];  // first global node id of each level, + total
    double thr[kMaxLevel + 1];       // flag threshold per level
    int64_t sx, sy, sz;              // caller-layout strides of the density
};

__device__ inline int level_of(const RgConst &k, int g) {
    int l = 0;
    while (l + 1 < k.n_levels && g >= k.nodeoff[l + 1]) ++l;
    return l;
}

__device__ inline int64_t cell_at(const RgConst &k, int64_t base, int x, int y, int z) {
    return base + x * k.sx + y * k.sy + z * k.sz;
}

// mean of the 8 cells of child `kid` (caller layout base) under parent cell
// (x, y, z), summed in child-cell order
__device__ inline double parent_mean(const RgConst &k, const double *rho, const int64_t *kid_base, int x, int y,
                                     int z) {
    const int64_t b = kid_base[(x >> 2) * 4 + (y >> 2) * 2 + (z >> 2)];
    const int bx = 2 * (x & 3), by = 2 * (y & 3), bz = 2 * (z & 3);
    double s = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c)
            for (int e = 0; e < 2; ++e) s += rho[cell_at(k, b, bx + a, by + c, bz + e)];
    return s / 8.0;
}

__device__ inline double block_max(double v, double *lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double r = lds[0];
    for (int i = 1; i < kRgT / 64; ++i) r = fmax(r, lds[i]);
    __syncthreads();
    return r;
}

// one work-group per node: criterion marks
__global__ __launch_bounds__(kRgT) void k_rg_flags(RgConst k, const LevelDesc *__restrict__ lv,
                                                   const double *__restrict__ rho, int32_t *__restrict__ marks) {
    __shared__ double lds[kRgT / 64];
    __shared__ int64_t kid_base[8];
    const int g = blockIdx.x;
    const int l = level_of(k, g);
    const LevelDesc L = lv[l];
    const int node = g - k.nodeoff[l];
    if (node >= L.n_int) {
        const int64_t b = L.out_base[node];
        double m = -INFINITY;
        for (int c = threadIdx.x; c < kCells; c += kRgT) m = fmax(m, rho[cell_at(k, b, c >> 6, (c >> 3) & 7, c & 7)]);
        m = block_max(m, lds);
        if (threadIdx.x == 0 && l < k.l_max && m > k.thr[l]) marks[g] = 1;
        return;
    }
    const LevelDesc C = lv[l + 1];
    bool all_leaves = true;
    for (int i = 0; i < 8; ++i) all_leaves = all_leaves && L.child[node * 8 + i] >= C.n_int;
    if (!all_leaves) return;
    if (threadIdx.x < 8) kid_base[threadIdx.x] = C.out_base[L.child[node * 8 + threadIdx.x]];
    __syncthreads();
    // children's cells against the next level's threshold, means against this one's
    double kid = -INFINITY, mean = -INFINITY;
    for (int c = threadIdx.x; c < 8 * kCells; c += kRgT) {
        const int i = c >> 9, q = c & 511;
        kid = fmax(kid, rho[cell_at(k, kid_base[i], q >> 6, (q >> 3) & 7, q & 7)]);
    }
    for (int c = threadIdx.x; c < kCells; c += kRgT)
        mean = fmax(mean, parent_mean(k, rho, kid_base, c >> 6, (c >> 3) & 7, c & 7));
    kid = block_max(kid, lds);
    mean = block_max(mean, lds);
    if (threadIdx.x == 0) {
        const bool kid_flag = l + 1 < k.l_max && kid > k.thr[l + 1];
        if (!kid_flag && !(mean > k.thr[l])) marks[g] = 4;
    }
}

__device__ inline int dir_index(int dx, int dy, int dz) { return (dx + 1) * 9 + (dy + 1) * 3 + dz + 1; }

// one pass of the balance cascade: every refined leaf refines the coarser
// leaves covering its missing same-level neighbours
__global__ __launch_bounds__(kRgT) void k_rg_balance(RgConst k, const LevelDesc *__restrict__ lv,
                                                     int32_t *marks) {
    const int g = blockIdx.x * kRgT + threadIdx.x;
    if (g >= k.n_total) return;
    const int l = level_of(k, g);
    const LevelDesc L = lv[l];
    const int node = g - k.nodeoff[l];
    if (node < L.n_int || l == 0) return;
    if (!(__atomic_load_n(&marks[g], __ATOMIC_RELAXED) & 3)) return;
    const int n = 1 << l;
    const int x = L.coord[node * 3], y = L.coord[node * 3 + 1], z = L.coord[node * 3 + 2];
    const LevelDesc P = lv[l - 1];
    const int par = L.parent[node];
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                if (!dx && !dy && !dz) continue;
                const int qx = x + dx, qy = y + dy, qz = z + dz;
                if (qx < 0 || qy < 0 || qz < 0 || qx >= n || qy >= n || qz >= n) continue;
                if (L.nbr[node * 27 + dir_index(dx, dy, dz)] >= 0) continue;
                const int cov = P.nbr[par * 27 + dir_index((qx >> 1) - (x >> 1), (qy >> 1) - (y >> 1),
                                                           (qz >> 1) - (z >> 1))];
                if (cov >= P.n_int) atomicOr(&marks[k.nodeoff[l - 1] + cov], 2);
            }
}

// de-refinements that would break the balance: one wavefront per node, a
// lane per (neighbour, child) pair
__global__ __launch_bounds__(64) void k_rg_cancel(RgConst k, const LevelDesc *__restrict__ lv, int32_t *marks) {
    const int g = blockIdx.x;
    if (!(marks[g] & 4)) return;
    const int l = level_of(k, g);
    const LevelDesc L = lv[l], C = lv[l + 1];
    const int node = g - k.nodeoff[l];
    const int px = L.coord[node * 3], py = L.coord[node * 3 + 1], pz = L.coord[node * 3 + 2];
    bool bad = false;
    if (threadIdx.x < 8) bad = marks[k.nodeoff[l + 1] + L.child[node * 8 + threadIdx.x]] & 3;
    for (int t = threadIdx.x; t < 27 * 8; t += 64) {
        const int d = t >> 3, i = t & 7;
        if (d == 13) continue;
        const int q = L.nbr[node * 27 + d];
        if (q < 0 || q >= L.n_int) continue;
        const int c = L.child[q * 8 + i];
        const int cx = C.coord[c * 3], cy = C.coord[c * 3 + 1], cz = C.coord[c * 3 + 2];
        const bool touch = cx >= 2 * px - 1 && cx <= 2 * px + 2 && cy >= 2 * py - 1 && cy <= 2 * py + 2 &&
                           cz >= 2 * pz - 1 && cz <= 2 * pz + 2;
        if (touch && (c < C.n_int || (marks[k.nodeoff[l + 1] + c] & 3))) bad = true;
    }
    if (__any(bad) && threadIdx.x == 0) marks[g] |= 8;
}

__device__ inline bool derefined(int32_t m) { return (m & 4) && !(m & 8); }

// number of new leaves each node emits
__global__ __launch_bounds__(kRgT) void k_rg_count(RgConst k, const LevelDesc *__restrict__ lv,
                                                   const int32_t *__restrict__ marks, int32_t *__restrict__ cnt) {
    const int g = blockIdx.x * kRgT + threadIdx.x;
    if (g >= k.n_total) return;
    const int l = level_of(k, g);
    const LevelDesc L = lv[l];
    const int node = g - k.nodeoff[l];
    int c;
    if (node < L.n_int) {
        c = derefined(marks[g]) ? 1 : 0;
    } else if (l > 0 && derefined(marks[k.nodeoff[l - 1] + L.parent[node]])) {
        c = 0;
    } else {
        c = (marks[g] & 3) ? 8 : 1;
    }
    cnt[g] = c;
}

// exclusive scan of the counts in one work-group (fixed order); off[n] = total
__global__ __launch_bounds__(1024) void k_rg_scan(const int32_t *__restrict__ cnt, int32_t *__restrict__ off,
                                                  int n) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int b = t * per, e = min(n, b + per);
    int32_t s = 0;
    for (int i = b; i < e; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - s;
    for (int i = b; i < e; ++i) {
        off[i] = run;
        run += cnt[i];
    }
    if (t == 1023) off[n] = part[1023];
}

// one work-group per emitting node: new leaves and their densities (leaf
// layout, cells z fastest)
__global__ __launch_bounds__(kRgT) void k_rg_emit(RgConst k, const LevelDesc *__restrict__ lv,
                                                  const double *__restrict__ rho, const int32_t *__restrict__ marks,
                                                  const int32_t *__restrict__ cnt, const int32_t *__restrict__ off,
                                                  octo_leaf *__restrict__ out_leaf, double *__restrict__ out_rho) {
    __shared__ int64_t kid_base[8];
    const int g = blockIdx.x;
    const int c = cnt[g];
    if (c == 0) return;
    const int l = level_of(k, g);
    const LevelDesc L = lv[l];
    const int node = g - k.nodeoff[l];
    const int o = off[g];
    const int x = L.coord[node * 3], y = L.coord[node * 3 + 1], z = L.coord[node * 3 + 2];
    if (node < L.n_int) {  // de-refined: the node becomes a leaf
        const LevelDesc C = lv[l + 1];
        if (threadIdx.x < 8) kid_base[threadIdx.x] = C.out_base[L.child[node * 8 + threadIdx.x]];
        __syncthreads();
        if (threadIdx.x == 0) out_leaf[o] = octo_leaf{l, x, y, z};
        for (int q = threadIdx.x; q < kCells; q += kRgT)
            out_rho[(int64_t)o * kCells + q] = parent_mean(k, rho, kid_base, q >> 6, (q >> 3) & 7, q & 7);
        return;
    }
    const int64_t b = L.out_base[node];
    if (c == 1) {
        if (threadIdx.x == 0) out_leaf[o] = octo_leaf{l, x, y, z};
        for (int q = threadIdx.x; q < kCells; q += kRgT)
            out_rho[(int64_t)o * kCells + q] = rho[cell_at(k, b, q >> 6, (q >> 3) & 7, q & 7)];
        return;
    }
    // refined: 8 children, child (a, c, e) at a*4 + c*2 + e
    if (threadIdx.x < 8) {
        const int a = threadIdx.x >> 2, cc = (threadIdx.x >> 1) & 1, e = threadIdx.x & 1;
        out_leaf[o + threadIdx.x] = octo_leaf{l + 1, 2 * x + a, 2 * y + cc, 2 * z + e};
    }
    for (int q = threadIdx.x; q < 8 * kCells; q += kRgT) {
        const int i = q >> 9, s = q & 511;
        const int a = i >> 2, cc = (i >> 1) & 1, e = i & 1;
        const int cx = s >> 6, cy = (s >> 3) & 7, cz = s & 7;
        out_rho[(int64_t)(o + i) * kCells + s] =
            rho[cell_at(k, b, 4 * a + (cx >> 1), 4 * cc + (cy >> 1), 4 * e + (cz >> 1))];
    }
}

}  // namespace

void regrid_device(octo_ctx *ctx, octo_tree *t, int l_max, double rho_r, RegridOut &r) {
    const Layout &Ly = t->layout;
    const int nl = Ly.n_levels;
    RgConst k{};
    k.n_levels = nl;
    k.l_max = l_max;
    int total = 0;
    for (int l = 0; l < nl; ++l) {
        k.nodeoff[l] = total;
        total += Ly.lv[l].n_nodes;
    }
    k.nodeoff[nl] = total;
    k.n_total = total;
    for (int l = 0; l <= kMaxLevel; ++l) k.thr[l] = std::ldexp(rho_r, 3 * (l + 1 - l_max));  // exact powers of 8
    k.sx = Ly.sx;
    k.sy = Ly.sy;
    k.sz = Ly.sz;
    hipStream_t q = ctx->stream;
    const LevelDesc *dl = t->plan.d_levels;
    const double *rho = t->rho;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    r.ctx = ctx;

    // marks, counts and offsets first; the outputs once their size is known
    const size_t o_cnt = al((size_t)total * 4), o_off = o_cnt + al((size_t)total * 4);
    r.scratch_bytes = o_off + al((size_t)(total + 1) * 4);
    r.scratch = ctx->dev_alloc(r.scratch_bytes);
    char *base = (char *)r.scratch;
    int32_t *marks = (int32_t *)base, *cnt = (int32_t *)(base + o_cnt), *off = (int32_t *)(base + o_off);
    check_hip(hipMemsetAsync(marks, 0, (size_t)total * 4, q), "regrid marks");
    hipLaunchKernelGGL(k_rg_flags, dim3(total), dim3(kRgT), 0, q, k, dl, rho, marks);
    const int nb = (total + kRgT - 1) / kRgT;
    // each pass carries the cascade at least one level up; nl passes reach the root
    for (int i = 0; i < nl; ++i) hipLaunchKernelGGL(k_rg_balance, dim3(nb), dim3(kRgT), 0, q, k, dl, marks);
    hipLaunchKernelGGL(k_rg_cancel, dim3(total), dim3(64), 0, q, k, dl, marks);
    hipLaunchKernelGGL(k_rg_count, dim3(nb), dim3(kRgT), 0, q, k, dl, marks, cnt);
    hipLaunchKernelGGL(k_rg_scan, dim3(1), dim3(1024), 0, q, cnt, off, total);
    std::vector<int32_t> hm(total);
    int32_t n_new = 0;
    check_hip(hipMemcpyAsync(hm.data(), marks, (size_t)total * 4, hipMemcpyDeviceToHost, q), "marks copy");
    check_hip(hipMemcpyAsync(&n_new, off + total, 4, hipMemcpyDeviceToHost, q), "count copy");
    check_hip(hipStreamSynchronize(q), "regrid");
    for (int g = 0; g < total; ++g) {
        const int32_t m = hm[g];
        if (m & 1)
            r.refined++;
        else if (m & 2)
            r.balance_refined++;
        if ((m & 4) && !(m & 8)) r.derefined++;
    }

    r.out_bytes = al((size_t)n_new * sizeof(octo_leaf)) + al((size_t)n_new * kCells * 8);
    r.out = ctx->dev_alloc(r.out_bytes);
    octo_leaf *out_leaf = (octo_leaf *)r.out;
    r.rho = (double *)((char *)r.out + al((size_t)n_new * sizeof(octo_leaf)));
    hipLaunchKernelGGL(k_rg_emit, dim3(total), dim3(kRgT), 0, q, k, dl, rho, marks, cnt, off, out_leaf, r.rho);
    check_hip(hipGetLastError(), "regrid emit");
    r.leaves = out_leaf;
    r.n_leaves = n_new;
    r.levels = std::min(nl + 1, kMaxLevel + 1);  // a regrid refines by one level at most
}

RegridOut::~RegridOut() {
    if (!ctx) return;
    hipStreamSynchronize(ctx->stream);
    if (scratch) ctx->dev_free(scratch, scratch_bytes);
    if (out) ctx->dev_free(out, out_bytes);
}

}  // namespace octo
