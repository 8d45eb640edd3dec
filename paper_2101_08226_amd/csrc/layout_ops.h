// Per-thread steps of the device tree layout (csrc/layout.hip): a leaf list
// becomes the per-level node tables of the layout described in
// octo_internal.h (nodes numbered interior first, then record leaves, then
// other leaves, each group in Morton order), with the checks of the host
// builder (duplicates, overlaps, gaps, 2:1 nesting).
//
// The cells, work arrays and keys are described with LayK in octo_internal.h.
// The includer defines the atomic operations LAY_CAS32(p, cmp, val),
// LAY_ADD64(p, v) and LAY_MIN64(p, v) (each returns the old value).
#pragma once

#include <cstdint>

#include "octo_internal.h"

namespace octo {

__host__ __device__ inline uint32_t lay_morton(int x, int y, int z) {
    uint32_t m = 0;
    for (int b = 0; b < kMaxLevel; ++b)
        m |= (uint32_t)((x >> b) & 1) << (3 * b + 2) | (uint32_t)((y >> b) & 1) << (3 * b + 1) |
             (uint32_t)((z >> b) & 1) << (3 * b);
    return m;
}

__host__ __device__ inline void lay_unmorton(uint32_t m, int &x, int &y, int &z) {
    x = y = z = 0;
    for (int b = 0; b < kMaxLevel; ++b) {
        x |= (int)((m >> (3 * b + 2)) & 1) << b;
        y |= (int)((m >> (3 * b + 1)) & 1) << b;
        z |= (int)((m >> (3 * b)) & 1) << b;
    }
}

__device__ inline void lay_error(const LayK &k, uint64_t code, int64_t item) {
    LAY_MIN64(&k.ctl[1], (unsigned long long)(code << 32 | (uint64_t)(item & 0xffffffff)));
}

__device__ inline void lay_append(const LayK &k, int l, uint32_t m, int32_t leaf, int64_t item) {
    const unsigned long long s = LAY_ADD64(&k.ctl[0], 1ull);
    if ((int64_t)s >= k.cap) {
        lay_error(k, kLayFull, item);
        return;
    }
    k.node_lm[s] = (uint64_t)l << 32 | m;
    k.node_leaf[s] = leaf;
}

// a leaf's own cell (duplicates fail the exchange)
__device__ inline void lay_mark_leaf(const LayK &k, int64_t i) {
    const octo_leaf f = k.leaf[i];
    if (f.level < 0 || f.level >= k.levels) {
        lay_error(k, kLayLevel, i);
        return;
    }
    const int n = 1 << f.level;
    if (f.ix < 0 || f.iy < 0 || f.iz < 0 || f.ix >= n || f.iy >= n || f.iz >= n) {
        lay_error(k, kLayIndex, i);
        return;
    }
    const uint32_t m = lay_morton(f.ix, f.iy, f.iz);
    if (LAY_CAS32(&k.cell[k.goff[f.level] + m], 0, kMarkLeaf) != 0) {
        lay_error(k, kLayDup, i);
        return;
    }
    lay_append(k, f.level, m, (int32_t)i, i);
}

// a leaf's ancestors, up to the first one already present (its marker walks
// on); an ancestor marked as a leaf is an overlap
__device__ inline void lay_mark_ancestors(const LayK &k, int64_t i) {
    const octo_leaf f = k.leaf[i];
    if (f.level < 0 || f.level >= k.levels) return;
    const int n = 1 << f.level;
    if (f.ix < 0 || f.iy < 0 || f.iz < 0 || f.ix >= n || f.iy >= n || f.iz >= n) return;
    int x = f.ix, y = f.iy, z = f.iz;
    for (int l = f.level - 1; l >= 0; --l) {
        x >>= 1;
        y >>= 1;
        z >>= 1;
        const uint32_t m = lay_morton(x, y, z);
        const int32_t old = LAY_CAS32(&k.cell[k.goff[l] + m], 0, kMarkInt);
        if (old == 0) {
            lay_append(k, l, m, -1, i);
            continue;
        }
        if (old == kMarkLeaf) lay_error(k, kLayInside, i);
        return;
    }
}

__device__ inline int64_t lay_count(const LayK &k) {
    const int64_t c = (int64_t)k.ctl[0];
    return c < k.cap ? c : k.cap;
}

// class, flags and sort key of appended node s (s < cap: padding past the count)
__device__ inline void lay_classify(const LayK &k, int64_t s) {
    k.val[s] = (int32_t)s;
    if (s >= lay_count(k)) {
        k.key[s] = kKeyPad;
        return;
    }
    const uint64_t lm = k.node_lm[s];
    const int l = (int)(lm >> 32);
    const uint32_t m = (uint32_t)lm;
    int x, y, z;
    lay_unmorton(m, x, y, z);
    const int n = 1 << l;
    const int32_t *g = k.cell + k.goff[l];
    int cls;
    if (k.node_leaf[s] < 0) {
        // interior: all 8 children present (levels below it exist)
        const int32_t *gc = k.cell + k.goff[l + 1] + ((int64_t)m << 3);
        int ic = 0;
        bool gap = false;
        for (int c = 0; c < 8; ++c) {
            const int32_t v = gc[c];
            gap |= v == 0;
            ic |= v == kMarkInt;
        }
        if (gap) lay_error(k, kLayGap, (int64_t)l << 27 | m);  // the node, as level << 27 | Morton index
        k.info[s] = ic;
        cls = 0;
    } else {
        bool rec = false, nest = false;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    const int qx = x + dx, qy = y + dy, qz = z + dz;
                    if (qx < 0 || qy < 0 || qz < 0 || qx >= n || qy >= n || qz >= n) continue;
                    const uint32_t mq = lay_morton(qx, qy, qz);
                    if (g[mq] != kMarkInt) continue;
                    rec = true;
                    // the neighbour's children on the sides towards this leaf are leaves
                    const int32_t *gc = k.cell + k.goff[l + 1] + ((int64_t)mq << 3);
                    for (int c = 0; c < 8; ++c) {
                        const int cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
                        if ((dx > 0 && cx) || (dx < 0 && !cx) || (dy > 0 && cy) || (dy < 0 && !cy) ||
                            (dz > 0 && cz) || (dz < 0 && !cz))
                            continue;
                        nest |= gc[c] == kMarkInt;
                    }
                }
        if (nest) lay_error(k, kLayNest, k.node_leaf[s]);
        // a leaf neighbour of the parent (cross-level partners one level up)
        bool x2 = false;
        if (l > 0) {
            const int px = x >> 1, py = y >> 1, pz = z >> 1, pn = n >> 1;
            const int32_t *gp = k.cell + k.goff[l - 1];
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        const int qx = px + dx, qy = py + dy, qz = pz + dz;
                        if (qx < 0 || qy < 0 || qz < 0 || qx >= pn || qy >= pn || qz >= pn) continue;
                        x2 |= gp[lay_morton(qx, qy, qz)] == kMarkLeaf;
                    }
        }
        k.info[s] = (rec ? kLeafX1 | kLeafLacc : 0) | (x2 ? kLeafX2 : 0);
        cls = rec ? 1 : 2;
    }
    k.key[s] = (uint64_t)l << 29 | (uint64_t)cls << 27 | m;
}

// first sorted position of each (level, class)
__device__ inline void lay_bounds(const LayK &k, int64_t i) {
    if (i >= lay_count(k)) return;
    const uint64_t a = k.skey[i] >> 27;
    if (i == 0 || (k.skey[i - 1] >> 27) != a) {
        const int l = (int)(a >> 2), c = (int)(a & 3);
        k.ctl[2 + 3 * l + c] = (unsigned long long)i;
    }
}

__device__ inline int64_t lay_level_start(const LayK &k, int l) {
    unsigned long long s = k.ctl[2 + 3 * l];
    for (int c = 1; c < 3; ++c) s = k.ctl[2 + 3 * l + c] < s ? k.ctl[2 + 3 * l + c] : s;
    return (int64_t)s;
}

// node index within its level into the node's cell
__device__ inline void lay_index(const LayK &k, int64_t i) {
    if (i >= lay_count(k)) return;
    const int32_t s = k.sval[i];
    const uint64_t lm = k.node_lm[s];
    const int l = (int)(lm >> 32);
    k.cell[k.goff[l] + (uint32_t)lm] = (int32_t)(i - lay_level_start(k, l)) + kIdxBase;
    k.host[2 * i] = k.info[s];
}

// parent index (for the host's work lists)
__device__ inline void lay_parent(const LayK &k, int64_t i) {
    if (i >= lay_count(k)) return;
    const uint64_t lm = k.node_lm[k.sval[i]];
    const int l = (int)(lm >> 32);
    k.host[2 * i + 1] = l > 0 ? k.cell[k.goff[l - 1] + ((uint32_t)lm >> 3)] - kIdxBase : -1;
}

// the tables of the node at sorted position i
__device__ inline void lay_tables(const LayK &k, const LayTables &t, int64_t i) {
    if (i >= lay_count(k)) return;
    const int32_t s = k.sval[i];
    const uint64_t lm = k.node_lm[s];
    const int l = (int)(lm >> 32);
    const uint32_t m = (uint32_t)lm;
    const int64_t idx = i - lay_level_start(k, l);
    int x, y, z;
    lay_unmorton(m, x, y, z);
    const int n = 1 << l;
    const int32_t *g = k.cell + k.goff[l];
    int32_t *nb = t.nbr[l] + 27 * idx;
    for (int o = 0; o < 27; ++o) {
        const int qx = x + o / 9 - 1, qy = y + (o / 3) % 3 - 1, qz = z + o % 3 - 1;
        int32_t v = -1;
        // the root has no neighbour entries, itself included
        if (l > 0 && qx >= 0 && qy >= 0 && qz >= 0 && qx < n && qy < n && qz < n) {
            const int32_t c = g[lay_morton(qx, qy, qz)];
            v = c ? c - kIdxBase : -1;
        }
        nb[o] = v;
    }
    if (idx < t.n_int[l]) {
        const int32_t *gc = k.cell + k.goff[l + 1] + ((int64_t)m << 3);
        for (int c = 0; c < 8; ++c) t.child[l][8 * idx + c] = gc[c] - kIdxBase;
    }
    t.parent[l][idx] = l > 0 ? k.cell[k.goff[l - 1] + (m >> 3)] - kIdxBase : -1;
    t.coord[l][3 * idx] = x;
    t.coord[l][3 * idx + 1] = y;
    t.coord[l][3 * idx + 2] = z;
    const int32_t leaf = k.node_leaf[s];
    t.out_base[l][idx] = leaf >= 0 ? (int64_t)leaf * kCells : -1;
}

// clear the cell of appended node s
__device__ inline void lay_clear(const LayK &k, int64_t s) {
    if (s >= lay_count(k)) return;
    const uint64_t lm = k.node_lm[s];
    k.cell[k.goff[(int)(lm >> 32)] + (uint32_t)lm] = 0;
}

}  // namespace octo
