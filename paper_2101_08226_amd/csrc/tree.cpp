// Host side of the octree: validation and layout of a leaf list, adaptive
// refinement from a density field, interaction stencils and work plans.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <unordered_map>
#include <unordered_set>

#include "runtime.h"

namespace octo {

void fail(octo_status code, const std::string &msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(OCTO_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

inline uint64_t key(int l, int x, int y, int z) {
    return ((uint64_t)l << 60) | ((uint64_t)x << 40) | ((uint64_t)y << 20) | (uint64_t)z;
}

inline uint64_t morton(int x, int y, int z) {
    uint64_t m = 0;
    for (int b = 0; b < 20; ++b) {
        m |= (uint64_t)((x >> b) & 1) << (3 * b + 2);
        m |= (uint64_t)((y >> b) & 1) << (3 * b + 1);
        m |= (uint64_t)((z >> b) & 1) << (3 * b);
    }
    return m;
}

struct Node {
    int l, x, y, z;
    bool leaf;
    int64_t leaf_index;  // caller order, -1 for interior
};

}  // namespace

Layout build_layout(const octo_leaf *leaves, int64_t n, int grid_level) {
    if (n <= 0 || !leaves) fail(OCTO_E_INVALID, "empty leaf list");
    std::vector<Node> nodes;
    nodes.reserve((size_t)n * 8 / 7 + 8);
    std::vector<int> parent;  // global index of each node's parent, -1 at the root
    parent.reserve(nodes.capacity());
    std::unordered_map<uint64_t, int> at;
    at.reserve((size_t)n * 2);
    int deepest = 0;
    for (int64_t k = 0; k < n; ++k) {
        const octo_leaf &f = leaves[k];
        if (f.level < 0 || f.level > kMaxLevel) fail(OCTO_E_INVALID, "leaf " + std::to_string(k) + ": level out of range");
        int m = 1 << f.level;
        if (f.ix < 0 || f.iy < 0 || f.iz < 0 || f.ix >= m || f.iy >= m || f.iz >= m)
            fail(OCTO_E_INVALID, "leaf " + std::to_string(k) + ": index out of range");
        if (!at.emplace(key(f.level, f.ix, f.iy, f.iz), (int)nodes.size()).second)
            fail(OCTO_E_INVALID, "leaf " + std::to_string(k) + ": duplicate");
        nodes.push_back(Node{f.level, f.ix, f.iy, f.iz, true, k});
        parent.push_back(-1);
        deepest = std::max(deepest, f.level);
    }
    // ancestors, and every node's parent
    for (int64_t k = 0; k < n; ++k) {
        int child = (int)k;
        int x = nodes[k].x, y = nodes[k].y, z = nodes[k].z;
        for (int l = nodes[k].l - 1; l >= 0; --l) {
            x >>= 1;
            y >>= 1;
            z >>= 1;
            auto ins = at.emplace(key(l, x, y, z), (int)nodes.size());
            const int p = ins.first->second;
            parent[child] = p;
            if (!ins.second) {
                if (nodes[p].leaf) fail(OCTO_E_INVALID, "leaf " + std::to_string(k) + " lies inside another leaf");
                break;
            }
            nodes.push_back(Node{l, x, y, z, false, -1});
            parent.push_back(-1);
            child = p;
        }
    }
    if (!at.count(key(0, 0, 0, 0))) fail(OCTO_E_INVALID, "no root");
    const int nn = (int)nodes.size();
    // children from the parent links; every interior node needs all 8
    std::vector<int> childg((size_t)nn * 8, -1);
    for (int i = 0; i < nn; ++i) {
        if (parent[i] < 0) continue;
        const Node &a = nodes[i];
        childg[(size_t)parent[i] * 8 + (((a.x & 1) << 2) | ((a.y & 1) << 1) | (a.z & 1))] = i;
    }
    std::vector<std::vector<int>> per(deepest + 1);
    for (int i = 0; i < nn; ++i) per[nodes[i].l].push_back(i);
    for (int i = 0; i < nn; ++i) {
        const Node &p = nodes[i];
        if (p.leaf) continue;
        for (int c = 0; c < 8; ++c)
            if (childg[(size_t)i * 8 + c] < 0)
                fail(OCTO_E_INVALID, "the leaves leave a gap below node (" + std::to_string(p.l) + "," +
                                         std::to_string(p.x) + "," + std::to_string(p.y) + "," + std::to_string(p.z) +
                                         ")");
    }
    // compact copies of the per-node data the passes below walk
    std::vector<uint8_t> isleaf(nn);
    std::vector<int32_t> pos((size_t)nn * 3);
    for (int i = 0; i < nn; ++i) {
        isleaf[i] = nodes[i].leaf;
        pos[3 * (size_t)i] = nodes[i].x;
        pos[3 * (size_t)i + 1] = nodes[i].y;
        pos[3 * (size_t)i + 2] = nodes[i].z;
    }
    // same-level neighbours, level by level from the parents' neighbours: the
    // node at q exists when the node at q/2 exists and is interior.  Per axis,
    // a coordinate of parity b moved by d in {-1, 0, 1} lands in the parent
    // cell offset (b + d) >> 1 (floor) at child parity (b + d) & 1.
    std::vector<int> nbrg((size_t)nn * 27, -1);
    for (int l = 1; l <= deepest; ++l) {
        const int m = 1 << l;
        for (int i : per[l]) {
            const int ax = pos[3 * (size_t)i], ay = pos[3 * (size_t)i + 1], az = pos[3 * (size_t)i + 2];
            const int *pn = &nbrg[(size_t)parent[i] * 27];
            const int p = parent[i];
            int *out = &nbrg[(size_t)i * 27];
            for (int dx = -1; dx <= 1; ++dx) {
                const int qx = ax + dx;
                if (qx < 0 || qx >= m) continue;
                const int px = ((ax & 1) + dx) >> 1, cx = (qx & 1) << 2;
                for (int dy = -1; dy <= 1; ++dy) {
                    const int qy = ay + dy;
                    if (qy < 0 || qy >= m) continue;
                    const int py = ((ay & 1) + dy) >> 1, cy = (qy & 1) << 1;
                    for (int dz = -1; dz <= 1; ++dz) {
                        const int qz = az + dz;
                        if (qz < 0 || qz >= m) continue;
                        const int pz = ((az & 1) + dz) >> 1;
                        const int d = (px + 1) * 9 + (py + 1) * 3 + pz + 1;
                        const int pq = d == 13 ? p : pn[d];
                        if (pq < 0 || isleaf[pq]) continue;
                        out[(dx + 1) * 9 + (dy + 1) * 3 + dz + 1] = childg[(size_t)pq * 8 + (cx | cy | (qz & 1))];
                    }
                }
            }
        }
    }
    // proper nesting: no leaf touches an interior node one level finer
    for (int i = 0; i < nn; ++i) {
        if (!isleaf[i]) continue;
        for (int o = 0; o < 27; ++o) {
            const int b = nbrg[(size_t)i * 27 + o];
            if (b < 0 || isleaf[b]) continue;
            int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
            // children of b on the faces/edges/corner towards a
            for (int c = 0; c < 8; ++c) {
                int cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
                if ((dx > 0 && cx) || (dx < 0 && !cx) || (dy > 0 && cy) || (dy < 0 && !cy) || (dz > 0 && cz) ||
                    (dz < 0 && !cz))
                    continue;
                if (!isleaf[childg[(size_t)b * 8 + c]])
                    fail(OCTO_E_INVALID, "leaves are not properly nested (2:1 balance)");
            }
        }
    }

    Layout L;
    L.n_levels = deepest + 1;
    L.leaves.assign(leaves, leaves + n);
    L.n_leaf_cells = n * 512;
    L.lv.resize(L.n_levels);
    // classification: interior, record leaf (touches an interior node of its level), other leaf
    std::vector<int> cls(nn);
    for (int i = 0; i < nn; ++i) {
        if (!isleaf[i]) {
            cls[i] = 0;
            continue;
        }
        bool rec = false;
        for (int o = 0; o < 27 && !rec; ++o) {
            const int b = nbrg[(size_t)i * 27 + o];
            if (b >= 0 && !isleaf[b]) rec = true;
        }
        cls[i] = rec ? 1 : 2;
    }
    // per level: sort (class, Morton key) pairs, then number the nodes
    std::vector<int> idx(nn);
    std::vector<std::pair<uint64_t, int>> ord;
    for (int l = 0; l < L.n_levels; ++l) {
        auto &v = per[l];
        ord.clear();
        for (int i : v) ord.emplace_back(((uint64_t)cls[i] << 62) | morton(nodes[i].x, nodes[i].y, nodes[i].z), i);
        std::sort(ord.begin(), ord.end());
        HostLevel &h = L.lv[l];
        h.n_nodes = (int)v.size();
        h.n_int = 0;
        h.n_rec = 0;
        for (int k = 0; k < h.n_nodes; ++k) {
            v[k] = ord[k].second;
            idx[v[k]] = k;
            h.n_int += cls[v[k]] == 0;
            h.n_rec += cls[v[k]] <= 1;
        }
    }
    const int64_t gn = grid_level >= 0 ? (int64_t)8 << grid_level : 0;
    if (grid_level >= 0) {
        L.sx = gn * gn;
        L.sy = gn;
        L.sz = 1;
    }
    for (int l = 0; l < L.n_levels; ++l) {
        HostLevel &h = L.lv[l];
        auto &v = per[l];
        h.nbr.assign((size_t)h.n_nodes * 27, -1);
        h.child.assign((size_t)h.n_int * 8, -1);
        h.parent.assign(h.n_nodes, -1);
        h.coord.assign((size_t)h.n_nodes * 3, 0);
        h.out_base.assign(h.n_nodes, -1);
        h.flags.assign(h.n_nodes, 0);
        h.int_child.assign(h.n_int, 0);
        for (int k = 0; k < h.n_nodes; ++k) {
            const int i = v[k];
            const Node &a = nodes[i];
            h.coord[3 * k] = a.x;
            h.coord[3 * k + 1] = a.y;
            h.coord[3 * k + 2] = a.z;
            for (int o = 0; o < 27; ++o) {
                const int b = nbrg[(size_t)i * 27 + o];
                h.nbr[27 * k + o] = b < 0 ? -1 : idx[b];
            }
            if (l > 0) h.parent[k] = idx[parent[i]];
            if (!a.leaf) {
                for (int c = 0; c < 8; ++c) {
                    const int ch = childg[(size_t)i * 8 + c];
                    h.child[8 * k + c] = idx[ch];
                    if (!isleaf[ch]) h.int_child[k] = 1;
                }
            } else {
                if (grid_level >= 0)
                    h.out_base[k] = ((int64_t)8 * a.x * gn + 8 * a.y) * gn + 8 * a.z;
                else
                    h.out_base[k] = a.leaf_index * 512;
                int32_t f = 0;
                if (k < h.n_rec) f |= kLeafX1 | kLeafLacc;
                if (l > 0) {
                    const int *pn = &nbrg[(size_t)parent[i] * 27];
                    for (int o = 0; o < 27; ++o)
                        if (pn[o] >= 0 && isleaf[pn[o]]) f |= kLeafX2;
                }
                h.flags[k] = f;
            }
        }
    }
    return L;
}

std::vector<octo_leaf> adaptive_leaves(octo_boxmax_fn boxmax, void *user, int max_level, double threshold) {
    if (!boxmax) fail(OCTO_E_INVALID, "no boxmax callback");
    if (max_level < 0 || max_level > kMaxLevel) fail(OCTO_E_INVALID, "max_level out of range");
    std::vector<std::unordered_set<uint64_t>> interior(max_level + 1);
    std::vector<std::array<int, 3>> cur{{0, 0, 0}};
    for (int l = 0; l < max_level && !cur.empty(); ++l) {
        double w = 1.0 / (double)(1 << l);
        std::vector<double> lo(3 * cur.size()), hi(3 * cur.size()), bm(cur.size());
        for (size_t i = 0; i < cur.size(); ++i)
            for (int d = 0; d < 3; ++d) {
                lo[3 * i + d] = cur[i][d] * w - 0.5;
                hi[3 * i + d] = lo[3 * i + d] + w;
            }
        boxmax((int64_t)cur.size(), lo.data(), hi.data(), bm.data(), user);
        std::vector<std::array<int, 3>> nxt;
        for (size_t i = 0; i < cur.size(); ++i) {
            if (!(bm[i] > threshold)) continue;
            interior[l].insert(key(l, cur[i][0], cur[i][1], cur[i][2]));
            for (int c = 0; c < 8; ++c)
                nxt.push_back({2 * cur[i][0] + (c >> 2), 2 * cur[i][1] + ((c >> 1) & 1), 2 * cur[i][2] + (c & 1)});
        }
        cur.swap(nxt);
    }
    auto exists = [&](int l, int x, int y, int z) {
        int m = 1 << l;
        if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m) return false;
        if (l == 0) return true;
        return interior[l - 1].count(key(l - 1, x >> 1, y >> 1, z >> 1)) > 0;
    };
    // proper nesting: refine every leaf that touches an interior node one level finer
    for (bool changed = true; changed;) {
        changed = false;
        for (int l = max_level - 1; l >= 0; --l) {
            std::vector<uint64_t> add;
            for (uint64_t k : interior[l + 1]) {
                int x = (int)((k >> 40) & 0xFFFFF), y = (int)((k >> 20) & 0xFFFFF), z = (int)(k & 0xFFFFF);
                for (int o = 0; o < 27; ++o) {
                    int nx = x + o / 9 - 1, ny = y + (o / 3) % 3 - 1, nz = z + o % 3 - 1;
                    if (nx < 0 || ny < 0 || nz < 0) continue;
                    int px = nx >> 1, py = ny >> 1, pz = nz >> 1;
                    if (!exists(l, px, py, pz)) continue;
                    uint64_t pk = key(l, px, py, pz);
                    if (!interior[l].count(pk)) add.push_back(pk);
                }
            }
            for (uint64_t k : add)
                if (interior[l].insert(k).second) changed = true;
        }
    }
    std::vector<octo_leaf> out;
    for (int l = 0; l <= max_level; ++l) {
        std::vector<std::array<int, 3>> nodes;
        if (l == 0)
            nodes.push_back({0, 0, 0});
        else
            for (uint64_t k : interior[l - 1]) {
                int x = (int)((k >> 40) & 0xFFFFF), y = (int)((k >> 20) & 0xFFFFF), z = (int)(k & 0xFFFFF);
                for (int c = 0; c < 8; ++c) nodes.push_back({2 * x + (c >> 2), 2 * y + ((c >> 1) & 1), 2 * z + (c & 1)});
            }
        for (auto &a : nodes)
            if (!interior[l].count(key(l, a[0], a[1], a[2]))) out.push_back(octo_leaf{l, a[0], a[1], a[2]});
    }
    std::sort(out.begin(), out.end(), [](const octo_leaf &a, const octo_leaf &b) {
        if (a.level != b.level) return a.level < b.level;
        if (a.ix != b.ix) return a.ix < b.ix;
        if (a.iy != b.iy) return a.iy < b.iy;
        return a.iz < b.iz;
    });
    return out;
}

// Stencils of one opening angle for levels >= 1.  For a cell of parity p
// (its index modulo 2 per axis) and an offset d to another cell of the same
// level, the parents' offset is floor((p + d) / 2).  Multipole partners are
// well separated with parents that are not; near partners are neither (d != 0).
Stencil make_stencil(double theta) {
    Stencil s;
    s.theta = theta;
    const double t2 = theta * theta;
    auto fdiv2 = [](int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); };
    std::vector<std::array<int, 3>> m2l[8], nr[8];
    for (int p = 0; p < 8; ++p) {
        int px = p >> 2, py = (p >> 1) & 1, pz = p & 1;
        for (int dx = -7; dx <= 7; ++dx)
            for (int dy = -7; dy <= 7; ++dy)
                for (int dz = -7; dz <= 7; ++dz) {
                    int Dx = fdiv2(px + dx), Dy = fdiv2(py + dy), Dz = fdiv2(pz + dz);
                    double d2 = (double)(dx * dx + dy * dy + dz * dz);
                    double D2 = (double)(Dx * Dx + Dy * Dy + Dz * Dz);
                    if (t2 * D2 > 1.0) continue;  // parents well separated
                    if (std::abs(dx) > 5 || std::abs(dy) > 5 || std::abs(dz) > 5)
                        fail(OCTO_E_UNSUPPORTED, "stencil reach above 5 cells");
                    if (t2 * d2 > 1.0)
                        m2l[p].push_back({dx, dy, dz});
                    else if (dx || dy || dz)
                        nr[p].push_back({dx, dy, dz});
                }
    }
    // neighbour sub-grids (slot (ox+1)*9 + (oy+1)*3 + oz+1) that an entry
    // reaches from any cell of target class p: a wavefront skips the entry
    // when none of them holds a source
    auto touch = [](int p, const std::array<int, 3> &d) {
        int px = p >> 2, py = (p >> 1) & 1, pz = p & 1;
        int32_t m = 0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j)
                for (int k = 0; k < 4; ++k) {
                    int sx = 2 * i + px + d[0], sy = 2 * j + py + d[1], sz = 2 * k + pz + d[2];
                    auto o = [](int v) { return v < 0 ? 0 : (v < 8 ? 1 : 2); };
                    m |= 1 << (o(sx) * 9 + o(sy) * 3 + o(sz));
                }
        return m;
    };
    for (int p = 0; p < 8; ++p) {
        s.m2l_beg[p] = (int)s.m2l.size();
        for (auto &d : m2l[p]) {
            s.m2l.push_back(pack_off(d[0], d[1], d[2]));
            s.m2l_touch.push_back(touch(p, d));
        }
        s.near_beg[p] = (int)s.nearo.size();
        for (auto &d : nr[p]) {
            s.nearo.push_back(pack_off(d[0], d[1], d[2]));
            s.near_touch.push_back(touch(p, d));
        }
        s.leaf_beg[p] = (int)s.leaf.size();
        for (int pass = 0; pass < 2; ++pass)
            for (auto &d : (pass == 0 ? m2l[p] : nr[p])) s.leaf.push_back(pack_off(d[0], d[1], d[2]));
    }
    // cross-level near partners at AMR boundaries: every offset of the
    // target classes' near lists once, with the classes whose list holds it
    // and, per class, the neighbour sub-grids it reaches.  The separation of
    // a target cell centre and a source point is a multiple of an
    // odd-integer vector n: (h/4) n with n = 1 - 2o - 4d per axis for the
    // child o (0 or 1 per axis) of a same-level cell at offset d (one level
    // down), and (h/2) n with n = 2b - 1 - 4d for a cell one level up at
    // offset d from the target's parent cell, b being the target's own index
    // bit; the table holds 1/|n| and n/|n|^3 per entry for the 8 children,
    // then for the 8 target classes.
    {
        int cls[11][11][11] = {};
        for (int p = 0; p < 8; ++p)
            for (auto &d : nr[p]) cls[d[0] + 5][d[1] + 5][d[2] + 5] |= 1 << p;
        s.xl_reach = 0;
        for (int dx = -5; dx <= 5; ++dx)
            for (int dy = -5; dy <= 5; ++dy)
                for (int dz = -5; dz <= 5; ++dz) {
                    const int c = cls[dx + 5][dy + 5][dz + 5];
                    if (!c) continue;
                    const std::array<int, 3> d{dx, dy, dz};
                    s.xl_off.push_back(pack_off(dx, dy, dz));
                    s.xl_cls.push_back(c);
                    for (int p = 0; p < 8; ++p) s.xl_touch.push_back((c >> p & 1) ? touch(p, d) : 0);
                    s.xl_reach = std::max(s.xl_reach, std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))));
                    for (int pass = 0; pass < 2; ++pass)
                        for (int j = 0; j < 8; ++j) {
                            const int bit[3] = {j >> 2, (j >> 1) & 1, j & 1};
                            double n[3], n2 = 0;
                            for (int a = 0; a < 3; ++a) {
                                n[a] = pass == 0 ? 1 - 2 * bit[a] - 4 * d[a] : 2 * bit[a] - 1 - 4 * d[a];
                                n2 += n[a] * n[a];
                            }
                            const double r = std::sqrt(n2);
                            s.xl_w.push_back(1.0 / r);
                            for (int a = 0; a < 3; ++a) s.xl_w.push_back(n[a] / (r * r * r));
                        }
                }
    }
    // near-field weights by |d| pattern (shared by all target classes, small
    // enough to stay in the scalar cache)
    s.leaf_tab.assign(kNearTab * 4, 0.0);
    for (int a = 0; a <= 5; ++a)
        for (int b = 0; b <= 5; ++b)
            for (int c = 0; c <= 5; ++c) {
                if (!(a | b | c)) continue;
                double r = std::sqrt((double)(a * a + b * b + c * c));
                double w0 = 1.0 / r;
                double w3 = w0 * w0 * w0;
                double *t = &s.leaf_tab[4 * ((a * 6 + b) * 6 + c)];
                t[0] = w0;
                t[1] = a * w3;
                t[2] = b * w3;
                t[3] = c * w3;
            }
    // near-field entries per target class grouped by sign octant, as offsets
    // into the parity-split halo: a target at x = 2i + px reads halo cell
    // ux = x + dx + 5, of class (px + dx + 5) & 1 at lattice index
    // i + ((px + dx + 5) >> 1), so the offset is the same for every cell of
    // the class.  An entry with a zero component may sit in either octant of
    // that axis (its weight there is zero); such entries are moved between
    // octants to lower the padding to whole blocks of 8, so that every
    // wavefront of a work-group walks about the same number of blocks (the
    // slowest sets the work-group's time): a local search over single moves
    // that accepts moves which do not raise the padding, from a fixed seed
    // (deterministic), keeping the best assignment seen.
    auto pad8 = [](int n) { return (8 - n % 8) % 8; };
    for (int p = 0; p < 8; ++p) {
        int px = p >> 2, py = (p >> 1) & 1, pz = p & 1;
        std::vector<std::array<int, 3>> all;
        for (int pass = 0; pass < 2; ++pass)
            for (auto &d : (pass == 0 ? m2l[p] : nr[p])) all.push_back(d);
        std::vector<int> oct(all.size()), cnt(8, 0);
        for (size_t e = 0; e < all.size(); ++e) {
            const auto &d = all[e];
            oct[e] = ((d[0] < 0) << 2) | ((d[1] < 0) << 1) | (d[2] < 0);
            ++cnt[oct[e]];
        }
        std::vector<int> movable;
        for (size_t e = 0; e < all.size(); ++e)
            if (!all[e][0] || !all[e][1] || !all[e][2]) movable.push_back((int)e);
        auto total_pad = [&]() {
            int t = 0;
            for (int o = 0; o < 8; ++o) t += pad8(cnt[o]);
            return t;
        };
        const int floor_pad = pad8((int)all.size());
        std::vector<int> best = oct;
        int best_pad = total_pad(), cur_pad = best_pad;
        uint64_t rng = 0x9e3779b97f4a7c15ull + (uint64_t)p;
        for (int iter = 0; iter < 200000 && best_pad > floor_pad && !movable.empty(); ++iter) {
            rng = rng * 6364136223846793005ull + 1442695040888963407ull;
            const int e = movable[(rng >> 33) % movable.size()];
            const auto &d = all[e];
            const int freeb = (d[0] == 0 ? 4 : 0) | (d[1] == 0 ? 2 : 0) | (d[2] == 0 ? 1 : 0);
            const int o1 = oct[e], o2 = o1 ^ (freeb & (int)(rng >> 20));
            if (o2 == o1) continue;
            const int delta = pad8(cnt[o1] - 1) + pad8(cnt[o2] + 1) - pad8(cnt[o1]) - pad8(cnt[o2]);
            if (delta > 0) continue;
            --cnt[o1];
            ++cnt[o2];
            oct[e] = o2;
            cur_pad += delta;
            if (cur_pad < best_pad) {
                best_pad = cur_pad;
                best = oct;
            }
        }
        oct = best;
        for (int o = 0; o < 8; ++o) {
            s.leaf_oct_beg[p * 9 + o] = (int)s.leaf_off.size();
            for (size_t e = 0; e < all.size(); ++e) {
                const auto &d = all[e];
                if (oct[e] != o) continue;
                int ux = px + d[0] + 5, uy = py + d[1] + 5, uz = pz + d[2] + 5;
                int q = ((ux & 1) << 2) | ((uy & 1) << 1) | (uz & 1);
                s.leaf_off.push_back(q * kNearQ + (ux >> 1) * kNearX + (uy >> 1) * kNearY + (uz >> 1));
                // weight row as a byte offset into the FP64 table (4 values a row)
                s.leaf_widx.push_back(32 * ((std::abs(d[0]) * 6 + std::abs(d[1])) * 6 + std::abs(d[2])));
            }
            // pad to whole blocks of 8 with entries of zero weight (row 0,
            // d = 0) that read the target's own halo cell
            while ((s.leaf_off.size() - s.leaf_oct_beg[p * 9 + o]) % 8) {
                s.leaf_off.push_back(0);
                s.leaf_widx.push_back(0);
            }
        }
        s.leaf_oct_beg[p * 9 + 8] = (int)s.leaf_off.size();
    }
    s.leaf_oct_beg[72] = (int)s.leaf_off.size();
    s.m2l_beg[8] = (int)s.m2l.size();
    s.near_beg[8] = (int)s.nearo.size();
    s.leaf_beg[8] = (int)s.leaf.size();
    // the same multipole entries grouped by the parity class of the source
    // cell, stored as offsets in the staged halo of that class.  The halo
    // lattice index of a source cell is its parent cell's offset from the
    // node plus 2 (multipole partners have parents at most 2 parent cells
    // away per axis for theta > 1/3): a target at x = 2i + px reads lattice
    // index ((x + dx) >> 1) + 2 = i + ((px + dx + 4) >> 1), so the offset is
    // the same for every cell of the target class
    for (int p = 0; p < 8; ++p) {
        int px = p >> 2, py = (p >> 1) & 1, pz = p & 1;
        for (int q = 0; q < 8; ++q) {
            s.m2l_src_beg[p * 9 + q] = (int)s.m2l_src.size();
            s.m2l_src_any[p * 8 + q] = 0;
            for (auto &d : m2l[p]) {
                int qq = (((px + d[0]) & 1) << 2) | (((py + d[1]) & 1) << 1) | ((pz + d[2]) & 1);
                if (qq == q) {
                    for (int a = 0; a < 3; ++a) {
                        const int pa = a == 0 ? px : (a == 1 ? py : pz);
                        if (pa + d[a] + 4 < 0 || pa + d[a] + 4 > 9)
                            fail(OCTO_E_UNSUPPORTED, "multipole partner beyond the staged halo");
                    }
                    s.m2l_src.push_back(((px + d[0] + 4) >> 1) * kHaloX + ((py + d[1] + 4) >> 1) * kHaloY +
                                        ((pz + d[2] + 4) >> 1));
                    s.m2l_src_touch.push_back(touch(p, d));
                    s.m2l_src_d.push_back(pack_off(d[0], d[1], d[2]));
                    s.m2l_src_any[p * 8 + q] |= s.m2l_src_touch.back();
                }
            }
        }
        s.m2l_src_beg[p * 9 + 8] = (int)s.m2l_src.size();
    }
    s.m2l_src_beg[72] = (int)s.m2l_src.size();
    // staging table of the near-field halo (independent of theta): which
    // neighbour sub-grid and storage index (parity-major: class << 6 | the
    // 4x4x4 lattice index) each thread loads, and where it goes in the halo
    s.near_stage.assign(kNearStage, -1);
    for (int c = 0; c < 18 * 18 * 18; ++c) {
        const int ux = c / 324, uy = (c / 18) % 18, uz = c % 18;
        const int sx = ux - 5, sy = uy - 5, sz = uz - 5;
        const int slot = ((sx >> 3) + 1) * 9 + ((sy >> 3) + 1) * 3 + ((sz >> 3) + 1);
        const int ax = sx & 7, ay = sy & 7, az = sz & 7;
        const int store = ((((ax & 1) << 2) | ((ay & 1) << 1) | (az & 1)) << 6) | ((ax >> 1) << 4) | ((ay >> 1) << 2) |
                          (az >> 1);
        const int q = ((ux & 1) << 2) | ((uy & 1) << 1) | (uz & 1);
        const int dest = q * kNearQ + (ux >> 1) * kNearX + (uy >> 1) * kNearY + (uz >> 1);
        s.near_stage[c] = slot | store << 5 | dest << 14;
    }
    return s;
}

// ---------------------------------------------------------------- plans

namespace {
inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

size_t plan_bytes(const PlanHost &ph) {
    Plan p;
    std::vector<char> img;
    return plan_layout(ph, nullptr, p, img);
}

// Lay the plan out in a device block starting at `dev`: set the Plan's device
// pointers and write the part that must be uploaded (descriptors and work
// items) into `image`; the per-item partial sums follow it.  Returns the
// total size of the block.
size_t plan_layout(const PlanHost &ph, void *dev, Plan &p, std::vector<char> &image) {
    char *base = (char *)dev;
    size_t off = 0;
    image.clear();
    auto put = [&](const void *src, size_t bytes) -> void * {
        void *dst = base + off;
        size_t n = al(bytes);
        image.resize(off + n, 0);
        if (bytes) memcpy(image.data() + off, src, bytes);
        off += n;
        return dst;
    };
    auto reserve = [&](size_t bytes) -> void * {
        void *dst = base + off;
        off += al(bytes);
        return dst;
    };
    p.n_trees = (int)ph.trees.size();
    p.n_m2l = (int)ph.m2l.size();
    p.n_leaf = (int)ph.leaf.size();
    p.n_p2m = (int)ph.p2m.size();
    p.n_m2l_nodes = (int)ph.m2l_nodes.size();
    p.n_m2l_leaf = (int)ph.m2l_leaf.size();
    p.n_levels_max = (int)ph.interior.size();
    p.d_levels = (LevelDesc *)put(ph.levels.data(), ph.levels.size() * sizeof(LevelDesc));
    p.d_trees = (TreeDesc *)put(ph.trees.data(), ph.trees.size() * sizeof(TreeDesc));
    p.d_m2l = (M2LItem *)put(ph.m2l.data(), ph.m2l.size() * sizeof(M2LItem));
    p.d_leaf = (LeafItem *)put(ph.leaf.data(), ph.leaf.size() * sizeof(LeafItem));
    p.d_p2m = (NodeItem *)put(ph.p2m.data(), ph.p2m.size() * sizeof(NodeItem));
    p.d_m2l_nodes = (M2LItem *)put(ph.m2l_nodes.data(), ph.m2l_nodes.size() * sizeof(M2LItem));
    p.d_m2l_leaf = (M2LItem *)put(ph.m2l_leaf.data(), ph.m2l_leaf.size() * sizeof(M2LItem));
    p.lds_min_level = (int)ph.interior.size();
    for (const M2LItem &q : ph.m2l_nodes) p.lds_min_level = std::min(p.lds_min_level, ph.levels[q.ld].level);
    std::vector<NodeItem> all;
    p.n_interior.clear();
    p.interior_off.clear();
    for (auto &v : ph.interior) {
        p.interior_off.push_back(all.size());
        p.n_interior.push_back((int)v.size());
        all.insert(all.end(), v.begin(), v.end());
    }
    p.d_interior = (NodeItem *)put(all.data(), all.size() * sizeof(NodeItem));
    all.clear();
    p.n_l2l.clear();
    p.l2l_off.clear();
    for (size_t l = 0; l < ph.interior.size(); ++l) {
        p.l2l_off.push_back(all.size());
        const size_t n = l < ph.l2l.size() ? ph.l2l[l].size() : 0;
        p.n_l2l.push_back((int)n);
        if (n) all.insert(all.end(), ph.l2l[l].begin(), ph.l2l[l].end());
    }
    p.d_l2l = (NodeItem *)put(all.data(), all.size() * sizeof(NodeItem));
    // coarse levels (few L2L nodes, many partial slots): separate wide sum
    p.sum_parts_level.assign(ph.interior.size(), 0);
    for (size_t l = 0; l < ph.interior.size(); ++l) {
        if (!p.n_l2l[l]) continue;
        int max_parts = 1;
        for (const NodeItem &q : ph.l2l[l]) max_parts = std::max(max_parts, ph.levels[q.ld].n_parts);
        p.sum_parts_level[l] = (max_parts > 1 && ph.l2l[l].size() <= 128) ? 1 : 0;
    }
    p.d_tree_leaf_beg = (int32_t *)put(ph.tree_leaf_beg.data(), ph.tree_leaf_beg.size() * sizeof(int32_t));
    p.d_tree_m2l_beg = (int32_t *)put(ph.tree_m2l_beg.data(), ph.tree_m2l_beg.size() * sizeof(int32_t));
    p.d_tree_m2ln_beg = (int32_t *)put(ph.tree_m2ln_beg.data(), ph.tree_m2ln_beg.size() * sizeof(int32_t));
    p.d_tree_m2lf_beg = (int32_t *)put(ph.tree_m2lf_beg.data(), ph.tree_m2lf_beg.size() * sizeof(int32_t));
    // the stats reduction's counters start at zero (uploaded with the image)
    const std::vector<int32_t> zeros(ph.trees.size(), 0);
    p.d_stat_done = (int32_t *)put(zeros.data(), zeros.size() * sizeof(int32_t));
    p.d_stat = (double *)reserve(ph.leaf.size() * kStat * sizeof(double));
    p.d_leaf_cnt = (int64_t *)reserve(ph.leaf.size() * sizeof(int64_t));
    // per-item pair counts: per-wavefront items, LDS-staged nodes, LDS-staged leaf targets
    p.d_m2l_cnt = (int64_t *)reserve((ph.m2l.size() + ph.m2l_nodes.size() + ph.m2l_leaf.size()) * sizeof(int64_t));
    p.d_out = (double *)reserve(ph.trees.size() * 12 * sizeof(double));
    p.d_stat_part = (double *)reserve(ph.trees.size() * kStatBlocks * 12 * sizeof(double));
    p.trees_host = ph.trees;
    return off;
}

// Synchronous upload (tree and batch set-up).
void plan_upload(const PlanHost &ph, void *dev, Plan &p, hipStream_t s) {
    std::vector<char> img;
    plan_layout(ph, dev, p, img);
    check_hip(hipMemcpyAsync(dev, img.data(), img.size(), hipMemcpyHostToDevice, s), "plan upload");
    check_hip(hipStreamSynchronize(s), "plan upload");
}

}  // namespace octo
