// The device layout's per-thread steps (csrc/layout_ops.h) run one thread
// after another on the CPU, in a shuffled order, with plain-memory versions
// of the atomic operations; a std::stable_sort stands in for the device's
// radix sort.  Reads a leaf list, writes the control words, the per-node host
// words and (when the list is valid) every level's tables.  Test harness
// only: built by tests/test_layout_emu.py.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <numeric>
#include <random>
#include <vector>

static inline int cas32(int *p, int c, int v) {
    const int o = *p;
    if (o == c) *p = v;
    return o;
}
static inline unsigned long long add64(unsigned long long *p, unsigned long long v) {
    const unsigned long long o = *p;
    *p += v;
    return o;
}
static inline unsigned long long min64(unsigned long long *p, unsigned long long v) {
    const unsigned long long o = *p;
    if (v < o) *p = v;
    return o;
}
#define LAY_CAS32(p, c, v) cas32((p), (c), (v))
#define LAY_ADD64(p, v) add64((p), (v))
#define LAY_MIN64(p, v) min64((p), (v))
#include "layout_ops.h"

using namespace octo;

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n = 0;
    int levels = 0;
    unsigned seed = 0;
    bool ok = fread(&n, 8, 1, f) == 1 && fread(&levels, 4, 1, f) == 1 && fread(&seed, 4, 1, f) == 1;
    std::vector<octo_leaf> leaves(n > 0 ? n : 0);
    ok = ok && n > 0 && fread(leaves.data(), sizeof(octo_leaf), n, f) == (size_t)n;
    fclose(f);
    if (!ok) return 2;
    int64_t cells = 0;
    for (int l = 0; l < levels; ++l) cells += 1ll << (3 * l);
    std::vector<int32_t> cell(cells, 0);
    const int64_t cap = n + (n + 6) / 7 + 16;
    std::vector<unsigned long long> ctl(kCtlWords);
    std::vector<uint64_t> node_lm(cap), key(cap), skey(cap);
    std::vector<int32_t> node_leaf(cap), val(cap), sval(cap), info(cap), host(2 * cap);
    LayK k{};
    k.leaf = leaves.data();
    k.n_leaf = n;
    k.cell = cell.data();
    int64_t c = 0;
    for (int l = 0; l <= kMaxLevel + 1; ++l) {
        k.goff[l] = c;
        if (l < levels) c += 1ll << (3 * l);
    }
    k.levels = levels;
    k.cap = cap;
    k.ctl = ctl.data();
    k.node_lm = node_lm.data();
    k.node_leaf = node_leaf.data();
    k.key = key.data();
    k.val = val.data();
    k.skey = skey.data();
    k.sval = sval.data();
    k.info = info.data();
    k.host = host.data();
    for (int i = 0; i < kCtlWords; ++i) ctl[i] = i == 0 ? 0 : ~0ull;
    std::mt19937 rng(seed);
    std::vector<int64_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::shuffle(ord.begin(), ord.end(), rng);
    for (int64_t i : ord) lay_mark_leaf(k, i);
    std::shuffle(ord.begin(), ord.end(), rng);
    for (int64_t i : ord) lay_mark_ancestors(k, i);
    for (int64_t s = 0; s < cap; ++s) lay_classify(k, s);
    std::vector<int64_t> p(cap);
    std::iota(p.begin(), p.end(), 0);
    std::stable_sort(p.begin(), p.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    for (int64_t i = 0; i < cap; ++i) {
        skey[i] = key[p[i]];
        sval[i] = val[p[i]];
    }
    for (int64_t i = 0; i < cap; ++i) lay_bounds(k, i);
    for (int64_t i = 0; i < cap; ++i) lay_index(k, i);
    for (int64_t i = 0; i < cap; ++i) lay_parent(k, i);
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(ctl.data(), 8, kCtlWords, o);
    fwrite(&cap, 8, 1, o);
    fwrite(host.data(), 4, 2 * cap, o);
    if (ctl[1] == ~0ull) {
        // the per-level counts as the library derives them, then the tables
        const int64_t count = (int64_t)ctl[0], none = INT64_MAX;
        auto at = [&](int l, int cc) { return ctl[2 + 3 * l + cc] == ~0ull ? none : (int64_t)ctl[2 + 3 * l + cc]; };
        auto start = [&](int l) { return std::min({at(l, 0), at(l, 1), at(l, 2)}); };
        int nl = 0;
        while (nl < k.levels && start(nl) != none) ++nl;
        LayTables t{};
        std::vector<std::vector<int32_t>> nb(nl), ch(nl), pa(nl), co(nl);
        std::vector<std::vector<int64_t>> ob(nl);
        std::vector<int64_t> nn(nl), ni(nl);
        for (int l = 0; l < nl; ++l) {
            const int64_t end = l + 1 < nl ? start(l + 1) : count;
            nn[l] = end - start(l);
            ni[l] = std::min({at(l, 1), at(l, 2), end}) - start(l);
            nb[l].assign(nn[l] * 27, -99);
            ch[l].assign(ni[l] * 8, -99);
            pa[l].assign(nn[l], -99);
            co[l].assign(nn[l] * 3, -99);
            ob[l].assign(nn[l], -99);
            t.nbr[l] = nb[l].data();
            t.child[l] = ch[l].data();
            t.parent[l] = pa[l].data();
            t.coord[l] = co[l].data();
            t.out_base[l] = ob[l].data();
            t.n_int[l] = (int)ni[l];
        }
        for (int64_t i = 0; i < cap; ++i) lay_tables(k, t, i);
        fwrite(&nl, 4, 1, o);
        for (int l = 0; l < nl; ++l) {
            fwrite(&nn[l], 8, 1, o);
            fwrite(&ni[l], 8, 1, o);
            fwrite(nb[l].data(), 4, nb[l].size(), o);
            fwrite(ch[l].data(), 4, ch[l].size(), o);
            fwrite(pa[l].data(), 4, pa[l].size(), o);
            fwrite(co[l].data(), 4, co[l].size(), o);
            fwrite(ob[l].data(), 8, ob[l].size(), o);
        }
    }
    for (int64_t s = 0; s < cap; ++s) lay_clear(k, s);
    int64_t dirty = 0;
    for (int32_t v : cell) dirty += v != 0;
    fwrite(&dirty, 8, 1, o);
    fclose(o);
    return 0;
}
