// Host-only introspection entry points (include/octo_host.h).
#include <algorithm>
#include <cmath>

#include "octo_host.h"
#include "runtime.h"

using namespace octo;

namespace octo {
void set_error(const std::string &m);
}

template <typename F>
static octo_status guard_h(F &&f) {
    try {
        f();
        return OCTO_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return OCTO_E_INVALID;
    }
}

extern "C" {

octo_status octo_host_stencil_sizes(double theta, int32_t *out) {
    return guard_h([&] {
        if (!out) fail(OCTO_E_INVALID, "out is NULL");
        if (!(theta >= 0.34 && theta < 1.0)) fail(OCTO_E_UNSUPPORTED, "theta must lie in [0.34, 1)");
        Stencil s = make_stencil(theta);
        for (int p = 0; p < 8; ++p) {
            out[p] = s.m2l_beg[p + 1] - s.m2l_beg[p];
            out[8 + p] = s.near_beg[p + 1] - s.near_beg[p];
            int reach = 0;
            for (int k = s.leaf_beg[p]; k < s.leaf_beg[p + 1]; ++k) {
                int v = s.leaf[k];
                int dx = (int)(int8_t)(v & 255), dy = (int)(int8_t)((v >> 8) & 255), dz = (int)(int8_t)((v >> 16) & 255);
                reach = std::max(reach, std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))));
            }
            out[16 + p] = reach;
        }
    });
}

octo_status octo_host_near_lists(double theta, int32_t *beg, int32_t *d, int64_t cap, int64_t *n) {
    return guard_h([&] {
        if (!beg || !n) fail(OCTO_E_INVALID, "NULL output");
        if (!(theta >= 0.34 && theta < 1.0)) fail(OCTO_E_UNSUPPORTED, "theta must lie in [0.34, 1)");
        Stencil s = make_stencil(theta);
        for (int k = 0; k < 73; ++k) beg[k] = s.leaf_oct_beg[k];
        *n = (int64_t)s.leaf_off.size();
        if (!d || cap < *n) return;
        // back from halo offsets to d: a target of class p reads halo cell
        // u = x + d + 5 of parity class q at lattice index (u >> 1)
        for (int p = 0; p < 8; ++p) {
            const int pc[3] = {p >> 2, (p >> 1) & 1, p & 1};
            for (int k = s.leaf_oct_beg[9 * p]; k < s.leaf_oct_beg[9 * p + 8]; ++k) {
                if (s.leaf_widx[k] == 0) {  // padding (row of d = 0)
                    d[k] = 0;
                    continue;
                }
                const int off = s.leaf_off[k], q = off / kNearQ, r = off % kNearQ;
                const int lat[3] = {r / kNearX, (r % kNearX) / kNearY, (r % kNearX) % kNearY};
                int dd[3];
                for (int a = 0; a < 3; ++a) dd[a] = 2 * lat[a] + ((q >> (2 - a)) & 1) - pc[a] - 5;
                d[k] = pack_off(dd[0], dd[1], dd[2]);
            }
        }
    });
}

octo_status octo_host_near_stage(int32_t *out, int64_t cap, int64_t *n) {
    return guard_h([&] {
        if (!n) fail(OCTO_E_INVALID, "NULL output");
        Stencil s = make_stencil(0.5);  // the table does not depend on theta
        *n = (int64_t)s.near_stage.size();
        if (!out || cap < *n) return;
        for (size_t k = 0; k < s.near_stage.size(); ++k) out[k] = s.near_stage[k];
    });
}

octo_status octo_host_layout(const octo_leaf *leaves, int64_t n_leaves, int32_t *n_levels, int64_t *out) {
    return guard_h([&] {
        if (!n_levels || !out) fail(OCTO_E_INVALID, "NULL output");
        Layout L = build_layout(leaves, n_leaves, -1);
        *n_levels = L.n_levels;
        for (int l = 0; l <= kMaxLevel; ++l) {
            const bool have = l < L.n_levels;
            out[3 * l] = have ? L.lv[l].n_nodes : 0;
            out[3 * l + 1] = have ? L.lv[l].n_int : 0;
            out[3 * l + 2] = have ? L.lv[l].n_rec - L.lv[l].n_int : 0;
        }
    });
}

octo_status octo_host_level_tables(const octo_leaf *leaves, int64_t n_leaves, int32_t level, int64_t *sizes,
                                   const octo_level_tables *out) {
    return guard_h([&] {
        if (!sizes) fail(OCTO_E_INVALID, "NULL sizes");
        const Layout L = build_layout(leaves, n_leaves, -1);
        if (level < 0 || level >= L.n_levels) fail(OCTO_E_INVALID, "level out of range");
        const HostLevel &h = L.lv[level];
        sizes[0] = h.n_nodes;
        sizes[1] = h.n_int;
        sizes[2] = h.n_rec;
        if (!out) return;
        auto put = [](auto *dst, const auto &v) {
            if (dst)
                for (size_t i = 0; i < v.size(); ++i) dst[i] = v[i];
        };
        put(out->nbr, h.nbr);
        put(out->child, h.child);
        put(out->parent, h.parent);
        put(out->coord, h.coord);
        put(out->out_base, h.out_base);
        put(out->flags, h.flags);
        put(out->int_child, h.int_child);
    });
}

octo_status octo_host_adaptive_leaves(octo_boxmax_fn boxmax, void *user, int max_level, double threshold,
                                      octo_leaf *out, int64_t cap, int64_t *n) {
    return guard_h([&] {
        if (!n) fail(OCTO_E_INVALID, "n is NULL");
        std::vector<octo_leaf> v = adaptive_leaves(boxmax, user, max_level, threshold);
        *n = (int64_t)v.size();
        if (out && cap >= (int64_t)v.size()) std::copy(v.begin(), v.end(), out);
    });
}

}  // extern "C"
