// HIP kernels of the gravity solve for gfx950 (wave64).
//
// Method (Octo-Tiger, Sec. 2.2): leaf cells are point masses; multipoles
// (mass, centre of mass, raw 2nd and 3rd moments) are composed upward; cells
// of one level that are well separated while their parents are not interact
// through a third-order multipole-to-local expansion plus the
// angular-momentum correction; leaf pairs that are not covered that way are
// summed directly; expansions are shifted downward and evaluated at the
// leaves (phi, g = -grad phi).
//
// Work decomposition: one 64-lane wavefront = one parity class (64 cells) of
// one 8^3 node, so every lane of a wavefront walks the same stencil of
// neighbour offsets; work-group ids are remapped so that consecutive items
// land on the same XCD (each XCD has its own L2).
#include <hip/hip_runtime.h>

#include "octo_internal.h"
#include "runtime.h"

namespace octo {

namespace {

constexpr int kXcd = 8;

// blockIdx -> item: the hardware deals work-groups round-robin over the XCDs;
// give each XCD a contiguous slice of the item list instead.
__device__ inline int xcd_item(int n_items) {
    const int b = blockIdx.x;
    const int per = (n_items + kXcd - 1) / kXcd;
    return (b % kXcd) * per + b / kXcd;
}

__device__ inline int grid_for_items(int n) { return n; }

__device__ inline void local_xyz(int s, int &x, int &y, int &z) {
    const int p = s >> 6, q = s & 63;
    x = ((q >> 4) << 1) | (p >> 2);
    y = (((q >> 2) & 3) << 1) | ((p >> 1) & 1);
    z = ((q & 3) << 1) | (p & 1);
}

__device__ inline int store_idx(int x, int y, int z) {
    return ((((x & 1) << 2) | ((y & 1) << 1) | (z & 1)) << 6) | (((x >> 1) << 4) | ((y >> 1) << 2) | (z >> 1));
}

__device__ inline double centre(int gi, double h) { return (gi + 0.5) * h - 0.5; }

__device__ inline void unpack(int32_t off, int &dx, int &dy, int &dz) {
    dx = (int)(int8_t)(off & 255);
    dy = (int)(int8_t)((off >> 8) & 255);
    dz = (int)(int8_t)((off >> 16) & 255);
}

// a pointer into device memory as a global-address-space pointer: its loads
// are global loads, which count only against the vector-memory counter
template <typename T>
using GPtr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ inline GPtr<T> gptr(T *p) {
    return (GPtr<T>)p;
}

__device__ inline int nbr_slot(int sx, int sy, int sz) {
    return ((sx >> 3) + 1) * 9 + ((sy >> 3) + 1) * 3 + ((sz >> 3) + 1);
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The sum over the 64 lanes of a wavefront in lane 63 (other lanes hold
// partial sums), by data-parallel moves within and across the four 16-lane
// rows: pairs, quads, row_shr 4 and 8 (the row total in lane 15 of each
// row), then lane 15 of rows 0 and 2 into rows 1 and 3, and lane 31 into rows
// 2 and 3.  A fixed order: the same inputs give the same bits.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ inline double wave_total_lane63(double v) {
    v += dpp_move<0xb1, 0xf>(v);   // quad_perm 1,0,3,2
    v += dpp_move<0x4e, 0xf>(v);   // quad_perm 2,3,0,1
    v += dpp_move<0x114, 0xf>(v);  // row_shr 4
    v += dpp_move<0x118, 0xf>(v);  // row_shr 8
    v += dpp_move<0x142, 0xa>(v);  // row_bcast 15 (rows 1, 3)
    v += dpp_move<0x143, 0xc>(v);  // row_bcast 31 (rows 2, 3)
    return v;
}

// packed symmetric index helpers for 3rd-order tensors:
// xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
// sum_{bc} T_abc u_b u_c for each a
__device__ inline void t3_uu(const double *T, double ux, double uy, double uz, double &ox, double &oy,
                             double &oz) {
    const double xx = ux * ux, yy = uy * uy, zz = uz * uz, xy = ux * uy, xz = ux * uz, yz = uy * uz;
    ox = T[0] * xx + T[3] * yy + T[5] * zz + 2.0 * (T[1] * xy + T[2] * xz + T[4] * yz);
    oy = T[1] * xx + T[6] * yy + T[8] * zz + 2.0 * (T[3] * xy + T[4] * xz + T[7] * yz);
    oz = T[2] * xx + T[7] * yy + T[9] * zz + 2.0 * (T[4] * xy + T[5] * xz + T[8] * yz);
}

// traces t_a = T_abb
__device__ inline void t3_trace(const double *T, double &tx, double &ty, double &tz) {
    tx = T[0] + T[3] + T[5];
    ty = T[1] + T[6] + T[8];
    tz = T[2] + T[7] + T[9];
}

// Trace-free parts of the raw moments.  Every contraction the multipole step
// makes is with a derivative tensor D^(k) of 1/r, k >= 2, which is trace-free
// in every index pair (1/r is harmonic), so only these parts contribute:
//   Q' = Q - (tr Q / 3) I,  O'_abc = O_abc - (d_ab t_c + d_ac t_b + d_bc t_a) / 5,
// t_a = O_abb.  Stored as independent components: q5 = xx xy xz yy yz
// (zz = -xx - yy); o7 = xxx xxy xxz xyy xyz yyy yyz (xzz = -xxx - xyy,
// yzz = -xxy - yyy, zzz = -xxz - yyz).
__device__ inline void detrace_q(const double *Q, double *q5) {
    const double t = (Q[0] + Q[3] + Q[5]) * (1.0 / 3.0);
    q5[0] = Q[0] - t;
    q5[1] = Q[1];
    q5[2] = Q[2];
    q5[3] = Q[3] - t;
    q5[4] = Q[4];
}
__device__ inline void detrace_o(const double *O, double *o7) {
    double tx, ty, tz;
    t3_trace(O, tx, ty, tz);
    tx *= 0.2;
    ty *= 0.2;
    tz *= 0.2;
    o7[0] = O[0] - 3.0 * tx;
    o7[1] = O[1] - ty;
    o7[2] = O[2] - tz;
    o7[3] = O[3] - tx;
    o7[4] = O[4];
    o7[5] = O[6] - 3.0 * ty;
    o7[6] = O[7] - tz;
}

// (O':RR)_a = sum_bc O'_abc R_b R_c for a trace-free O' (o7 packing), given
// e = xx - zz, f = yy - zz, u = 2xy, v = 2xz, w = 2yz of R.
template <typename T>
__device__ inline void o7_rr(const T *o, T e, T f, T u, T v, T w, T &ox, T &oy, T &oz) {
    const T xzz = -(o[0] + o[3]), yzz = -(o[1] + o[5]);
    ox = o[0] * e + o[3] * f + o[1] * u + o[2] * v + o[4] * w;
    oy = o[1] * e + o[5] * f + o[3] * u + o[4] * v + o[6] * w;
    oz = o[2] * e + o[6] * f + o[4] * u + xzz * v + yzz * w;
}

}  // namespace

// ------------------------------------------------------------------ P2M
// Leaf cells become point masses m = rho h^3 at their centres (the record
// leaves' trivial multipole records are written once, k_leaf_records); each
// mass also goes into its parent cell's child-mass record.  SRC: the second
// source (a density rate) instead of the density; its leaf cells are point
// sources at the same centres, with zero dipole.
template <bool SRC>
__global__ __launch_bounds__(256) void k_p2m(const LevelDesc *__restrict__ L, const TreeDesc *__restrict__ T,
                                             const NodeItem *__restrict__ items, int n_items) {
    const int it = blockIdx.x >> 1;
    if (it >= n_items) return;
    const NodeItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const TreeDesc td = T[ld.tree];
    const int node = item.node;
    const int s = ((blockIdx.x & 1) << 8) | threadIdx.x;
    int x, y, z;
    local_xyz(s, x, y, z);
    const double h = ld.h;
    const int64_t off = gptr(ld.out_base)[node] + x * td.sx + y * td.sy + z * td.sz;
    const double m = gptr(SRC ? td.src : td.rho)[off] * (h * h * h);
    const size_t ci = (size_t)node * kCells + s;
    gptr(ld.mass)[ci] = m;
    if (ld.parent_ld >= 0) {
        // the parent cell's list of child masses (cross-level near pairs)
        const LevelDesc pl = L[ld.parent_ld];
        const GPtr<const int32_t> coord = gptr(ld.coord);
        const int px = 4 * (coord[3 * node] & 1) + (x >> 1), py = 4 * (coord[3 * node + 1] & 1) + (y >> 1),
                  pz = 4 * (coord[3 * node + 2] & 1) + (z >> 1);
        const size_t pc = (size_t)gptr(ld.parent)[node] * kCells + store_idx(px, py, pz);
        gptr(pl.cm)[pc * 8 + (((x & 1) << 2) | ((y & 1) << 1) | (z & 1))] = m;
    }
}

// The multipole record of the record leaves' cells, which no solve changes:
// centre of mass at the cell centre, zero second and third moments, zero
// dipole of a second source.  Written once per tree (with its work plan),
// so the leaf-mass pass writes the masses only.
__global__ __launch_bounds__(256) void k_leaf_records(const LevelDesc *__restrict__ L,
                                                      const NodeItem *__restrict__ items, int n_items) {
    const int it = blockIdx.x >> 1;
    if (it >= n_items) return;
    const NodeItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const int node = item.node;
    if (node >= ld.n_rec) return;
    const int s = ((blockIdx.x & 1) << 8) | threadIdx.x;
    int x, y, z;
    local_xyz(s, x, y, z);
    const double h = ld.h;
    const size_t S = (size_t)ld.n_rec * kCells, ci = (size_t)node * kCells + s;
    ld.mp[ci] = centre(8 * ld.coord[3 * node] + x, h);
    ld.mp[S + ci] = centre(8 * ld.coord[3 * node + 1] + y, h);
    ld.mp[2 * S + ci] = centre(8 * ld.coord[3 * node + 2] + z, h);
    for (int c = 3; c < kRec; ++c) ld.mp[c * S + ci] = 0.0;
    for (int c = 0; c < 3; ++c) ld.dip[c * S + ci] = 0.0;
}

// ------------------------------------------------------------------ M2M
// Parent multipole from its 8 children: mass, centre of mass, and the raw
// 2nd/3rd moments about it (parallel-axis shifts; the children's dipoles
// about their own centres of mass vanish).
__global__ __launch_bounds__(256) void k_m2m(const LevelDesc *__restrict__ L, const NodeItem *__restrict__ items,
                                             int n_items) {
    const int it = blockIdx.x >> 1;
    if (it >= n_items) return;
    const NodeItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const LevelDesc cl = L[ld.child_ld];
    // the two levels' arrays as global pointers (global loads count only
    // against the vector-memory counter)
    const GPtr<const int32_t> child = gptr(ld.child), ccoord = gptr(cl.coord);
    const GPtr<const double> cmass = gptr(cl.mass), cmp = gptr(cl.mp);
    const GPtr<double> mass = gptr(ld.mass), mp = gptr(ld.mp);
    const int node = item.node;
    const int s = ((blockIdx.x & 1) << 8) | threadIdx.x;
    int x, y, z;
    local_xyz(s, x, y, z);
    const size_t CS = (size_t)cl.n_rec * kCells;
    int cn[8], cs[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int cx = 2 * x + (c >> 2), cy = 2 * y + ((c >> 1) & 1), cz = 2 * z + (c & 1);
        cn[c] = child[node * 8 + ((cx >> 3) << 2) + ((cy >> 3) << 1) + (cz >> 3)];
        cs[c] = store_idx(cx & 7, cy & 7, cz & 7);
    }
    auto child_com = [&](int c, double &zx, double &zy, double &zz) {
        const size_t ci = (size_t)cn[c] * kCells + cs[c];
        if (cn[c] < cl.n_rec) {
            zx = cmp[ci];
            zy = cmp[CS + ci];
            zz = cmp[2 * CS + ci];
        } else {
            const int cx = 2 * x + (c >> 2), cy = 2 * y + ((c >> 1) & 1), cz = 2 * z + (c & 1);
            const int ch = child[node * 8 + ((cx >> 3) << 2) + ((cy >> 3) << 1) + (cz >> 3)];
            zx = centre(8 * ccoord[3 * ch] + (cx & 7), cl.h);
            zy = centre(8 * ccoord[3 * ch + 1] + (cy & 7), cl.h);
            zz = centre(8 * ccoord[3 * ch + 2] + (cz & 7), cl.h);
        }
    };
    double m = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const double cm = cmass[(size_t)cn[c] * kCells + cs[c]];
        double zx, zy, zz;
        child_com(c, zx, zy, zz);
        m += cm;
        mx += cm * zx;
        my += cm * zy;
        mz += cm * zz;
    }
    double Zx, Zy, Zz;
    if (m > 0.0) {
        Zx = mx / m;
        Zy = my / m;
        Zz = mz / m;
    } else {
        Zx = centre(8 * gptr(ld.coord)[3 * node] + x, ld.h);
        Zy = centre(8 * gptr(ld.coord)[3 * node + 1] + y, ld.h);
        Zz = centre(8 * gptr(ld.coord)[3 * node + 2] + z, ld.h);
    }
    double Q[6] = {0, 0, 0, 0, 0, 0};
    double O[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int c = 0; c < 8; ++c) {
        const size_t ci = (size_t)cn[c] * kCells + cs[c];
        const double cm = cmass[ci];
        double zx, zy, zz;
        child_com(c, zx, zy, zz);
        const double sx = zx - Zx, sy = zy - Zy, sz = zz - Zz;
        double q[6] = {0, 0, 0, 0, 0, 0}, o[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (cn[c] < cl.n_rec) {
#pragma unroll
            for (int k = 0; k < 6; ++k) q[k] = cmp[(3 + k) * CS + ci];
#pragma unroll
            for (int k = 0; k < 10; ++k) o[k] = cmp[(9 + k) * CS + ci];
        }
        // second moments: q_ab + m s_a s_b
        Q[0] += q[0] + cm * sx * sx;
        Q[1] += q[1] + cm * sx * sy;
        Q[2] += q[2] + cm * sx * sz;
        Q[3] += q[3] + cm * sy * sy;
        Q[4] += q[4] + cm * sy * sz;
        Q[5] += q[5] + cm * sz * sz;
        // third moments: o_abc + q_ab s_c + q_ac s_b + q_bc s_a + m s_a s_b s_c
        // q packed: xx0 xy1 xz2 yy3 yz4 zz5
        O[0] += o[0] + 3.0 * q[0] * sx + cm * sx * sx * sx;                      // xxx
        O[1] += o[1] + q[0] * sy + 2.0 * q[1] * sx + cm * sx * sx * sy;          // xxy
        O[2] += o[2] + q[0] * sz + 2.0 * q[2] * sx + cm * sx * sx * sz;          // xxz
        O[3] += o[3] + q[3] * sx + 2.0 * q[1] * sy + cm * sx * sy * sy;          // xyy
        O[4] += o[4] + q[1] * sz + q[2] * sy + q[4] * sx + cm * sx * sy * sz;    // xyz
        O[5] += o[5] + q[5] * sx + 2.0 * q[2] * sz + cm * sx * sz * sz;          // xzz
        O[6] += o[6] + 3.0 * q[3] * sy + cm * sy * sy * sy;                      // yyy
        O[7] += o[7] + q[3] * sz + 2.0 * q[4] * sy + cm * sy * sy * sz;          // yyz
        O[8] += o[8] + q[5] * sy + 2.0 * q[4] * sz + cm * sy * sz * sz;          // yzz
        O[9] += o[9] + 3.0 * q[5] * sz + cm * sz * sz * sz;                      // zzz
    }
    const size_t pi = (size_t)node * kCells + s;
    const size_t PS = (size_t)ld.n_rec * kCells;
    mass[pi] = m;
    mp[pi] = Zx;
    mp[PS + pi] = Zy;
    mp[2 * PS + pi] = Zz;
#pragma unroll
    for (int k = 0; k < 6; ++k) mp[(3 + k) * PS + pi] = Q[k];
#pragma unroll
    for (int k = 0; k < 10; ++k) mp[(9 + k) * PS + pi] = O[k];
}

// Second source: moments of orders 0-3 of the children's second-source
// multipoles about the parent's density centre of mass (written by k_m2m),
// where the dipole does not vanish: with s = z_c - Z,
//   M1 += d + m s,  M2_ab += q_ab + d_a s_b + d_b s_a + m s_a s_b,
//   M3_abc += o_abc + (q_ab s_c + q_ac s_b + q_bc s_a)
//            + (d_a s_b s_c + d_b s_a s_c + d_c s_a s_b) + m s_a s_b s_c.
__global__ __launch_bounds__(256) void k_m2m_src(const LevelDesc *__restrict__ L, const NodeItem *__restrict__ items,
                                                 int n_items) {
    const int it = blockIdx.x >> 1;
    if (it >= n_items) return;
    const NodeItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const LevelDesc cl = L[ld.child_ld];
    // the two levels' arrays as global pointers (global loads count only
    // against the vector-memory counter)
    const GPtr<const int32_t> child = gptr(ld.child), ccoord = gptr(cl.coord);
    const GPtr<const double> cmass = gptr(cl.mass), cmp = gptr(cl.mp), cdip = gptr(cl.dip);
    const GPtr<double> mass = gptr(ld.mass), mp = gptr(ld.mp), dip = gptr(ld.dip);
    const int node = item.node;
    const int s = ((blockIdx.x & 1) << 8) | threadIdx.x;
    int x, y, z;
    local_xyz(s, x, y, z);
    const size_t CS = (size_t)cl.n_rec * kCells;
    const size_t pi = (size_t)node * kCells + s;
    const size_t PS = (size_t)ld.n_rec * kCells;
    const double Zx = mp[pi], Zy = mp[PS + pi], Zz = mp[2 * PS + pi];
    double m = 0.0, D[3] = {0, 0, 0};
    double Q[6] = {0, 0, 0, 0, 0, 0};
    double O[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int c = 0; c < 8; ++c) {
        const int cx = 2 * x + (c >> 2), cy = 2 * y + ((c >> 1) & 1), cz = 2 * z + (c & 1);
        const int cn = child[node * 8 + ((cx >> 3) << 2) + ((cy >> 3) << 1) + (cz >> 3)];
        const size_t ci = (size_t)cn * kCells + store_idx(cx & 7, cy & 7, cz & 7);
        const double cm = cmass[ci];
        double zx, zy, zz;
        double d[3] = {0, 0, 0}, q[6] = {0, 0, 0, 0, 0, 0}, o[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (cn < cl.n_rec) {
            zx = cmp[ci];
            zy = cmp[CS + ci];
            zz = cmp[2 * CS + ci];
#pragma unroll
            for (int k = 0; k < 3; ++k) d[k] = cdip[k * CS + ci];
#pragma unroll
            for (int k = 0; k < 6; ++k) q[k] = cmp[(3 + k) * CS + ci];
#pragma unroll
            for (int k = 0; k < 10; ++k) o[k] = cmp[(9 + k) * CS + ci];
        } else {
            zx = centre(8 * ccoord[3 * cn] + (cx & 7), cl.h);
            zy = centre(8 * ccoord[3 * cn + 1] + (cy & 7), cl.h);
            zz = centre(8 * ccoord[3 * cn + 2] + (cz & 7), cl.h);
        }
        const double sx = zx - Zx, sy = zy - Zy, sz = zz - Zz;
        m += cm;
        D[0] += d[0] + cm * sx;
        D[1] += d[1] + cm * sy;
        D[2] += d[2] + cm * sz;
        // q packed: xx0 xy1 xz2 yy3 yz4 zz5
        Q[0] += q[0] + 2.0 * d[0] * sx + cm * sx * sx;
        Q[1] += q[1] + d[0] * sy + d[1] * sx + cm * sx * sy;
        Q[2] += q[2] + d[0] * sz + d[2] * sx + cm * sx * sz;
        Q[3] += q[3] + 2.0 * d[1] * sy + cm * sy * sy;
        Q[4] += q[4] + d[1] * sz + d[2] * sy + cm * sy * sz;
        Q[5] += q[5] + 2.0 * d[2] * sz + cm * sz * sz;
        O[0] += o[0] + 3.0 * q[0] * sx + 3.0 * d[0] * sx * sx + cm * sx * sx * sx;                          // xxx
        O[1] += o[1] + q[0] * sy + 2.0 * q[1] * sx + d[1] * sx * sx + 2.0 * d[0] * sx * sy + cm * sx * sx * sy;  // xxy
        O[2] += o[2] + q[0] * sz + 2.0 * q[2] * sx + d[2] * sx * sx + 2.0 * d[0] * sx * sz + cm * sx * sx * sz;  // xxz
        O[3] += o[3] + q[3] * sx + 2.0 * q[1] * sy + d[0] * sy * sy + 2.0 * d[1] * sx * sy + cm * sx * sy * sy;  // xyy
        O[4] += o[4] + q[1] * sz + q[2] * sy + q[4] * sx + d[0] * sy * sz + d[1] * sx * sz + d[2] * sx * sy +
                cm * sx * sy * sz;                                                                           // xyz
        O[5] += o[5] + q[5] * sx + 2.0 * q[2] * sz + d[0] * sz * sz + 2.0 * d[2] * sx * sz + cm * sx * sz * sz;  // xzz
        O[6] += o[6] + 3.0 * q[3] * sy + 3.0 * d[1] * sy * sy + cm * sy * sy * sy;                          // yyy
        O[7] += o[7] + q[3] * sz + 2.0 * q[4] * sy + d[2] * sy * sy + 2.0 * d[1] * sy * sz + cm * sy * sy * sz;  // yyz
        O[8] += o[8] + q[5] * sy + 2.0 * q[4] * sz + d[1] * sz * sz + 2.0 * d[2] * sy * sz + cm * sy * sz * sz;  // yzz
        O[9] += o[9] + 3.0 * q[5] * sz + 3.0 * d[2] * sz * sz + cm * sz * sz * sz;                          // zzz
    }
    mass[pi] = m;
#pragma unroll
    for (int k = 0; k < 3; ++k) dip[k * PS + pi] = D[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) mp[(3 + k) * PS + pi] = Q[k];
#pragma unroll
    for (int k = 0; k < 10; ++k) mp[(9 + k) * PS + pi] = O[k];
}

// ------------------------------------------------------------------ M2L
// Multipole-to-local of one ordered pair A <- B (R = z_A - z_B), truncated
// at total order 3 (L^(n) takes source moments of order <= 3 - n), with the
// angular-momentum correction: C_A += -(1/6) [M3_B - (m_B/m_A) M3_A] : D4(R).
// G is applied once at the end.
// Accumulators of one target: L0, L1 directly; L2 and L3 as the sums
// T2 = sum m f2 R R and T3 = sum m f3 R R R, from which L2 = -(T2 + s1 I)
// and L3 = -(T3 + sym(I U)) are formed once at the end (finish_l2_l3), with
// s1 = sum m f1 and U = sum m f2 R taken from the traces of T2 and T3: the
// derivative tensors of 1/r are trace-free (f2 r^2 = -3 f1, f3 r^2 = -5 f2),
// so tr T2 = -3 s1 and the (a,a,c) trace of T3 is -5 U_c; C is the correction.
template <typename T>
struct Acc {
    T L0, L1[3], L2[6], L3[10];
    double C[3];
    T A2, A3;  // FP64 density solves: parts of L0 (m2l_pair_f64)
};

template <typename T>
__device__ inline void acc_zero(Acc<T> &a) {
    a.L0 = (T)0;
    a.A2 = (T)0;
    a.A3 = (T)0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a.L1[k] = (T)0;
        a.C[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) a.L2[k] = (T)0;
#pragma unroll
    for (int k = 0; k < 10; ++k) a.L3[k] = (T)0;
}

// After the last pair: the unscaled sums of m2l_pair_f64 to the common form.
template <bool DIP, typename T>
__device__ inline void acc_close(Acc<T> &a) {
    a.L0 = -(a.L0 + 1.5 * a.A2 + 2.5 * a.A3);
#pragma unroll
    for (int k = 0; k < 10; ++k) a.L3[k] *= -15.0;
}

// L2 = -(T2 + s1 I); L3_abc = -(T3_abc + d_ab U_c + d_ac U_b + d_bc U_a),
// with s1 = -tr(T2) / 3 and U_c = -(T3_xxc + T3_yyc + T3_zzc) / 5 (T3 as
// scaled by acc_close, L2 holding T2 and the dipole terms, whose trace is
// the dipole's part of -3 s1)
template <typename T>
__device__ inline void finish_l2_l3(Acc<T> &a) {
    const T s1 = -(a.L2[0] + a.L2[3] + a.L2[5]) * (T)(1.0 / 3.0);
    const T Ux = -(a.L3[0] + a.L3[3] + a.L3[5]) * (T)0.2;
    const T Uy = -(a.L3[1] + a.L3[6] + a.L3[8]) * (T)0.2;
    const T Uz = -(a.L3[2] + a.L3[7] + a.L3[9]) * (T)0.2;
    a.L2[0] = -(a.L2[0] + s1);
    a.L2[1] = -a.L2[1];
    a.L2[2] = -a.L2[2];
    a.L2[3] = -(a.L2[3] + s1);
    a.L2[4] = -a.L2[4];
    a.L2[5] = -(a.L2[5] + s1);
    const T three = (T)3;
    a.L3[0] = -(a.L3[0] + three * Ux);
    a.L3[1] = -(a.L3[1] + Uy);
    a.L3[2] = -(a.L3[2] + Uz);
    a.L3[3] = -(a.L3[3] + Ux);
    a.L3[4] = -a.L3[4];
    a.L3[5] = -(a.L3[5] + Ux);
    a.L3[6] = -(a.L3[6] + three * Uy);
    a.L3[7] = -(a.L3[7] + Uz);
    a.L3[8] = -(a.L3[8] + Uy);
    a.L3[9] = -(a.L3[9] + three * Uz);
}

// Multipole-to-local of one ordered pair, on trace-free source moments (q5,
// o7 packing); with D^(k) the derivative tensors of 1/r at R:
//   L0 -= m f0 + (1/2) f2 R.Q'.R - (1/6) f3 O'.RRR
//   L1_a -= (m f1 + (1/2) f3 R.Q'.R) R_a + f2 (Q'R)_a
// (the trace terms f1 tr Q, f2 tr O vanish).  DIP: the source also has a
// dipole d (second source expanded about the density's centres): L0 += d.D1,
// L1_a += d_b D2_ab, L2_ab += d_c D3_abc, i.e. with w = d.R: L0 += f1 w;
// L1_a += f2 w R_a + f1 d_a; L2_ab += f3 w R_a R_b + f2 (w d_ab + R_a d_b +
// R_b d_a).  Correction: n = O'_B - mu O'_A is trace-free, so n : D4 reduces
// to f4 (n:RR . R) R + 3 f3 (n:RR), with n:RR = O'_B:RR - mu O'_A:RR.
//
// In FP64, with the radial chain's
// constant factors folded into the coefficients.  With g = 1/|R| and
// p_n = g^(2n+1): f0 = g, f1 = -p1, f2 = 3 p2, f3 = -15 p3, f4 = 105 p4, so
//   L0 = -(A0 + 3/2 A2 + 5/2 A3), A0 = sum m g, A2 = sum p2 R.Q'.R,
//        A3 = sum p3 O':RRR (A0 kept in L0 until acc_close);
//   L1_a += (m p1 + 15/2 p3 R.Q'.R) R_a - 3 p2 (Q'R)_a;
//   T2 += 3 m p2 RR;  T3 += m p3 RRR (scaled by -15 in acc_close);
//   C_a += 15/2 p3 (n:RR)_a - 35/2 p4 (n:RR.R) R_a.
// DIP (a second source with a dipole d about the density's centre, w = d.R,
// no correction): A0 also sums p1 w; the L1 coefficient gains 3 p2 w and
// L1_a gains -p1 d_a; T2 += 15 p3 w RR; and L2_ab -= 3 p2 (d_a R_b + d_b R_a).
// Every update is one fused multiply-add.
template <bool LEAF_TARGET, bool DIP>
__device__ inline void m2l_pair_f64(double Rx, double Ry, double Rz, double mB, const double *q, const double *o,
                                    const double *dp, double mu, const double *oA, bool amc, Acc<double> &a) {
    const double r2 = Rx * Rx + Ry * Ry + Rz * Rz;
    // 1/|R|: the hardware estimate, then the second-order correction
    // (1 - e)^(-1/2) ~ 1 + e/2 + 3e^2/8 with e = 1 - r2 y0^2 (r2 is positive
    // and normal: distinct cells)
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e0 = __builtin_fma(-r2, y0 * y0, 1.0);
    const double g = __builtin_fma(y0 * e0, __builtin_fma(e0, 0.375, 0.5), y0);
    const double s = g * g, p1 = g * s, p2 = p1 * s, p3 = p2 * s;
    // quadrupole contractions
    const double qzz = -(q[0] + q[3]);
    const double QRx = q[0] * Rx + q[1] * Ry + q[2] * Rz;
    const double QRy = q[1] * Rx + q[3] * Ry + q[4] * Rz;
    const double QRz = q[2] * Rx + q[4] * Ry + qzz * Rz;
    const double RQR = Rx * QRx + Ry * QRy + Rz * QRz;
    // octupole contractions
    const double xx = Rx * Rx, yy = Ry * Ry, zz = Rz * Rz, xy = Rx * Ry, xz = Rx * Rz, yz = Ry * Rz;
    const double e = xx - zz, f = yy - zz, u = 2.0 * xy, v = 2.0 * xz, w = 2.0 * yz;
    double ORx, ORy, ORz;
    o7_rr(o, e, f, u, v, w, ORx, ORy, ORz);
    const double ORRR = Rx * ORx + Ry * ORy + Rz * ORz;
    double dx = 0.0, dy = 0.0, dz = 0.0, dw = 0.0;
    if (DIP) {
        dx = dp[0];
        dy = dp[1];
        dz = dp[2];
        dw = dx * Rx + dy * Ry + dz * Rz;
    }
    a.L0 = __builtin_fma(mB, g, a.L0);
    if (DIP) a.L0 = __builtin_fma(p1, dw, a.L0);
    a.A2 = __builtin_fma(p2, RQR, a.A2);
    a.A3 = __builtin_fma(p3, ORRR, a.A3);
    const double mp1 = mB * p1, k2 = 3.0 * p2, k3 = 7.5 * p3;
    const double mp1w = DIP ? __builtin_fma(k2, dw, mp1) : mp1;
    const double c = __builtin_fma(k3, RQR, mp1w);
    a.L1[0] = __builtin_fma(-k2, QRx, __builtin_fma(c, Rx, a.L1[0]));
    a.L1[1] = __builtin_fma(-k2, QRy, __builtin_fma(c, Ry, a.L1[1]));
    a.L1[2] = __builtin_fma(-k2, QRz, __builtin_fma(c, Rz, a.L1[2]));
    if (DIP) {
        a.L1[0] = __builtin_fma(-p1, dx, a.L1[0]);
        a.L1[1] = __builtin_fma(-p1, dy, a.L1[1]);
        a.L1[2] = __builtin_fma(-p1, dz, a.L1[2]);
    }
    if (!LEAF_TARGET) {
        const double m2 = mB * k2;
        const double e2 = DIP ? __builtin_fma(2.0 * k3, dw, m2) : m2;
        a.L2[0] = __builtin_fma(e2, xx, a.L2[0]);
        a.L2[1] = __builtin_fma(e2, xy, a.L2[1]);
        a.L2[2] = __builtin_fma(e2, xz, a.L2[2]);
        a.L2[3] = __builtin_fma(e2, yy, a.L2[3]);
        a.L2[4] = __builtin_fma(e2, yz, a.L2[4]);
        a.L2[5] = __builtin_fma(e2, zz, a.L2[5]);
        if (DIP) {
            const double fx = k2 * dx, fy = k2 * dy, fz = k2 * dz;
            a.L2[0] = __builtin_fma(-2.0 * fx, Rx, a.L2[0]);
            a.L2[1] = __builtin_fma(-fx, Ry, __builtin_fma(-fy, Rx, a.L2[1]));
            a.L2[2] = __builtin_fma(-fx, Rz, __builtin_fma(-fz, Rx, a.L2[2]));
            a.L2[3] = __builtin_fma(-2.0 * fy, Ry, a.L2[3]);
            a.L2[4] = __builtin_fma(-fy, Rz, __builtin_fma(-fz, Ry, a.L2[4]));
            a.L2[5] = __builtin_fma(-2.0 * fz, Rz, a.L2[5]);
        }
        const double m3 = mB * p3;
        const double m3x = m3 * Rx, m3y = m3 * Ry, m3z = m3 * Rz;
        a.L3[0] = __builtin_fma(m3x, xx, a.L3[0]);
        a.L3[1] = __builtin_fma(m3x, xy, a.L3[1]);
        a.L3[2] = __builtin_fma(m3x, xz, a.L3[2]);
        a.L3[3] = __builtin_fma(m3x, yy, a.L3[3]);
        a.L3[4] = __builtin_fma(m3x, yz, a.L3[4]);
        a.L3[5] = __builtin_fma(m3x, zz, a.L3[5]);
        a.L3[6] = __builtin_fma(m3y, yy, a.L3[6]);
        a.L3[7] = __builtin_fma(m3y, yz, a.L3[7]);
        a.L3[8] = __builtin_fma(m3z, yz, a.L3[8]);
        a.L3[9] = __builtin_fma(m3z, zz, a.L3[9]);
    }
    if (!DIP && amc) {
        // n:RR = O'_B:RR - mu O'_A:RR; a leaf target is a point mass at its
        // cell centre (no third moment), so there n:RR = O'_B:RR
        double nx = ORx, ny = ORy, nz = ORz, nR = ORRR;
        if (!LEAF_TARGET) {
            double ax, ay, az;
            o7_rr(oA, e, f, u, v, w, ax, ay, az);
            nx = __builtin_fma(-mu, ax, ORx);
            ny = __builtin_fma(-mu, ay, ORy);
            nz = __builtin_fma(-mu, az, ORz);
            nR = __builtin_fma(-mu, ax * Rx + ay * Ry + az * Rz, ORRR);
        }
        const double kR = (-17.5 * (p3 * s)) * nR;
        a.C[0] = __builtin_fma(kR, Rx, __builtin_fma(k3, nx, a.C[0]));
        a.C[1] = __builtin_fma(kR, Ry, __builtin_fma(k3, ny, a.C[1]));
        a.C[2] = __builtin_fma(kR, Rz, __builtin_fma(k3, nz, a.C[2]));
    }
}

// The pair routine of the per-wavefront multipole kernel and of the
// LDS-staged kernel's FP64 variants.
template <bool LEAF_TARGET, bool DIP, typename T>
__device__ inline void m2l_pair(double Rx, double Ry, double Rz, double mB, const double *q, const double *o,
                                const double *D, double mu, const double *oA, bool amc, Acc<T> &a) {
    static_assert(sizeof(T) == sizeof(double), "the FP64 pair routine");
    m2l_pair_f64<LEAF_TARGET, DIP>(Rx, Ry, Rz, mB, q, o, D, mu, oA, amc, a);
}

// The same pair in FP32 (mixed precision: the multipole bulk in FP32,
// accumulated in FP32), the correction's per-pair term accumulated in FP64.
// Same operations and constants as m2l_pair_f64, with 1/|R| from the
// hardware estimate alone (about 1 ulp in FP32).
template <bool LEAF_TARGET>
__device__ inline void m2l_pair_f32(float Rx, float Ry, float Rz, float mB, const float *q, const float *o, float mu,
                                    const float *oA, bool amc, Acc<float> &a) {
    const float r2 = Rx * Rx + Ry * Ry + Rz * Rz;
    const float g = __builtin_amdgcn_rsqf(r2);
    const float s = g * g, p1 = g * s, p2 = p1 * s, p3 = p2 * s;
    const float qzz = -(q[0] + q[3]);
    const float QRx = q[0] * Rx + q[1] * Ry + q[2] * Rz;
    const float QRy = q[1] * Rx + q[3] * Ry + q[4] * Rz;
    const float QRz = q[2] * Rx + q[4] * Ry + qzz * Rz;
    const float RQR = Rx * QRx + Ry * QRy + Rz * QRz;
    const float xx = Rx * Rx, yy = Ry * Ry, zz = Rz * Rz, xy = Rx * Ry, xz = Rx * Rz, yz = Ry * Rz;
    const float e = xx - zz, f = yy - zz, u = 2.0f * xy, v = 2.0f * xz, w = 2.0f * yz;
    float ORx, ORy, ORz;
    o7_rr(o, e, f, u, v, w, ORx, ORy, ORz);
    const float ORRR = Rx * ORx + Ry * ORy + Rz * ORz;
    a.L0 = __builtin_fmaf(mB, g, a.L0);
    a.A2 = __builtin_fmaf(p2, RQR, a.A2);
    a.A3 = __builtin_fmaf(p3, ORRR, a.A3);
    const float mp1 = mB * p1, k2 = 3.0f * p2, k3 = 7.5f * p3;
    const float c = __builtin_fmaf(k3, RQR, mp1);
    a.L1[0] = __builtin_fmaf(-k2, QRx, __builtin_fmaf(c, Rx, a.L1[0]));
    a.L1[1] = __builtin_fmaf(-k2, QRy, __builtin_fmaf(c, Ry, a.L1[1]));
    a.L1[2] = __builtin_fmaf(-k2, QRz, __builtin_fmaf(c, Rz, a.L1[2]));
    if (!LEAF_TARGET) {
        const float m2 = mB * k2;
        a.L2[0] = __builtin_fmaf(m2, xx, a.L2[0]);
        a.L2[1] = __builtin_fmaf(m2, xy, a.L2[1]);
        a.L2[2] = __builtin_fmaf(m2, xz, a.L2[2]);
        a.L2[3] = __builtin_fmaf(m2, yy, a.L2[3]);
        a.L2[4] = __builtin_fmaf(m2, yz, a.L2[4]);
        a.L2[5] = __builtin_fmaf(m2, zz, a.L2[5]);
        const float m3 = mB * p3;
        const float m3x = m3 * Rx, m3y = m3 * Ry, m3z = m3 * Rz;
        a.L3[0] = __builtin_fmaf(m3x, xx, a.L3[0]);
        a.L3[1] = __builtin_fmaf(m3x, xy, a.L3[1]);
        a.L3[2] = __builtin_fmaf(m3x, xz, a.L3[2]);
        a.L3[3] = __builtin_fmaf(m3x, yy, a.L3[3]);
        a.L3[4] = __builtin_fmaf(m3x, yz, a.L3[4]);
        a.L3[5] = __builtin_fmaf(m3x, zz, a.L3[5]);
        a.L3[6] = __builtin_fmaf(m3y, yy, a.L3[6]);
        a.L3[7] = __builtin_fmaf(m3y, yz, a.L3[7]);
        a.L3[8] = __builtin_fmaf(m3z, yz, a.L3[8]);
        a.L3[9] = __builtin_fmaf(m3z, zz, a.L3[9]);
    }
    if (amc) {
        float nx = ORx, ny = ORy, nz = ORz, nR = ORRR;
        if (!LEAF_TARGET) {
            float ax, ay, az;
            o7_rr(oA, e, f, u, v, w, ax, ay, az);
            nx = __builtin_fmaf(-mu, ax, ORx);
            ny = __builtin_fmaf(-mu, ay, ORy);
            nz = __builtin_fmaf(-mu, az, ORz);
            nR = __builtin_fmaf(-mu, ax * Rx + ay * Ry + az * Rz, ORRR);
        }
        const float kR = (-17.5f * (p3 * s)) * nR;
        a.C[0] += (double)__builtin_fmaf(kR, Rx, k3 * nx);
        a.C[1] += (double)__builtin_fmaf(kR, Ry, k3 * ny);
        a.C[2] += (double)__builtin_fmaf(kR, Rz, k3 * nz);
    }
}

template <bool LEAF_TARGET, bool DIP, typename T>
__device__ void m2l_item(const LevelDesc &ld, const TreeDesc &td, const StencilDev &st, const M2LItem item,
                         const int *s_nbr, int64_t *cnt_out, bool count) {
    const int lane = threadIdx.x;
    const int node = item.node, p = item.parity;
    const int s = (p << 6) | lane;
    int x, y, z;
    local_xyz(s, x, y, z);
    const size_t S = (size_t)ld.n_rec * kCells;
    const size_t ti = (size_t)node * kCells + s;
    const double zAx = ld.mp[ti], zAy = ld.mp[S + ti], zAz = ld.mp[2 * S + ti];
    const double mA = ld.mass[ti];
    double OA[10], oA[7];
#pragma unroll
    for (int k = 0; k < 10; ++k) OA[k] = DIP ? 0.0 : ld.mp[(9 + k) * S + ti];
    detrace_o(OA, oA);
    // the correction is applied to every lane (a uniform branch); targets
    // without mass drop it at the end
    const bool amc = !DIP && td.amc;
    const double imA = mA > 0.0 ? 1.0 / mA : 0.0;
    Acc<T> a;
    acc_zero(a);
    int cnt = 0;
    const int n_src_max = LEAF_TARGET ? ld.n_int : ld.n_rec;  // leaf <- leaf pairs are direct
    double Dp[3] = {0.0, 0.0, 0.0};
    double q5[5], o7[7];
    if (ld.level == 0) {
        // root: every other root cell is a candidate; multipole iff well separated
        const int parts = LEAF_TARGET ? 1 : ld.n_parts;
        const int k0 = kCells * item.chunk / parts, k1 = kCells * (item.chunk + 1) / parts;
        for (int k = k0; k < k1; ++k) {
            int bx, by, bz;
            local_xyz(k, bx, by, bz);
            const int dx = bx - x, dy = by - y, dz = bz - z;
            const double d2 = (double)(dx * dx + dy * dy + dz * dz);
            if (!(st.theta2 * d2 > 1.0) || 0 >= n_src_max) continue;
            const size_t si = k;  // root node 0
            const double mB = ld.mass[si];
            double Q[6], O[10];
#pragma unroll
            for (int q = 0; q < 6; ++q) Q[q] = ld.mp[(3 + q) * S + si];
#pragma unroll
            for (int q = 0; q < 10; ++q) O[q] = ld.mp[(9 + q) * S + si];
            if (DIP)
                for (int q = 0; q < 3; ++q) Dp[q] = ld.dip[q * S + si];
            detrace_q(Q, q5);
            detrace_o(O, o7);
            m2l_pair<LEAF_TARGET, DIP, T>(zAx - ld.mp[si], zAy - ld.mp[S + si], zAz - ld.mp[2 * S + si], mB, q5, o7,
                                          Dp, mB * imA, oA, amc, a);
            if (count) ++cnt;
        }
    } else {
        const int beg = st.m2l_beg[p], len = st.m2l_beg[p + 1] - beg;
        const int parts = LEAF_TARGET ? 1 : ld.n_parts;
        const int k0 = beg + len * item.chunk / parts, k1 = beg + len * (item.chunk + 1) / parts;
        // neighbour sub-grids holding sources for this target (uniform)
        int src_mask = 0;
        for (int b = 0; b < 27; ++b) src_mask |= (s_nbr[b] >= 0 && s_nbr[b] < n_src_max) ? (1 << b) : 0;
        src_mask = __builtin_amdgcn_readfirstlane(src_mask);
        for (int k = k0; k < k1; ++k) {
            if (!(st.m2l_touch[k] & src_mask)) continue;  // no lane reaches a source
            int dx, dy, dz;
            unpack(st.m2l[k], dx, dy, dz);
            const int sx = x + dx, sy = y + dy, sz = z + dz;
            const int nb = s_nbr[nbr_slot(sx, sy, sz)];
            if (nb < 0 || nb >= n_src_max) continue;
            const size_t si = (size_t)nb * kCells + store_idx(sx & 7, sy & 7, sz & 7);
            const double mB = ld.mass[si];
            double Q[6], O[10];
#pragma unroll
            for (int q = 0; q < 6; ++q) Q[q] = ld.mp[(3 + q) * S + si];
#pragma unroll
            for (int q = 0; q < 10; ++q) O[q] = ld.mp[(9 + q) * S + si];
            if (DIP)
                for (int q = 0; q < 3; ++q) Dp[q] = ld.dip[q * S + si];
            detrace_q(Q, q5);
            detrace_o(O, o7);
            m2l_pair<LEAF_TARGET, DIP, T>(zAx - ld.mp[si], zAy - ld.mp[S + si], zAz - ld.mp[2 * S + si], mB, q5, o7,
                                          Dp, mB * imA, oA, amc, a);
            if (count) ++cnt;
        }
    }
    acc_close<DIP>(a);
    if (!(mA > 0.0)) a.C[0] = a.C[1] = a.C[2] = 0.0;
    const double G = td.G;
    if (LEAF_TARGET) {
        const size_t LS = (size_t)(ld.n_rec - ld.n_int) * kCells;
        const size_t li = (size_t)(node - ld.n_int) * kCells + s;
        ld.lacc[li] = G * (double)a.L0;
        ld.lacc[LS + li] = G * (double)a.L1[0];
        ld.lacc[2 * LS + li] = G * (double)a.L1[1];
        ld.lacc[3 * LS + li] = G * (double)a.L1[2];
        ld.lacc[4 * LS + li] = G * a.C[0];
        ld.lacc[5 * LS + li] = G * a.C[1];
        ld.lacc[6 * LS + li] = G * a.C[2];
    } else {
        finish_l2_l3(a);
        const size_t IS = (size_t)ld.n_int * kCells;
        double *out = ld.loc + (size_t)item.chunk * kLoc * IS + (size_t)node * kCells + s;
        out[0] = G * (double)a.L0;
#pragma unroll
        for (int k = 0; k < 3; ++k) out[(1 + k) * IS] = G * (double)a.L1[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) out[(4 + k) * IS] = G * (double)a.L2[k];
#pragma unroll
        for (int k = 0; k < 10; ++k) out[(10 + k) * IS] = G * (double)a.L3[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) out[(20 + k) * IS] = G * a.C[k];
    }
    const int tot = wave_sum(cnt);
    if (lane == 0) *cnt_out = tot;
}

template <typename T, bool DIP>
__global__ __launch_bounds__(64) void k_m2l(const LevelDesc *__restrict__ L, const TreeDesc *__restrict__ TD,
                                            const M2LItem *__restrict__ items, int n_items, StencilDev st,
                                            int64_t *__restrict__ cnt, int count) {
    const int it = xcd_item(n_items);
    if (it >= n_items) return;
    const M2LItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const TreeDesc td = TD[ld.tree];
    __shared__ int s_nbr[27];
    if (threadIdx.x < 27) s_nbr[threadIdx.x] = ld.nbr[item.node * 27 + threadIdx.x];
    __syncthreads();
    if (item.node < ld.n_int)
        m2l_item<false, DIP, T>(ld, td, st, item, s_nbr, cnt + it, count != 0);
    else
        m2l_item<true, DIP, T>(ld, td, st, item, s_nbr, cnt + it, count != 0);
}


#ifndef OCTO_M2L_UNROLL
#define OCTO_M2L_UNROLL 1
#endif

// Multipole-to-local for all 512 cells of one interior node (LEAF: of one
// leaf node next to interior nodes of its level, whose cells take only L0, L1
// and the correction from the interior cells), with the source halo staged in
// LDS one parity class at a time: the cells of one parity class whose parent
// cells lie within 2 parent cells of the node form an 8x8x8 lattice, one cell
// per thread; each staged cell holds its mass, centre of mass and trace-free
// moments (16 FP64 values in 8 double2 planes, 68 KB: two work-groups per CU,
// four wavefronts per SIMD, at most 128 VGPRs; DIP: + the dipole, 10 planes,
// 85 KB, one work-group per CU).  Every wavefront (one target parity class)
// walks the part of its stencil whose sources fall in the staged class.
template <typename T, bool DIP, bool AMC, bool LEAF>
__global__ __launch_bounds__(512, DIP ? 2 : 4) void k_m2l_lds(const LevelDesc *__restrict__ L, const TreeDesc *__restrict__ TD,
                                                 const M2LItem *__restrict__ items, int n_items, StencilDev st,
                                                 int64_t *__restrict__ cnt_out, int count) {
    const int it = xcd_item(n_items);
    if (it >= n_items) return;
    const M2LItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const TreeDesc td = TD[ld.tree];
    const int node = item.node;
    // halo of one source class: 8x8x8 lattice, x-planes padded to 68 so that
    // the 8 lanes of each 16-byte LDS read phase (4 z x 2 x positions, see
    // the lane order below) hit distinct banks
    constexpr int NV = DIP ? 10 : 8;  // double2 planes per source cell
    constexpr int HY = kHaloY, HX = kHaloX, HN = kHaloN;
    // FP32 (mixed precision): 4 float4 planes per source cell, positions as
    // offsets from the cell centres (see stage_class)
    constexpr bool F32 = sizeof(T) == 4;
    static_assert(!(F32 && DIP), "the second-source multipole work runs in FP64");
    __shared__ __align__(16) unsigned char s_raw[(F32 ? 4 : NV) * HN * 16];
    auto s_src = reinterpret_cast<double2 (*)[HN]>(s_raw);
    auto s_src4 = reinterpret_cast<float4 (*)[HN]>(s_raw);
    __shared__ int s_nbr[27];
    __shared__ int s_cnt[8];
    const int tid = threadIdx.x;
    // wave-uniform (one wavefront per parity class): keep it in a scalar register
    const int p = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    if (tid < 27) s_nbr[tid] = ld.nbr[node * 27 + tid];
    // wavefront p holds target class p (parity-major storage: cell
    // p << 6 | i << 4 | j << 2 | k at lattice position (i, j, k)); lane
    // j << 4 | i << 2 | k, so that consecutive lanes run over k, then i
    const int s = (p << 6) | (((lane >> 2) & 3) << 4) | ((lane >> 4) << 2) | (lane & 3);
    int x, y, z;
    local_xyz(s, x, y, z);
    const size_t S = (size_t)ld.n_rec * kCells;
    const size_t ti = (size_t)node * kCells + s;
    const double zAx = ld.mp[ti], zAy = ld.mp[S + ti], zAz = ld.mp[2 * S + ti];
    const double mA = ld.mass[ti];
    double OA[10], oA[7];
#pragma unroll
    for (int k = 0; k < 10; ++k) OA[k] = DIP ? 0.0 : ld.mp[(9 + k) * S + ti];
    detrace_o(OA, oA);
    // the correction (a compile-time choice) is applied to every lane;
    // targets without mass drop it at the end
    constexpr bool amc = AMC && !DIP;
    const bool counting = count != 0;
    const double imA = mA > 0.0 ? 1.0 / mA : 0.0;
    // FP32: the target's offset from its cell centre and its moments in FP32;
    // the cells' centres are exact multiples of h - 1/2 (h a power of 2)
    const double hc = ld.h;
    const int gx0 = 8 * ld.coord[3 * node], gy0 = 8 * ld.coord[3 * node + 1], gz0 = 8 * ld.coord[3 * node + 2];
    float dAx = 0.f, dAy = 0.f, dAz = 0.f, oAf[7];
    if constexpr (F32) {
        dAx = (float)(zAx - centre(gx0 + x, hc));
        dAy = (float)(zAy - centre(gy0 + y, hc));
        dAz = (float)(zAz - centre(gz0 + z, hc));
#pragma unroll
        for (int k = 0; k < 7; ++k) oAf[k] = (float)oA[k];
    }
    const float imAf = (float)imA;
    Acc<T> a;
    acc_zero(a);
    int cnt = 0;
    __syncthreads();
    // this item's share of the source parity classes; its partial locals go
    // to slot `chunk` and are summed by the downward pass
    const int q0 = LEAF ? 0 : 8 * item.chunk / ld.n_parts, q1 = LEAF ? 8 : 8 * (item.chunk + 1) / ld.n_parts;
    // sources: interior nodes and record leaves of this level; a leaf target's only the interior ones
    const int n_src = LEAF ? ld.n_int : ld.n_rec;
    // the neighbour sub-grids that hold sources (uniform; all 27 inside the
    // domain's interior): source classes no entry of any target class reaches
    // are skipped; leaf targets also skip the entries that reach none of them
    int src_mask = 0, q_need = 0;
    for (int b = 0; b < 27; ++b) src_mask |= (s_nbr[b] >= 0 && s_nbr[b] < n_src) ? (1 << b) : 0;
    src_mask = __builtin_amdgcn_readfirstlane(src_mask);
    for (int q = 0; q < 8; ++q)
        for (int pp = 0; pp < 8; ++pp)
            if (st.m2l_src_any[pp * 8 + q] & src_mask) q_need |= 1 << q;
    // Source class q staged in LDS, one cell per thread: lattice index
    // i in [0,8) <-> local coordinate 2i - 4 + parity.  Cells that are not
    // sources get mass -0.0 (counted as absent, contributes exact zeros) and
    // a far-away centre.  The loads go through the global address space (a
    // generic load also counts as an LDS access); the other work-group on
    // the CU computes while this one stages.
    const GPtr<const double> gmass = gptr(ld.mass), gmp = gptr(ld.mp), gdip = gptr(ld.dip);
    const int cx = tid >> 6, cy = (tid >> 3) & 7, cz = tid & 7;
    auto stage_class = [&](int q) {
        const int sx = 2 * cx - 4 + (q >> 2), sy = 2 * cy - 4 + ((q >> 1) & 1), sz = 2 * cz - 4 + (q & 1);
        const int nb = s_nbr[nbr_slot(sx, sy, sz)];
        const bool present = nb >= 0 && nb < n_src;
        const size_t si = present ? (size_t)nb * kCells + store_idx(sx & 7, sy & 7, sz & 7) : 0;
        const int c = cx * HX + cy * HY + cz;
        if constexpr (F32) {
            // (m, dz_x, dz_y, dz_z) (q5_0..q5_3) (q5_4, o7_0..o7_2) (o7_3..o7_6),
            // dz the centre of mass minus the cell centre
            double a[10];
            if (present) {
                a[0] = gmass[si];
#pragma unroll
                for (int k = 0; k < 9; ++k) a[1 + k] = gmp[k * S + si];
                a[1] -= centre(gx0 + sx, hc);
                a[2] -= centre(gy0 + sy, hc);
                a[3] -= centre(gz0 + sz, hc);
            } else {
                a[0] = -0.0;
#pragma unroll
                for (int k = 1; k < 10; ++k) a[k] = 0.0;
            }
            double q5[5];
            detrace_q(&a[4], q5);
            s_src4[0][c] = make_float4((float)a[0], (float)a[1], (float)a[2], (float)a[3]);
            s_src4[1][c] = make_float4((float)q5[0], (float)q5[1], (float)q5[2], (float)q5[3]);
            __builtin_amdgcn_sched_barrier(0);
            double o[10], o7[7];
#pragma unroll
            for (int k = 0; k < 10; ++k) o[k] = present ? gmp[(9 + k) * S + si] : 0.0;
            detrace_o(o, o7);
            s_src4[2][c] = make_float4((float)q5[4], (float)o7[0], (float)o7[1], (float)o7[2]);
            s_src4[3][c] = make_float4((float)o7[3], (float)o7[4], (float)o7[5], (float)o7[6]);
            return;
        }
        // record planes: (m, zx) (zy, zz) (q5_0, q5_1) (q5_2, q5_3) (q5_4, o7_0)
        // (o7_1, o7_2) (o7_3, o7_4) (o7_5, o7_6) [(d_x, d_y) (d_z, 0)], staged in
        // two passes (mass, centre and second moments; then third moments and
        // dipole) so that few values are live next to the accumulators
        double a[10];
        if (present) {
            a[0] = gmass[si];
#pragma unroll
            for (int k = 0; k < 9; ++k) a[1 + k] = gmp[k * S + si];
        } else {
            a[0] = -0.0;
            a[1] = a[2] = a[3] = 1.0e3;
#pragma unroll
            for (int k = 4; k < 10; ++k) a[k] = 0.0;
        }
        double q5[5];
        detrace_q(&a[4], q5);
        s_src[0][c] = make_double2(a[0], a[1]);
        s_src[1][c] = make_double2(a[2], a[3]);
        s_src[2][c] = make_double2(q5[0], q5[1]);
        s_src[3][c] = make_double2(q5[2], q5[3]);
        __builtin_amdgcn_sched_barrier(0);
        double o[10], o7[7];
        if (present) {
#pragma unroll
            for (int k = 0; k < 10; ++k) o[k] = gmp[(9 + k) * S + si];
        } else {
#pragma unroll
            for (int k = 0; k < 10; ++k) o[k] = 0.0;
        }
        detrace_o(o, o7);
        s_src[4][c] = make_double2(q5[4], o7[0]);
        s_src[5][c] = make_double2(o7[1], o7[2]);
        s_src[6][c] = make_double2(o7[3], o7[4]);
        s_src[7][c] = make_double2(o7[5], o7[6]);
        if (DIP) {
            double d[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) d[k] = present ? gdip[k * S + si] : 0.0;
            s_src[8 % NV][c] = make_double2(d[0], d[1]);
            s_src[9 % NV][c] = make_double2(d[2], 0.0);
        }
    };
    // second source (one work-group per CU, registers to spare): the next
    // class's raw values are loaded into registers while this class is
    // walked, and stored after the barrier that ends the walk
    double pv[23];
    auto load_regs = [&](int q) {
        const int sx = 2 * cx - 4 + (q >> 2), sy = 2 * cy - 4 + ((q >> 1) & 1), sz = 2 * cz - 4 + (q & 1);
        const int nb = s_nbr[nbr_slot(sx, sy, sz)];
        if (nb >= 0 && nb < n_src) {
            const size_t si = (size_t)nb * kCells + store_idx(sx & 7, sy & 7, sz & 7);
            pv[0] = gmass[si];
#pragma unroll
            for (int k = 0; k < kRec; ++k) pv[1 + k] = gmp[k * S + si];
#pragma unroll
            for (int k = 0; k < 3; ++k) pv[20 + k] = gdip[k * S + si];
        } else {
            pv[0] = -0.0;
            pv[1] = pv[2] = pv[3] = 1.0e3;
#pragma unroll
            for (int k = 4; k < 23; ++k) pv[k] = 0.0;
        }
    };
    auto store_regs = [&]() {
        const int c = cx * HX + cy * HY + cz;
        double q5[5], o7[7];
        detrace_q(&pv[4], q5);
        detrace_o(&pv[10], o7);
        s_src[0][c] = make_double2(pv[0], pv[1]);
        s_src[1][c] = make_double2(pv[2], pv[3]);
        s_src[2][c] = make_double2(q5[0], q5[1]);
        s_src[3][c] = make_double2(q5[2], q5[3]);
        s_src[4][c] = make_double2(q5[4], o7[0]);
        s_src[5][c] = make_double2(o7[1], o7[2]);
        s_src[6][c] = make_double2(o7[3], o7[4]);
        s_src[7][c] = make_double2(o7[5], o7[6]);
        s_src[8 % NV][c] = make_double2(pv[20], pv[21]);
        s_src[9 % NV][c] = make_double2(pv[22], 0.0);
    };
    // the needed classes of this item's share, in order (uniform)
    auto next_class = [&](int q) {
        for (++q; q < q1; ++q)
            if ((q_need >> q) & 1) break;
        return q;
    };
    int q = next_class(q0 - 1);
    if constexpr (DIP) {
        if (q < q1) load_regs(q);
    }
    while (q < q1) {
        if constexpr (DIP)
            store_regs();
        else
            stage_class(q);
        __syncthreads();
        const int beg = st.m2l_src_beg[p * 9 + q], end = st.m2l_src_beg[p * 9 + q + 1];
        const int hb = (x >> 1) * HX + (y >> 1) * HY + (z >> 1);
        if (counting) {
            // pairs with a present source (absent sources carry -0.0), in a
            // pass of their own so that the multipole loop carries no count;
            // four independent counts keep several LDS reads in flight
            int c4[4] = {0, 0, 0, 0};
            int k = beg;
            for (; k + 3 < end; k += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    c4[u] += signbit(F32 ? (double)s_src4[0][hb + st.m2l_src[k + u]].x
                                         : s_src[0][hb + st.m2l_src[k + u]].x) ? 0 : 1;
            }
            for (; k < end; ++k)
                c4[0] += signbit(F32 ? (double)s_src4[0][hb + st.m2l_src[k]].x : s_src[0][hb + st.m2l_src[k]].x) ? 0 : 1;
            cnt += c4[0] + c4[1] + c4[2] + c4[3];
        }
        auto pair = [&](int k) {
            const int h = hb + st.m2l_src[k];  // the offset is uniform over the wavefront
            if constexpr (F32) {
                // R = z_A - z_B = (c_A - c_B) + (dz_A - dz_B), c_A - c_B = -h d exactly
                int dx, dy, dz;
                unpack(st.m2l_src_d[k], dx, dy, dz);
                const float4 e0 = s_src4[0][h], e1 = s_src4[1][h], e2 = s_src4[2][h], e3 = s_src4[3][h];
                const float qf[5] = {e1.x, e1.y, e1.z, e1.w, e2.x};
                const float of[7] = {e2.y, e2.z, e2.w, e3.x, e3.y, e3.z, e3.w};
                m2l_pair_f32<LEAF>((dAx - e0.y) + (float)(-hc * dx), (dAy - e0.z) + (float)(-hc * dy),
                                   (dAz - e0.w) + (float)(-hc * dz), e0.x, qf, of, e0.x * imAf, oAf, amc, a);
            } else {
                double r[2 * NV];
#pragma unroll
                for (int j = 0; j < NV; ++j) {
                    const double2 e = s_src[j][h];
                    r[2 * j] = e.x;
                    r[2 * j + 1] = e.y;
                }
                m2l_pair<LEAF, DIP, T>(zAx - r[1], zAy - r[2], zAz - r[3], r[0], &r[4], &r[9], &r[16 % (2 * NV)],
                                       r[0] * imA, oA, amc, a);
            }
        };
        if (LEAF) {
#pragma unroll OCTO_M2L_UNROLL
            for (int k = beg; k < end; ++k)
                if (st.m2l_src_touch[k] & src_mask) pair(k);  // uniform
        } else {
            // Entries that reach only absent sub-grids (domain boundary) cost
            // their full work: a per-entry skip breaks the interleaving and is
            // slower overall.
#pragma unroll OCTO_M2L_UNROLL
            for (int k = beg; k < end; ++k) pair(k);
        }
        const int qn = next_class(q);
        if constexpr (DIP) {
            if (qn < q1) load_regs(qn);
        }
        __syncthreads();
        q = qn;
    }
    acc_close<DIP>(a);
    if (!(mA > 0.0)) a.C[0] = a.C[1] = a.C[2] = 0.0;
    const double G = td.G;
    if (LEAF) {
        const size_t LS = (size_t)(ld.n_rec - ld.n_int) * kCells;
        const size_t li = (size_t)(node - ld.n_int) * kCells + s;
        ld.lacc[li] = G * (double)a.L0;
#pragma unroll
        for (int k = 0; k < 3; ++k) ld.lacc[(1 + k) * LS + li] = G * (double)a.L1[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) ld.lacc[(4 + k) * LS + li] = G * a.C[k];
    } else {
        finish_l2_l3(a);
        const size_t IS = (size_t)ld.n_int * kCells;
        double *out = ld.loc + (size_t)item.chunk * kLoc * IS + (size_t)node * kCells + s;
        out[0] = G * (double)a.L0;
#pragma unroll
        for (int k = 0; k < 3; ++k) out[(1 + k) * IS] = G * (double)a.L1[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) out[(4 + k) * IS] = G * (double)a.L2[k];
#pragma unroll
        for (int k = 0; k < 10; ++k) out[(10 + k) * IS] = G * (double)a.L3[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) out[(20 + k) * IS] = G * a.C[k];
    }
    const int tot = wave_sum(cnt);
    if (lane == 0) s_cnt[p] = tot;
    __syncthreads();
    if (tid == 0) {
        int64_t sum = 0;
        for (int k = 0; k < 8; ++k) sum += s_cnt[k];
        cnt_out[it] = sum;
    }
}

// ------------------------------------------------------------------ partial slots
// Sum the partial-locals slots of one level into slot 0, one thread per
// (cell, component) (coarse levels, where few cells have many slots).
__global__ __launch_bounds__(256) void k_sum_parts(const LevelDesc *__restrict__ L, const NodeItem *__restrict__ items,
                                                   int n_items) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_items * kCells * kLoc) return;
    const int it = i / (kCells * kLoc), r = i % (kCells * kLoc);
    const int c = r / kCells, cell = r % kCells;
    const NodeItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const size_t IS = (size_t)ld.n_int * kCells;
    const GPtr<double> dst = gptr(ld.loc) + c * IS + (size_t)item.node * kCells + cell;
    double v = *dst;
    for (int part = 1; part < ld.n_parts; ++part) v += dst[(size_t)part * kLoc * IS];
    *dst = v;
}

// ------------------------------------------------------------------ L2L
// v += the parent expansion P (kLoc values) shifted by d = (dx, dy, dz):
// Taylor shift of the order-3 local polynomial; the correction C is a
// uniform acceleration and is inherited.
__device__ inline void l2l_shift(const double *P, double dx, double dy, double dz, double *v) {
    const double *P2 = P + 4, *P3 = P + 10;
    double Tx, Ty, Tz;  // sum_bc L3_abc d_b d_c
    t3_uu(P3, dx, dy, dz, Tx, Ty, Tz);
    const double L2dx = P2[0] * dx + P2[1] * dy + P2[2] * dz;
    const double L2dy = P2[1] * dx + P2[3] * dy + P2[4] * dz;
    const double L2dz = P2[2] * dx + P2[4] * dy + P2[5] * dz;
    v[0] += P[0] + P[1] * dx + P[2] * dy + P[3] * dz + 0.5 * (L2dx * dx + L2dy * dy + L2dz * dz) +
            (Tx * dx + Ty * dy + Tz * dz) * (1.0 / 6.0);
    v[1] += P[1] + L2dx + 0.5 * Tx;
    v[2] += P[2] + L2dy + 0.5 * Ty;
    v[3] += P[3] + L2dz + 0.5 * Tz;
    // L2_ab += sum_c L3_abc d_c
    v[4] += P2[0] + P3[0] * dx + P3[1] * dy + P3[2] * dz;  // xx
    v[5] += P2[1] + P3[1] * dx + P3[3] * dy + P3[4] * dz;  // xy
    v[6] += P2[2] + P3[2] * dx + P3[4] * dy + P3[5] * dz;  // xz
    v[7] += P2[3] + P3[3] * dx + P3[6] * dy + P3[7] * dz;  // yy
    v[8] += P2[4] + P3[4] * dx + P3[7] * dy + P3[8] * dz;  // yz
    v[9] += P2[5] + P3[5] * dx + P3[8] * dy + P3[9] * dz;  // zz
#pragma unroll
    for (int c = 10; c < kLoc; ++c) v[c] += P[c];
}

// Interior cells with an interior child: sum the partial locals, then add the
// parent's expansion shifted to this cell's centre of mass.
__global__ __launch_bounds__(256) void k_l2l(const LevelDesc *__restrict__ L, const NodeItem *__restrict__ items,
                                             int n_items, int parts_done) {
    const int it = blockIdx.x >> 1;
    if (it >= n_items) return;
    const NodeItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const int node = item.node;
    const int s = ((blockIdx.x & 1) << 8) | threadIdx.x;
    const size_t IS = (size_t)ld.n_int * kCells;
    const size_t ci = (size_t)node * kCells + s;
    const GPtr<double> loc = gptr(ld.loc);
    double v[kLoc];
#pragma unroll
    for (int c = 0; c < kLoc; ++c) v[c] = loc[c * IS + ci];
    for (int part = 1; part < (parts_done ? 1 : ld.n_parts); ++part) {
        const GPtr<const double> src = loc + (size_t)part * kLoc * IS + ci;
#pragma unroll
        for (int c = 0; c < kLoc; ++c) v[c] += src[c * IS];
    }
    // the 64 parent cells over this node (a 4x4x4 block of the parent) staged
    // in LDS, component by component; lane q of every wavefront reads block
    // cell q
    __shared__ double s_par[3 + kLoc][64];
    const bool has_parent = ld.parent_ld >= 0;  // uniform
    if (has_parent) {
        const LevelDesc pl = L[ld.parent_ld];
        const int pn = gptr(ld.parent)[node];
        const GPtr<const int32_t> coord = gptr(ld.coord);
        const GPtr<const double> pmp = gptr(pl.mp), ploc = gptr(pl.loc);
        const int ox = 4 * (coord[3 * node] & 1), oy = 4 * (coord[3 * node + 1] & 1), oz = 4 * (coord[3 * node + 2] & 1);
        const size_t PIS = (size_t)pl.n_int * kCells, PRS = (size_t)pl.n_rec * kCells;
        for (int t = threadIdx.x; t < (3 + kLoc) * 64; t += 256) {
            const int c = t >> 6, j = t & 63;
            const size_t pi = (size_t)pn * kCells + store_idx(ox + (j >> 4), oy + ((j >> 2) & 3), oz + (j & 3));
            s_par[c][j] = c < 3 ? pmp[c * PRS + pi] : ploc[(c - 3) * PIS + pi];
        }
    }
    __syncthreads();
    if (has_parent) {
        int x, y, z;
        local_xyz(s, x, y, z);
        const int j = ((x >> 1) << 4) | ((y >> 1) << 2) | (z >> 1);
        const size_t RS = (size_t)ld.n_rec * kCells;
        const GPtr<const double> mp = gptr(ld.mp);
        const double dx = mp[ci] - s_par[0][j], dy = mp[RS + ci] - s_par[1][j], dz = mp[2 * RS + ci] - s_par[2][j];
        double P[kLoc];
#pragma unroll
        for (int c = 0; c < kLoc; ++c) P[c] = s_par[3 + c][j];
        l2l_shift(P, dx, dy, dz, v);
    }
#pragma unroll
    for (int c = 0; c < kLoc; ++c) loc[c * IS + ci] = v[c];
}

// ------------------------------------------------------------------ leaves
// Per leaf cell: direct point-mass sums over same-level leaf partners (the
// stencil of parents that are not well separated), over the children of
// nearby interior cells and over nearby coarser leaves (properly nested AMR
// boundaries), plus the parent's expansion shifted to the cell centre and
// the cell's own multipole-to-local sums; writes phi and g = -grad phi and
// per-wavefront sums for the net force and torque.
__device__ inline float rsqrt_t(float v) { return rsqrtf(v); }

template <typename T>
__device__ inline const T *weights(const StencilDev &st);
template <>
__device__ inline const double *weights<double>(const StencilDev &st) {
    return st.leaf_tab;
}
template <>
__device__ inline const float *weights<float>(const StencilDev &st) {
    return st.leaf_tab32;
}

// Near-field entries of one sign octant (SX, SY, SZ = +1 or -1: the signs of
// d, zero counted as +1, applied at compile time to the |d| weights):
// phi sum += m / |d|, g sums += m d / |d|^3, in blocks of 8 entries whose
// offsets and weight indices are fetched together (uniform over the
// wavefront: scalar loads), two accumulator sets.  Each octant's list is
// padded to whole blocks with zero-weight entries (weight row 0).  COUNT:
// absent partners carry mass -1 and are masked; real entries (w0 > 0) with
// a present partner are counted.
template <typename T, bool COUNT, int SX, int SY, int SZ>
__device__ inline void near_octant(const T *__restrict__ s_m, int base, const int32_t *__restrict__ off,
                                   const int32_t *__restrict__ widx, const T *__restrict__ tab, int beg, int end,
                                   T *acc, int &cnt) {
    auto add = [&](T m, const T *w, int set) {
        T mm = m;
        if (COUNT) {
            const bool ok = m >= (T)0;
            mm = ok ? m : (T)0;
            cnt += (ok && w[0] > (T)0) ? 1 : 0;
        }
        T *a = acc + 4 * set;
        a[0] += mm * w[0];
        if (SX > 0) a[1] += mm * w[1]; else a[1] -= mm * w[1];
        if (SY > 0) a[2] += mm * w[2]; else a[2] -= mm * w[2];
        if (SZ > 0) a[3] += mm * w[3]; else a[3] -= mm * w[3];
    };
    // weight rows addressed by an unsigned 32-bit byte offset from the table
    // base (stored for the FP64 table), so the scalar load takes it as its
    // offset operand
    auto row = [&](int wb) {
        return (const T *)((const char *)tab + (sizeof(T) == 8 ? (unsigned)wb : (unsigned)wb >> 1));
    };
    for (int k = beg; k < end; k += 8) {
        int o[8], wi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            o[u] = off[k + u];
            wi[u] = widx[k + u];
        }
        T m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) m[u] = s_m[base + o[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) add(m[u], row(wi[u]), u & 1);
    }
}
__device__ inline double rsqrt_t(double v) { return rsqrt(v); }


template <typename T>
__device__ inline const T *xl_weights(const StencilDev &st);
template <>
__device__ inline const double *xl_weights<double>(const StencilDev &st) {
    return st.xl_w;
}
template <>
__device__ inline const float *xl_weights<float>(const StencilDev &st) {
    return st.xl_w32;
}

// Cross-level pairs of the leaf cells of one node at AMR boundaries, direct
// point masses added to phi, g: interior cells of this level near a cell (X1:
// each of their 8 children, one level down) and leaves one level up near the
// cell's parent cell (X2).  Called by the whole work-group once the
// same-level sums have read s_m.  The separation of a target centre and a
// source point is (h/4) n (X1) or (h/2) n (X2) for an odd-integer vector n
// fixed per entry and child (X1) or per entry and target class (X2), so the
// weights 1/|n| and n/|n|^3 are table rows, the same for the whole
// wavefront.  X1 reads each source cell's 8 child masses as one 64-byte
// record (the level's cm array, filled by the leaf-mass pass); X2 stages the (4 + 2r)^3
// cells of the parent level around the node's 4^3 parent cells in s_m (r:
// the largest offset component; masses of leaves, -1 (COUNT) or 0
// elsewhere; x2v: this thread's cell, loaded by xl_x2_load).  s_nbr: the 27
// same-level neighbours of the node.
// The X2 source of thread tid (one cell of the block per thread), loaded
// together with the same-level halo and stored once the walk is done.
template <typename T, bool COUNT>
__device__ inline T xl_x2_load(const LevelDesc *__restrict__ L, const LevelDesc &ld, int flags, const StencilDev &st,
                               const int *s_pnbr, int node, int tid) {
    const int R = st.xl_reach, E = 4 + 2 * R;
    if (!(flags & kLeafX2) || ld.parent_ld < 0 || tid >= E * E * E) return (T)0;
    const LevelDesc pl = L[ld.parent_ld];
    const GPtr<const int32_t> coord = gptr(ld.coord);
    const int sx = 4 * (coord[3 * node] & 1) - R + tid / (E * E), sy = 4 * (coord[3 * node + 1] & 1) - R + (tid / E) % E,
              sz = 4 * (coord[3 * node + 2] & 1) - R + tid % E;
    const int nb = s_pnbr[nbr_slot(sx, sy, sz)];
    return nb >= pl.n_int ? (T)gptr(pl.mass)[(size_t)nb * kCells + store_idx(sx & 7, sy & 7, sz & 7)]
                          : (T)(COUNT ? -1 : 0);
}

template <typename T, bool COUNT>
__device__ inline void cross_level(const LevelDesc *__restrict__ L, const LevelDesc &ld, int flags,
                                   const StencilDev &st, T *s_m, const int *s_nbr, T x2v, int node,
                                   int tid, int x, int y, int z, int p, T &phi_t, T &gx_t, T &gy_t, T &gz_t,
                                   int &cnt) {
    const bool x1 = (flags & kLeafX1) != 0, x2 = (flags & kLeafX2) != 0 && ld.parent_ld >= 0;
    if (!x1 && !x2) return;  // uniform over the work-group
    const int R = st.xl_reach, E = 4 + 2 * R, E3 = E * E * E;
    const double h = ld.h;
    const T *W = xl_weights<T>(st);
    if (x2) {
        __syncthreads();  // the same-level sums are done with s_m
        if (tid < E3) s_m[tid] = x2v;
        __syncthreads();
    }
    if (x1) {
        // the child masses of this level's interior cells, 8 per cell in one
        // 64-byte record (the children next to a leaf are leaves, written by
        // the leaf-mass pass)
        const GPtr<const double> cmass = gptr(ld.cm);
        int int_mask = 0;  // neighbour sub-grids that are interior (uniform)
        for (int b = 0; b < 27; ++b) int_mask |= (s_nbr[b] >= 0 && s_nbr[b] < ld.n_int) ? (1 << b) : 0;
        int_mask = __builtin_amdgcn_readfirstlane(int_mask);
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int k = 0; k < st.n_xl; ++k) {
            // no lane of the class reaches an interior cell: skip (uniform)
            if (!(st.xl_touch[8 * k + p] & int_mask)) continue;
            int dx, dy, dz;
            unpack(st.xl_off[k], dx, dy, dz);
            const int sx = x + dx, sy = y + dy, sz = z + dz;
            const int nb = s_nbr[nbr_slot(sx, sy, sz)];
            const bool inner = nb >= 0 && nb < ld.n_int;
            const size_t at = inner ? ((size_t)nb * kCells + store_idx(sx & 7, sy & 7, sz & 7)) * 8 : 0;
            T m[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) m[c] = (T)cmass[at + c];
            const T *w = W + 64 * k;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const T mc = inner ? m[c] : (T)0;
                a0 += mc * w[4 * c];
                a1 += mc * w[4 * c + 1];
                a2 += mc * w[4 * c + 2];
                a3 += mc * w[4 * c + 3];
            }
            if (COUNT) cnt += inner ? 8 : 0;
        }
        // separation (h/4) n: phi -= m / |R|, g -= m R / |R|^3
        const T s1 = (T)(4.0 / h), s2 = (T)(16.0 / (h * h));
        phi_t -= a0 * s1;
        gx_t -= a1 * s2;
        gy_t -= a2 * s2;
        gz_t -= a3 * s2;
    }
    if (x2) {
        // the target's parent cell at (x >> 1, ...) in the node's 4^3 block;
        // its class among the parent level's cells decides the near list
        const int ix = x >> 1, iy = y >> 1, iz = z >> 1;
        const int pp = ((ix & 1) << 2) | ((iy & 1) << 1) | (iz & 1);
        const int base = ((ix + R) * E + (iy + R)) * E + (iz + R);
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int k = 0; k < st.n_xl; ++k) {
            int dx, dy, dz;
            unpack(st.xl_off[k], dx, dy, dz);
            const bool member = (st.xl_cls[k] >> pp) & 1;
            const T m = s_m[base + (dx * E + dy) * E + dz];
            T mm;
            if (COUNT) {
                const bool ok = member && m >= (T)0;
                mm = ok ? m : (T)0;
                cnt += ok ? 1 : 0;
            } else {
                mm = member ? m : (T)0;
            }
            const T *w = W + 64 * k + 32 + 4 * p;
            a0 += mm * w[0];
            a1 += mm * w[1];
            a2 += mm * w[2];
            a3 += mm * w[3];
        }
        // separation (h/2) n
        const T s1 = (T)(2.0 / h), s2 = (T)(4.0 / (h * h));
        phi_t -= a0 * s1;
        gx_t -= a1 * s2;
        gy_t -= a2 * s2;
        gz_t -= a3 * s2;
    }
}

// COUNT: count the evaluated pairs (solves that report statistics); without
// it absent partners are stored as zero masses and the loop is unmasked
// (identical results: adding 0 * w changes nothing).
template <typename T, bool COUNT>
__global__ __launch_bounds__(512) void k_near(const LevelDesc *__restrict__ L, const TreeDesc *__restrict__ TD,
                                              const LeafItem *__restrict__ items, int n_items, StencilDev st,
                                              int64_t *__restrict__ cnt_out) {
    const int it = xcd_item(n_items);
    if (it >= n_items) return;
    const LeafItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const TreeDesc td = TD[ld.tree];
    const int tid = threadIdx.x;
    // wave-uniform (one wavefront per parity class): keep it in a scalar register
    const int p = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int node = item.node;
    // masses of the 18^3 cells within 5 cells of this node, split by parity
    // class; -1 (COUNT) or 0 where the cell is not a leaf of this level
    // (absent or interior)
    __shared__ T s_m[kNearN];
    __shared__ int s_nbr[27];
    __shared__ int s_pnbr[27];
    if (tid < 27) {
        s_nbr[tid] = gptr(ld.nbr)[node * 27 + tid];
        if (ld.parent_ld >= 0) s_pnbr[tid] = gptr(L[ld.parent_ld].nbr)[gptr(ld.parent)[node] * 27 + tid];
    }
    __syncthreads();
    const T x2v = xl_x2_load<T, COUNT>(L, ld, item.flags, st, s_pnbr, node, tid);
    if (ld.level > 0) {
        // all 12 loads of this thread in flight before any store; the cell
        // indices come from the staging table (the same for every
        // work-group), not from per-thread integer arithmetic.  The neighbour
        // lookups (LDS) all come first and the mass loads go through the
        // global address space: a generic (flat) load also counts as an LDS
        // access, so each LDS wait would otherwise wait for the loads issued
        // before it and the 12 loads would run one after the other.
        constexpr int NU = kNearStage / 512;
        const GPtr<const int32_t> stage = gptr(st.near_stage);
        const GPtr<const double> mass = gptr(ld.mass);
        int e[NU], nb[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) e[u] = stage[u * 512 + tid];
#pragma unroll
        for (int u = 0; u < NU; ++u) nb[u] = e[u] >= 0 ? s_nbr[e[u] & 31] : -1;
        T v[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u)
            v[u] = nb[u] >= ld.n_int ? (T)mass[(size_t)nb[u] * kCells + ((e[u] >> 5) & 511)] : (T)(COUNT ? -1 : 0);
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if (e[u] >= 0) s_m[e[u] >> 14] = v[u];
    }
    __syncthreads();
    const int s = tid;  // parity-major storage: wavefront p holds class p
    int x, y, z;
    local_xyz(s, x, y, z);
    const double h = ld.h;
    int cnt = 0;

    // same-level leaf partners: phi = -(1/h) sum m w0, g = (1/h^2) sum m w1
    T sp = 0, sgx = 0, sgy = 0, sgz = 0;
    if (ld.level == 0) {
        for (int k = 0; k < kCells; ++k) {
            if (k == s) continue;
            int bx, by, bz;
            local_xyz(k, bx, by, bz);
            const T dx = (T)(bx - x), dy = (T)(by - y), dz = (T)(bz - z);
            const T w0 = rsqrt_t(dx * dx + dy * dy + dz * dz);
            const T m = (T)ld.mass[k];
            const T mw0 = m * w0, mw3 = mw0 * w0 * w0;
            sp += mw0;
            sgx += mw3 * dx;
            sgy += mw3 * dy;
            sgz += mw3 * dz;
            ++cnt;
        }
    } else {
        const int base = (x >> 1) * kNearX + (y >> 1) * kNearY + (z >> 1);
        const int *ob = st.leaf_oct_beg + p * 9;
        const T *tab = weights<T>(st);
        T acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        near_octant<T, COUNT, 1, 1, 1>(s_m, base, st.leaf_off, st.leaf_widx, tab, ob[0], ob[1], acc, cnt);
        near_octant<T, COUNT, 1, 1, -1>(s_m, base, st.leaf_off, st.leaf_widx, tab, ob[1], ob[2], acc, cnt);
        near_octant<T, COUNT, 1, -1, 1>(s_m, base, st.leaf_off, st.leaf_widx, tab, ob[2], ob[3], acc, cnt);
        near_octant<T, COUNT, 1, -1, -1>(s_m, base, st.leaf_off, st.leaf_widx, tab, ob[3], ob[4], acc, cnt);
        near_octant<T, COUNT, -1, 1, 1>(s_m, base, st.leaf_off, st.leaf_widx, tab, ob[4], ob[5], acc, cnt);
        near_octant<T, COUNT, -1, 1, -1>(s_m, base, st.leaf_off, st.leaf_widx, tab, ob[5], ob[6], acc, cnt);
        near_octant<T, COUNT, -1, -1, 1>(s_m, base, st.leaf_off, st.leaf_widx, tab, ob[6], ob[7], acc, cnt);
        near_octant<T, COUNT, -1, -1, -1>(s_m, base, st.leaf_off, st.leaf_widx, tab, ob[7], ob[8], acc, cnt);
        sp = acc[0] + acc[4];
        sgx = acc[1] + acc[5];
        sgy = acc[2] + acc[6];
        sgz = acc[3] + acc[7];
    }
    const T ih = (T)(1.0 / h);
    T phi_t = -sp * ih;
    T gx_t = sgx * ih * ih, gy_t = sgy * ih * ih, gz_t = sgz * ih * ih;

    cross_level<T, COUNT>(L, ld, item.flags, st, s_m, s_nbr, x2v, node, tid, x, y, z, p, phi_t, gx_t, gy_t, gz_t,
                          cnt);
    // direct sums enter the FP64 accumulation: phi and g of this cell's
    // direct partners, G applied
    const size_t NS = (size_t)(ld.n_nodes - ld.n_int) * kCells;
    const size_t ni = (size_t)(node - ld.n_int) * kCells + s;
    const GPtr<double> nf = gptr(ld.nf);
    nf[ni] = td.G * (double)phi_t;
    nf[NS + ni] = td.G * (double)gx_t;
    nf[2 * NS + ni] = td.G * (double)gy_t;
    nf[3 * NS + ni] = td.G * (double)gz_t;
    if (COUNT) {
        const int tot = wave_sum(cnt);
        __shared__ int s_c[8];
        if (lane == 0) s_c[p] = tot;
        __syncthreads();
        if (tid == 0) {
            int64_t c = 0;
            for (int w = 0; w < 8; ++w) c += s_c[w];
            cnt_out[it] = c;
        }
    }
}

// Leaf cells, after the downward pass: the direct sums from the near-field
// kernel, the cell's own multipole-to-local sums (record leaves) and the
// parent's expansion shifted to the cell centre give phi and g = -grad phi,
// written in the caller's layout, plus per-node partial sums of the
// diagnostics.  SRC (second-source solve): the potential only.
template <bool SRC>
__global__ __launch_bounds__(512) void k_l2p(const LevelDesc *__restrict__ L, const TreeDesc *__restrict__ TD,
                                             const LeafItem *__restrict__ items, int n_items,
                                             double *__restrict__ stat, int stats) {
    const int it = xcd_item(n_items);
    if (it >= n_items) return;
    const LeafItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const TreeDesc td = TD[ld.tree];
    const int tid = threadIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int node = item.node;
    const int s = tid;
    int x, y, z;
    local_xyz(s, x, y, z);
    const double h = ld.h;
    // the level's arrays as global pointers: their loads then count only
    // against the vector-memory counter, so waits for the scalar loads of
    // the descriptors do not also wait for them
    const GPtr<const int32_t> coord = gptr(ld.coord);
    const GPtr<const double> nf = gptr(ld.nf), lacc = gptr(ld.lacc);
    const int gx0 = 8 * coord[3 * node], gy0 = 8 * coord[3 * node + 1], gz0 = 8 * coord[3 * node + 2];
    const double cx = centre(gx0 + x, h), cy = centre(gy0 + y, h), cz = centre(gz0 + z, h);
    const size_t NS = (size_t)(ld.n_nodes - ld.n_int) * kCells;
    const size_t ni = (size_t)(node - ld.n_int) * kCells + s;
    double phi = nf[ni];
    double gx = nf[NS + ni], gy = nf[2 * NS + ni], gz = nf[3 * NS + ni];

    // own multipole-to-local sums (record leaves)
    if (item.flags & kLeafLacc) {
        const size_t LS = (size_t)(ld.n_rec - ld.n_int) * kCells;
        const size_t li = (size_t)(node - ld.n_int) * kCells + s;
        phi += lacc[li];
        gx += -lacc[LS + li] + lacc[4 * LS + li];
        gy += -lacc[2 * LS + li] + lacc[5 * LS + li];
        gz += -lacc[3 * LS + li] + lacc[6 * LS + li];
    }
    // parent expansion shifted to the cell centre, evaluated there.  The 64
    // parent cells over this node (a 4x4x4 block of the parent) are staged in
    // LDS by the whole work-group, component by component, then each is read
    // by the 8 cells under it (lane q of every wavefront reads block cell q)
    __shared__ double s_par[3 + kLoc][64];
    const bool has_parent = ld.parent_ld >= 0;  // uniform
    if (has_parent) {
        const LevelDesc pl = L[ld.parent_ld];
        const int pn = gptr(ld.parent)[node];
        const int ox = 4 * (coord[3 * node] & 1), oy = 4 * (coord[3 * node + 1] & 1), oz = 4 * (coord[3 * node + 2] & 1);
        const GPtr<const int32_t> pcoord = gptr(pl.coord);
        const GPtr<const double> pmp = gptr(pl.mp), ploc = gptr(pl.loc);
        const size_t PIS = (size_t)pl.n_int * kCells, PRS = (size_t)pl.n_rec * kCells;
        // a deferred parent: the sum of its partial slots (in slot order), then
        // the grandparent's finished expansions over the block (2x2x2 cells)
        // shifted in.  The grandparent values are loaded first, by threads
        // that stage only three parent values, so that both loads overlap
        const int parts = (item.flags & kLeafDefer) ? pl.n_parts : 1;
        const bool gp_stage = (item.flags & kLeafDefer) && pl.parent_ld >= 0;  // uniform
        constexpr int kGpFirst = 512 - (3 + kLoc) * 8;
        __shared__ double s_gp[3 + kLoc][8];
        double gpv = 0.0;
        if (gp_stage && tid >= kGpFirst) {
            const LevelDesc gl = L[pl.parent_ld];
            const int gn = gptr(pl.parent)[pn];
            const int gx = 4 * (pcoord[3 * pn] & 1) + (ox >> 1), gy = 4 * (pcoord[3 * pn + 1] & 1) + (oy >> 1),
                      gz = 4 * (pcoord[3 * pn + 2] & 1) + (oz >> 1);
            const int c = (tid - kGpFirst) >> 3, k = (tid - kGpFirst) & 7;
            const size_t gi = (size_t)gn * kCells + store_idx(gx + (k >> 2), gy + ((k >> 1) & 1), gz + (k & 1));
            gpv = c < 3 ? gptr(gl.mp)[c * (size_t)gl.n_rec * kCells + gi]
                        : gptr(gl.loc)[(c - 3) * (size_t)gl.n_int * kCells + gi];
        }
        for (int t = tid; t < (3 + kLoc) * 64; t += 512) {
            const int c = t >> 6, j = t & 63;
            const size_t pi = (size_t)pn * kCells + store_idx(ox + (j >> 4), oy + ((j >> 2) & 3), oz + (j & 3));
            double v;
            if (c < 3) {
                v = pmp[c * PRS + pi];
            } else {
                v = ploc[(c - 3) * PIS + pi];
                for (int part = 1; part < parts; ++part) v += ploc[((size_t)part * kLoc + c - 3) * PIS + pi];
            }
            s_par[c][j] = v;
        }
        if (gp_stage) {
            // the L2L shift of the 64 block cells, by one wavefront
            if (tid >= kGpFirst) s_gp[(tid - kGpFirst) >> 3][(tid - kGpFirst) & 7] = gpv;
            __syncthreads();
            if (tid < 64) {
                const int j = tid, k = ((j >> 5) << 2) | (((j >> 3) & 1) << 1) | ((j >> 1) & 1);
                double P[kLoc], v[kLoc];
#pragma unroll
                for (int c = 0; c < kLoc; ++c) {
                    P[c] = s_gp[3 + c][k];
                    v[c] = s_par[3 + c][j];
                }
                l2l_shift(P, s_par[0][j] - s_gp[0][k], s_par[1][j] - s_gp[1][k], s_par[2][j] - s_gp[2][k], v);
#pragma unroll
                for (int c = 0; c < kLoc; ++c) s_par[3 + c][j] = v[c];
            }
        }
    }
    __syncthreads();
    if (has_parent) {
        const int j = ((x >> 1) << 4) | ((y >> 1) << 2) | (z >> 1);
        const double dx = cx - s_par[0][j], dy = cy - s_par[1][j], dz = cz - s_par[2][j];
        double P[kLoc];
#pragma unroll
        for (int c = 0; c < kLoc; ++c) P[c] = s_par[3 + c][j];
        const double *P2 = P + 4, *P3 = P + 10;
        double Tx, Ty, Tz;
        t3_uu(P3, dx, dy, dz, Tx, Ty, Tz);
        const double L2dx = P2[0] * dx + P2[1] * dy + P2[2] * dz;
        const double L2dy = P2[1] * dx + P2[3] * dy + P2[4] * dz;
        const double L2dz = P2[2] * dx + P2[4] * dy + P2[5] * dz;
        phi += P[0] + P[1] * dx + P[2] * dy + P[3] * dz + 0.5 * (L2dx * dx + L2dy * dy + L2dz * dz) +
               (Tx * dx + Ty * dy + Tz * dz) * (1.0 / 6.0);
        gx += -(P[1] + L2dx + 0.5 * Tx) + P[20];
        gy += -(P[2] + L2dy + 0.5 * Ty) + P[21];
        gz += -(P[3] + L2dz + 0.5 * Tz) + P[22];
    }
    const int64_t o = gptr(ld.out_base)[node] + x * td.sx + y * td.sy + z * td.sz;
    gptr(td.phi)[o] = phi;
    if (SRC) return;
    const GPtr<double> g = gptr(td.g);
    g[o] = gx;
    g[td.n_leaf_cells + o] = gy;
    g[2 * td.n_leaf_cells + o] = gz;
    if (!stats) return;  // uniform

    // per-wavefront partial sums for the diagnostics; |g| and |x| only set
    // the scales that the net force and torque are divided by, so the
    // hardware reciprocal square root is accurate enough for them
    const double m = gptr(ld.mass)[(size_t)node * kCells + s];
    const double fx = m * gx, fy = m * gy, fz = m * gz;
    const double g2 = gx * gx + gy * gy + gz * gz, x2 = cx * cx + cy * cy + cz * cz;
    const double gn = g2 > 0.0 ? g2 * __builtin_amdgcn_rsq(g2) : 0.0;
    const double xn = x2 > 0.0 ? x2 * __builtin_amdgcn_rsq(x2) : 0.0;
    double v[kStat] = {m, fx, fy, fz, cy * fz - cz * fy, cz * fx - cx * fz, cx * fy - cy * fx, m * gn, xn * m * gn};
#pragma unroll
    for (int k = 0; k < kStat; ++k) v[k] = wave_total_lane63(v[k]);
    __shared__ double s_v[8][kStat];
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < kStat; ++k) s_v[p][k] = v[k];
    }
    __syncthreads();
    if (tid < kStat) {
        double acc = 0.0;
        for (int w = 0; w < 8; ++w) acc += s_v[w][tid];
        stat[(size_t)it * kStat + tid] = acc;
    }
}

// ------------------------------------------------------------------ stats
// Per tree, kStatBlocks work-groups each sum a contiguous share of the
// per-node partials (and of the pair counts) in a fixed order and write
// them to a slot of their own; the last work-group of the tree to finish (a
// counter, reset by that work-group for the next solve) adds the slots in
// slot order.  The same inputs give the same bits however the work-groups
// are scheduled.
constexpr int kStatT = 256;

__global__ __launch_bounds__(kStatT) void k_stats(const int32_t *__restrict__ leaf_beg,
                                                  const int32_t *__restrict__ m2l_beg,
                                                  const int32_t *__restrict__ m2ln_beg,
                                                  const int32_t *__restrict__ m2lf_beg, int n_m2l, int n_m2ln,
                                                  const double *__restrict__ stat,
                                                  const int64_t *__restrict__ leaf_cnt,
                                                  const int64_t *__restrict__ m2l_cnt, double *__restrict__ part,
                                                  int *__restrict__ done, double *__restrict__ out, int counts) {
    const int t = blockIdx.x / kStatBlocks, b = blockIdx.x % kStatBlocks;
    auto share = [&](const int32_t *beg, int &i0, int &i1) {
        const int lo = beg[t], n = beg[t + 1] - lo, per = (n + kStatBlocks - 1) / kStatBlocks;
        i0 = lo + min(n, b * per);
        i1 = lo + min(n, (b + 1) * per);
    };
    __shared__ double sh[kStat][kStatT / 64];
    __shared__ long long shc[3][kStatT / 64];
    __shared__ int s_last;
    double acc[kStat];
#pragma unroll
    for (int k = 0; k < kStat; ++k) acc[k] = 0.0;
    long long c_m2l = 0, c_dir = 0, c_lds = 0;
    int i0, i1;
    share(leaf_beg, i0, i1);
    for (int i = i0 + threadIdx.x; i < i1; i += kStatT) {
#pragma unroll
        for (int k = 0; k < kStat; ++k) acc[k] += stat[(size_t)i * kStat + k];
        if (counts) c_dir += leaf_cnt[i];
    }
    // pair counts only when the kernels counted them (zero otherwise)
    if (counts) {
        share(m2l_beg, i0, i1);
        for (int i = i0 + threadIdx.x; i < i1; i += kStatT) c_m2l += m2l_cnt[i];
        share(m2ln_beg, i0, i1);
        for (int i = i0 + threadIdx.x; i < i1; i += kStatT) c_lds += m2l_cnt[n_m2l + i];
        share(m2lf_beg, i0, i1);
        for (int i = i0 + threadIdx.x; i < i1; i += kStatT) c_m2l += m2l_cnt[n_m2l + n_m2ln + i];
    }
#pragma unroll
    for (int k = 0; k < kStat; ++k) acc[k] = wave_sum(acc[k]);
    c_m2l = wave_sum(c_m2l);
    c_dir = wave_sum(c_dir);
    c_lds = wave_sum(c_lds);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < kStat; ++k) sh[k][wv] = acc[k];
        shc[0][wv] = c_m2l + c_lds;
        shc[1][wv] = c_dir;
        shc[2][wv] = c_lds;
    }
    __syncthreads();
    // this work-group's slot: 9 sums, multipole pairs, direct pairs, LDS-kernel pairs
    double *slot = part + ((size_t)t * kStatBlocks + b) * 12;
    if (threadIdx.x < kStat) {
        double v = 0.0;
        for (int w = 0; w < kStatT / 64; ++w) v += sh[threadIdx.x][w];
        slot[threadIdx.x] = v;
    } else if (threadIdx.x < kStat + 3) {
        long long v = 0;
        for (int w = 0; w < kStatT / 64; ++w) v += shc[threadIdx.x - kStat][w];
        slot[threadIdx.x] = (double)v;  // exact below 2^53
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&done[t], 1) == kStatBlocks - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (threadIdx.x < 12) {
        const double *ps = part + (size_t)t * kStatBlocks * 12;
        double v = 0.0;
        for (int j = 0; j < kStatBlocks; ++j) v += ps[j * 12 + threadIdx.x];
        out[t * 12 + threadIdx.x] = v;
    }
    if (threadIdx.x == 0) done[t] = 0;  // ready for the next solve
}

// ------------------------------------------------------------------ launch

void launch_leaf_records(const Plan &p, hipStream_t s) {
    if (p.n_p2m)
        hipLaunchKernelGGL(k_leaf_records, dim3(2 * p.n_p2m), dim3(256), 0, s, p.d_levels, p.d_p2m, p.n_p2m);
    check_hip(hipGetLastError(), "kernel launch");
}

void launch_solve(const Plan &p, const StencilDev &st, const LaunchOpts &o, hipStream_t s) {
    auto mark = [&](int i) {
        if (o.phase_events) check_hip(hipEventRecord(o.phase_events[i], s), "phase event");
    };
    const bool src = o.source;
    // mixed precision: the LDS-staged multipole kernels in FP32 (the
    // per-wavefront kernel of the root and level 1 and the second source stay FP64)
    const bool f32 = o.precision == OCTO_MIXED;
    // net force and torque reductions: with statistics (which also count
    // pairs) or on their own; never for the second source
    const bool reduce = !src && (o.count || o.reduce);
    mark(0);
    if (p.n_p2m)
        hipLaunchKernelGGL(k_p2m<false>, dim3(2 * p.n_p2m), dim3(256), 0, s, p.d_levels, p.d_trees, p.d_p2m, p.n_p2m);
    if (src) {
        // the density's centres of mass first, then the second source's
        // leaf cells (which replace the leaf masses for the near field)
        for (int l = p.n_levels_max - 1; l >= 0; --l) {
            const int n = p.n_interior[l];
            if (n)
                hipLaunchKernelGGL(k_m2m, dim3(2 * n), dim3(256), 0, s, p.d_levels, p.d_interior + p.interior_off[l],
                                   n);
        }
        if (p.n_p2m)
            hipLaunchKernelGGL(k_p2m<true>, dim3(2 * p.n_p2m), dim3(256), 0, s, p.d_levels, p.d_trees, p.d_p2m,
                               p.n_p2m);
    }
    mark(1);
    // the near field needs only the leaf masses: it runs on its own stream,
    // concurrently with the upward pass, the multipole phase and the downward pass
    const bool near_fork = o.aux_near && p.n_leaf;
    hipStream_t sn = near_fork ? o.aux_near : s;
    if (near_fork) {
        check_hip(hipEventRecord(o.fork_near, s), "fork");
        check_hip(hipStreamWaitEvent(o.aux_near, o.fork_near, 0), "fork");
    }
    if (p.n_leaf) {
        const bool count = o.count && !src;
        const int grid = ((p.n_leaf + kXcd - 1) / kXcd) * kXcd;
        auto near = o.precision == OCTO_MIXED ? (count ? k_near<float, true> : k_near<float, false>)
                                              : (count ? k_near<double, true> : k_near<double, false>);
        hipLaunchKernelGGL(near, dim3(grid), dim3(512), 0, sn, p.d_levels, p.d_trees, p.d_leaf, p.n_leaf, st,
                           p.d_leaf_cnt);
    }
    if (near_fork) check_hip(hipEventRecord(o.join_near, o.aux_near), "join");
    mark(2);
    // With a second stream, the levels below the shallowest LDS-staged level
    // (the root and other sparse levels) go there: their upward pass, their
    // per-wavefront multipole work (with the leaf targets of every level) and
    // their downward pass depend only on each other and on the deeper
    // levels' upward pass, so they overlap the LDS-staged kernel.  M2L at a
    // level reads only that level's multipoles.
    const bool fork = o.aux && (p.n_m2l || p.n_m2l_leaf) && p.n_m2l_nodes;
    const int lsplit = fork ? std::min(p.lds_min_level, p.n_levels_max) : 0;
    auto upward = [&](int l, hipStream_t q) {
        const int n = p.n_interior[l];
        if (n)
            hipLaunchKernelGGL(src ? k_m2m_src : k_m2m, dim3(2 * n), dim3(256), 0, q, p.d_levels,
                               p.d_interior + p.interior_off[l], n);
    };
    // the L2L pass covers the interior nodes with an interior child; the
    // others are finished by their leaves in k_l2p
    auto downward = [&](int l, hipStream_t q) {
        const int n = p.n_l2l[l];
        if (!n) return;
        // levels with few nodes sum their many partial slots in a separate wide pass
        const bool wide = p.sum_parts_level.size() > (size_t)l && p.sum_parts_level[l];
        if (wide)
            hipLaunchKernelGGL(k_sum_parts, dim3((n * kCells * kLoc + 255) / 256), dim3(256), 0, q, p.d_levels,
                               p.d_l2l + p.l2l_off[l], n);
        hipLaunchKernelGGL(k_l2l, dim3(2 * n), dim3(256), 0, q, p.d_levels, p.d_l2l + p.l2l_off[l], n, wide ? 1 : 0);
    };
    // the LDS-staged multipole kernel (dense levels, on the main stream)
    auto lds_levels = [&]() {
        if (!p.n_m2l_nodes) return;
        const int grid = ((p.n_m2l_nodes + kXcd - 1) / kXcd) * kXcd;
        auto k = src ? k_m2l_lds<double, true, false, false>
                     : f32 ? (o.amc ? k_m2l_lds<float, false, true, false> : k_m2l_lds<float, false, false, false>)
                           : (o.amc ? k_m2l_lds<double, false, true, false> : k_m2l_lds<double, false, false, false>);
        hipLaunchKernelGGL(k, dim3(grid), dim3(512), 0, s, p.d_levels, p.d_trees, p.d_m2l_nodes, p.n_m2l_nodes, st,
                           p.d_m2l_cnt + p.n_m2l, o.count ? 1 : 0);
    };
    for (int l = p.n_levels_max - 1; l >= lsplit; --l) upward(l, s);
    hipStream_t sm = fork ? o.aux : s;
    if (fork) {
        check_hip(hipEventRecord(o.fork, s), "fork");
        check_hip(hipStreamWaitEvent(o.aux, o.fork, 0), "fork");
        // the near field overlaps the upward pass (a chain of small
        // launches) but not the LDS-staged kernel: run together, the two
        // fill the same CUs and each slows the other by more than it gains
        if (near_fork) check_hip(hipStreamWaitEvent(s, o.join_near, 0), "join");
        // issued before the other stream's work, so that a graph replay
        // dispatches it as soon as the dense levels' upward pass is done
        lds_levels();
    }
    for (int l = lsplit - 1; l >= 0; --l) upward(l, sm);
    mark(3);
    if (p.n_m2l) {
        const int grid = ((p.n_m2l + kXcd - 1) / kXcd) * kXcd;
        auto k = src ? k_m2l<double, true> : k_m2l<double, false>;
        hipLaunchKernelGGL(k, dim3(grid), dim3(64), 0, sm, p.d_levels, p.d_trees, p.d_m2l, p.n_m2l, st, p.d_m2l_cnt,
                           o.count ? 1 : 0);
    }
    if (p.n_m2l_leaf) {
        const int grid = ((p.n_m2l_leaf + kXcd - 1) / kXcd) * kXcd;
        auto k = src ? k_m2l_lds<double, true, false, true>
                     : f32 ? (o.amc ? k_m2l_lds<float, false, true, true> : k_m2l_lds<float, false, false, true>)
                           : (o.amc ? k_m2l_lds<double, false, true, true> : k_m2l_lds<double, false, false, true>);
        hipLaunchKernelGGL(k, dim3(grid), dim3(512), 0, sm, p.d_levels, p.d_trees, p.d_m2l_leaf, p.n_m2l_leaf, st,
                           p.d_m2l_cnt + p.n_m2l + p.n_m2l_nodes, o.count ? 1 : 0);
    }
    for (int l = 0; l < lsplit; ++l) downward(l, sm);
    if (fork) check_hip(hipEventRecord(o.join, o.aux), "join");
    mark(8);
    if (!fork) lds_levels();
    if (fork) check_hip(hipStreamWaitEvent(s, o.join, 0), "join");
    mark(4);
    for (int l = lsplit; l < p.n_levels_max; ++l) downward(l, s);
    mark(5);
    if (near_fork) check_hip(hipStreamWaitEvent(s, o.join_near, 0), "join");
    if (p.n_leaf) {
        const int grid = ((p.n_leaf + kXcd - 1) / kXcd) * kXcd;
        hipLaunchKernelGGL(src ? k_l2p<true> : k_l2p<false>, dim3(grid), dim3(512), 0, s, p.d_levels, p.d_trees,
                           p.d_leaf, p.n_leaf, p.d_stat, reduce ? 1 : 0);
    }
    mark(6);
    // the reductions only when they are asked for (a solve with statistics)
    if (reduce)
        hipLaunchKernelGGL(k_stats, dim3(p.n_trees * kStatBlocks), dim3(kStatT), 0, s, p.d_tree_leaf_beg,
                           p.d_tree_m2l_beg, p.d_tree_m2ln_beg, p.d_tree_m2lf_beg, p.n_m2l, p.n_m2l_nodes, p.d_stat,
                           p.d_leaf_cnt, p.d_m2l_cnt, p.d_stat_part, p.d_stat_done, p.d_out, o.count ? 1 : 0);
    mark(7);
    check_hip(hipGetLastError(), "kernel launch");
}

}  // namespace octo

namespace octo {

// ------------------------------------------------------------------ coupling
// Gravity source terms of the hydrodynamic update (Sec. 2.3, source vector S
// with the right-hand sides of the momentum and energy equations, Sec. 2.1):
//   S_s = rho g + Omega x s
//   S_E = 1/2 (phi drho/dt - rho dphi/dt) + rho Omega . (x x g)
// for every leaf cell (x = cell centre), arrays in the caller's layout.
__global__ __launch_bounds__(512) void k_sources(const LevelDesc *__restrict__ L, const TreeDesc *__restrict__ TD,
                                                 const LeafItem *__restrict__ items, int n_items, double ox, double oy,
                                                 double oz, const double *__restrict__ rho, const double *__restrict__ sv,
                                                 const double *__restrict__ phi, const double *__restrict__ g,
                                                 const double *__restrict__ drho, const double *__restrict__ dphi,
                                                 double *__restrict__ src_s, double *__restrict__ src_e) {
    const int it = blockIdx.x;
    if (it >= n_items) return;
    const LeafItem item = items[it];
    const LevelDesc ld = L[item.ld];
    const TreeDesc td = TD[ld.tree];
    const int node = item.node;
    const int s = threadIdx.x;
    int x, y, z;
    local_xyz(s, x, y, z);
    const double h = ld.h;
    const double cx = centre(8 * ld.coord[3 * node] + x, h), cy = centre(8 * ld.coord[3 * node + 1] + y, h),
                 cz = centre(8 * ld.coord[3 * node + 2] + z, h);
    const int64_t n = td.n_leaf_cells;
    const int64_t o = ld.out_base[node] + x * td.sx + y * td.sy + z * td.sz;
    const double r = rho[o], gx = g[o], gy = g[n + o], gz = g[2 * n + o];
    const double sx = sv[o], sy = sv[n + o], sz = sv[2 * n + o];
    src_s[o] = r * gx + (oy * sz - oz * sy);
    src_s[n + o] = r * gy + (oz * sx - ox * sz);
    src_s[2 * n + o] = r * gz + (ox * sy - oy * sx);
    const double dr = drho ? drho[o] : 0.0, dp = dphi ? dphi[o] : 0.0;
    // x cross g
    const double xgx = cy * gz - cz * gy, xgy = cz * gx - cx * gz, xgz = cx * gy - cy * gx;
    src_e[o] = 0.5 * (phi[o] * dr - r * dp) + r * (ox * xgx + oy * xgy + oz * xgz);
}

// Energy update after a potential solve (Sec. 2.3): E += 1/2 rho (phi_before - phi_after).
__global__ __launch_bounds__(256) void k_energy_update(int64_t n, const double *__restrict__ rho,
                                                       const double *__restrict__ before,
                                                       const double *__restrict__ after, double *__restrict__ E) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) E[i] += 0.5 * rho[i] * (before[i] - after[i]);
}

void launch_sources(const Plan &p, const double omega[3], const double *rho, const double *s, const double *phi,
                    const double *g, const double *drho, const double *dphi, double *src_s, double *src_e,
                    hipStream_t st) {
    if (!p.n_leaf) return;
    hipLaunchKernelGGL(k_sources, dim3(p.n_leaf), dim3(512), 0, st, p.d_levels, p.d_trees, p.d_leaf, p.n_leaf,
                       omega[0], omega[1], omega[2], rho, s, phi, g, drho, dphi, src_s, src_e);
    check_hip(hipGetLastError(), "sources launch");
}

void launch_energy_update(int64_t n, const double *rho, const double *before, const double *after, double *E,
                          hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_energy_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, rho, before, after,
                       E);
    check_hip(hipGetLastError(), "energy update launch");
}

}  // namespace octo
