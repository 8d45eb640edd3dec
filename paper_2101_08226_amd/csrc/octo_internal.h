// Internal data layout shared by the host runtime and the HIP kernels.
//
// Device layout of one tree (all arrays in HBM, owned by the tree):
//  * Per level l, nodes are numbered [0, n_int) interior, [n_int, n_rec) leaf
//    nodes that touch an interior node of their level ("record leaves": they
//    take part in multipole interactions), [n_rec, n_nodes) other leaves;
//    each group is in Morton order.
//  * Cells inside a node are stored parity-major: storage index
//    s = parity * 64 + q with parity = (x&1)<<2 | (y&1)<<1 | (z&1) and
//    q = (x>>1)<<4 | (y>>1)<<2 | (z>>1) for local cell (x, y, z).  One
//    64-lane wavefront holds one parity class of one node, so all its lanes
//    share one interaction stencil.
//  * Per-cell fields are structure-of-arrays: component c of node n cell s
//    lives at base[c * (count * 512) + n * 512 + s].
#pragma once

#include <cstdint>

#include "octo.h"

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#define __device__
#endif
#endif

namespace octo {

constexpr int kCells = 512;
constexpr int kMaxLevel = 9;  // deepest supported level (finest cells 1/4096)

// multipole record of a cell (besides its mass): centre of mass (3), raw
// second moments (6: xx xy xz yy yz zz), raw third moments (10: xxx xxy xxz
// xyy xyz xzz yyy yyz yzz zzz), all about the centre of mass
constexpr int kRec = 19;
// local expansion of an interior cell: L0, L1 (3), L2 (6), L3 (10) and the
// angular-momentum correction C (3), same packing as the moments
constexpr int kLoc = 23;
// multipole-to-local accumulators of a record leaf: L0, L1 (3), C (3)
constexpr int kLacc = 7;
// per leaf work item partial sums: M, F (3), T (3), S_F, S_T
constexpr int kStat = 9;
// work-groups per tree of the final statistics reduction (each a slot of 12
// values: the 9 sums and 3 pair counts)
constexpr int kStatBlocks = 16;
// halo of one source parity class in the LDS-staged multipole kernel: an
// 8x8x8 lattice (the class's cells whose parent cells lie within 2 parent
// cells of the node), x-planes padded to 68 (index ix * kHaloX + iy * kHaloY + iz)
constexpr int kHaloY = 8, kHaloX = 68, kHaloN = 8 * kHaloX;
// leaf-mass halo of the near-field kernel: the 18^3 cells within 5 cells of a
// node, split by parity class into eight 9x9x9 lattices (lattice index
// (ux>>1, uy>>1, uz>>1) of halo cell u = local + 5 at ix * kNearX + iy * kNearY
// + iz; rows and planes padded so that the lanes of a wavefront, one parity
// class of targets, read distinct LDS banks), class q at q * kNearQ
constexpr int kNearY = 12, kNearX = 112, kNearQ = 9 * kNearX, kNearN = 8 * kNearQ;
// staging of that halo by the 512 threads of a near-field work-group: entry
// u * 512 + t (u < 12) names the halo cell c = u * 512 + t (ux = c / 324,
// uy = (c / 18) % 18, uz = c % 18, local coordinate u - 5) as
// slot | store << 5 | dest << 14: the neighbour slot of the sub-grid holding
// it, its storage index there and its index in the parity-split halo; -1
// past the 18^3 cells
constexpr int kNearStage = 12 * 512;
// near-field weights by |d| pattern: index (|dx| * 6 + |dy|) * 6 + |dz|
constexpr int kNearTab = 216;


struct LevelDesc {
    int32_t level, n_nodes, n_int, n_rec;
    int32_t parent_ld;  // descriptor of level - 1 of the same tree (-1 at the root)
    int32_t child_ld;   // descriptor of level + 1 (-1 if the level has no interior nodes)
    int32_t n_parts;    // slots of partial interior locals (chunked multipole work)
    int32_t tree;       // index of the tree descriptor
    double h;           // cell width
    const int32_t *nbr;       // n_nodes * 27: same-level neighbour node (dx,dy,dz) at (dx+1)*9+(dy+1)*3+dz+1, -1 = none
    const int32_t *child;     // n_int * 8: child node at level + 1, child (cx,cy,cz) at cx*4+cy*2+cz
    const int32_t *parent;    // n_nodes: parent node at level - 1 (-1 at the root)
    const int32_t *coord;     // n_nodes * 3: node index at this level
    const int64_t *out_base;  // n_nodes: caller-layout offset of local cell (0,0,0) (leaf nodes), -1 otherwise
    double *mass;             // n_nodes * 512
    double *mp;               // kRec * n_rec * 512
    double *loc;              // n_parts * kLoc * n_int * 512 (slot-major)
    double *lacc;             // kLacc * (n_rec - n_int) * 512
    double *nf;               // 4 * (n_nodes - n_int) * 512: direct-sum phi, g of leaf cells
    double *dip;              // 3 * n_rec * 512: dipole of a second source about the density's centres
    double *cm;               // n_int * 512 * 8: per interior cell (storage index s), the masses of its 8 child
                              // cells (a*4 + b*2 + c for child (2x+a, 2y+b, 2z+c)), written by the leaf-mass pass
                              // where the child node is a leaf (the only children the cross-level pairs read)
};

struct TreeDesc {
    const double *rho;  // caller layout
    double *phi;        // caller layout, set per solve
    double *g;          // 3 x n_leaf_cells, set per solve (NULL in second-source solves)
    const double *src;  // second source (a density rate), caller layout, set per second-source solve
    int64_t n_leaf_cells;
    int64_t sx, sy, sz;  // caller-layout strides of local cell (x, y, z)
    double G;
    int32_t amc;
    int32_t pad;
};

// one wavefront of multipole-to-local work: 64 target cells of one parity
// class of one node, stencil entries [len*chunk/n_parts, len*(chunk+1)/n_parts)
struct M2LItem {
    int32_t ld, node, parity, chunk;
};

// kLeafDefer: the leaf's parent has no interior child, so no L2L pass
// finishes the parent's expansion: the leaf kernel sums the parent's partial
// slots and shifts the grandparent's expansion in itself (each parent cell is
// under exactly one leaf's 4x4x4 block, so no cell is done twice)
enum : int32_t { kLeafX1 = 1, kLeafX2 = 2, kLeafLacc = 4, kLeafDefer = 8 };

// one work-group of leaf work: the 512 cells of one leaf node (8 wavefronts,
// one per parity class)
struct LeafItem {
    int32_t ld, node, pad, flags;
};

struct NodeItem {
    int32_t ld, node;
};

// interaction stencils for one opening angle (levels >= 1), per parity class;
// offsets packed as (dx & 255) | (dy & 255) << 8 | (dz & 255) << 16
struct StencilDev {
    const int32_t *m2l;    // well separated, parents not
    const int32_t *m2l_touch;   // per m2l entry: mask of the 27 neighbour sub-grids it reaches from the class
    const int32_t *leaf;   // m2l followed by near (packed offsets)
    // near-field entries per target class, grouped by the sign octant o of d
    // (o = (dx<0)<<2 | (dy<0)<<1 | (dz<0)): offset into the parity-split halo
    // relative to the target's lattice position, and weight-table row as a
    // byte offset into the FP64 table (half of it into the FP32 table)
    const int32_t *leaf_off;
    const int32_t *leaf_widx;
    const double *leaf_tab;   // kNearTab x 4: 1/|d|, |dx|/|d|^3, |dy|/|d|^3, |dz|/|d|^3
    const float *leaf_tab32;  // the same weights rounded to FP32 (mixed precision)
    const int32_t *near_stage;  // kNearStage staging entries of the near-field halo
    const int32_t *m2l_src;  // m2l entries regrouped by source parity class, as halo offsets: the entry
                             // (dx,dy,dz) of target class p reads halo index (x>>1, y>>1, z>>1) + offset
    // cross-level near partners (AMR boundaries): the offsets d (not well
    // separated, parents not, d != 0) of all target classes once each; per
    // entry the mask of the classes whose near list holds it, per (entry,
    // class) the neighbour sub-grids it reaches, and 16 weight rows of 4
    // (1/|n|, n/|n|^3): rows 0-7 for the children of a same-level interior
    // cell, rows 8-15 per target class for a cell one level up
    const int32_t *xl_off;
    const int32_t *xl_cls;
    const int32_t *xl_touch;
    const double *xl_w;
    const float *xl_w32;
    int32_t n_xl;
    int32_t xl_reach;  // largest |component| of an entry (the staged blocks' margin)
    int32_t m2l_beg[9];
    int32_t leaf_beg[9];
    int32_t leaf_oct_beg[73];  // target class p, octant o: [p*9+o, p*9+o+1)
    int32_t m2l_src_beg[73];  // target class p, source class q: [p*9+q, p*9+q+1)
    const int32_t *m2l_src_touch;  // per m2l_src entry: mask of the 27 neighbour sub-grids it reaches
    const int32_t *m2l_src_d;      // per m2l_src entry: the offset d (source cell minus target cell), packed
    int32_t m2l_src_any[64];       // target class p, source class q: union of the group's touch masks
    double theta2;
};

// Device tree layout (csrc/layout.hip, csrc/layout_ops.h).  Node presence
// lives in one dense cell per node position and level (Morton index within the
// level): 0 absent, kMarkLeaf / kMarkInt while the node set is built and
// classified, then kIdxBase + the node's index in its level.
constexpr int32_t kMarkLeaf = 1, kMarkInt = 2, kIdxBase = 16;
// error codes, lowest first wins (then the lowest item)
enum : uint64_t { kLayLevel = 1, kLayIndex = 2, kLayDup = 3, kLayInside = 4, kLayGap = 5, kLayNest = 6, kLayFull = 7 };
// sort key: level << 29 | class << 27 | Morton index (class 0 interior, 1
// record leaf, 2 other leaf); padding sorts last
constexpr uint64_t kKeyPad = (1ull << 33) - 1;
constexpr int kKeyBits = 33;
// control words: [0] nodes appended, [1] first error (code << 32 | item),
// [2 + 3 * level + class] first sorted position of (level, class)
constexpr int kCtlWords = 2 + 3 * (kMaxLevel + 1);

struct LayK {
    const octo_leaf *leaf;
    int64_t n_leaf;
    int32_t *cell;                  // dense presence cells of levels [0, levels)
    int64_t goff[kMaxLevel + 2];    // first cell of each level: sum of 8^k, k < l
    int32_t levels;
    int64_t cap;                    // node capacity
    unsigned long long *ctl;        // kCtlWords control words
    uint64_t *node_lm;              // per appended node: level << 32 | Morton index
    int32_t *node_leaf;             // its position in the leaf list, -1 for interior
    uint64_t *key;                  // sort input (key, slot)
    int32_t *val;
    const uint64_t *skey;           // sort output
    const int32_t *sval;
    int32_t *info;                  // per slot: kLeaf* flags of a leaf; 1 if an interior node has an interior child
    int32_t *host;                  // per sorted position: info, parent index (downloaded)
};

// the tables of a laid-out tree, per level
struct LayTables {
    int32_t *nbr[kMaxLevel + 1], *child[kMaxLevel + 1], *parent[kMaxLevel + 1], *coord[kMaxLevel + 1];
    int64_t *out_base[kMaxLevel + 1];
    int32_t n_int[kMaxLevel + 1];
};

__host__ __device__ inline int32_t pack_off(int dx, int dy, int dz) {
    return (dx & 255) | ((dy & 255) << 8) | ((dz & 255) << 16);
}

}  // namespace octo
