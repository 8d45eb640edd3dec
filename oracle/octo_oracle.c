/*
 * octo_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU reference for the gravity solve of
 * Octo-Tiger (Marcello et al., "Octo-Tiger: a new, 3D hydrodynamic code for
 * stellar mergers that uses HPX parallelisation", Sec. 2.2 "Gravity Update and
 * the Angular Momentum Correction").  It exists to check the HIP library; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the HIP library.
 *
 * What it computes (each step follows the paper's order):
 *   - the octree of 8x8x8 sub-grids (Sec. 2.4): a node is a leaf or has 8
 *     children; neighbouring sub-grids differ by at most one level;
 *   - leaf cells are point masses m = rho h^3 at their centres (the cell-mass
 *     definition used by the diagnostics of Sec. 4);
 *   - upward pass: multipoles of a cell are composed from its 8 children
 *     (Sec. 2.2); moments are raw moments about the cell's centre of mass, up
 *     to third order;
 *   - interactions: two cells at the same level whose opening angle
 *     dx/|x_A - x_B| is below theta are well separated; they interact through
 *     the multipole expansion when they are well separated and their parents
 *     are not (Sec. 2.2, opening criterion).  The candidate pairs are produced
 *     by the recursion that definition implies, starting from all pairs of
 *     distinct root cells;  pairs that are never well separated are summed
 *     directly as point masses;
 *   - the angular-momentum correction (Sec. 2.2): the third-order part of
 *     the pair force is applied as a uniform acceleration of each cell, which
 *     removes the pair torque while keeping the pair forces equal and
 *     opposite;
 *   - downward pass: the expansion of each child is derived from its parent's
 *     (Sec. 2.2); leaves evaluate phi and g = -grad phi (Sec. 2.1);
 *   - the time derivative of the potential (Sec. 2.1: the energy equation's
 *     gravity source uses it, computed by the same FMM with the density rate
 *     as source): a second, signed source is expanded about the density's
 *     centres of mass (so it has a dipole) and goes through the same
 *     interaction lists; orc_solve_source.
 *
 * Readings where the paper is silent are listed in the design notes; the ones
 * this file relies on: expansion order p = 3; expansion centres are centres of
 * mass; the opening test uses geometric cell centres, evaluated on integer
 * offsets as (theta*theta)*|d|^2 > 1 in IEEE double; no self-interaction.
 *
 * Everything is FP64, plain loops, full (unpacked) tensors.  Parallelism is
 * an OpenMP loop over root cells; each task writes only into its own subtree,
 * so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMAXLEV 9 /* levels 0..8 */

typedef struct {
    double m, z[3];
    double M1[3]; /* dipole about z: zero for the density (z is its centre of
                     mass), nonzero for a second source expanded about the
                     density's centres */
    double M2[3][3];
    double M3[3][3][3];
    double L0, L1[3], L2[3][3], L3[3][3][3], C[3];
} ocell;

typedef struct {
    int level, n[3];
    int leaf;
    int parent;
    int child[8]; /* child (cx,cy,cz) at index (cx*2+cy)*2+cz */
    int out;      /* position in the caller's leaf list, -1 if interior */
    ocell *cell;  /* 512 cells, local (ix,iy,iz) at (ix*8+iy)*8+iz */
    double *rho;  /* leaves only */
    unsigned char *mark;
} onode;

typedef struct {
    int64_t m2l, direct, m2l_leaf_leaf;
} ocount;

typedef struct {
    int nlev; /* deepest level + 1 */
    int nnodes, cap;
    onode *nodes;
    int *lut[OMAXLEV]; /* per level: (2^l)^3 node ids or -1 */
    int nleaves;
    int *leaf_node;
    ocount last; /* interaction counts of the last solve (marked targets only) */
    int centres; /* expansion centres of interior cells: 0 centre of mass (the
                    default); 1 geometric centre, dipole kept; 2 geometric
                    centre, dipole dropped (see orc_tree_set_centres) */
    char err[256];
} otree;

/* Kernel of the interaction: phi(x) = -G sum_j m_j K(x - y_j).
 * mode 0: Newtonian K = 1/|R|.
 * mode 1: a cubic polynomial K(R) = sum c_b R^b over the 20 monomials of
 *         degree <= 3, enumerated bx = 0..3, by = 0..3-bx, bz = 0..3-bx-by.
 *         A third-order expansion of such a kernel is exact, which lets tests
 *         compare the whole tree machinery with brute force. */
typedef struct {
    int mode;
    double coef[20];
    int pw[20][3];
    double theta2; /* theta*theta */
    double G;
    int amc;
    ocount *cnt; /* counts of the current task */
} oparams;

/* ------------------------------------------------------------------------ */
/* Tree                                                                      */
/* ------------------------------------------------------------------------ */

static int lut_size(int l) { return 1 << (3 * l); }

static int lut_index(int l, int x, int y, int z) { return (x << (2 * l)) | (y << l) | z; }

static int lut_get(const otree *t, int l, int x, int y, int z) {
    if (l < 0 || l >= OMAXLEV || !t->lut[l]) return -1;
    int m = 1 << l;
    if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m) return -1;
    return t->lut[l][lut_index(l, x, y, z)];
}

static int new_node(otree *t, int l, int x, int y, int z, int leaf) {
    if (t->nnodes == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 64;
        t->nodes = (onode *)realloc(t->nodes, sizeof(onode) * (size_t)t->cap);
    }
    int id = t->nnodes++;
    onode *n = &t->nodes[id];
    memset(n, 0, sizeof(*n));
    n->level = l;
    n->n[0] = x;
    n->n[1] = y;
    n->n[2] = z;
    n->leaf = leaf;
    n->parent = -1;
    n->out = -1;
    for (int c = 0; c < 8; ++c) n->child[c] = -1;
    if (!t->lut[l]) {
        t->lut[l] = (int *)malloc(sizeof(int) * (size_t)lut_size(l));
        for (int i = 0; i < lut_size(l); ++i) t->lut[l][i] = -1;
    }
    t->lut[l][lut_index(l, x, y, z)] = id;
    return id;
}

void orc_tree_free(otree *t) {
    if (!t) return;
    for (int i = 0; i < t->nnodes; ++i) {
        free(t->nodes[i].cell);
        free(t->nodes[i].rho);
        free(t->nodes[i].mark);
    }
    free(t->nodes);
    for (int l = 0; l < OMAXLEV; ++l) free(t->lut[l]);
    free(t->leaf_node);
    free(t);
}

const char *orc_tree_error(const otree *t) { return t ? t->err : "null tree"; }

/* Build the tree from a leaf list (level, nx, ny, nz per leaf) and the density
 * of each leaf's 512 cells.  Returns NULL-free tree with err[0] != 0 on failure
 * (caller checks orc_tree_error). */
otree *orc_tree_new(int nleaves, const int32_t *leaves, const double *rho) {
    otree *t = (otree *)calloc(1, sizeof(otree));
    if (nleaves <= 0) {
        snprintf(t->err, sizeof t->err, "no leaves");
        return t;
    }
    t->nleaves = nleaves;
    t->leaf_node = (int *)malloc(sizeof(int) * (size_t)nleaves);
    /* 1. leaves */
    for (int k = 0; k < nleaves; ++k) {
        int l = leaves[4 * k], x = leaves[4 * k + 1], y = leaves[4 * k + 2], z = leaves[4 * k + 3];
        if (l < 0 || l >= OMAXLEV) {
            snprintf(t->err, sizeof t->err, "leaf %d: level %d out of range", k, l);
            return t;
        }
        int m = 1 << l;
        if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m) {
            snprintf(t->err, sizeof t->err, "leaf %d: index out of range", k);
            return t;
        }
        if (lut_get(t, l, x, y, z) >= 0) {
            snprintf(t->err, sizeof t->err, "leaf %d: duplicate", k);
            return t;
        }
        int id = new_node(t, l, x, y, z, 1);
        t->nodes[id].out = k;
        t->leaf_node[k] = id;
        if (t->nlev < l + 1) t->nlev = l + 1;
    }
    /* 2. ancestors */
    for (int k = 0; k < nleaves; ++k) {
        int id = t->leaf_node[k];
        int l = t->nodes[id].level, x = t->nodes[id].n[0], y = t->nodes[id].n[1], z = t->nodes[id].n[2];
        for (int pl = l - 1; pl >= 0; --pl) {
            x >>= 1;
            y >>= 1;
            z >>= 1;
            int p = lut_get(t, pl, x, y, z);
            if (p >= 0) {
                if (t->nodes[p].leaf) {
                    snprintf(t->err, sizeof t->err, "leaf %d overlaps a coarser leaf", k);
                    return t;
                }
                break; /* the rest of the chain exists already */
            }
            new_node(t, pl, x, y, z, 0);
        }
    }
    if (lut_get(t, 0, 0, 0, 0) < 0) {
        snprintf(t->err, sizeof t->err, "no root");
        return t;
    }
    /* 3. every interior node has all 8 children */
    for (int id = 0; id < t->nnodes; ++id) {
        onode *n = &t->nodes[id];
        if (n->leaf) continue;
        for (int c = 0; c < 8; ++c) {
            int cx = 2 * n->n[0] + (c >> 2), cy = 2 * n->n[1] + ((c >> 1) & 1), cz = 2 * n->n[2] + (c & 1);
            int ch = lut_get(t, n->level + 1, cx, cy, cz);
            if (ch < 0) {
                snprintf(t->err, sizeof t->err, "gap: node (%d,%d,%d,%d) misses child %d", n->level, n->n[0],
                         n->n[1], n->n[2], c);
                return t;
            }
            t->nodes[id].child[c] = ch;
            t->nodes[ch].parent = id;
        }
    }
    /* 4. proper nesting across faces, edges and corners: a leaf may not touch
     *    an interior node one level finer. */
    for (int k = 0; k < nleaves; ++k) {
        const onode *n = &t->nodes[t->leaf_node[k]];
        int l = n->level;
        for (int o = 0; o < 27; ++o) {
            int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
            if (!ox && !oy && !oz) continue;
            int px = n->n[0] + ox, py = n->n[1] + oy, pz = n->n[2] + oz;
            int m = 1 << l;
            if (px < 0 || py < 0 || pz < 0 || px >= m || py >= m || pz >= m) continue;
            int p = lut_get(t, l, px, py, pz);
            if (p < 0 || t->nodes[p].leaf) continue;
            for (int c = 0; c < 8; ++c) {
                int bx = c >> 2, by = (c >> 1) & 1, bz = c & 1;
                /* child of p touches n iff on each axis it sits on the side facing n */
                if ((ox == 1 && bx != 0) || (ox == -1 && bx != 1)) continue;
                if ((oy == 1 && by != 0) || (oy == -1 && by != 1)) continue;
                if ((oz == 1 && bz != 0) || (oz == -1 && bz != 1)) continue;
                if (!t->nodes[t->nodes[p].child[c]].leaf) {
                    snprintf(t->err, sizeof t->err, "2:1 balance violated next to leaf %d", k);
                    return t;
                }
            }
        }
    }
    /* 5. storage and density */
    for (int id = 0; id < t->nnodes; ++id) {
        onode *n = &t->nodes[id];
        n->cell = (ocell *)calloc(512, sizeof(ocell));
        n->mark = (unsigned char *)calloc(512, 1);
        if (n->leaf) {
            n->rho = (double *)malloc(512 * sizeof(double));
            const double *src = rho + (size_t)n->out * 512;
            for (int i = 0; i < 512; ++i) {
                if (!(src[i] >= 0.0) || !isfinite(src[i])) {
                    snprintf(t->err, sizeof t->err, "leaf %d: density not finite and >= 0", n->out);
                    return t;
                }
                n->rho[i] = src[i];
            }
        }
    }
    return t;
}

int orc_tree_nlev(const otree *t) { return t->nlev; }

/* Ordered-pair counts of the last solve: multipole interactions, direct
 * point-mass pairs, and the multipole interactions between two leaf cells
 * (which reduce to point-mass pairs). */
void orc_last_counts(const otree *t, int64_t *out) {
    out[0] = t->last.m2l;
    out[1] = t->last.direct;
    out[2] = t->last.m2l_leaf_leaf;
}
int orc_tree_nnodes(const otree *t) { return t->nnodes; }

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

static double cell_width(int l) { return 1.0 / (double)(8 << l); }

/* centre of cell with global index i at level l: -1/2 + (i + 1/2) h */
static double centre(int l, int i) { return (i + 0.5) * cell_width(l) - 0.5; }

typedef struct {
    int node, loc;
} cref;

static ocell *C(const otree *t, cref a) { return &t->nodes[a.node].cell[a.loc]; }

static void gidx(const otree *t, cref a, int g[3]) {
    const onode *n = &t->nodes[a.node];
    g[0] = 8 * n->n[0] + (a.loc >> 6);
    g[1] = 8 * n->n[1] + ((a.loc >> 3) & 7);
    g[2] = 8 * n->n[2] + (a.loc & 7);
}

static int is_leaf(const otree *t, cref a) { return t->nodes[a.node].leaf; }

/* the 8 child cells of an interior cell */
static void children(const otree *t, cref a, cref out[8]) {
    const onode *n = &t->nodes[a.node];
    int lx = a.loc >> 6, ly = (a.loc >> 3) & 7, lz = a.loc & 7;
    int k = 0;
    for (int ox = 0; ox < 2; ++ox)
        for (int oy = 0; oy < 2; ++oy)
            for (int oz = 0; oz < 2; ++oz) {
                int cx = 2 * lx + ox, cy = 2 * ly + oy, cz = 2 * lz + oz; /* 0..15 within the 2x2x2 children */
                int ch = n->child[((cx >> 3) * 2 + (cy >> 3)) * 2 + (cz >> 3)];
                out[k].node = ch;
                out[k].loc = ((cx & 7) * 8 + (cy & 7)) * 8 + (cz & 7);
                ++k;
            }
}

/* well separated: theta' = dx/|x_A - x_B| < theta, on integer offsets */
static int well_separated(const otree *t, cref a, cref b, const oparams *p) {
    int ga[3], gb[3];
    gidx(t, a, ga);
    gidx(t, b, gb);
    double dx = ga[0] - gb[0], dy = ga[1] - gb[1], dz = ga[2] - gb[2];
    double d2 = dx * dx + dy * dy + dz * dz;
    return p->theta2 * d2 > 1.0;
}

/* ------------------------------------------------------------------------ */
/* Derivative tensors D^(k)(R) = grad^k K(R), k = 0..4                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    double d0, d1[3], d2[3][3], d3[3][3][3], d4[3][3][3][3];
} dtens;

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

static void dtensors_newton(const double R[3], dtens *D) {
    /* radial derivatives f_k = (r^-1 d/dr)^k r^-1 */
    double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    double r = sqrt(r2);
    double f0 = 1.0 / r;
    double f1 = -f0 / r2;
    double f2 = -3.0 * f1 / r2;
    double f3 = -5.0 * f2 / r2;
    double f4 = -7.0 * f3 / r2;
    D->d0 = f0;
    for (int a = 0; a < 3; ++a) {
        D->d1[a] = f1 * R[a];
        for (int b = 0; b < 3; ++b) {
            D->d2[a][b] = f2 * R[a] * R[b] + f1 * kd(a, b);
            for (int c = 0; c < 3; ++c) {
                D->d3[a][b][c] = f3 * R[a] * R[b] * R[c] + f2 * (kd(a, b) * R[c] + kd(a, c) * R[b] + kd(b, c) * R[a]);
                for (int d = 0; d < 3; ++d) {
                    D->d4[a][b][c][d] =
                        f4 * R[a] * R[b] * R[c] * R[d] +
                        f3 * (kd(a, b) * R[c] * R[d] + kd(a, c) * R[b] * R[d] + kd(a, d) * R[b] * R[c] +
                              kd(b, c) * R[a] * R[d] + kd(b, d) * R[a] * R[c] + kd(c, d) * R[a] * R[b]) +
                        f2 * (kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c));
                }
            }
        }
    }
}

/* d^alpha/dR^alpha of R^beta, alpha given as per-axis counts */
static double mono_deriv(const int beta[3], const int alpha[3], const double R[3]) {
    double v = 1.0;
    for (int d = 0; d < 3; ++d) {
        if (alpha[d] > beta[d]) return 0.0;
        for (int q = 0; q < alpha[d]; ++q) v *= (double)(beta[d] - q);
        for (int q = 0; q < beta[d] - alpha[d]; ++q) v *= R[d];
    }
    return v;
}

static double poly_deriv(const oparams *p, const int *axes, int k, const double R[3]) {
    int alpha[3] = {0, 0, 0};
    for (int i = 0; i < k; ++i) alpha[axes[i]]++;
    double s = 0.0;
    for (int m = 0; m < 20; ++m) s += p->coef[m] * mono_deriv(p->pw[m], alpha, R);
    return s;
}

static void dtensors_poly(const oparams *p, const double R[3], dtens *D) {
    int ax[4] = {0, 0, 0, 0};
    D->d0 = poly_deriv(p, ax, 0, R);
    for (ax[0] = 0; ax[0] < 3; ++ax[0]) {
        D->d1[ax[0]] = poly_deriv(p, ax, 1, R);
        for (ax[1] = 0; ax[1] < 3; ++ax[1]) {
            D->d2[ax[0]][ax[1]] = poly_deriv(p, ax, 2, R);
            for (ax[2] = 0; ax[2] < 3; ++ax[2]) {
                D->d3[ax[0]][ax[1]][ax[2]] = poly_deriv(p, ax, 3, R);
                for (ax[3] = 0; ax[3] < 3; ++ax[3]) D->d4[ax[0]][ax[1]][ax[2]][ax[3]] = poly_deriv(p, ax, 4, R);
            }
        }
    }
}

static void dtensors(const oparams *p, const double R[3], dtens *D) {
    if (p->mode == 0)
        dtensors_newton(R, D);
    else
        dtensors_poly(p, R, D);
}

/* ------------------------------------------------------------------------ */
/* The operators                                                             */
/* ------------------------------------------------------------------------ */

/* Multipole of a leaf cell: a point mass at its centre. */
static void p2m(otree *t, cref a) {
    const onode *n = &t->nodes[a.node];
    ocell *c = C(t, a);
    int g[3];
    gidx(t, a, g);
    double h = cell_width(n->level);
    c->m = n->rho[a.loc] * h * h * h;
    for (int d = 0; d < 3; ++d) c->z[d] = centre(n->level, g[d]);
    memset(c->M1, 0, sizeof c->M1);
    memset(c->M2, 0, sizeof c->M2);
    memset(c->M3, 0, sizeof c->M3);
}

/* Raw moments (orders 0-3) of the children's multipoles about the point z:
 * each child's moments about its own centre z_c are shifted by s = z_c - z
 * (binomial expansion of (x - z)^n = ((x - z_c) + s)^n). */
static void compose(const ocell *const ch[8], const double z[3], ocell *p) {
    p->m = 0.0;
    memset(p->M1, 0, sizeof p->M1);
    memset(p->M2, 0, sizeof p->M2);
    memset(p->M3, 0, sizeof p->M3);
    for (int k = 0; k < 8; ++k) {
        const ocell *c = ch[k];
        double s[3];
        for (int d = 0; d < 3; ++d) s[d] = c->z[d] - z[d];
        p->m += c->m;
        for (int i = 0; i < 3; ++i) {
            p->M1[i] += c->M1[i] + c->m * s[i];
            for (int j = 0; j < 3; ++j) {
                p->M2[i][j] += c->M2[i][j] + c->M1[i] * s[j] + c->M1[j] * s[i] + c->m * s[i] * s[j];
                for (int l = 0; l < 3; ++l)
                    p->M3[i][j][l] += c->M3[i][j][l] + c->M2[i][j] * s[l] + c->M2[i][l] * s[j] + c->M2[j][l] * s[i] +
                                      c->M1[i] * s[j] * s[l] + c->M1[j] * s[i] * s[l] + c->M1[l] * s[i] * s[j] +
                                      c->m * s[i] * s[j] * s[l];
            }
        }
    }
}

/* Compose a cell's multipole from its 8 children: total mass, centre of mass,
 * and raw second and third moments about that centre (the children's dipoles
 * about their own centres of mass vanish, and so does the parent's about its
 * own: it is set to zero rather than left at its rounding residue). */
static void m2m(otree *t, cref a) {
    cref ch[8];
    children(t, a, ch);
    ocell *p = C(t, a);
    const ocell *cc[8];
    double m = 0.0, mz[3] = {0, 0, 0};
    for (int k = 0; k < 8; ++k) {
        cc[k] = C(t, ch[k]);
        m += cc[k]->m;
        for (int d = 0; d < 3; ++d) mz[d] += cc[k]->m * cc[k]->z[d];
    }
    double z[3];
    if (m > 0.0 && t->centres == 0) {
        for (int d = 0; d < 3; ++d) z[d] = mz[d] / m;
    } else {
        int g[3];
        gidx(t, a, g);
        for (int d = 0; d < 3; ++d) z[d] = centre(t->nodes[a.node].level, g[d]);
    }
    compose(cc, z, p);
    for (int d = 0; d < 3; ++d) p->z[d] = z[d];
    if (t->centres != 1) memset(p->M1, 0, sizeof p->M1);
}

/* Second source (a density rate): leaf cells are point sources s h^3 at
 * their centres (which are also the density's centres of mass). */
static void p2m_src(otree *t, cref a, const double *src) {
    const onode *n = &t->nodes[a.node];
    ocell *c = C(t, a);
    double h = cell_width(n->level);
    c->m = src[(size_t)n->out * 512 + a.loc] * h * h * h;
    memset(c->M1, 0, sizeof c->M1);
    memset(c->M2, 0, sizeof c->M2);
    memset(c->M3, 0, sizeof c->M3);
}

/* Second source, interior cells: moments of orders 0-3 about the density's
 * centre of mass z (already in the cell), dipole included. */
static void m2m_src(otree *t, cref a) {
    cref ch[8];
    children(t, a, ch);
    ocell *p = C(t, a);
    const ocell *cc[8];
    for (int k = 0; k < 8; ++k) cc[k] = C(t, ch[k]);
    double z[3] = {p->z[0], p->z[1], p->z[2]};
    compose(cc, z, p);
}

/* Multipole-to-local: the Taylor expansion about z_A of the potential of
 * B's multipole, truncated at total order 3 (L^(n) keeps source orders
 * m <= 3 - n), plus the angular-momentum correction of A. */
static void m2l_cells(const ocell *A, const ocell *B, const oparams *p, double *L0, double L1[3], double L2[3][3],
                      double L3[3][3][3], double Cc[3]) {
    double R[3];
    for (int d = 0; d < 3; ++d) R[d] = A->z[d] - B->z[d];
    dtens D;
    dtensors(p, R, &D);
    const double G = p->G;
    /* L^(n) = -G sum_{k <= 3-n} ((-1)^k / k!) M^(k)_B : D^(n+k) */
    double q1 = 0.0, q2 = 0.0, q3 = 0.0;
    for (int a = 0; a < 3; ++a) {
        q1 += B->M1[a] * D.d1[a];
        for (int b = 0; b < 3; ++b) {
            q2 += B->M2[a][b] * D.d2[a][b];
            for (int c = 0; c < 3; ++c) q3 += B->M3[a][b][c] * D.d3[a][b][c];
        }
    }
    *L0 += -G * (B->m * D.d0 - q1 + 0.5 * q2 - q3 / 6.0);
    for (int a = 0; a < 3; ++a) {
        double s1 = 0.0, s = 0.0;
        for (int b = 0; b < 3; ++b) {
            s1 += B->M1[b] * D.d2[a][b];
            for (int c = 0; c < 3; ++c) s += B->M2[b][c] * D.d3[a][b][c];
        }
        L1[a] += -G * (B->m * D.d1[a] - s1 + 0.5 * s);
        for (int b = 0; b < 3; ++b) {
            double s2 = 0.0;
            for (int c = 0; c < 3; ++c) s2 += B->M1[c] * D.d3[a][b][c];
            L2[a][b] += -G * (B->m * D.d2[a][b] - s2);
            for (int c = 0; c < 3; ++c) L3[a][b][c] += -G * B->m * D.d3[a][b][c];
        }
    }
    /* Correction: the order-3 pair force F3 = (G/6)(m_B M3_A - m_A M3_B) : D^(4)
     * acts on A as the uniform acceleration F3/m_A. */
    if (p->amc && A->m > 0.0) {
        double ratio = B->m / A->m;
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d) s += (B->M3[b][c][d] - ratio * A->M3[b][c][d]) * D.d4[a][b][c][d];
            Cc[a] += -G * s / 6.0;
        }
    }
}

static void m2l(otree *t, cref a, cref b, const oparams *p) {
    ocell *A = C(t, a);
    if (p->cnt) {
        p->cnt->m2l++;
        if (is_leaf(t, a) && is_leaf(t, b)) p->cnt->m2l_leaf_leaf++;
    }
    m2l_cells(A, C(t, b), p, &A->L0, A->L1, A->L2, A->L3, A->C);
}

/* Point-mass interaction of leaf cell a with leaf cell b (a receives). */
static void direct(otree *t, cref a, cref b, const oparams *p) {
    if (!t->nodes[a.node].mark[a.loc]) return;
    if (p->cnt) p->cnt->direct++;
    ocell *A = C(t, a);
    const ocell *B = C(t, b);
    double R[3];
    for (int d = 0; d < 3; ++d) R[d] = A->z[d] - B->z[d];
    dtens D;
    dtensors(p, R, &D);
    A->L0 += -p->G * B->m * D.d0;
    for (int d = 0; d < 3; ++d) A->L1[d] += -p->G * B->m * D.d1[d];
}

/* Candidate pair (a receives from b), same level, a != b. */
static void interact(otree *t, cref a, cref b, const oparams *p) {
    if (!t->nodes[a.node].mark[a.loc]) return;
    if (well_separated(t, a, b, p)) {
        m2l(t, a, b, p);
        return;
    }
    int la = is_leaf(t, a), lb = is_leaf(t, b);
    cref ca[8], cb[8];
    if (la && lb) {
        direct(t, a, b, p);
    } else if (la) {
        children(t, b, cb); /* leaves, by proper nesting */
        for (int j = 0; j < 8; ++j) direct(t, a, cb[j], p);
    } else if (lb) {
        children(t, a, ca);
        for (int i = 0; i < 8; ++i) direct(t, ca[i], b, p);
    } else {
        children(t, a, ca);
        children(t, b, cb);
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) interact(t, ca[i], cb[j], p);
    }
}

/* Pairs of distinct children of one interior cell (their parents coincide and
 * so are not well separated), then recurse. */
static void siblings(otree *t, cref a, const oparams *p) {
    if (is_leaf(t, a) || !t->nodes[a.node].mark[a.loc]) return;
    cref ca[8];
    children(t, a, ca);
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j)
            if (i != j) interact(t, ca[i], ca[j], p);
    for (int i = 0; i < 8; ++i) siblings(t, ca[i], p);
}

/* Shift the expansion of parent cell P to child cell Q (Taylor series of the
 * order-3 local polynomial about the new centre); the correction is a uniform
 * acceleration and is inherited unchanged. */
static void l2l(const ocell *P, ocell *Q) {
    double d[3];
    for (int i = 0; i < 3; ++i) d[i] = Q->z[i] - P->z[i];
    double s0 = P->L0;
    for (int a = 0; a < 3; ++a) {
        s0 += P->L1[a] * d[a];
        for (int b = 0; b < 3; ++b) {
            s0 += 0.5 * P->L2[a][b] * d[a] * d[b];
            for (int c = 0; c < 3; ++c) s0 += P->L3[a][b][c] * d[a] * d[b] * d[c] / 6.0;
        }
    }
    Q->L0 += s0;
    for (int a = 0; a < 3; ++a) {
        double s1 = P->L1[a];
        for (int b = 0; b < 3; ++b) {
            s1 += P->L2[a][b] * d[b];
            for (int c = 0; c < 3; ++c) s1 += 0.5 * P->L3[a][b][c] * d[b] * d[c];
        }
        Q->L1[a] += s1;
        for (int b = 0; b < 3; ++b) {
            double s2 = P->L2[a][b];
            for (int c = 0; c < 3; ++c) s2 += P->L3[a][b][c] * d[c];
            Q->L2[a][b] += s2;
            for (int c = 0; c < 3; ++c) Q->L3[a][b][c] += P->L3[a][b][c];
        }
        Q->C[a] += P->C[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Solve                                                                     */
/* ------------------------------------------------------------------------ */

static void init_params(oparams *p, double theta, double G, int amc, int mode, const double *coef) {
    memset(p, 0, sizeof *p);
    p->theta2 = theta * theta;
    p->G = G;
    p->amc = amc;
    p->mode = mode;
    int m = 0;
    for (int bx = 0; bx <= 3; ++bx)
        for (int by = 0; by <= 3 - bx; ++by)
            for (int bz = 0; bz <= 3 - bx - by; ++bz) {
                p->pw[m][0] = bx;
                p->pw[m][1] = by;
                p->pw[m][2] = bz;
                p->coef[m] = coef ? coef[m] : 0.0;
                ++m;
            }
}

static void mark_up(otree *t, int node, int loc) {
    int l = t->nodes[node].level;
    int g[3];
    cref a = {node, loc};
    gidx(t, a, g);
    for (int pl = l; pl >= 0; --pl) {
        int sh = l - pl;
        int gx = g[0] >> sh, gy = g[1] >> sh, gz = g[2] >> sh;
        int id = lut_get(t, pl, gx >> 3, gy >> 3, gz >> 3);
        t->nodes[id].mark[((gx & 7) * 8 + (gy & 7)) * 8 + (gz & 7)] = 1;
    }
}

/* Solve for phi and g at every leaf cell (sample == NULL), or only at the
 * listed leaf cells (global leaf-cell ids leaf*512 + local), restricting the
 * interaction recursion to targets on their ancestor chains.
 * phi: n_out, g: 3 x n_out (SoA), where n_out = nleaves*512 (full) or nsample.
 * Returns 0 on success. */
static int solve_impl(otree *t, const oparams *pp, const double *src, const int64_t *sample, int64_t nsample,
                      int nthreads, double *phi, double *g) {
    oparams p = *pp;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* per-level node lists */
    int *cnt = (int *)calloc(OMAXLEV, sizeof(int));
    int **lev = (int **)calloc(OMAXLEV, sizeof(int *));
    for (int id = 0; id < t->nnodes; ++id) cnt[t->nodes[id].level]++;
    for (int l = 0; l < OMAXLEV; ++l) {
        lev[l] = (int *)malloc(sizeof(int) * (size_t)(cnt[l] + 1));
        cnt[l] = 0;
    }
    for (int id = 0; id < t->nnodes; ++id) {
        int l = t->nodes[id].level;
        lev[l][cnt[l]++] = id;
    }
    /* reset */
#pragma omp parallel for schedule(static)
    for (int id = 0; id < t->nnodes; ++id) {
        for (int i = 0; i < 512; ++i) {
            ocell *c = &t->nodes[id].cell[i];
            c->L0 = 0.0;
            memset(c->L1, 0, sizeof c->L1);
            memset(c->L2, 0, sizeof c->L2);
            memset(c->L3, 0, sizeof c->L3);
            memset(c->C, 0, sizeof c->C);
        }
        memset(t->nodes[id].mark, sample ? 0 : 1, 512);
    }
    if (sample) {
        for (int64_t s = 0; s < nsample; ++s) {
            int64_t gid = sample[s];
            if (gid < 0 || gid >= (int64_t)t->nleaves * 512) return 2;
            mark_up(t, t->leaf_node[gid / 512], (int)(gid % 512));
        }
    }
    /* upward: leaves become point masses, then compose level by level */
#pragma omp parallel for schedule(static)
    for (int id = 0; id < t->nnodes; ++id)
        if (t->nodes[id].leaf)
            for (int i = 0; i < 512; ++i) p2m(t, (cref){id, i});
    for (int l = t->nlev - 2; l >= 0; --l) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < cnt[l]; ++k) {
            int id = lev[l][k];
            if (t->nodes[id].leaf) continue;
            for (int i = 0; i < 512; ++i) m2m(t, (cref){id, i});
        }
    }
    /* a second source: its moments about the density's expansion centres */
    if (src) {
#pragma omp parallel for schedule(static)
        for (int id = 0; id < t->nnodes; ++id)
            if (t->nodes[id].leaf)
                for (int i = 0; i < 512; ++i) p2m_src(t, (cref){id, i}, src);
        for (int l = t->nlev - 2; l >= 0; --l) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < cnt[l]; ++k) {
                int id = lev[l][k];
                if (t->nodes[id].leaf) continue;
                for (int i = 0; i < 512; ++i) m2m_src(t, (cref){id, i});
            }
        }
    }
    /* interactions: all ordered pairs of distinct root cells are candidates */
    int root = lut_get(t, 0, 0, 0, 0);
    ocount *counts = (ocount *)calloc(512, sizeof(ocount));
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < 512; ++i) {
        oparams pt = p;
        pt.cnt = &counts[i];
        cref a = {root, i};
        for (int j = 0; j < 512; ++j)
            if (j != i) interact(t, a, (cref){root, j}, &pt);
        siblings(t, a, &pt);
    }
    t->last.m2l = t->last.direct = t->last.m2l_leaf_leaf = 0;
    for (int i = 0; i < 512; ++i) {
        t->last.m2l += counts[i].m2l;
        t->last.direct += counts[i].direct;
        t->last.m2l_leaf_leaf += counts[i].m2l_leaf_leaf;
    }
    free(counts);
    /* downward */
    for (int l = 1; l < t->nlev; ++l) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < cnt[l]; ++k) {
            int id = lev[l][k];
            onode *n = &t->nodes[id];
            const onode *pn = &t->nodes[n->parent];
            for (int i = 0; i < 512; ++i) {
                if (!n->mark[i]) continue;
                int lx = i >> 6, ly = (i >> 3) & 7, lz = i & 7;
                int px = (4 * (n->n[0] & 1)) + (lx >> 1), py = (4 * (n->n[1] & 1)) + (ly >> 1),
                    pz = (4 * (n->n[2] & 1)) + (lz >> 1);
                l2l(&pn->cell[(px * 8 + py) * 8 + pz], &n->cell[i]);
            }
        }
    }
    /* leaves: phi = L0, g = -grad phi = -L1 + C */
    int64_t nout = sample ? nsample : (int64_t)t->nleaves * 512;
    for (int64_t s = 0; s < nout; ++s) {
        int64_t gid = sample ? sample[s] : s;
        const ocell *c = &t->nodes[t->leaf_node[gid / 512]].cell[gid % 512];
        phi[s] = c->L0;
        if (g)
            for (int d = 0; d < 3; ++d) g[d * nout + s] = -c->L1[d] + c->C[d];
    }
    for (int l = 0; l < OMAXLEV; ++l) free(lev[l]);
    free(lev);
    free(cnt);
    return 0;
}

/* Expansion centres of interior cells for later solves of the density.
 * The paper says multipoles and expansions are taken relative to cell
 * centres (Sec. 2.2); the default reading is the centre of mass (mode 0),
 * about which the dipole vanishes and the correction cancels the pair torque
 * exactly.  Mode 1 expands about geometric centres and carries the dipole
 * through every shift and interaction (a complete expansion about another
 * point); mode 2 expands about geometric centres and drops the dipole, as an
 * implementation that assumes it vanishes would.  Used only to study the
 * static-sphere residuals of Sec. 3.4; the correction is not exact for modes
 * 1 and 2.  Returns 0, or 1 for an unknown mode. */
int orc_tree_set_centres(otree *t, int mode) {
    if (!t || mode < 0 || mode > 2) return 1;
    t->centres = mode;
    return 0;
}

int orc_solve(otree *t, double theta, double G, int amc, int mode, const double *coef, const int64_t *sample,
              int64_t nsample, int nthreads, double *phi, double *g) {
    if (!t || t->err[0]) return 1;
    oparams p;
    init_params(&p, theta, G, amc, mode, coef);
    return solve_impl(t, &p, NULL, sample, nsample, nthreads, phi, g);
}

/* The potential of a second, signed source s (a density rate, per leaf cell in
 * the same layout as the density) with the density's tree, interaction lists
 * and expansion centres: the FMM applied to the time derivative of the density
 * gives the time derivative of the potential (Sec. 2.1, the energy equation's
 * source term).  With the same centres the discrete operator is the same
 * symmetric matrix as for the density, so sum_i (phi_i s_i - rho_i dphi_i) h_i^3
 * vanishes up to rounding.  Only the potential is returned; the correction
 * (which acts on forces) is not applied.  The tree's moments afterwards are
 * those of s. */
int orc_solve_source(otree *t, double theta, double G, int mode, const double *coef, const double *src,
                     const int64_t *sample, int64_t nsample, int nthreads, double *phi) {
    if (!t || t->err[0] || !src) return 1;
    oparams p;
    init_params(&p, theta, G, 0, mode, coef);
    return solve_impl(t, &p, src, sample, nsample, nthreads, phi, NULL);
}

/* Moments of cell (level, global index) after the last solve:
 * out[0] = m, out[1..3] = z, out[4..12] = M2 (row-major), out[13..39] = M3,
 * out[40..42] = M1. */
int orc_cell_moments(const otree *t, int level, int gx, int gy, int gz, double *out) {
    int id = lut_get(t, level, gx >> 3, gy >> 3, gz >> 3);
    if (id < 0) return 1;
    const ocell *c = &t->nodes[id].cell[((gx & 7) * 8 + (gy & 7)) * 8 + (gz & 7)];
    out[0] = c->m;
    for (int d = 0; d < 3; ++d) out[1 + d] = c->z[d];
    memcpy(out + 4, c->M2, 9 * sizeof(double));
    memcpy(out + 13, c->M3, 27 * sizeof(double));
    memcpy(out + 40, c->M1, 3 * sizeof(double));
    return 0;
}

/* Leaf-cell centres (3 x n SoA) and masses (n) in leaf-list order. */
void orc_leaf_cells(const otree *t, double *x, double *m) {
    int64_t n = (int64_t)t->nleaves * 512;
    for (int k = 0; k < t->nleaves; ++k) {
        const onode *nd = &t->nodes[t->leaf_node[k]];
        double h = cell_width(nd->level);
        for (int i = 0; i < 512; ++i) {
            int64_t s = (int64_t)k * 512 + i;
            int g[3];
            gidx(t, (cref){t->leaf_node[k], i}, g);
            for (int d = 0; d < 3; ++d) x[d * n + s] = centre(nd->level, g[d]);
            m[s] = nd->rho[i] * h * h * h;
        }
    }
}

/* Derivative tensors of the kernel at R (for tests): out = d0, d1(3), d2(9),
 * d3(27), d4(81). */
void orc_dtensors(const double *R, int mode, const double *coef, double *out) {
    oparams p;
    init_params(&p, 0.5, 1.0, 1, mode, coef);
    dtens D;
    dtensors(&p, R, &D);
    out[0] = D.d0;
    memcpy(out + 1, D.d1, 3 * sizeof(double));
    memcpy(out + 4, D.d2, 9 * sizeof(double));
    memcpy(out + 13, D.d3, 27 * sizeof(double));
    memcpy(out + 40, D.d4, 81 * sizeof(double));
}

/* One multipole-to-local interaction between two free cells (for tests).
 * a, b: m, z(3), M2(9), M3(27) as in orc_cell_moments.
 * out: L0, L1(3), L2(9), L3(27), C(3) = 43 values for A receiving from B. */
void orc_m2l_pair(const double *a, const double *b, double G, int amc, int mode, const double *coef, double *out) {
    oparams p;
    init_params(&p, 0.5, G, amc, mode, coef);
    ocell A, B;
    memset(&A, 0, sizeof A);
    memset(&B, 0, sizeof B);
    A.m = a[0];
    B.m = b[0];
    memcpy(A.z, a + 1, 3 * sizeof(double));
    memcpy(B.z, b + 1, 3 * sizeof(double));
    memcpy(A.M2, a + 4, 9 * sizeof(double));
    memcpy(B.M2, b + 4, 9 * sizeof(double));
    memcpy(A.M3, a + 13, 27 * sizeof(double));
    memcpy(B.M3, b + 13, 27 * sizeof(double));
    m2l_cells(&A, &B, &p, &A.L0, A.L1, A.L2, A.L3, A.C);
    out[0] = A.L0;
    memcpy(out + 1, A.L1, 3 * sizeof(double));
    memcpy(out + 4, A.L2, 9 * sizeof(double));
    memcpy(out + 13, A.L3, 27 * sizeof(double));
    memcpy(out + 40, A.C, 3 * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Direct N^2 summation with Neumaier compensation                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    double s, c;
} nsum;

static void nadd(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

/* phi_i = -G sum_{j != i} m_j K(x_i - x_j), g_i = -grad phi, for targets
 * i in [i0, i1).  x: 3 x n SoA; outputs are (i1 - i0) and 3 x (i1 - i0). */
void orc_direct(int64_t n, const double *x, const double *m, double G, int mode, const double *coef, int64_t i0,
                int64_t i1, int nthreads, double *phi, double *g) {
    oparams p;
    init_params(&p, 0.5, G, 1, mode, coef);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t nt = i1 - i0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = i0; i < i1; ++i) {
        nsum sp = {0, 0}, sg[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double R[3] = {x[i] - x[j], x[n + i] - x[n + j], x[2 * n + i] - x[2 * n + j]};
            double d0, d1[3];
            if (p.mode == 0) {
                double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
                double r = sqrt(r2);
                d0 = 1.0 / r;
                for (int d = 0; d < 3; ++d) d1[d] = -R[d] / (r2 * r);
            } else {
                int ax[1] = {0};
                d0 = poly_deriv(&p, ax, 0, R);
                for (ax[0] = 0; ax[0] < 3; ++ax[0]) d1[ax[0]] = poly_deriv(&p, ax, 1, R);
            }
            nadd(&sp, -G * m[j] * d0);
            for (int d = 0; d < 3; ++d) nadd(&sg[d], G * m[j] * d1[d]);
        }
        phi[i - i0] = sp.s + sp.c;
        for (int d = 0; d < 3; ++d) g[d * nt + (i - i0)] = sg[d].s + sg[d].c;
    }
}

/* Direct sum at arbitrary target points xt (3 x nt SoA) from all sources;
 * a source at exactly the target position is skipped (no self-interaction). */
void orc_direct_points(int64_t n, const double *x, const double *m, int64_t nt, const double *xt, double G, int mode,
                       const double *coef, int nthreads, double *phi, double *g) {
    oparams p;
    init_params(&p, 0.5, G, 1, mode, coef);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        nsum sp = {0, 0}, sg[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = 0; j < n; ++j) {
            double R[3] = {xt[i] - x[j], xt[nt + i] - x[n + j], xt[2 * nt + i] - x[2 * n + j]};
            if (R[0] == 0.0 && R[1] == 0.0 && R[2] == 0.0) continue;
            double d0, d1[3];
            if (p.mode == 0) {
                double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
                double r = sqrt(r2);
                d0 = 1.0 / r;
                for (int d = 0; d < 3; ++d) d1[d] = -R[d] / (r2 * r);
            } else {
                int ax[1] = {0};
                d0 = poly_deriv(&p, ax, 0, R);
                for (ax[0] = 0; ax[0] < 3; ++ax[0]) d1[ax[0]] = poly_deriv(&p, ax, 1, R);
            }
            nadd(&sp, -G * m[j] * d0);
            for (int d = 0; d < 3; ++d) nadd(&sg[d], G * m[j] * d1[d]);
        }
        phi[i] = sp.s + sp.c;
        for (int d = 0; d < 3; ++d) g[d * nt + i] = sg[d].s + sg[d].c;
    }
}
