// Self-consistent-field (SCF) iteration for a synchronously rotating binary
// of two polytropes (Sec. 4.1, "The Initial Stellar Model") on the n^3 grid of
// a uniform tree, every step on the device.
//
// Work per iteration: four streaming passes over the grid (star finding,
// normalisation, moments of the stars, new density), three one-block kernels
// for the scalars (centres, orbit, L1 and the constants) and the potential
// solve.  Every maximum (centre cells, L1) is a reduction with a total order
// (larger value first, then smaller flat index), so it is exact and
// independent of the launch shape; the sums are reduced in a fixed order
// (per-block partials, then one block), so results repeat bit for bit.
//
// Star membership is decided on integers: cell centres and the split between
// the sides are multiples of h/2 (the split is a cell centre or a cell face),
// so |x_i - x_c| < |x_split - x_c| is the comparison of squared offsets in
// half-cell units, which is what the floating-point comparison of those
// distances decides.
//
// This file is compiled without floating-point contraction, so each step
// rounds as written.
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"

namespace octo {
namespace {

constexpr int kT = 256;          // threads per block
constexpr int kMaxParts = 2048;  // partial results per streaming pass (blocks)
constexpr int kUnr = 4;          // cells per thread with their loads in flight together
constexpr int kSums = 11;        // moments gathered by the moments pass
constexpr int64_t kNone = INT64_MAX;

struct ScfConst {
    int lg, n;        // log2 of cells per axis, cells per axis
    int64_t cells;    // n^3
    double h, vol;    // cell width, cell volume
    double M[2];      // target masses
    double npoly, f, rho_floor, J0;
};

// Device-resident state of the iteration.
struct ScfDev {
    int64_t s2;       // split in half-cell units: x = s2 h / 2 - 1/2
    double K;         // polytropic constant in force
    int64_t c[2];     // centre cells
    int64_t r2[2];    // star radii |s2 - (2 i_c + 1)| in half-cell units
    double q[2];      // normalisation factors (step 1)
    double m[2];      // star masses of the current density
    double omega, xc, yc, a;
    double C[2], K_new;
    int64_t l1, s2_new;
};

struct Arg {
    double v;
    int64_t i;
};

__device__ inline void take(Arg &a, double v, int64_t i) {
    if (v > a.v || (v == a.v && i < a.i)) {
        a.v = v;
        a.i = i;
    }
}

__device__ inline Arg wave_arg(Arg a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Arg b;
        b.v = __shfl_xor(a.v, o, 64);
        b.i = __shfl_xor(a.i, o, 64);
        take(a, b.v, b.i);
    }
    return a;
}

// Block-wide maximum; the result is valid in thread 0.
__device__ inline Arg block_arg(Arg a, Arg *lds) {
    a = wave_arg(a);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) lds[w] = a;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) take(a, lds[k].v, lds[k].i);
    __syncthreads();
    return a;
}

__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// grids up to 512^3 cells: flat indices fit 32 bits
__device__ inline void cell_ijk(uint32_t g, const ScfConst &k, int &i, int &j, int &l) {
    i = (int)(g >> (2 * k.lg));
    j = (int)(g >> k.lg) & (k.n - 1);
    l = (int)g & (k.n - 1);
}

__device__ inline double centre_of(int i, double h) { return (i + 0.5) * h - 0.5; }

// Side 0 (accretor) holds the cells whose centre lies below the split.
// Offsets and radii in half-cell units stay below 2^11 (n <= 512), their
// squares and sums below 2^31.
__device__ inline int side_of(int i, int64_t s2) { return 2 * i + 1 < (int)s2 ? 0 : 1; }

struct Star {
    int ci, cj, cl;
    int r2sq;  // squared radius in half-cell units
};

__device__ inline Star star_of(int64_t c, int64_t r2, const ScfConst &k) {
    Star s;
    cell_ijk((uint32_t)c, k, s.ci, s.cj, s.cl);
    s.r2sq = (int)(r2 * r2);
    return s;
}

__device__ inline bool inside(const Star &s, int i, int j, int l) {
    const int di = i - s.ci, dj = j - s.cj, dl = l - s.cl;
    return 4 * (di * di + dj * dj + dl * dl) < s.r2sq;
}

__device__ inline int64_t half_radius(int64_t s2, int64_t c, const ScfConst &k) {
    const int64_t ci = c >> (2 * k.lg);
    const int64_t d = s2 - (2 * ci + 1);
    return d < 0 ? -d : d;
}

__device__ inline void store_arg(Arg a[2], double *bv, int64_t *bi) {
    __shared__ Arg lds[kT / 64];
    for (int s = 0; s < 2; ++s) {
        const Arg r = block_arg(a[s], lds);
        if (threadIdx.x == 0) {
            bv[2 * blockIdx.x + s] = r.v;
            bi[2 * blockIdx.x + s] = r.i;
        }
    }
}

__global__ void k_scf_init(ScfDev *st, int64_t s2, double K) {
    st->s2 = s2;
    st->K = K;
}

// Streaming pass over the grid, with the densest cell of each side of the
// split in the pass's output density as a by-product.
//   MODE 0: read the density (star finding);
//   MODE 1: step 1, multiply each star's cells by its normalisation factor;
//   MODE 2: step 6, the new density from the potential (split = new L1).
template <int MODE>
__global__ __launch_bounds__(kT) void k_scf_pass(ScfConst k, const ScfDev *__restrict__ st, double *rho,
                                                 const double *__restrict__ phi, double *__restrict__ bv,
                                                 int64_t *__restrict__ bi) {
    const int64_t s2 = MODE == 2 ? st->s2_new : st->s2;
    Star S[2];
    double C[2] = {0.0, 0.0}, q[2] = {1.0, 1.0}, w2 = 0.0, xc = 0.0, yc = 0.0, kn = 1.0;
    if (MODE != 0)
        for (int s = 0; s < 2; ++s) S[s] = star_of(st->c[s], MODE == 2 ? half_radius(s2, st->c[s], k) : st->r2[s], k);
    if (MODE == 1) {
        q[0] = st->q[0];
        q[1] = st->q[1];
    }
    if (MODE == 2) {
        C[0] = st->C[0];
        C[1] = st->C[1];
        w2 = 0.5 * st->omega * st->omega;
        xc = st->xc;
        yc = st->yc;
        kn = st->K_new * (k.npoly + 1.0);
    }
    Arg best[2] = {{-INFINITY, kNone}, {-INFINITY, kNone}};
    const uint32_t cells = (uint32_t)k.cells, stride = gridDim.x * kT;
    const double *src = MODE == 2 ? phi : rho;
    for (uint32_t g0 = blockIdx.x * kT + threadIdx.x; g0 < cells; g0 += kUnr * stride) {
        double in[kUnr];
#pragma unroll
        for (int u = 0; u < kUnr; ++u) {
            const uint32_t g = g0 + u * stride;
            in[u] = g < cells ? src[g] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kUnr; ++u) {
            const uint32_t g = g0 + u * stride;
            if (g >= cells) break;
            int i, j, l;
            cell_ijk(g, k, i, j, l);
            const int s = side_of(i, s2);
            double v = in[u];
            if (MODE == 1) {
                if (inside(S[s], i, j, l)) {
                    v = v * q[s];
                    rho[g] = v;
                }
            } else if (MODE == 2) {
                const double dx = centre_of(i, k.h) - xc, dy = centre_of(j, k.h) - yc;
                const double pe = in[u] - w2 * (dx * dx + dy * dy);
                const double H = inside(S[s], i, j, l) ? C[s] - pe : -1.0;
                v = H > 0.0 ? pow(H / kn, k.npoly) : 0.0;
                v = v < k.rho_floor ? k.rho_floor : v;
                rho[g] = v;
            }
            take(best[s], v, g);
        }
    }
    store_arg(best, bv, bi);
}

// Centre cells from the pass partials; radii about the split.  advance:
// the split and K of the iteration just finished take over first.
__global__ __launch_bounds__(kT) void k_scf_centres(ScfConst k, ScfDev *st, const double *__restrict__ bv,
                                                    const int64_t *__restrict__ bi, int nparts, int advance) {
    __shared__ Arg lds[kT / 64];
    Arg a[2] = {{-INFINITY, kNone}, {-INFINITY, kNone}};
    for (int p = threadIdx.x; p < nparts; p += kT)
        for (int s = 0; s < 2; ++s) take(a[s], bv[2 * p + s], bi[2 * p + s]);
    for (int s = 0; s < 2; ++s) a[s] = block_arg(a[s], lds);
    if (threadIdx.x == 0) {
        if (advance) {
            st->s2 = st->s2_new;
            st->K = st->K_new;
        }
        for (int s = 0; s < 2; ++s) {
            // an empty side: every candidate ties at -inf, the smallest index wins
            const int64_t c = a[s].i == kNone ? 0 : a[s].i;
            st->c[s] = c;
            st->r2[s] = half_radius(st->s2, c, k);
        }
    }
}

// Moments of the grid and of each star about the current split:
// [0..2] sum rho, rho x, rho y over the grid; [3 + 4s ..] sum rho, rho x,
// rho y, rho z over star s.
__global__ __launch_bounds__(kT) void k_scf_moments(ScfConst k, const ScfDev *__restrict__ st,
                                                    const double *__restrict__ rho, double *__restrict__ part) {
    const Star S[2] = {star_of(st->c[0], st->r2[0], k), star_of(st->c[1], st->r2[1], k)};
    const int64_t s2 = st->s2;
    double acc[kSums];
    for (int q = 0; q < kSums; ++q) acc[q] = 0.0;
    const uint32_t cells = (uint32_t)k.cells, stride = gridDim.x * kT;
    for (uint32_t g0 = blockIdx.x * kT + threadIdx.x; g0 < cells; g0 += kUnr * stride) {
        double in[kUnr];
#pragma unroll
        for (int u = 0; u < kUnr; ++u) {
            const uint32_t g = g0 + u * stride;
            in[u] = g < cells ? rho[g] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kUnr; ++u) {
            const uint32_t g = g0 + u * stride;
            if (g >= cells) break;
            int i, j, l;
            cell_ijk(g, k, i, j, l);
            const double r = in[u];
            const double x = centre_of(i, k.h), y = centre_of(j, k.h), z = centre_of(l, k.h);
            acc[0] += r;
            acc[1] += r * x;
            acc[2] += r * y;
            const int s = side_of(i, s2);
            if (inside(S[s], i, j, l)) {
                acc[3 + 4 * s] += r;
                acc[4 + 4 * s] += r * x;
                acc[5 + 4 * s] += r * y;
                acc[6 + 4 * s] += r * z;
            }
        }
    }
    __shared__ double lds[kT / 64][kSums];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int q = 0; q < kSums; ++q) {
        const double v = wsum(acc[q]);
        if (l == 0) lds[w][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kSums) {
        double v = 0.0;
        for (int u = 0; u < kT / 64; ++u) v += lds[u][threadIdx.x];
        part[(int64_t)blockIdx.x * kSums + threadIdx.x] = v;
    }
}

// Totals of the moments (fixed order); normalisation factors (step 1), the
// rotation axis (step 2), the separation and Omega (step 3).
__global__ __launch_bounds__(kT) void k_scf_orbit(ScfConst k, ScfDev *st, const double *__restrict__ part,
                                                  int nparts) {
    __shared__ double lds[kT / 64][kSums];
    __shared__ double tot[kSums];
    double acc[kSums];
    for (int q = 0; q < kSums; ++q) acc[q] = 0.0;
    for (int p = threadIdx.x; p < nparts; p += kT)
        for (int q = 0; q < kSums; ++q) acc[q] += part[(int64_t)p * kSums + q];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int q = 0; q < kSums; ++q) {
        const double v = wsum(acc[q]);
        if (l == 0) lds[w][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kSums) {
        double v = 0.0;
        for (int u = 0; u < kT / 64; ++u) v += lds[u][threadIdx.x];
        tot[threadIdx.x] = v * k.vol;  // vol is a power of two: exact
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double M = tot[0];
        st->xc = tot[1] / M;
        st->yc = tot[2] / M;
        double cm[2][3];
        for (int s = 0; s < 2; ++s) {
            const double ms = tot[3 + 4 * s];
            st->m[s] = ms;
            st->q[s] = k.M[s] / ms;
            for (int d = 0; d < 3; ++d) cm[s][d] = tot[4 + 4 * s + d] / ms;
        }
        const double dx = cm[1][0] - cm[0][0], dy = cm[1][1] - cm[0][1], dz = cm[1][2] - cm[0][2];
        const double a = sqrt(dx * dx + dy * dy + dz * dz);
        st->a = a;
        st->omega = k.J0 * (k.M[0] + k.M[1]) / (k.M[0] * k.M[1] * a * a);
    }
}

// Step 4 and 5: L1 on the row through the accretor's centre, the
// integration constants and the new K; records the iteration's scalars.
__global__ __launch_bounds__(kT) void k_scf_row(ScfConst k, ScfDev *st, const double *__restrict__ rho,
                                                const double *__restrict__ phi, octo_scf_state *hist) {
    __shared__ Arg lds[kT / 64];
    int i1, j1, l1c, i2, j2, l2c;
    cell_ijk(st->c[0], k, i1, j1, l1c);
    cell_ijk(st->c[1], k, i2, j2, l2c);
    const double w2 = 0.5 * st->omega * st->omega, xc = st->xc, yc = st->yc;
    auto peff = [&](int64_t g) {
        int i, j, l;
        cell_ijk(g, k, i, j, l);
        const double dx = centre_of(i, k.h) - xc, dy = centre_of(j, k.h) - yc;
        return phi[g] - w2 * (dx * dx + dy * dy);
    };
    const int lo = i1 < i2 ? i1 : i2, hi = i1 < i2 ? i2 : i1;
    Arg a = {-INFINITY, kNone};
    for (int i = lo + 1 + (int)threadIdx.x; i < hi; i += kT) {
        const int64_t g = ((int64_t)i << (2 * k.lg)) | ((int64_t)j1 << k.lg) | (int64_t)l1c;
        take(a, peff(g), g);
    }
    a = block_arg(a, lds);
    if (threadIdx.x == 0) {
        const int64_t l1 = a.i == kNone ? 0 : a.i;
        const int64_t c1 = st->c[0], c2 = st->c[1];
        const double n = k.npoly;
        const double pe1 = peff(c1), phiC = peff(c2), peL = peff(l1);
        const double C1 = st->K * (1.0 + n) * pow(rho[c1], 1.0 / n) + pe1;
        const double C2 = (1.0 - k.f) * phiC + k.f * peL;
        const double Kn = (C2 - phiC) / ((n + 1.0) * pow(rho[c2], 1.0 / n));
        const int64_t il = l1 >> (2 * k.lg);
        st->C[0] = C1;
        st->C[1] = C2;
        st->K_new = Kn;
        st->l1 = l1;
        st->s2_new = 2 * il + 1;
        octo_scf_state r;
        r.omega = st->omega;
        r.K = Kn;
        r.C1 = C1;
        r.C2 = C2;
        r.x_L1 = centre_of((int)il, k.h);
        r.a = st->a;
        r.mass1 = st->m[0];
        r.mass2 = st->m[1];
        r.c1 = c1;
        r.c2 = c2;
        r.l1 = l1;
        *hist = r;
    }
}

// Scratch of one call: state, partials, iteration records.  Either taken
// from the context's allocator for the call (owned), or carved out of
// caller-provided device memory (the fixed per-device array below).
struct Scratch {
    octo_ctx *ctx = nullptr;
    void *mem = nullptr;
    size_t bytes = 0;
    bool owned = false;
    ScfDev *st = nullptr;
    double *part = nullptr, *bv = nullptr;
    int64_t *bi = nullptr;
    octo_scf_state *hist = nullptr;
    double *g = nullptr;
    struct Offsets {
        size_t part, bv, bi, hist, g, total;
    };
    static Offsets offsets(int n_hist, int64_t g_doubles) {
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        Offsets o;
        o.part = al(sizeof(ScfDev));
        o.bv = o.part + al((size_t)kMaxParts * kSums * 8);
        o.bi = o.bv + al((size_t)kMaxParts * 2 * 8);
        o.hist = o.bi + al((size_t)kMaxParts * 2 * 8);
        o.g = o.hist + al((size_t)(n_hist > 0 ? n_hist : 1) * sizeof(octo_scf_state));
        o.total = o.g + al((size_t)g_doubles * 8);
        return o;
    }
    void carve(const Offsets &o, int64_t g_doubles) {
        char *b = (char *)mem;
        st = (ScfDev *)b;
        part = (double *)(b + o.part);
        bv = (double *)(b + o.bv);
        bi = (int64_t *)(b + o.bi);
        hist = (octo_scf_state *)(b + o.hist);
        g = g_doubles ? (double *)(b + o.g) : nullptr;
    }
    Scratch(octo_ctx *c, int n_hist, int64_t g_doubles) : ctx(c), owned(true) {
        const Offsets o = offsets(n_hist, g_doubles);
        bytes = o.total;
        mem = ctx->dev_alloc(bytes);
        carve(o, g_doubles);
    }
    // one step's scratch inside `dev` (capacity `cap` bytes, checked by the caller)
    Scratch(octo_ctx *c, void *dev) : ctx(c), mem(dev) {
        const Offsets o = offsets(1, 0);
        bytes = o.total;
        carve(o, 0);
    }
    ~Scratch() {
        if (mem && owned) {
            hipStreamSynchronize(ctx->stream);
            ctx->dev_free(mem, bytes);
        }
    }
};

// Fixed scratch of the allocation-free step (octo_scf_step_noalloc): one
// array per device for the whole process.  Its size covers the largest step
// layout (kMaxParts partials, one record), the same for every grid level.
constexpr size_t kFixedScratchBytes = 256 * 1024;
__device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;                          // guards the address table
void *g_fixed_ptr[kMaxDevices] = {};            // device address of `scratch`, per device
std::mutex g_fixed_use[kMaxDevices];            // one step at a time on a device's array

ScfConst make_const(int level, const octo_scf_params &p) {
    ScfConst k;
    k.lg = level + 3;
    k.n = 8 << level;
    k.cells = (int64_t)k.n * k.n * k.n;
    k.h = 1.0 / k.n;
    k.vol = k.h * k.h * k.h;
    k.M[0] = p.M1;
    k.M[1] = p.M2;
    k.npoly = p.n;
    k.f = p.f;
    k.rho_floor = p.rho_floor;
    const double mu = p.M1 * p.M2 / (p.M1 + p.M2);
    k.J0 = mu * p.a0 * p.a0 * std::sqrt(p.G * (p.M1 + p.M2) / std::pow(p.a0, 3.0));
    return k;
}

int parts_for(int64_t cells) {
    const int64_t per = (int64_t)kT * 2 * kUnr;
    const int64_t p = (cells + per - 1) / per;
    return (int)(p < 1 ? 1 : (p > kMaxParts ? kMaxParts : p));
}

template <int MODE>
void pass(const ScfConst &k, const Scratch &s, int np, double *rho, const double *phi, hipStream_t q) {
    hipLaunchKernelGGL(k_scf_pass<MODE>, dim3(np), dim3(kT), 0, q, k, s.st, rho, phi, s.bv, s.bi);
}

// star finding (centres, radii) from the last pass, then the moments
void stars_and_moments(const ScfConst &k, const Scratch &s, int np, const double *rho, int advance,
                       hipStream_t q) {
    hipLaunchKernelGGL(k_scf_centres, dim3(1), dim3(kT), 0, q, k, s.st, s.bv, s.bi, np, advance);
    hipLaunchKernelGGL(k_scf_moments, dim3(np), dim3(kT), 0, q, k, s.st, rho, s.part);
    hipLaunchKernelGGL(k_scf_orbit, dim3(1), dim3(kT), 0, q, k, s.st, s.part, np);
}

// step 1 on `rho` in place (the densest cells of the split's sides are in
// the pass partials); leaves the normalised density's centres and moments
void normalise(const ScfConst &k, const Scratch &s, int np, double *rho, int advance, hipStream_t q) {
    stars_and_moments(k, s, np, rho, advance, q);
    pass<1>(k, s, np, rho, nullptr, q);
    stars_and_moments(k, s, np, rho, 0, q);
}

// steps 4-6 after the moments of the normalised density: rho_out may be rho
void finish_step(const ScfConst &k, const Scratch &s, int np, const double *rho, const double *phi,
                 double *rho_out, octo_scf_state *rec, hipStream_t q) {
    hipLaunchKernelGGL(k_scf_row, dim3(1), dim3(kT), 0, q, k, s.st, rho, phi, rec);
    pass<2>(k, s, np, rho_out, phi, q);
}

}  // namespace

void scf_step(octo_ctx *ctx, int level, const octo_scf_params &p, double K, int64_t s2, const double *rho,
              const double *phi, double *rho_out, octo_scf_state *state) {
    const ScfConst k = make_const(level, p);
    const int np = parts_for(k.cells);
    hipStream_t q = ctx->stream;
    Scratch s(ctx, 1, 0);
    hipLaunchKernelGGL(k_scf_init, dim3(1), dim3(1), 0, q, s.st, s2, K);
    pass<0>(k, s, np, const_cast<double *>(rho), nullptr, q);  // MODE 0 only reads
    stars_and_moments(k, s, np, rho, 0, q);
    finish_step(k, s, np, rho, phi, rho_out, s.hist, q);
    check_hip(hipMemcpyAsync(state, s.hist, sizeof(octo_scf_state), hipMemcpyDeviceToHost, q), "state copy");
    check_hip(hipStreamSynchronize(q), "scf step");
}

void scf_fixed_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) fail(OCTO_E_DEVICE, "device index beyond the fixed-scratch table");
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    if (g_fixed_ptr[device]) return;
    // the caller has made `device` current: the address is that device's copy
    void *p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "fixed scratch address");
    if (!p) fail(OCTO_E_DEVICE, "fixed scratch has no device address");
    g_fixed_ptr[device] = p;
}

size_t scf_fixed_scratch_bytes() { return kFixedScratchBytes; }

void scf_step_noalloc(octo_ctx *ctx, int level, const octo_scf_params &p, double K, int64_t s2, const double *rho,
                      const double *phi, double *rho_out, octo_scf_state *state) {
    const int dev = ctx->device;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_fixed_mu);
        if (dev >= 0 && dev < kMaxDevices) base = g_fixed_ptr[dev];
    }
    if (!base) fail(OCTO_E_STATE, "fixed scratch of device " + std::to_string(dev) + " not set up");
    const size_t need = Scratch::offsets(1, 0).total;
    if (need > kFixedScratchBytes)
        fail(OCTO_E_INVALID, "step needs " + std::to_string(need) + " bytes of scratch, the fixed array holds " +
                                 std::to_string(kFixedScratchBytes));
    const ScfConst k = make_const(level, p);
    const int np = parts_for(k.cells);
    hipStream_t q = ctx->stream;
    // steps on one device share the array: the lock keeps them apart (each
    // returns only after its stream has drained)
    std::lock_guard<std::mutex> use(g_fixed_use[dev]);
    Scratch s(ctx, base);
    // every field of the state, the partials and the record is written by
    // the step's kernels before it is read; k_scf_init sets the split and K
    hipLaunchKernelGGL(k_scf_init, dim3(1), dim3(1), 0, q, s.st, s2, K);
    pass<0>(k, s, np, const_cast<double *>(rho), nullptr, q);  // MODE 0 only reads
    stars_and_moments(k, s, np, rho, 0, q);
    finish_step(k, s, np, rho, phi, rho_out, s.hist, q);
    check_hip(hipMemcpyAsync(state, s.hist, sizeof(octo_scf_state), hipMemcpyDeviceToHost, q), "state copy");
    check_hip(hipStreamSynchronize(q), "scf step");
}

void scf_run(octo_ctx *ctx, octo_tree *t, int level, const octo_opts &o, const octo_scf_params &p, int64_t s2,
             int iterations, double *rho_out, double *phi_out, octo_scf_state *history) {
    const ScfConst k = make_const(level, p);
    const int np = parts_for(k.cells);
    hipStream_t q = ctx->stream;
    Scratch s(ctx, iterations, 3 * k.cells);
    double *rho = t->rho;  // the tree's density: the solve reads it in place
    std::vector<TreeDesc> want = t->plan.trees_host;
    want[0].phi = phi_out;
    want[0].g = s.g;
    want[0].G = p.G;
    want[0].amc = o.amc ? 1 : 0;
    auto solve = [&] { run_plan(ctx, t->plan, t->graphs, want, &o, false); };

    hipLaunchKernelGGL(k_scf_init, dim3(1), dim3(1), 0, q, s.st, s2, p.K0);
    pass<0>(k, s, np, rho, nullptr, q);
    for (int it = 0; it < iterations; ++it) {
        normalise(k, s, np, rho, it > 0, q);  // step 1
        solve();                               // step 7 of the previous iteration
        finish_step(k, s, np, rho, phi_out, rho, s.hist + it, q);  // steps 4-6 (2-3 in the moments)
    }
    normalise(k, s, np, rho, iterations > 0, q);
    solve();
    if (rho_out)
        check_hip(hipMemcpyAsync(rho_out, rho, (size_t)k.cells * 8, hipMemcpyDeviceToDevice, q), "density copy");
    if (history && iterations > 0)
        check_hip(hipMemcpyAsync(history, s.hist, (size_t)iterations * sizeof(octo_scf_state),
                                 hipMemcpyDeviceToHost, q),
                  "history copy");
    tree_release(t, q);
    check_hip(hipStreamSynchronize(q), "scf run");
}

}  // namespace octo
