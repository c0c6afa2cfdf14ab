// Register-resident mass-matrix solve for 2D FP32 problems that fit the chip.
//
// Same mathematics as k_cg.hip (mixed-precision iterative refinement: FP64
// solution and residual outside, FP32 conjugate gradients with FP64 dot products
// inside), organised around the cost of grid-wide synchronisation on a
// multi-die GPU:
//
//  * every workgroup owns one tile of RX x RY nodes for the whole solve and keeps
//    its CG vectors (p, s, r, w and the correction d per field) in registers and
//    the tile's stencil coefficients in LDS; the FP64 solution stays in
//    owner-only global memory; within the tile, neighbours are exchanged through
//    LDS;
//  * across tiles only the boundary values travel, published to full-size
//    exchange arrays with device-coherent stores and read back with
//    device-coherent loads, so no cache flush is ever needed;
//  * the inner CG is the Chronopoulos-Gear variant: both dot products of an
//    iteration are reduced together, so an iteration needs one grid barrier.
//    The new residual r' = r - alpha (w + beta s) of a neighbour tile's boundary
//    node is recomputed from its published (r, w, s) with the same FP32
//    operations its owner uses, so the halo is bit-identical;
//  * the grid barrier is a two-level arrival tree on counters (no single
//    serialised atomic); the last arriving workgroup reduces the per-workgroup
//    FP64 partials in a fixed order and publishes the totals, so every workgroup
//    takes identical decisions and the result is deterministic.
//  Every wait is bounded: a timed-out wait raises an abort flag that ends the
//  solve in every workgroup.
#include "p2m_internal.hpp"

namespace p2m {

namespace {

constexpr int RX = 128;           // tile width in nodes
constexpr int RY = 32;            // tile height
constexpr int RNPT = 8;           // nodes per thread
constexpr int RBS = RX * RY / RNPT;  // threads per workgroup; a wave covers RNPT/2 rows
constexpr int LW = RX + 2;        // LDS row stride including the halo ring
constexpr int LH = RY + 2;
constexpr int kGroups = 16;       // fan-in of the first barrier level
constexpr int kNV = 3 * kMaxFields;
constexpr long kSpinMax = 1L << 22;

struct RSync {
    unsigned* ctr;    // [kGroups * 32] group arrival counters (128-byte apart)
    unsigned* root;   // root arrival counter
    unsigned* rel;    // release epoch
    unsigned* abort;  // set on a timed-out wait
    double* part;     // [2][nblocks][kNV] per-workgroup partials
    double* tot;      // [2][kNV] totals
};

struct RArgs {
    Mesh m;
    int tiles_x;
    float* coef;       // [4][nn]  D, E, N, NE  (orphan diagonals set to 1 here)
    float* b;          // [F][nn]  (orphan entries set to 0 here)
    const float* w;    // [nn]
    float* xout;       // [F][nn]  start (USER) on entry, result on exit
    double* x64;       // [F][nn]  FP64 solution, owner-only
    float* pubR;       // [2][F][nn] published boundary values
    float* pubW;
    float* pubS;
    double* pubX;      // [F][nn]
    RSync sy;
    int start;
    p2m_solve_opts opts;
    p2m_report* rep;
};

// device-coherent (L2-bypassing) accesses for data that crosses workgroups
__device__ __forceinline__ void st_c(float* p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_c(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_c(const float* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_c(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_c(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Buffer-resource accesses: a 128-bit descriptor (base, size) in scalar
// registers plus a 32-bit element offset, so the per-node offsets are shared by
// all arrays.  AUX 0 = plain (owner-only data), 16 = device-coherent (sc1).
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kPlain = 0, kCoherent = 16;
__device__ __forceinline__ rsrc_t mkrs(const void* p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}
template <int AUX>
__device__ __forceinline__ float ldf(rsrc_t r, int i) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ void stf(rsrc_t r, int i, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, i * 4, 0, AUX);
}
template <int AUX>
__device__ __forceinline__ double ldd(rsrc_t r, int i) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ void std8(rsrc_t r, int i, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, i * 8, 0, AUX);
}

// Block sum of NV doubles per thread in a fixed order; totals land in out[0..NV).
template <int NV>
__device__ __forceinline__ void block_sum_to(double (&v)[NV], double* lds /* [RBS/64][NV] */,
                                             double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double s = v[j];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_down(s, d, 64);
        if (lane == 0) lds[wave * NV + j] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int wv = 0; wv < RBS / 64; ++wv) s += lds[wv * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Grid barrier that also sums the workgroups' partials vals[0..nv) (FP64).  On
// return vals[0..nv) holds the totals in every workgroup.  Returns false after
// an abort.
__device__ bool sync_reduce(const RSync& s, unsigned epoch, double* vals, int nv, int nblocks) {
    __shared__ int s_role;
    __shared__ int s_ok;
    double* part = s.part + (size_t)(epoch & 1) * nblocks * kNV;
    double* tot = s.tot + (size_t)(epoch & 1) * kNV;
    if (threadIdx.x < nv) st_c(&part[(size_t)blockIdx.x * kNV + threadIdx.x], vals[threadIdx.x]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int ng = nblocks < kGroups ? nblocks : kGroups;
    if (threadIdx.x == 0) {
        int role = 0;
        const int g = blockIdx.x % kGroups;
        const unsigned gsize = (unsigned)((nblocks - g + kGroups - 1) / kGroups);
        const unsigned old = __hip_atomic_fetch_add(&s.ctr[g * 32], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == epoch * gsize) {
            const unsigned o2 = __hip_atomic_fetch_add(s.root, 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            if (o2 + 1 == epoch * (unsigned)ng) role = 1;
        }
        s_role = role;
    }
    __syncthreads();
    if (s_role) {
        // the last arriver: value j is summed by the 32 lanes of segment j, lane l
        // over blocks l, l+32, ..., then a fixed shuffle tree
        const int seg = threadIdx.x >> 5, l = threadIdx.x & 31;
        for (int jv = seg; jv < kNV; jv += RBS / 32) {
            double acc = 0.0;
            if (jv < nv)
                for (int bk = l; bk < nblocks; bk += 32) acc += ld_c(&part[(size_t)bk * kNV + jv]);
#pragma unroll
            for (int d = 16; d >= 1; d >>= 1) acc += __shfl_down(acc, d, 32);
            if (jv < nv && l == 0) st_c(&tot[jv], acc);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(s.rel, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) {
        int ok = 1;
        long spins = 0;
        while (ld_c(s.rel) < epoch) {
            if (ld_c(s.abort) != 0u || ++spins > kSpinMax) {
                __hip_atomic_store(s.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    if (threadIdx.x < nv) vals[threadIdx.x] = ld_c(&tot[threadIdx.x]);
    __syncthreads();
    return s_ok != 0;
}

// global index of local tile coordinate (lc, lr), periodic
__device__ __forceinline__ int gidx(const Mesh& m, int i0, int j0, int lc, int lr) {
    int gc = i0 + lc, gr = j0 + lr;
    if (gc < 0) gc += m.nx;
    if (gc >= m.nx) gc -= m.nx;
    if (gr < 0) gr += m.ny;
    if (gr >= m.ny) gr -= m.ny;
    return gc + m.nx * gr;
}

// halo slot h -> local (lc, lr) on the ring around a TXa x TYa tile
__device__ __forceinline__ bool halo_slot(int h, int txa, int tya, int& lc, int& lr) {
    const int row = txa + 2;
    if (h < row) { lr = -1; lc = h - 1; return true; }
    h -= row;
    if (h < row) { lr = tya; lc = h - 1; return true; }
    h -= row;
    if (h < tya) { lc = -1; lr = h; return true; }
    h -= tya;
    if (h < tya) { lc = txa; lr = h; return true; }
    return false;
}

__device__ __forceinline__ bool on_boundary(int lc, int lr, int txa, int tya) {
    return lc == 0 || lr == 0 || lc == txa - 1 || lr == tya - 1;
}

template <int F>
__global__ __launch_bounds__(RBS) void k_cgr(RArgs a) {
    const Mesh& m = a.m;
    const int nn = m.nn;
    const int nblocks = gridDim.x;
    const int tile = blockIdx.x;
    const int i0 = (tile % a.tiles_x) * RX;
    const int j0 = (tile / a.tiles_x) * RY;
    const int txa = min(RX, m.nx - i0), tya = min(RY, m.ny - j0);
    // node j of this thread: tile row (RNPT/2)*wave + j/2, column lane + 64*(j%2);
    // a wave covers whole rows, so every global access of a wave is a 64-wide
    // contiguous run and LDS accesses are conflict-free
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = (RNPT / 2) * wave;
    const int nhalo = 2 * (txa + 2) + 2 * tya;
    auto nrow = [&](int j) { return row0 + (j >> 1); };
    auto ncol = [&](int j) { return lane + 64 * (j & 1); };
    auto active = [&](int j) { return nrow(j) < tya && ncol(j) < txa; };
    const int kb = (j0 + row0) * m.nx + i0 + lane;  // global index of node 0
    auto gk = [&](int j) { return kb + (j >> 1) * m.nx + 64 * (j & 1); };
    // per-field descriptors of the owner-only and the published arrays
    const size_t fb4 = (size_t)nn * 4, fb8 = (size_t)nn * 8;
    auto rs_x64 = [&](int f) { return mkrs(a.x64 + (size_t)f * nn, fb8); };
    auto rs_d = [&](int f) { return mkrs(a.xout + (size_t)f * nn, fb4); };
    auto rs_b = [&](int f) { return mkrs(a.b + (size_t)f * nn, fb4); };
    auto rs_pubX = [&](int f) { return mkrs(a.pubX + (size_t)f * nn, fb8); };
    auto rs_pub = [&](float* base, int par, int f) {
        return mkrs(base + ((size_t)par * F + f) * nn, fb4);
    };

    // LDS: stencil coefficients of the tile plus its left column and bottom row,
    // and one exchange area used as F FP32 planes or as one FP64 plane
    constexpr int CW = RX + 1, CN = (RY + 1) * (RX + 1);
    constexpr size_t XB = (size_t)F * LH * LW * sizeof(float) > (size_t)LH * LW * sizeof(double)
                              ? (size_t)F * LH * LW * sizeof(float)
                              : (size_t)LH * LW * sizeof(double);
    __shared__ float cf[4 * CN];
    __shared__ __align__(16) unsigned char xbuf[XB];
    float* lf = (float*)xbuf;       // plane f at lf + f * LH * LW
    double* ld64 = (double*)xbuf;
    __shared__ double red_lds[(RBS / 64) * kNV];
    __shared__ double vals[kNV];
    __shared__ double s_bb[F], s_gam[F], s_alpha[F], s_relres[F], s_target[F];
    __shared__ float s_af[F], s_bf[F];
    __shared__ int s_iters[F], s_refines[F], s_done[F], s_inner[F], s_zero[F];
    __shared__ uint32_t s_flags;
    __shared__ int s_any;

    auto lidx = [&](int lc, int lr) { return (lr + 1) * LW + (lc + 1); };
    // per-field flags read once into a register after each decision point
    auto inner_mask = [&]() {
        uint32_t mk = 0;
#pragma unroll
        for (int f = 0; f < F; ++f)
            if (s_inner[f]) mk |= 1u << f;
        return mk;
    };
    auto cidx = [&](int lc, int lr) { return (lr + 1) * CW + (lc + 1); };
    const int q0 = lidx(lane, row0);   // LDS index of node 0; node j: + (j/2)*LW + 64*(j%2)
    const int qc0 = cidx(lane, row0);
    auto qj = [&](int j) { return q0 + (j >> 1) * LW + 64 * (j & 1); };
    auto qcj = [&](int j) { return qc0 + (j >> 1) * CW + 64 * (j & 1); };

    float vp[F][RNPT], vd[F][RNPT], vs[F][RNPT], vr[F][RNPT], vw[F][RNPT];

    if (threadIdx.x < F) {
        const int f = threadIdx.x;
        s_iters[f] = 0; s_refines[f] = 0; s_done[f] = 0; s_inner[f] = 0; s_zero[f] = 0;
        s_relres[f] = 0.0; s_bb[f] = 0.0;
    }
    if (threadIdx.x == 0) s_flags = 0u;

    uint32_t amask = 0, bmask = 0;  // active nodes; active nodes on the tile boundary
#pragma unroll
    for (int j = 0; j < RNPT; ++j) {
        if (!active(j)) continue;
        amask |= 1u << j;
        const int lc = ncol(j), lr = nrow(j);
        if (lc == 0 || lr == 0 || lc == txa - 1 || lr == tya - 1) bmask |= 1u << j;
    }

    // ---- P: coefficients into LDS, orphan regularisation, FP64 start vector ----
#pragma unroll
    for (int j = 0; j < RNPT; ++j) {
        if (!(amask & (1u << j))) continue;
        const int k = gk(j);
        const int q = qcj(j);
        const float wk = a.w[k];
        const bool orphan = !(wk > 0.f);
        if (orphan) a.coef[k] = 1.f;
        cf[q] = orphan ? 1.f : a.coef[k];
        cf[CN + q] = a.coef[(size_t)nn + k];
        cf[2 * CN + q] = a.coef[(size_t)2 * nn + k];
        cf[3 * CN + q] = a.coef[(size_t)3 * nn + k];
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const size_t o = (size_t)f * nn + k;
            double x0;
            if (orphan) {
                a.b[o] = 0.f;
                x0 = 0.0;
            } else if (a.start == P2M_START_FLIP) {
                x0 = (double)a.b[o] / (double)wk;
            } else if (a.start == P2M_START_ZERO) {
                x0 = 0.0;
            } else {
                x0 = (double)a.xout[o];
            }
            a.x64[o] = x0;
            a.xout[o] = 0.f;  // xout holds the FP32 correction d during the solve
        }
        if (orphan && a.rep) {
            atomicAdd(&a.rep->n_orphan, 1);
            atomicOr(&a.rep->flags, (uint32_t)P2M_FLAG_ORPHAN);
        }
    }
    // left column / bottom row: only their E, N, NE are used, never modified here
    for (int h = threadIdx.x; h < txa + 1 + tya; h += RBS) {
        int lc, lr;
        if (h < txa + 1) { lr = -1; lc = h - 1; } else { lc = -1; lr = h - (txa + 1); }
        const int k = gidx(m, i0, j0, lc, lr);
        const int q = cidx(lc, lr);
        cf[CN + q] = a.coef[(size_t)nn + k];
        cf[2 * CN + q] = a.coef[(size_t)2 * nn + k];
        cf[3 * CN + q] = a.coef[(size_t)3 * nn + k];
    }
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
        for (int j = 0; j < RNPT; ++j) vp[f][j] = vd[f][j] = vs[f][j] = vr[f][j] = vw[f][j] = 0.f;
    __syncthreads();

    unsigned epoch = 0;
    int ex = 0;  // exchange parity of pubR / pubW / pubS
    bool alive = true;

    // w = M r at the owned nodes for every inner-active field (r in the exchange
    // planes); node-major so each node's seven coefficients are read once
    auto spmv_all = [&](uint32_t imask) {
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            const int qc = qcj(j), q = qj(j);
            const float cD = cf[qc], cE = cf[CN + qc], cEw = cf[CN + qc - 1];
            const float cN = cf[2 * CN + qc], cNs = cf[2 * CN + qc - CW];
            const float cNE = cf[3 * CN + qc], cNEsw = cf[3 * CN + qc - CW - 1];
            const bool on = amask & (1u << j);
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                const float* L = lf + (size_t)f * LH * LW;
                float acc = cD * L[q];
                acc = fmaf(cE, L[q + 1], acc);
                acc = fmaf(cEw, L[q - 1], acc);
                acc = fmaf(cN, L[q + LW], acc);
                acc = fmaf(cNs, L[q - LW], acc);
                acc = fmaf(cNE, L[q + LW + 1], acc);
                acc = fmaf(cNEsw, L[q - LW - 1], acc);
                vw[f][j] = on ? acc : 0.f;
            }
        }
    };

    for (int outer = 0; alive; ++outer) {
        // ---- fold the correction into x64, publish the boundary x64 ------------
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (s_done[f]) continue;
            const rsrc_t rx = rs_x64(f), rpx = rs_pubX(f);
#pragma unroll
            for (int j = 0; j < RNPT; ++j) {
                if (!(amask & (1u << j))) continue;
                const int kk = gk(j);
                const double xv = ldd<kPlain>(rx, kk) + (double)vd[f][j];
                std8<kPlain>(rx, kk, xv);
                if (bmask & (1u << j)) std8<kCoherent>(rpx, kk, xv);
            }
#pragma unroll
            for (int j = 0; j < RNPT; ++j) vd[f][j] = 0.f;
        }
        __syncthreads();
        alive = sync_reduce(a.sy, ++epoch, vals, 0, nblocks);
        if (!alive) break;

        // ---- R: r = b - M x64 in FP64; r_T = (float) r -------------------------
        {
            double pr[3 * F];
#pragma unroll
            for (int q = 0; q < 3 * F; ++q) pr[q] = 0.0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (s_done[f]) continue;
                const rsrc_t rx = rs_x64(f), rpx = rs_pubX(f), rb = rs_b(f), rd = rs_d(f);
                const rsrc_t rpr = rs_pub(a.pubR, ex, f);
#pragma unroll
                for (int j = 0; j < RNPT; ++j)
                    if (amask & (1u << j)) ld64[qj(j)] = ldd<kPlain>(rx, gk(j));
                for (int h = threadIdx.x; h < nhalo; h += RBS) {
                    int lc, lr;
                    if (!halo_slot(h, txa, tya, lc, lr)) continue;
                    ld64[lidx(lc, lr)] = ldd<kCoherent>(rpx, gidx(m, i0, j0, lc, lr));
                }
                __syncthreads();
                // the FP32 residual goes to the (now free) correction array xout and
                // is loaded into registers after the barrier
#pragma unroll 1
                for (int j = 0; j < RNPT; ++j) {
                    if (!(amask & (1u << j))) continue;
                    const int q = qj(j), qc = qcj(j);
                    const double mx = (double)cf[qc] * ld64[q] + (double)cf[CN + qc] * ld64[q + 1] +
                                      (double)cf[CN + qc - 1] * ld64[q - 1] +
                                      (double)cf[2 * CN + qc] * ld64[q + LW] +
                                      (double)cf[2 * CN + qc - CW] * ld64[q - LW] +
                                      (double)cf[3 * CN + qc] * ld64[q + LW + 1] +
                                      (double)cf[3 * CN + qc - CW - 1] * ld64[q - LW - 1];
                    const int kk = gk(j);
                    const double bk = (double)ldf<kPlain>(rb, kk);
                    const double r64 = bk - mx;
                    const float rt = (float)r64;
                    stf<kPlain>(rd, kk, rt);
                    pr[f] += r64 * r64;
                    pr[F + f] += (double)rt * (double)rt;
                    if (outer == 0) pr[2 * F + f] += bk * bk;
                    if (bmask & (1u << j)) stf<kCoherent>(rpr, kk, rt);
                }
                __syncthreads();
            }
            block_sum_to<3 * F>(pr, red_lds, vals);
        }
        alive = sync_reduce(a.sy, ++epoch, vals, 3 * F, nblocks);
        if (!alive) break;
        if (threadIdx.x == 0) {
            int any = 0;
            for (int f = 0; f < F; ++f) {
                if (s_done[f]) continue;
                s_refines[f] += 1;
                if (outer == 0) s_bb[f] = vals[2 * F + f];
                const double bb = s_bb[f];
                if (bb == 0.0) {
                    s_zero[f] = 1; s_done[f] = 1; s_relres[f] = 0.0;
                    continue;
                }
                const double rr = vals[f];
                const double relres = sqrt(rr / bb);
                s_relres[f] = relres;
                if (relres <= a.opts.tol || outer >= a.opts.max_refine ||
                    s_iters[f] >= a.opts.maxit || !(relres == relres)) {
                    s_done[f] = 1;
                    if (!(relres <= a.opts.tol)) s_flags |= P2M_FLAG_NOT_CONVERGED;
                    continue;
                }
                s_gam[f] = vals[F + f];
                const double goal = 0.25 * a.opts.tol * a.opts.tol * bb;
                const double rel = a.opts.inner_rtol * a.opts.inner_rtol * rr;
                s_target[f] = goal > rel ? goal : rel;
                s_inner[f] = 1;
                any = 1;
            }
            s_any = any;
        }
        __syncthreads();
        if (!s_any) break;

        // ---- CG start: w = M r, delta = (w, r); p = s = d = 0 -------------------
        uint32_t imask = inner_mask();
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (!(imask & (1u << f))) continue;
            float* L = lf + (size_t)f * LH * LW;
            const rsrc_t rd = rs_d(f);
#pragma unroll
            for (int j = 0; j < RNPT; ++j) {
                vr[f][j] = 0.f;
                if (amask & (1u << j)) {
                    vr[f][j] = ldf<kPlain>(rd, gk(j));
                    stf<kPlain>(rd, gk(j), 0.f);
                    L[qj(j)] = vr[f][j];
                }
            }
        }
        for (int h = threadIdx.x; h < nhalo; h += RBS) {
            int lc, lr;
            if (!halo_slot(h, txa, tya, lc, lr)) continue;
            const int gh = gidx(m, i0, j0, lc, lr);
            float hv[F];
#pragma unroll
            for (int f = 0; f < F; ++f) hv[f] = ldf<kCoherent>(rs_pub(a.pubR, ex, f), gh);
#pragma unroll
            for (int f = 0; f < F; ++f)
                if (imask & (1u << f)) lf[(size_t)f * LH * LW + lidx(lc, lr)] = hv[f];
        }
        __syncthreads();
        ex ^= 1;
        {
            spmv_all(imask);
            double pd[F];
#pragma unroll
            for (int f = 0; f < F; ++f) pd[f] = 0.0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                const rsrc_t rr = rs_pub(a.pubR, ex, f), rw = rs_pub(a.pubW, ex, f),
                             rs = rs_pub(a.pubS, ex, f);
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    vs[f][j] = 0.f;
                    vp[f][j] = 0.f;
                    vd[f][j] = 0.f;
                    if (!(amask & (1u << j))) continue;
                    pd[f] += (double)vw[f][j] * (double)vr[f][j];
                    if (bmask & (1u << j)) {
                        stf<kCoherent>(rr, gk(j), vr[f][j]);
                        stf<kCoherent>(rw, gk(j), vw[f][j]);
                        stf<kCoherent>(rs, gk(j), 0.f);
                    }
                }
            }
            __syncthreads();
            block_sum_to<F>(pd, red_lds, vals);
        }
        alive = sync_reduce(a.sy, ++epoch, vals, F, nblocks);
        if (!alive) break;
        if (threadIdx.x == 0) {
            for (int f = 0; f < F; ++f) {
                if (!s_inner[f]) continue;
                if (!(vals[f] > 0.0)) {
                    s_inner[f] = 0; s_done[f] = 1;
                    s_flags |= P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED;
                    continue;
                }
                s_alpha[f] = s_gam[f] / vals[f];
                s_af[f] = (float)s_alpha[f];
                s_bf[f] = 0.f;
            }
        }
        __syncthreads();

        // ---- inner iterations (one barrier each) -------------------------------
        while (alive) {
            imask = inner_mask();
            float af[F], bf[F];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                af[f] = s_af[f];
                bf[f] = s_bf[f];
            }
            // halo first (its loads are the longest latency): the neighbours' new
            // residual from their published state, all fields' loads in flight
            for (int h = threadIdx.x; h < nhalo; h += RBS) {
                int lc, lr;
                if (!halo_slot(h, txa, tya, lc, lr)) continue;
                const int gh = gidx(m, i0, j0, lc, lr);
                float ro[F], wo[F], so[F];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    ro[f] = ldf<kCoherent>(rs_pub(a.pubR, ex, f), gh);
                    wo[f] = ldf<kCoherent>(rs_pub(a.pubW, ex, f), gh);
                    so[f] = ldf<kCoherent>(rs_pub(a.pubS, ex, f), gh);
                }
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    if (!(imask & (1u << f))) continue;
                    const float sn = fmaf(bf[f], so[f], wo[f]);
                    lf[(size_t)f * LH * LW + lidx(lc, lr)] = fmaf(-af[f], sn, ro[f]);
                }
            }
            // local updates and the new residual into LDS
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                const float al = af[f], be = bf[f];
                float* L = lf + (size_t)f * LH * LW;
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    vp[f][j] = fmaf(be, vp[f][j], vr[f][j]);
                    vd[f][j] = fmaf(al, vp[f][j], vd[f][j]);
                    vs[f][j] = fmaf(be, vs[f][j], vw[f][j]);
                    vr[f][j] = fmaf(-al, vs[f][j], vr[f][j]);
                    if (amask & (1u << j)) L[qj(j)] = vr[f][j];
                }
            }
            __syncthreads();
            ex ^= 1;
            {
                spmv_all(imask);
                double pg[2 * F];
#pragma unroll
                for (int q = 0; q < 2 * F; ++q) pg[q] = 0.0;
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    if (!(imask & (1u << f))) continue;
                    const rsrc_t rr = rs_pub(a.pubR, ex, f), rw = rs_pub(a.pubW, ex, f),
                                 rs = rs_pub(a.pubS, ex, f);
#pragma unroll
                    for (int j = 0; j < RNPT; ++j) {
                        if (!(amask & (1u << j))) continue;
                        pg[f] += (double)vr[f][j] * (double)vr[f][j];
                        pg[F + f] += (double)vw[f][j] * (double)vr[f][j];
                        if (bmask & (1u << j)) {
                            stf<kCoherent>(rr, gk(j), vr[f][j]);
                            stf<kCoherent>(rw, gk(j), vw[f][j]);
                            stf<kCoherent>(rs, gk(j), vs[f][j]);
                        }
                    }
                }
                __syncthreads();
                block_sum_to<2 * F>(pg, red_lds, vals);
            }
            alive = sync_reduce(a.sy, ++epoch, vals, 2 * F, nblocks);
            if (!alive) break;
            if (threadIdx.x == 0) {
                int any = 0;
                for (int f = 0; f < F; ++f) {
                    if (!s_inner[f]) continue;
                    const double gam = vals[f], del = vals[F + f];
                    s_iters[f] += 1;
                    if (!(gam > s_target[f]) || s_iters[f] >= a.opts.maxit) {
                        s_inner[f] = 0;
                        continue;
                    }
                    const double beta = gam / s_gam[f];
                    const double den = del - beta * gam / s_alpha[f];
                    if (!(den > 0.0) || !(gam == gam)) {
                        s_inner[f] = 0;
                        s_flags |= P2M_FLAG_BREAKDOWN;
                        continue;
                    }
                    s_alpha[f] = gam / den;
                    s_gam[f] = gam;
                    s_af[f] = (float)s_alpha[f];
                    s_bf[f] = (float)beta;
                    any = 1;
                }
                s_any = any;
            }
            __syncthreads();
            if (!s_any) break;
        }
    }

    if (!alive && threadIdx.x == 0) s_flags |= P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED;
    __syncthreads();
    // result: the FP64 solution rounded to FP32 (0 for fields with b == 0)
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const rsrc_t rx = rs_x64(f), rd = rs_d(f);
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            if (!(amask & (1u << j))) continue;
            stf<kPlain>(rd, gk(j), s_zero[f] ? 0.f : (float)ldd<kPlain>(rx, gk(j)));
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.rep) {
        for (int f = 0; f < F; ++f) {
            a.rep->iters[f] = s_iters[f];
            a.rep->refines[f] = s_refines[f];
            a.rep->rel_residual[f] = s_relres[f];
        }
        if (s_flags) atomicOr(&a.rep->flags, s_flags);
    }
}

__global__ void k_sync_clear(unsigned* ctr, unsigned* root, unsigned* rel, unsigned* abort_) {
    const int t = threadIdx.x;
    if (t < kGroups * 32) ctr[t] = 0u;
    if (t < 32) { root[t] = 0u; rel[t] = 0u; abort_[t] = 0u; }
}

const void* cgr_kernel(int F) {
    switch (F) {
        case 1: return (const void*)k_cgr<1>;
        case 2: return (const void*)k_cgr<2>;
        case 3: return (const void*)k_cgr<3>;
    }
    return nullptr;
}

}  // namespace

// workspace bytes of the register-resident solve (beyond b, w, coef and x)
size_t cgr_workspace_bytes(const Mesh& m, int F, int blocks) {
    auto al = [](size_t v) { return (v + kAlign - 1) / kAlign * kAlign; };
    size_t s = 0;
    s += al((size_t)F * m.nn * sizeof(double));           // x64
    s += 3 * al((size_t)2 * F * m.nn * sizeof(float));    // pubR, pubW, pubS
    s += al((size_t)F * m.nn * sizeof(double));           // pubX
    s += al((size_t)kGroups * 32 * sizeof(unsigned));     // ctr
    s += 3 * al(32 * sizeof(unsigned));                   // root, rel, abort
    s += al((size_t)2 * blocks * kNV * sizeof(double));   // part
    s += al((size_t)2 * kNV * sizeof(double));            // tot
    return s;
}

int cgr_tiles(const Mesh& m) { return ((m.nx + RX - 1) / RX) * ((m.ny + RY - 1) / RY); }

bool cgr_supported(const Mesh& m, int F, int device) {
    if (m.dim != 2 || F < 1 || F > 3) return false;
    int cus = 0, per = 0, coop = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess ||
        !coop)
        return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, cgr_kernel(F), RBS, 0) != hipSuccess)
        return false;
    return cgr_tiles(m) <= per * cus;
}

hipError_t launch_cg_resident(const Mesh& m, int F, float* coef, float* b, const float* w,
                              float* x, int start, void* ws, const p2m_solve_opts& opts,
                              p2m_report* rep, hipStream_t stream) {
    auto al = [](size_t v) { return (v + kAlign - 1) / kAlign * kAlign; };
    const int blocks = cgr_tiles(m);
    char* p = (char*)ws;
    RArgs a;
    a.m = m;
    a.tiles_x = (m.nx + RX - 1) / RX;
    a.coef = coef;
    a.b = b;
    a.w = w;
    a.xout = x;
    a.start = start;
    a.opts = opts;
    a.rep = rep;
    a.x64 = (double*)p; p += al((size_t)F * m.nn * sizeof(double));
    a.pubR = (float*)p; p += al((size_t)2 * F * m.nn * sizeof(float));
    a.pubW = (float*)p; p += al((size_t)2 * F * m.nn * sizeof(float));
    a.pubS = (float*)p; p += al((size_t)2 * F * m.nn * sizeof(float));
    a.pubX = (double*)p; p += al((size_t)F * m.nn * sizeof(double));
    a.sy.ctr = (unsigned*)p; p += al((size_t)kGroups * 32 * sizeof(unsigned));
    a.sy.root = (unsigned*)p; p += al(32 * sizeof(unsigned));
    a.sy.rel = (unsigned*)p; p += al(32 * sizeof(unsigned));
    a.sy.abort = (unsigned*)p; p += al(32 * sizeof(unsigned));
    a.sy.part = (double*)p; p += al((size_t)2 * blocks * kNV * sizeof(double));
    a.sy.tot = (double*)p;
    hipLaunchKernelGGL(k_sync_clear, dim3(1), dim3(kGroups * 32), 0, stream, a.sy.ctr, a.sy.root,
                       a.sy.rel, a.sy.abort);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void* fn = cgr_kernel(F);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(RBS), args, 0, stream);
}

}  // namespace p2m
