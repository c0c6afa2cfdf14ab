// Device-side pieces shared by the two tile solvers (k_cgr.hip: one tile per
// workgroup, state in registers; k_cgb.hip: several tiles and instances per
// workgroup, state streamed): the tile geometry, the device-coherent accesses,
// buffer descriptors, the fixed-order block and grid reductions and the
// two-level barrier.  Both solvers take every floating-point decision through
// these helpers, so a tile computes the same bits in either kernel.
#pragma once

#include "p2m_internal.hpp"

namespace p2m {

namespace {

constexpr int RX = kSolveTileX;     // tile width in nodes
constexpr int RY = kSolveTileY;     // tile height
constexpr int RNPT = 8;           // nodes per thread
constexpr int RBS = RX * RY / RNPT;  // threads per workgroup; a wave covers RNPT/2 rows
constexpr int LW = RX + 2;        // LDS row stride including the halo ring
constexpr int LH = RY + 2;
constexpr int kGroups = 16;       // fan-in of the first barrier level
constexpr int kNV = 3 * kMaxFields;

struct RSync {
    unsigned* ctr;    // [kGroups * 32] group arrival counters (128-byte apart)
    unsigned* root;   // root arrival counter
    unsigned* rel;    // [kGroups * 32] release epoch, one copy per group (128-byte apart)
    unsigned* abort;  // set on a timed-out wait
    double* part;     // [2][nblocks][kNV] per-workgroup partials
    double* tot;      // [2][kNV] totals
    long spin;        // polls before a wait gives up (kSolveSpinDefault; < 0: at once)
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

// Lane moves of a double through the VALU's data-parallel primitives (DPP), both
// halves; every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const u32x2 u = __builtin_bit_cast(u32x2, v);
    u32x2 r;
    r.x = (unsigned)__builtin_amdgcn_mov_dpp((int)u.x, CTRL, 0xF, 0xF, false);
    r.y = (unsigned)__builtin_amdgcn_mov_dpp((int)u.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const u32x2 u = __builtin_bit_cast(u32x2, v);
    u32x2 r;
    r.x = (unsigned)__builtin_amdgcn_readlane((int)u.x, lane);
    r.y = (unsigned)__builtin_amdgcn_readlane((int)u.y, lane);
    return __builtin_bit_cast(double, r);
}
// Sum over each 16-lane row of the wave, exact in the row's first lane: lane pairs,
// then quads, then quads two apart (row rotation by 4), then the row's halves
// (rotation by 8).  Register-to-register moves: no LDS round trip per step.
__device__ __forceinline__ double row_sum16(double s) {
    s += dpp_d<0xB1>(s);    // quad_perm [1,0,3,2]
    s += dpp_d<0x4E>(s);    // quad_perm [2,3,0,1]
    s += dpp_d<0x124>(s);   // row_ror:4
    s += dpp_d<0x128>(s);   // row_ror:8
    return s;
}

// A boundary column's (r, w, s) are published as one record per node (r at f, w at
// F + f, s at 2F + f, padded to whole 16-byte units): a neighbour reads a ring
// column slot with dwordx4 loads from one place instead of 3F scattered words.  The
// boundary rows stay in field planes, where a wave's accesses are contiguous.
constexpr int rec_floats(int F) { return (3 * F + 3) / 4 * 4; }
struct F4 {
    float v[4];
};
// 16 bytes at byte offset vo + so (so uniform, kept out of the per-lane address); the
// result is read through a bit cast to a plain struct (element access on the
// builtin's vector result is lowered to a single-dword load by this compiler)
template <int AUX>
__device__ __forceinline__ void ld4f(rsrc_t r, int vo, int so, float* o) {
    const F4 q = __builtin_bit_cast(F4, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, AUX));
    o[0] = q.v[0];
    o[1] = q.v[1];
    o[2] = q.v[2];
    o[3] = q.v[3];
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int AUX>
__device__ __forceinline__ void st4f(rsrc_t r, int vo, int so, const float* v) {
    u32x4 q;
    q.x = __builtin_bit_cast(unsigned, v[0]);
    q.y = __builtin_bit_cast(unsigned, v[1]);
    q.z = __builtin_bit_cast(unsigned, v[2]);
    q.w = __builtin_bit_cast(unsigned, v[3]);
    __builtin_amdgcn_raw_buffer_store_b128(q, r, vo, so, AUX);
}
template <int AUX>
__device__ __forceinline__ void st1f(rsrc_t r, int vo, int so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, AUX);
}

// Block sum of NV doubles per thread in a fixed order; totals land in out[0..NV).
// Per wave: the four row sums (row_sum16) added as (r0 + r1) + (r2 + r3); then the
// waves' sums in wave order.
template <int NV>
__device__ __forceinline__ void block_sum_to(double (&v)[NV], double* lds /* [RBS/64][NV] */,
                                             double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double r = row_sum16(v[j]);
        const double s = (readlane_d(r, 0) + readlane_d(r, 16)) + (readlane_d(r, 32) + readlane_d(r, 48));
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

// Sum of the partials (bk, jv) over bk < nblocks for every jv < nv, handed to
// out(jv, sum).  The fixed order that every solve uses: value jv is summed by the
// 32 lanes of segment jv, lane l over blocks l, l+32, ... in increasing order, then
// the two row sums of the segment (row_sum16) added in row order.  Called by all
// threads of one workgroup (every wave runs the same number of segment steps, so
// the lane moves see every lane active).  Loads go out kPartBatch at a time before
// they are added (in the same order), so a lane waits once per batch, not once per
// block.
static_assert(kNV % 2 == 0 && (RBS / 32) % 2 == 0 && RBS % 64 == 0,
              "both segments of a wave take the same number of steps");
// Partial (bk, jv) is part[bk * sb + jv * sv]: block-major (sb = kNV, sv = 1) or
// value-major (sb = 1, sv = the block count), where a segment's lanes read
// consecutive words.  The layout changes addresses only, never the order.
template <typename Out>
__device__ __forceinline__ void sum_partials(const double* part, int nblocks, int nv, size_t sb,
                                             size_t sv, Out out) {
    constexpr int kPartBatch = 8;
    const int seg = threadIdx.x >> 5, l = threadIdx.x & 31;
    for (int jv = seg; jv < kNV; jv += RBS / 32) {
        double acc = 0.0;
        if (jv < nv)
            for (int b0 = l; b0 < nblocks; b0 += 32 * kPartBatch) {
                double v[kPartBatch];
#pragma unroll
                for (int u = 0; u < kPartBatch; ++u) {
                    const int bk = b0 + 32 * u;
                    v[u] = bk < nblocks ? ld_c(&part[(size_t)bk * sb + (size_t)jv * sv]) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kPartBatch; ++u)
                    if (b0 + 32 * u < nblocks) acc += v[u];
            }
        const double r = row_sum16(acc);
        const double lo = readlane_d(r, 0) + readlane_d(r, 16);
        const double hi = readlane_d(r, 32) + readlane_d(r, 48);
        if (jv < nv && l == 0) out(jv, (threadIdx.x & 32) ? hi : lo);
    }
}

// Arrival at the two-level barrier tree (thread 0 only): the group counter of
// this workgroup, then, for the last of its group, the root counter.  Counters
// only grow; epoch e is complete when they reach e times their fan-in.  Returns
// true in the last arriving workgroup of the grid.
__device__ __forceinline__ bool tree_arrive(const RSync& s, unsigned epoch, int nblocks) {
    const int ng = nblocks < kGroups ? nblocks : kGroups;
    const int g = blockIdx.x % kGroups;
    const unsigned gsize = (unsigned)((nblocks - g + kGroups - 1) / kGroups);
    const unsigned old = __hip_atomic_fetch_add(&s.ctr[g * 32], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == epoch * gsize) {
        const unsigned o2 = __hip_atomic_fetch_add(s.root, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (o2 + 1 == epoch * (unsigned)ng) return true;
    }
    return false;
}

// Bounded wait for the release of `epoch` (thread 0 only).  A wait that times
// out, or that sees the abort flag, raises the abort flag and returns false.
__device__ __forceinline__ bool tree_wait(const RSync& s, unsigned epoch) {
    long spins = 0;
    const unsigned* rel = s.rel + (blockIdx.x % kGroups) * 32;
    while (ld_c(rel) < epoch) {
        if (ld_c(s.abort) != 0u || ++spins > s.spin) {
            __hip_atomic_store(s.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// The release goes to every group's copy, so each copy is polled by one group's
// workgroups only.
__device__ __forceinline__ void tree_release(const RSync& s, unsigned epoch) {
#pragma unroll
    for (int g = 0; g < kGroups; ++g)
        __hip_atomic_store(s.rel + g * 32, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier that also sums the workgroups' partials vals[0..nv) (FP64).  Every
// workgroup stores its partials, arrives, waits for the release and then sums all
// partials itself in the fixed order of sum_partials, so every workgroup holds
// the same totals without a second exchange.  The partials are double-buffered
// by epoch parity: epoch e + 2 overwrites epoch e's buffer only after every
// workgroup has passed epoch e + 1, i.e. finished reading it.  On return
// vals[0..nv) holds the totals.  Returns false after an abort.
__device__ bool sync_reduce(const RSync& s, unsigned epoch, double* vals, int nv, int nblocks) {
    __shared__ int s_ok;
    const double* part = s.part + (size_t)(epoch & 1) * nblocks * kNV;
    // value-major partials: the readers' lanes of one value read consecutive words
    if (threadIdx.x < nv)
        st_c(&s.part[(size_t)(epoch & 1) * nblocks * kNV + (size_t)threadIdx.x * nblocks + blockIdx.x],
             vals[threadIdx.x]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (tree_arrive(s, epoch, nblocks)) tree_release(s, epoch);
        s_ok = tree_wait(s, epoch) ? 1 : 0;
    }
    __syncthreads();
    const bool ok = s_ok != 0;
    if (ok && nv > 0)
        sum_partials(part, nblocks, nv, 1, (size_t)nblocks, [&](int jv, double v) { vals[jv] = v; });
    __syncthreads();
    return ok;
}

// ---------------------------------------------------------------------------
// Floating-point steps, written with explicit fused operations so that the
// rounding of every value is fixed by the source and not by contraction.
// ---------------------------------------------------------------------------

// FP64 accumulation of the product of two FP32 values (exact product, one
// rounding)
__device__ __forceinline__ double dot_acc(double acc, float a, float b) {
    return __fma_rn((double)a, (double)b, acc);
}
__device__ __forceinline__ double sq_acc(double acc, double a) { return __fma_rn(a, a, acc); }

// FP64 stencil product (M x)_k from seven coefficients and the seven values
// (centre, +x, -x, +y, -y, +x+y, -x-y)
__device__ __forceinline__ double stencil64(float cD, float cE, float cEw, float cN, float cNs,
                                            float cNE, float cNEsw, double x0, double xe,
                                            double xw, double xn, double xs, double xne,
                                            double xsw) {
    double acc = __dmul_rn((double)cD, x0);
    acc = __fma_rn((double)cE, xe, acc);
    acc = __fma_rn((double)cEw, xw, acc);
    acc = __fma_rn((double)cN, xn, acc);
    acc = __fma_rn((double)cNs, xs, acc);
    acc = __fma_rn((double)cNE, xne, acc);
    acc = __fma_rn((double)cNEsw, xsw, acc);
    return acc;
}

// FP32 stencil product, same order
__device__ __forceinline__ float stencil32(float cD, float cE, float cEw, float cN, float cNs,
                                           float cNE, float cNEsw, float x0, float xe, float xw,
                                           float xn, float xs, float xne, float xsw) {
    float acc = __fmul_rn(cD, x0);
    acc = fmaf(cE, xe, acc);
    acc = fmaf(cEw, xw, acc);
    acc = fmaf(cN, xn, acc);
    acc = fmaf(cNs, xs, acc);
    acc = fmaf(cNE, xne, acc);
    acc = fmaf(cNEsw, xsw, acc);
    return acc;
}

// Jacobi preconditioner: the inverse of the regularised diagonal, 1 / M(k,k)
// (correctly rounded), and 1 for an orphan node (w_k == 0, identity row).
__device__ __forceinline__ float jacobi_inv(float diag, float wk) {
    return wk > 0.f ? __frcp_rn(diag) : 1.0f;
}

// Jacobi-preconditioned Chronopoulos-Gear updates of one node, u = r / M(k,k):
// p = u + beta p, d = d + alpha p, s = w + beta s, r = r - alpha s (w = M u of the
// previous iteration).  Returns the new u.
__device__ __forceinline__ float pcg_update(float al, float be, float dinv, float& p, float& d,
                                            float& s, float& r, float w) {
    const float u = __fmul_rn(r, dinv);
    p = fmaf(be, p, u);
    d = fmaf(al, p, d);
    s = fmaf(be, s, w);
    r = fmaf(-al, s, r);
    return __fmul_rn(r, dinv);
}

// a neighbour's new preconditioned residual from its published (r, w, s):
// (r - alpha (w + beta s)) / M(k,k), the same operations as pcg_update
__device__ __forceinline__ float halo_u(float al, float be, float dinv, float r, float w,
                                        float s) {
    return __fmul_rn(fmaf(-al, fmaf(be, s, w), r), dinv);
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

// halo slot h -> local (lc, lr) on the ring around a TXa x TYa tile: the row below,
// the row above (txa + 2 each, corners included), the left column, the right
// column (tya each).  Written with selects: assignments through the references in
// branches were lowered through a stack slot in scratch memory.
__device__ __forceinline__ bool halo_slot(int h, int txa, int tya, int& lc, int& lr) {
    const int row = txa + 2;
    const bool below = h < row, above = !below && h < 2 * row;
    const int hc = h - 2 * row;                 // column part: left, then right
    const bool left = hc < tya;
    lc = below ? h - 1 : (above ? h - row - 1 : (left ? -1 : txa));
    lr = below ? -1 : (above ? tya : (left ? hc : hc - tya));
    return h < 2 * row + 2 * tya;
}

__device__ __forceinline__ bool on_boundary(int lc, int lr, int txa, int tya) {
    return lc == 0 || lr == 0 || lc == txa - 1 || lr == tya - 1;
}


}  // namespace

}  // namespace p2m
