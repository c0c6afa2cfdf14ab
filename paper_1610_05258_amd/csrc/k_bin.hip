// Binning of particles by cell: a stable counting sort.
//
//   locate_count : FP64 locate of every particle, cell key, per-cell counts
//                  (integer atomics: order-independent, so the counts are exact);
//                  the value an atomic returns gives each particle a distinct
//                  slot of its cell (its rank), in an order that depends on timing
//   exclusive_scan: cell_start = exclusive prefix sum of the counts
//   place        : perm[cell_start[key] + rank] = particle (no atomics)
//   segment_sort : every cell sorts its slots by original index, which makes the
//                  permutation exactly the stable (cell, original index) order
//
// The result does not depend on the order in which the atomics were served.
#include "p2m_internal.hpp"

namespace p2m {

namespace {

constexpr int kBlock = kBinBlock;

__global__ void k_report_clear(p2m_report* rep) {
    int t = threadIdx.x;
    if (t < 8) {
        rep->iters[t] = 0;
        rep->refines[t] = 0;
        rep->rel_residual[t] = 0.0;
    }
    if (t == 0) {
        rep->flags = 0u;
        rep->n_orphan = 0;
        rep->n_invalid = 0;
        rep->reserved = 0;
    }
}

// Fill of n ints; with rep, block 0 also zeroes that report (one launch for both).
__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t value, size_t n,
                           p2m_report* __restrict__ rep) {
    if (rep && blockIdx.x == 0) {
        const int t = threadIdx.x;
        if (t < 8) {
            rep->iters[t] = 0;
            rep->refines[t] = 0;
            rep->rel_residual[t] = 0.0;
        }
        if (t == 0) {
            rep->flags = 0u;
            rep->n_orphan = 0;
            rep->n_invalid = 0;
            rep->reserved = 0;
        }
    }
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = value;
}

// Lanes of a wave whose keys are equal form a group; returns the mask of this
// lane's group (0 for inactive lanes).  Wave-uniform loop over distinct keys.
__device__ __forceinline__ uint64_t match_any(int key, bool active) {
    uint64_t remaining = __ballot(active);
    uint64_t mine = 0;
    while (remaining) {
        const int leader = __ffsll((unsigned long long)remaining) - 1;
        const int lkey = __builtin_amdgcn_readlane(key, leader);   // leader is wave-uniform
        const bool same = active && key == lkey;
        const uint64_t grp = __ballot(same);
        if (same) mine = grp;
        remaining &= ~grp;
    }
    return mine;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Locate of particle i of one problem (lanes with i >= np take part in the wave
// operations only), its key cell0 + cell or -1, the count of its cell and its
// rank in the cell (the slot it takes, 0 .. count - 1).  One atomic per distinct
// cell per wave: particles arrive spatially coherent in typical inputs, so this
// removes most same-address atomic traffic; a group's lanes take consecutive
// slots from the value the atomic returns.  Split in two so that a thread can
// have several atomics in flight: locate_count_issue locates and issues the
// atomic, locate_count_finish waits for its value and writes key and rank.
struct LocState {
    int k;           // key or -1
    int first;       // value returned to the group leader (the group's first slot)
    uint64_t grp;    // lanes of this lane's group
    bool in;         // i < np
};

// (px, py: the particle's coordinates, loaded by the caller; py unused in 1D)
template <typename T>
__device__ __forceinline__ LocState locate_count_issue(const Mesh& m, T px, T py, int i,
                                                       int cell0, int32_t* __restrict__ counts,
                                                       p2m_report* __restrict__ rep) {
    LocState st;
    st.in = i < m.np;
    bool fin_x = true, fin_y = true;
    int cx = 0, cy = 0;
    double xi, eta;
    bool ok = false;
    if (st.in) {
        ok = locate_axis((double)px, m.nx, m.inv_hx, cx, xi, fin_x);
        if (m.dim == 2) ok = locate_axis((double)py, m.ny, m.inv_hy, cy, eta, fin_y) && ok;
    }
    st.k = ok ? cell0 + cx + m.nx * cy : -1;
    st.grp = match_any(st.k, ok);
    const int lane = threadIdx.x & 63;
    st.first = 0;
    if (ok && lane == __ffsll((unsigned long long)st.grp) - 1)
        st.first = atomicAdd(&counts[st.k], (int)__popcll(st.grp));
    if (st.in && !ok && rep) {
        const uint32_t f = (fin_x && fin_y) ? P2M_FLAG_RANGE : P2M_FLAG_NONFINITE;
        atomicOr(&rep->flags, f);
        atomicAdd(&rep->n_invalid, 1);
    }
    return st;
}

__device__ __forceinline__ void locate_count_finish(const LocState& st, int i,
                                                    int32_t* __restrict__ key,
                                                    int32_t* __restrict__ rank) {
    const int lane = threadIdx.x & 63;
    const bool ok = st.k >= 0;
    const int leader = ok ? __ffsll((unsigned long long)st.grp) - 1 : lane;
    const int first = __shfl(st.first, leader, 64);
    if (st.in) {
        key[i] = st.k;
        rank[i] = ok ? first + (int)__popcll(st.grp & lanemask_lt()) : -1;
    }
}

// kLocItems particles per thread: item u of block b covers particles
// [(b * kLocItems + u) * kBlock, ... + kBlock), so each wave step is 64
// consecutive particles.  Every coordinate is loaded before the first atomic
// and all items' atomics are issued before any is awaited (one memory counter
// covers loads and atomics in issue order).
constexpr int kLocItems = 4;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_locate_count(Mesh m, Particles<T> P,
                                                         int32_t* __restrict__ key,
                                                         int32_t* __restrict__ rank,
                                                         int32_t* __restrict__ counts,
                                                         p2m_report* __restrict__ rep) {
    const int base = blockIdx.x * (kBlock * kLocItems) + threadIdx.x;
    T px[kLocItems], py[kLocItems];
#pragma unroll
    for (int u = 0; u < kLocItems; ++u) {
        const int i = base + u * kBlock;
        px[u] = py[u] = (T)0;
        if (i < m.np) {
            px[u] = P.x[i];
            if (m.dim == 2) py[u] = P.y[i];
        }
    }
    LocState st[kLocItems];
#pragma unroll
    for (int u = 0; u < kLocItems; ++u)
        st[u] = locate_count_issue<T>(m, px[u], py[u], base + u * kBlock, 0, counts, rep);
#pragma unroll
    for (int u = 0; u < kLocItems; ++u) locate_count_finish(st[u], base + u * kBlock, key, rank);
}

// batch: block b covers particles [(b - lb) * kBinBlock, ...) of instance lmap[b]
__global__ void k_locate_count_batch(const BatchInst* __restrict__ inst,
                                     const int32_t* __restrict__ lmap, int32_t* __restrict__ key,
                                     int32_t* __restrict__ rank, int32_t* __restrict__ counts) {
    const BatchInst& I = inst[lmap[blockIdx.x]];
    const int i = (blockIdx.x - I.lb) * kBinBlock + threadIdx.x;
    float px = 0.f, py = 0.f;
    if (i < I.m.np) {
        px = I.P.x[i];
        if (I.m.dim == 2) py = I.P.y[i];
    }
    const LocState st = locate_count_issue<float>(I.m, px, py, i, I.no, counts, I.rep);
    locate_count_finish(st, i, key + I.po, rank + I.po);
}

__global__ void k_report_clear_n(p2m_report* __restrict__ reps, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = t / 32, q = t % 32;
    if (r >= n) return;
    p2m_report* rep = reps + r;
    if (q < 8) {
        rep->iters[q] = 0;
        rep->refines[q] = 0;
        rep->rel_residual[q] = 0.0;
    }
    if (q == 8) {
        rep->flags = 0u;
        rep->n_orphan = 0;
        rep->n_invalid = 0;
        rep->reserved = 0;
    }
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts (three phases: block sums, scan of the block
// sums by one block, per-block scan plus offset)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Block-wide exclusive scan of one int per thread (blockDim.x == kBlock); also
// returns the block total.
__device__ __forceinline__ int block_exclusive_scan(int v, int& total) {
    __shared__ int wave_tot[kBlock / 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int inc = wave_inclusive_scan(v);
    if (lane == 63) wave_tot[wave] = inc;
    __syncthreads();
    int off = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) off += wave_tot[w];
        total += wave_tot[w];
    }
    __syncthreads();
    return off + inc - v;
}

// Single-pass exclusive scan with decoupled look-back.  Workgroups take tile
// numbers in launch order from a counter, so every predecessor of a tile has
// started; a tile publishes its own sum (AGG), looks back over its predecessors'
// words (64 at a time, one per lane of wave 0) until it meets an inclusive prefix
// (PRE), and publishes its own inclusive prefix.  A word holds the flag in bits
// 62-63 and the value (< 2^31) in bits 0-31; the words and the counter start at
// zero (the caller clears them with the counts).
constexpr unsigned long long kScanAgg = 1ull << 62, kScanPre = 2ull << 62;
constexpr long kScanSpinMax = 1L << 26;

__global__ __launch_bounds__(kBlock) void k_scan_lookback(const int32_t* __restrict__ in, int n,
                                                          int32_t* __restrict__ out,
                                                          unsigned long long* status,
                                                          unsigned* tile_ctr) {
    __shared__ int s_tile, s_excl;
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const int tile = s_tile;
    const int base = tile * kScanTile + threadIdx.x * kScanItems;
    int vals[kScanItems];
    int s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        vals[j] = (base + j < n) ? in[base + j] : 0;
        s += vals[j];
    }
    int total;
    int ex = block_exclusive_scan(s, total);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane == 0)
            __hip_atomic_store(&status[tile], (tile == 0 ? kScanPre : kScanAgg) | (unsigned)total,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int excl = 0;
        int end = tile;  // predecessors [end - 64, end) are examined in one step
        long spins = 0;
        while (end > 0) {
            const int idx = end - 1 - lane;
            const unsigned long long w =
                idx >= 0 ? __hip_atomic_load(&status[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                         : kScanPre;
            const unsigned flag = (unsigned)(w >> 62);
            const uint64_t pre = __ballot(flag == 2u), inv = __ballot(flag == 0u);
            const int first = pre ? __ffsll((unsigned long long)pre) - 1 : 63;
            const uint64_t upto = first >= 63 ? ~0ull : ((1ull << (first + 1)) - 1);
            if (inv & upto) {  // a word this step needs is not published yet
                if (++spins > kScanSpinMax) break;
                continue;
            }
            int v = lane <= first ? (int)(w & 0xffffffffull) : 0;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
            excl += v;
            if (pre) break;
            end -= 64;
        }
        if (lane == 0) {
            if (tile > 0)
                __hip_atomic_store(&status[tile], kScanPre | (unsigned)(excl + total),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_excl = excl;
        }
    }
    __syncthreads();
    ex += s_excl;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = ex;
        ex += vals[j];
    }
    if (tile == (n + kScanTile - 1) / kScanTile - 1 && threadIdx.x == kBlock - 1)
        out[n] = s_excl + total;  // grand total
}

// Every located particle goes to its slot cell_start[key] + rank.  With
// ncells >= 0, slots [valid, np) (after every valid particle) are set to -1.
__global__ void k_place(int np, const int32_t* __restrict__ key, const int32_t* __restrict__ rank,
                        const int32_t* __restrict__ cell_start, int32_t* __restrict__ perm,
                        int ncells) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    if (ncells >= 0 && i >= cell_start[ncells]) perm[i] = -1;
    const int k = key[i];
    if (k >= 0) perm[cell_start[k] + rank[i]] = i;
}

// Every cell's slots sorted by original index, one thread per cell.  A cell of
// at most kSortReg particles is held in registers and, when out of order, sorted
// by a fixed network (8 or 16 wide).  Larger cells are sorted in place by
// insertion.  A workgroup's kBlock consecutive cells own one contiguous range of
// perm: when it fits kSortStage entries it is loaded into LDS and written back
// with coalesced accesses (only if some cell was out of order); otherwise every
// thread works on global memory directly.
constexpr int kSortReg = 16;
constexpr int kSortStage = 4096;   // perm entries staged per workgroup (16 KB)

// Batcher's odd-even merge sort network on N (a power of two) registers; every
// bound is a compile-time constant, so the network unrolls to N log^2 N / 4
// compare-exchanges.
template <int N>
__device__ __forceinline__ void sort_network(int (&v)[N]) {
#pragma unroll
    for (int p = 1; p < N; p <<= 1)
#pragma unroll
        for (int k = p; k >= 1; k >>= 1)
#pragma unroll
            for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
                for (int i = 0; i < k; ++i)
                    if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        const int a = v[i + j], b = v[i + j + k];
                        v[i + j] = min(a, b);
                        v[i + j + k] = max(a, b);
                    }
}

// Sorts a segment of n <= N entries (padded with the largest int) in registers;
// writes it back only when it was out of order.  Returns whether it wrote.
template <int N>
__device__ __forceinline__ bool sort_small(int32_t* __restrict__ seg, int n) {
    int v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = (j < n) ? seg[j] : 0x7fffffff;
    bool sorted = true;
#pragma unroll
    for (int j = 1; j < N; ++j) sorted = sorted && v[j - 1] <= v[j];
    if (sorted) return false;
    sort_network<N>(v);
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (j < n) seg[j] = v[j];
    return true;
}

__device__ __forceinline__ bool rank_sort_small(int32_t* __restrict__ seg, int n) {
    return n <= 8 ? sort_small<8>(seg, n) : sort_small<kSortReg>(seg, n);
}

__device__ __forceinline__ bool insertion_sort(int32_t* __restrict__ seg, int n) {
    bool moved = false;
    for (int i = 1; i < n; ++i) {
        const int x = seg[i];
        int j = i - 1;
        while (j >= 0 && seg[j] > x) {
            seg[j + 1] = seg[j];
            --j;
            moved = true;
        }
        seg[j + 1] = x;
    }
    return moved;
}

__global__ __launch_bounds__(kBlock) void k_segment_sort(int ncells,
                                                         const int32_t* __restrict__ cell_start,
                                                         int32_t* __restrict__ perm) {
    __shared__ int32_t st[kSortStage];
    const int c0 = blockIdx.x * kBlock;
    const int c1 = min(c0 + kBlock, ncells);
    const int c = c0 + (int)threadIdx.x;
    const int lo = cell_start[c0], hi = cell_start[c1];
    const int s = c < c1 ? cell_start[c] : lo, e = c < c1 ? cell_start[c + 1] : lo;
    const int n = e - s;
    if (hi - lo > kSortStage) {  // uniform over the workgroup
        if (n > kSortReg) insertion_sort(perm + s, n);
        else if (n > 1) rank_sort_small(perm + s, n);
        return;
    }
    // every load of the stage goes out before the first LDS write (a loop that
    // stores each load to LDS would wait for each load in turn)
    constexpr int kStageIt = kSortStage / kBlock;
    static_assert(kSortStage % kBlock == 0, "whole staging rounds");
    int32_t tmp[kStageIt];
#pragma unroll
    for (int u = 0; u < kStageIt; ++u) {
        const int t = lo + (int)threadIdx.x + u * kBlock;
        tmp[u] = t < hi ? perm[t] : 0;
    }
#pragma unroll
    for (int u = 0; u < kStageIt; ++u) {
        const int t = lo + (int)threadIdx.x + u * kBlock;
        if (t < hi) st[t - lo] = tmp[u];
    }
    __syncthreads();
    bool moved = false;
    if (n > kSortReg) moved = insertion_sort(st + (s - lo), n);
    else if (n > 1) moved = rank_sort_small(st + (s - lo), n);
    if (!__syncthreads_or(moved)) return;
    for (int t = lo + (int)threadIdx.x; t < hi; t += kBlock) perm[t] = st[t - lo];
}

inline int grid_for(size_t n, int block) { return (int)((n + block - 1) / block); }

}  // namespace

hipError_t launch_report_clear(p2m_report* rep, hipStream_t stream) {
    if (!rep) return hipSuccess;
    hipLaunchKernelGGL(k_report_clear, dim3(1), dim3(64), 0, stream, rep);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t value, size_t n, hipStream_t stream,
                           p2m_report* rep) {
    if (n == 0 && !rep) return hipSuccess;
    int grid = (int)((n + kBlock - 1) / kBlock);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid), dim3(kBlock), 0, stream, p, value, n, rep);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_locate_count(const Mesh& m, Particles<T> P, int32_t* key, int32_t* rank,
                               int32_t* counts, p2m_report* rep, hipStream_t stream) {
    if (m.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_locate_count<T>, dim3(grid_for(m.np, kBlock * kLocItems)), dim3(kBlock),
                       0, stream, m, P, key, rank, counts, rep);
    return hipGetLastError();
}
template hipError_t launch_locate_count<float>(const Mesh&, Particles<float>, int32_t*, int32_t*,
                                               int32_t*, p2m_report*, hipStream_t);
template hipError_t launch_locate_count<double>(const Mesh&, Particles<double>, int32_t*,
                                                int32_t*, int32_t*, p2m_report*, hipStream_t);

// status words (one per tile) and the tile counter; zero before each scan
size_t scan_workspace_bytes(int n) {
    const size_t nb = (size_t)(n + kScanTile - 1) / kScanTile;
    return (nb + 1) * sizeof(unsigned long long);
}

hipError_t launch_exclusive_scan(const int32_t* counts, int32_t* out, int n, void* scan_ws,
                                 hipStream_t stream) {
    const int nb = (n + kScanTile - 1) / kScanTile;
    unsigned long long* status = (unsigned long long*)scan_ws;
    unsigned* ctr = (unsigned*)(status + nb);
    if (nb == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, out, 0, (size_t)1,
                           (p2m_report*)nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_lookback, dim3(nb), dim3(kBlock), 0, stream, counts, n, out, status,
                       ctr);
    return hipGetLastError();
}

hipError_t launch_place(const Mesh& m, const int32_t* key, const int32_t* rank,
                        const int32_t* cell_start, int32_t* perm, hipStream_t stream) {
    if (m.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_place, dim3(grid_for(m.np, kBlock)), dim3(kBlock), 0, stream, m.np, key,
                       rank, cell_start, perm, m.nn);
    return hipGetLastError();
}

hipError_t launch_report_clear_n(p2m_report* reps, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_report_clear_n, dim3(grid_for((size_t)n * 32, kBlock)), dim3(kBlock), 0,
                       stream, reps, n);
    return hipGetLastError();
}

hipError_t launch_locate_count_batch(const BatchInst* inst, const int32_t* lmap, int nblocks,
                                     int32_t* key, int32_t* rank, int32_t* counts,
                                     hipStream_t stream) {
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_locate_count_batch, dim3(nblocks), dim3(kBinBlock), 0, stream, inst, lmap,
                       key, rank, counts);
    return hipGetLastError();
}

hipError_t launch_place_flat(int np, const int32_t* key, const int32_t* rank,
                             const int32_t* cell_start, int32_t* perm, hipStream_t stream) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_place, dim3(grid_for(np, kBlock)), dim3(kBlock), 0, stream, np, key,
                       rank, cell_start, perm, -1);
    return hipGetLastError();
}

hipError_t launch_segment_sort_flat(int ncells, const int32_t* cell_start, int32_t* perm,
                                    hipStream_t stream) {
    if (ncells == 0) return hipSuccess;
    hipLaunchKernelGGL(k_segment_sort, dim3(grid_for(ncells, kBlock)), dim3(kBlock), 0, stream,
                       ncells, cell_start, perm);
    return hipGetLastError();
}

hipError_t launch_segment_sort(const Mesh& m, const int32_t* cell_start, int32_t* perm,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_segment_sort, dim3(grid_for(m.nn, kBlock)), dim3(kBlock), 0, stream,
                       m.nn, cell_start, perm);
    return hipGetLastError();
}

}  // namespace p2m
