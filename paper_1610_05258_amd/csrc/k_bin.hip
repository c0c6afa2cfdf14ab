// Binning of particles by cell: a stable counting sort.
//
//   locate_count : FP64 locate of every particle, cell key, per-cell counts
//                  (integer atomics: order-independent, so the counts are exact);
//                  the value an atomic returns gives each particle a distinct
//                  slot of its cell (its rank), in an order that depends on timing
//   exclusive_scan: cell_start = exclusive prefix sum of the counts (one kernel,
//                  decoupled look-back over the predecessor tiles)
//   place        : perm[cell_start[key] + rank] = particle (no atomics)
//   segment_sort : every cell sorts its slots by original index, which makes the
//                  permutation exactly the stable (cell, original index) order
//
// The result does not depend on the order in which the atomics were served.
//
// Every wait is bounded.  If the scan's look-back gives up on a predecessor, it
// raises P2M_FLAG_BIN_TIMEOUT and an abort word; place then leaves every cell
// empty (cell_start all 0, perm all -1), so whatever reads the binning stays in
// bounds and the caller sees the flag.
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
// exclusive scan of int32 counts: one kernel, each workgroup scans a tile of
// kScanTile counts and adds the prefix of its predecessors found by look-back
// ---------------------------------------------------------------------------
// 32 counts per thread (read and written as 16-byte vectors): a tile of 8192 keeps
// the look-back chain short (128 tiles for 2^20 cells)
constexpr int kScanItems = 32;
constexpr int kScanTile = kBlock * kScanItems;
typedef int i32x4 __attribute__((ext_vector_type(4)));

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
// 62-63 and the value (< 2^31) in bits 0-31; the words, the counter and the abort
// word start at zero (the caller clears them with the counts).
//
// The wait for an unpublished word is bounded by spin_max polls (spin_max < 0:
// no poll at all, the first unpublished word ends the wait; a test hook for the
// timeout path).  A tile that gives up still publishes a (wrong) PRE so that its
// successors finish, sets the abort word and raises P2M_FLAG_BIN_TIMEOUT in the
// nrep reports; k_place then discards the whole scan.
constexpr unsigned long long kScanAgg = 1ull << 62, kScanPre = 2ull << 62;

__global__ __launch_bounds__(kBlock) void k_scan_lookback(const int32_t* __restrict__ in, int n,
                                                          int32_t* __restrict__ out,
                                                          unsigned long long* status,
                                                          unsigned* tile_ctr, unsigned* abort_word,
                                                          long spin_max,
                                                          p2m_report* __restrict__ reps,
                                                          int nrep) {
    __shared__ int s_tile, s_excl;
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const int tile = s_tile;
    const int base = tile * kScanTile + threadIdx.x * kScanItems;
    // a full run of 16-byte aligned arrays: vector accesses
    const bool whole = base + kScanItems <= n && (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
    int vals[kScanItems];
    if (whole) {
#pragma unroll
        for (int j = 0; j < kScanItems; j += 4) {
            const i32x4 q = *(const i32x4*)(in + base + j);
            vals[j] = q.x;
            vals[j + 1] = q.y;
            vals[j + 2] = q.z;
            vals[j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) vals[j] = (base + j < n) ? in[base + j] : 0;
    }
    int s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s += vals[j];
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
        bool gave_up = false;
        while (end > 0) {
            const int idx = end - 1 - lane;
            const unsigned long long w =
                (idx >= 0 && spin_max >= 0)
                    ? __hip_atomic_load(&status[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    : (idx >= 0 ? 0ull : kScanPre);
            const unsigned flag = (unsigned)(w >> 62);
            const uint64_t pre = __ballot(flag == 2u), inv = __ballot(flag == 0u);
            const int first = pre ? __ffsll((unsigned long long)pre) - 1 : 63;
            const uint64_t upto = first >= 63 ? ~0ull : ((1ull << (first + 1)) - 1);
            if (inv & upto) {  // a word this step needs is not published yet
                if (++spins > spin_max) {
                    gave_up = true;
                    break;
                }
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
            if (gave_up) {
                __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int r = 0; r < nrep; ++r) atomicOr(&reps[r].flags, (uint32_t)P2M_FLAG_BIN_TIMEOUT);
            }
        }
    }
    __syncthreads();
    ex += s_excl;
    if (whole) {
#pragma unroll
        for (int j = 0; j < kScanItems; j += 4) {
            i32x4 q;
            q.x = ex;
            q.y = q.x + vals[j];
            q.z = q.y + vals[j + 1];
            q.w = q.z + vals[j + 2];
            ex = q.w + vals[j + 3];
            *(i32x4*)(out + base + j) = q;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            if (base + j < n) out[base + j] = ex;
            ex += vals[j];
        }
    }
    if (tile == (n + kScanTile - 1) / kScanTile - 1 && threadIdx.x == kBlock - 1)
        out[n] = s_excl + total;  // grand total
}

// Every located particle goes to its slot cell_start[key] + rank.  With
// fill_tail, slots [valid, np) (after every valid particle) are set to -1.
// When the scan has aborted (abort word set), the binning is discarded instead:
// cell_start[0..ncells] = 0 and perm[0..np) = -1, so every cell is empty.  A
// thread takes kPlaceItems indices, blockDim apart; the grid covers max(np,
// ncells + 1) indices.  Its loads (the abort word, the valid count, keys and
// ranks) go out together, then its cell_start gathers: two round trips per wave.
constexpr int kPlaceItems = 4;

__global__ void k_place(int np, const int32_t* __restrict__ key, const int32_t* __restrict__ rank,
                        int32_t* __restrict__ cell_start, int32_t* __restrict__ perm, int ncells,
                        int fill_tail, const unsigned* __restrict__ abort_word) {
    const int i0 = blockIdx.x * blockDim.x * kPlaceItems + threadIdx.x;
    const unsigned ab = __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int valid = fill_tail ? cell_start[ncells] : np;
    int k[kPlaceItems], r[kPlaceItems];
#pragma unroll
    for (int u = 0; u < kPlaceItems; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        k[u] = i < np ? key[i] : -1;
        r[u] = i < np ? rank[i] : 0;
    }
    if (ab != 0u) {
#pragma unroll
        for (int u = 0; u < kPlaceItems; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < np) perm[i] = -1;
            if (i <= ncells) cell_start[i] = 0;
        }
        return;
    }
    int st[kPlaceItems];
#pragma unroll
    for (int u = 0; u < kPlaceItems; ++u) st[u] = k[u] >= 0 ? cell_start[k[u]] : 0;
#pragma unroll
    for (int u = 0; u < kPlaceItems; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        if (i >= np) continue;
        if (i >= valid) perm[i] = -1;
        if (k[u] >= 0) perm[st[u] + r[u]] = i;
    }
}

// Every cell's slots sorted by original index.  A workgroup owns kBlock
// consecutive cells, which own one contiguous range of perm; when that range
// fits kSortStage entries it is loaded into LDS and written back with coalesced
// accesses (only if some cell was out of order), otherwise the sort works on
// global memory in place.  A cell of at most kSortReg particles is sorted by its
// own thread in registers with a fixed network (8 or 16 wide).  Larger cells
// are sorted one after the other by the whole workgroup with a merge network of
// n log^2 n / 4 compare-exchanges (bounded work whatever the crowding).
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

// One segment of n entries sorted ascending by all kBlock threads of the
// workgroup (every thread calls it; seg is LDS or global memory private to the
// workgroup).  Bitonic sort in the form whose comparators all put the smaller
// value at the lower index: each merge of two sorted halves of a block of k
// first compares i with its mirror k - 1 - i, then half-cleans at distances
// k/4, ..., 1.  The segment is padded to the next power of two P with virtual
// +infinity entries; a comparator whose upper index is >= n would leave both
// entries in place, so it is skipped and the padding is never stored.  The
// values are distinct particle numbers.  Returns (to every thread) whether any
// entry moved.
__device__ __forceinline__ bool block_sort_segment(int32_t* seg, int n, int* moved_flag) {
    int P = 1;
    while (P < n) P <<= 1;
    if (threadIdx.x == 0) *moved_flag = 0;
    __syncthreads();
    int moved = 0;
    for (int k = 2; k <= P; k <<= 1) {
        const int half = k >> 1;
        for (int q = threadIdx.x; q < P / 2; q += kBlock) {
            const int blk = q / half, off = q - blk * half;
            const int i = blk * k + off, j = blk * k + k - 1 - off;
            if (j < n) {
                const int a = seg[i], b = seg[j];
                if (a > b) {
                    seg[i] = b;
                    seg[j] = a;
                    moved = 1;
                }
            }
        }
        __syncthreads();
        for (int d = k >> 2; d >= 1; d >>= 1) {
            for (int q = threadIdx.x; q < P / 2; q += kBlock) {
                const int blk = q / d;
                const int i = blk * 2 * d + (q - blk * d), j = i + d;
                if (j < n) {
                    const int a = seg[i], b = seg[j];
                    if (a > b) {
                        seg[i] = b;
                        seg[j] = a;
                        moved = 1;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (moved) *moved_flag = 1;
    __syncthreads();
    const int any = *moved_flag;
    __syncthreads();
    return any != 0;
}

__global__ __launch_bounds__(kBlock) void k_segment_sort(int ncells,
                                                         const int32_t* __restrict__ cell_start,
                                                         int32_t* __restrict__ perm) {
    __shared__ int32_t st[kSortStage];
    __shared__ int big[kBlock];
    __shared__ int n_big, s_flag;
    const int c0 = blockIdx.x * kBlock;
    const int c1 = min(c0 + kBlock, ncells);
    const int c = c0 + (int)threadIdx.x;
    const int lo = cell_start[c0], hi = cell_start[c1];
    const int s = c < c1 ? cell_start[c] : lo, e = c < c1 ? cell_start[c + 1] : lo;
    const int n = e - s;
    if (threadIdx.x == 0) n_big = 0;
    const bool staged = hi - lo <= kSortStage;   // uniform over the workgroup
    if (staged) {
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
    }
    __syncthreads();
    // large cells are listed (in any order: cells are independent) and sorted
    // after the small ones; the LDS and global forms are written out separately
    // so that each compiles to its own memory instructions
    if (n > kSortReg) big[atomicAdd(&n_big, 1)] = (int)threadIdx.x;
    if (!staged) {
        if (n > 1 && n <= kSortReg) rank_sort_small(perm + s, n);
        __syncthreads();
        const int nb = n_big;
        for (int k = 0; k < nb; ++k) {
            const int cc = c0 + big[k];
            const int bs = cell_start[cc];
            block_sort_segment(perm + bs, cell_start[cc + 1] - bs, &s_flag);
        }
        return;
    }
    bool moved = false;
    if (n > 1 && n <= kSortReg) moved = rank_sort_small(st + (s - lo), n);
    __syncthreads();
    const int nb = n_big;
    for (int k = 0; k < nb; ++k) {
        const int cc = c0 + big[k];
        const int bs = cell_start[cc];
        moved = block_sort_segment(st + (bs - lo), cell_start[cc + 1] - bs, &s_flag) || moved;
    }
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

// words of the scan workspace: status[nb], then the tile counter and the abort word
static unsigned* scan_ctr(void* scan_ws, int n) {
    return (unsigned*)((unsigned long long*)scan_ws + (n + kScanTile - 1) / kScanTile);
}

hipError_t launch_exclusive_scan(const int32_t* counts, int32_t* out, int n, void* scan_ws,
                                 long spin_max, p2m_report* reps, int nrep, hipStream_t stream) {
    const int nb = (n + kScanTile - 1) / kScanTile;
    unsigned long long* status = (unsigned long long*)scan_ws;
    unsigned* ctr = scan_ctr(scan_ws, n);
    if (nb == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, out, 0, (size_t)1,
                           (p2m_report*)nullptr);
        return hipGetLastError();
    }
    if (!reps) nrep = 0;
    hipLaunchKernelGGL(k_scan_lookback, dim3(nb), dim3(kBlock), 0, stream, counts, n, out, status,
                       ctr, ctr + 1, spin_max, reps, nrep);
    return hipGetLastError();
}

hipError_t launch_place(const Mesh& m, const int32_t* key, const int32_t* rank, int32_t* cell_start,
                        int32_t* perm, const void* scan_ws, hipStream_t stream) {
    if (m.np == 0) return hipSuccess;
    const int nidx = m.np > m.nn + 1 ? m.np : m.nn + 1;
    hipLaunchKernelGGL(k_place, dim3(grid_for(nidx, kBlock * kPlaceItems)), dim3(kBlock), 0, stream,
                       m.np, key, rank, cell_start, perm, m.nn, 1, scan_ctr((void*)scan_ws, m.nn) + 1);
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

hipError_t launch_place_flat(int np, int ncells, const int32_t* key, const int32_t* rank,
                             int32_t* cell_start, int32_t* perm, const void* scan_ws,
                             hipStream_t stream) {
    if (np == 0) return hipSuccess;
    const int nidx = np > ncells + 1 ? np : ncells + 1;
    hipLaunchKernelGGL(k_place, dim3(grid_for(nidx, kBlock * kPlaceItems)), dim3(kBlock), 0, stream,
                       np, key, rank, cell_start, perm, ncells, 0, scan_ctr((void*)scan_ws, ncells) + 1);
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
