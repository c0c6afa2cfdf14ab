// Scatter of the particle-quadrature system and the FLIP / PIC finalize.
//
// For a mesh tile of TS x TS nodes one workgroup
//   1. walks the (TS+1) x (TS+1) cells that touch the tile (one extra row and
//      column below / left of it, periodic), one thread per cell.  Each thread
//      reads its cell's particles in binned order and accumulates, per cell, the
//      corner parts of w_i = sum v psi_i, b_i = sum v A psi_i and of the mass
//      matrix M_ij = sum v psi_i psi_j (Sec. 2.3 eqs. (11)-(12), Sec. 2.4) in
//      registers, then stores them in LDS;
//   2. one thread per node adds the parts of the (up to) four cells around the
//      node in a fixed order and writes b, w and the stencil of M.
// No float atomics: the sums are deterministic and independent of the launch.
//
// Per cell (corners c00, c10, c11, c01 = lower-left, lower-right, upper-right,
// upper-left) the parts are: diagonal D_c for each corner; the bottom edge
// (c00-c10) and top edge (c01-c11) entries of E; the left edge (c00-c01) and
// right edge (c10-c11) entries of N; the diagonal edge (c00-c11) entry of NE;
// w_c and b_f,c for each corner.
#include <type_traits>

#include "p2m_internal.hpp"

namespace p2m {

namespace {

// quantity slots of the per-cell parts
enum : int {
    Q_D00 = 0, Q_D10, Q_D11, Q_D01,
    Q_EB, Q_ET, Q_NL, Q_NR, Q_NE,
    Q_W00, Q_W10, Q_W11, Q_W01,
    Q_B = 13   // then 4 per field: b00, b10, b11, b01
};

// A cell's sums run over its particles one after the other.  Plain FP32 sums
// lose about sqrt(n) units of rounding over n terms: harmless at the usual few
// particles per cell, not for crowded cells.  Cells of more than
// kCompensateAbove particles are therefore summed apart, by the whole
// workgroup: every thread sums a strided share of the cell's particles with
// Kahan's compensation, and the shares are added in thread order, again
// compensated (FP32 arithmetic throughout, error about two roundings whatever
// the count).  Which cells take that path depends on the data only, so results
// stay deterministic.
constexpr int kCompensateAbove = 32;

template <bool KAHAN, typename T>
__device__ __forceinline__ void acc_add(T& s, T& c, T x) {
    if (KAHAN) {
        const T y = x - c;
        const T t = s + y;
        c = (t - s) - y;
        s = t;
    } else {
        s += x;
    }
}

// One particle (corner weights, volume, values av[f] = av[f * stride]) added
// to a cell's parts acc (and their compensations cmp when KAHAN).
template <bool KAHAN, typename T, int F, int NQ>
__device__ __forceinline__ void acc_particle(T (&acc)[NQ], T (&cmp)[NQ], T c00, T c10, T c11,
                                             T c01, T v, const T* av, int stride) {
    const T v00 = v * c00, v10 = v * c10, v11 = v * c11, v01 = v * c01;
    acc_add<KAHAN>(acc[Q_D00], cmp[Q_D00], v00 * c00);
    acc_add<KAHAN>(acc[Q_D10], cmp[Q_D10], v10 * c10);
    acc_add<KAHAN>(acc[Q_D11], cmp[Q_D11], v11 * c11);
    acc_add<KAHAN>(acc[Q_D01], cmp[Q_D01], v01 * c01);
    acc_add<KAHAN>(acc[Q_EB], cmp[Q_EB], v00 * c10);
    acc_add<KAHAN>(acc[Q_ET], cmp[Q_ET], v01 * c11);
    acc_add<KAHAN>(acc[Q_NL], cmp[Q_NL], v00 * c01);
    acc_add<KAHAN>(acc[Q_NR], cmp[Q_NR], v10 * c11);
    acc_add<KAHAN>(acc[Q_NE], cmp[Q_NE], v00 * c11);
    acc_add<KAHAN>(acc[Q_W00], cmp[Q_W00], v00);
    acc_add<KAHAN>(acc[Q_W10], cmp[Q_W10], v10);
    acc_add<KAHAN>(acc[Q_W11], cmp[Q_W11], v11);
    acc_add<KAHAN>(acc[Q_W01], cmp[Q_W01], v01);
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const T a = av[f * stride];
        acc_add<KAHAN>(acc[Q_B + 4 * f + 0], cmp[Q_B + 4 * f + 0], v00 * a);
        acc_add<KAHAN>(acc[Q_B + 4 * f + 1], cmp[Q_B + 4 * f + 1], v10 * a);
        acc_add<KAHAN>(acc[Q_B + 4 * f + 2], cmp[Q_B + 4 * f + 2], v11 * a);
        acc_add<KAHAN>(acc[Q_B + 4 * f + 3], cmp[Q_B + 4 * f + 3], v01 * a);
    }
}

// Staged 2D scatter.  A workgroup owns a TS x TS node tile and the (TS+1)^2 cells
// around it.  The particles of those cells (their perm segments) are processed in
// chunks of CH slots: first every thread loads particles slot-parallel (perm reads
// coalesced, coordinate gathers independent of each other), locates them in FP64
// and stages the four corner weights, the volume and the values in LDS; then one
// thread per cell walks its slots in binned order and accumulates the cell's parts
// in registers.  Chunks run in order, so every sum keeps the binned particle order.
// perm holds particle numbers offset by po (batches number all particles in one
// space); tile is the tile index within the problem.
template <typename T, int F, int TS, int CH>
__device__ __forceinline__ void assemble2d_tile(const Mesh& m, const Particles<T>& P,
                                                const T* __restrict__ values,
                                                const int32_t* __restrict__ perm, int po,
                                                const int32_t* __restrict__ cell_start,
                                                T* __restrict__ b, T* __restrict__ w,
                                                T* __restrict__ coef, int tiles_x, int tile) {
    constexpr int HS = TS + 1;
    constexpr int HC = HS * HS;
    constexpr int NT = (HC + 63) / 64 * 64;     // threads: one per cell
    constexpr int NQ = Q_B + 4 * F;
    constexpr int NS = 5 + F;                   // staged values per slot
    constexpr int SPT = (CH + NT - 1) / NT;     // staged slots per thread and chunk
    constexpr size_t SLOT_B = (size_t)NS * CH * sizeof(T);
    constexpr size_t PART_B = (size_t)NQ * HC * sizeof(T);
    constexpr size_t RED_B = (size_t)NQ * (NT + 1) * sizeof(T);   // crowded-cell shares
    constexpr size_t SMEM_B = SLOT_B > PART_B ? (SLOT_B > RED_B ? SLOT_B : RED_B)
                                              : (PART_B > RED_B ? PART_B : RED_B);
    static_assert(NQ <= NT, "one thread per quantity in the crowded-cell sums");
    __shared__ __align__(16) unsigned char smem[SMEM_B];
    __shared__ int c_seg[HC], c_off[HC + 1];
    __shared__ short big_cell[HC];              // crowded cells of the tile
    __shared__ int n_big;
    __shared__ short cmap[2][CH];               // slot of a chunk -> its cell (2 buffers)
    __shared__ int wsum[NT / 64];
    T* st = (T*)smem;                           // st[q * CH + slot]
    T(*part)[HC] = (T(*)[HC])smem;              // after the chunks: part[q][cell]

    const int i0 = (tile % tiles_x) * TS;
    const int j0 = (tile / tiles_x) * TS;
    const T v_uni = (T)m.v_uniform;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;

    // cell segments and their exclusive prefix (cells beyond the mesh: empty;
    // crowded cells are listed and left out of the staged chunks)
    if (t == 0) n_big = 0;
    int cnt = 0;
    if (t < HC) {
        const int hx = t % HS, hy = t / HS;
        int gi = i0 - 1 + hx, gj = j0 - 1 + hy;
        int s0 = 0;
        if (gi < m.nx && gj < m.ny) {
            if (gi < 0) gi += m.nx;
            if (gj < 0) gj += m.ny;
            const int c = gi + m.nx * gj;
            s0 = cell_start[c];
            cnt = cell_start[c + 1] - s0;
        }
        c_seg[t] = s0;
    }
    __syncthreads();
    if (cnt > kCompensateAbove) {
        big_cell[atomicAdd(&n_big, 1)] = (short)t;   // any order: cells are independent
        cnt = 0;
    }
    int inc = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int woff = 0;
    for (int wv = 0; wv < wave; ++wv) woff += wsum[wv];
    if (t < HC) c_off[t] = woff + inc - cnt;
    if (t == NT - 1) c_off[HC] = woff + inc;
    __syncthreads();
    const int total = c_off[HC];
    const int my_lo = (t < HC) ? c_off[t] : 0, my_hi = (t < HC) ? c_off[t + 1] : 0;

    T acc[NQ], cmp[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = cmp[q] = (T)0;

    // Chunks of CH slots, pipelined two deep: while chunk c is accumulated, the
    // particle data of chunk c+1 and the particle numbers of chunk c+2 are in
    // flight.  cmap (slot of a chunk -> its cell) is double-buffered; every sum
    // still runs over a cell's slots in binned order.
    const int nch = (total + CH - 1) / CH;
    auto fill_cmap = [&](int c) {  // cell threads mark their slots of chunk c
        const int cb = c * CH, ce = min(cb + CH, total);
        const int a0 = max(my_lo, cb), a1 = min(my_hi, ce);
        short* cm = cmap[c & 1];
        for (int sl = a0; sl < a1; ++sl) cm[sl - cb] = (short)t;
    };
    auto load_perm = [&](int c, int (&pi)[SPT]) {  // particle numbers of chunk c
        const int cb = c * CH, ce = min(cb + CH, total);
        const short* cm = cmap[c & 1];
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int sl = cb + t + u * NT;
            pi[u] = -1;
            if (sl < ce) {
                const int hc = cm[sl - cb];
                pi[u] = perm[c_seg[hc] + (sl - c_off[hc])] - po;
            }
        }
    };
    auto load_vals = [&](const int (&pi)[SPT], T (&px)[SPT], T (&py)[SPT], T (&pv)[SPT],
                         T (&pa)[SPT][F]) {
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            if (pi[u] < 0) continue;
            const int i = pi[u];
            px[u] = P.x[i];
            py[u] = P.y[i];
            pv[u] = P.vol ? P.vol[i] : v_uni;
#pragma unroll
            for (int f = 0; f < F; ++f) pa[u][f] = values[(size_t)f * m.np + i];
        }
    };
    int piA[SPT], piB[SPT];
    T pxA[SPT], pyA[SPT], pvA[SPT], paA[SPT][F];
    T pxB[SPT], pyB[SPT], pvB[SPT], paB[SPT][F];
    if (nch > 0) {
        fill_cmap(0);
        if (nch > 1) fill_cmap(1);
        __syncthreads();
        load_perm(0, piA);
        load_vals(piA, pxA, pyA, pvA, paA);
        if (nch > 1) load_perm(1, piB);
        __syncthreads();  // cmap[0] is read above and refilled (chunk 2) in the first pass
    }
    for (int c = 0; c < nch; ++c) {
        const int cb = c * CH, ce = min(cb + CH, total);
        // stage chunk c: FP64 locate of the loaded positions into LDS
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            if (piA[u] < 0) continue;
            int cx, cy;
            double xi, eta;
            bool fx, fy;
            locate_axis((double)pxA[u], m.nx, m.inv_hx, cx, xi, fx);
            locate_axis((double)pyA[u], m.ny, m.inv_hy, cy, eta, fy);
            T c00, c10, c11, c01;
            corner_weights<T>(xi, eta, c00, c10, c11, c01);
            const int o = t + u * NT;
            st[0 * CH + o] = c00;
            st[1 * CH + o] = c10;
            st[2 * CH + o] = c11;
            st[3 * CH + o] = c01;
            st[4 * CH + o] = pvA[u];
#pragma unroll
            for (int f = 0; f < F; ++f) st[(5 + f) * CH + o] = paA[u][f];
        }
        // chunk c's cmap buffer is free (its particle numbers are loaded): chunk c+2's
        if (c + 2 < nch) fill_cmap(c + 2);
        __syncthreads();
        // chunk c+1's particle data, then chunk c+2's particle numbers, in flight
        // during the accumulation of chunk c
        int piN[SPT];
#pragma unroll
        for (int u = 0; u < SPT; ++u) piN[u] = -1;
        if (c + 1 < nch) {
            load_vals(piB, pxB, pyB, pvB, paB);
            if (c + 2 < nch) load_perm(c + 2, piN);
        }
        // accumulate: one thread per cell, its slots in order
        const int a0 = max(my_lo, cb), a1 = min(my_hi, ce);
        for (int sl = a0; sl < a1; ++sl) {
            const int o = sl - cb;
            acc_particle<false, T, F>(acc, cmp, st[0 * CH + o], st[1 * CH + o], st[2 * CH + o],
                                      st[3 * CH + o], st[4 * CH + o], st + 5 * CH + o, CH);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            piA[u] = piB[u];
            pxA[u] = pxB[u];
            pyA[u] = pyB[u];
            pvA[u] = pvB[u];
#pragma unroll
            for (int f = 0; f < F; ++f) paA[u][f] = paB[u][f];
            piB[u] = piN[u];
        }
    }
    // crowded cells, one after the other: thread t sums slots t, t + NT, ... of
    // the cell with compensation; then thread q adds quantity q's NT shares in
    // thread order, compensated; the cell's own thread takes the totals
    const int nbig = n_big;
    T* red = (T*)smem;                          // red[q * NT + thread], totals at NQ * NT
    for (int kb = 0; kb < nbig; ++kb) {
        const int hc = big_cell[kb];
        const int hx = hc % HS, hy = hc / HS;
        int gi = i0 - 1 + hx, gj = j0 - 1 + hy;
        if (gi < 0) gi += m.nx;
        if (gj < 0) gj += m.ny;
        const int c = gi + m.nx * gj;
        const int s0 = c_seg[hc], n = cell_start[c + 1] - s0;
        T sa[NQ], sc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) sa[q] = sc[q] = (T)0;
        for (int sl = t; sl < n; sl += NT) {
            const int i = perm[s0 + sl] - po;
            int cx, cy;
            double xi, eta;
            bool fx, fy;
            locate_axis((double)P.x[i], m.nx, m.inv_hx, cx, xi, fx);
            locate_axis((double)P.y[i], m.ny, m.inv_hy, cy, eta, fy);
            T c00, c10, c11, c01;
            corner_weights<T>(xi, eta, c00, c10, c11, c01);
            const T v = P.vol ? P.vol[i] : v_uni;
            acc_particle<true, T, F>(sa, sc, c00, c10, c11, c01, v, values + i, m.np);
        }
        __syncthreads();     // the staging area is free (previous cell's totals read)
#pragma unroll
        for (int q = 0; q < NQ; ++q) red[q * NT + t] = sa[q] - sc[q];
        __syncthreads();
        if (t < NQ) {
            T s1 = (T)0, c1 = (T)0;
            for (int u = 0; u < NT; ++u) acc_add<true>(s1, c1, red[t * NT + u]);
            red[NQ * NT + t] = s1 - c1;
        }
        __syncthreads();
        if (t == hc) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] = red[NQ * NT + q];
        }
    }
    if (nbig > 0) __syncthreads();
    if (t < HC) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[q][t] = acc[q];
    }
    __syncthreads();

    if (t >= TS * TS) return;
    const int li = t % TS, lj = t / TS;
    const int gi = i0 + li, gj = j0 + lj;
    if (gi >= m.nx || gj >= m.ny) return;
    const int k = gi + m.nx * gj;
    // halo coordinates of the cells around node (gi, gj)
    const int cA = (li + 1) + HS * (lj + 1);  // cell (i, j): node is its c00
    const int cB = li + HS * (lj + 1);        // cell (i-1, j): node is its c10
    const int cC = li + HS * lj;              // cell (i-1, j-1): node is its c11
    const int cD = (li + 1) + HS * lj;        // cell (i, j-1): node is its c01
    w[k] = ((part[Q_W00][cA] + part[Q_W10][cB]) + part[Q_W11][cC]) + part[Q_W01][cD];
#pragma unroll
    for (int f = 0; f < F; ++f) {
        b[(size_t)f * m.nn + k] = ((part[Q_B + 4 * f + 0][cA] + part[Q_B + 4 * f + 1][cB]) +
                                   part[Q_B + 4 * f + 2][cC]) +
                                  part[Q_B + 4 * f + 3][cD];
    }
    if (coef) {
        coef[k] = ((part[Q_D00][cA] + part[Q_D10][cB]) + part[Q_D11][cC]) + part[Q_D01][cD];
        coef[(size_t)m.nn + k] = part[Q_EB][cA] + part[Q_ET][cD];       // M(k, k+x)
        coef[(size_t)2 * m.nn + k] = part[Q_NL][cA] + part[Q_NR][cB];   // M(k, k+y)
        coef[(size_t)3 * m.nn + k] = part[Q_NE][cA];                    // M(k, k+x+y)
    }
}

template <typename T, int F, int TS, int CH>
__global__ __launch_bounds__(((TS + 1) * (TS + 1) + 63) / 64 * 64) void k_assemble2d(
    Mesh m, Particles<T> P, const T* __restrict__ values, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ cell_start, T* __restrict__ b, T* __restrict__ w,
    T* __restrict__ coef, int tiles_x) {
    assemble2d_tile<T, F, TS, CH>(m, P, values, perm, 0, cell_start, b, w, coef, tiles_x,
                                  blockIdx.x);
}

// batch: tile t belongs to instance amap[t]; the instance's b, w and coef blocks
// start at F*no, no and 4*no
template <int F, int TS, int CH>
__global__ __launch_bounds__(((TS + 1) * (TS + 1) + 63) / 64 * 64) void k_assemble2d_batch(
    const BatchInst* __restrict__ inst, const int32_t* __restrict__ amap,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ cell_start,
    float* __restrict__ b, float* __restrict__ w, float* __restrict__ coef) {
    const BatchInst& I = inst[amap[blockIdx.x]];
    assemble2d_tile<float, F, TS, CH>(I.m, I.P, I.values, perm, I.po, cell_start + I.no,
                                      b + (size_t)F * I.no, w + I.no, coef + (size_t)4 * I.no,
                                      I.atx, blockIdx.x - I.at);
}

// 1D: a tile of TS nodes and the TS+1 cells touching it (one extra on the left).
// Per cell: diagonal parts at the left / right node, the edge entry, w and b at
// both nodes.
template <typename T, int F, int TS>
__global__ __launch_bounds__(TS) void k_assemble1d(Mesh m, Particles<T> P,
                                                  const T* __restrict__ values,
                                                  const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ cell_start,
                                                  T* __restrict__ b, T* __restrict__ w,
                                                  T* __restrict__ coef) {
    constexpr int HC = TS + 1;
    constexpr int NQ = 5 + 2 * F;  // DL, DR, E, WL, WR, then bL, bR per field
    __shared__ T part[NQ][HC];
    const int i0 = blockIdx.x * TS;
    const T v_uni = (T)m.v_uniform;
    // one cell per thread, its particles in binned order; a cell of more than
    // kCompensateAbove particles is summed with Kahan's compensation
    auto cell_sums = [&](auto kahan, int s, int e, T (&acc)[NQ], T (&cmp)[NQ]) {
        constexpr bool K = decltype(kahan)::value;
        for (int kk = s; kk < e; ++kk) {
            const int i = perm[kk];
            int cx;
            double xi;
            bool fx;
            locate_axis((double)P.x[i], m.nx, m.inv_hx, cx, xi, fx);
            const T cl = (T)__dsub_rn(1.0, xi), cr = (T)xi;
            const T v = P.vol ? P.vol[i] : v_uni;
            const T vl = v * cl, vr = v * cr;
            acc_add<K>(acc[0], cmp[0], vl * cl);
            acc_add<K>(acc[1], cmp[1], vr * cr);
            acc_add<K>(acc[2], cmp[2], vl * cr);
            acc_add<K>(acc[3], cmp[3], vl);
            acc_add<K>(acc[4], cmp[4], vr);
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const T a = values[(size_t)f * m.np + i];
                acc_add<K>(acc[5 + 2 * f], cmp[5 + 2 * f], vl * a);
                acc_add<K>(acc[6 + 2 * f], cmp[6 + 2 * f], vr * a);
            }
        }
    };
    for (int hc = threadIdx.x; hc < HC; hc += TS) {
        int gi = i0 - 1 + hc;
        if (gi >= m.nx) continue;
        if (gi < 0) gi += m.nx;
        T acc[NQ], cmp[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = cmp[q] = (T)0;
        const int s = cell_start[gi], e = cell_start[gi + 1];
        const bool crowded = e - s > kCompensateAbove;
        if (crowded) cell_sums(std::true_type{}, s, e, acc, cmp);
        else cell_sums(std::false_type{}, s, e, acc, cmp);
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[q][hc] = crowded ? acc[q] - cmp[q] : acc[q];
    }
    __syncthreads();
    const int gi = i0 + threadIdx.x;
    if (gi >= m.nx) return;
    const int cA = threadIdx.x + 1;  // cell i: node is its left end
    const int cB = threadIdx.x;      // cell i-1: node is its right end
    w[gi] = part[3][cA] + part[4][cB];
#pragma unroll
    for (int f = 0; f < F; ++f) b[(size_t)f * m.nn + gi] = part[5 + 2 * f][cA] + part[6 + 2 * f][cB];
    if (coef) {
        coef[gi] = part[0][cA] + part[1][cB];
        coef[(size_t)m.nn + gi] = part[2][cA];
    }
}

template <typename T>
__global__ void k_finalize(int nn, int F, const T* __restrict__ b, const T* __restrict__ w,
                           int pic, T measure, T* __restrict__ out,
                           p2m_report* __restrict__ rep) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    bool orphan = false;
    if (k < nn) {
        const T wk = w[k];
        orphan = !(wk > (T)0);
        for (int f = 0; f < F; ++f) {
            const T bk = b[(size_t)f * nn + k];
            T o;
            if (pic) o = bk / measure;
            else o = orphan ? (T)0 : bk / wk;
            out[(size_t)f * nn + k] = o;
        }
    }
    if (rep) {
        // one atomic per wave that holds an orphan
        uint64_t mask = __ballot(k < nn && orphan);
        if (mask && (threadIdx.x & 63) == __ffsll((unsigned long long)mask) - 1) {
            atomicAdd(&rep->n_orphan, (int)__popcll(mask));
            atomicOr(&rep->flags, (uint32_t)P2M_FLAG_ORPHAN);
        }
    }
}

// staged slots per chunk: the staging area stays within 32 KB
template <typename T, int F>
constexpr int stage_chunk() {
    return ((int)(32768 / ((5 + F) * sizeof(T))) > 2048 ? 2048
                                                        : (int)(32768 / ((5 + F) * sizeof(T)))) /
           64 * 64;
}

template <int F>
hipError_t assemble_batch_f(const BatchInst* inst, const int32_t* amap, int ntiles,
                            const int32_t* perm, const int32_t* cs, float* b, float* w,
                            float* coef, hipStream_t stream) {
    constexpr int TS = assemble_tile(F, 4);
    constexpr int CH = stage_chunk<float, F>();
    constexpr int NT = ((TS + 1) * (TS + 1) + 63) / 64 * 64;
    hipLaunchKernelGGL((k_assemble2d_batch<F, TS, CH>), dim3(ntiles), dim3(NT), 0, stream, inst,
                       amap, perm, cs, b, w, coef);
    return hipGetLastError();
}

template <typename T, int F, int TS>
hipError_t assemble2d_ts(const Mesh& m, Particles<T> P, const T* values, const int32_t* perm,
                         const int32_t* cs, T* b, T* w, T* coef, hipStream_t stream) {
    constexpr int CH = stage_chunk<T, F>();
    constexpr int NT = ((TS + 1) * (TS + 1) + 63) / 64 * 64;
    const int tx = (m.nx + TS - 1) / TS, ty = (m.ny + TS - 1) / TS;
    hipLaunchKernelGGL((k_assemble2d<T, F, TS, CH>), dim3(tx * ty), dim3(NT), 0, stream, m, P,
                       values, perm, cs, b, w, coef, tx);
    return hipGetLastError();
}

// tile: 0 = the default node tile (15 x 15 where its parts fit 64 KB of LDS, else
// 8 x 8), 8 = 8 x 8
template <typename T, int F>
hipError_t assemble_f(const Mesh& m, Particles<T> P, const T* values, const int32_t* perm,
                      const int32_t* cs, T* b, T* w, T* coef, int tile, hipStream_t stream) {
    if (m.dim == 1) {
        constexpr int TS = 256;
        int grid = (m.nx + TS - 1) / TS;
        hipLaunchKernelGGL((k_assemble1d<T, F, TS>), dim3(grid), dim3(TS), 0, stream, m, P, values,
                           perm, cs, b, w, coef);
        return hipGetLastError();
    }
    // tile 15x15 unless the per-cell parts of its 16x16 cells exceed 64 KB; chunk
    // of staged slots sized to keep the staging area within 32 KB
    static_assert(Q_B == 13, "assemble_tile assumes 13 + 4F parts per cell");
    constexpr int TS = assemble_tile(F, (int)sizeof(T));
    if (tile == 8 && TS != 8)
        return assemble2d_ts<T, F, 8>(m, P, values, perm, cs, b, w, coef, stream);
    return assemble2d_ts<T, F, TS>(m, P, values, perm, cs, b, w, coef, stream);
}

}  // namespace

template <typename T>
hipError_t launch_assemble(const Mesh& m, Particles<T> P, const T* values, int F,
                           const int32_t* perm, const int32_t* cell_start, T* b, T* w, T* coef,
                           hipStream_t stream, int tile) {
    switch (F) {
        case 1: return assemble_f<T, 1>(m, P, values, perm, cell_start, b, w, coef, tile, stream);
        case 2: return assemble_f<T, 2>(m, P, values, perm, cell_start, b, w, coef, tile, stream);
        case 3: return assemble_f<T, 3>(m, P, values, perm, cell_start, b, w, coef, tile, stream);
        case 4: return assemble_f<T, 4>(m, P, values, perm, cell_start, b, w, coef, tile, stream);
        case 5: return assemble_f<T, 5>(m, P, values, perm, cell_start, b, w, coef, tile, stream);
        case 6: return assemble_f<T, 6>(m, P, values, perm, cell_start, b, w, coef, tile, stream);
        case 7: return assemble_f<T, 7>(m, P, values, perm, cell_start, b, w, coef, tile, stream);
        case 8: return assemble_f<T, 8>(m, P, values, perm, cell_start, b, w, coef, tile, stream);
        default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_assemble<float>(const Mesh&, Particles<float>, const float*, int,
                                           const int32_t*, const int32_t*, float*, float*, float*,
                                           hipStream_t, int);
template hipError_t launch_assemble<double>(const Mesh&, Particles<double>, const double*, int,
                                            const int32_t*, const int32_t*, double*, double*,
                                            double*, hipStream_t, int);

hipError_t launch_assemble_batch(int F, const BatchInst* inst, const int32_t* amap, int ntiles,
                                 const int32_t* perm, const int32_t* cell_start, float* b,
                                 float* w, float* coef, hipStream_t stream) {
    if (ntiles == 0) return hipSuccess;
    switch (F) {
        case 1: return assemble_batch_f<1>(inst, amap, ntiles, perm, cell_start, b, w, coef, stream);
        case 2: return assemble_batch_f<2>(inst, amap, ntiles, perm, cell_start, b, w, coef, stream);
        case 3: return assemble_batch_f<3>(inst, amap, ntiles, perm, cell_start, b, w, coef, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_finalize(const Mesh& m, int F, const T* b, const T* w, int pic, T* out,
                           p2m_report* rep, hipStream_t stream) {
    const int block = 256;
    int grid = (m.nn + block - 1) / block;
    hipLaunchKernelGGL(k_finalize<T>, dim3(grid), dim3(block), 0, stream, m.nn, F, b, w, pic,
                       (T)m.cell_measure, out, rep);
    return hipGetLastError();
}
template hipError_t launch_finalize<float>(const Mesh&, int, const float*, const float*, int,
                                           float*, p2m_report*, hipStream_t);
template hipError_t launch_finalize<double>(const Mesh&, int, const double*, const double*, int,
                                            double*, p2m_report*, hipStream_t);

}  // namespace p2m
