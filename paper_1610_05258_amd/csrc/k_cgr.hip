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
//  * the inner CG is the Chronopoulos-Gear variant of Jacobi-preconditioned CG
//    (u = r / diag M, w = M u): the three dot products of an iteration, (r, u),
//    (w, u) and (r, r), are reduced together, so an iteration needs one grid
//    barrier.  The new u' = (r - alpha (w + beta s)) / diag M of a neighbour
//    tile's boundary node is recomputed from its published (r, w, s) with the
//    same FP32 operations its owner uses, so the halo is bit-identical;
//  * each workgroup also keeps the ring's copies of p and d (the same FP32
//    operations on the same values as their owners), so the correction of an
//    inner solve is folded into x inside the next residual phase: the ring's new
//    x is its owner's published x plus the ring copy of d, and no barrier
//    separates the fold from the residual;
//  * the grid barrier adds one to a counter and polls it; after it every
//    workgroup sums the per-workgroup FP64 partials in the same fixed order, so
//    every workgroup takes identical decisions and the result is deterministic.
//  Every wait is bounded: a timed-out wait raises an abort flag that ends the
//  solve in every workgroup.
#include "cg_common.hpp"

namespace p2m {

namespace {

struct RArgs {
    Mesh m;
    int tiles_x;
    float* coef;       // [4][nn]  D, E, N, NE  (orphan diagonals set to 1 here)
    float* b;          // [F][nn]  (orphan entries set to 0 here)
    const float* w;    // [nn]
    float* xout;       // [F][nn]  start (USER) on entry, result on exit
    double* x64;       // [F][nn]  FP64 solution, owner-only
    float* pubR;       // [2][F][nn] published values of the boundary rows
    float* pubW;
    float* pubS;
    float* pubC;       // [2][nn][rec_floats(F)] published records of the boundary columns
    double* pubX;      // [2][F][nn] published boundary x64, by refinement parity
    RSync sy;
    int start;
    p2m_solve_opts opts;
    p2m_report* rep;
};

constexpr int NH = 2 * (RX + 2) + 2 * RY;   // ring slots of a full tile

// the start x0 of node k of field f as the P phase computes it (0 at an orphan,
// w == 0); the ring's start in the first residual phase
__device__ __forceinline__ double start_value(const RArgs& a, int f, int k) {
    if (a.start == P2M_START_ZERO) return 0.0;
    const float wk = a.w[k];
    if (!(wk > 0.f)) return 0.0;
    const size_t o = (size_t)f * a.m.nn + k;
    return a.start == P2M_START_FLIP ? (double)a.b[o] / (double)wk : (double)a.xout[o];
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
    static_assert(NH <= RBS, "one ring slot per thread");
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
    auto rs_pubX = [&](int par, int f) { return mkrs(a.pubX + ((size_t)par * F + f) * nn, fb8); };
    auto rs_pub = [&](float* base, int par, int f) {
        return mkrs(base + ((size_t)par * F + f) * nn, fb4);
    };
    constexpr int RS = rec_floats(F);
    auto rs_col = [&](int par) {
        return mkrs(a.pubC + (size_t)par * nn * RS, (size_t)nn * RS * 4);
    };

    // LDS: stencil coefficients of the tile plus its left column and bottom row,
    // and one exchange area used as F FP32 planes or as one FP64 plane
    constexpr int CW = RX + 1, CN = (RY + 1) * (RX + 1);
    // xbuf: the F FP32 planes of the CG iterations, or (residual phase) one FP64
    // plane of x followed by one FP32 plane of b
    constexpr size_t XB = (size_t)(F > 3 ? F : 3) * LH * LW * sizeof(float);
    __shared__ float cf[4 * CN];
    __shared__ float dv[LH * LW];   // Jacobi inverse diagonal of the tile and its ring
    __shared__ __align__(16) unsigned char xbuf[XB];
    float* lf = (float*)xbuf;       // plane f at lf + f * LH * LW
    double* ld64 = (double*)xbuf;
    float* lb = (float*)(ld64 + LH * LW);
    // the ring's copies of p (field f at f * NH) and d (at (F + f) * NH), slot h
    // held by thread h
    __shared__ float rpd[2 * F * NH];
    __shared__ double red_lds[(RBS / 64) * kNV];
    __shared__ double vals[kNV];
    __shared__ double s_bb[F], s_gam[F], s_alpha[F], s_relres[F], s_target[F];
    __shared__ float s_af[F], s_bf[F];
    __shared__ int s_iters[F], s_refines[F], s_done[F], s_inner[F], s_zero[F], s_res[F];
    __shared__ uint32_t s_flags;

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
        s_res[f] = 0; s_relres[f] = 0.0; s_bb[f] = 0.0;
    }
    if (threadIdx.x == 0) s_flags = 0u;

    // active nodes; those on the tile boundary; on a boundary row; on a boundary column
    uint32_t amask = 0, bmask = 0, rmask = 0, cmask = 0;
#pragma unroll
    for (int j = 0; j < RNPT; ++j) {
        if (!active(j)) continue;
        amask |= 1u << j;
        const int lc = ncol(j), lr = nrow(j);
        if (lr == 0 || lr == tya - 1) rmask |= 1u << j;
        if (lc == 0 || lc == txa - 1) cmask |= 1u << j;
    }
    bmask = rmask | cmask;

    // left column / bottom row (only their E, N, NE are used, never modified here)
    // and the ring's inverse diagonals (an orphan's is 1 whatever its stored
    // diagonal): at most one slot of each per thread, both slots' loads issued
    // before either LDS write
    static_assert(RX + 1 + RY <= RBS, "one left-column or bottom-row slot per thread");
    {
        const int h = threadIdx.x;
        int eq = -1, dq = -1;
        float e1 = 0.f, e2 = 0.f, e3 = 0.f, dc = 0.f, dw = 0.f;
        if (h < txa + 1 + tya) {
            int lc, lr;
            if (h < txa + 1) { lr = -1; lc = h - 1; } else { lc = -1; lr = h - (txa + 1); }
            const int k = gidx(m, i0, j0, lc, lr);
            eq = cidx(lc, lr);
            e1 = a.coef[(size_t)nn + k];
            e2 = a.coef[(size_t)2 * nn + k];
            e3 = a.coef[(size_t)3 * nn + k];
        }
        int lc, lr;
        if (h < nhalo && halo_slot(h, txa, tya, lc, lr)) {
            const int k = gidx(m, i0, j0, lc, lr);
            dq = lidx(lc, lr);
            dc = a.coef[k];
            dw = a.w[k];
        }
        if (eq >= 0) {
            cf[CN + eq] = e1;
            cf[2 * CN + eq] = e2;
            cf[3 * CN + eq] = e3;
        }
        if (dq >= 0) dv[dq] = jacobi_inv(dc, dw);
    }
    // ---- P: coefficients into LDS, orphan regularisation, FP64 start vector ----
    // Every load is issued before the first store: the memory counter covers loads
    // and stores in issue order, so a load issued after a store would also wait for
    // the store.
    {
        float pw[RNPT], pc[4][RNPT], px[F][RNPT];
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            if (!(amask & (1u << j))) continue;
            const int k = gk(j);
            pw[j] = a.w[k];
#pragma unroll
            for (int c = 0; c < 4; ++c) pc[c][j] = a.coef[(size_t)c * nn + k];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const size_t o = (size_t)f * nn + k;
                px[f][j] = a.start == P2M_START_USER ? a.xout[o] : a.b[o];
            }
        }
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            if (!(amask & (1u << j))) continue;
            const int k = gk(j);
            const int q = qcj(j);
            const float wk = pw[j];
            const bool orphan = !(wk > 0.f);
            const float dk = pc[0][j];
            if (orphan) a.coef[k] = 1.f;
            cf[q] = orphan ? 1.f : dk;
            dv[qj(j)] = jacobi_inv(dk, wk);
            cf[CN + q] = pc[1][j];
            cf[2 * CN + q] = pc[2][j];
            cf[3 * CN + q] = pc[3][j];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const size_t o = (size_t)f * nn + k;
                double x0;
                if (orphan) {
                    a.b[o] = 0.f;
                    x0 = 0.0;
                } else if (a.start == P2M_START_FLIP) {
                    x0 = (double)px[f][j] / (double)wk;
                } else if (a.start == P2M_START_ZERO) {
                    x0 = 0.0;
                } else {
                    x0 = (double)px[f][j];
                }
                a.x64[o] = x0;
                // the start's boundary values, read by the second residual phase
                // (the first computes the ring's start itself)
                if (bmask & (1u << j)) std8<kCoherent>(rs_pubX(0, f), k, x0);
            }
            if (orphan && a.rep) {
                atomicAdd(&a.rep->n_orphan, 1);
                atomicOr(&a.rep->flags, (uint32_t)P2M_FLAG_ORPHAN);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
        for (int j = 0; j < RNPT; ++j) vp[f][j] = vd[f][j] = vs[f][j] = vr[f][j] = vw[f][j] = 0.f;
    __syncthreads();

    unsigned epoch = 0;
    int ex = 0;  // exchange parity of pubR / pubW / pubS
    bool alive = true;

    // w = M u at the owned nodes for every inner-active field (u in the exchange
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
                const float acc = stencil32(cD, cE, cEw, cN, cNs, cNE, cNEsw, L[q], L[q + 1],
                                            L[q - 1], L[q + LW], L[q - LW], L[q + LW + 1],
                                            L[q - LW - 1]);
                vw[f][j] = on ? acc : 0.f;
            }
        }
    };

    // the boundary's (r, w, s) of every inner-active field into the exchange
    // planes of parity ex
    auto publish_rws = [&](uint32_t imask) {
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (!(imask & (1u << f))) continue;
            const rsrc_t rr = rs_pub(a.pubR, ex, f), rw = rs_pub(a.pubW, ex, f),
                         rs = rs_pub(a.pubS, ex, f);
#pragma unroll
            for (int j = 0; j < RNPT; ++j) {
                if (rmask & (1u << j)) {
                    stf<kCoherent>(rr, gk(j), vr[f][j]);
                    stf<kCoherent>(rw, gk(j), vw[f][j]);
                    stf<kCoherent>(rs, gk(j), vs[f][j]);
                }
            }
        }
        // boundary columns: whole records, 16 bytes a store (an idle field's slots
        // carry its frozen values, which no reader uses)
        const rsrc_t rc = rs_col(ex);
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            if (!(cmask & (1u << j))) continue;
            float rec[RS];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                rec[f] = vr[f][j];
                rec[F + f] = vw[f][j];
                rec[2 * F + f] = vs[f][j];
            }
#pragma unroll
            for (int c = 3 * F; c < RS; ++c) rec[c] = 0.f;
#pragma unroll
            for (int c = 0; c < RS / 4; ++c) st4f<kCoherent>(rc, gk(j) * (RS * 4), 16 * c, rec + 4 * c);
        }
    };

    for (int outer = 0; alive; ++outer) {
        // ---- R: x += d (outer > 0: the correction of the last inner solve), then
        //      r = b - M x in FP64 and r_T = (float) r.  The ring's x is its owner's
        //      published x plus the ring copy of d, or (outer 0) the start computed
        //      from the inputs the owner computes it from, so no barrier separates
        //      the fold (or the start) from the residual.  With outer > 0, x rounded
        //      to FP32 is stored as the result: final if this residual ends the
        //      field's solve, overwritten by the next residual phase otherwise.
        {
            const int pin = (outer + 1) & 1, pout = outer & 1;   // pubX parity read / written
            double pr[3 * F];
#pragma unroll
            for (int q = 0; q < 3 * F; ++q) pr[q] = 0.0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (s_done[f]) continue;
                const rsrc_t rx = rs_x64(f), rb = rs_b(f);
                const rsrc_t rpr = rs_pub(a.pubR, ex, f), rpc = rs_col(ex);
                // every load of the field is issued before the first LDS write or
                // global store: the ring slot of this thread (at most one), then x and
                // b of the own nodes (a node outside the mesh reads element 0, never
                // written)
                int hq = -1;
                double hx = 0.0;
                if (threadIdx.x < nhalo) {
                    int lc, lr;
                    halo_slot(threadIdx.x, txa, tya, lc, lr);
                    hq = lidx(lc, lr);
                    const int gh = gidx(m, i0, j0, lc, lr);
                    hx = outer > 0 ? ldd<kCoherent>(rs_pubX(pin, f), gh) +
                                         (double)rpd[(F + f) * NH + threadIdx.x]
                                   : start_value(a, f, gh);
                }
                double xo[RNPT];
                float bo[RNPT];
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    const int kk = (amask & (1u << j)) ? gk(j) : 0;
                    xo[j] = ldd<kPlain>(rx, kk);
                    bo[j] = ldf<kPlain>(rb, kk);
                }
                if (outer > 0) {
#pragma unroll
                    for (int j = 0; j < RNPT; ++j) xo[j] += (double)vd[f][j];
                }
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    if (!(amask & (1u << j))) continue;
                    ld64[qj(j)] = xo[j];
                    lb[qj(j)] = bo[j];
                }
                if (hq >= 0) ld64[hq] = hx;
                if (outer > 0) {
                    const rsrc_t ro = rs_d(f), rpx = rs_pubX(pout, f);
#pragma unroll
                    for (int j = 0; j < RNPT; ++j) {
                        if (!(amask & (1u << j))) continue;
                        const int kk = gk(j);
                        std8<kPlain>(rx, kk, xo[j]);
                        stf<kPlain>(ro, kk, (float)xo[j]);
                        if (bmask & (1u << j)) std8<kCoherent>(rpx, kk, xo[j]);
                    }
                }
                __syncthreads();
                // the FP32 residual replaces b in LDS (a node's b is read only by its
                // own thread) and goes into the registers of the CG start; b was staged
                // in LDS with x, so the loop issues no global load that would wait on
                // its stores
#pragma unroll 1
                for (int j = 0; j < RNPT; ++j) {
                    if (!(amask & (1u << j))) continue;
                    const int q = qj(j), qc = qcj(j);
                    const double mx = stencil64(
                        cf[qc], cf[CN + qc], cf[CN + qc - 1], cf[2 * CN + qc], cf[2 * CN + qc - CW],
                        cf[3 * CN + qc], cf[3 * CN + qc - CW - 1], ld64[q], ld64[q + 1],
                        ld64[q - 1], ld64[q + LW], ld64[q - LW], ld64[q + LW + 1],
                        ld64[q - LW - 1]);
                    const int kk = gk(j);
                    const double bk = (double)lb[q];
                    const double r64 = bk - mx;
                    const float rt = (float)r64;
                    lb[q] = rt;
                    pr[f] = sq_acc(pr[f], r64);
                    if (outer == 0) pr[2 * F + f] = sq_acc(pr[2 * F + f], bk);
                    if (rmask & (1u << j)) stf<kCoherent>(rpr, kk, rt);
                    if (cmask & (1u << j)) st1f<kCoherent>(rpc, kk * (RS * 4), 4 * f, rt);
                }
#pragma unroll
                for (int j = 0; j < RNPT; ++j)
                    if (amask & (1u << j)) vr[f][j] = lb[qj(j)];
                __syncthreads();
            }
            block_sum_to<3 * F>(pr, red_lds, vals);
        }
        alive = sync_reduce(a.sy, ++epoch, vals, 3 * F, nblocks);
        if (!alive) break;
        // refinement decision, one thread per field
        if (threadIdx.x < F && !s_done[threadIdx.x]) {
            const int f = threadIdx.x;
            s_refines[f] += 1;
            s_res[f] = outer > 0;
            if (outer == 0) s_bb[f] = vals[2 * F + f];
            const double bb = s_bb[f];
            const double rr = vals[f];
            const double relres = bb == 0.0 ? 0.0 : sqrt(rr / bb);
            s_relres[f] = relres;
            if (bb == 0.0) {
                s_zero[f] = 1;
                s_done[f] = 1;
            } else if (relres <= a.opts.tol || outer >= a.opts.max_refine ||
                       s_iters[f] >= a.opts.maxit || !(relres == relres)) {
                s_done[f] = 1;
                if (!(relres <= a.opts.tol)) atomicOr(&s_flags, (uint32_t)P2M_FLAG_NOT_CONVERGED);
            } else {
                const double goal = 0.25 * a.opts.tol * a.opts.tol * bb;
                const double rel = a.opts.inner_rtol * a.opts.inner_rtol * rr;
                s_target[f] = goal > rel ? goal : rel;
                s_inner[f] = 1;
            }
        }
        __syncthreads();
        uint32_t imask = inner_mask();
        if (!imask) break;

        // ---- CG start: u = r / diag, w = M u, delta = (w, u), gamma = (r, u);
        //      p = s = d = 0, and the ring copies of p and d (r is in registers
        //      since the residual phase) ----------------------------------------
        if (threadIdx.x < nhalo) {
            const int h = threadIdx.x;
            int lc, lr;
            halo_slot(h, txa, tya, lc, lr);
            const int gh = gidx(m, i0, j0, lc, lr);
            float hv[F];
            if (lr >= 0 && lr < tya) {   // a column slot: the neighbour's record
                float rec[4];
                ld4f<kCoherent>(rs_col(ex), gh * (RS * 4), 0, rec);
#pragma unroll
                for (int f = 0; f < F; ++f) hv[f] = rec[f];
            } else {
#pragma unroll
                for (int f = 0; f < F; ++f) hv[f] = ldf<kCoherent>(rs_pub(a.pubR, ex, f), gh);
            }
            const float dh = dv[lidx(lc, lr)];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                lf[(size_t)f * LH * LW + lidx(lc, lr)] = __fmul_rn(hv[f], dh);
                rpd[f * NH + h] = 0.f;
                rpd[(F + f) * NH + h] = 0.f;
            }
        }
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (!(imask & (1u << f))) continue;
            float* L = lf + (size_t)f * LH * LW;
#pragma unroll
            for (int j = 0; j < RNPT; ++j)
                if (amask & (1u << j)) L[qj(j)] = __fmul_rn(vr[f][j], dv[qj(j)]);
        }
        __syncthreads();
        ex ^= 1;
        {
            spmv_all(imask);
            // the boundary's (r, w, s) go out as soon as w is known, so their
            // latency overlaps the dot products; nothing loads from global memory
            // between them and the barrier, which waits for them
            publish_rws(imask);
            double pd[2 * F];
#pragma unroll
            for (int f = 0; f < 2 * F; ++f) pd[f] = 0.0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    vs[f][j] = 0.f;
                    vp[f][j] = 0.f;
                    vd[f][j] = 0.f;
                    if (!(amask & (1u << j))) continue;
                    const float uj = lf[(size_t)f * LH * LW + qj(j)];
                    pd[f] = dot_acc(pd[f], vw[f][j], uj);
                    pd[F + f] = dot_acc(pd[F + f], vr[f][j], uj);
                }
            }
            block_sum_to<2 * F>(pd, red_lds, vals);
        }
        alive = sync_reduce(a.sy, ++epoch, vals, 2 * F, nblocks);
        if (!alive) break;
        if (threadIdx.x < F && s_inner[threadIdx.x]) {
            const int f = threadIdx.x;
            const double del = vals[f], gam = vals[F + f];
            if (!(del > 0.0) || !(gam > 0.0)) {
                s_inner[f] = 0;
                s_done[f] = 1;
                atomicOr(&s_flags, (uint32_t)(P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED));
            } else {
                s_gam[f] = gam;
                s_alpha[f] = gam / del;
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
            // residual from their published state, all fields' loads in flight; the
            // ring copies of p and d advance with the u they held
            if (threadIdx.x < nhalo) {
                const int h = threadIdx.x;
                int lc, lr;
                halo_slot(h, txa, tya, lc, lr);
                const int gh = gidx(m, i0, j0, lc, lr);
                float ro[F], wo[F], so[F];
                if (lr >= 0 && lr < tya) {   // a column slot: the neighbour's record
                    float rec[RS];
                    const rsrc_t rc = rs_col(ex);
#pragma unroll
                    for (int c = 0; c < RS / 4; ++c) ld4f<kCoherent>(rc, gh * (RS * 4), 16 * c, rec + 4 * c);
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        ro[f] = rec[f];
                        wo[f] = rec[F + f];
                        so[f] = rec[2 * F + f];
                    }
                } else {
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        ro[f] = ldf<kCoherent>(rs_pub(a.pubR, ex, f), gh);
                        wo[f] = ldf<kCoherent>(rs_pub(a.pubW, ex, f), gh);
                        so[f] = ldf<kCoherent>(rs_pub(a.pubS, ex, f), gh);
                    }
                }
                const int q = lidx(lc, lr);
                const float dh = dv[q];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    if (!(imask & (1u << f))) continue;
                    float* L = lf + (size_t)f * LH * LW;
                    const float pn = fmaf(bf[f], rpd[f * NH + h], L[q]);
                    rpd[f * NH + h] = pn;
                    rpd[(F + f) * NH + h] = fmaf(af[f], pn, rpd[(F + f) * NH + h]);
                    L[q] = halo_u(af[f], bf[f], dh, ro[f], wo[f], so[f]);
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
                    const float un = pcg_update(al, be, dv[qj(j)], vp[f][j], vd[f][j], vs[f][j],
                                                vr[f][j], vw[f][j]);
                    if (amask & (1u << j)) L[qj(j)] = un;
                }
            }
            __syncthreads();
            ex ^= 1;
            {
                spmv_all(imask);
                publish_rws(imask);
                double pg[3 * F];
#pragma unroll
                for (int q = 0; q < 3 * F; ++q) pg[q] = 0.0;
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    if (!(imask & (1u << f))) continue;
#pragma unroll
                    for (int j = 0; j < RNPT; ++j) {
                        if (!(amask & (1u << j))) continue;
                        const float uj = lf[(size_t)f * LH * LW + qj(j)];
                        pg[f] = dot_acc(pg[f], vr[f][j], uj);
                        pg[F + f] = dot_acc(pg[F + f], vw[f][j], uj);
                        pg[2 * F + f] = dot_acc(pg[2 * F + f], vr[f][j], vr[f][j]);
                    }
                }
                // no barrier before the block sum: it orders its own LDS use, and the
                // planes are written next after the grid barrier
                block_sum_to<3 * F>(pg, red_lds, vals);
            }
            alive = sync_reduce(a.sy, ++epoch, vals, 3 * F, nblocks);
            if (!alive) break;
            // CG step decision, one thread per field
            if (threadIdx.x < F && s_inner[threadIdx.x]) {
                const int f = threadIdx.x;
                const double gam = vals[f], del = vals[F + f], rho = vals[2 * F + f];
                s_iters[f] += 1;
                if (!(rho > s_target[f]) || s_iters[f] >= a.opts.maxit) {
                    s_inner[f] = 0;
                } else {
                    const double beta = gam / s_gam[f];
                    const double den = del - beta * gam / s_alpha[f];
                    if (!(den > 0.0) || !(gam > 0.0)) {
                        s_inner[f] = 0;
                        atomicOr(&s_flags, (uint32_t)P2M_FLAG_BREAKDOWN);
                    } else {
                        s_alpha[f] = gam / den;
                        s_gam[f] = gam;
                        s_af[f] = (float)s_alpha[f];
                        s_bf[f] = (float)beta;
                    }
                }
            }
            __syncthreads();
            if (!inner_mask()) break;
        }
        // the iteration state is dead until the next CG start sets it: constant
        // here, it holds no registers through the residual phase (d does: the
        // residual phase folds it into x)
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
            for (int j = 0; j < RNPT; ++j) vp[f][j] = vs[f][j] = vr[f][j] = vw[f][j] = 0.f;
    }

    if (!alive && threadIdx.x == 0) s_flags |= P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED;
    __syncthreads();
    // result of the fields that no residual phase with outer > 0 ended (solved by
    // the start, b == 0, or an aborted solve): the FP64 solution rounded to FP32, 0
    // for fields with b == 0
    {
        float res[F][RNPT];
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (alive && s_res[f] && !s_zero[f]) continue;
#pragma unroll
            for (int j = 0; j < RNPT; ++j)
                if (amask & (1u << j)) res[f][j] = (float)ldd<kPlain>(rs_x64(f), gk(j));
        }
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (alive && s_res[f] && !s_zero[f]) continue;
#pragma unroll
            for (int j = 0; j < RNPT; ++j)
                if (amask & (1u << j)) stf<kPlain>(rs_d(f), gk(j), s_zero[f] ? 0.f : res[f][j]);
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

// barrier counters to zero; with rep, that report too (one launch for both)
__global__ void k_sync_clear(unsigned* ctr, unsigned* root, unsigned* rel, unsigned* abort_,
                             p2m_report* rep) {
    const int t = threadIdx.x;
    if (t < kGroups * 32) { ctr[t] = 0u; rel[t] = 0u; }
    if (t < 32) { root[t] = 0u; abort_[t] = 0u; }
    if (rep) {
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
    s += al((size_t)2 * m.nn * rec_floats(F) * sizeof(float));   // pubC
    s += al((size_t)2 * F * m.nn * sizeof(double));       // pubX
    s += al((size_t)kGroups * 32 * sizeof(unsigned));     // ctr
    s += al((size_t)kGroups * 32 * sizeof(unsigned));     // rel
    s += 2 * al(32 * sizeof(unsigned));                   // root, abort
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
                              p2m_report* rep, bool clear_rep, long spin, hipStream_t stream) {
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
    a.pubC = (float*)p; p += al((size_t)2 * m.nn * rec_floats(F) * sizeof(float));
    a.pubX = (double*)p; p += al((size_t)2 * F * m.nn * sizeof(double));
    a.sy.ctr = (unsigned*)p; p += al((size_t)kGroups * 32 * sizeof(unsigned));
    a.sy.root = (unsigned*)p; p += al(32 * sizeof(unsigned));
    a.sy.rel = (unsigned*)p; p += al((size_t)kGroups * 32 * sizeof(unsigned));
    a.sy.abort = (unsigned*)p; p += al(32 * sizeof(unsigned));
    a.sy.part = (double*)p; p += al((size_t)2 * blocks * kNV * sizeof(double));
    a.sy.tot = (double*)p;
    a.sy.spin = spin;
    hipLaunchKernelGGL(k_sync_clear, dim3(1), dim3(kGroups * 32), 0, stream, a.sy.ctr, a.sy.root,
                       a.sy.rel, a.sy.abort, clear_rep ? rep : (p2m_report*)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void* fn = cgr_kernel(F);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {&a};
    // An ordinary launch: the stream has finished every earlier kernel, and the
    // grid (one workgroup per compute unit at most, checked by cgr_supported) is
    // then resident as a whole.  The barrier is the kernel's own counter tree, not
    // the cooperative-groups one, and every wait in it is bounded.  (A cooperative
    // launch added ~30 us of queue gaps around each solve.)
    return hipLaunchKernel(fn, dim3(blocks), dim3(RBS), args, 0, stream);
}

}  // namespace p2m
