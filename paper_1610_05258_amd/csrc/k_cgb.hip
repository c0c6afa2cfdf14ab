// Batched mass-matrix solve: many independent 2D FP32 problems of uneven size in
// one persistent launch.
//
// The mathematics and every rounding step are those of the register-resident
// solve (k_cgr.hip): FP64 solution, FP64 residual and refinement outside, FP32
// Jacobi-preconditioned Chronopoulos-Gear conjugate gradients with FP64 dot
// products inside, on the same RX x RY node tiles with the same node-to-thread
// mapping.  What changes is the ownership:
//
//  * the solver tiles of all instances are numbered in one list (instance by
//    instance); workgroup g owns tiles g, g + G, g + 2G, ... for the whole solve
//    and streams each tile's CG vectors (p, d, s, r, w per field) from owner-only
//    arrays and its stencil coefficients into LDS, phase by phase;
//  * a tile's partial sums are formed exactly as in the resident kernel (same
//    thread sums, same block tree) and stored per tile;
//  * a synchronisation is two passes of the grid barrier tree: after the first
//    (all tile partials stored) the workgroup assigned to an instance reduces
//    that instance's tile partials in the resident kernel's fixed order (tile l,
//    l+32, ... per lane, then the 32-lane tree) and publishes its totals; after
//    the second every workgroup reads all totals and takes every instance's
//    decisions redundantly.  (A counter per instance would be cheaper in
//    passes, but many workgroups adding to one address serialise on it.);
//  * all instances step through the same phase sequence (fold, residual, CG
//    start, inner iterations); an (instance, field) pair that has converged, or
//    whose inner solve has ended, idles until the phase it needs comes round.
//
// Each (instance, field) pair therefore performs the operations of the resident
// solve of that instance alone, in the same order: the batched result equals the
// single-problem result bit for bit.
#include <string.h>

#include "cg_common.hpp"

namespace p2m {

namespace {

struct BArgs {
    const BatchInst* inst;
    int nprob;
    const int32_t* rmap;
    const int32_t* order;   // dealing order of the tiles (null: 0, 1, 2, ...)
    int ntiles;
    float* coef;        // [4][nn] blocks at 4*no (orphan diagonals set to 1 here)
    float* b;           // [F][nn] blocks at F*no (orphan entries set to 0 here)
    const float* w;     // [nn] blocks at no
    float* sP;          // CG state [F][nn] blocks at F*no, owner-only
    float* sD;
    float* sS;
    float* sR;
    float* sW;
    double* x64;        // [F][nn] blocks at F*no, owner-only
    float* pubR;        // [2][F][nn] blocks at 2*F*no, published boundary-row values
    float* pubW;
    float* pubS;
    float* pubC;        // [2][nn][rec_floats(F)] blocks at 2*rec_floats(F)*no, boundary-column records
    double* pubX;       // [F][nn] blocks at F*no
    RSync sy;           // part: [2][ntiles][kNV]; tot: [2][nprob][kNV]
    int start;
    p2m_solve_opts opts;
};

template <int F>
__global__ __launch_bounds__(RBS) void k_cgb(BArgs a) {
    const int G = gridDim.x, g = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = (RNPT / 2) * wave;

    constexpr int CW = RX + 1, CN = (RY + 1) * (RX + 1);
    // xbuf: the F FP32 planes of the CG iterations, or (residual phase) one FP64
    // plane of x followed by one FP32 plane of b
    constexpr size_t XB = (size_t)(F > 3 ? F : 3) * LH * LW * sizeof(float);
    static_assert(2 * (RX + 2) + 2 * RY <= RBS, "one ring slot per thread");
    __shared__ float cf[4 * CN];
    __shared__ float dv[LH * LW];   // Jacobi inverse diagonal of the tile and its ring
    __shared__ __align__(16) unsigned char xbuf[XB];
    float* lf = (float*)xbuf;
    double* ld64 = (double*)xbuf;
    float* lb = (float*)(ld64 + LH * LW);
    __shared__ double red_lds[(RBS / 64) * kNV];
    __shared__ double tv[kNV];                         // block sums of the current tile
    __shared__ double vals[3 * kBatchMaxPairs];        // instance totals, [k * nv + j]
    __shared__ double s_bb[kBatchMaxPairs], s_gam[kBatchMaxPairs], s_alpha[kBatchMaxPairs],
        s_relres[kBatchMaxPairs], s_target[kBatchMaxPairs];
    __shared__ float s_af[kBatchMaxPairs], s_bf[kBatchMaxPairs];
    __shared__ int s_iters[kBatchMaxPairs], s_refines[kBatchMaxPairs];
    __shared__ unsigned char s_done[kBatchMaxPairs], s_inner[kBatchMaxPairs],
        s_zero[kBatchMaxPairs];
    __shared__ uint32_t s_flags[kBatchMaxInstances];
    // the tiles of this workgroup: instance and tile number inside the instance
    __shared__ int t_k[kBatchMaxOwn], t_lt[kBatchMaxOwn];
    __shared__ int s_nown, s_ok;

    const int nprob = a.nprob;
    auto lidx = [&](int lc, int lr) { return (lr + 1) * LW + (lc + 1); };
    auto cidx = [&](int lc, int lr) { return (lr + 1) * CW + (lc + 1); };
    const int q0 = lidx(lane, row0);
    const int qc0 = cidx(lane, row0);
    auto qj = [&](int j) { return q0 + (j >> 1) * LW + 64 * (j & 1); };
    auto qcj = [&](int j) { return qc0 + (j >> 1) * CW + 64 * (j & 1); };
    auto nrow = [&](int j) { return row0 + (j >> 1); };
    auto ncol = [&](int j) { return lane + 64 * (j & 1); };

    // ---- set-up: own tiles, instance runs, per-pair state ---------------------
    if (threadIdx.x == 0) {
        int n = 0;
        for (int i = g; i < a.ntiles; i += G) {
            const int t = a.order ? a.order[i] : i;
            const int k = a.rmap[t];
            t_k[n] = k;
            t_lt[n] = t - a.inst[k].rt;
            ++n;
        }
        s_nown = n;
    }
    for (int p = threadIdx.x; p < nprob * F; p += RBS) {
        s_iters[p] = 0; s_refines[p] = 0; s_done[p] = 0; s_inner[p] = 0; s_zero[p] = 0;
        s_relres[p] = 0.0; s_bb[p] = 0.0;
    }
    for (int k = threadIdx.x; k < nprob; k += RBS) s_flags[k] = 0u;
    __syncthreads();
    const int nown = s_nown;

    // per-tile geometry and masks of this thread
    int k = 0, i0 = 0, j0 = 0, nx = 0, ny = 0, no = 0, nn = 0, txa = 0, tya = 0, nhalo = 0;
    uint32_t amask = 0, bmask = 0, rmask = 0, cmask = 0;   // active; boundary; boundary row; column
    int kb = 0;
    int cur = 0;   // the current tile's number in the batch
    auto set_tile = [&](int ti) {
        k = t_k[ti];
        const int lt = t_lt[ti];
        const BatchInst& I = a.inst[k];
        i0 = (lt % I.rtx) * RX;
        j0 = (lt / I.rtx) * RY;
        nx = I.m.nx;
        ny = I.m.ny;
        no = I.no;
        cur = I.rt + lt;
        nn = nx * ny;
        txa = min(RX, nx - i0);
        tya = min(RY, ny - j0);
        nhalo = 2 * (txa + 2) + 2 * tya;
        amask = 0;
        rmask = 0;
        cmask = 0;
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            const int lc = ncol(j), lr = nrow(j);
            if (!(lr < tya && lc < txa)) continue;
            amask |= 1u << j;
            if (lr == 0 || lr == tya - 1) rmask |= 1u << j;
            if (lc == 0 || lc == txa - 1) cmask |= 1u << j;
        }
        bmask = rmask | cmask;
        kb = (j0 + row0) * nx + i0 + lane;
    };
    auto gk = [&](int j) { return kb + (j >> 1) * nx + 64 * (j & 1); };
    auto ghalo = [&](int lc, int lr) {
        int gc = i0 + lc, gr = j0 + lr;
        if (gc < 0) gc += nx;
        if (gc >= nx) gc -= nx;
        if (gr < 0) gr += ny;
        if (gr >= ny) gr -= ny;
        return gc + nx * gr;
    };
    // descriptors of the current tile's instance blocks
    auto rs_f4 = [&](float* base, int f) {
        return mkrs(base + (size_t)F * no + (size_t)f * nn, (size_t)nn * 4);
    };
    auto rs_f8 = [&](double* base, int f) {
        return mkrs(base + (size_t)F * no + (size_t)f * nn, (size_t)nn * 8);
    };
    // The streamed CG state (p, d, s, r, w) is tile-blocked: tile T's block of
    // F x kTS floats holds field f at f * kTS, and this thread's nodes j = 0..3 and
    // j = 4..7 in two runs of four at 4 t and 4 RBS + 4 t, so a thread moves its
    // eight values of a vector with two 16-byte accesses.  Slots of nodes outside
    // the mesh are moved too and read as 0.
    static_assert(RNPT == 8, "two runs of four per thread");
    constexpr int kTS = RBS * RNPT;
    auto st_blk = [&](float* base, int f) {
        return base + ((size_t)cur * F + f) * kTS + (size_t)threadIdx.x * 4;
    };
    auto ld8 = [&](const float* q, float (&v)[RNPT]) {
        const float4 a0 = *reinterpret_cast<const float4*>(q);
        const float4 a1 = *reinterpret_cast<const float4*>(q + RBS * 4);
        const float t8[RNPT] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
        for (int j = 0; j < RNPT; ++j) v[j] = (amask & (1u << j)) ? t8[j] : 0.f;
    };
    auto st8 = [&](float* q, const float (&v)[RNPT]) {
        *reinterpret_cast<float4*>(q) = make_float4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<float4*>(q + RBS * 4) = make_float4(v[4], v[5], v[6], v[7]);
    };
    auto slot = [](int j) { return (j >> 2) * (RBS * 4) + (j & 3); };
    auto rs_pub = [&](float* base, int par, int f) {
        return mkrs(base + (size_t)2 * F * no + ((size_t)par * F + f) * nn, (size_t)nn * 4);
    };
    constexpr int RS = rec_floats(F);
    auto rs_col = [&](int par) {
        return mkrs(a.pubC + (size_t)2 * RS * no + (size_t)par * nn * RS, (size_t)nn * RS * 4);
    };
    auto inner_mask = [&]() {
        uint32_t mk = 0;
#pragma unroll
        for (int f = 0; f < F; ++f)
            if (s_inner[k * F + f]) mk |= 1u << f;
        return mk;
    };
    // the tile's stencil coefficients (and its left column / bottom row) into LDS,
    // with the Jacobi inverse diagonals of the tile and its ring when asked
    auto load_coef = [&](bool with_dinv) {
        const float* c = a.coef + (size_t)4 * no;
        const float* w = a.w + no;
        // every load before the first LDS write (a node outside the mesh reads
        // element 0 and is not written)
        float c0[RNPT], c1[RNPT], c2[RNPT], c3[RNPT], wv[RNPT];
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            const int kk = (amask & (1u << j)) ? gk(j) : 0;
            c0[j] = c[kk];
            c1[j] = c[(size_t)nn + kk];
            c2[j] = c[(size_t)2 * nn + kk];
            c3[j] = c[(size_t)3 * nn + kk];
            wv[j] = with_dinv ? w[kk] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            if (!(amask & (1u << j))) continue;
            const int q = qcj(j);
            cf[q] = c0[j];
            if (with_dinv) dv[qj(j)] = jacobi_inv(c0[j], wv[j]);
            cf[CN + q] = c1[j];
            cf[2 * CN + q] = c2[j];
            cf[3 * CN + q] = c3[j];
        }
        for (int h = threadIdx.x; h < txa + 1 + tya; h += RBS) {
            int lc, lr;
            if (h < txa + 1) { lr = -1; lc = h - 1; } else { lc = -1; lr = h - (txa + 1); }
            const int kk = ghalo(lc, lr);
            const int q = cidx(lc, lr);
            cf[CN + q] = c[(size_t)nn + kk];
            cf[2 * CN + q] = c[(size_t)2 * nn + kk];
            cf[3 * CN + q] = c[(size_t)3 * nn + kk];
        }
        if (with_dinv)
            for (int h = threadIdx.x; h < nhalo; h += RBS) {
                int lc, lr;
                if (!halo_slot(h, txa, tya, lc, lr)) continue;
                const int kk = ghalo(lc, lr);
                dv[lidx(lc, lr)] = jacobi_inv(c[kk], w[kk]);
            }
    };
    // store the current tile's block sums tv[0..nv) as its partials
    auto store_partials = [&](unsigned epoch, int nv) {
        double* part = a.sy.part + (size_t)(epoch & 1) * a.ntiles * kNV;
        // value-major: the lanes summing one value read consecutive words
        if (threadIdx.x < nv) st_c(&part[(size_t)threadIdx.x * a.ntiles + cur], tv[threadIdx.x]);
    };

    // Synchronisation `epoch` with nv values per instance: barrier (partials
    // stored), reduction of the assigned instances, barrier (totals stored),
    // totals into vals; with nv == 0 only the first barrier.  The barrier tree
    // counts its passes (tep), whatever the number of passes per epoch.
    // Returns false after an abort.
    unsigned tep = 0;
    auto sync_batch = [&](unsigned epoch, int nv) -> bool {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int par = epoch & 1;
        const double* part = a.sy.part + (size_t)par * a.ntiles * kNV;
        double* tot = a.sy.tot + (size_t)par * nprob * kNV;
        ++tep;
        if (threadIdx.x == 0) {
            if (tree_arrive(a.sy, tep, G)) tree_release(a.sy, tep);
            s_ok = tree_wait(a.sy, tep) ? 1 : 0;
        }
        __syncthreads();
        if (!s_ok) return false;
        if (nv == 0) return true;
        if (g < nprob) {
            for (int kk = g; kk < nprob; kk += G) {
                const BatchInst& I = a.inst[kk];
                double* tk = tot + (size_t)kk * kNV;
                sum_partials(part + I.rt, I.nrt, nv, 1, (size_t)a.ntiles,
                             [&](int jv, double v) { st_c(&tk[jv], v); });
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        ++tep;
        if (threadIdx.x == 0) {
            if (tree_arrive(a.sy, tep, G)) tree_release(a.sy, tep);
            s_ok = tree_wait(a.sy, tep) ? 1 : 0;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nprob * nv; i += RBS) {
            const int kk = i / nv, jv = i - kk * nv;
            vals[i] = ld_c(&tot[(size_t)kk * kNV + jv]);
        }
        __syncthreads();
        return s_ok != 0;
    };

    float vp[F][RNPT], vd[F][RNPT], vs[F][RNPT], vr[F][RNPT], vw[F][RNPT];

    // ---- P: orphan regularisation, FP64 start vector, d = 0 -------------------
    for (int ti = 0; ti < nown; ++ti) {
        set_tile(ti);
        const BatchInst& I = a.inst[k];
        float* c = a.coef + (size_t)4 * no;
        float* bb = a.b + (size_t)F * no;
        const float* w = a.w + no;
        double* x64 = a.x64 + (size_t)F * no;
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            if (!(amask & (1u << j))) continue;
            const int kk = gk(j);
            const float wk = w[kk];
            const bool orphan = !(wk > 0.f);
            if (orphan) c[kk] = 1.f;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const size_t o = (size_t)f * nn + kk;
                double x0;
                if (orphan) {
                    bb[o] = 0.f;
                    x0 = 0.0;
                } else if (a.start == P2M_START_FLIP) {
                    x0 = (double)bb[o] / (double)wk;
                } else if (a.start == P2M_START_ZERO) {
                    x0 = 0.0;
                } else {
                    x0 = (double)I.out[o];
                }
                x64[o] = x0;
                // the start's boundary values for the first residual (the first
                // fold, which would add d = 0, is skipped)
                if (bmask & (1u << j)) std8<kCoherent>(rs_f8(a.pubX, f), kk, x0);
            }
            if (orphan && I.rep) {
                atomicAdd(&I.rep->n_orphan, 1);
                atomicOr(&I.rep->flags, (uint32_t)P2M_FLAG_ORPHAN);
            }
        }
        // d = 0 (every slot of the tile's block)
        const float zero8[RNPT] = {};
#pragma unroll
        for (int f = 0; f < F; ++f) st8(st_blk(a.sD, f), zero8);
    }
    __syncthreads();

    unsigned epoch = 0;
    int ex = 0;
    bool alive = true;

    // w = M r at the owned nodes of the current tile for the fields in imask
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

    // the current tile's CG state (p, d, s, r, w) of every inner-active field into
    // the owner-only arrays, and its boundary (r, w, s) into the exchange planes
    // of parity ex ^ 1 (r only with_r: at the CG start it is already stored)
    auto store_state = [&](uint32_t imask, bool with_r) {
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (!(imask & (1u << f))) continue;
            const rsrc_t rr = rs_pub(a.pubR, ex ^ 1, f), rw = rs_pub(a.pubW, ex ^ 1, f),
                         rs = rs_pub(a.pubS, ex ^ 1, f), rc = rs_col(ex ^ 1);
            st8(st_blk(a.sP, f), vp[f]);
            st8(st_blk(a.sD, f), vd[f]);
            st8(st_blk(a.sS, f), vs[f]);
            if (with_r) st8(st_blk(a.sR, f), vr[f]);
            st8(st_blk(a.sW, f), vw[f]);
#pragma unroll
            for (int j = 0; j < RNPT; ++j) {
                if (!(amask & (1u << j))) continue;
                const int kk = gk(j);
                if (rmask & (1u << j)) {
                    stf<kCoherent>(rr, kk, vr[f][j]);
                    stf<kCoherent>(rw, kk, vw[f][j]);
                    stf<kCoherent>(rs, kk, vs[f][j]);
                }
                if (cmask & (1u << j)) {
                    const int vo = kk * (RS * 4);
                    st1f<kCoherent>(rc, vo, 4 * f, vr[f][j]);
                    st1f<kCoherent>(rc, vo, 4 * (F + f), vw[f][j]);
                    st1f<kCoherent>(rc, vo, 4 * (2 * F + f), vs[f][j]);
                }
            }
        }
    };

    for (int outer = 0; alive; ++outer) {
        // ---- fold the correction into x64, publish the boundary x64 ------------
        // (outer 0: the start vector, published by the P phase)
        for (int ti = 0; ti < nown && outer > 0; ++ti) {
            set_tile(ti);
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (s_done[k * F + f]) continue;
                const rsrc_t rx = rs_f8(a.x64, f), rpx = rs_f8(a.pubX, f);
                // the field's loads go out together, ahead of its stores (a load
                // issued after a store waits for it); a node outside the mesh reads
                // element 0
                double xo[RNPT];
                float dd[RNPT];
                ld8(st_blk(a.sD, f), dd);
#pragma unroll
                for (int j = 0; j < RNPT; ++j) xo[j] = ldd<kPlain>(rx, (amask & (1u << j)) ? gk(j) : 0);
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    if (!(amask & (1u << j))) continue;
                    const int kk = gk(j);
                    const double xv = xo[j] + (double)dd[j];
                    std8<kPlain>(rx, kk, xv);
                    if (bmask & (1u << j)) std8<kCoherent>(rpx, kk, xv);
                }
            }
        }
        alive = sync_batch(++epoch, 0);
        if (!alive) break;

        // ---- R: r = b - M x64 in FP64; r_T = (float) r -------------------------
        for (int ti = 0; ti < nown; ++ti) {
            set_tile(ti);
            bool all_done = true;
#pragma unroll
            for (int f = 0; f < F; ++f) all_done = all_done && s_done[k * F + f];
            if (all_done) continue;
            load_coef(false);
            double pr[3 * F];
#pragma unroll
            for (int q = 0; q < 3 * F; ++q) pr[q] = 0.0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (s_done[k * F + f]) continue;
                const rsrc_t rx = rs_f8(a.x64, f), rpx = rs_f8(a.pubX, f), rb = rs_f4(a.b, f);
                float* const rr = st_blk(a.sR, f);
                const rsrc_t rpr = rs_pub(a.pubR, ex, f), rpc = rs_col(ex);
                // every load of the field is issued before the first LDS write: the
                // ring slot of this thread (at most one), then x and b of the own
                // nodes (a node outside the mesh reads element 0, never written)
                int hq = -1;
                double hx = 0.0;
                if (threadIdx.x < nhalo) {
                    int lc, lr;
                    if (halo_slot(threadIdx.x, txa, tya, lc, lr)) {
                        hq = lidx(lc, lr);
                        hx = ldd<kCoherent>(rpx, ghalo(lc, lr));
                    }
                }
                double xo[RNPT];
                float bo[RNPT];
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    const int kk = (amask & (1u << j)) ? gk(j) : 0;
                    xo[j] = ldd<kPlain>(rx, kk);
                    bo[j] = ldf<kPlain>(rb, kk);
                }
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    if (!(amask & (1u << j))) continue;
                    ld64[qj(j)] = xo[j];
                    lb[qj(j)] = bo[j];
                }
                if (hq >= 0) ld64[hq] = hx;
                __syncthreads();
                // b was staged in LDS with x: the loop issues no global load that would
                // wait on its stores
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
                    rr[slot(j)] = rt;
                    pr[f] = sq_acc(pr[f], r64);
                    if (outer == 0) pr[2 * F + f] = sq_acc(pr[2 * F + f], bk);
                    if (rmask & (1u << j)) stf<kCoherent>(rpr, kk, rt);
                    if (cmask & (1u << j)) st1f<kCoherent>(rpc, kk * (RS * 4), 4 * f, rt);
                }
                __syncthreads();
            }
            block_sum_to<3 * F>(pr, red_lds, tv);
            store_partials(epoch + 1, 3 * F);
        }
        alive = sync_batch(++epoch, 3 * F);
        if (!alive) break;
        int any = 0;
        if (threadIdx.x < nprob) {
            const int kk = threadIdx.x;
            for (int f = 0; f < F; ++f) {
                const int p = kk * F + f;
                const double* v = vals + (size_t)kk * 3 * F;
                if (s_done[p]) continue;
                s_refines[p] += 1;
                if (outer == 0) s_bb[p] = v[2 * F + f];
                const double bb = s_bb[p];
                if (bb == 0.0) {
                    s_zero[p] = 1; s_done[p] = 1; s_relres[p] = 0.0;
                    continue;
                }
                const double rr = v[f];
                const double relres = sqrt(rr / bb);
                s_relres[p] = relres;
                if (relres <= a.opts.tol || outer >= a.opts.max_refine ||
                    s_iters[p] >= a.opts.maxit || !(relres == relres)) {
                    s_done[p] = 1;
                    if (!(relres <= a.opts.tol)) s_flags[kk] |= P2M_FLAG_NOT_CONVERGED;
                    continue;
                }
                const double goal = 0.25 * a.opts.tol * a.opts.tol * bb;
                const double rel = a.opts.inner_rtol * a.opts.inner_rtol * rr;
                s_target[p] = goal > rel ? goal : rel;
                s_inner[p] = 1;
                any = 1;
            }
        }
        if (!__syncthreads_or(any)) break;

        // ---- CG start: u = r / diag, w = M u, delta = (w, u), gamma = (r, u);
        //      p = s = d = 0 -----------------------------------------------------
        for (int ti = 0; ti < nown; ++ti) {
            set_tile(ti);
            const uint32_t imask = inner_mask();
            if (!imask) continue;
            load_coef(true);
            __syncthreads();
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                float* L = lf + (size_t)f * LH * LW;
                ld8(st_blk(a.sR, f), vr[f]);
#pragma unroll
                for (int j = 0; j < RNPT; ++j)
                    if (amask & (1u << j)) L[qj(j)] = __fmul_rn(vr[f][j], dv[qj(j)]);
            }
            for (int h = threadIdx.x; h < nhalo; h += RBS) {
                int lc, lr;
                if (!halo_slot(h, txa, tya, lc, lr)) continue;
                const int gh = ghalo(lc, lr);
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
                for (int f = 0; f < F; ++f)
                    if (imask & (1u << f))
                        lf[(size_t)f * LH * LW + lidx(lc, lr)] = __fmul_rn(hv[f], dh);
            }
            __syncthreads();
            spmv_all(imask);
            double pd[2 * F];
#pragma unroll
            for (int f = 0; f < 2 * F; ++f) pd[f] = 0.0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    vp[f][j] = vd[f][j] = vs[f][j] = 0.f;
                    if (!(amask & (1u << j))) continue;
                    const float uj = lf[(size_t)f * LH * LW + qj(j)];
                    pd[f] = dot_acc(pd[f], vw[f][j], uj);
                    pd[F + f] = dot_acc(pd[F + f], vr[f][j], uj);
                }
            }
            __syncthreads();
            block_sum_to<2 * F>(pd, red_lds, tv);
            store_partials(epoch + 1, 2 * F);
            store_state(imask, false);
        }
        ex ^= 1;
        alive = sync_batch(++epoch, 2 * F);
        if (!alive) break;
        if (threadIdx.x < nprob) {
            const int kk = threadIdx.x;
            for (int f = 0; f < F; ++f) {
                const int p = kk * F + f;
                if (!s_inner[p]) continue;
                const double del = vals[(size_t)kk * 2 * F + f];
                const double gam = vals[(size_t)kk * 2 * F + F + f];
                if (!(del > 0.0) || !(gam > 0.0)) {
                    s_inner[p] = 0; s_done[p] = 1;
                    s_flags[kk] |= P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED;
                    continue;
                }
                s_gam[p] = gam;
                s_alpha[p] = gam / del;
                s_af[p] = (float)s_alpha[p];
                s_bf[p] = 0.f;
            }
        }
        __syncthreads();

        // ---- inner iterations (one barrier each) -------------------------------
        while (alive) {
            for (int ti = 0; ti < nown; ++ti) {
                set_tile(ti);
                const uint32_t imask = inner_mask();
                if (!imask) continue;
                float af[F], bf[F];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    af[f] = s_af[k * F + f];
                    bf[f] = s_bf[k * F + f];
                }
                // every load of the tile is issued before any result is used: own
                // coefficients and state, then the ring (diagonal and weight, the
                // published state, and the edge coefficients of the left column and
                // bottom row); one ring slot per thread (nhalo < RBS)
                const float* c = a.coef + (size_t)4 * no;
                const float* w = a.w + no;
                float cD[RNPT], cE[RNPT], cN[RNPT], cNE[RNPT];
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    cD[j] = cE[j] = cN[j] = cNE[j] = 0.f;
                    if (!(amask & (1u << j))) continue;
                    const int kk = gk(j);
                    cD[j] = c[kk];
                    cE[j] = c[(size_t)nn + kk];
                    cN[j] = c[(size_t)2 * nn + kk];
                    cNE[j] = c[(size_t)3 * nn + kk];
                }
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    if (!(imask & (1u << f))) {
#pragma unroll
                        for (int j = 0; j < RNPT; ++j)
                            vp[f][j] = vd[f][j] = vs[f][j] = vr[f][j] = vw[f][j] = 0.f;
                        continue;
                    }
                    ld8(st_blk(a.sP, f), vp[f]);
                    ld8(st_blk(a.sD, f), vd[f]);
                    ld8(st_blk(a.sS, f), vs[f]);
                    ld8(st_blk(a.sR, f), vr[f]);
                    ld8(st_blk(a.sW, f), vw[f]);
                }
                {
                    int lc = 0, lr = 0;
                    if (threadIdx.x < nhalo && halo_slot(threadIdx.x, txa, tya, lc, lr)) {
                        const int gh = ghalo(lc, lr);
                        // a neighbour's stored diagonal may predate its owner's orphan
                        // fix in this launch: the orphan test reads w, never rewritten
                        const float dh = jacobi_inv(c[gh], w[gh]);
                        float ro[F], wo[F], so[F];
                        if (lr >= 0 && lr < tya) {   // a column slot: the neighbour's record
                            float rec[RS];
                            const rsrc_t rc = rs_col(ex);
#pragma unroll
                            for (int c4 = 0; c4 < RS / 4; ++c4)
                                ld4f<kCoherent>(rc, gh * (RS * 4), 16 * c4, rec + 4 * c4);
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
                        // edge coefficients: bottom row lc in [-1, txa), left column
                        // lr in [0, tya) (the only ring slots the stencil reads)
                        if ((lr == -1 && lc < txa) || (lc == -1 && lr >= 0 && lr < tya)) {
                            const int q = cidx(lc, lr);
                            cf[CN + q] = c[(size_t)nn + gh];
                            cf[2 * CN + q] = c[(size_t)2 * nn + gh];
                            cf[3 * CN + q] = c[(size_t)3 * nn + gh];
                        }
#pragma unroll
                        for (int f = 0; f < F; ++f) {
                            if (!(imask & (1u << f))) continue;
                            lf[(size_t)f * LH * LW + lidx(lc, lr)] =
                                halo_u(af[f], bf[f], dh, ro[f], wo[f], so[f]);
                        }
                    }
                }
                // own nodes: coefficients into LDS, the updates, u into the planes.
                // The own diagonal is already regularised (1 for an orphan, written
                // by this workgroup), so its reciprocal is the Jacobi factor.
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    if (!(amask & (1u << j))) continue;
                    const int qc = qcj(j);
                    cf[qc] = cD[j];
                    cf[CN + qc] = cE[j];
                    cf[2 * CN + qc] = cN[j];
                    cf[3 * CN + qc] = cNE[j];
                }
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    if (!(imask & (1u << f))) continue;
                    const float al = af[f], be = bf[f];
                    float* L = lf + (size_t)f * LH * LW;
#pragma unroll
                    for (int j = 0; j < RNPT; ++j) {
                        if (!(amask & (1u << j))) continue;
                        L[qj(j)] = pcg_update(al, be, jacobi_inv(cD[j], 1.f), vp[f][j], vd[f][j],
                                              vs[f][j], vr[f][j], vw[f][j]);
                    }
                }
                __syncthreads();
                spmv_all(imask);
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
                __syncthreads();
                block_sum_to<3 * F>(pg, red_lds, tv);
                store_partials(epoch + 1, 3 * F);
                // the tile's state and its published boundary go out last: a load
                // issued after a store waits for it
                store_state(imask, true);
            }
            ex ^= 1;
            alive = sync_batch(++epoch, 3 * F);
            if (!alive) break;
            int more = 0;
            if (threadIdx.x < nprob) {
                const int kk = threadIdx.x;
                for (int f = 0; f < F; ++f) {
                    const int p = kk * F + f;
                    if (!s_inner[p]) continue;
                    const double gam = vals[(size_t)kk * 3 * F + f];
                    const double del = vals[(size_t)kk * 3 * F + F + f];
                    const double rho = vals[(size_t)kk * 3 * F + 2 * F + f];
                    s_iters[p] += 1;
                    if (!(rho > s_target[p]) || s_iters[p] >= a.opts.maxit) {
                        s_inner[p] = 0;
                        continue;
                    }
                    const double beta = gam / s_gam[p];
                    const double den = del - beta * gam / s_alpha[p];
                    if (!(den > 0.0) || !(gam > 0.0)) {
                        s_inner[p] = 0;
                        s_flags[kk] |= P2M_FLAG_BREAKDOWN;
                        continue;
                    }
                    s_alpha[p] = gam / den;
                    s_gam[p] = gam;
                    s_af[p] = (float)s_alpha[p];
                    s_bf[p] = (float)beta;
                    more = 1;
                }
            }
            if (!__syncthreads_or(more)) break;
        }
    }

    if (!alive)
        for (int kk = threadIdx.x; kk < nprob; kk += RBS)
            s_flags[kk] |= P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED;
    __syncthreads();
    // result: the FP64 solution rounded to FP32 (0 for fields with b == 0)
    for (int ti = 0; ti < nown; ++ti) {
        set_tile(ti);
        float* out = a.inst[k].out;
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const rsrc_t rx = rs_f8(a.x64, f);
            const rsrc_t ro = mkrs(out + (size_t)f * nn, (size_t)nn * 4);
            const bool zero = s_zero[k * F + f] != 0;
#pragma unroll
            for (int j = 0; j < RNPT; ++j) {
                if (!(amask & (1u << j))) continue;
                stf<kPlain>(ro, gk(j), zero ? 0.f : (float)ldd<kPlain>(rx, gk(j)));
            }
        }
    }
    if (g == 0) {
        for (int kk = threadIdx.x; kk < nprob; kk += RBS) {
            p2m_report* rep = a.inst[kk].rep;
            if (!rep) continue;
            for (int f = 0; f < F; ++f) {
                rep->iters[f] = s_iters[kk * F + f];
                rep->refines[f] = s_refines[kk * F + f];
                rep->rel_residual[f] = s_relres[kk * F + f];
            }
            if (s_flags[kk]) atomicOr(&rep->flags, s_flags[kk]);
        }
    }
}

__global__ void k_sync_clear_b(unsigned* ctr, unsigned* root, unsigned* rel, unsigned* abort_) {
    for (int t = threadIdx.x; t < kGroups * 32; t += blockDim.x) {
        ctr[t] = 0u;
        rel[t] = 0u;
    }
    for (int t = threadIdx.x; t < 32; t += blockDim.x) {
        root[t] = 0u;
        abort_[t] = 0u;
    }
}

size_t al(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// one-instance table for a single problem solved by k_cgb: the entry is copied
// word by word from the kernel argument, every tile maps to instance 0
__global__ void k_single_table(BatchInst inst, int ntiles, uint32_t* __restrict__ tbl,
                               int32_t* __restrict__ rmap) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int kWords = (int)(sizeof(BatchInst) / sizeof(uint32_t));
    static_assert(sizeof(BatchInst) % sizeof(uint32_t) == 0, "table entry in words");
    if (t < kWords) tbl[t] = reinterpret_cast<const uint32_t*>(&inst)[t];
    if (t < ntiles) rmap[t] = 0;
}

}  // namespace

const void* cgb_kernel(int F) {
    switch (F) {
        case 1: return (const void*)k_cgb<1>;
        case 2: return (const void*)k_cgb<2>;
        case 3: return (const void*)k_cgb<3>;
    }
    return nullptr;
}

// Workgroups of the batched solve: one per CU at most (co-residency of the whole
// grid is what the barriers need), no more than the tiles, and enough that no
// workgroup owns more than kBatchMaxOwn tiles.  0 when the batch does not fit.
int cgb_grid(int F, int ntiles, int device) {
    const void* fn = cgb_kernel(F);
    if (!fn || ntiles < 1) return 0;
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, RBS, 0) != hipSuccess || per < 1)
        return 0;
    const long cap = (long)per * cus;
    const int G = (int)(ntiles < cap ? ntiles : cap);
    if ((long)G * kBatchMaxOwn < ntiles) return 0;
    return G;
}

size_t cgb_workspace_bytes(int F, int nprob, int ntiles, size_t nodes) {
    size_t s = 0;
    s += 5 * al((size_t)F * ntiles * RX * RY * sizeof(float));   // p, d, s, r, w (tile-blocked)
    s += al((size_t)F * nodes * sizeof(double));          // x64
    s += 3 * al((size_t)2 * F * nodes * sizeof(float));   // pubR, pubW, pubS
    s += al((size_t)2 * nodes * rec_floats(F) * sizeof(float));   // pubC
    s += al((size_t)F * nodes * sizeof(double));          // pubX
    s += al((size_t)kGroups * 32 * sizeof(unsigned));     // ctr
    s += al((size_t)kGroups * 32 * sizeof(unsigned));     // rel
    s += 2 * al(32 * sizeof(unsigned));                   // root, abort
    s += al((size_t)2 * ntiles * kNV * sizeof(double));   // part
    s += al((size_t)2 * nprob * kNV * sizeof(double));    // tot
    return s;
}

static int single_tiles(const Mesh& m) {
    return ((m.nx + RX - 1) / RX) * ((m.ny + RY - 1) / RY);
}

size_t cgt_workspace_bytes(const Mesh& m, int F) {
    const int nt = single_tiles(m);
    return al(sizeof(BatchInst)) + al((size_t)nt * sizeof(int32_t)) +
           cgb_workspace_bytes(F, 1, nt, (size_t)m.nn);
}

int cgt_grid(const Mesh& m, int F, int groups, int device) {
    if (m.dim != 2 || F < 1 || F > kResidentMaxFields) return 0;
    const int nt = single_tiles(m);
    const int cap = cgb_grid(F, nt, device);
    if (cap < 1) return 0;
    int G = groups > 0 && groups < cap ? groups : cap;
    if ((long)G * kBatchMaxOwn < nt) G = cap;
    return G;
}

hipError_t launch_cg_tiles(const Mesh& m, int F, float* coef, float* b, const float* w, float* x,
                           int start, void* ws, const p2m_solve_opts& opts, p2m_report* rep,
                           int groups, int device, long spin, hipStream_t stream) {
    const int nt = single_tiles(m);
    const int G = cgt_grid(m, F, groups, device);
    if (G < 1) return hipErrorInvalidValue;
    char* p = (char*)ws;
    BatchInst inst;
    memset(&inst, 0, sizeof(inst));
    inst.m = m;
    inst.out = x;
    inst.rep = rep;
    inst.rtx = (m.nx + RX - 1) / RX;
    inst.nrt = nt;
    BatchInst* tbl = (BatchInst*)p;
    p += al(sizeof(BatchInst));
    int32_t* rmap = (int32_t*)p;
    p += al((size_t)nt * sizeof(int32_t));
    const int nthreads = nt > 64 ? nt : 64;
    hipLaunchKernelGGL(k_single_table, dim3((nthreads + 255) / 256), dim3(256), 0, stream, inst, nt,
                       (uint32_t*)tbl, rmap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BatchSolveBufs bb;
    bb.inst = tbl;
    bb.nprob = 1;
    bb.rmap = rmap;
    bb.order = nullptr;
    bb.ntiles = nt;
    bb.coef = coef;
    bb.b = b;
    bb.w = w;
    bb.ws = p;
    bb.spin = spin;
    return launch_cg_batch(F, bb, (size_t)m.nn, G, start, opts, stream);
}

hipError_t launch_cg_batch(int F, const BatchSolveBufs& bb, size_t nodes, int grid, int start,
                           const p2m_solve_opts& opts, hipStream_t stream) {
    if (grid < 1 || bb.nprob < 1 || bb.nprob > kBatchMaxInstances ||
        bb.nprob * F > kBatchMaxPairs || (long)grid * kBatchMaxOwn < bb.ntiles)
        return hipErrorInvalidValue;
    const void* fn = cgb_kernel(F);
    if (!fn) return hipErrorInvalidValue;
    char* p = (char*)bb.ws;
    BArgs a;
    a.inst = bb.inst;
    a.nprob = bb.nprob;
    a.rmap = bb.rmap;
    a.order = bb.order;
    a.ntiles = bb.ntiles;
    a.coef = bb.coef;
    a.b = bb.b;
    a.w = bb.w;
    a.start = start;
    a.opts = opts;
    const size_t f4 = al((size_t)F * bb.ntiles * RX * RY * sizeof(float));
    a.sP = (float*)p; p += f4;
    a.sD = (float*)p; p += f4;
    a.sS = (float*)p; p += f4;
    a.sR = (float*)p; p += f4;
    a.sW = (float*)p; p += f4;
    a.x64 = (double*)p; p += al((size_t)F * nodes * sizeof(double));
    a.pubR = (float*)p; p += al((size_t)2 * F * nodes * sizeof(float));
    a.pubW = (float*)p; p += al((size_t)2 * F * nodes * sizeof(float));
    a.pubS = (float*)p; p += al((size_t)2 * F * nodes * sizeof(float));
    a.pubC = (float*)p; p += al((size_t)2 * nodes * rec_floats(F) * sizeof(float));
    a.pubX = (double*)p; p += al((size_t)F * nodes * sizeof(double));
    a.sy.ctr = (unsigned*)p; p += al((size_t)kGroups * 32 * sizeof(unsigned));
    a.sy.root = (unsigned*)p; p += al(32 * sizeof(unsigned));
    a.sy.rel = (unsigned*)p; p += al((size_t)kGroups * 32 * sizeof(unsigned));
    a.sy.abort = (unsigned*)p; p += al(32 * sizeof(unsigned));
    a.sy.part = (double*)p; p += al((size_t)2 * bb.ntiles * kNV * sizeof(double));
    a.sy.tot = (double*)p;
    a.sy.spin = bb.spin;
    hipLaunchKernelGGL(k_sync_clear_b, dim3(1), dim3(512), 0, stream, a.sy.ctr, a.sy.root,
                       a.sy.rel, a.sy.abort);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* args[] = {&a};
    return hipLaunchKernel(fn, dim3(grid), dim3(RBS), args, 0, stream);
}

}  // namespace p2m
