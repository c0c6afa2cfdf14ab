// Register-resident mass-matrix solve with a degree-2 Chebyshev polynomial
// preconditioner (2D FP32, F <= 3).
//
// The same organisation as the Jacobi-preconditioned resident solve (k_cgr.hip):
// one 128 x 32 node tile per workgroup for the whole solve, CG vectors in
// registers, the tile's stencil in LDS, boundary values exchanged through
// device-coherent exchange planes, one grid barrier per CG iteration
// (Chronopoulos-Gear form), FP64 dot products, FP64 residual and refinement.
// Only the preconditioner differs: u = P r with
//
//     P = p(D^-1 M) D^-1,   p(lambda) = c0 + c1 lambda,
//
// the polynomial for which lambda p(lambda) = 1 - T2((hi + lo - 2 lambda) /
// (hi - lo)) / T2((hi + lo) / (hi - lo)) (T2 the Chebyshev polynomial of degree 2),
// i.e. u = c0 y + c1 D^-1 M y with y = D^-1 r.  Every particle of the P1 mass
// matrix touches at most three hats, so (sum_a psi_a x_a)^2 <= 3 sum_a psi_a^2
// x_a^2 and the eigenvalues of D^-1 M lie in (0, 3]; p is positive below
// hi + lo = 3.3, so P is symmetric positive definite and CG applies.  On the
// particle sets of the benchmarks it takes the iteration count from 13 to 8
// (8 particles per cell) and from about 60 to 35 (2 per cell).
//
// The extra product M y needs y on a ring two nodes deep around the tile: the
// boundary bands published by every tile are two nodes wide, and a tile rebuilds
// y = D^-1 (r - alpha (w + beta s)) on the whole two-deep ring from its
// neighbours' published (r, w, s) with the same FP32 operations the owners use,
// then u on the tile and its one-deep ring, so every halo value is bit-identical
// to its owner's.  Still one grid barrier per iteration.  As in the Jacobi kernel,
// each workgroup keeps the one-deep ring's copies of p and d (the owners' FP32
// operations on the same values), so the correction of an inner solve is folded
// into x inside the next residual phase, with no barrier of its own.
#include "cg_common.hpp"

namespace p2m {

namespace {

constexpr int G2 = 2;                    // ring depth
constexpr int LW2 = RX + 2 * G2;         // LDS row stride of the value planes
constexpr int LH2 = RY + 2 * G2;
constexpr int CW2 = RX + 2 * G2 - 1;     // coefficient region: [-G2, RX + G2 - 2] per axis
constexpr int CH2 = RY + 2 * G2 - 1;
constexpr int CN2 = CW2 * CH2;
constexpr int NH1 = 2 * (RX + 2) + 2 * RY;   // one-deep ring slots of a full tile

// the one-deep ring slot of local (lc, lr) in halo_slot's order, or -1
__device__ __forceinline__ int ring1_index(int lc, int lr, int txa, int tya) {
    const int row = txa + 2;
    if (lr == -1 && lc >= -1 && lc <= txa) return lc + 1;
    if (lr == tya && lc >= -1 && lc <= txa) return row + lc + 1;
    if (lc == -1 && lr >= 0 && lr < tya) return 2 * row + lr;
    if (lc == txa && lr >= 0 && lr < tya) return 2 * row + tya + lr;
    return -1;
}

struct CArgs {
    Mesh m;
    int tiles_x;
    float* coef;
    float* b;
    const float* w;
    float* xout;
    double* x64;
    float* pubR;
    float* pubW;
    float* pubS;
    float* pubC;
    double* pubX;      // [2][F][nn] published one-deep boundary of x64, by refinement parity
    RSync sy;
    int start;
    float c0, c1;      // the preconditioner polynomial
    p2m_solve_opts opts;
    p2m_report* rep;
};

// ring slot h (0 <= h < 2 G2 (txa + 2 G2) + 2 G2 tya) -> local (lc, lr): first the
// 2 G2 full rows below and above the tile, then the side columns.  Written with
// selects: assignments through the references in branches were lowered through
// a stack slot in scratch memory.
__device__ __forceinline__ bool ring2_slot(int h, int txa, int tya, int& lc, int& lr) {
    const int row = txa + 2 * G2;
    const int nrows = 2 * G2 * row;
    const bool in_rows = h < nrows;
    const int rr = h / row;
    const int hc = in_rows ? 0 : h - nrows;
    const int cc = hc / tya;
    const int lc_r = h - rr * row - G2;
    const int lr_r = rr < G2 ? rr - G2 : tya + (rr - G2);
    const int lr_c = hc - cc * tya;
    const int lc_c = cc < G2 ? cc - G2 : txa + (cc - G2);
    lc = in_rows ? lc_r : lc_c;
    lr = in_rows ? lr_r : lr_c;
    return h < nrows + 2 * G2 * tya;
}

// Jacobi-preconditioned CG update of one node with the previous preconditioned
// residual u_old given (it is no longer r / diag): p = u_old + beta p,
// d = d + alpha p, s = w + beta s, r = r - alpha s; returns y = r / diag.
__device__ __forceinline__ float pcg_update_u(float al, float be, float dinv, float u_old, float& p,
                                              float& d, float& s, float& r, float w) {
    p = fmaf(be, p, u_old);
    d = fmaf(al, p, d);
    s = fmaf(be, s, w);
    r = fmaf(-al, s, r);
    return __fmul_rn(r, dinv);
}

template <int F>
__global__ __launch_bounds__(RBS) void k_cgrc(CArgs a) {
    const Mesh& m = a.m;
    const int nn = m.nn;
    const int nblocks = gridDim.x;
    const int tile = blockIdx.x;
    const int i0 = (tile % a.tiles_x) * RX;
    const int j0 = (tile / a.tiles_x) * RY;
    const int txa = min(RX, m.nx - i0), tya = min(RY, m.ny - j0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = (RNPT / 2) * wave;
    const int nring2 = 2 * G2 * (txa + 2 * G2) + 2 * G2 * tya;   // two-deep ring
    const int nring1 = 2 * (txa + 2) + 2 * tya;                  // one-deep ring
    static_assert(2 * (RX + 2) + 2 * RY <= RBS, "one one-deep ring slot per thread");
    auto nrow = [&](int j) { return row0 + (j >> 1); };
    auto ncol = [&](int j) { return lane + 64 * (j & 1); };
    auto active = [&](int j) { return nrow(j) < tya && ncol(j) < txa; };
    const int kb = (j0 + row0) * m.nx + i0 + lane;
    auto gk = [&](int j) { return kb + (j >> 1) * m.nx + 64 * (j & 1); };
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

    constexpr size_t XB = (size_t)(F > 3 ? F : 3) * LH2 * LW2 * sizeof(float);
    __shared__ float cf[4 * CN2];
    __shared__ float dv[LH2 * LW2];
    __shared__ __align__(16) unsigned char xbuf[XB];
    float* lf = (float*)xbuf;
    double* ld64 = (double*)xbuf;
    float* lb = (float*)(ld64 + LH2 * LW2);
    // the one-deep ring's copies of p (field f at f * NH1) and d (at (F + f) * NH1)
    __shared__ float rpd[2 * F * NH1];
    __shared__ double red_lds[(RBS / 64) * kNV];
    __shared__ double vals[kNV];
    __shared__ double s_bb[F], s_gam[F], s_alpha[F], s_relres[F], s_target[F];
    __shared__ float s_af[F], s_bf[F];
    __shared__ int s_iters[F], s_refines[F], s_done[F], s_inner[F], s_zero[F], s_res[F];
    __shared__ uint32_t s_flags;
    __shared__ int s_any;

    auto lidx = [&](int lc, int lr) { return (lr + G2) * LW2 + (lc + G2); };
    auto cidx = [&](int lc, int lr) { return (lr + G2) * CW2 + (lc + G2); };
    auto inner_mask = [&]() {
        uint32_t mk = 0;
#pragma unroll
        for (int f = 0; f < F; ++f)
            if (s_inner[f]) mk |= 1u << f;
        return mk;
    };
    const int q0 = lidx(lane, row0);
    const int qc0 = cidx(lane, row0);
    auto qj = [&](int j) { return q0 + (j >> 1) * LW2 + 64 * (j & 1); };
    auto qcj = [&](int j) { return qc0 + (j >> 1) * CW2 + 64 * (j & 1); };
    const float c0 = a.c0, c1 = a.c1;

    float vp[F][RNPT], vd[F][RNPT], vs[F][RNPT], vr[F][RNPT], vw[F][RNPT];

    if (threadIdx.x < F) {
        const int f = threadIdx.x;
        s_iters[f] = 0; s_refines[f] = 0; s_done[f] = 0; s_inner[f] = 0; s_zero[f] = 0;
        s_res[f] = 0; s_relres[f] = 0.0; s_bb[f] = 0.0;
    }
    if (threadIdx.x == 0) s_flags = 0u;

    // active nodes; the one-deep boundary (the residual phase's exchange); the
    // two-deep bands published for the iterations: rows, columns
    uint32_t amask = 0, b1mask = 0, rmask = 0, cmask = 0;
#pragma unroll
    for (int j = 0; j < RNPT; ++j) {
        if (!active(j)) continue;
        amask |= 1u << j;
        const int lc = ncol(j), lr = nrow(j);
        if (lr < G2 || lr >= tya - G2) rmask |= 1u << j;
        if (lc < G2 || lc >= txa - G2) cmask |= 1u << j;
        if (lr == 0 || lr == tya - 1 || lc == 0 || lc == txa - 1) b1mask |= 1u << j;
    }
    const uint32_t bmask = rmask | cmask;

    // my one-deep ring slot (the extra stencil product is evaluated there too)
    int r1c = 0, r1r = 0;
    const bool has_r1 = (int)threadIdx.x < nring1 && halo_slot(threadIdx.x, txa, tya, r1c, r1r);

    // coefficients of the region around the tile ([-2, txa] x [-2, tya] minus the
    // tile: one entry per thread; a node's diagonal is 1 where it is an orphan),
    // and the inverse diagonals of the two-deep ring
    {
        const int cw = txa + 2 * G2 - 1, chh = tya + 2 * G2 - 1;
        const int nreg = cw * chh - txa * tya;
        static_assert(CN2 - RX * RY <= RBS, "one coefficient-region slot per thread");
        const int h = threadIdx.x;
        int eq = -1;
        float e0 = 0.f, e1 = 0.f, e2 = 0.f, e3 = 0.f, ew = 0.f;
        if (h < nreg) {
            // walk the region row by row, skipping the tile
            int lc = 0, lr = 0;
            {
                int hh = h;
                const int below = G2 * cw;   // rows -G2 .. -1
                if (hh < below) {
                    lr = hh / cw - G2;
                    lc = hh % cw - G2;
                } else {
                    hh -= below;
                    const int side = (cw - txa);   // per tile row: G2 left, G2 - 1 right
                    if (hh < side * tya) {
                        lr = hh / side;
                        const int s2 = hh % side;
                        lc = s2 < G2 ? s2 - G2 : txa + (s2 - G2);
                    } else {
                        hh -= side * tya;
                        lr = tya + hh / cw;
                        lc = hh % cw - G2;
                    }
                }
            }
            const int k = gidx(m, i0, j0, lc, lr);
            eq = cidx(lc, lr);
            e0 = a.coef[k];
            e1 = a.coef[(size_t)nn + k];
            e2 = a.coef[(size_t)2 * nn + k];
            e3 = a.coef[(size_t)3 * nn + k];
            ew = a.w[k];
        }
        if (eq >= 0) {
            cf[eq] = ew > 0.f ? e0 : 1.f;
            cf[CN2 + eq] = e1;
            cf[2 * CN2 + eq] = e2;
            cf[3 * CN2 + eq] = e3;
        }
        for (int hh = threadIdx.x; hh < nring2; hh += RBS) {
            int lc, lr;
            if (!ring2_slot(hh, txa, tya, lc, lr)) continue;
            const int k = gidx(m, i0, j0, lc, lr);
            dv[lidx(lc, lr)] = jacobi_inv(a.coef[k], a.w[k]);
        }
    }
    // ---- P: own coefficients into LDS, orphan regularisation, FP64 start ----------
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
            cf[CN2 + q] = pc[1][j];
            cf[2 * CN2 + q] = pc[2][j];
            cf[3 * CN2 + q] = pc[3][j];
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
                // the start's one-deep boundary, read by the second residual phase
                // (the first computes the ring's start itself)
                if (b1mask & (1u << j)) std8<kCoherent>(rs_pubX(0, f), k, x0);
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
    int ex = 0;
    bool alive = true;

    // M applied at LDS position q (plane L) with the coefficients at qc
    auto stencil_at = [&](const float* L, int q, int qc) {
        return stencil32(cf[qc], cf[CN2 + qc], cf[CN2 + qc - 1], cf[2 * CN2 + qc],
                         cf[2 * CN2 + qc - CW2], cf[3 * CN2 + qc], cf[3 * CN2 + qc - CW2 - 1], L[q],
                         L[q + 1], L[q - 1], L[q + LW2], L[q - LW2], L[q + LW2 + 1],
                         L[q - LW2 - 1]);
    };

    // The planes hold y = D^-1 r on the tile and the two-deep ring: replace them
    // with u = c0 y + c1 D^-1 (M y) on the tile and the one-deep ring (the values a
    // tile's own stencil product reads).  Node by node, as the stencil product
    // below: a node's seven coefficients serve every field.  The new values wait in
    // vw (dead here: the update has consumed w, the stencil product after this
    // recomputes it) until every thread has read the planes.
    auto precondition = [&](uint32_t imask) {
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            const int qc = qcj(j), q = qj(j);
            const float cD = cf[qc], cE = cf[CN2 + qc], cEw = cf[CN2 + qc - 1];
            const float cN = cf[2 * CN2 + qc], cNs = cf[2 * CN2 + qc - CW2];
            const float cNE = cf[3 * CN2 + qc], cNEsw = cf[3 * CN2 + qc - CW2 - 1];
            const float di = dv[q];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                const float* L = lf + (size_t)f * LH2 * LW2;
                const float t = stencil32(cD, cE, cEw, cN, cNs, cNE, cNEsw, L[q], L[q + 1], L[q - 1],
                                          L[q + LW2], L[q - LW2], L[q + LW2 + 1], L[q - LW2 - 1]);
                vw[f][j] = fmaf(c1, __fmul_rn(di, t), __fmul_rn(c0, L[q]));
            }
        }
        float ur[F];
#pragma unroll
        for (int f = 0; f < F; ++f) ur[f] = 0.f;
        if (has_r1) {
            const int q = lidx(r1c, r1r), qc = cidx(r1c, r1r);
            const float di = dv[q];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                const float* L = lf + (size_t)f * LH2 * LW2;
                ur[f] = fmaf(c1, __fmul_rn(di, stencil_at(L, q, qc)), __fmul_rn(c0, L[q]));
            }
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (!(imask & (1u << f))) continue;
            float* L = lf + (size_t)f * LH2 * LW2;
#pragma unroll
            for (int j = 0; j < RNPT; ++j)
                if (amask & (1u << j)) L[qj(j)] = vw[f][j];
            if (has_r1) L[lidx(r1c, r1r)] = ur[f];
        }
        __syncthreads();
    };

    // w = M u at the owned nodes for every inner-active field
    auto spmv_all = [&](uint32_t imask) {
#pragma unroll
        for (int j = 0; j < RNPT; ++j) {
            const int qc = qcj(j), q = qj(j);
            const float cD = cf[qc], cE = cf[CN2 + qc], cEw = cf[CN2 + qc - 1];
            const float cN = cf[2 * CN2 + qc], cNs = cf[2 * CN2 + qc - CW2];
            const float cNE = cf[3 * CN2 + qc], cNEsw = cf[3 * CN2 + qc - CW2 - 1];
            const bool on = amask & (1u << j);
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                const float* L = lf + (size_t)f * LH2 * LW2;
                const float acc = stencil32(cD, cE, cEw, cN, cNs, cNE, cNEsw, L[q], L[q + 1],
                                            L[q - 1], L[q + LW2], L[q - LW2], L[q + LW2 + 1],
                                            L[q - LW2 - 1]);
                vw[f][j] = on ? acc : 0.f;
            }
        }
    };

    // the two-deep bands' (r, w, s) into the exchange planes of parity ex
    auto publish_rws = [&](uint32_t imask) {
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (!(imask & (1u << f))) continue;
            const rsrc_t rr = rs_pub(a.pubR, ex, f), rw = rs_pub(a.pubW, ex, f),
                         rs = rs_pub(a.pubS, ex, f), rc = rs_col(ex);
#pragma unroll
            for (int j = 0; j < RNPT; ++j) {
                if (rmask & (1u << j)) {
                    stf<kCoherent>(rr, gk(j), vr[f][j]);
                    stf<kCoherent>(rw, gk(j), vw[f][j]);
                    stf<kCoherent>(rs, gk(j), vs[f][j]);
                }
                if (cmask & (1u << j)) {
                    const int vo = gk(j) * (RS * 4);
                    st1f<kCoherent>(rc, vo, 4 * f, vr[f][j]);
                    st1f<kCoherent>(rc, vo, 4 * (F + f), vw[f][j]);
                    st1f<kCoherent>(rc, vo, 4 * (2 * F + f), vs[f][j]);
                }
            }
        }
    };

    for (int outer = 0; alive; ++outer) {
        // ---- fold (outer > 0): x64 += d, x rounded to FP32 stored as the result
        //      (final if the next residual ends the field's solve, overwritten by a
        //      later fold otherwise), the one-deep boundary of x published with the
        //      parity of this refinement -------------------------------------------
        const int pin = (outer + 1) & 1, pout = outer & 1;   // pubX parity read / written
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (s_done[f] || outer == 0) continue;
            const rsrc_t rx = rs_x64(f), ro = rs_d(f), rpx = rs_pubX(pout, f);
            double xo[RNPT];
#pragma unroll
            for (int j = 0; j < RNPT; ++j) xo[j] = ldd<kPlain>(rx, (amask & (1u << j)) ? gk(j) : 0);
#pragma unroll
            for (int j = 0; j < RNPT; ++j) {
                if (!(amask & (1u << j))) continue;
                const int kk = gk(j);
                const double xv = xo[j] + (double)vd[f][j];
                std8<kPlain>(rx, kk, xv);
                stf<kPlain>(ro, kk, (float)xv);
                if (b1mask & (1u << j)) std8<kCoherent>(rpx, kk, xv);
            }
#pragma unroll
            for (int j = 0; j < RNPT; ++j) vd[f][j] = 0.f;
        }

        // ---- R: r = b - M x in FP64 (one-deep ring) and r_T = (float) r, published
        //      on the two-deep bands.  The ring's x is its owner's x of the previous
        //      refinement (published with the other parity) plus the ring copy of
        //      d, or (outer 0) the start computed from the inputs the owner computes
        //      it from, so no barrier separates the fold (or the start) from the
        //      residual. -------------------------------------------------------------
        {
            double pr[3 * F];
#pragma unroll
            for (int q = 0; q < 3 * F; ++q) pr[q] = 0.0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (s_done[f]) continue;
                const rsrc_t rx = rs_x64(f), rb = rs_b(f);
                const rsrc_t rpr = rs_pub(a.pubR, ex, f), rpc = rs_col(ex);
                // every load of the field is issued before the first LDS write or
                // global store
                int hq = -1;
                double hx = 0.0;
                if (has_r1) {
                    hq = lidx(r1c, r1r);
                    const int gh = gidx(m, i0, j0, r1c, r1r);
                    if (outer > 0) {
                        hx = ldd<kCoherent>(rs_pubX(pin, f), gh) +
                             (double)rpd[(F + f) * NH1 + threadIdx.x];
                    } else if (a.start != P2M_START_ZERO) {
                        const float wk = a.w[gh];
                        const size_t o = (size_t)f * nn + gh;
                        if (wk > 0.f)
                            hx = a.start == P2M_START_FLIP ? (double)a.b[o] / (double)wk
                                                           : (double)a.xout[o];
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
#pragma unroll 1
                for (int j = 0; j < RNPT; ++j) {
                    if (!(amask & (1u << j))) continue;
                    const int q = qj(j), qc = qcj(j);
                    const double mx = stencil64(
                        cf[qc], cf[CN2 + qc], cf[CN2 + qc - 1], cf[2 * CN2 + qc],
                        cf[2 * CN2 + qc - CW2], cf[3 * CN2 + qc], cf[3 * CN2 + qc - CW2 - 1],
                        ld64[q], ld64[q + 1], ld64[q - 1], ld64[q + LW2], ld64[q - LW2],
                        ld64[q + LW2 + 1], ld64[q - LW2 - 1]);
                    const int kk = gk(j);
                    const double bk = (double)lb[q];
                    const double r64 = bk - mx;
                    const float rt = (float)r64;
                    lb[q] = rt;   // replaces b (read by this thread only)
                    pr[f] = sq_acc(pr[f], r64);
                    if (outer == 0) pr[2 * F + f] = sq_acc(pr[2 * F + f], bk);
                    if (rmask & (1u << j)) stf<kCoherent>(rpr, kk, rt);
                    if (cmask & (1u << j)) st1f<kCoherent>(rpc, kk * (RS * 4), 4 * f, rt);
                }
                // the FP32 residual goes into the registers of the CG start
#pragma unroll
                for (int j = 0; j < RNPT; ++j)
                    if (amask & (1u << j)) vr[f][j] = lb[qj(j)];
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
                s_res[f] = outer > 0;
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

        // ---- CG start: y = D^-1 r (tile and two-deep ring), u = P r, w = M u,
        //      delta = (w, u), gamma = (r, u); p = s = d = 0, and the ring copies of
        //      p and d ------------------------------------------------------------
        uint32_t imask = inner_mask();
        if (has_r1) {
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                rpd[f * NH1 + threadIdx.x] = 0.f;
                rpd[(F + f) * NH1 + threadIdx.x] = 0.f;
            }
        }
        for (int h = threadIdx.x; h < nring2; h += RBS) {
            int lc, lr;
            if (!ring2_slot(h, txa, tya, lc, lr)) continue;
            const int gh = gidx(m, i0, j0, lc, lr);
            float hv[F];
            if (lr >= 0 && lr < tya) {   // a column band: the neighbour's record
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
                if (imask & (1u << f)) lf[(size_t)f * LH2 * LW2 + lidx(lc, lr)] = __fmul_rn(hv[f], dh);
        }
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if (!(imask & (1u << f))) continue;
            float* L = lf + (size_t)f * LH2 * LW2;
#pragma unroll
            for (int j = 0; j < RNPT; ++j)
                if (amask & (1u << j)) L[qj(j)] = __fmul_rn(vr[f][j], dv[qj(j)]);
        }
        __syncthreads();
        precondition(imask);
        ex ^= 1;
        {
            spmv_all(imask);
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
                    const float uj = lf[(size_t)f * LH2 * LW2 + qj(j)];
                    pd[f] = dot_acc(pd[f], vw[f][j], uj);
                    pd[F + f] = dot_acc(pd[F + f], vr[f][j], uj);
                }
            }
            block_sum_to<2 * F>(pd, red_lds, vals);
            publish_rws(imask);
        }
        alive = sync_reduce(a.sy, ++epoch, vals, 2 * F, nblocks);
        if (!alive) break;
        if (threadIdx.x == 0) {
            for (int f = 0; f < F; ++f) {
                if (!s_inner[f]) continue;
                const double del = vals[f], gam = vals[F + f];
                if (!(del > 0.0) || !(gam > 0.0)) {
                    s_inner[f] = 0; s_done[f] = 1;
                    s_flags |= P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED;
                    continue;
                }
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
            // y on the two-deep ring from the neighbours' published state
            for (int h = threadIdx.x; h < nring2; h += RBS) {
                int lc, lr;
                if (!ring2_slot(h, txa, tya, lc, lr)) continue;
                const int gh = gidx(m, i0, j0, lc, lr);
                float ro[F], wo[F], so[F];
                if (lr >= 0 && lr < tya) {
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
                // a one-deep ring slot: its copies of p and d advance with the u it
                // held (the planes hold u there until this overwrites it with y)
                const int h1 = ring1_index(lc, lr, txa, tya);
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    if (!(imask & (1u << f))) continue;
                    float* L = lf + (size_t)f * LH2 * LW2;
                    if (h1 >= 0) {
                        const float pn = fmaf(bf[f], rpd[f * NH1 + h1], L[q]);
                        rpd[f * NH1 + h1] = pn;
                        rpd[(F + f) * NH1 + h1] = fmaf(af[f], pn, rpd[(F + f) * NH1 + h1]);
                    }
                    L[q] = halo_u(af[f], bf[f], dh, ro[f], wo[f], so[f]);
                }
            }
            // local updates with the previous u (still in the planes), y = D^-1 r
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (!(imask & (1u << f))) continue;
                const float al = af[f], be = bf[f];
                float* L = lf + (size_t)f * LH2 * LW2;
#pragma unroll
                for (int j = 0; j < RNPT; ++j) {
                    const int q = qj(j);
                    const float yn = pcg_update_u(al, be, dv[q], L[q], vp[f][j], vd[f][j], vs[f][j],
                                                  vr[f][j], vw[f][j]);
                    if (amask & (1u << j)) L[q] = yn;
                }
            }
            __syncthreads();
            precondition(imask);
            ex ^= 1;
            {
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
                        const float uj = lf[(size_t)f * LH2 * LW2 + qj(j)];
                        pg[f] = dot_acc(pg[f], vr[f][j], uj);
                        pg[F + f] = dot_acc(pg[F + f], vw[f][j], uj);
                        pg[2 * F + f] = dot_acc(pg[2 * F + f], vr[f][j], vr[f][j]);
                    }
                }
                // no barrier before the block sum: it orders its own LDS use, and the
                // planes are written next after the grid barrier
                block_sum_to<3 * F>(pg, red_lds, vals);
                publish_rws(imask);
            }
            alive = sync_reduce(a.sy, ++epoch, vals, 3 * F, nblocks);
            if (!alive) break;
            if (threadIdx.x == 0) {
                int any = 0;
                for (int f = 0; f < F; ++f) {
                    if (!s_inner[f]) continue;
                    const double gam = vals[f], del = vals[F + f], rho = vals[2 * F + f];
                    s_iters[f] += 1;
                    if (!(rho > s_target[f]) || s_iters[f] >= a.opts.maxit) {
                        s_inner[f] = 0;
                        continue;
                    }
                    const double beta = gam / s_gam[f];
                    const double den = del - beta * gam / s_alpha[f];
                    if (!(den > 0.0) || !(gam > 0.0)) {
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

__global__ void k_sync_clear_c(unsigned* ctr, unsigned* root, unsigned* rel, unsigned* abort_,
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

const void* cgrc_kernel(int F) {
    switch (F) {
        case 1: return (const void*)k_cgrc<1>;
        case 2: return (const void*)k_cgrc<2>;
        case 3: return (const void*)k_cgrc<3>;
    }
    return nullptr;
}

}  // namespace

// The preconditioner polynomial: lambda p(lambda) = 1 - T2((hi + lo - 2 lambda) /
// (hi - lo)) / T2(sigma), sigma = (hi + lo) / (hi - lo), gives p = c0 + c1 lambda with
// c0 = 4 sigma / (delta (2 sigma^2 - 1)) and c1 = -2 / (delta^2 (2 sigma^2 - 1)),
// delta = (hi - lo) / 2.  [lo, hi] = [0.2, 3.1]: p > 0 below hi + lo = 3.3, above the
// eigenvalue bound 3 of D^-1 M.
void cgrc_coefficients(float& c0, float& c1) {
    const double lo = 0.2, hi = 3.1;
    const double delta = 0.5 * (hi - lo), sigma = (hi + lo) / (hi - lo);
    const double den = 2.0 * sigma * sigma - 1.0;
    c0 = (float)(4.0 * sigma / (delta * den));
    c1 = (float)(-2.0 / (delta * delta * den));
}

bool cgrc_supported(const Mesh& m, int F, int device) {
    if (m.dim != 2 || F < 1 || F > 3) return false;
    int cus = 0, per = 0, coop = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess ||
        !coop)
        return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, cgrc_kernel(F), RBS, 0) != hipSuccess)
        return false;
    return cgr_tiles(m) <= per * cus;
}

hipError_t launch_cg_resident_cheb(const Mesh& m, int F, float* coef, float* b, const float* w,
                                   float* x, int start, void* ws, const p2m_solve_opts& opts,
                                   p2m_report* rep, bool clear_rep, long spin, hipStream_t stream) {
    auto al = [](size_t v) { return (v + kAlign - 1) / kAlign * kAlign; };
    const int blocks = cgr_tiles(m);
    char* p = (char*)ws;
    CArgs a;
    a.m = m;
    a.tiles_x = (m.nx + RX - 1) / RX;
    a.coef = coef;
    a.b = b;
    a.w = w;
    a.xout = x;
    a.start = start;
    a.opts = opts;
    a.rep = rep;
    cgrc_coefficients(a.c0, a.c1);
    // the carve-up of the Jacobi resident solve's workspace (cgr_workspace_bytes)
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
    hipLaunchKernelGGL(k_sync_clear_c, dim3(1), dim3(kGroups * 32), 0, stream, a.sy.ctr, a.sy.root,
                       a.sy.rel, a.sy.abort, clear_rep ? rep : (p2m_report*)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void* fn = cgrc_kernel(F);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {&a};
    // an ordinary launch, as for the Jacobi resident solve: the grid (one workgroup per
    // compute unit at most, checked by cgrc_supported) is resident as a whole once the
    // stream's earlier kernels have finished; every wait of the barrier is bounded
    return hipLaunchKernel(fn, dim3(blocks), dim3(RBS), args, 0, stream);
}

}  // namespace p2m
