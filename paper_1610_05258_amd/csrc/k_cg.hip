// Mass-matrix solve M Abar = b (Sec. 2.4 eqs. (13), (19)) for F fields at once.
//
// Mixed-precision iterative refinement around conjugate gradients:
//   outer: the solution is kept in FP64 (x64); the true residual
//          r = b - M x64 is evaluated in FP64 from the stored coefficients;
//          stop when ||r||_2 / ||b||_2 <= tol for every field;
//   inner: Jacobi-preconditioned CG in T (FP32 on the FP32 path) on the
//          correction M d = r (u = r / diag M), with the stencil product, axpy
//          and vector updates in T, every field sharing each coefficient read,
//          and all dot products accumulated in FP64; the next outer step folds
//          d into x64 in FP64.
// The whole solve is one persistent kernel: grid-wide barriers separate the
// phases; reductions are per-block FP64 partials that every block sums in the
// same fixed order, so all blocks take identical decisions and the result is
// deterministic.  Every loop is bounded (maxit, max_refine), and so is every
// wait in the grid barrier: a wait that times out ends the solve in every block
// with the breakdown flag.
//
// Stencil storage (symmetric, periodic): D_k = M(k,k), E_k = M(k,k+x),
// N_k = M(k,k+y), NE_k = M(k,k+x+y) in 2D; D_k, E_k = M(k,k+1) in 1D.  The third
// form (an irregular sparse matrix, the particle mass matrix of a triangulation)
// keeps D_k and then every row's off-diagonal entries in up to `ew` slots, slot j
// of row k at [nn + j nn + k] with its column in ecol[j nn + k] (-1 ends the row).
#include <atomic>
#include <type_traits>

#include "cg_common.hpp"

namespace p2m {

namespace {

constexpr int kCgBlock = 256;
constexpr int kSlots = 3 * kMaxFields;  // partial slots per block and phase
// Grid-barrier words after the partials: the two-level counter tree of the tile
// solvers (group counters, root, per-group release copies, abort flag), zeroed
// before each launch.
constexpr int kBarWords = 2 * kGroups * 32 + 2 * 32;
constexpr size_t kBarBytes = (size_t)kBarWords * sizeof(unsigned);

__device__ __forceinline__ RSync bar_of(unsigned* w, long spin) {
    RSync s;
    s.spin = spin;
    s.ctr = w;
    s.root = w + kGroups * 32;
    s.rel = w + kGroups * 32 + 32;
    s.abort = w + 2 * kGroups * 32 + 32;
    s.part = nullptr;
    s.tot = nullptr;
    return s;
}

// Grid-wide barrier number `epoch` (1, 2, ...) of a launch whose blocks are all
// resident (the grid is sized from the occupancy).  The solve's vectors are
// exchanged through ordinary cached stores, so the barrier orders them itself:
// every wave waits for its own stores (the workgroup barrier does not), then one
// thread writes the XCD's L2 back (agent-scope release), arrives at the counter
// tree, waits for the release and invalidates the cached lines (agent-scope
// acquire) before the block goes on.  Returns false after a wait timed out here
// or in another block (the abort flag).
__device__ bool grid_barrier(const RSync& s, unsigned epoch) {
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (tree_arrive(s, epoch, gridDim.x)) tree_release(s, epoch);
        const bool ok = tree_wait(s, epoch);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    return s_ok != 0;
}

__global__ void k_bar_clear(unsigned* w) {
    for (int i = threadIdx.x; i < kBarWords; i += blockDim.x) w[i] = 0u;
}

template <typename T>
struct CgArgs {
    Mesh m;
    T* coef;           // stencil of M; the diagonal of orphan rows is set to 1 here
    T* b;              // right-hand sides; orphan entries are set to 0 here
    T* xout;           // [F][nn] correction d during the solve, the result at the end
    double* x64;       // [2][F][nn] solution in FP64 (ping-pong)
    T* r;
    T* p0;
    T* p1;
    T* q;
    double* partials;  // [2][gridDim][kSlots]
    T* dinv;           // [nn] inverse of the regularised diagonal (written here)
    const T* w;        // [nn] FLIP volumes (orphans: w == 0)
    int start;         // P2M_START_FLIP / ZERO / USER (xout holds the user start)
    long spin;         // polls before a grid-barrier wait gives up (< 0: at once)
    const int32_t* ecol;  // columns of the sparse-row form ([ew][nn]), else unused
    int ew;               // slots per row of that form
    p2m_solve_opts opts;
    p2m_report* rep;
};

struct Nbr {
    int k, xp, xm, yp, ym, pp, mm;
};

// neighbour indices of node k: k+x, k-x, k+y, k-y, k+x+y, k-x-y (2D); k+1, k-1 (1D)
template <int DIM>
__device__ __forceinline__ Nbr neighbours(const Mesh& m, int k) {
    Nbr n;
    n.k = k;
    if (DIM == 3) {
        n.xp = n.xm = n.yp = n.ym = n.pp = n.mm = k;
        return n;
    }
    if (DIM == 1) {
        n.xp = (k + 1 == m.nx) ? 0 : k + 1;
        n.xm = (k == 0) ? m.nx - 1 : k - 1;
        n.yp = n.ym = n.pp = n.mm = k;
        return n;
    }
    const int j = k / m.nx, i = k - j * m.nx;
    const int ip = (i + 1 == m.nx) ? 0 : i + 1, im = (i == 0) ? m.nx - 1 : i - 1;
    const int jp = (j + 1 == m.ny) ? 0 : j + 1, jm = (j == 0) ? m.ny - 1 : j - 1;
    n.xp = ip + m.nx * j;
    n.xm = im + m.nx * j;
    n.yp = i + m.nx * jp;
    n.ym = i + m.nx * jm;
    n.pp = ip + m.nx * jp;
    n.mm = im + m.nx * jm;
    return n;
}

// coefficients of row k: D_k, E_k, E_{k-x}, N_k, N_{k-y}, NE_k, NE_{k-x-y}
template <typename T>
struct Row {
    T d, e, ew, n, ns, ne, nesw;
};

template <typename T, int DIM>
__device__ __forceinline__ Row<T> load_row(const T* __restrict__ coef, int nn, const Nbr& n) {
    Row<T> r;
    r.d = coef[n.k];
    if (DIM == 3) {
        r.e = r.ew = r.n = r.ns = r.ne = r.nesw = (T)0;
        return r;
    }
    r.e = coef[(size_t)nn + n.k];
    r.ew = coef[(size_t)nn + n.xm];
    if (DIM == 2) {
        r.n = coef[(size_t)2 * nn + n.k];
        r.ns = coef[(size_t)2 * nn + n.ym];
        r.ne = coef[(size_t)3 * nn + n.k];
        r.nesw = coef[(size_t)3 * nn + n.mm];
    } else {
        r.n = r.ns = r.ne = r.nesw = (T)0;
    }
    return r;
}

// (M v)_k for a vector given by an accessor v(idx), in arithmetic type A
template <int DIM, typename A, typename T, typename V>
__device__ __forceinline__ A apply_row(const Row<T>& c, const Nbr& n, V&& v,
                                       const T* __restrict__ coef, const int32_t* __restrict__ ecol,
                                       int nn, int ew) {
    if (DIM == 3) {
        A s = (A)c.d * v(n.k);
        for (int j = 0; j < ew; ++j) {
            const int col = ecol[(size_t)j * nn + n.k];
            if (col < 0) break;
            s += (A)coef[(size_t)(j + 1) * nn + n.k] * v(col);
        }
        return s;
    }
    A s = (A)c.d * v(n.k) + (A)c.e * v(n.xp) + (A)c.ew * v(n.xm);
    if (DIM == 2)
        s += (A)c.n * v(n.yp) + (A)c.ns * v(n.ym) + (A)c.ne * v(n.pp) + (A)c.nesw * v(n.mm);
    return s;
}

// block-wide sum of NV doubles per thread; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* [4][NV] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double s = v[j];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_down(s, d, 64);
        v[j] = s;
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double s = 0.0;
            for (int w = 0; w < kCgBlock / 64; ++w) s += lds[w * NV + j];
            v[j] = s;
        }
    }
    __syncthreads();
}

template <int NV>
__device__ __forceinline__ void store_partials(double* __restrict__ dst, const double (&v)[NV]) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) dst[(size_t)blockIdx.x * kSlots + j] = v[j];
    }
}

// Sum of one phase's per-block partials over all blocks in a fixed order; every
// block computes the same totals into tot[0..NV).
template <int NV>
__device__ __forceinline__ void grid_total(const double* __restrict__ part, int nblocks,
                                           double* tot, double* lds) {
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int bk = threadIdx.x; bk < nblocks; bk += kCgBlock) {
        const double* pb = part + (size_t)bk * kSlots;
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] += pb[j];
    }
    block_sum<NV>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) tot[j] = acc[j];
    }
    __syncthreads();
}

__device__ __forceinline__ float recip(float d) { return __frcp_rn(d); }
__device__ __forceinline__ double recip(double d) { return 1.0 / d; }

template <typename T, int DIM, int F>
__global__ __launch_bounds__(kCgBlock) void k_cg(CgArgs<T> a) {
    const Mesh& m = a.m;
    const int nn = m.nn;
    const int nblocks = gridDim.x;
    const RSync bar =
        bar_of((unsigned*)((char*)a.partials + (size_t)2 * nblocks * kSlots * sizeof(double)),
               a.spin);
    unsigned epoch = 0;
    // a grid of one workgroup (small problems) synchronises with the workgroup
    // barrier, which also orders its global-memory accesses; the grid barrier's
    // device-wide handshake would cost microseconds per step
    auto gsync = [&]() -> bool {
        if (nblocks == 1) {
            __syncthreads();
            return true;
        }
        return grid_barrier(bar, ++epoch);
    };
    const size_t xstride = (size_t)F * nn;

    __shared__ double lds[(kCgBlock / 64) * kSlots];
    __shared__ double tot[kSlots];
    // per-field solver state, identical in every block
    __shared__ double s_bb[F], s_rho[F], s_target[F], s_alpha[F], s_beta[F], s_relres[F];
    __shared__ int s_iters[F], s_refines[F], s_done[F], s_inner[F], s_zero[F], s_xb[F];
    __shared__ uint32_t s_flags;
    __shared__ int s_any;

    // Totals of a phase's NV partials per thread into tot[0..NV): block sum, then
    // over the blocks in the fixed order of grid_total.  A grid of one block takes
    // its block sum as the total (what grid_total would add to it: zeros) and
    // needs no global exchange.
    auto phase_total = [&](auto& part, int ph) -> bool {
        constexpr int NV = sizeof(part) / sizeof(double);
        block_sum<NV>(part, lds);
        if (nblocks == 1) {
            if (threadIdx.x == 0) {
#pragma unroll
                for (int j = 0; j < NV; ++j) tot[j] = part[j];
            }
            __syncthreads();
            return true;
        }
        store_partials<NV>(a.partials + (ph & 1) * ((size_t)nblocks * kSlots), part);
        if (!gsync()) return false;
        grid_total<NV>(a.partials + (ph & 1) * ((size_t)nblocks * kSlots), nblocks, tot, lds);
        return true;
    };

    if (threadIdx.x < F) {
        const int f = threadIdx.x;
        s_iters[f] = 0;
        s_refines[f] = 0;
        s_done[f] = 0;
        s_inner[f] = 0;
        s_zero[f] = 0;
        s_xb[f] = 0;
        s_relres[f] = 0.0;
        s_bb[f] = 0.0;
        s_beta[f] = 0.0;
    }
    if (threadIdx.x == 0) s_flags = 0u;
    __syncthreads();

    int phase = 0;
    const int k0 = blockIdx.x * kCgBlock + threadIdx.x;
    const int kstride = nblocks * kCgBlock;
    T* p_old = a.p0;
    T* p_new = a.p1;

    // ---- P: orphan regularisation and the FP64 start vector -------------------
    // A node with w_i == 0 has every coefficient of its row and column equal to 0
    // (all particle weights of that node vanish); its row becomes the identity
    // with b_i = 0, so Abar_i = 0.  Start: FLIP = b/w, ZERO, USER = xout.
    for (int k = k0; k < nn; k += kstride) {
        const T wk = a.w[k];
        const bool orphan = !(wk > (T)0);
        if (orphan) a.coef[k] = (T)1;
        a.dinv[k] = orphan ? (T)1 : recip(a.coef[k]);
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const size_t o = (size_t)f * nn + k;
            double x0;
            if (orphan) {
                a.b[o] = (T)0;
                x0 = 0.0;
            } else if (a.start == P2M_START_FLIP) {
                x0 = (double)a.b[o] / (double)wk;
            } else if (a.start == P2M_START_ZERO) {
                x0 = 0.0;
            } else {
                x0 = (double)a.xout[o];
            }
            a.x64[o] = x0;
        }
        if (orphan && a.rep) {
            atomicAdd(&a.rep->n_orphan, 1);
            atomicOr(&a.rep->flags, (uint32_t)P2M_FLAG_ORPHAN);
        }
    }
    bool alive = gsync();

    for (int outer = 0; alive; ++outer) {
        // ---- R: fold the correction into x64 and evaluate r = b - M x64 in FP64 --
        // slots: [f] ||r64||^2, [F+f] (r_T, u) with r_T = (T)r64, u = r_T / diag,
        // [2F+f] ||b||^2 (first pass)
        {
            double part[3 * F];
#pragma unroll
            for (int j = 0; j < 3 * F; ++j) part[j] = 0.0;
            for (int k = k0; k < nn; k += kstride) {
                const Nbr n = neighbours<DIM>(m, k);
                const Row<T> c = load_row<T, DIM>(a.coef, nn, n);
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    if (s_done[f]) continue;
                    const double* xf = a.x64 + s_xb[f] * xstride + (size_t)f * nn;
                    const T* df = a.xout + (size_t)f * nn;
                    const bool fold = outer > 0;
                    auto y = [&](int idx) -> double {
                        return fold ? xf[idx] + (double)df[idx] : xf[idx];
                    };
                    const double mx = apply_row<DIM, double>(c, n, y, a.coef, a.ecol, nn, a.ew);
                    const double bk = (double)a.b[(size_t)f * nn + k];
                    const double r64 = bk - mx;
                    const T rt = (T)r64;
                    a.r[(size_t)f * nn + k] = rt;
                    a.x64[(s_xb[f] ^ 1) * xstride + (size_t)f * nn + k] = y(k);
                    part[f] += r64 * r64;
                    part[F + f] += (double)rt * (double)(rt * a.dinv[k]);
                    if (outer == 0) part[2 * F + f] += bk * bk;
                }
            }
            alive = phase_total(part, phase);
        }
        ++phase;
        if (!alive) break;
        if (threadIdx.x == 0) {
            int any = 0;
            for (int f = 0; f < F; ++f) {
                if (s_done[f]) continue;
                s_xb[f] ^= 1;  // the folded solution now lives in the other buffer
                s_refines[f] += 1;
                if (outer == 0) s_bb[f] = tot[2 * F + f];
                const double bb = s_bb[f];
                if (bb == 0.0) {  // b == 0: the solution is 0
                    s_zero[f] = 1;
                    s_done[f] = 1;
                    s_relres[f] = 0.0;
                    continue;
                }
                const double rr = tot[f];
                const double relres = sqrt(rr / bb);
                s_relres[f] = relres;
                if (relres <= a.opts.tol || outer >= a.opts.max_refine ||
                    s_iters[f] >= a.opts.maxit || !(relres == relres)) {
                    s_done[f] = 1;
                    if (!(relres <= a.opts.tol)) s_flags |= P2M_FLAG_NOT_CONVERGED;
                    continue;
                }
                s_rho[f] = tot[F + f];
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

        // ---- inner CG on M d = r, d starts at 0 ---------------------------------
        for (int it = 0;; ++it) {
            // A: p_new = u + beta p_old with u = r / diag (at the node and its
            //    neighbours), q = M p_new
            {
                double part[F];
#pragma unroll
                for (int j = 0; j < F; ++j) part[j] = 0.0;
                for (int k = k0; k < nn; k += kstride) {
                    const Nbr n = neighbours<DIM>(m, k);
                    const Row<T> c = load_row<T, DIM>(a.coef, nn, n);
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        if (!s_inner[f]) continue;
                        const T* rf = a.r + (size_t)f * nn;
                        const T* pf = p_old + (size_t)f * nn;
                        const T beta = (T)s_beta[f];
                        const bool first = (it == 0);
                        auto pv = [&](int idx) -> T {
                            const T u = rf[idx] * a.dinv[idx];
                            return first ? u : u + beta * pf[idx];
                        };
                        const T pk = pv(n.k);
                        const T qk = apply_row<DIM, T>(c, n, pv, a.coef, a.ecol, nn, a.ew);
                        p_new[(size_t)f * nn + k] = pk;
                        a.q[(size_t)f * nn + k] = qk;
                        part[f] += (double)pk * (double)qk;
                    }
                }
                alive = phase_total(part, phase);
            }
            ++phase;
            if (!alive) break;
            if (threadIdx.x == 0) {
                for (int f = 0; f < F; ++f) {
                    if (!s_inner[f]) continue;
                    const double pq = tot[f];
                    if (!(pq > 0.0) || !(s_rho[f] == s_rho[f])) {
                        // indefinite or non-finite: stop this field with its last x64
                        s_inner[f] = 0;
                        s_done[f] = 1;
                        s_flags |= P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED;
                        continue;
                    }
                    s_alpha[f] = s_rho[f] / pq;
                }
            }
            __syncthreads();
            // B: d += alpha p_new (d = alpha p_new on the first step), r -= alpha q;
            //    partials (r, u) and (r, r)
            {
                double part[2 * F];
#pragma unroll
                for (int j = 0; j < 2 * F; ++j) part[j] = 0.0;
                for (int k = k0; k < nn; k += kstride) {
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        if (!s_inner[f]) continue;
                        const T al = (T)s_alpha[f];
                        const size_t o = (size_t)f * nn + k;
                        const T dk = (it == 0) ? (T)0 : a.xout[o];
                        a.xout[o] = dk + al * p_new[o];
                        const T rn = a.r[o] - al * a.q[o];
                        a.r[o] = rn;
                        part[f] += (double)rn * (double)(rn * a.dinv[k]);
                        part[F + f] += (double)rn * (double)rn;
                    }
                }
                alive = phase_total(part, phase);
            }
            ++phase;
            if (!alive) break;
            if (threadIdx.x == 0) {
                int any = 0;
                for (int f = 0; f < F; ++f) {
                    if (!s_inner[f]) continue;
                    const double rho_new = tot[f], rr = tot[F + f];
                    s_beta[f] = rho_new / s_rho[f];
                    s_rho[f] = rho_new;
                    s_iters[f] += 1;
                    if (!(rr > s_target[f]) || s_iters[f] >= a.opts.maxit) {
                        s_inner[f] = 0;
                        continue;
                    }
                    any = 1;
                }
                s_any = any;
            }
            __syncthreads();
            T* tmp = p_old;
            p_old = p_new;
            p_new = tmp;
            if (!s_any) break;
        }
    }

    // a timed-out barrier ends the solve: the last FP64 solution is the result
    if (!alive && threadIdx.x == 0) s_flags |= P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED;
    __syncthreads();
    // result: the FP64 solution rounded to T (0 for fields with b == 0)
    for (int k = k0; k < nn; k += kstride) {
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const size_t o = (size_t)f * nn + k;
            a.xout[o] = s_zero[f] ? (T)0 : (T)a.x64[s_xb[f] * xstride + o];
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

template <typename T, int DIM>
const void* cg_kernel(int F) {
    switch (F) {
        case 1: return (const void*)k_cg<T, DIM, 1>;
        case 2: return (const void*)k_cg<T, DIM, 2>;
        case 3: return (const void*)k_cg<T, DIM, 3>;
        case 4: return (const void*)k_cg<T, DIM, 4>;
        case 5: return (const void*)k_cg<T, DIM, 5>;
        case 6: return (const void*)k_cg<T, DIM, 6>;
        case 7: return (const void*)k_cg<T, DIM, 7>;
        case 8: return (const void*)k_cg<T, DIM, 8>;
    }
    return nullptr;
}

// the sparse-row form is used by the FP64 solves only
template <typename T>
const void* cg_kernel_for(int dim, int F) {
    if (dim == 1) return cg_kernel<T, 1>(F);
    if (dim == 2) return cg_kernel<T, 2>(F);
    if constexpr (std::is_same<T, double>::value) {
        if (dim == 3) return cg_kernel<T, 3>(F);
    }
    return nullptr;
}

}  // namespace

// the partials, then the grid-barrier words
size_t cg_partials_bytes(int blocks) {
    return (size_t)2 * blocks * kSlots * sizeof(double) + kBarBytes;
}

namespace {

// Workgroups of one solve variant that are resident at once on the device: its
// occupancy per compute unit (at most 2) times the compute units.  Kept per
// device and variant after the first query.
constexpr int kMaxDevices = 16;

template <typename T>
int cg_variant_blocks(int device, int dim, int F) {
    static std::atomic<int> cache[kMaxDevices][4][kMaxFields + 1];
    const bool cached = device >= 0 && device < kMaxDevices;
    if (cached) {
        const int v = cache[device][dim][F].load(std::memory_order_relaxed);
        if (v > 0) return v;
    }
    int cus = 0, b = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    const void* fn = cg_kernel_for<T>(dim, F);
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, kCgBlock, 0) != hipSuccess)
        return 0;
    if (b > 2) b = 2;
    if (b < 1) return 0;
    if (cached) cache[device][dim][F].store(b * cus, std::memory_order_relaxed);
    return b * cus;
}

}  // namespace

// The largest grid any variant may take (workspace layouts are sized for it); a
// launch takes at most its own variant's resident grid.
template <typename T>
int cg_max_blocks(int device) {
    int most = 0;
    for (int F = 1; F <= kMaxFields; ++F) {
        for (int dim = 1; dim <= 3; ++dim) {
            if (!cg_kernel_for<T>(dim, F)) continue;
            const int v = cg_variant_blocks<T>(device, dim, F);
            if (v <= 0) return 0;
            if (v > most) most = v;
        }
    }
    return most;
}
template int cg_max_blocks<float>(int);
template int cg_max_blocks<double>(int);

template <typename T>
hipError_t launch_cg(const Mesh& m, int F, T* coef, T* b, const T* w, T* x, int start,
                     const CgWorkspace& ws, const p2m_solve_opts& opts, p2m_report* rep,
                     hipStream_t stream) {
    CgArgs<T> a;
    a.m = m;
    a.coef = coef;
    a.b = b;
    a.w = w;
    a.start = start;
    a.xout = x;
    a.x64 = ws.x64;
    a.r = (T*)ws.r;
    a.p0 = (T*)ws.p0;
    a.p1 = (T*)ws.p1;
    a.q = (T*)ws.q;
    a.partials = ws.partials;
    a.dinv = (T*)ws.dinv;
    a.spin = ws.spin;
    a.ecol = ws.ell_col;
    a.ew = ws.ell_w;
    a.opts = opts;
    a.rep = rep;
    void* args[] = {&a};
    const void* fn = cg_kernel_for<T>(m.dim, F);
    if (!fn || (m.dim == 3 && !ws.ell_col)) return hipErrorInvalidValue;
    // An ordinary launch: the stream has finished every earlier kernel, and the
    // grid (at most this variant's occupancy per compute unit) is then resident as
    // a whole.  The barrier is the kernel's own, with bounded waits; a cooperative
    // launch added tens of microseconds of queue overhead per solve.  The grid
    // never exceeds ws.blocks, which the partials were sized for.
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    const int resident = cg_variant_blocks<T>(device, m.dim, F);
    if (resident <= 0) return hipErrorInvalidValue;
    const int blocks = ws.blocks < resident ? ws.blocks : resident;
    if (blocks > 1) {
        unsigned* bar =
            (unsigned*)((char*)ws.partials + (size_t)2 * blocks * kSlots * sizeof(double));
        hipLaunchKernelGGL(k_bar_clear, dim3(1), dim3(256), 0, stream, bar);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipLaunchKernel(fn, dim3(blocks), dim3(kCgBlock), args, 0, stream);
}
template hipError_t launch_cg<float>(const Mesh&, int, float*, float*, const float*, float*, int,
                                     const CgWorkspace&, const p2m_solve_opts&, p2m_report*,
                                     hipStream_t);
template hipError_t launch_cg<double>(const Mesh&, int, double*, double*, const double*, double*,
                                      int, const CgWorkspace&, const p2m_solve_opts&, p2m_report*,
                                      hipStream_t);

}  // namespace p2m
