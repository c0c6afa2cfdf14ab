// The paper-exact 1D assignments (Table 1; Sec. 2.4 eq. (20); Appendix B), FP64.
//
// In 1D the particle "triangulation" of Sec. 2 is the order of the particles
// along the periodic segment, and the particle hat psi_mu is the P1 hat on the
// sorted particles (Sec. 3.1).  Every integral is the exact integral of that
// particle interpolant or of the mesh interpolant against the hats, either
// exactly (both factors are linear between merged breakpoints, so Simpson's
// rule on each piece is exact) or with the Appendix-B rule (on every gap of the
// target hats, the parabola through the source interpolant at both ends and the
// midpoint, integrated exactly against the two hats of the gap).
//
// The kernels, in call order:
//   k_x1d_keys     wrapped position of every binned particle (sort key)
//   k_x1d_sort     per cell, (position, particle number) order: cells of up to
//                  32 particles by their own thread, larger ones by the whole
//                  workgroup with the merge network of the binning sort
//   k_x1d_setup    gaps g_k, volumes v_k = (g_{k-1} + g_k) / 2 (eq. (4)) and the
//                  values in sorted order
//   k_x1d_eval_p   the particle interpolant at every node and element midpoint
//   k_x1d_c_appb / k_x1d_c_exact + k_x1d_c_sum
//                  c_j = int A psi_j (mesh hats)                 (P2M)
//   k_x1d_eval_m / k_x1d_cp_appb / k_x1d_cp_exact + k_x1d_c_sum
//                  c'_mu = int Abar psi_mu (particle hats)       (M2P)
//   k_x1d_mass_mesh / k_x1d_mass_part
//                  the stencils of the consistent mass matrices: mesh 2h/3, h/6;
//                  particles (g_{k-1} + g_k)/3, g_k/6 (cyclic tridiagonal)
//   k_x1d_div / k_x1d_scatter
//                  lumped divisions and the result in caller order
// The mass solves themselves run in the streaming CG kernel (k_cg.hip) on these
// stencils.
#include "p2m_internal.hpp"

namespace p2m {

namespace {

constexpr int kB = 256;
constexpr int kSortSmall = 32;

inline int grid_of(size_t n) { return (int)((n + kB - 1) / kB); }

// position wrapped into [0, L): valid inputs satisfy 0 <= x < L + h
__device__ __forceinline__ double wrap_pos(double x, double L) { return x < L ? x : x - L; }

__device__ __forceinline__ bool pair_less(double ka, int ia, double kb, int ib) {
    return ka < kb || (ka == kb && ia < ib);
}

__global__ void k_x1d_keys(int N, const double* __restrict__ x, const int32_t* __restrict__ perm,
                           double L, double* __restrict__ key, int32_t* __restrict__ idx) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= N) return;
    const int p = perm[k];
    key[k] = wrap_pos(x[p], L);
    idx[k] = p;
}

// Sort of one segment of (key, idx) pairs by the whole workgroup: the bitonic
// network whose comparators all put the smaller pair at the lower index (each
// merge first compares i with its mirror, then half-cleans), with comparators
// beyond the segment skipped (virtual +infinity padding never moves).
__device__ void block_sort_pairs(double* key, int32_t* idx, int n) {
    int P = 1;
    while (P < n) P <<= 1;
    for (int k = 2; k <= P; k <<= 1) {
        const int half = k >> 1;
        for (int q = threadIdx.x; q < P / 2; q += kB) {
            const int blk = q / half, off = q - blk * half;
            const int i = blk * k + off, j = blk * k + k - 1 - off;
            if (j < n && pair_less(key[j], idx[j], key[i], idx[i])) {
                const double tk = key[i];
                const int ti = idx[i];
                key[i] = key[j];
                idx[i] = idx[j];
                key[j] = tk;
                idx[j] = ti;
            }
        }
        __syncthreads();
        for (int d = k >> 2; d >= 1; d >>= 1) {
            for (int q = threadIdx.x; q < P / 2; q += kB) {
                const int blk = q / d;
                const int i = blk * 2 * d + (q - blk * d), j = i + d;
                if (j < n && pair_less(key[j], idx[j], key[i], idx[i])) {
                    const double tk = key[i];
                    const int ti = idx[i];
                    key[i] = key[j];
                    idx[i] = idx[j];
                    key[j] = tk;
                    idx[j] = ti;
                }
            }
            __syncthreads();
        }
    }
}

// Every cell's (key, idx) pairs in ascending (key, idx) order, in place.
__global__ __launch_bounds__(kB) void k_x1d_sort(int ncells, const int32_t* __restrict__ cs,
                                                 double* __restrict__ key,
                                                 int32_t* __restrict__ idx) {
    __shared__ int big[kB];
    __shared__ int n_big;
    const int c0 = blockIdx.x * kB;
    const int c = c0 + (int)threadIdx.x;
    if (threadIdx.x == 0) n_big = 0;
    __syncthreads();
    int s = 0, n = 0;
    if (c < ncells) {
        s = cs[c];
        n = cs[c + 1] - s;
    }
    if (n > kSortSmall) {
        big[atomicAdd(&n_big, 1)] = c;   // any order: cells are independent
    } else if (n > 1) {
        // insertion sort of at most kSortSmall pairs
        for (int i = s + 1; i < s + n; ++i) {
            const double kv = key[i];
            const int iv = idx[i];
            int j = i - 1;
            while (j >= s && pair_less(kv, iv, key[j], idx[j])) {
                key[j + 1] = key[j];
                idx[j + 1] = idx[j];
                --j;
            }
            key[j + 1] = kv;
            idx[j + 1] = iv;
        }
    }
    __syncthreads();
    const int nb = n_big;
    for (int k = 0; k < nb; ++k) {
        const int cc = big[k];
        const int bs = cs[cc];
        block_sort_pairs(key + bs, idx + bs, cs[cc + 1] - bs);
    }
}

// gaps, volumes (eq. (4)) and values in sorted order; volumes also in caller order
__global__ void k_x1d_setup(int N, double L, const double* __restrict__ key,
                            const int32_t* __restrict__ idx, const double* __restrict__ values,
                            int F, int np, double* __restrict__ gap, double* __restrict__ vol_s,
                            double* __restrict__ vol_c, double* __restrict__ As) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= N) return;
    const double xk = key[k];
    const double g = (k + 1 < N) ? key[k + 1] - xk : (key[0] + L) - xk;
    const double gm = (k > 0) ? xk - key[k - 1] : (key[0] + L) - key[N - 1];
    gap[k] = g;
    const double v = 0.5 * (g + gm);
    vol_s[k] = v;
    const int p = idx[k];
    vol_c[p] = v;
    for (int f = 0; f < F; ++f) As[(size_t)f * N + k] = values[(size_t)f * np + p];
}

// the periodic piecewise-linear interpolant through (key[k], A[k]) at y in [0, L)
__device__ __forceinline__ double interp_sorted(const double* __restrict__ key,
                                                const double* __restrict__ A, int N, double L,
                                                double y) {
    // a: the last knot with key <= y (none: the last knot, one period back)
    int lo = 0, hi = N;   // first index with key > y
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key[mid] <= y) lo = mid + 1;
        else hi = mid;
    }
    const int a = lo - 1;
    double xa, xb, fa, fb;
    if (a < 0) {
        xa = key[N - 1] - L;
        fa = A[N - 1];
        xb = key[0];
        fb = A[0];
    } else {
        xa = key[a];
        fa = A[a];
        if (a + 1 < N) {
            xb = key[a + 1];
            fb = A[a + 1];
        } else {
            xb = key[0] + L;
            fb = A[0];
        }
    }
    const double slope = (fb - fa) / (xb - xa);
    return slope * (y - xa) + fa;
}

// node j at j h (h = L / n), its gap to the next node (the last one ends at L)
__device__ __forceinline__ double node_x(int j, double h) { return (double)j * h; }
__device__ __forceinline__ double node_gap(int j, int n, double h, double L) {
    return (j + 1 < n ? node_x(j + 1, h) : L) - node_x(j, h);
}

// particle interpolant at node j and at the midpoint of element j, every field
__global__ void k_x1d_eval_p(int n, double h, double L, int N, const double* __restrict__ key,
                             const double* __restrict__ As, int F, double* __restrict__ fn,
                             double* __restrict__ fm) {
    const int j = blockIdx.x * kB + threadIdx.x;
    if (j >= n) return;
    const double xj = node_x(j, h);
    const double mj = xj + 0.5 * node_gap(j, n, h, L);
    for (int f = 0; f < F; ++f) {
        const double* A = As + (size_t)f * N;
        fn[(size_t)f * n + j] = N > 0 ? interp_sorted(key, A, N, L, xj) : 0.0;
        fm[(size_t)f * n + j] = N > 0 ? interp_sorted(key, A, N, L, wrap_pos(mj, L)) : 0.0;
    }
}

// Appendix-B rule on the mesh hats: c_j = g_j/6 (f(x_j) + 2 f(m_j)) + g_{j-1}/6 (f(x_j) + 2 f(m_{j-1}))
__global__ void k_x1d_c_appb(int n, double h, double L, int F, const double* __restrict__ fn,
                             const double* __restrict__ fm, double* __restrict__ c) {
    const int j = blockIdx.x * kB + threadIdx.x;
    if (j >= n) return;
    const int jm = j > 0 ? j - 1 : n - 1;
    const double g = node_gap(j, n, h, L), gm = node_gap(jm, n, h, L);
    for (int f = 0; f < F; ++f) {
        const double fj = fn[(size_t)f * n + j];
        const double own = g / 6.0 * (fj + 2.0 * fm[(size_t)f * n + j]);
        const double prev = gm / 6.0 * (fj + 2.0 * fm[(size_t)f * n + jm]);
        c[(size_t)f * n + j] = own + prev;
    }
}

// Simpson on one piece [a, b] with f linear on it (fm its mean) against the two
// hats of the gap [left, right] that contains the piece
__device__ __forceinline__ void piece(double a, double b, double fa, double fb, double left,
                                      double right, double& to_left, double& to_right) {
    const double span = right - left;
    const double m = 0.5 * (a + b);
    const double fm = 0.5 * (fa + fb);
    const double la = (right - a) / span, lm = (right - m) / span, lb = (right - b) / span;
    const double h6 = (b - a) / 6.0;
    to_left += h6 * (fa * la + 4.0 * fm * lm + fb * lb);
    to_right += h6 * (fa * (1.0 - la) + 4.0 * fm * (1.0 - lm) + fb * (1.0 - lb));
}

// first index with key > y / with key >= y
__device__ __forceinline__ int upper_idx(const double* __restrict__ key, int N, double y) {
    int lo = 0, hi = N;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key[mid] <= y) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int lower_idx(const double* __restrict__ key, int N, double y) {
    int lo = 0, hi = N;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key[mid] < y) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Exact overlaps with the mesh hats, element by element: element j is cut by the
// particles strictly inside it; er[j] goes to node j, el[j] to node j + 1.
__global__ void k_x1d_c_exact(int n, double h, double L, int N, const double* __restrict__ key,
                              const double* __restrict__ As, int F, const double* __restrict__ fn,
                              double* __restrict__ to_lo, double* __restrict__ to_hi) {
    const int j = blockIdx.x * kB + threadIdx.x;
    if (j >= n) return;
    const double left = node_x(j, h);
    const double right = j + 1 < n ? node_x(j + 1, h) : L;
    const int k0 = upper_idx(key, N, left), k1 = lower_idx(key, N, right);
    for (int f = 0; f < F; ++f) {
        const double* A = As + (size_t)f * N;
        double lo = 0.0, hi = 0.0;
        double a = left, fa = fn[(size_t)f * n + j];
        for (int k = k0; k < k1; ++k) {
            piece(a, key[k], fa, A[k], left, right, lo, hi);
            a = key[k];
            fa = A[k];
        }
        piece(a, right, fa, fn[(size_t)f * n + (j + 1 < n ? j + 1 : 0)], left, right, lo, hi);
        to_lo[(size_t)f * n + j] = lo;
        to_hi[(size_t)f * n + j] = hi;
    }
}

// c_k = to_lo[k] + to_hi[k - 1] (periodic)
__global__ void k_x1d_c_sum(int K, int F, const double* __restrict__ to_lo,
                            const double* __restrict__ to_hi, double* __restrict__ c) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= K) return;
    const int km = k > 0 ? k - 1 : K - 1;
    for (int f = 0; f < F; ++f) c[(size_t)f * K + k] = to_lo[(size_t)f * K + k] + to_hi[(size_t)f * K + km];
}

// the mesh interpolant of nodal values Ab at y in [0, L)
__device__ __forceinline__ double interp_mesh(const double* __restrict__ Ab, int n, double h,
                                              double inv_h, double L, double y) {
    int j = (int)floor(y * inv_h);
    if (j < 0) j = 0;
    if (j > n - 1) j = n - 1;
    while (j > 0 && node_x(j, h) > y) --j;
    while (j + 1 < n && node_x(j + 1, h) <= y) ++j;
    const double xa = node_x(j, h), xb = j + 1 < n ? node_x(j + 1, h) : L;
    const double fa = Ab[j], fb = Ab[j + 1 < n ? j + 1 : 0];
    const double slope = (fb - fa) / (xb - xa);
    return slope * (y - xa) + fa;
}

// mesh interpolant at every sorted particle and at the midpoint of its gap
__global__ void k_x1d_eval_m(int N, int n, double h, double inv_h, double L,
                             const double* __restrict__ key, const double* __restrict__ gap,
                             const double* __restrict__ Ab, int F, double* __restrict__ fk,
                             double* __restrict__ fmid) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= N) return;
    const double xk = key[k];
    const double mk = wrap_pos(xk + 0.5 * gap[k], L);
    for (int f = 0; f < F; ++f) {
        const double* A = Ab + (size_t)f * n;
        fk[(size_t)f * N + k] = interp_mesh(A, n, h, inv_h, L, xk);
        fmid[(size_t)f * N + k] = interp_mesh(A, n, h, inv_h, L, mk);
    }
}

// Appendix-B rule on the particle hats
__global__ void k_x1d_cp_appb(int N, int F, const double* __restrict__ gap,
                              const double* __restrict__ fk, const double* __restrict__ fmid,
                              double* __restrict__ c) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= N) return;
    const int km = k > 0 ? k - 1 : N - 1;
    for (int f = 0; f < F; ++f) {
        const double fv = fk[(size_t)f * N + k];
        const double own = gap[k] / 6.0 * (fv + 2.0 * fmid[(size_t)f * N + k]);
        const double prev = gap[km] / 6.0 * (fv + 2.0 * fmid[(size_t)f * N + km]);
        c[(size_t)f * N + k] = own + prev;
    }
}

// Exact overlaps with the particle hats, gap by gap: gap k = [x_k, x_{k+1}] is cut
// by the nodes strictly inside it (the last gap runs past L to x_0 + L)
__global__ void k_x1d_cp_exact(int N, int n, double h, double inv_h, double L,
                               const double* __restrict__ key, const double* __restrict__ gap,
                               const double* __restrict__ Ab, const double* __restrict__ fk, int F,
                               double* __restrict__ to_lo, double* __restrict__ to_hi) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= N) return;
    const double left = key[k];
    const double right = k + 1 < N ? key[k + 1] : key[0] + L;
    // node jj of the periodic continuation: node jj mod n, shifted by whole periods
    auto nodepos = [&](int jj) { return node_x(jj % n, h) + (double)(jj / n) * L; };
    // the first node strictly right of `left`
    int j = (int)floor(left * inv_h);
    if (j < 0) j = 0;
    while (j > 0 && nodepos(j) > left) --j;
    while (nodepos(j) <= left) ++j;
    const int kn = k + 1 < N ? k + 1 : 0;
    for (int f = 0; f < F; ++f) {
        const double* A = Ab + (size_t)f * n;
        double lo = 0.0, hi = 0.0;
        double a = left, fa = fk[(size_t)f * N + k];
        for (int jj = j;; ++jj) {
            const int jw = jj % n;
            const double xn = nodepos(jj);
            if (!(xn < right)) break;
            piece(a, xn, fa, A[jw], left, right, lo, hi);
            a = xn;
            fa = A[jw];
        }
        piece(a, right, fa, fk[(size_t)f * N + kn], left, right, lo, hi);
        to_lo[(size_t)f * N + k] = lo;
        to_hi[(size_t)f * N + k] = hi;
    }
}

// consistent mesh mass matrix of 1D P1 hats: 2h/3 on the diagonal, h/6 beside it;
// w = h (no orphans); b = c
__global__ void k_x1d_mass_mesh(int n, double L, double* __restrict__ coef, double* __restrict__ w) {
    const int j = blockIdx.x * kB + threadIdx.x;
    if (j >= n) return;
    const double h = L / (double)n;
    coef[j] = 2.0 * h / 3.0;
    coef[(size_t)n + j] = h / 6.0;
    w[j] = h;
}

// consistent particle mass matrix on the sorted particles: (g_{k-1} + g_k)/3 and g_k/6
__global__ void k_x1d_mass_part(int N, const double* __restrict__ gap, double* __restrict__ coef) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= N) return;
    const int km = k > 0 ? k - 1 : N - 1;
    coef[k] = gap[km] / 3.0 + gap[k] / 3.0;
    coef[(size_t)N + k] = gap[k] / 6.0;
}

// out[f][k] = c[f][k] / d[k] (d == nullptr: / s)
__global__ void k_x1d_div(int K, int F, const double* __restrict__ c, const double* __restrict__ d,
                          double s, double* __restrict__ out) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= K) return;
    const double den = d ? d[k] : s;
    for (int f = 0; f < F; ++f) out[(size_t)f * K + k] = c[(size_t)f * K + k] / den;
}

// sorted-order values to caller order; particles left out of the binning get NaN
__global__ void k_x1d_fill_nan(size_t n, double* __restrict__ out) {
    const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) out[i] = __builtin_nan("");
}
__global__ void k_x1d_scatter(int N, int F, int np, const int32_t* __restrict__ idx,
                              const double* __restrict__ xs, double* __restrict__ out) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= N) return;
    const int p = idx[k];
    for (int f = 0; f < F; ++f) out[(size_t)f * np + p] = xs[(size_t)f * N + k];
}

}  // namespace

#define X1D_TRY(e)                                 \
    do {                                           \
        hipError_t e_ = (e);                       \
        if (e_ != hipSuccess) return e_;           \
    } while (0)

hipError_t x1d_sort(const Mesh& m, int N, const double* x, const int32_t* perm,
                    const int32_t* cs, double* key, int32_t* idx, hipStream_t stream) {
    if (N == 0) return hipSuccess;
    const double L = m.cell_measure * m.nx;
    hipLaunchKernelGGL(k_x1d_keys, dim3(grid_of(N)), dim3(kB), 0, stream, N, x, perm, L, key, idx);
    X1D_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_x1d_sort, dim3(grid_of(m.nx)), dim3(kB), 0, stream, m.nx, cs, key, idx);
    return hipGetLastError();
}

hipError_t x1d_setup(int N, double L, const double* key, const int32_t* idx, const double* values,
                     int F, int np, double* gap, double* vol_s, double* vol_c, double* As,
                     hipStream_t stream) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_x1d_setup, dim3(grid_of(N)), dim3(kB), 0, stream, N, L, key, idx, values,
                       F, np, gap, vol_s, vol_c, As);
    return hipGetLastError();
}

hipError_t x1d_p2m_overlap(const Mesh& m, int N, const double* key, const double* As, int F,
                           int quad, double* fn, double* fm, double* t_lo, double* t_hi,
                           double* c, hipStream_t stream) {
    const int n = m.nx;
    const double h = m.cell_measure, L = h * n;
    hipLaunchKernelGGL(k_x1d_eval_p, dim3(grid_of(n)), dim3(kB), 0, stream, n, h, L, N, key, As, F,
                       fn, fm);
    X1D_TRY(hipGetLastError());
    if (quad == P2M_QUAD_APPB) {
        hipLaunchKernelGGL(k_x1d_c_appb, dim3(grid_of(n)), dim3(kB), 0, stream, n, h, L, F, fn, fm,
                           c);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_x1d_c_exact, dim3(grid_of(n)), dim3(kB), 0, stream, n, h, L, N, key, As, F,
                       fn, t_lo, t_hi);
    X1D_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_x1d_c_sum, dim3(grid_of(n)), dim3(kB), 0, stream, n, F, t_lo, t_hi, c);
    return hipGetLastError();
}

hipError_t x1d_m2p_overlap(const Mesh& m, int N, const double* key, const double* gap,
                           const double* nodal, int F, int quad, double* fk, double* fmid,
                           double* t_lo, double* t_hi, double* c, hipStream_t stream) {
    if (N == 0) return hipSuccess;
    const int n = m.nx;
    const double h = m.cell_measure, L = h * n;
    hipLaunchKernelGGL(k_x1d_eval_m, dim3(grid_of(N)), dim3(kB), 0, stream, N, n, h, m.inv_hx, L, key,
                       gap, nodal, F, fk, fmid);
    X1D_TRY(hipGetLastError());
    if (quad == P2M_QUAD_APPB) {
        hipLaunchKernelGGL(k_x1d_cp_appb, dim3(grid_of(N)), dim3(kB), 0, stream, N, F, gap, fk, fmid,
                           c);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_x1d_cp_exact, dim3(grid_of(N)), dim3(kB), 0, stream, N, n, h, m.inv_hx, L,
                       key, gap, nodal, fk, F, t_lo, t_hi);
    X1D_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_x1d_c_sum, dim3(grid_of(N)), dim3(kB), 0, stream, N, F, t_lo, t_hi, c);
    return hipGetLastError();
}

hipError_t x1d_mass_mesh(int n, double L, double* coef, double* w, hipStream_t stream) {
    hipLaunchKernelGGL(k_x1d_mass_mesh, dim3(grid_of(n)), dim3(kB), 0, stream, n, L, coef, w);
    return hipGetLastError();
}

hipError_t x1d_mass_part(int N, const double* gap, double* coef, hipStream_t stream) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_x1d_mass_part, dim3(grid_of(N)), dim3(kB), 0, stream, N, gap, coef);
    return hipGetLastError();
}

hipError_t x1d_div(int K, int F, const double* c, const double* d, double s, double* out,
                   hipStream_t stream) {
    if (K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_x1d_div, dim3(grid_of(K)), dim3(kB), 0, stream, K, F, c, d, s, out);
    return hipGetLastError();
}

hipError_t x1d_scatter(int N, int F, int np, const int32_t* idx, const double* xs, double* out,
                       hipStream_t stream) {
    if (np > 0) {
        const size_t tot = (size_t)F * np;
        hipLaunchKernelGGL(k_x1d_fill_nan, dim3(grid_of(tot)), dim3(kB), 0, stream, tot, out);
        X1D_TRY(hipGetLastError());
    }
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_x1d_scatter, dim3(grid_of(N)), dim3(kB), 0, stream, N, F, np, idx, xs, out);
    return hipGetLastError();
}

}  // namespace p2m
