// Mesh->particle interpolation and the 1D delta particle->mesh assignment.
//
// gather  : Abarbar_mu = sum_i Abar_i psi_i(r_mu) (Sec. 2.2 eq. (10), read at r_mu).
//           One thread per particle in the caller's order: positions and outputs
//           are read and written coalesced; the 2 or 3 nodal values per field
//           come from the L2/MALL-resident nodal arrays.
// delta1d : Abar_i = sum_mu A_mu psi_mu(x_i) (Sec. 2.2 eq. (9)) with 1D particle
//           hats on the particles sorted along the periodic axis: the linear
//           interpolation between the two consecutive particles that bracket
//           node i.  Positions are compared in the cell coordinate s = c + xi of
//           the locate step and particles are ordered by (s, original index).
#include "p2m_internal.hpp"

namespace p2m {

namespace {

constexpr int kGatherGroup = 4;

__device__ __forceinline__ void flag_invalid(p2m_report* rep, bool finite) {
    if (rep) atomicOr(&rep->flags, finite ? (uint32_t)P2M_FLAG_RANGE : (uint32_t)P2M_FLAG_NONFINITE);
}

// kGatherItems particles per thread (item u of block b: particles
// [(b * kGatherItems + u) * blockDim, ...), coalesced per item): every position
// is loaded, then every nodal value, then the outputs are stored, so a thread
// waits for two memory round trips in all.
constexpr int kGatherItems = 4;

template <typename T>
__global__ void k_gather2d(Mesh m, Particles<T> P, const T* __restrict__ nodal, int F,
                           T* __restrict__ out, p2m_report* __restrict__ rep) {
    const int base = blockIdx.x * blockDim.x * kGatherItems + threadIdx.x;
    T px[kGatherItems], py[kGatherItems];
#pragma unroll
    for (int u = 0; u < kGatherItems; ++u) {
        const int i = base + u * (int)blockDim.x;
        px[u] = py[u] = (T)0;
        if (i < m.np) {
            px[u] = P.x[i];
            py[u] = P.y[i];
        }
    }
    int n0[kGatherItems], n1[kGatherItems], n2[kGatherItems];
    T l0[kGatherItems], l1[kGatherItems], l2[kGatherItems];
    bool ok[kGatherItems];
#pragma unroll
    for (int u = 0; u < kGatherItems; ++u) {
        const int i = base + u * (int)blockDim.x;
        int cx = 0, cy = 0;
        double xi = 0.0, eta = 0.0;
        bool fx = true, fy = true;
        ok[u] = false;
        if (i < m.np) {
            ok[u] = locate_axis((double)px[u], m.nx, m.inv_hx, cx, xi, fx);
            ok[u] = locate_axis((double)py[u], m.ny, m.inv_hy, cy, eta, fy) && ok[u];
            if (!ok[u]) flag_invalid(rep, fx && fy);
        }
        if (!ok[u]) cx = cy = 0, xi = eta = 0.0;
        const int i1 = (cx + 1 == m.nx) ? 0 : cx + 1;
        const int j1 = (cy + 1 == m.ny) ? 0 : cy + 1;
        const bool lower = xi >= eta;
        n0[u] = cx + m.nx * cy;
        n1[u] = lower ? i1 + m.nx * cy : i1 + m.nx * j1;
        n2[u] = lower ? i1 + m.nx * j1 : cx + m.nx * j1;
        T c00, c10, c11, c01;
        corner_weights<T>(xi, eta, c00, c10, c11, c01);
        l0[u] = c00;
        l1[u] = lower ? c10 : c11;
        l2[u] = lower ? c11 : c01;
    }
    for (int f = 0; f < F; ++f) {
        const T* a = nodal + (size_t)f * m.nn;
        T v[kGatherItems][3];
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            v[u][0] = a[n0[u]];
            v[u][1] = a[n1[u]];
            v[u][2] = a[n2[u]];
        }
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            const int i = base + u * (int)blockDim.x;
            if (i < m.np)
                out[(size_t)f * m.np + i] =
                    ok[u] ? l0[u] * v[u][0] + l1[u] * v[u][1] + l2[u] * v[u][2] : (T)NAN;
        }
    }
}

template <typename T>
__global__ void k_gather1d(Mesh m, Particles<T> P, const T* __restrict__ nodal, int F,
                           T* __restrict__ out, p2m_report* __restrict__ rep) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.np) return;
    int cx;
    double xi;
    bool fx;
    bool ok = locate_axis((double)P.x[i], m.nx, m.inv_hx, cx, xi, fx);
    if (!ok) {
        for (int f = 0; f < F; ++f) out[(size_t)f * m.np + i] = (T)NAN;
        flag_invalid(rep, fx);
        return;
    }
    const int n1 = (cx + 1 == m.nx) ? 0 : cx + 1;
    const T l0 = (T)__dsub_rn(1.0, xi), l1 = (T)xi;
    for (int f0 = 0; f0 < F; f0 += kGatherGroup) {
        T v[kGatherGroup][2];
#pragma unroll
        for (int g = 0; g < kGatherGroup; ++g) {
            if (f0 + g >= F) break;
            const T* a = nodal + (size_t)(f0 + g) * m.nn;
            v[g][0] = a[cx];
            v[g][1] = a[n1];
        }
#pragma unroll
        for (int g = 0; g < kGatherGroup; ++g) {
            if (f0 + g >= F) break;
            out[(size_t)(f0 + g) * m.np + i] = l0 * v[g][0] + l1 * v[g][1];
        }
    }
}

// offset of particle p inside its cell
template <typename T>
__device__ __forceinline__ double cell_offset(const Mesh& m, const T* x, int p) {
    int c;
    double xi;
    bool fin;
    locate_axis((double)x[p], m.nx, m.inv_hx, c, xi, fin);
    return xi;
}

// (xi, idx) lexicographic comparisons
__device__ __forceinline__ bool lex_less(double xa, int ia, double xb, int ib) {
    return xa < xb || (xa == xb && ia < ib);
}

template <typename T>
__global__ void k_delta1d(Mesh m, Particles<T> P, const T* __restrict__ values, int F,
                          const int32_t* __restrict__ perm, const int32_t* __restrict__ cs,
                          T* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.nx) return;
    const int n = m.nx;
    const int total = cs[n];
    if (total == 0) {
        for (int f = 0; f < F; ++f) out[(size_t)f * m.nn + i] = (T)0;
        return;
    }
    // particle a: last in (s, idx) order with s <= i
    int a = -1, ca = -1;
    double xa = 0.0;
    // b: the particle after a
    int b = -1, cb = -1;
    double xb = 0.0;
    {
        // inside cell i: the particles sitting exactly on node i (xi == 0) and the
        // first particle strictly inside the cell
        int z = -1;
        int f_in = -1;
        double x_in = 0.0;
        for (int k = cs[i]; k < cs[i + 1]; ++k) {
            const int p = perm[k];
            const double xi = cell_offset(m, P.x, p);
            if (xi == 0.0) {
                if (p > z) z = p;
            } else if (f_in < 0 || lex_less(xi, p, x_in, f_in)) {
                f_in = p;
                x_in = xi;
            }
        }
        if (z >= 0) {
            a = z; ca = i; xa = 0.0;
            if (f_in >= 0) { b = f_in; cb = i; xb = x_in; }
        } else {
            // nearest non-empty cell to the left (cyclic; may come back to cell i)
            for (int step = 1; step <= n; ++step) {
                const int c = (i - step + n) % n;
                if (cs[c + 1] > cs[c]) {
                    for (int k = cs[c]; k < cs[c + 1]; ++k) {
                        const int p = perm[k];
                        const double xi = cell_offset(m, P.x, p);
                        if (a < 0 || lex_less(xa, a, xi, p)) { a = p; xa = xi; }
                    }
                    ca = c;
                    break;
                }
            }
            if (f_in >= 0) { b = f_in; cb = i; xb = x_in; }
        }
        if (b < 0) {
            // the first particle of the nearest non-empty cell to the right (cyclic)
            for (int step = 1; step <= n; ++step) {
                const int c = (i + step) % n;
                if (cs[c + 1] > cs[c]) {
                    for (int k = cs[c]; k < cs[c + 1]; ++k) {
                        const int p = perm[k];
                        const double xi = cell_offset(m, P.x, p);
                        if (b < 0 || lex_less(xi, p, xb, b)) { b = p; xb = xi; }
                    }
                    cb = c;
                    break;
                }
            }
        }
    }
    const double dn = (double)n;
    const double sa = (double)ca + xa;
    const double sb = (double)cb + xb;
    double da = (double)i - sa;
    if (da < 0.0) da += dn;
    double db;
    if (b == a) {
        db = dn - da;
    } else {
        db = sb - (double)i;
        if (db < 0.0) db += dn;
        if (db == 0.0) db = dn;
    }
    const double frac = da / (da + db);
    for (int f = 0; f < F; ++f) {
        const double va = (double)values[(size_t)f * m.np + a];
        const double vb = (double)values[(size_t)f * m.np + b];
        out[(size_t)f * m.nn + i] = (T)(va + (vb - va) * frac);
    }
}

}  // namespace

template <typename T>
hipError_t launch_gather(const Mesh& m, Particles<T> P, const T* nodal, int F, T* out,
                         p2m_report* rep, hipStream_t stream) {
    if (m.np == 0) return hipSuccess;
    const int block = 256;
    if (m.dim == 2) {
        const int grid = (int)(((size_t)m.np + (size_t)block * kGatherItems - 1) /
                               ((size_t)block * kGatherItems));
        hipLaunchKernelGGL(k_gather2d<T>, dim3(grid), dim3(block), 0, stream, m, P, nodal, F, out, rep);
    } else {
        const int grid = (m.np + block - 1) / block;
        hipLaunchKernelGGL(k_gather1d<T>, dim3(grid), dim3(block), 0, stream, m, P, nodal, F, out, rep);
    }
    return hipGetLastError();
}
template hipError_t launch_gather<float>(const Mesh&, Particles<float>, const float*, int, float*,
                                         p2m_report*, hipStream_t);
template hipError_t launch_gather<double>(const Mesh&, Particles<double>, const double*, int,
                                          double*, p2m_report*, hipStream_t);

template <typename T>
hipError_t launch_delta1d(const Mesh& m, Particles<T> P, const T* values, int F,
                          const int32_t* perm, const int32_t* cell_start, T* out,
                          hipStream_t stream) {
    const int block = 256;
    const int grid = (m.nx + block - 1) / block;
    hipLaunchKernelGGL(k_delta1d<T>, dim3(grid), dim3(block), 0, stream, m, P, values, F, perm,
                       cell_start, out);
    return hipGetLastError();
}
template hipError_t launch_delta1d<float>(const Mesh&, Particles<float>, const float*, int,
                                          const int32_t*, const int32_t*, float*, hipStream_t);
template hipError_t launch_delta1d<double>(const Mesh&, Particles<double>, const double*, int,
                                           const int32_t*, const int32_t*, double*, hipStream_t);

}  // namespace p2m
