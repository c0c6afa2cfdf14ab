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

// Cell corners and P1 weights of particle i's triangle (the "/" split); ok is
// false for a particle that cannot be located (flagged, NaN output).
template <typename T>
struct GatherGeom {
    int n0, n1, n2;
    T l0, l1, l2;
    bool ok;
};

template <typename T>
__device__ __forceinline__ GatherGeom<T> gather_geom(const Mesh& m, T px, T py, bool in,
                                                     p2m_report* rep) {
    GatherGeom<T> g;
    int cx = 0, cy = 0;
    double xi = 0.0, eta = 0.0;
    bool fx = true, fy = true;
    g.ok = false;
    if (in) {
        g.ok = locate_axis((double)px, m.nx, m.inv_hx, cx, xi, fx);
        g.ok = locate_axis((double)py, m.ny, m.inv_hy, cy, eta, fy) && g.ok;
        if (!g.ok) flag_invalid(rep, fx && fy);
    }
    if (!g.ok) cx = cy = 0, xi = eta = 0.0;
    const int i1 = (cx + 1 == m.nx) ? 0 : cx + 1;
    const int j1 = (cy + 1 == m.ny) ? 0 : cy + 1;
    const bool lower = xi >= eta;
    g.n0 = cx + m.nx * cy;
    g.n1 = lower ? i1 + m.nx * cy : i1 + m.nx * j1;
    g.n2 = lower ? i1 + m.nx * j1 : cx + m.nx * j1;
    T c00, c10, c11, c01;
    corner_weights<T>(xi, eta, c00, c10, c11, c01);
    g.l0 = c00;
    g.l1 = lower ? c10 : c11;
    g.l2 = lower ? c11 : c01;
    return g;
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
    GatherGeom<T> g[kGatherItems];
#pragma unroll
    for (int u = 0; u < kGatherItems; ++u)
        g[u] = gather_geom<T>(m, px[u], py[u], base + u * (int)blockDim.x < m.np, rep);
    for (int f = 0; f < F; ++f) {
        const T* a = nodal + (size_t)f * m.nn;
        T v[kGatherItems][3];
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            v[u][0] = a[g[u].n0];
            v[u][1] = a[g[u].n1];
            v[u][2] = a[g[u].n2];
        }
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            const int i = base + u * (int)blockDim.x;
            if (i < m.np)
                out[(size_t)f * m.np + i] =
                    g[u].ok ? g[u].l0 * v[u][0] + g[u].l1 * v[u][1] + g[u].l2 * v[u][2] : (T)NAN;
        }
    }
}

// The same from a node-major copy nm[k * F + f] of the nodal values: one load of
// F consecutive values per corner instead of F loads.
template <typename T, int F>
__global__ void k_gather2d_nm(Mesh m, Particles<T> P, const T* __restrict__ nm,
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
    GatherGeom<T> g[kGatherItems];
#pragma unroll
    for (int u = 0; u < kGatherItems; ++u)
        g[u] = gather_geom<T>(m, px[u], py[u], base + u * (int)blockDim.x < m.np, rep);
    T v[kGatherItems][3][F];
#pragma unroll
    for (int u = 0; u < kGatherItems; ++u)
#pragma unroll
        for (int f = 0; f < F; ++f) {
            v[u][0][f] = nm[(size_t)g[u].n0 * F + f];
            v[u][1][f] = nm[(size_t)g[u].n1 * F + f];
            v[u][2][f] = nm[(size_t)g[u].n2 * F + f];
        }
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            const int i = base + u * (int)blockDim.x;
            if (i < m.np)
                out[(size_t)f * m.np + i] =
                    g[u].ok ? g[u].l0 * v[u][0][f] + g[u].l1 * v[u][1][f] + g[u].l2 * v[u][2][f]
                            : (T)NAN;
        }
}

// nm[k * F + f] = nodal[f * nn + k]
template <typename T>
__global__ void k_node_major(const T* __restrict__ nodal, int F, int nn, T* __restrict__ nm) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    for (int f = 0; f < F; ++f) nm[(size_t)k * F + f] = nodal[(size_t)f * nn + k];
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
                         p2m_report* rep, hipStream_t stream, void* ws, size_t ws_bytes) {
    if (m.np == 0) return hipSuccess;
    const int block = 256;
    if (m.dim == 2) {
        const int grid = (int)(((size_t)m.np + (size_t)block * kGatherItems - 1) /
                               ((size_t)block * kGatherItems));
        if (ws && F >= 2 && F <= 4 && ws_bytes >= (size_t)F * m.nn * sizeof(T)) {
            T* nm = (T*)ws;
            hipLaunchKernelGGL(k_node_major<T>, dim3((m.nn + block - 1) / block), dim3(block), 0,
                               stream, nodal, F, m.nn, nm);
            switch (F) {
                case 2:
                    hipLaunchKernelGGL((k_gather2d_nm<T, 2>), dim3(grid), dim3(block), 0, stream, m,
                                       P, nm, out, rep);
                    break;
                case 3:
                    hipLaunchKernelGGL((k_gather2d_nm<T, 3>), dim3(grid), dim3(block), 0, stream, m,
                                       P, nm, out, rep);
                    break;
                default:
                    hipLaunchKernelGGL((k_gather2d_nm<T, 4>), dim3(grid), dim3(block), 0, stream, m,
                                       P, nm, out, rep);
            }
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_gather2d<T>, dim3(grid), dim3(block), 0, stream, m, P, nodal, F, out, rep);
    } else {
        const int grid = (m.np + block - 1) / block;
        hipLaunchKernelGGL(k_gather1d<T>, dim3(grid), dim3(block), 0, stream, m, P, nodal, F, out, rep);
    }
    return hipGetLastError();
}
template hipError_t launch_gather<float>(const Mesh&, Particles<float>, const float*, int, float*,
                                         p2m_report*, hipStream_t, void*, size_t);
template hipError_t launch_gather<double>(const Mesh&, Particles<double>, const double*, int,
                                          double*, p2m_report*, hipStream_t, void*, size_t);

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
