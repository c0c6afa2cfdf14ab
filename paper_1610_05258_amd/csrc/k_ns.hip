// The mesh half of the particle fluid solver of Sec. 3.3 (Taylor-Green vortex
// sheet) on the periodic "/"-split P1 mesh with square cells of side h:
//
//   coef    : stencil arrays of the two symmetric systems the mass-matrix solver
//             takes (D, E, N, NE per node, and the diagonal as w):
//               viscous  I + s K, s = dt nu / h^2, K the P1 stiffness matrix, which
//                        on right isosceles triangles is the five-point Laplacian;
//               pressure K with node 0 held at 0 (its row and column replaced by
//                        the identity, which changes p by a constant only);
//   div     : right-hand side of the pressure system, -(1/dt) (D U*)_k with
//             (D U)_k = int psi_k div U_h;
//   correct : the projection U^{n+1} = U* - dt M_L^{-1} G p, (G p)_k = int psi_k
//             grad p_h, M_L = h^2 (row sums of the P1 mesh mass matrix);
//   advect  : mid-point advection of the particles, r* = r + (dt/2) a with a the
//             interpolated U^{n+1}, r <- r + dt U^{n+1}(r*), wrapped into [0, L).
//
// Every node sees the six triangles around it: of cell (i, j) both triangles
// (the node is their corner n00), of cell (i-1, j) the lower one (corner n10), of
// cell (i-1, j-1) both (corner n11) and of cell (i, j-1) the upper one (corner
// n01).  On a triangle the P1 derivatives are node differences over h; the
// integral of a hat over a triangle is h^2/6.  The node sums are formed in FP64
// and rounded once.
#include "p2m_internal.hpp"

namespace p2m {

namespace {

struct Nbr {
    int i, j, im, jm, ip, jp;
};

__device__ __forceinline__ Nbr nbr(int k, int nx, int ny) {
    Nbr q;
    q.i = k % nx;
    q.j = k / nx;
    q.im = q.i == 0 ? nx - 1 : q.i - 1;
    q.jm = q.j == 0 ? ny - 1 : q.j - 1;
    q.ip = q.i + 1 == nx ? 0 : q.i + 1;
    q.jp = q.j + 1 == ny ? 0 : q.j + 1;
    return q;
}

__global__ void k_ns_coef(int nx, int ny, float s, float* __restrict__ cv, float* __restrict__ wv,
                          float* __restrict__ cp, float* __restrict__ wp) {
    const int nn = nx * ny;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    const float dv = (float)(1.0 + 4.0 * (double)s);
    cv[k] = dv;
    cv[nn + k] = -s;
    cv[2 * nn + k] = -s;
    cv[3 * nn + k] = 0.f;
    wv[k] = dv;
    // node 0's couplings: its own E and N, the E of (nx-1, 0) and the N of (0, ny-1)
    const int i = k % nx, j = k / nx;
    const bool pin = k == 0;
    const bool e0 = pin || (i == nx - 1 && j == 0);
    const bool n0 = pin || (i == 0 && j == ny - 1);
    const float dp = pin ? 1.f : 4.f;
    cp[k] = dp;
    cp[nn + k] = e0 ? 0.f : -1.f;
    cp[2 * nn + k] = n0 ? 0.f : -1.f;
    cp[3 * nn + k] = 0.f;
    wp[k] = dp;
}

// rhs_k = scale * sum of the six triangles' divergence differences (lower triangle
// of cell c: u10 - u00 + v11 - v10; upper: u11 - u01 + v01 - v00), scale =
// -(h/6)/dt; with pin, 0 at the held node 0
__global__ void k_ns_div(int nx, int ny, double scale, int pin, const float* __restrict__ U,
                         float* __restrict__ rhs) {
    const int nn = nx * ny;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    const Nbr q = nbr(k, nx, ny);
    const float* u = U;
    const float* v = U + nn;
    auto at = [&](const float* a, int ii, int jj) { return (double)a[ii + nx * jj]; };
    // cell (ci, cj) with upper-right corner (ci1, cj1)
    auto dl = [&](int ci, int cj, int ci1, int cj1) {
        return (at(u, ci1, cj) - at(u, ci, cj)) + (at(v, ci1, cj1) - at(v, ci1, cj));
    };
    auto du = [&](int ci, int cj, int ci1, int cj1) {
        return (at(u, ci1, cj1) - at(u, ci, cj1)) + (at(v, ci, cj1) - at(v, ci, cj));
    };
    const double sum = dl(q.i, q.j, q.ip, q.jp) + du(q.i, q.j, q.ip, q.jp) +
                       dl(q.im, q.j, q.i, q.jp) + dl(q.im, q.jm, q.i, q.j) +
                       du(q.im, q.jm, q.i, q.j) + du(q.i, q.jm, q.ip, q.j);
    rhs[k] = (pin && k == 0) ? 0.f : (float)(scale * sum);
}

// U^{n+1}_k = U*_k - factor * (sum of the six triangles' gradient differences),
// lower triangle of cell c: (p10 - p00, p11 - p10); upper: (p11 - p01, p01 - p00);
// factor = dt / (6 h)
__global__ void k_ns_correct(int nx, int ny, double factor, const float* __restrict__ Us,
                             const float* __restrict__ p, float* __restrict__ Un) {
    const int nn = nx * ny;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    const Nbr q = nbr(k, nx, ny);
    auto at = [&](int ii, int jj) { return (double)p[ii + nx * jj]; };
    double gx = 0.0, gy = 0.0;
    auto gl = [&](int ci, int cj, int ci1, int cj1) {
        gx += at(ci1, cj) - at(ci, cj);
        gy += at(ci1, cj1) - at(ci1, cj);
    };
    auto gu = [&](int ci, int cj, int ci1, int cj1) {
        gx += at(ci1, cj1) - at(ci, cj1);
        gy += at(ci, cj1) - at(ci, cj);
    };
    gl(q.i, q.j, q.ip, q.jp);
    gu(q.i, q.j, q.ip, q.jp);
    gl(q.im, q.j, q.i, q.jp);
    gl(q.im, q.jm, q.i, q.j);
    gu(q.im, q.jm, q.i, q.j);
    gu(q.i, q.jm, q.ip, q.j);
    Un[k] = (float)((double)Us[k] - factor * gx);
    Un[nn + k] = (float)((double)Us[nn + k] - factor * gy);
}

__device__ __forceinline__ double wrap(double x, double len) {
    return __dsub_rn(x, len * floor(x / len));
}

// U at an FP64 position (its triangle's three nodes, FP64 weights); false when the
// position cannot be located
__device__ __forceinline__ bool interp2(const Mesh& m, const float* __restrict__ U, double x,
                                        double y, double& ux, double& uy, bool& finite) {
    int cx = 0, cy = 0;
    double xi = 0.0, eta = 0.0;
    bool fx = true, fy = true;
    bool ok = locate_axis(x, m.nx, m.inv_hx, cx, xi, fx);
    ok = locate_axis(y, m.ny, m.inv_hy, cy, eta, fy) && ok;
    finite = fx && fy;
    if (!ok) return false;
    const int i1 = cx + 1 == m.nx ? 0 : cx + 1;
    const int j1 = cy + 1 == m.ny ? 0 : cy + 1;
    double c00, c10, c11, c01;
    corner_weights<double>(xi, eta, c00, c10, c11, c01);
    const int k00 = cx + m.nx * cy, k10 = i1 + m.nx * cy, k11 = i1 + m.nx * j1, k01 = cx + m.nx * j1;
    const float* v = U + m.nn;
    ux = c00 * U[k00] + c10 * U[k10] + c11 * U[k11] + c01 * U[k01];
    uy = c00 * v[k00] + c10 * v[k10] + c11 * v[k11] + c01 * v[k01];
    return true;
}

// x, y and xo, yo may be the same arrays (each thread reads its particle before
// writing it)
__global__ void k_ns_advect(Mesh m, double lx, double ly, double dt, const float* x,
                            const float* y, const float* __restrict__ a,
                            const float* __restrict__ U, float* xo, float* yo,
                            p2m_report* __restrict__ rep) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.np) return;
    const double x0 = x[i], y0 = y[i];
    const double xm = wrap(x0 + 0.5 * dt * (double)a[i], lx);
    const double ym = wrap(y0 + 0.5 * dt * (double)a[m.np + i], ly);
    double ux = 0.0, uy = 0.0;
    bool finite = true;
    if (!interp2(m, U, xm, ym, ux, uy, finite)) {
        if (rep) atomicOr(&rep->flags, finite ? (uint32_t)P2M_FLAG_RANGE : (uint32_t)P2M_FLAG_NONFINITE);
        xo[i] = NAN;
        yo[i] = NAN;
        return;
    }
    xo[i] = (float)wrap(x0 + dt * ux, lx);
    yo[i] = (float)wrap(y0 + dt * uy, ly);
}

// ---------------------------------------------------------------------------
// Direct solves of the mesh systems by the 2D discrete Fourier transform:
// I + s K and K are circulant on the periodic mesh, diagonal in the 2D discrete
// Fourier basis with eigenvalues 1 + s lam and lam, lam(kx, ky) = 4 - 2 cos(2 pi
// kx / nx) - 2 cos(2 pi ky / ny) (the five-point symbol); K's zero mode is the
// constant, left at 0 (zero-mean pressure).  Transforms in FP64: row transforms
// of one length per workgroup (radix-2 Stockham in LDS, natural order in and out;
// other lengths by Bluestein's algorithm over a power-of-two convolution), a tiled
// transpose between the two directions.
// ---------------------------------------------------------------------------
constexpr int kFftMaxN = 2048;   // 2n complex doubles of LDS = 64 KB

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// radix-2 Stockham transform of x[0..n), n = 2^logn, in LDS (y: scratch of the
// same size); the result ends in x (the two pointers are swapped per pass).  The
// workgroup's threads share the work; the caller synchronises before.
__device__ __forceinline__ void fft_lds(double2*& x, double2*& y, int n, int logn, double sign) {
    const int half = n >> 1;
    for (int ls = 0; ls < logn; ++ls) {
        const int ns = 1 << ls;
        for (int j = threadIdx.x; j < half; j += blockDim.x) {
            const int k = j & (ns - 1);
            const double2 a = x[j], b0 = x[j + half];
            double sn, cs;
            sincospi(sign * (double)k / (double)ns, &sn, &cs);
            const double2 b = make_double2(b0.x * cs - b0.y * sn, b0.x * sn + b0.y * cs);
            const int d = ((j >> ls) << (ls + 1)) + k;
            y[d] = cadd(a, b);
            y[d + ns] = csub(a, b);
        }
        __syncthreads();
        double2* t = x;
        x = y;
        y = t;
    }
}

// rows of length n = 2^logn, one per workgroup; sign -1 forward, +1 inverse
// (unnormalised); REAL_IN reads reals of type R (imaginary part 0), REAL_OUT writes
// the real part times scale as R
template <bool REAL_IN, bool REAL_OUT, typename R>
__global__ void k_fft_rows(const void* __restrict__ in, void* __restrict__ out, int n, int logn,
                           double sign, double scale) {
    extern __shared__ double2 fsh[];
    double2* x = fsh;
    double2* y = fsh + n;
    const size_t base = (size_t)blockIdx.x * n;
    for (int t = threadIdx.x; t < n; t += blockDim.x)
        x[t] = REAL_IN ? make_double2((double)((const R*)in)[base + t], 0.0)
                       : ((const double2*)in)[base + t];
    __syncthreads();
    fft_lds(x, y, n, logn, sign);
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        if (REAL_OUT)
            ((R*)out)[base + t] = (R)(x[t].x * scale);
        else
            ((double2*)out)[base + t] = x[t];
    }
}

// Rows of any length n <= kFftMaxN / 2 by Bluestein's chirp-z algorithm: with
// c_j = exp(-i pi j^2 / n), the DFT is X_k = c_k sum_j (x_j c_j) conj(c_{k-j}), a
// circular convolution of length M = 2^logm >= 2n - 1 done by two radix-2
// transforms and the transform bhat of the chirp (k_fft_chirp).  The inverse
// (sign +1) conjugates on the way in and out.  Arguments as k_fft_rows.
__device__ __forceinline__ double2 chirp(int j, int n) {
    double sn, cs;
    sincospi(-(double)(((long long)j * j) % (2LL * n)) / (double)n, &sn, &cs);
    return make_double2(cs, sn);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// bhat = FFT_M(b), b_m = conj(c_m) for 0 <= m < n, b_{M-m} = conj(c_m) for
// 0 < m < n, 0 elsewhere; one workgroup
__global__ void k_fft_chirp(double2* __restrict__ bhat, int n, int m, int logm) {
    extern __shared__ double2 fsh[];
    double2* x = fsh;
    double2* y = fsh + m;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const int j = t < n ? t : (t > m - n ? m - t : -1);
        double2 v = make_double2(0.0, 0.0);
        if (j >= 0) {
            const double2 c = chirp(j, n);
            v = make_double2(c.x, -c.y);
        }
        x[t] = v;
    }
    __syncthreads();
    fft_lds(x, y, m, logm, -1.0);
    for (int t = threadIdx.x; t < m; t += blockDim.x) bhat[t] = x[t];
}

template <bool REAL_IN, bool REAL_OUT, typename R>
__global__ void k_fft_rows_chirp(const void* __restrict__ in, void* __restrict__ out, int n, int m,
                                 int logm, const double2* __restrict__ bhat, double sign,
                                 double scale) {
    extern __shared__ double2 fsh[];
    double2* x = fsh;
    double2* y = fsh + m;
    const size_t base = (size_t)blockIdx.x * n;
    const bool inv = sign > 0.0;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (t < n) {
            v = REAL_IN ? make_double2((double)((const R*)in)[base + t], 0.0)
                        : ((const double2*)in)[base + t];
            if (inv) v.y = -v.y;
            v = cmul(v, chirp(t, n));
        }
        x[t] = v;
    }
    __syncthreads();
    fft_lds(x, y, m, logm, -1.0);
    for (int t = threadIdx.x; t < m; t += blockDim.x) x[t] = cmul(x[t], bhat[t]);
    __syncthreads();
    fft_lds(x, y, m, logm, 1.0);
    const double im = 1.0 / (double)m;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        double2 v = cmul(x[t], chirp(t, n));
        v = make_double2(v.x * im, (inv ? -v.y : v.y) * im);
        if (REAL_OUT)
            ((R*)out)[base + t] = (R)(v.x * scale);
        else
            ((double2*)out)[base + t] = v;
    }
}

// out[b][c][r] = in[b][r][c] for nb matrices of R x C, 32 x 32 tiles through LDS
__global__ void k_transpose_c(const double2* __restrict__ in, double2* __restrict__ out, int R, int C) {
    __shared__ double2 tile[32][33];
    const size_t mb = (size_t)blockIdx.z * R * C;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    for (int dy = threadIdx.y; dy < 32; dy += blockDim.y) {
        const int r = r0 + dy, c = c0 + threadIdx.x;
        if (r < R && c < C) tile[dy][threadIdx.x] = in[mb + (size_t)r * C + c];
    }
    __syncthreads();
    for (int dy = threadIdx.y; dy < 32; dy += blockDim.y) {
        const int c = c0 + dy, r = r0 + threadIdx.x;
        if (r < R && c < C) out[mb + (size_t)c * R + r] = tile[threadIdx.x][dy];
    }
}

// spectrum [nb][nx][ny] (row kx, column ky) divided by the system's eigenvalue:
// 1 + s lam (viscous), lam (pressure; the zero mode set to 0), or the consistent
// P1 mass matrix of the "/" split, s (1/2 + (cos tx + cos ty + cos(tx + ty)) / 6)
// with s = hx hy (mass)
__global__ void k_fft_divide(double2* __restrict__ a, int nx, int ny, int nb, double s, int mode) {
    const size_t nn = (size_t)nx * ny;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * nb) return;
    const size_t e = t % nn;
    const int kx = (int)(e / ny), ky = (int)(e % ny);
    double2 v = a[t];
    if (mode == kFftMass) {
        const double m = s * (0.5 + (cospi(2.0 * kx / nx) + cospi(2.0 * ky / ny) +
                                     cospi(2.0 * kx / nx + 2.0 * ky / ny)) / 6.0);
        a[t] = make_double2(v.x / m, v.y / m);
        return;
    }
    const double lam = 4.0 - 2.0 * cospi(2.0 * kx / nx) - 2.0 * cospi(2.0 * ky / ny);
    if (mode == kFftPressure) {
        if (kx == 0 && ky == 0) v = make_double2(0.0, 0.0);
        else v = make_double2(v.x / lam, v.y / lam);
    } else {
        const double d = 1.0 + s * lam;
        v = make_double2(v.x / d, v.y / d);
    }
    a[t] = v;
}

inline int grid_of(int n, int b) { return (n + b - 1) / b; }

inline int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace


// a side the row transforms take: a power of two up to kFftMaxN, or any length up
// to kFftMaxN / 2 (Bluestein, convolution length at most kFftMaxN)
static bool fft_side(int n) {
    return n >= 2 && (((n & (n - 1)) == 0 && n <= kFftMaxN) || 2 * n - 1 <= kFftMaxN);
}

bool fft_supported(const Mesh& m) { return m.dim == 2 && fft_side(m.nx) && fft_side(m.ny); }

// two complex planes of nb fields, then the chirp transforms of the two sides
size_t fft_workspace_bytes(const Mesh& m, int nb) {
    return ((size_t)2 * nb * m.nn + 2 * kFftMaxN) * sizeof(double2);
}

template <typename Real>
hipError_t launch_fft_solve(const Mesh& m, int nb, double s, int mode, const Real* rhs, Real* x,
                            void* ws, hipStream_t stream) {
    double2* fa = (double2*)ws;
    double2* fb = fa + (size_t)nb * m.nn;
    double2* chirp_tab[2] = {fb + (size_t)nb * m.nn, fb + (size_t)nb * m.nn + kFftMaxN};
    auto conv_len = [](int n) {
        int lg = 0;
        while ((1 << lg) < 2 * n - 1) ++lg;
        return lg;
    };
    // the chirp transform of each side that is not a power of two (x: table 0, y: 1)
    const int sides[2] = {m.nx, m.ny};
    for (int d = 0; d < 2; ++d) {
        const int n = sides[d];
        if ((n & (n - 1)) == 0) continue;
        const int lg = conv_len(n), mm = 1 << lg;
        const int threads = mm / 2 < 256 ? (mm / 2 < 64 ? 64 : mm / 2) : 256;
        hipLaunchKernelGGL(k_fft_chirp, dim3(1), dim3(threads), (size_t)2 * mm * sizeof(double2),
                           stream, chirp_tab[d], n, mm, lg);
        const hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess) return e0;
    }
    const int nx = m.nx, ny = m.ny, lx = ilog2(nx), ly = ilog2(ny);
    auto rows = [&](int n, int nrows, const void* in, void* out, double sign, double scale,
                    bool real_in, bool real_out) {
        if ((n & (n - 1)) != 0) {   // Bluestein
            const int lg = conv_len(n), mm = 1 << lg;
            const int threads = mm / 2 < 256 ? (mm / 2 < 64 ? 64 : mm / 2) : 256;
            const size_t shm = (size_t)2 * mm * sizeof(double2);
            const double2* tab = chirp_tab[n == m.nx ? 0 : 1];
            if (real_in)
                hipLaunchKernelGGL((k_fft_rows_chirp<true, false, Real>), dim3(nrows), dim3(threads), shm,
                                   stream, in, out, n, mm, lg, tab, sign, scale);
            else if (real_out)
                hipLaunchKernelGGL((k_fft_rows_chirp<false, true, Real>), dim3(nrows), dim3(threads), shm,
                                   stream, in, out, n, mm, lg, tab, sign, scale);
            else
                hipLaunchKernelGGL((k_fft_rows_chirp<false, false, Real>), dim3(nrows), dim3(threads),
                                   shm, stream, in, out, n, mm, lg, tab, sign, scale);
            return hipGetLastError();
        }
        const int threads = n / 2 < 256 ? (n / 2 < 64 ? 64 : n / 2) : 256;
        const size_t shm = (size_t)2 * n * sizeof(double2);
        const int lg = ilog2(n);
        if (real_in)
            hipLaunchKernelGGL((k_fft_rows<true, false, Real>), dim3(nrows), dim3(threads), shm, stream, in, out,
                               n, lg, sign, scale);
        else if (real_out)
            hipLaunchKernelGGL((k_fft_rows<false, true, Real>), dim3(nrows), dim3(threads), shm, stream, in, out,
                               n, lg, sign, scale);
        else
            hipLaunchKernelGGL((k_fft_rows<false, false, Real>), dim3(nrows), dim3(threads), shm, stream, in, out,
                               n, lg, sign, scale);
        return hipGetLastError();
    };
    auto transpose = [&](const double2* in, double2* out, int R, int C) {
        hipLaunchKernelGGL(k_transpose_c, dim3(grid_of(C, 32), grid_of(R, 32), nb), dim3(32, 8), 0, stream,
                           in, out, R, C);
        return hipGetLastError();
    };
    (void)lx;
    (void)ly;
    hipError_t e;
    if ((e = rows(nx, nb * ny, rhs, fa, -1.0, 1.0, true, false)) != hipSuccess) return e;
    if ((e = transpose(fa, fb, ny, nx)) != hipSuccess) return e;
    if ((e = rows(ny, nb * nx, fb, fa, -1.0, 1.0, false, false)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fft_divide, dim3(grid_of(nb * m.nn, 256)), dim3(256), 0, stream, fa, nx, ny, nb,
                       s, mode);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = rows(ny, nb * nx, fa, fb, 1.0, 1.0, false, false)) != hipSuccess) return e;
    if ((e = transpose(fb, fa, nx, ny)) != hipSuccess) return e;
    return rows(nx, nb * ny, fa, x, 1.0, 1.0 / ((double)nx * ny), false, true);
}
template hipError_t launch_fft_solve<double>(const Mesh&, int, double, int, const double*, double*,
                                             void*, hipStream_t);

hipError_t launch_ns_fft_solve(const Mesh& m, int nb, double s, int pressure, const float* rhs,
                               float* x, void* ws, hipStream_t stream) {
    return launch_fft_solve<float>(m, nb, s, pressure ? kFftPressure : kFftViscous, rhs, x, ws,
                                   stream);
}

hipError_t launch_ns_coef(const Mesh& m, float s, float* cv, float* wv, float* cp, float* wp,
                          hipStream_t stream) {
    hipLaunchKernelGGL(k_ns_coef, dim3(grid_of(m.nn, 256)), dim3(256), 0, stream, m.nx, m.ny, s,
                       cv, wv, cp, wp);
    return hipGetLastError();
}

hipError_t launch_ns_div(const Mesh& m, double scale, int pin, const float* U, float* rhs,
                         hipStream_t stream) {
    hipLaunchKernelGGL(k_ns_div, dim3(grid_of(m.nn, 256)), dim3(256), 0, stream, m.nx, m.ny, scale,
                       pin, U, rhs);
    return hipGetLastError();
}

hipError_t launch_ns_correct(const Mesh& m, double factor, const float* Us, const float* p,
                             float* Un, hipStream_t stream) {
    hipLaunchKernelGGL(k_ns_correct, dim3(grid_of(m.nn, 256)), dim3(256), 0, stream, m.nx, m.ny,
                       factor, Us, p, Un);
    return hipGetLastError();
}

hipError_t launch_ns_advect(const Mesh& m, double lx, double ly, double dt, const float* x,
                            const float* y, const float* a, const float* U, float* xo, float* yo,
                            p2m_report* rep, hipStream_t stream) {
    if (m.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ns_advect, dim3(grid_of(m.np, 256)), dim3(256), 0, stream, m, lx, ly, dt,
                       x, y, a, U, xo, yo, rep);
    return hipGetLastError();
}

}  // namespace p2m
