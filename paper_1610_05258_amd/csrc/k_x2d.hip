// Paper-exact 2D assignment (Sec. 3.2; Appendix B): P1 hats on the periodic
// Delaunay triangulation of the particles, all in FP64.
//
//   k_x2d_pos      binned order: wrapped positions, values and the cell of every
//                  located particle (slot k = position in the binned order)
//   k_x2d_star     per particle, its Delaunay neighbours counter-clockwise by gift
//                  wrapping over the particles of the surrounding mesh cells, widened
//                  ring by ring until no particle outside the searched rings can
//                  change them (twice the largest circumradius within the searched
//                  radius); the volume int psi_mu is a third of the area of the
//                  triangles (mu, n_j, n_j+1).
//   k_x2d_check    every triangle (mu, a, b) must appear in the lists of a and b too
//   k_x2d_locate   the particle interpolant of eq. (1) at the points of a regular
//                  grid (mesh nodes, or nodes and edge midpoints): the triangle that
//                  holds the point is found by a walk from the nearest particle
//   k_x2d_rhs_mesh int A psi_j over the six mesh triangles around node j with the
//                  Appendix-B rule (A at vertices and midpoints from k_x2d_locate)
//   k_x2d_rhs_part int Abar psi_mu over the triangles around particle mu with the
//                  Appendix-B rule (Abar the mesh interpolant)
//   k_x2d_mpart    the consistent particle mass matrix in the sparse-row form of
//                  the streaming CG (diagonal, then the off-diagonal slots)
//   k_x2d_mmesh    the consistent mesh mass stencil (D, E, N, NE)
// The mass systems are solved by the streaming CG (k_cg.hip).
#include "p2m_internal.hpp"

namespace p2m {

namespace {

constexpr int kB = 128;
constexpr int kCap = P2M_X2D_MAXDEG;   // neighbours per particle
constexpr int kRingMax = 8;            // mesh-cell rings searched around a particle
constexpr int kWalkMax = 1024;         // triangles a point-location walk may visit

inline int grid_of(size_t n) { return (int)((n + kB - 1) / kB); }

struct Geo {
    int nx, ny, N;
    int r0;   // first ring count the triangulation tries
    double lx, ly, hx, hy, inv_hx, inv_hy;
};

__device__ __forceinline__ int floor_div(int a, int n) {
    return a >= 0 ? a / n : -((-a + n - 1) / n);
}
__device__ __forceinline__ int pack_shift(int sx, int sy) { return (sx + 128) | ((sy + 128) << 8); }
__device__ __forceinline__ int shift_x(int s) { return (s & 255) - 128; }
__device__ __forceinline__ int shift_y(int s) { return ((s >> 8) & 255) - 128; }

__device__ __forceinline__ void flag(p2m_report* rep, uint32_t f) {
    if (rep) atomicOr(&rep->flags, f);
}

// ---------------------------------------------------------------------------
__global__ void k_x2d_pos(Geo g, const int32_t* __restrict__ perm, const double* __restrict__ x,
                          const double* __restrict__ y, const double* __restrict__ values, int F,
                          int np, double* __restrict__ xs, double* __restrict__ ys,
                          int32_t* __restrict__ cell, double* __restrict__ As) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= g.N) return;
    const int p = perm[k];
    const double px = x[p], py = y[p];
    int cx, cy;
    double xi, eta;
    bool fx, fy;
    locate_axis(px, g.nx, g.inv_hx, cx, xi, fx);
    locate_axis(py, g.ny, g.inv_hy, cy, eta, fy);
    // a position in [L, L + h) belongs to cell 0 (the binning's wrap); move it there
    xs[k] = __dmul_rn(px, g.inv_hx) >= (double)g.nx ? px - g.lx : px;
    ys[k] = __dmul_rn(py, g.inv_hy) >= (double)g.ny ? py - g.ly : py;
    cell[k] = cx + g.nx * cy;
    if (values)
        for (int f = 0; f < F; ++f) As[(size_t)f * g.N + k] = values[(size_t)f * np + p];
}

// ---------------------------------------------------------------------------
// The Delaunay neighbours of slot k, counter-clockwise, by gift wrapping over the
// particles of the mesh cells within r rings of its own (coordinates relative to
// the particle).  The nearest particle is a Delaunay neighbour.  From a neighbour
// u, the next one is the particle c left of the edge (k, u) whose circle through
// k, u and c has its centre first along the edge's bisector: centre
// u / 2 + t (-u_y, u_x) with t = (|c|^2 - u.c) / (2 u x c), smallest t (an empty
// circle).  The centres are the Voronoi vertices; when twice the largest circle
// radius is within the searched radius (every particle left out is at least
// r min(hx, hy) away), no particle outside the rings can change the result;
// otherwise the search widens by a ring.
// One particle per group of G lanes: each lane scans every G-th cell of the
// search square, and the group agrees on the winner of every scan with a
// butterfly of lane exchanges (every lane ends with the same winner: the
// comparison of two candidates evaluates the same two products on both lanes).
struct Cand {
    double n, d;     // key n / d (d > 0)
    double vx, vy;   // position relative to the particle
    int q, s;        // slot and packed image shift; q < 0: none
};

// a before b: smaller key, ties to the smaller (slot, shift)
__device__ __forceinline__ bool before_cand(const Cand& a, const Cand& b) {
    if (a.q < 0) return false;
    if (b.q < 0) return true;
    const double l = a.n * b.d, r = b.n * a.d;
    if (l != r) return l < r;
    return a.q != b.q ? a.q < b.q : a.s < b.s;
}

// a found candidate before the wrap's best so far: one lane per particle scans in a
// fixed order, and equal keys there mean four points on one circle (a triangulation
// that is not unique), so the first found stands; a group breaks ties as above so
// that its winner does not depend on how the cells were dealt to its lanes
template <int G>
__device__ __forceinline__ bool before_wrap(const Cand& a, const Cand& b) {
    if constexpr (G == 1) return b.q < 0 || a.n * b.d < b.n * a.d;
    return before_cand(a, b);
}

template <int G>
__device__ __forceinline__ Cand group_min(Cand v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
        Cand o;
        o.n = __shfl_xor(v.n, m, G);
        o.d = __shfl_xor(v.d, m, G);
        o.vx = __shfl_xor(v.vx, m, G);
        o.vy = __shfl_xor(v.vy, m, G);
        o.q = __shfl_xor(v.q, m, G);
        o.s = __shfl_xor(v.s, m, G);
        if (before_cand(o, v)) v = o;
    }
    return v;
}

template <int G>
__device__ __forceinline__ int group_or(int v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v |= __shfl_xor(v, m, G);
    return v;
}

// the particles of every G-th cell of the (2r + 1)^2 square around (cx, cy),
// starting at this lane's cell
template <int G, typename Fn>
__device__ __forceinline__ void for_lane_candidates(const Geo& g, const int32_t* __restrict__ cs,
                                                    int cx, int cy, int r, int lane, Fn&& fn) {
    if constexpr (G == 1) {   // row by row
        for (int dy = -r; dy <= r; ++dy) {
            const int ay = cy + dy;
            const int sy = floor_div(ay, g.ny);
            const int row = g.nx * (ay - sy * g.ny);
            for (int dx = -r; dx <= r; ++dx) {
                const int ax = cx + dx;
                const int sx = floor_div(ax, g.nx);
                const int cc = (ax - sx * g.nx) + row;
                const int q1 = cs[cc + 1];
                for (int q = cs[cc]; q < q1; ++q) fn(q, sx, sy);
            }
        }
    } else {   // cells lane, lane + G, ... of the square in row-major order
        const int side = 2 * r + 1, ncell = side * side;
        for (int ci = lane; ci < ncell; ci += G) {
            const int dyy = ci / side, dxx = ci - dyy * side;
            const int ax = cx + dxx - r, ay = cy + dyy - r;
            const int sx = floor_div(ax, g.nx), sy = floor_div(ay, g.ny);
            const int cc = (ax - sx * g.nx) + g.nx * (ay - sy * g.ny);
            const int q1 = cs[cc + 1];
            for (int q = cs[cc]; q < q1; ++q) fn(q, sx, sy);
        }
    }
}

template <int G>
__global__ __launch_bounds__(kB) void k_x2d_star(Geo g, const double* __restrict__ xs,
                                                 const double* __restrict__ ys,
                                                 const int32_t* __restrict__ cell,
                                                 const int32_t* __restrict__ cs,
                                                 int32_t* __restrict__ deg, int32_t* __restrict__ nbr,
                                                 int32_t* __restrict__ nsh, double* __restrict__ vol,
                                                 p2m_report* rep) {
    // plain rounding, no fused multiply-adds: the decisions below compare cross
    // products of nearly parallel vectors, and the same expression must give the
    // same result in every particle's computation
#pragma clang fp contract(off)
    const int tid = blockIdx.x * kB + threadIdx.x;
    const int k = tid / G, lane = tid - k * G;
    if (k >= g.N) return;   // the whole group
    const double px = xs[k], py = ys[k];
    const int c = cell[k];
    const int cy = c / g.nx, cx = c - cy * g.nx;
    const double hmin = g.hx < g.hy ? g.hx : g.hy;
    int32_t* nk = nbr + (size_t)k * kCap;
    int32_t* sk = nsh + (size_t)k * kCap;
    int n = 0;
    bool ok = false, bad = false;
    for (int r = g.r0; r <= kRingMax && !ok && !bad; ++r) {
        // the nearest particle image
        Cand b;
        b.q = -1;
        int dup = 0;
        for_lane_candidates<G>(g, cs, cx, cy, r, lane, [&](int q, int sx, int sy) {
            if (q == k && sx == 0 && sy == 0) return;
            Cand e;
            e.vx = (xs[q] - px) + sx * g.lx;
            e.vy = (ys[q] - py) + sy * g.ly;
            e.n = e.vx * e.vx + e.vy * e.vy;
            e.d = 1.0;
            e.q = q;
            e.s = pack_shift(sx, sy);
            if (!(e.n > 0.0)) dup = 1;   // two particles at one position
            if (before_cand(e, b)) b = e;
        });
        b = group_min<G>(b);
        bad = group_or<G>(dup) != 0;
        if (bad || b.q < 0) continue;
        const int q0 = b.q, s0 = b.s;
        int cq = q0, csh = s0;
        double ux = b.vx, uy = b.vy, rmax2 = 0.0;
        bool closed = false;
        n = 0;
        while (n < kCap) {
            if (lane == 0) {
                nk[n] = cq;
                sk[n] = csh;
            }
            ++n;
            // the particle left of (k, u) whose circle through k and u has its centre
            // first along the bisector: t = num / den, den = 2 u x c > 0
            Cand e;
            e.q = -1;
            for_lane_candidates<G>(g, cs, cx, cy, r, lane, [&](int q, int sx, int sy) {
                if (q == k && sx == 0 && sy == 0) return;
                const int sh = pack_shift(sx, sy);
                if (q == cq && sh == csh) return;   // the edge's own end
                const double rx = (xs[q] - px) + sx * g.lx;
                const double ry = (ys[q] - py) + sy * g.ly;
                const double cr = ux * ry - uy * rx;
                if (!(cr > 0.0)) return;
                Cand f;
                f.n = rx * rx + ry * ry - (ux * rx + uy * ry);
                f.d = 2.0 * cr;
                f.vx = rx;
                f.vy = ry;
                f.q = q;
                f.s = sh;
                if (before_wrap<G>(f, e)) e = f;
            });
            e = group_min<G>(e);
            if (e.q < 0) break;   // nothing on the left: the cell is open at this radius
            const double bt = e.n / e.d;
            const double ox = 0.5 * ux - bt * uy, oy = 0.5 * uy + bt * ux;
            const double rho2 = ox * ox + oy * oy;
            rmax2 = rho2 > rmax2 ? rho2 : rmax2;
            if (e.q == q0 && e.s == s0) {
                closed = true;
                break;
            }
            cq = e.q;
            csh = e.s;
            ux = e.vx;
            uy = e.vy;
        }
        const double reach = r * hmin * (1.0 - 1e-9);
        ok = closed && n >= 3 && 4.0 * rmax2 <= reach * reach;
    }
    if (!ok) {
        for (int i = lane; i < kCap; i += G) {
            nk[i] = -1;
            sk[i] = 0;
        }
        if (lane == 0) {
            deg[k] = 0;
            vol[k] = __builtin_nan("");
            flag(rep, P2M_FLAG_TRIANGULATION);
        }
        return;
    }
    for (int i = n + lane; i < kCap; i += G) {
        nk[i] = -1;
        sk[i] = 0;
    }
    if (lane != 0) return;
    deg[k] = n;
    double area2 = 0.0;
    double ax0 = 0.0, ay0 = 0.0, fx0 = 0.0, fy0 = 0.0;
    for (int i = 0; i < n; ++i) {
        const int q = nk[i], sh = sk[i];
        const double rx = (xs[q] - px) + shift_x(sh) * g.lx;
        const double ry = (ys[q] - py) + shift_y(sh) * g.ly;
        if (i == 0) {
            fx0 = rx;
            fy0 = ry;
        } else {
            area2 += ax0 * ry - ay0 * rx;
        }
        ax0 = rx;
        ay0 = ry;
    }
    area2 += ax0 * fy0 - ay0 * fx0;
    vol[k] = area2 / 6.0;   // a third of the triangles' total area (area2 / 2)
}

// position of neighbour entry j of slot u among u's list, or -1
// (a list is kCap = 32 words, 128 bytes, in a 256-byte aligned workspace: four
// entries per 16-byte load)
__device__ __forceinline__ int find_entry(const int32_t* __restrict__ nbr,
                                          const int32_t* __restrict__ nsh, int du, int u, int q,
                                          int s) {
    const int4* nb = (const int4*)(nbr + (size_t)u * kCap);
    const int4* ns = (const int4*)(nsh + (size_t)u * kCap);
    for (int j = 0; j < du; j += 4) {
        const int4 a = nb[j >> 2], b = ns[j >> 2];
        if (a.x == q && b.x == s) return j;
        if (j + 1 < du && a.y == q && b.y == s) return j + 1;
        if (j + 2 < du && a.z == q && b.z == s) return j + 2;
        if (j + 3 < du && a.w == q && b.w == s) return j + 3;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Triangle (k, a, b) with a, b consecutive in k's list is (a, b, k) seen from a:
// in a's list, b must come right before k.  A failure marks the triangulation.
__global__ void k_x2d_check(Geo g, const int32_t* __restrict__ deg, const int32_t* __restrict__ nbr,
                            const int32_t* __restrict__ nsh, p2m_report* rep) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= g.N) return;
    const int d = deg[k];
    if (d == 0) return;   // flagged by the star kernel
    bool ok = true;
    for (int i = 0; i < d && ok; ++i) {
        const int a = nbr[(size_t)k * kCap + i], sa = nsh[(size_t)k * kCap + i];
        const int i1 = (i + 1 == d) ? 0 : i + 1;
        const int b = nbr[(size_t)k * kCap + i1], sb = nsh[(size_t)k * kCap + i1];
        const int da = deg[a];
        // k and b as seen from a's image
        const int sk = pack_shift(-shift_x(sa), -shift_y(sa));
        const int sba = pack_shift(shift_x(sb) - shift_x(sa), shift_y(sb) - shift_y(sa));
        const int j = find_entry(nbr, nsh, da, a, k, sk);
        if (j < 0) {
            ok = false;
            break;
        }
        const int jp = (j == 0) ? da - 1 : j - 1;
        if (nbr[(size_t)a * kCap + jp] != b || nsh[(size_t)a * kCap + jp] != sba) ok = false;
    }
    if (!ok) flag(rep, P2M_FLAG_TRIANGULATION);
}

// ---------------------------------------------------------------------------
// The particle interpolant at grid point (I, J) of a gx x gy grid with spacing
// (dx, dy) (the nodes: the mesh itself; nodes and midpoints: half the spacing).
// out[f][J gx + I]; NaN where the walk fails.
struct Vtx {
    int q, sx, sy;
};

__global__ __launch_bounds__(kB) void k_x2d_locate(Geo g, int gx, int gy, double dx, double dy,
                                                   const double* __restrict__ xs,
                                                   const double* __restrict__ ys,
                                                   const int32_t* __restrict__ cs,
                                                   const int32_t* __restrict__ deg,
                                                   const int32_t* __restrict__ nbr,
                                                   const int32_t* __restrict__ nsh,
                                                   const double* __restrict__ As, int F,
                                                   double* __restrict__ out, p2m_report* rep) {
#pragma clang fp contract(off)   // orientation signs in plain rounding
    const int P = blockIdx.x * kB + threadIdx.x;
    if (P >= gx * gy) return;
    const int J = P / gx, I = P - J * gx;
    const double zx = I * dx, zy = J * dy;
    // cell of the point (points on a cell edge belong to the cell above / right)
    int cx = (int)floor(zx * g.inv_hx), cy = (int)floor(zy * g.inv_hy);
    cx = cx < 0 ? 0 : (cx >= g.nx ? g.nx - 1 : cx);
    cy = cy < 0 ? 0 : (cy >= g.ny ? g.ny - 1 : cy);
    const double hmin = g.hx < g.hy ? g.hx : g.hy;

    // nearest particle image
    double best = 1e300;
    Vtx a = {-1, 0, 0};
    for (int r = 0; r <= kRingMax; ++r) {
        for (int ddy = -r; ddy <= r; ++ddy) {
            const bool edge_row = (ddy == -r || ddy == r);
            const int step = edge_row ? 1 : 2 * r;
            for (int ddx = -r; ddx <= r; ddx += (step > 0 ? step : 1)) {
                const int ax = cx + ddx, ay = cy + ddy;
                const int sx = floor_div(ax, g.nx), sy = floor_div(ay, g.ny);
                const int cc = (ax - sx * g.nx) + g.nx * (ay - sy * g.ny);
                const int q1 = cs[cc + 1];
                for (int q = cs[cc]; q < q1; ++q) {
                    const double rx = (xs[q] - zx) + sx * g.lx;
                    const double ry = (ys[q] - zy) + sy * g.ly;
                    const double d2 = rx * rx + ry * ry;
                    if (d2 < best) {
                        best = d2;
                        a.q = q;
                        a.sx = sx;
                        a.sy = sy;
                    }
                }
                if (step == 0) break;
            }
        }
        const double reach = r * hmin;
        if (a.q >= 0 && best <= reach * reach) break;
    }
    bool ok = a.q >= 0 && deg[a.q] >= 3;
    double la = 0.0, lb = 0.0, lc = 0.0;
    Vtx b = {0, 0, 0}, c = {0, 0, 0};
    auto entry = [&](const Vtx& u, int j) -> Vtx {
        const int s = nsh[(size_t)u.q * kCap + j];
        return Vtx{nbr[(size_t)u.q * kCap + j], u.sx + shift_x(s), u.sy + shift_y(s)};
    };
    auto rel = [&](const Vtx& v, double& rx, double& ry) {
        rx = (xs[v.q] - zx) + v.sx * g.lx;
        ry = (ys[v.q] - zy) + v.sy * g.ly;
    };
    // the neighbour that comes right before v in u's list (the third vertex of
    // the triangle across edge (u, v) from the current one)
    auto before = [&](const Vtx& u, const Vtx& v, Vtx& x) -> bool {
        const int du = deg[u.q];
        if (du < 3) return false;
        const int j = find_entry(nbr, nsh, du, u.q, v.q, pack_shift(v.sx - u.sx, v.sy - u.sy));
        if (j < 0) return false;
        x = entry(u, j == 0 ? du - 1 : j - 1);
        return true;
    };
    if (ok) {
        b = entry(a, 0);
        c = entry(a, 1);
        ok = false;
        for (int step = 0; step < kWalkMax; ++step) {
            double ax_, ay_, bx_, by_, cx_, cy_;
            rel(a, ax_, ay_);
            rel(b, bx_, by_);
            rel(c, cx_, cy_);
            // twice the signed areas of (a, b, z), (b, c, z), (c, a, z) with z at 0
            const double oab = ax_ * by_ - ay_ * bx_;
            const double obc = bx_ * cy_ - by_ * cx_;
            const double oca = cx_ * ay_ - cy_ * ax_;
            Vtx x;
            if (oab < 0.0) {
                if (!before(a, b, x)) break;
                c = b;
                b = x;   // (a, x, b)
            } else if (obc < 0.0) {
                if (!before(b, c, x)) break;
                a = b;
                b = x;   // (b, x, c)
            } else if (oca < 0.0) {
                if (!before(c, a, x)) break;
                b = x;
                const Vtx t = a;
                a = c;
                c = t;   // (c, x, a)
            } else {
                const double s = oab + obc + oca;
                la = obc / s;
                lb = oca / s;
                lc = oab / s;
                ok = s > 0.0;
                break;
            }
        }
    }
    if (!ok) {
        for (int f = 0; f < F; ++f) out[(size_t)f * gx * gy + P] = __builtin_nan("");
        flag(rep, P2M_FLAG_TRIANGULATION);
        return;
    }
    for (int f = 0; f < F; ++f) {
        const double* A = As + (size_t)f * g.N;
        out[(size_t)f * gx * gy + P] = la * A[a.q] + lb * A[b.q] + lc * A[c.q];
    }
}

// ---------------------------------------------------------------------------
// Appendix-B rule on one triangle for its vertex a: |T| (Qa/30 - (Qb + Qc)/60 +
// 2 (Qab + Qac)/15 + Qbc/15)
__device__ __forceinline__ double appb(double area, double qa, double qb, double qc, double qab,
                                       double qac, double qbc) {
    return area * (qa / 30.0 - (qb + qc) / 60.0 + 2.0 * (qab + qac) / 15.0 + qbc / 15.0);
}

// b_j over the six triangles of the "/" split around node (i, j); H [F][2ny][2nx]
// holds A on the half-spacing grid (node (i, j) at (2i, 2j)).
__global__ void k_x2d_rhs_mesh(Geo g, int F, const double* __restrict__ H, double* __restrict__ b) {
    const int k = blockIdx.x * kB + threadIdx.x;
    const int nn = g.nx * g.ny;
    if (k >= nn) return;
    const int j = k / g.nx, i = k - j * g.nx;
    const int gx = 2 * g.nx, gy = 2 * g.ny;
    // the other two vertices of each triangle, in half-spacing offsets
    const int ob[6][2] = {{2, 0}, {2, 2}, {-2, 0}, {-2, -2}, {-2, -2}, {0, -2}};
    const int oc[6][2] = {{2, 2}, {0, 2}, {0, 2}, {0, -2}, {-2, 0}, {2, 0}};
    const double area = 0.5 * g.hx * g.hy;
    for (int f = 0; f < F; ++f) {
        const double* Hf = H + (size_t)f * gx * gy;
        auto at = [&](int di, int dj) -> double {
            int I = 2 * i + di, Jj = 2 * j + dj;
            I = I < 0 ? I + gx : (I >= gx ? I - gx : I);
            Jj = Jj < 0 ? Jj + gy : (Jj >= gy ? Jj - gy : Jj);
            return Hf[(size_t)Jj * gx + I];
        };
        const double qa = at(0, 0);
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int bx = ob[t][0], by = ob[t][1], cx = oc[t][0], cy = oc[t][1];
            s += appb(area, qa, at(bx, by), at(cx, cy), at(bx / 2, by / 2), at(cx / 2, cy / 2),
                      at((bx + cx) / 2, (by + cy) / 2));
        }
        b[(size_t)f * nn + k] = s;
    }
}

// the mesh interpolant (eq. (3) hats, "/" split) at a point of the plane
__device__ __forceinline__ double mesh_at(const Geo& g, const double* __restrict__ nodal, double x,
                                          double y) {
    x -= floor(x / g.lx) * g.lx;
    y -= floor(y / g.ly) * g.ly;
    int cx, cy;
    double xi, eta;
    bool fx, fy;
    locate_axis(x, g.nx, g.inv_hx, cx, xi, fx);
    locate_axis(y, g.ny, g.inv_hy, cy, eta, fy);
    double c00, c10, c11, c01;
    corner_weights<double>(xi, eta, c00, c10, c11, c01);
    const int i1 = (cx + 1 == g.nx) ? 0 : cx + 1, j1 = (cy + 1 == g.ny) ? 0 : cy + 1;
    return c00 * nodal[cx + g.nx * cy] + c10 * nodal[i1 + g.nx * cy] +
           c11 * nodal[i1 + g.nx * j1] + c01 * nodal[cx + g.nx * j1];
}

// c_mu over the triangles (mu, n_i, n_i+1) of slot k; c [F][N]
__global__ void k_x2d_rhs_part(Geo g, int F, const double* __restrict__ xs,
                               const double* __restrict__ ys, const int32_t* __restrict__ deg,
                               const int32_t* __restrict__ nbr, const int32_t* __restrict__ nsh,
                               const double* __restrict__ nodal, double* __restrict__ c) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= g.N) return;
    const int d = deg[k];
    const int nn = g.nx * g.ny;
    const double px = xs[k], py = ys[k];
    for (int f = 0; f < F; ++f) {
        const double* Af = nodal + (size_t)f * nn;
        if (d == 0) {
            c[(size_t)f * g.N + k] = __builtin_nan("");
            continue;
        }
        const double qp = mesh_at(g, Af, px, py);
        double s = 0.0;
        int q = nbr[(size_t)k * kCap + d - 1], sh = nsh[(size_t)k * kCap + d - 1];
        double ax = (xs[q] - px) + shift_x(sh) * g.lx, ay = (ys[q] - py) + shift_y(sh) * g.ly;
        double qa = mesh_at(g, Af, px + ax, py + ay);
        double qpa = mesh_at(g, Af, px + 0.5 * ax, py + 0.5 * ay);
        for (int i = 0; i < d; ++i) {
            q = nbr[(size_t)k * kCap + i];
            sh = nsh[(size_t)k * kCap + i];
            const double bx = (xs[q] - px) + shift_x(sh) * g.lx;
            const double by = (ys[q] - py) + shift_y(sh) * g.ly;
            const double qb = mesh_at(g, Af, px + bx, py + by);
            const double qpb = mesh_at(g, Af, px + 0.5 * bx, py + 0.5 * by);
            const double qab = mesh_at(g, Af, px + 0.5 * (ax + bx), py + 0.5 * (ay + by));
            const double area = 0.5 * (ax * by - ay * bx);   // triangle (mu, a, b)
            s += appb(area, qp, qa, qb, qpa, qpb, qab);
            ax = bx;
            ay = by;
            qa = qb;
            qpa = qpb;
        }
        c[(size_t)f * g.N + k] = s;
    }
}

// m_part in the CG's sparse-row form: coef[k] = sum |T| / 6; slot i of row k is the
// neighbour n_i with (|T_{i-1}| + |T_i|) / 12, T_i = (mu, n_i, n_i+1).
__global__ void k_x2d_mpart(Geo g, const double* __restrict__ xs, const double* __restrict__ ys,
                            const int32_t* __restrict__ deg, const int32_t* __restrict__ nbr,
                            const int32_t* __restrict__ nsh, double* __restrict__ coef,
                            int32_t* __restrict__ ecol) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= g.N) return;
    const size_t N = (size_t)g.N;
    const int d = deg[k];
    const double px = xs[k], py = ys[k];
    auto rel = [&](int i, double& rx, double& ry) {
        const int q = nbr[(size_t)k * kCap + i], s = nsh[(size_t)k * kCap + i];
        rx = (xs[q] - px) + shift_x(s) * g.lx;
        ry = (ys[q] - py) + shift_y(s) * g.ly;
    };
    double diag = 0.0;
    if (d > 0) {
        double ax, ay, bx, by;
        rel(d - 1, ax, ay);
        rel(0, bx, by);
        double aprev = 0.5 * (ax * by - ay * bx);   // T_{d-1} = (mu, n_{d-1}, n_0)
        for (int i = 0; i < d; ++i) {
            const int i1 = (i + 1 == d) ? 0 : i + 1;
            double cx_, cy_;
            rel(i1, cx_, cy_);
            const double ai = 0.5 * (bx * cy_ - by * cx_);   // T_i = (mu, n_i, n_{i+1})
            diag += ai;
            coef[N + (size_t)i * N + k] = (aprev + ai) / 12.0;
            ecol[(size_t)i * N + k] = nbr[(size_t)k * kCap + i];
            aprev = ai;
            bx = cx_;
            by = cy_;
        }
    }
    coef[k] = diag / 6.0;
    for (int i = d; i < kCap; ++i) {
        coef[N + (size_t)i * N + k] = 0.0;
        ecol[(size_t)i * N + k] = -1;
    }
}

// consistent mesh mass stencil (Sec. 2.4 on the "/" split): D = hx hy / 2 and
// E = N = NE = hx hy / 12; w = hx hy (its row sums, the FLIP start's volumes)
__global__ void k_x2d_mmesh(int nn, double cm, double* __restrict__ coef, double* __restrict__ w) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= nn) return;
    coef[k] = 0.5 * cm;
    coef[(size_t)nn + k] = cm / 12.0;
    coef[(size_t)2 * nn + k] = cm / 12.0;
    coef[(size_t)3 * nn + k] = cm / 12.0;
    w[k] = cm;
}

// caller-order triangulation (deg, neighbours as caller numbers, shifts)
__global__ void k_x2d_export(Geo g, const int32_t* __restrict__ perm, const int32_t* __restrict__ deg,
                             const int32_t* __restrict__ nbr, const int32_t* __restrict__ nsh,
                             int32_t* __restrict__ deg_out, int32_t* __restrict__ nbr_out,
                             int32_t* __restrict__ sh_out) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= g.N) return;
    const int p = perm[k], d = deg[k];
    deg_out[p] = d;
    for (int i = 0; i < kCap; ++i) {
        nbr_out[(size_t)p * kCap + i] = i < d ? perm[nbr[(size_t)k * kCap + i]] : -1;
        sh_out[(size_t)p * kCap + i] = i < d ? nsh[(size_t)k * kCap + i] : 0;
    }
}

__global__ void k_x2d_clear_export(int np, int32_t* __restrict__ deg_out,
                                   int32_t* __restrict__ nbr_out, int32_t* __restrict__ sh_out) {
    const int p = blockIdx.x * kB + threadIdx.x;
    if (p >= np) return;
    deg_out[p] = 0;
    for (int i = 0; i < kCap; ++i) {
        nbr_out[(size_t)p * kCap + i] = -1;
        sh_out[(size_t)p * kCap + i] = 0;
    }
}

Geo geo_of(const Mesh& m, int N, double lx, double ly) {
    Geo g;
    g.nx = m.nx;
    g.ny = m.ny;
    g.N = N;
    g.lx = lx;
    g.ly = ly;
    g.hx = lx / m.nx;
    g.hy = ly / m.ny;
    g.inv_hx = m.inv_hx;
    g.inv_hy = m.inv_hy;
    // dense particles (six or more per cell) usually close their cells within one
    // ring, sparser ones within two
    g.r0 = (m.nn > 0 && N >= 6 * (long)m.nn) ? 1 : 2;
    return g;
}

}  // namespace

#define X2D_TRY(e)                           \
    do {                                     \
        hipError_t e_ = (e);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

hipError_t x2d_triangulate(const X2dArgs& a, hipStream_t stream) {
    if (a.N == 0) return hipSuccess;
    const Geo g = geo_of(a.m, a.N, a.lx, a.ly);
    hipLaunchKernelGGL(k_x2d_pos, dim3(grid_of(a.N)), dim3(kB), 0, stream, g, a.perm, a.x, a.y,
                       a.values, a.F, a.m.np, a.xs, a.ys, a.cell, a.As);
    X2D_TRY(hipGetLastError());
    // lanes per particle: about 2^19 lanes in flight (what 256 compute units hold),
    // at most 16; with more particles than that a particle has one lane
    int G = 1;
    while (G < 16 && (size_t)a.N * G < ((size_t)1 << 19)) G *= 2;
    if ((size_t)a.N * G > (size_t)INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid(grid_of((size_t)a.N * G));
    switch (G) {
        case 1:
            hipLaunchKernelGGL(k_x2d_star<1>, grid, dim3(kB), 0, stream, g, a.xs, a.ys, a.cell, a.cs,
                               a.deg, a.nbr, a.nsh, a.vol, a.rep);
            break;
        case 2:
            hipLaunchKernelGGL(k_x2d_star<2>, grid, dim3(kB), 0, stream, g, a.xs, a.ys, a.cell, a.cs,
                               a.deg, a.nbr, a.nsh, a.vol, a.rep);
            break;
        case 4:
            hipLaunchKernelGGL(k_x2d_star<4>, grid, dim3(kB), 0, stream, g, a.xs, a.ys, a.cell, a.cs,
                               a.deg, a.nbr, a.nsh, a.vol, a.rep);
            break;
        case 8:
            hipLaunchKernelGGL(k_x2d_star<8>, grid, dim3(kB), 0, stream, g, a.xs, a.ys, a.cell, a.cs,
                               a.deg, a.nbr, a.nsh, a.vol, a.rep);
            break;
        default:
            hipLaunchKernelGGL(k_x2d_star<16>, grid, dim3(kB), 0, stream, g, a.xs, a.ys, a.cell,
                               a.cs, a.deg, a.nbr, a.nsh, a.vol, a.rep);
            break;
    }
    X2D_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_x2d_check, dim3(grid_of(a.N)), dim3(kB), 0, stream, g, a.deg, a.nbr, a.nsh,
                       a.rep);
    return hipGetLastError();
}

hipError_t x2d_export(const X2dArgs& a, int32_t* deg_out, int32_t* nbr_out, int32_t* sh_out,
                      hipStream_t stream) {
    if (a.m.np > 0) {
        hipLaunchKernelGGL(k_x2d_clear_export, dim3(grid_of(a.m.np)), dim3(kB), 0, stream, a.m.np,
                           deg_out, nbr_out, sh_out);
        X2D_TRY(hipGetLastError());
    }
    if (a.N == 0) return hipSuccess;
    const Geo g = geo_of(a.m, a.N, a.lx, a.ly);
    hipLaunchKernelGGL(k_x2d_export, dim3(grid_of(a.N)), dim3(kB), 0, stream, g, a.perm, a.deg,
                       a.nbr, a.nsh, deg_out, nbr_out, sh_out);
    return hipGetLastError();
}

hipError_t x2d_locate(const X2dArgs& a, bool half, double* out, hipStream_t stream) {
    const Geo g = geo_of(a.m, a.N, a.lx, a.ly);
    const int gx = half ? 2 * a.m.nx : a.m.nx, gy = half ? 2 * a.m.ny : a.m.ny;
    const double dx = half ? 0.5 * g.hx : g.hx, dy = half ? 0.5 * g.hy : g.hy;
    hipLaunchKernelGGL(k_x2d_locate, dim3(grid_of((size_t)gx * gy)), dim3(kB), 0, stream, g, gx, gy,
                       dx, dy, a.xs, a.ys, a.cs, a.deg, a.nbr, a.nsh, a.As, a.F, out, a.rep);
    return hipGetLastError();
}

hipError_t x2d_rhs_mesh(const X2dArgs& a, const double* H, double* b, hipStream_t stream) {
    const Geo g = geo_of(a.m, a.N, a.lx, a.ly);
    hipLaunchKernelGGL(k_x2d_rhs_mesh, dim3(grid_of(a.m.nn)), dim3(kB), 0, stream, g, a.F, H, b);
    return hipGetLastError();
}

hipError_t x2d_mass_mesh(const X2dArgs& a, double* coef, double* w, hipStream_t stream) {
    hipLaunchKernelGGL(k_x2d_mmesh, dim3(grid_of(a.m.nn)), dim3(kB), 0, stream, a.m.nn,
                       a.m.cell_measure, coef, w);
    return hipGetLastError();
}

hipError_t x2d_rhs_part(const X2dArgs& a, const double* nodal, double* c, hipStream_t stream) {
    if (a.N == 0) return hipSuccess;
    const Geo g = geo_of(a.m, a.N, a.lx, a.ly);
    hipLaunchKernelGGL(k_x2d_rhs_part, dim3(grid_of(a.N)), dim3(kB), 0, stream, g, a.F, a.xs, a.ys,
                       a.deg, a.nbr, a.nsh, nodal, c);
    return hipGetLastError();
}

hipError_t x2d_mass_part(const X2dArgs& a, double* coef, int32_t* ecol, hipStream_t stream) {
    if (a.N == 0) return hipSuccess;
    const Geo g = geo_of(a.m, a.N, a.lx, a.ly);
    hipLaunchKernelGGL(k_x2d_mpart, dim3(grid_of(a.N)), dim3(kB), 0, stream, g, a.xs, a.ys, a.deg,
                       a.nbr, a.nsh, coef, ecol);
    return hipGetLastError();
}

}  // namespace p2m
