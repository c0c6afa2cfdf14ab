// Paper-exact 2D assignment (Sec. 3.2; Appendix B): P1 hats on the periodic
// Delaunay triangulation of the particles, all in FP64.
//
//   k_x2d_pos      binned order: wrapped positions, values and the cell of every
//                  located particle (slot k = position in the binned order)
//   k_x2d_star     per particle, its Voronoi cell by clipping a square with the
//                  bisectors of the particles of the surrounding mesh cells, ring by
//                  ring, until no particle outside the searched rings can cut it
//                  (twice the farthest vertex within the searched radius).  The
//                  bisectors that bound the cell name the Delaunay neighbours,
//                  counter-clockwise; the volume int psi_mu is a third of the area of
//                  the triangles (mu, n_j, n_j+1).
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
constexpr int kCap = P2M_X2D_MAXDEG;   // neighbours per particle, vertices per Voronoi cell
constexpr int kRingMax = 8;            // mesh-cell rings searched around a particle
constexpr int kWalkMax = 1024;         // triangles a point-location walk may visit

inline int grid_of(size_t n) { return (int)((n + kB - 1) / kB); }

struct Geo {
    int nx, ny, N;
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
// Voronoi cell of slot k.  The polygon is kept counter-clockwise around the
// particle in coordinates relative to it; edge i runs from vertex i to vertex
// i + 1 and carries the site whose bisector it lies on (slot, packed image shift;
// -1 for the starting square).
__global__ __launch_bounds__(kB) void k_x2d_star(Geo g, const double* __restrict__ xs,
                                                 const double* __restrict__ ys,
                                                 const int32_t* __restrict__ cell,
                                                 const int32_t* __restrict__ cs,
                                                 int32_t* __restrict__ deg, int32_t* __restrict__ nbr,
                                                 int32_t* __restrict__ nsh, double* __restrict__ vol,
                                                 p2m_report* rep) {
    const int k = blockIdx.x * kB + threadIdx.x;
    if (k >= g.N) return;
    const double px = xs[k], py = ys[k];
    const int c = cell[k];
    const int cy = c / g.nx, cx = c - cy * g.nx;
    const double hmin = g.hx < g.hy ? g.hx : g.hy;
    const double hmax = g.hx < g.hy ? g.hy : g.hx;

    double vx[2][kCap], vy[2][kCap];
    int lq[2][kCap], ls[2][kCap];
    int cur = 0, n = 4;
    const double S = 2.0 * (kRingMax + 1) * hmax;
    vx[0][0] = -S; vy[0][0] = -S;
    vx[0][1] = S;  vy[0][1] = -S;
    vx[0][2] = S;  vy[0][2] = S;
    vx[0][3] = -S; vy[0][3] = S;
    for (int i = 0; i < 4; ++i) {
        lq[0][i] = -1;
        ls[0][i] = 0;
    }
    double rmax2 = 2.0 * S * S;
    bool secure = false, bad = false;

    for (int r = 0; r <= kRingMax && !secure && !bad; ++r) {
        for (int dy = -r; dy <= r && !bad; ++dy) {
            const bool edge_row = (dy == -r || dy == r);
            const int step = edge_row ? 1 : 2 * r;   // interior rows: only the two ends
            for (int dx = -r; dx <= r && !bad; dx += (step > 0 ? step : 1)) {
                const int ax = cx + dx, ay = cy + dy;
                const int sx = floor_div(ax, g.nx), sy = floor_div(ay, g.ny);
                const int cc = (ax - sx * g.nx) + g.nx * (ay - sy * g.ny);
                const int q1 = cs[cc + 1];
                for (int q = cs[cc]; q < q1; ++q) {
                    if (q == k && sx == 0 && sy == 0) continue;
                    const double rx = (xs[q] - px) + sx * g.lx;
                    const double ry = (ys[q] - py) + sy * g.ly;
                    const double d2 = rx * rx + ry * ry;
                    if (!(d2 > 0.0)) {   // two particles at one position
                        bad = true;
                        break;
                    }
                    if (0.25 * d2 >= rmax2) continue;   // its bisector misses the cell
                    // clip by { v : v.r <= |r|^2 / 2 }
                    const double hh = 0.5 * d2;
                    const int nxt = cur ^ 1;
                    int m = 0;
                    double di = vx[cur][0] * rx + vy[cur][0] * ry - hh;
                    for (int i = 0; i < n; ++i) {
                        const int j = (i + 1 == n) ? 0 : i + 1;
                        const double dj = vx[cur][j] * rx + vy[cur][j] * ry - hh;
                        const bool ini = di <= 0.0, inj = dj <= 0.0;
                        if (ini) {
                            if (m >= kCap) {
                                bad = true;
                                break;
                            }
                            vx[nxt][m] = vx[cur][i];
                            vy[nxt][m] = vy[cur][i];
                            lq[nxt][m] = lq[cur][i];
                            ls[nxt][m] = ls[cur][i];
                            ++m;
                        }
                        if (ini != inj) {
                            if (m >= kCap) {
                                bad = true;
                                break;
                            }
                            const double t = di / (di - dj);
                            vx[nxt][m] = vx[cur][i] + t * (vx[cur][j] - vx[cur][i]);
                            vy[nxt][m] = vy[cur][i] + t * (vy[cur][j] - vy[cur][i]);
                            lq[nxt][m] = ini ? q : lq[cur][i];
                            ls[nxt][m] = ini ? pack_shift(sx, sy) : ls[cur][i];
                            ++m;
                        }
                        di = dj;
                    }
                    if (bad) break;
                    cur = nxt;
                    n = m;
                    rmax2 = 0.0;
                    for (int i = 0; i < n; ++i) {
                        const double e = vx[cur][i] * vx[cur][i] + vy[cur][i] * vy[cur][i];
                        rmax2 = e > rmax2 ? e : rmax2;
                    }
                }
                if (step == 0) break;   // r == 0: the one cell
            }
        }
        // every particle not yet seen is at least r hmin away (the rings cover the
        // cells within r of the particle's own); its bisector is then at least
        // r hmin / 2 away and cannot cut a cell whose vertices are all closer
        const double reach = r * hmin * (1.0 - 1e-9);
        if (r >= 1 && 4.0 * rmax2 <= reach * reach) secure = true;
    }
    if (!secure || bad || n < 3) {
        deg[k] = 0;
        vol[k] = __builtin_nan("");
        flag(rep, P2M_FLAG_TRIANGULATION);
        return;
    }
    deg[k] = n;
    double area2 = 0.0;
    double ax0 = 0.0, ay0 = 0.0, fx0 = 0.0, fy0 = 0.0;
    for (int i = 0; i < n; ++i) {
        const int q = lq[cur][i], s = ls[cur][i];
        nbr[(size_t)k * kCap + i] = q;
        nsh[(size_t)k * kCap + i] = s;
        const double rx = (xs[q] - px) + shift_x(s) * g.lx;
        const double ry = (ys[q] - py) + shift_y(s) * g.ly;
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
    for (int i = n; i < kCap; ++i) {
        nbr[(size_t)k * kCap + i] = -1;
        nsh[(size_t)k * kCap + i] = 0;
    }
    vol[k] = area2 / 6.0;   // a third of the triangles' total area (area2 / 2)
}

// position of neighbour entry j of slot u among u's list, or -1
__device__ __forceinline__ int find_entry(const int32_t* __restrict__ nbr,
                                          const int32_t* __restrict__ nsh, int du, int u, int q,
                                          int s) {
    for (int j = 0; j < du; ++j)
        if (nbr[(size_t)u * kCap + j] == q && nsh[(size_t)u * kCap + j] == s) return j;
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

// node values of a half-spacing grid H [F][2ny][2nx] (the delta P2M)
__global__ void k_x2d_nodes(Geo g, int F, const double* __restrict__ H, double* __restrict__ out) {
    const int k = blockIdx.x * kB + threadIdx.x;
    const int nn = g.nx * g.ny;
    if (k >= nn) return;
    const int j = k / g.nx, i = k - j * g.nx;
    const size_t gxy = (size_t)4 * nn;
    for (int f = 0; f < F; ++f)
        out[(size_t)f * nn + k] = H[(size_t)f * gxy + (size_t)(2 * j) * (2 * g.nx) + 2 * i];
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
    hipLaunchKernelGGL(k_x2d_star, dim3(grid_of(a.N)), dim3(kB), 0, stream, g, a.xs, a.ys, a.cell,
                       a.cs, a.deg, a.nbr, a.nsh, a.vol, a.rep);
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

hipError_t x2d_nodes(const X2dArgs& a, const double* H, double* out, hipStream_t stream) {
    const Geo g = geo_of(a.m, a.N, a.lx, a.ly);
    hipLaunchKernelGGL(k_x2d_nodes, dim3(grid_of(a.m.nn)), dim3(kB), 0, stream, g, a.F, H, out);
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
