"""Pins of the paper-exact 2D oracle (Sec. 3.2 particle Delaunay hats, Appendix B 2D
rule, Sec. 2.4 consistent mass matrices) against what geometry and the mathematics
fix: the empty-circumcircle property checked by brute force over every image, the
torus counts, the closed form of a hexagonal lattice, point location by brute force,
the element rule against independent Gauss quadrature of quadratics, constants,
exact nodal sampling, and second-order convergence on a smooth field."""
import numpy as np
import pytest

from oracle import p1
from oracle import paper2d as p2
from paper_1610_05258_amd import workloads as wl


def small_cloud(seed=5, n=6, ppc=2, lx=1.0, ly=0.75):
    x, y = wl.stratified_2d(seed, n, n, ppc, lx, ly)
    return x, y, lx, ly


def test_delaunay_empty_circumcircle_bruteforce():
    x, y, lx, ly = small_cloud()
    tri, sh = p2.periodic_delaunay(x, y, lx, ly)
    X, Y = p2.triangle_vertices(x, y, lx, ly, tri, sh)
    # every image of every particle in the 5 x 5 tiling
    ax = np.concatenate([x + sx * lx for sy in range(-2, 3) for sx in range(-2, 3)])
    ay = np.concatenate([y + sy * ly for sy in range(-2, 3) for sx in range(-2, 3)])
    for t in range(tri.shape[0]):
        (x0, x1, x2), (y0, y1, y2) = X[t], Y[t]
        d = 2.0 * (x0 * (y1 - y2) + x1 * (y2 - y0) + x2 * (y0 - y1))
        ux = ((x0**2 + y0**2) * (y1 - y2) + (x1**2 + y1**2) * (y2 - y0)
              + (x2**2 + y2**2) * (y0 - y1)) / d
        uy = ((x0**2 + y0**2) * (x2 - x1) + (x1**2 + y1**2) * (x0 - x2)
              + (x2**2 + y2**2) * (x1 - x0)) / d
        r2 = (x0 - ux) ** 2 + (y0 - uy) ** 2
        dist2 = (ax - ux) ** 2 + (ay - uy) ** 2
        # the three vertices lie on the circle; nothing lies inside it
        assert np.count_nonzero(dist2 < r2 * (1 - 1e-9)) == 0


def test_delaunay_torus_counts_and_area():
    x, y, lx, ly = small_cloud(seed=7, n=8, ppc=3)
    tri, sh = p2.periodic_delaunay(x, y, lx, ly)
    n = x.size
    assert tri.shape[0] == 2 * n                      # V - E + F = 0 on the torus
    X, Y = p2.triangle_vertices(x, y, lx, ly, tri, sh)
    a = p2.triangle_areas(X, Y)
    assert np.all(a > 0)
    assert abs(a.sum() - lx * ly) <= 1e-13 * lx * ly
    # every directed edge (with its relative shift) appears once, and its reverse once
    edges = {}
    for t in range(tri.shape[0]):
        for k in range(3):
            a0, a1 = k, (k + 1) % 3
            key = (tri[t, a0], tri[t, a1], *(sh[t, a1] - sh[t, a0]))
            edges[key] = edges.get(key, 0) + 1
    assert all(c == 1 for c in edges.values())
    for (i, j, dx, dy) in edges:
        assert (j, i, -dx, -dy) in edges
    v = p2.particle_volumes(x, y, lx, ly, tri, sh)
    assert abs(v.sum() - lx * ly) <= 1e-13 * lx * ly


def hex_lattice(nx=6, ny=4, a=0.5):
    j, i = np.divmod(np.arange(nx * ny), nx)
    x = (i + 0.5 * (j % 2)) * a
    y = j * a * np.sqrt(3.0) / 2.0
    return x, y, nx * a, ny * a * np.sqrt(3.0) / 2.0


def test_hexagonal_lattice_closed_form():
    x, y, lx, ly = hex_lattice()
    a = 0.5
    tri, sh = p2.periodic_delaunay(x, y, lx, ly)
    area = np.sqrt(3.0) / 4.0 * a * a
    X, Y = p2.triangle_vertices(x, y, lx, ly, tri, sh)
    np.testing.assert_allclose(p2.triangle_areas(X, Y), area, rtol=1e-12)
    v = p2.particle_volumes(x, y, lx, ly, tri, sh)
    np.testing.assert_allclose(v, 6 * area / 3.0, rtol=1e-12)   # the hexagon's area
    M = p2.particle_mass(x, y, lx, ly, tri, sh).toarray()
    np.testing.assert_allclose(np.diag(M), area, rtol=1e-12)      # 6 |T| / 6
    off = M - np.diag(np.diag(M))
    assert np.all(np.count_nonzero(off > 0, axis=1) == 6)
    np.testing.assert_allclose(off[off > 0], area / 6.0, rtol=1e-12)  # 2 |T| / 12
    np.testing.assert_allclose(M.sum(axis=1), v, rtol=1e-12)


def test_interpolant_against_bruteforce_location():
    x, y, lx, ly = small_cloud(seed=9, n=5, ppc=2)
    tri, sh = p2.periodic_delaunay(x, y, lx, ly)
    X, Y = p2.triangle_vertices(x, y, lx, ly, tri, sh)
    interp = p2.ParticleInterpolant(x, y, lx, ly)
    g = np.random.Generator(np.random.PCG64(1))
    A = g.standard_normal(x.size)
    qx = g.uniform(0, lx, 300)
    qy = g.uniform(0, ly, 300)
    got = interp(A, qx, qy)[0]
    for q in range(qx.size):
        found = None
        for t in range(tri.shape[0]):
            for sx in (-1, 0, 1):
                for sy in (-1, 0, 1):
                    px_ = X[t] + sx * lx
                    py_ = Y[t] + sy * ly
                    det = (px_[1] - px_[0]) * (py_[2] - py_[0]) - (py_[1] - py_[0]) * (px_[2] - px_[0])
                    l1 = ((qx[q] - px_[0]) * (py_[2] - py_[0]) - (qy[q] - py_[0]) * (px_[2] - px_[0])) / det
                    l2 = ((px_[1] - px_[0]) * (qy[q] - py_[0]) - (py_[1] - py_[0]) * (qx[q] - px_[0])) / det
                    l0 = 1 - l1 - l2
                    if min(l0, l1, l2) >= -1e-12:
                        found = l0 * A[tri[t, 0]] + l1 * A[tri[t, 1]] + l2 * A[tri[t, 2]]
        assert found is not None
        assert abs(found - got[q]) <= 1e-12 * max(1.0, abs(found))


def gauss_triangle(f, X, Y, order=6):
    """Integral of f over the triangle by the collapsed (Duffy) tensor Gauss rule,
    exact for polynomials of degree <= 2 order - 2."""
    u, wu = np.polynomial.legendre.leggauss(order)
    u = 0.5 * (u + 1)
    wu = 0.5 * wu
    s, t = np.meshgrid(u, u, indexing="ij")
    w = np.outer(wu, wu)
    l1 = s
    l2 = (1 - s) * t
    jac = (1 - s)
    l0 = 1 - l1 - l2
    px_ = l0 * X[0] + l1 * X[1] + l2 * X[2]
    py_ = l0 * Y[0] + l1 * Y[1] + l2 * Y[2]
    area2 = abs((X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]))
    return np.sum(w * jac * f(px_, py_, l0, l1, l2)) * area2


@pytest.mark.parametrize("seed", range(6))
def test_appb_rule_exact_on_quadratics(seed):
    g = np.random.Generator(np.random.PCG64(100 + seed))
    X = g.uniform(-1, 1, 3)
    Y = g.uniform(-1, 1, 3)
    if (X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]) < 0:
        X[[1, 2]] = X[[2, 1]]
        Y[[1, 2]] = Y[[2, 1]]
    c = g.standard_normal(6)

    def q(px_, py_):
        return c[0] + c[1] * px_ + c[2] * py_ + c[3] * px_ * px_ + c[4] * px_ * py_ + c[5] * py_ * py_

    area = 0.5 * ((X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]))
    mids = [(0.5 * (X[k] + X[(k + 1) % 3]), 0.5 * (Y[k] + Y[(k + 1) % 3])) for k in range(3)]
    got = p2.appb_triangle(area, q(X[0], Y[0]), q(X[1], Y[1]), q(X[2], Y[2]),
                           q(*mids[0]), q(*mids[1]), q(*mids[2]))
    for a in range(3):
        ref = gauss_triangle(lambda px_, py_, l0, l1, l2: q(px_, py_) * (l0, l1, l2)[a], X, Y)
        assert abs(got[a] - ref) <= 1e-13 * max(1.0, abs(ref))


def test_mesh_mass_fft_matches_element_assembly():
    nx, ny, lx, ly = 12, 8, 1.5, 1.0
    M = p2.mesh_mass_stencil(nx, ny, lx, ly)
    np.testing.assert_allclose(np.asarray(M.sum(axis=1)).ravel(), (lx / nx) * (ly / ny), rtol=1e-13)
    g = np.random.Generator(np.random.PCG64(2))
    b = g.standard_normal((2, nx * ny))
    x = p2.mesh_mass_solve(b, nx, ny, lx, ly)
    np.testing.assert_allclose(M @ x[0], b[0], atol=1e-12)
    np.testing.assert_allclose(M @ x[1], b[1], atol=1e-12)
    ev = np.linalg.eigvalsh(M.toarray()) / ((lx / nx) * (ly / ny))
    assert ev.min() > 0.25 - 1e-12 and ev.max() <= 1.0 + 1e-12


def test_constants_reproduced_by_every_kind():
    x, y = wl.stratified_2d(11, 8, 8, 4, 1.0, 1.0)
    P = p2.Paper2D(x, y, 8, 8, 1.0, 1.0)
    A = np.full((1, x.size), 2.5)
    for op in (P.p2m_delta, P.p2m_flip, P.p2m_mass, P.p2m_lumped):   # not PIC (eq. (11) with v_i = h^2)
        np.testing.assert_allclose(op(A), 2.5, rtol=1e-12, err_msg=op.__name__)
    nodal = np.full((1, 64), -1.25)
    for op in (P.m2p_delta, P.m2p_mass, P.m2p_lumped):
        np.testing.assert_allclose(op(nodal), -1.25, rtol=1e-12, err_msg=op.__name__)


def test_delta_samples_particles_at_nodes():
    """A node that carries a particle takes that particle's value (lambda = (1, 0, 0))."""
    nx = ny = 6
    lx = ly = 1.0
    xs, ys = wl.stratified_2d(12, nx, ny, 2, lx, ly)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x = np.concatenate([i.ravel() * lx / nx, xs])
    y = np.concatenate([j.ravel() * ly / ny, ys])
    P = p2.Paper2D(x, y, nx, ny, lx, ly)
    A = np.random.Generator(np.random.PCG64(3)).standard_normal((1, x.size))
    np.testing.assert_allclose(P.p2m_delta(A)[0], A[0, :nx * ny], rtol=1e-12, atol=1e-13)


def smooth(x, y, L):
    return np.sin(2 * np.pi * x / L) * np.cos(2 * np.pi * y / L) + 0.5 * np.cos(4 * np.pi * y / L)


def test_second_order_convergence():
    """Mass P2M and full-mass M2P of a smooth field converge at second order: halving
    the spacing of mesh and particles divides the nodal error by about four.  A dropped
    or misweighted term of the Appendix-B rule or of a mass matrix breaks this."""
    L = 1.0
    err_p2m, err_m2p = [], []
    for n in (16, 32, 64):
        x, y = wl.stratified_2d(13, n, n, 4, L, L)
        P = p2.Paper2D(x, y, n, n, L, L)
        nxg, nyg = P.node_xy()
        A = smooth(x, y, L)[None]
        err_p2m.append(np.abs(P.p2m_mass(A)[0] - smooth(nxg, nyg, L)).max())
        nodal = smooth(nxg, nyg, L)[None]
        err_m2p.append(np.abs(P.m2p_mass(nodal)[0] - smooth(x, y, L)).max())
    for e in (err_p2m, err_m2p):
        assert e[0] / e[1] > 3.0 and e[1] / e[2] > 3.0, e


def test_conservation_and_flip_volumes():
    """Full mass conserves against the volumes (1^T m = v^T on both sides, Sec. 2.4),
    and FLIP with the Delaunay volumes is eq. (11)-(12) of the existing oracle."""
    x, y = wl.stratified_2d(14, 10, 10, 3, 2.0, 1.0)
    P = p2.Paper2D(x, y, 10, 10, 2.0, 1.0)
    g = np.random.Generator(np.random.PCG64(4))
    A = g.standard_normal((2, x.size))
    Ab = P.p2m_mass(A)
    b = P.mesh_rhs(A)
    np.testing.assert_allclose(Ab.sum(axis=1) * (0.2 * 0.1), b.sum(axis=1), rtol=1e-11)
    nodal = g.standard_normal((1, 100))
    Abb = P.m2p_mass(nodal)
    np.testing.assert_allclose((Abb * P.vol).sum(axis=1), P.particle_rhs(nodal).sum(axis=1),
                               rtol=1e-11)
    np.testing.assert_allclose(P.p2m_flip(A), p1.flip(dict(P.prob), A)[0], rtol=1e-13)


def test_local_star_matches_periodic_triangulation():
    """The one-particle patch form gives each particle's neighbours of the full
    periodic triangulation (in counter-clockwise order)."""
    x, y = wl.stratified_2d(15, 10, 10, 3, 1.0, 1.0)
    tri, sh = p2.periodic_delaunay(x, y, 1.0, 1.0)
    for mu in range(0, x.size, 7):
        star = p2.local_star(x, y, 1.0, 1.0, mu, 0.45)
        assert star is not None
        want = set()
        for t in range(tri.shape[0]):
            for a in range(3):
                if tri[t, a] == mu:
                    for b in range(3):
                        if b != a:
                            want.add((int(tri[t, b]), *(int(v) for v in sh[t, b] - sh[t, a])))
        assert set(star) == want
        # counter-clockwise: consecutive neighbours turn left around mu
        for (i0, sx0, sy0), (i1, sx1, sy1) in zip(star, star[1:] + star[:1]):
            ax, ay = x[i0] + sx0 - x[mu], y[i0] + sy0 - y[mu]
            bx, by = x[i1] + sx1 - x[mu], y[i1] + sy1 - y[mu]
            assert ax * by - ay * bx > 0


def test_local_interpolant_matches_full_interpolant():
    """The one-point patch form gives the full periodic interpolant's value."""
    x, y = wl.stratified_2d(16, 12, 12, 2, 1.0, 1.0)
    interp = p2.ParticleInterpolant(x, y, 1.0, 1.0)
    g = np.random.Generator(np.random.PCG64(5))
    A = g.standard_normal((2, x.size))
    qx = g.uniform(0, 1.0, 40)
    qy = g.uniform(0, 1.0, 40)
    full = interp(A, qx, qy)
    for q in range(qx.size):
        v = p2.local_interpolant(x, y, 1.0, 1.0, A, qx[q], qy[q], 0.4)
        assert v is not None
        np.testing.assert_allclose(v, full[:, q], rtol=1e-12, atol=1e-13)
