"""Paper-exact 2D assignment methods (Sec. 3.2, Appendix B) on a periodic box.

Test infrastructure only (see the package docstring).

In 2D the particle hats psi_mu are the P1 hats of the periodic Delaunay
triangulation of the particles (Sec. 3.2; eq. (1) with those hats), the mesh hats
psi_i the P1 hats of the "/"-split square mesh.  Everything here is FP64:

* periodic Delaunay: the Delaunay triangulation of the 3 x 3 tiling of the box,
  keeping each triangle that has a vertex in the central tile, named canonically
  (particle ids, integer image shifts relative to the first vertex, counter-
  clockwise) and counted once.
* particle volume v_mu = int psi_mu = sum over incident triangles of |T| / 3
  (eq. (4) in 2D); mesh volume v_i = hx hy (eq. (5)).
* consistent mass matrices m_ab = int psi_a psi_b: on a triangle |T|/6 on the
  diagonal and |T|/12 off it (Sec. 2.4).  The mesh matrix is the 7-point stencil
  hx hy (1/2; 1/12 to the +-x, +-y, +-(x+y) neighbours), solved here by the FFT of
  its symbol; the particle matrix is assembled from the triangles and solved by a
  sparse LU factorisation.
* delta: Abar_i = A(r_i), the particle interpolant at the node (eq. (9)); M2P delta
  is the mesh interpolant at the particle (eq. (10)).
* Appendix-B rule (2D): on every triangle of the target triangulation, Q is the
  quadratic through the source interpolant at the three vertices and the three edge
  midpoints, and int_T Q lambda_a is integrated exactly.  With the P2 basis and
  int lambda_1^a lambda_2^b lambda_3^c = 2|T| a! b! c! / (a+b+c+2)! this is
  |T| (Q_a/30 - (Q_b + Q_c)/60 + 2 (Q_ab + Q_ac)/15 + Q_bc/15).
  P2M integrates A over the mesh triangles, M2P integrates Abar over the particle
  triangles (the same rule applied to the inverse projection, eq. (20)).

Methods (Table 1 rows): delta, FLIP and PIC (Sec. 2.3 with the Delaunay volumes),
mass-delta and full mass, and the two lumped variants.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.spatial import Delaunay

from . import p1


# ----------------------------------------------------------------------------
# periodic Delaunay triangulation of the particles
# ----------------------------------------------------------------------------
def _canonical(ids, sh):
    """Canonical name of one triangle: among its three rotations (orientation kept),
    the smallest tuple (ids, shifts relative to the first vertex)."""
    best = None
    for r in range(3):
        order = [(r + k) % 3 for k in range(3)]
        base = sh[order[0]]
        key = (int(ids[order[0]]), int(ids[order[1]]), int(ids[order[2]]),
               int(sh[order[1]][0] - base[0]), int(sh[order[1]][1] - base[1]),
               int(sh[order[2]][0] - base[0]), int(sh[order[2]][1] - base[1]))
        if best is None or key < best:
            best = key
    return best


def periodic_delaunay(x, y, lx, ly):
    """Periodic Delaunay triangulation of the particles (Sec. 3.2).

    Returns ``tri`` [T, 3] particle ids and ``sh`` [T, 3, 2] integer image shifts
    (vertex a sits at (x + sh[..,0] lx, y + sh[..,1] ly)); every triangle is
    counter-clockwise, named canonically and listed once, sorted by name.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.size
    tiles = [(sx, sy) for sy in (-1, 0, 1) for sx in (-1, 0, 1)]
    px = np.concatenate([x + sx * lx for sx, sy in tiles])
    py = np.concatenate([y + sy * ly for sx, sy in tiles])
    d = Delaunay(np.stack([px, py], axis=1))
    simp = d.simplices
    tile = simp // n
    pid = simp % n
    tsh = np.array(tiles, dtype=np.int64)[tile]           # [T, 3, 2]
    central = (tile == 4).any(axis=1)
    names = set()
    for t in np.nonzero(central)[0]:
        ids = pid[t]
        s = tsh[t]
        pa = np.array([px[simp[t, k]] for k in range(3)])
        pb = np.array([py[simp[t, k]] for k in range(3)])
        cross = (pa[1] - pa[0]) * (pb[2] - pb[0]) - (pb[1] - pb[0]) * (pa[2] - pa[0])
        if cross < 0:
            ids = ids[[0, 2, 1]]
            s = s[[0, 2, 1]]
        names.add(_canonical(ids, s))
    names = sorted(names)
    tri = np.array([k[:3] for k in names], dtype=np.int64).reshape(-1, 3)
    sh = np.zeros((len(names), 3, 2), dtype=np.int64)
    for t, k in enumerate(names):
        sh[t, 1] = k[3:5]
        sh[t, 2] = k[5:7]
    return tri, sh


def local_star(x, y, lx, ly, mu, radius):
    """Delaunay neighbours of particle mu (Sec. 3.2) from the particles within
    ``radius`` of it (every periodic image), counter-clockwise from the nearest one:
    a list of (particle id, sx, sy), or None when the patch is too small to decide
    (some circle through mu and two neighbours reaches beyond the patch: a point
    outside could then lie inside it)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ids, sxs, sys_, px, py = [], [], [], [], []
    for sy in (-1, 0, 1):
        for sx in (-1, 0, 1):
            dx = x + sx * lx - x[mu]
            dy = y + sy * ly - y[mu]
            keep = dx * dx + dy * dy <= radius * radius
            ids.append(np.nonzero(keep)[0])
            sxs.append(np.full(keep.sum(), sx))
            sys_.append(np.full(keep.sum(), sy))
            px.append(dx[keep])
            py.append(dy[keep])
    ids, sxs, sys_ = np.concatenate(ids), np.concatenate(sxs), np.concatenate(sys_)
    pts = np.stack([np.concatenate(px), np.concatenate(py)], axis=1)
    me = np.nonzero((ids == mu) & (sxs == 0) & (sys_ == 0))[0][0]
    d = Delaunay(pts)
    star = set()
    rmax = 0.0
    for t in d.simplices[(d.simplices == me).any(axis=1)]:
        P = pts[t]
        a = P[1] - P[0]
        b = P[2] - P[0]
        den = 2.0 * (a[0] * b[1] - a[1] * b[0])
        ux = (b[1] * (a @ a) - a[1] * (b @ b)) / den
        uy = (a[0] * (b @ b) - b[0] * (a @ a)) / den
        cx, cy = P[0][0] + ux, P[0][1] + uy
        rmax = max(rmax, np.hypot(cx, cy))          # circumradius seen from mu (on the circle)
        star.update(int(v) for v in t if v != me)
    if 2.0 * rmax > radius:
        return None
    star = list(star)
    ang = np.arctan2(pts[star, 1], pts[star, 0])
    order = [star[i] for i in np.argsort(ang)]
    near = min(range(len(order)), key=lambda i: pts[order[i]] @ pts[order[i]])
    order = order[near:] + order[:near]
    return [(int(ids[v]), int(sxs[v]), int(sys_[v])) for v in order]


def local_interpolant(x, y, lx, ly, values, qx, qy, radius):
    """The particle interpolant of eq. (1) at one point (qx, qy) from the Delaunay
    triangulation of the particles within ``radius`` of it (every periodic image), or
    None when the patch is too small to decide (the triangle holding the point has a
    circle reaching beyond the patch, so a point outside could lie inside it)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ids, px, py = [], [], []
    for sy in (-1, 0, 1):
        for sx in (-1, 0, 1):
            dx = x + sx * lx - qx
            dy = y + sy * ly - qy
            keep = dx * dx + dy * dy <= radius * radius
            ids.append(np.nonzero(keep)[0])
            px.append(dx[keep])
            py.append(dy[keep])
    ids = np.concatenate(ids)
    pts = np.stack([np.concatenate(px), np.concatenate(py)], axis=1)
    d = Delaunay(pts)
    s = int(d.find_simplex(np.zeros((1, 2)))[0])
    if s < 0:
        return None
    t = d.simplices[s]
    P = pts[t]
    a = P[1] - P[0]
    b = P[2] - P[0]
    den = 2.0 * (a[0] * b[1] - a[1] * b[0])
    ux = (b[1] * (a @ a) - a[1] * (b @ b)) / den
    uy = (a[0] * (b @ b) - b[0] * (a @ a)) / den
    cx, cy = P[0][0] + ux, P[0][1] + uy
    if np.hypot(cx, cy) + np.hypot(ux, uy) > radius:
        return None
    T = d.transform[s]
    l12 = T[:2, :] @ (np.zeros(2) - T[2, :])
    lam = np.array([l12[0], l12[1], 1.0 - l12.sum()])
    values = np.atleast_2d(np.asarray(values, dtype=np.float64))
    return (values[:, ids[t]] * lam).sum(axis=1)


def triangle_vertices(x, y, lx, ly, tri, sh):
    """Unrolled vertex coordinates [T, 3] (X, Y) of the triangles."""
    X = np.asarray(x, dtype=np.float64)[tri] + sh[..., 0] * lx
    Y = np.asarray(y, dtype=np.float64)[tri] + sh[..., 1] * ly
    return X, Y


def triangle_areas(X, Y):
    return 0.5 * ((X[:, 1] - X[:, 0]) * (Y[:, 2] - Y[:, 0])
                  - (Y[:, 1] - Y[:, 0]) * (X[:, 2] - X[:, 0]))


def particle_volumes(x, y, lx, ly, tri=None, sh=None):
    """v_mu = int psi_mu = sum of |T|/3 over the triangles incident to mu (eq. (4))."""
    if tri is None:
        tri, sh = periodic_delaunay(x, y, lx, ly)
    X, Y = triangle_vertices(x, y, lx, ly, tri, sh)
    a = triangle_areas(X, Y)
    return np.bincount(tri.ravel(), weights=np.repeat(a / 3.0, 3), minlength=len(x))


def particle_mass(x, y, lx, ly, tri, sh):
    """Consistent particle mass matrix m_mu,nu = int psi_mu psi_nu (Sec. 2.4), CSR."""
    X, Y = triangle_vertices(x, y, lx, ly, tri, sh)
    a = triangle_areas(X, Y)
    rows, cols, vals = [], [], []
    for i in range(3):
        for j in range(3):
            rows.append(tri[:, i])
            cols.append(tri[:, j])
            vals.append(a * (2.0 if i == j else 1.0) / 12.0)
    n = len(x)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


# ----------------------------------------------------------------------------
# the particle interpolant A(r) = sum_mu A_mu psi_mu(r) (eq. (1))
# ----------------------------------------------------------------------------
class ParticleInterpolant:
    """Point location in the tiled Delaunay triangulation and barycentric evaluation."""

    def __init__(self, x, y, lx, ly):
        self.x = np.asarray(x, dtype=np.float64)
        self.y = np.asarray(y, dtype=np.float64)
        self.lx, self.ly = float(lx), float(ly)
        n = self.x.size
        tiles = [(sx, sy) for sy in (-1, 0, 1) for sx in (-1, 0, 1)]
        px = np.concatenate([self.x + sx * lx for sx, sy in tiles])
        py = np.concatenate([self.y + sy * ly for sx, sy in tiles])
        self.d = Delaunay(np.stack([px, py], axis=1))
        self.n = n

    def weights(self, qx, qy):
        """Particle ids [3, Q] and barycentric weights [3, Q] of the points (wrapped
        into the box first)."""
        qx = np.mod(np.asarray(qx, dtype=np.float64), self.lx)
        qy = np.mod(np.asarray(qy, dtype=np.float64), self.ly)
        q = np.stack([qx, qy], axis=1)
        s = self.d.find_simplex(q)
        if np.any(s < 0):
            raise ValueError("point outside the tiled triangulation")
        T = self.d.transform[s]
        b = np.einsum("qij,qj->qi", T[:, :2, :], q - T[:, 2, :])
        lam = np.concatenate([b, 1.0 - b.sum(axis=1, keepdims=True)], axis=1)
        ids = self.d.simplices[s] % self.n
        return ids.T, lam.T

    def __call__(self, values, qx, qy):
        values = np.atleast_2d(np.asarray(values, dtype=np.float64))
        ids, lam = self.weights(qx, qy)
        return sum(lam[a] * values[:, ids[a]] for a in range(3))


# ----------------------------------------------------------------------------
# Appendix-B quadrature in 2D
# ----------------------------------------------------------------------------
def appb_triangle(area, qa, qb, qc, qab, qbc, qca):
    """int_T Q lambda_v for the three vertices v = a, b, c of T, where Q is the
    quadratic with vertex values qa, qb, qc and edge-midpoint values qab, qbc, qca
    (Appendix B, 2D)."""
    ta = area * (qa / 30.0 - (qb + qc) / 60.0 + 2.0 * (qab + qca) / 15.0 + qbc / 15.0)
    tb = area * (qb / 30.0 - (qc + qa) / 60.0 + 2.0 * (qbc + qab) / 15.0 + qca / 15.0)
    tc = area * (qc / 30.0 - (qa + qb) / 60.0 + 2.0 * (qca + qbc) / 15.0 + qab / 15.0)
    return ta, tb, tc


def mesh_triangles(nx, ny):
    """The 2 nx ny triangles of the "/"-split mesh as node triples (counter-clockwise)
    and their vertices on the half-spacing grid (I, J) [T, 3] (node (i, j) is
    (2i, 2j)), unwrapped so that midpoints are vertex averages."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    ip, jp = (i + 1) % nx, (j + 1) % ny
    n00, n10, n11, n01 = i + nx * j, ip + nx * j, ip + nx * jp, i + nx * jp
    lo = np.stack([n00, n10, n11], axis=1)
    up = np.stack([n00, n11, n01], axis=1)
    I0, J0 = 2 * i, 2 * j
    loI = np.stack([I0, I0 + 2, I0 + 2], axis=1)
    loJ = np.stack([J0, J0, J0 + 2], axis=1)
    upI = np.stack([I0, I0 + 2, I0], axis=1)
    upJ = np.stack([J0, J0 + 2, J0 + 2], axis=1)
    return (np.concatenate([lo, up]), np.concatenate([loI, upI]), np.concatenate([loJ, upJ]))


def mesh_rhs_appb(interp, values, nx, ny, lx, ly):
    """b_j = int A psi_j over the mesh triangles with the Appendix-B rule, [F, nx ny]."""
    values = np.atleast_2d(np.asarray(values, dtype=np.float64))
    hx, hy = lx / nx, ly / ny
    tri, TI, TJ = mesh_triangles(nx, ny)
    area = 0.5 * hx * hy

    def at(I, J):
        return interp(values, I * (0.5 * hx), J * (0.5 * hy))

    q = [at(TI[:, k], TJ[:, k]) for k in range(3)]
    m = [at((TI[:, k] + TI[:, (k + 1) % 3]) // 2, (TJ[:, k] + TJ[:, (k + 1) % 3]) // 2)
         for k in range(3)]                    # midpoints ab, bc, ca
    ta, tb, tc = appb_triangle(area, q[0], q[1], q[2], m[0], m[1], m[2])
    nn = nx * ny
    out = np.zeros((values.shape[0], nn))
    for f in range(values.shape[0]):
        out[f] = (np.bincount(tri[:, 0], weights=ta[f], minlength=nn)
                  + np.bincount(tri[:, 1], weights=tb[f], minlength=nn)
                  + np.bincount(tri[:, 2], weights=tc[f], minlength=nn))
    return out


def mesh_mass_stencil(nx, ny, lx, ly):
    """Consistent mesh mass matrix (Sec. 2.4) assembled from the element matrices, CSR."""
    hx, hy = lx / nx, ly / ny
    tri, _, _ = mesh_triangles(nx, ny)
    a = np.full(tri.shape[0], 0.5 * hx * hy)
    rows, cols, vals = [], [], []
    for i in range(3):
        for j in range(3):
            rows.append(tri[:, i])
            cols.append(tri[:, j])
            vals.append(a * (2.0 if i == j else 1.0) / 12.0)
    nn = nx * ny
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nn, nn))


def mesh_mass_solve(b, nx, ny, lx, ly):
    """m^-1 b for the consistent mesh mass matrix by the FFT of its symbol
    hx hy [1/2 + (cos tx + cos ty + cos(tx + ty)) / 6] (periodic, circulant)."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    hx, hy = lx / nx, ly / ny
    tx = 2.0 * np.pi * np.fft.fftfreq(nx)[None, :]
    ty = 2.0 * np.pi * np.fft.fftfreq(ny)[:, None]
    sym = hx * hy * (0.5 + (np.cos(tx) + np.cos(ty) + np.cos(tx + ty)) / 6.0)
    out = np.empty_like(b)
    for f in range(b.shape[0]):
        B = np.fft.fft2(b[f].reshape(ny, nx))
        out[f] = np.real(np.fft.ifft2(B / sym)).ravel()
    return out


def particle_rhs_appb(x, y, lx, ly, tri, sh, nodal, nx, ny):
    """c_nu = int Abar psi_nu over the particle triangles with the Appendix-B rule,
    Abar the mesh interpolant of eq. (3); [F, N_p]."""
    nodal = np.atleast_2d(np.asarray(nodal, dtype=np.float64))
    X, Y = triangle_vertices(x, y, lx, ly, tri, sh)
    area = triangle_areas(X, Y)
    prob = dict(dim=2, nx=nx, ny=ny, lx=lx, ly=ly)

    def at(px, py):
        pr = dict(prob, x=np.mod(px, lx), y=np.mod(py, ly))
        return p1.interpolate(pr, nodal)

    q = [at(X[:, k], Y[:, k]) for k in range(3)]
    m = [at(0.5 * (X[:, k] + X[:, (k + 1) % 3]), 0.5 * (Y[:, k] + Y[:, (k + 1) % 3]))
         for k in range(3)]
    ta, tb, tc = appb_triangle(area, q[0], q[1], q[2], m[0], m[1], m[2])
    n = len(x)
    out = np.zeros((nodal.shape[0], n))
    for f in range(nodal.shape[0]):
        out[f] = (np.bincount(tri[:, 0], weights=ta[f], minlength=n)
                  + np.bincount(tri[:, 1], weights=tb[f], minlength=n)
                  + np.bincount(tri[:, 2], weights=tc[f], minlength=n))
    return out


# ----------------------------------------------------------------------------
# Table 1 operators in 2D
# ----------------------------------------------------------------------------
class Paper2D:
    """The particles of one periodic 2D problem with their triangulation."""

    def __init__(self, x, y, nx, ny, lx, ly):
        self.x = np.asarray(x, dtype=np.float64)
        self.y = np.asarray(y, dtype=np.float64)
        self.nx, self.ny, self.lx, self.ly = int(nx), int(ny), float(lx), float(ly)
        self.tri, self.sh = periodic_delaunay(self.x, self.y, lx, ly)
        self.vol = particle_volumes(self.x, self.y, lx, ly, self.tri, self.sh)
        self.interp = ParticleInterpolant(self.x, self.y, lx, ly)
        self._mp_lu = None

    @property
    def prob(self):
        return dict(dim=2, nx=self.nx, ny=self.ny, lx=self.lx, ly=self.ly,
                    x=self.x, y=self.y, vol=self.vol)

    def node_xy(self):
        i, j = np.meshgrid(np.arange(self.nx), np.arange(self.ny), indexing="xy")
        return i.ravel() * (self.lx / self.nx), j.ravel() * (self.ly / self.ny)

    # P2M
    def p2m_delta(self, A):
        """eq. (9): Abar_i = A(r_i)."""
        nx_, ny_ = self.node_xy()
        return self.interp(A, nx_, ny_)

    def p2m_flip(self, A):
        """eqs. (11)-(12) with the Delaunay volumes."""
        return p1.flip(self.prob, np.atleast_2d(A))[0]

    def p2m_pic(self, A):
        """eq. (11) with v_i = hx hy (eq. (5))."""
        return p1.pic(self.prob, np.atleast_2d(A))[0]

    def mesh_rhs(self, A):
        return mesh_rhs_appb(self.interp, A, self.nx, self.ny, self.lx, self.ly)

    def p2m_mass(self, A):
        """Abar = m^-1 int A psi_j (mass-delta and full-mass P2M, Table 1)."""
        return mesh_mass_solve(self.mesh_rhs(A), self.nx, self.ny, self.lx, self.ly)

    def p2m_lumped(self, A):
        """Abar_i = (1 / v_i) int A psi_i (eq. (17), mesh side)."""
        return self.mesh_rhs(A) / ((self.lx / self.nx) * (self.ly / self.ny))

    # M2P
    def m2p_delta(self, nodal):
        """eq. (10): the mesh interpolant at the particles."""
        return p1.interpolate(self.prob, nodal)

    def particle_rhs(self, nodal):
        return particle_rhs_appb(self.x, self.y, self.lx, self.ly, self.tri, self.sh,
                                 nodal, self.nx, self.ny)

    def particle_mass(self):
        return particle_mass(self.x, self.y, self.lx, self.ly, self.tri, self.sh)

    def m2p_mass(self, nodal):
        """eq. (20): m_part Abarbar = int Abar psi_nu (full mass M2P)."""
        if self._mp_lu is None:
            self._mp_lu = spla.splu(self.particle_mass().tocsc())
        c = self.particle_rhs(nodal)
        return np.stack([self._mp_lu.solve(c[f]) for f in range(c.shape[0])])

    def m2p_lumped(self, nodal):
        """Abarbar_nu = (1 / v_nu) int Abar psi_nu (eq. (17), particle side)."""
        return self.particle_rhs(nodal) / self.vol

