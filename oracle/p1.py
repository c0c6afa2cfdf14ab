"""FP64 oracle of the particle<->mesh assignment as the GPU path computes it.

Test infrastructure only (see the package docstring): nothing in the product
imports this module.

The mesh is a periodic structured P1 mesh: ``n`` nodes per axis on ``[0, L)``,
node ``i`` at ``i*h`` with ``h = L/n``.  In 2D, node ``k = i + nx*j`` and every
square cell is split by its "/" diagonal (lower-left to upper-right node) into two
right triangles.  The mesh hats psi_i are the P1 functions that are 1 at their
node and fall linearly to 0 at the neighbouring nodes (Sec. 2, eq. (3); Sec. 3.1
and Sec. 3.2 describe the same linear hats).

Reading of the integrals (the method's central reading).  The paper reconstructs
the particle field with hats psi_mu on a Delaunay triangulation of the particles
(Sec. 2, eq. (1); Sec. 3.2), which this path does not build.  Every integral over
the domain is instead evaluated with the paper's own particle quadrature,
int f = sum_mu v_mu f(r_mu), the identity it uses for int A (Sec. 2.1) and for the
FLIP volume (Sec. 2.3, eq. (12)).  Hence

    b_i   = sum_mu v_mu A_mu psi_i(r_mu)                (right-hand side)
    w_i   = sum_mu v_mu psi_i(r_mu)                     (FLIP volume, eq. (12))
    M_ij  = sum_mu v_mu psi_i(r_mu) psi_j(r_mu)         (mass matrix m_ij, Sec. 2.4)

and the mass assignment (eqs. (13), (19): Abar = m^{-1} int A psi) solves
M Abar = b.  Under this inner product the preservation property (eq. (18)) holds
exactly, and FLIP is the row-sum lumping of the same system.

Other readings used here:
* locate: t = x * (n/L) in FP64 with n/L one FP64 division; c = floor(t),
  xi = t - c (exact); c == n wraps to cell 0; a position is valid iff t is finite
  and 0 <= t < n + 1.  Invalid particles are excluded and flagged.
* 2D triangle choice: xi >= eta is the lower triangle (n00, n10, n11) with
  barycentrics (1-xi, xi-eta, eta); otherwise the upper triangle (n00, n11, n01)
  with (1-eta, xi, eta-xi).
* orphan nodes (w_i == 0 exactly; "a node may even have a vanishing volume",
  Sec. 2.3) get Abar_i = 0; in the mass system their row and column are replaced
  by the identity with b_i = 0.
* particle volumes: an input array, or NULL meaning uniform area/N_p.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Report flag bits of the method (the numbers are part of the public contract).
FLAG_ORPHAN = 1 << 0
FLAG_RANGE = 1 << 3
FLAG_NONFINITE = 1 << 4


# ----------------------------------------------------------------------------
# locate (P1 element of a particle) and the P1 weights psi_i(r_mu)
# ----------------------------------------------------------------------------
def locate_axis(x, n, length):
    """Cell index and local offset along one axis.

    Returns (c, xi, valid, finite): c int64 cell in [0, n), xi in [0, 1) FP64.
    Follows the locate reading stated in the module docstring; the element that
    contains r_mu is what psi_i(r_mu) of eq. (3) needs.
    """
    x = np.asarray(x, dtype=np.float64)
    inv = np.float64(n) / np.float64(length)
    t = x * inv
    finite = np.isfinite(t)
    t0 = np.where(finite, t, 0.0)
    valid = finite & (t0 >= 0.0) & (t0 < n + 1)
    t0 = np.where(valid, t0, 0.0)
    cf = np.floor(t0)
    xi = t0 - cf
    c = cf.astype(np.int64)
    c = np.where(c == n, 0, c)
    return c, xi, valid, finite


def locate_1d(x, n, length):
    """1D locate: nodes (c, c+1 mod n) with P1 weights (1-xi, xi) (Sec. 3.1 hats)."""
    c, xi, valid, finite = locate_axis(x, n, length)
    nodes = np.stack([c, (c + 1) % n])
    lam = np.stack([1.0 - xi, xi])
    return dict(key=c, xi=xi, nodes=nodes, lam=lam, valid=valid, finite=finite)


def locate_2d(x, y, nx, ny, lx, ly):
    """2D locate on the "/"-split square mesh (Sec. 3.2 hats, split reading above).

    Returns nodes[3, N] and lam[3, N] with nodes[0] always the cell's lower-left
    node n00, and the cell key cx + nx*cy.
    """
    cx, xi, vx, fx = locate_axis(x, nx, lx)
    cy, eta, vy, fy = locate_axis(y, ny, ly)
    i1 = (cx + 1) % nx
    j1 = (cy + 1) % ny
    n00 = cx + nx * cy
    n10 = i1 + nx * cy
    n11 = i1 + nx * j1
    n01 = cx + nx * j1
    lower = xi >= eta
    nodes = np.stack([n00, np.where(lower, n10, n11), np.where(lower, n11, n01)])
    lam = np.stack([
        np.where(lower, 1.0 - xi, 1.0 - eta),
        np.where(lower, xi - eta, xi),
        np.where(lower, eta, eta - xi),
    ])
    return dict(key=n00, cx=cx, cy=cy, xi=xi, eta=eta, nodes=nodes, lam=lam,
                valid=vx & vy, finite=fx & fy)


def locate(prob):
    """Dispatch on the problem dimension. ``prob`` is a dict with dim, nx, ny, lx, ly, x, y."""
    if prob["dim"] == 1:
        return locate_1d(prob["x"], prob["nx"], prob["lx"])
    return locate_2d(prob["x"], prob["y"], prob["nx"], prob["ny"], prob["lx"], prob["ly"])


def n_nodes(prob):
    return prob["nx"] * (prob["ny"] if prob["dim"] == 2 else 1)


def cell_measure(prob):
    """Mesh volume v_i = int psi_i (eq. (5)) of every node of the uniform mesh: h (1D), hx*hy (2D)."""
    if prob["dim"] == 1:
        return prob["lx"] / prob["nx"]
    return (prob["lx"] / prob["nx"]) * (prob["ly"] / prob["ny"])


def particle_volumes(prob, n_particles):
    """v_mu of eq. (4): the given array, or uniform domain measure / N_p when absent."""
    v = prob.get("vol")
    if v is not None:
        return np.asarray(v, dtype=np.float64)
    area = prob["lx"] * (prob["ly"] if prob["dim"] == 2 else 1.0)
    return np.full(n_particles, area / n_particles)


# ----------------------------------------------------------------------------
# binning: stable counting sort of particles by cell
# ----------------------------------------------------------------------------
def bin_particles(key, valid, n_cells):
    """Stable sort of the valid particles by cell key.

    perm[k] is the original index of the k-th particle in (cell, original index)
    order; invalid particles are left out and the tail of perm is -1.
    cell_start is the exclusive prefix sum of the per-cell counts (length n_cells+1).
    Not a step of the paper (its triangulation library located particles); this
    is the locality device of the GPU path, defined as a plain stable sort.
    """
    key = np.asarray(key, dtype=np.int64)
    idx = np.flatnonzero(valid)
    order = np.argsort(key[idx], kind="stable")
    perm = np.full(key.shape[0], -1, dtype=np.int64)
    perm[: idx.size] = idx[order]
    counts = np.bincount(key[idx], minlength=n_cells)
    cell_start = np.zeros(n_cells + 1, dtype=np.int64)
    cell_start[1:] = np.cumsum(counts)
    return perm, cell_start


# ----------------------------------------------------------------------------
# scatter: b, w and the particle-quadrature mass matrix
# ----------------------------------------------------------------------------
def assemble(prob, values, want_matrix=True):
    """Scatter of one problem.

    b[f, i] = sum_mu v_mu A_f,mu psi_i(r_mu)     (numerator of eq. (11))
    w[i]    = sum_mu v_mu psi_i(r_mu)            (FLIP volume, eq. (12))
    M       = sum_mu v_mu psi_i(r_mu) psi_j(r_mu) (m_ij of Sec. 2.4 under particle quadrature)

    ``values`` is [F, N_p].  Invalid particles contribute nothing.
    Returns dict(b, w, M (scipy CSR or None), loc, v, flags).
    """
    values = np.atleast_2d(np.asarray(values, dtype=np.float64))
    loc = locate(prob)
    nn = n_nodes(prob)
    npart = values.shape[1]
    v = particle_volumes(prob, npart)
    ok = loc["valid"]
    nodes = loc["nodes"][:, ok]
    lam = loc["lam"][:, ok]
    vv = v[ok]
    k = nodes.shape[0]
    b = np.zeros((values.shape[0], nn))
    for f in range(values.shape[0]):
        af = values[f, ok]
        for a in range(k):
            b[f] += np.bincount(nodes[a], weights=vv * af * lam[a], minlength=nn)
    w = np.zeros(nn)
    for a in range(k):
        w += np.bincount(nodes[a], weights=vv * lam[a], minlength=nn)
    M = None
    if want_matrix:
        rows, cols, vals = [], [], []
        for a in range(k):
            for c in range(k):
                rows.append(nodes[a])
                cols.append(nodes[c])
                vals.append(vv * lam[a] * lam[c])
        M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nn, nn)).tocsr()
        M.sum_duplicates()
    flags = 0
    if not np.all(loc["finite"]):
        flags |= FLAG_NONFINITE
    if not np.all(loc["valid"] | ~loc["finite"]):
        flags |= FLAG_RANGE
    if np.any(w == 0.0):
        flags |= FLAG_ORPHAN
    return dict(b=b, w=w, M=M, loc=loc, v=v, flags=flags)


def stencil_coefficients(prob, M):
    """Read the symmetric stencil storage out of the CSR matrix.

    2D: D_k = M[k,k], E_k = M[k, k+x], N_k = M[k, k+y], NE_k = M[k, k+x+y]
    1D: D_k, E_k = M[k, k+1].  Only meaningful for n >= 3 per axis (for n == 2 the
    periodic neighbours coincide and the stencil splits one matrix entry in two).
    """
    M = M.tocsr()
    nx = prob["nx"]
    if prob["dim"] == 1:
        k = np.arange(nx)
        return dict(D=np.asarray(M[k, k]).ravel(), E=np.asarray(M[k, (k + 1) % nx]).ravel())
    ny = prob["ny"]
    j, i = np.divmod(np.arange(nx * ny), nx)
    kx = (i + 1) % nx + nx * j
    ky = i + nx * ((j + 1) % ny)
    kxy = (i + 1) % nx + nx * ((j + 1) % ny)
    k = np.arange(nx * ny)
    return dict(D=np.asarray(M[k, k]).ravel(), E=np.asarray(M[k, kx]).ravel(),
                N=np.asarray(M[k, ky]).ravel(), NE=np.asarray(M[k, kxy]).ravel())


# ----------------------------------------------------------------------------
# particle -> mesh: FLIP and PIC
# ----------------------------------------------------------------------------
def flip(prob, values):
    """FLIP assignment, Sec. 2.3 eqs. (11)-(12), Table 1: Abar_i = b_i / w_i; orphans -> 0."""
    a = assemble(prob, values, want_matrix=False)
    w = a["w"]
    out = np.where(w > 0.0, a["b"] / np.where(w > 0.0, w, 1.0), 0.0)
    return out, a


def pic(prob, values):
    """PIC assignment, Sec. 2.3 eq. (11) with the mesh volume of eq. (5): Abar_i = b_i / v_i."""
    a = assemble(prob, values, want_matrix=False)
    return a["b"] / cell_measure(prob), a


# ----------------------------------------------------------------------------
# particle -> mesh: mass assignment
# ----------------------------------------------------------------------------
def regularised_matrix(M, w):
    """M with orphan rows/columns (w_i == 0, hence all-zero) replaced by the identity."""
    orphan = (w == 0.0).astype(np.float64)
    return (M + sp.diags(orphan)).tocsr()


def cg_fp64(A, b, x0=None, rtol=1e-14, maxit=10000):
    """Textbook conjugate gradients in FP64 (Hestenes-Stiefel), stop at ||r|| <= rtol*||b||.

    The paper solves its mass systems with library solvers (Appendix A); any exact
    SPD solver computes the same Abar, and CG is used above the direct-solve size.
    """
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    r = b - A @ x
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0
    p = r.copy()
    rr = r @ r
    for it in range(maxit):
        if np.sqrt(rr) <= rtol * bn:
            return x, it
        q = A @ p
        alpha = rr / (p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxit


def pcg_jacobi_fp64(A, b, x0=None, rtol=1e-14, maxit=10000):
    """Textbook preconditioned CG in FP64 with the diagonal (Jacobi) preconditioner
    u = r / diag(A); stop at the unpreconditioned ||r|| <= rtol*||b||.  Same solution
    as cg_fp64 (the iteration, not the system, changes); with a unit diagonal the
    iterates are those of cg_fp64.  Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    dinv = 1.0 / A.diagonal()
    r = b - A @ x
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0
    u = dinv * r
    p = u.copy()
    ru = r @ u
    for it in range(maxit):
        if np.linalg.norm(r) <= rtol * bn:
            return x, it
        q = A @ p
        alpha = ru / (p @ q)
        x += alpha * p
        r -= alpha * q
        u = dinv * r
        ru_new = r @ u
        p = u + (ru_new / ru) * p
        ru = ru_new
    return x, maxit


def mass_solve(M, w, b, solver="auto", rtol=1e-14):
    """Solve M Abar_f = b_f for every field (Sec. 2.4 eqs. (13), (19); Table 1, mass rows)."""
    A = regularised_matrix(M, w)
    b = np.atleast_2d(b)
    nn = A.shape[0]
    if solver == "auto":
        solver = "direct" if nn <= 65536 else "cg"
    out = np.zeros_like(b)
    if solver == "dense":
        Ad = A.toarray()
        for f in range(b.shape[0]):
            out[f] = np.linalg.solve(Ad, b[f])
    elif solver == "direct":
        lu = spla.splu(A.tocsc())
        for f in range(b.shape[0]):
            out[f] = lu.solve(b[f])
    elif solver == "cg":
        for f in range(b.shape[0]):
            out[f], _ = cg_fp64(A, b[f], rtol=rtol)
    else:
        raise ValueError(solver)
    return out


def mass_assign(prob, values, solver="auto"):
    """Mass P2M of one problem (Table 1, mass-delta / full mass P2M column)."""
    a = assemble(prob, values, want_matrix=True)
    return mass_solve(a["M"], a["w"], a["b"], solver=solver), a


def relative_residual(M, w, b, x):
    """||b - M x||_2 / ||b||_2 per field with the regularised M (0 when b == 0 and x == 0)."""
    A = regularised_matrix(M, w)
    b = np.atleast_2d(b)
    x = np.atleast_2d(x)
    out = np.zeros(b.shape[0])
    for f in range(b.shape[0]):
        bn = np.linalg.norm(b[f])
        rn = np.linalg.norm(b[f] - A @ x[f])
        out[f] = rn / bn if bn > 0 else rn
    return out


# ----------------------------------------------------------------------------
# mesh -> particle: interpolation
# ----------------------------------------------------------------------------
def interpolate(prob, nodal):
    """Mesh->particle, Sec. 2.2 eq. (10) (read at r_mu): Abarbar_mu = sum_i Abar_i psi_i(r_mu).

    ``nodal`` is [F, N_n]; the result is [F, N_p] in the caller's particle order.
    Invalid particles get NaN.
    """
    nodal = np.atleast_2d(np.asarray(nodal, dtype=np.float64))
    loc = locate(prob)
    out = np.zeros((nodal.shape[0], loc["nodes"].shape[1]))
    for a in range(loc["nodes"].shape[0]):
        out += loc["lam"][a] * nodal[:, loc["nodes"][a]]
    out[:, ~loc["valid"]] = np.nan
    return out


# ----------------------------------------------------------------------------
# 1D delta assignment
# ----------------------------------------------------------------------------
def delta_1d(prob, values):
    """1D delta P2M, Sec. 2.2 eq. (9): Abar_i = sum_mu A_mu psi_mu(x_i).

    In 1D the particle hats are the P1 hats on the particles sorted along the
    periodic axis, so the particle interpolant at node x_i is the linear
    interpolation between the two consecutive particles that bracket it.
    Reading: positions are compared in the cell coordinate s = c + xi of the locate
    step (so a node and a particle coincide exactly when xi == 0); particles are
    ordered by (s, original index); a = the last particle with s_a <= i, b = the one
    after a (cyclically); with da = (i - s_a) mod n and db = (s_b - i) mod n
    (db = n when b is a), Abar_i = A_a + (A_b - A_a) * da / (da + db).
    """
    values = np.atleast_2d(np.asarray(values, dtype=np.float64))
    n = prob["nx"]
    loc = locate_1d(prob["x"], n, prob["lx"])
    ok = np.flatnonzero(loc["valid"])
    s = loc["key"][ok].astype(np.float64) + loc["xi"][ok]
    order = np.lexsort((ok, s))          # primary s, secondary original index
    s_sorted = s[order]
    idx_sorted = ok[order]
    m = s_sorted.size
    out = np.zeros((values.shape[0], n))
    if m == 0:
        return out
    for i in range(n):
        # last position with s <= i
        pos = np.searchsorted(s_sorted, float(i), side="right") - 1
        ia = pos % m                       # pos == -1 wraps to the last particle
        ib = (ia + 1) % m
        da = (float(i) - s_sorted[ia]) % n
        if m == 1:
            db = n - da
        else:
            db = (s_sorted[ib] - float(i)) % n
            if db == 0.0:
                db = float(n)
        A_a = values[:, idx_sorted[ia]]
        A_b = values[:, idx_sorted[ib]]
        out[:, i] = A_a + (A_b - A_a) * (da / (da + db))
    return out


def assemble_stencil(prob, values):
    """The same scatter as ``assemble`` but accumulating the mass matrix directly
    in its symmetric stencil storage with bincount (no sparse matrix), for large
    problems.  2D: D, E = M(k,k+x), N = M(k,k+y), NE = M(k,k+x+y) as the pairs of
    corners each particle's triangle touches; 1D: D, E = M(k,k+1).
    Valid for n >= 3 per axis (for n == 2 a periodic neighbour pair is stored
    twice and the split between the two slots differs from ``stencil_coefficients``).
    """
    values = np.atleast_2d(np.asarray(values, dtype=np.float64))
    loc = locate(prob)
    nn = n_nodes(prob)
    npart = values.shape[1]
    v = particle_volumes(prob, npart)
    ok = loc["valid"]
    vv = v[ok]
    out = {}
    if prob["dim"] == 1:
        c = loc["key"][ok]
        c1 = (c + 1) % prob["nx"]
        l0, l1 = loc["lam"][0][ok], loc["lam"][1][ok]
        out["D"] = np.bincount(c, vv * l0 * l0, nn) + np.bincount(c1, vv * l1 * l1, nn)
        out["E"] = np.bincount(c, vv * l0 * l1, nn)
        out["w"] = np.bincount(c, vv * l0, nn) + np.bincount(c1, vv * l1, nn)
        out["b"] = np.stack([np.bincount(c, vv * values[f, ok] * l0, nn) +
                             np.bincount(c1, vv * values[f, ok] * l1, nn)
                             for f in range(values.shape[0])])
        return out
    nx, ny = prob["nx"], prob["ny"]
    cx, cy = loc["cx"][ok], loc["cy"][ok]
    xi, eta = loc["xi"][ok], loc["eta"][ok]
    lower = xi >= eta
    i1, j1 = (cx + 1) % nx, (cy + 1) % ny
    n00, n10, n11, n01 = cx + nx * cy, i1 + nx * cy, i1 + nx * j1, cx + nx * j1
    # corner weights (0 for the corner outside the particle's triangle)
    w00 = np.where(lower, 1.0 - xi, 1.0 - eta)
    w10 = np.where(lower, xi - eta, 0.0)
    w11 = np.where(lower, eta, xi)
    w01 = np.where(lower, 0.0, eta - xi)
    bc = lambda idx, wt: np.bincount(idx, wt, nn)
    out["D"] = bc(n00, vv * w00 * w00) + bc(n10, vv * w10 * w10) + bc(n11, vv * w11 * w11) + bc(n01, vv * w01 * w01)
    out["E"] = bc(n00, vv * w00 * w10) + bc(n01, vv * w01 * w11)     # bottom and top edges
    out["N"] = bc(n00, vv * w00 * w01) + bc(n10, vv * w10 * w11)     # left and right edges
    out["NE"] = bc(n00, vv * w00 * w11)                               # the "/" diagonal
    out["w"] = bc(n00, vv * w00) + bc(n10, vv * w10) + bc(n11, vv * w11) + bc(n01, vv * w01)
    out["b"] = np.stack([bc(n00, vv * values[f, ok] * w00) + bc(n10, vv * values[f, ok] * w10) +
                         bc(n11, vv * values[f, ok] * w11) + bc(n01, vv * values[f, ok] * w01)
                         for f in range(values.shape[0])])
    return out


def stencil_matrix(prob, st):
    """CSR matrix of a symmetric periodic stencil (D, E, N, NE in 2D; D, E in 1D)."""
    nx = prob["nx"]
    if prob["dim"] == 1:
        k = np.arange(nx)
        rows = np.concatenate([k, k, (k + 1) % nx])
        cols = np.concatenate([k, (k + 1) % nx, k])
        vals = np.concatenate([st["D"], st["E"], st["E"]])
        return sp.coo_matrix((vals, (rows, cols)), shape=(nx, nx)).tocsr()
    ny = prob["ny"]
    nn = nx * ny
    j, i = np.divmod(np.arange(nn), nx)
    k = np.arange(nn)
    kx = (i + 1) % nx + nx * j
    ky = i + nx * ((j + 1) % ny)
    kxy = (i + 1) % nx + nx * ((j + 1) % ny)
    rows = np.concatenate([k, k, kx, k, ky, k, kxy])
    cols = np.concatenate([k, kx, k, ky, k, kxy, k])
    vals = np.concatenate([st["D"], st["E"], st["E"], st["N"], st["N"], st["NE"], st["NE"]])
    return sp.coo_matrix((vals, (rows, cols)), shape=(nn, nn)).tocsr()
