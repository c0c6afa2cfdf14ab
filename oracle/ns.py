"""FP64 oracle of the particle fluid solver of Sec. 3.3 (Taylor-Green vortex sheet).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: nothing in the product
imports this module, and it imports nothing from the product.

The paper states the flow problem (incompressible Navier-Stokes, Sec. 3.3), the
Taylor-Green solution, its parameters (u0 = 1, L = 1, nu = 0.005, Re = 200), the
error measure (eq. (29)), the particle count (as many particles as nodes) and the
time step (Courant number 0.5), and says only that the scheme is a standard
splitting approach with mid-point time integration and mesh derivatives.  The
scheme written here is this code's reading of that sentence (a fractional step for
equal-order P1 velocity and pressure); every step of it is stated below.

Mesh: the periodic P1 mesh of ``p1`` (n x n square cells of side h, "/" split).

One time step from particle velocities a_mu at positions r_mu:
1. P2M: Ubar = assign(a) per velocity component, with FLIP (Sec. 2.3) or the mass
   assignment (Sec. 2.4 read with the particle quadrature, ``p1.mass_assign``).
2. Viscous step, implicit: (M_L + dt nu K) U* = M_L Ubar, with K the P1 stiffness
   matrix (K_ij = int grad psi_i . grad psi_j) and M_L = h^2 I the row-sum lumping
   of the P1 mesh mass matrix.
3. Pressure Poisson: K p = -(1/dt) D U*, with (D U)_i = int psi_i div U_h.  K is
   singular (constants); node 0 is held at p = 0 (its row and column replaced by the
   identity, right-hand side 0), which changes p by a constant only.
4. Projection: U^{n+1} = U* - dt M_L^{-1} G p, with (G p)_i = int psi_i grad p_h.
5. M2P: a_mu <- U^{n+1}(r_mu) (interpolation, Sec. 2.2 eq. (10)).
6. Mid-point advection: r* = r + (dt/2) a_mu, r <- r + dt U^{n+1}(r*), wrapped
   into [0, L) per axis.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import p1

ASSIGN = ("flip", "mass")


def _cell_nodes(nx, ny):
    """Node numbers (n00, n10, n11, n01) of every cell, cell (i, j) at i + nx*j."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    ip, jp = (i + 1) % nx, (j + 1) % ny
    return i + nx * j, ip + nx * j, ip + nx * jp, i + nx * jp


def _triangles(nx, ny):
    """The two triangles of every cell with the gradients of their three hats
    (in units of 1/h): lower (n00, n10, n11) and upper (n00, n11, n01)."""
    n00, n10, n11, n01 = _cell_nodes(nx, ny)
    lower = ((n00, n10, n11), ((-1.0, 0.0), (1.0, -1.0), (0.0, 1.0)))
    upper = ((n00, n11, n01), ((0.0, -1.0), (1.0, 0.0), (-1.0, 1.0)))
    return (lower, upper)


def _mesh(prob):
    nx, ny = prob["nx"], prob["ny"]
    h = prob["lx"] / nx
    if abs(prob["ly"] / ny - h) > 1e-12 * h:
        raise ValueError("square cells only")
    return nx, ny, h


def stiffness_matrix(prob):
    """K_ij = sum over triangles of area * grad psi_i . grad psi_j (dimensionless)."""
    nx, ny, _ = _mesh(prob)
    n = nx * ny
    rows, cols, vals = [], [], []
    for nodes, grads in _triangles(nx, ny):
        for a in range(3):
            for b in range(3):
                ga, gb = np.array(grads[a]), np.array(grads[b])
                rows.append(nodes[a])
                cols.append(nodes[b])
                vals.append(np.full(nodes[a].shape, 0.5 * float(ga @ gb)))   # area h^2/2, grads /h
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def gradient_matrices(prob):
    """(Cx, Cy): C_ij = int psi_i grad psi_j = sum over triangles T of both nodes of
    (int_T psi_i) grad psi_j|_T, with int_T psi_i = area/3 = h^2/6."""
    nx, ny, h = _mesh(prob)
    n = nx * ny
    out = []
    for comp in range(2):
        rows, cols, vals = [], [], []
        for nodes, grads in _triangles(nx, ny):
            for a in range(3):
                for b in range(3):
                    rows.append(nodes[a])
                    cols.append(nodes[b])
                    vals.append(np.full(nodes[a].shape, (h / 6.0) * grads[b][comp]))
        out.append(sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                 shape=(n, n)))
    return out[0], out[1]


def divergence(C, U):
    """(D U)_i = int psi_i div U_h, U = [2, N_n]."""
    return C[0] @ U[0] + C[1] @ U[1]


def gradient(C, p):
    """(G p)_i = int psi_i grad p_h, as [2, N_n]."""
    return np.stack([C[0] @ p, C[1] @ p])


def pinned(K):
    """K with node 0's row and column replaced by the identity."""
    K = K.tolil()
    K[0, :] = 0.0
    K[:, 0] = 0.0
    K[0, 0] = 1.0
    return K.tocsc()


def mesh_step(prob, Ubar, dt, nu, ops=None):
    """Steps 2-4 on the mesh: (U*, p, U^{n+1})."""
    nx, ny, h = _mesh(prob)
    K, C, Kp = ops if ops is not None else operators(prob)
    n = nx * ny
    s = dt * nu / h ** 2
    A = (sp.identity(n, format="csc") + s * K).tocsc()
    Ustar = np.stack([spla.spsolve(A, Ubar[c]) for c in range(2)])
    rhs = -(1.0 / dt) * divergence(C, Ustar)
    rhs[0] = 0.0
    p = spla.spsolve(Kp, rhs)
    Unew = Ustar - (dt / h ** 2) * gradient(C, p)
    return Ustar, p, Unew


def operators(prob):
    K = stiffness_matrix(prob)
    return K, gradient_matrices(prob), pinned(K)


def wrap(x, length):
    return x - length * np.floor(x / length)


def assign(prob, a, method):
    if method == "flip":
        return p1.flip(prob, a)[0]
    if method == "mass":
        return p1.mass_assign(prob, a, solver="direct")[0]
    raise ValueError(method)


def step(prob, a, method, dt, nu, ops=None):
    """One time step (steps 1-6).  Returns (new problem dict, new particle
    velocities [2, N_p], U^{n+1} [2, N_n])."""
    Ubar = assign(prob, a, method)
    _, _, Unew = mesh_step(prob, Ubar, dt, nu, ops)
    a_new = p1.interpolate(prob, Unew)
    xm = wrap(prob["x"] + 0.5 * dt * a_new[0], prob["lx"])
    ym = wrap(prob["y"] + 0.5 * dt * a_new[1], prob["ly"])
    mid = dict(prob, x=xm, y=ym)
    am = p1.interpolate(mid, Unew)
    new = dict(prob, x=wrap(prob["x"] + dt * am[0], prob["lx"]),
               y=wrap(prob["y"] + dt * am[1], prob["ly"]))
    return new, a_new, Unew


def taylor_green(x, y, t, length=1.0, nu=0.005, u0=1.0):
    """The Taylor-Green vortex sheet of Sec. 3.3: u = f sin(kx) cos(ky),
    v = -f cos(kx) sin(ky), k = 2 pi / L, f = u0 exp(-2 nu k^2 t)."""
    k = 2.0 * np.pi / length
    f = u0 * np.exp(-2.0 * nu * k * k * t)
    return np.stack([f * np.sin(k * x) * np.cos(k * y), -f * np.cos(k * x) * np.sin(k * y)])
