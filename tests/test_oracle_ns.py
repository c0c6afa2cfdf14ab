"""Pins of the FP64 oracle of the particle fluid solver (oracle/ns.py, Sec. 3.3).

The scheme is this code's reading of the paper's one-sentence description (a
splitting approach with mid-point time integration and mesh derivatives); the pins
are facts that hold whatever the code: closed forms of the P1 operators on the "/"
mesh, identities of periodic integration by parts, consistency orders, the exact
Taylor-Green solution, and the paper's own observations (first order in dt; the
mass assignment more accurate than FLIP)."""
import numpy as np
import pytest

from oracle import ns

K2PI = 2.0 * np.pi


def mesh(n):
    return dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=np.zeros(1), y=np.zeros(1), vol=None)


def nodes(n):
    xs = np.arange(n) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    return X.ravel(), Y.ravel()


def test_stiffness_is_the_five_point_laplacian():
    """For right isosceles triangles the P1 stiffness matrix is 4 on the diagonal,
    -1 towards the four axis neighbours and 0 across the diagonals."""
    n = 6
    K = ns.stiffness_matrix(mesh(n)).toarray()
    ref = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            k = i + n * j
            ref[k, k] = 4.0
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ref[k, (i + di) % n + n * ((j + dj) % n)] -= 1.0
    assert np.array_equal(K, ref)


def test_gradient_operator_identities():
    """Periodic integration by parts: int psi_i d psi_j + int psi_j d psi_i = 0, so
    C + C^T = 0; the hats sum to one, so the rows and columns of C sum to 0."""
    Cx, Cy = ns.gradient_matrices(mesh(7))
    for C in (Cx, Cy):
        assert abs(C + C.T).max() == 0.0
        assert np.abs(np.asarray(C.sum(axis=0))).max() < 1e-15
        assert np.abs(np.asarray(C.sum(axis=1))).max() < 1e-15


def test_gradient_is_second_order_at_the_nodes():
    """(G p)_i / h^2 approximates grad p at node i to O(h^2) for a smooth p."""
    errs = []
    for n in (16, 32, 64):
        X, Y = nodes(n)
        p = np.sin(K2PI * X) * np.cos(K2PI * Y)
        G = ns.gradient(ns.gradient_matrices(mesh(n)), p) * n * n
        ex = np.stack([K2PI * np.cos(K2PI * X) * np.cos(K2PI * Y),
                       -K2PI * np.sin(K2PI * X) * np.sin(K2PI * Y)])
        errs.append(np.abs(G - ex).max() / K2PI)
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_viscous_step_on_the_taylor_green_mode():
    """The nodal Taylor-Green field is an eigenvector of the five-point K with
    eigenvalue 4 - 4 cos(kh) and is discretely divergence-free, so one mesh step
    scales it by exactly 1 / (1 + (dt nu / h^2) (4 - 4 cos(kh)))."""
    n = 24
    X, Y = nodes(n)
    tg = ns.taylor_green(X, Y, 0.0)
    h, dt, nu = 1.0 / n, 0.02, 0.05
    _, p, U = ns.mesh_step(mesh(n), tg, dt, nu)
    factor = 1.0 / (1.0 + dt * nu / h ** 2 * (4.0 - 4.0 * np.cos(K2PI * h)))
    assert np.abs(U - factor * tg).max() < 1e-13
    assert np.abs(p).max() < 1e-12


def test_projection_removes_a_gradient_field():
    """With nu = 0, a Taylor-Green field plus the gradient of phi = cos(kx) sin(2ky)/k
    comes back as the Taylor-Green field, to second order in h."""
    res = []
    for n in (16, 32, 64):
        X, Y = nodes(n)
        tg = ns.taylor_green(X, Y, 0.0)
        gphi = np.stack([-np.sin(K2PI * X) * np.sin(2 * K2PI * Y),
                         2.0 * np.cos(K2PI * X) * np.cos(2 * K2PI * Y)])
        _, _, U = ns.mesh_step(mesh(n), tg + gphi, 0.5 / n, 0.0)
        res.append(np.linalg.norm(U - tg) / np.linalg.norm(gphi))
    assert res[2] < 0.02 and 3.4 < res[0] / res[1] < 4.4 and 3.4 < res[1] / res[2] < 4.4


def test_mesh_step_conserves_momentum():
    """sum_i K_ij = 0 and sum_i C_ij = 0: the viscous and pressure steps leave the
    total momentum (lumped mass times velocity) unchanged."""
    n = 20
    U0 = np.random.default_rng(5).normal(size=(2, n * n))
    _, _, U = ns.mesh_step(mesh(n), U0, 0.01, 0.3)
    assert np.abs(U.sum(axis=1) - U0.sum(axis=1)).max() < 1e-11


def run_tg(n, method, T=0.25, ppc=2, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    x = ((i.ravel()[:, None] + g.uniform(0, 1, (n * n, ppc))) * h).ravel()
    y = ((j.ravel()[:, None] + g.uniform(0, 1, (n * n, ppc))) * h).ravel()
    prob = dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=x, y=y, vol=None)
    a = ns.taylor_green(x, y, 0.0)
    dt = 0.5 * h                       # Courant number 0.5 with u0 = 1
    steps = int(round(T / dt))
    ops = ns.operators(prob)
    for _ in range(steps):
        prob, a, _ = ns.step(prob, a, method, dt, 0.005, ops)
    ex = ns.taylor_green(prob["x"], prob["y"], steps * dt)
    return np.sqrt(((ex - a) ** 2).sum() / (ex ** 2).sum())


def test_taylor_green_first_order_and_mass_beats_flip():
    """Sec. 3.3: the velocity error against the exact solution falls as dt^1 at a
    fixed Courant number (here dt and h halve together), and the mass assignment is
    more accurate than FLIP."""
    e = {(n, m): run_tg(n, m) for n in (16, 32) for m in ns.ASSIGN}
    for m in ns.ASSIGN:
        assert 1.4 < e[(16, m)] / e[(32, m)] < 2.8, (m, e)
    for n in (16, 32):
        assert e[(n, "mass")] < 0.6 * e[(n, "flip")], e
