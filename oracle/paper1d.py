"""Paper-exact 1D assignment methods (Table 1) and the Sec. 3.1 top-hat experiment.

Test infrastructure only (see the package docstring).

In 1D the particle hats psi_mu are the P1 hats on the particles sorted along the
periodic segment (Sec. 2, eq. (1); Sec. 3.1), so the particle "triangulation" is
the sorted order.  Everything here is FP64 and follows the paper's definitions:

* particle volume v_mu = int psi_mu = (x_{mu+1} - x_{mu-1}) / 2      (eq. (4))
* mesh volume v_i = int psi_i = h                                     (eq. (5))
* consistent mass matrices m_ij = int psi_i psi_j                     (Sec. 2.4)
  mesh: 2h/3 on the diagonal, h/6 off it; particles: (D_{mu-1}+D_mu)/3 and D_mu/6
  with D_mu = x_{mu+1} - x_mu.
* the overlap integrals int A psi_j either exactly ("exact": both factors are
  piecewise linear, so on every piece between merged breakpoints the product is a
  quadratic and Simpson's rule is exact) or with the Appendix-B rule ("appB": per
  element, fit a parabola Q through A at both ends and the midpoint and integrate
  Q psi_j exactly; Q psi_j is a cubic, so Simpson's rule on the element is exact:
  int_e Q psi_j = |e|/6 (A(x_j) + 2 A(mid))).

Methods (Table 1 rows): delta, FLIP, mass-delta, full mass, and the two lumped
variants the paper lists without results.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import metrics


# ----------------------------------------------------------------------------
# periodic piecewise-linear interpolants
# ----------------------------------------------------------------------------
def periodic_sort(x, L=1.0):
    """Positions wrapped to [0, L) and the stable order along the segment."""
    xw = np.mod(np.asarray(x, dtype=np.float64), L)
    order = np.argsort(xw, kind="stable")
    return xw, order


def particle_volumes(x, L=1.0):
    """eq. (4) for 1D hats on sorted particles: v_mu = (x_{mu+1} - x_{mu-1}) / 2, periodic."""
    xw, order = periodic_sort(x, L)
    xs = xw[order]
    gap = np.diff(np.concatenate([xs, [xs[0] + L]]))     # D_mu = x_{mu+1} - x_mu
    vs = 0.5 * (gap + np.roll(gap, 1))
    v = np.empty_like(vs)
    v[order] = vs
    return v


def eval_pl(knots, vals, xq, L=1.0):
    """Evaluate the periodic piecewise-linear function through (knots, vals) at xq.

    knots need not be sorted; the function is sum_k vals_k psi_k with psi_k the
    periodic P1 hat on the sorted knots (eq. (1) for particles, eq. (3) for nodes).
    """
    kw, order = periodic_sort(knots, L)
    ks = kw[order]
    vs = np.asarray(vals, dtype=np.float64)[order]
    ext_k = np.concatenate([[ks[-1] - L], ks, [ks[0] + L]])
    ext_v = np.concatenate([[vs[-1]], vs, [vs[0]]])
    xq = np.mod(np.asarray(xq, dtype=np.float64), L)
    # np.interp needs increasing knots; duplicates are harmless for evaluation.
    return np.interp(xq, ext_k, ext_v)


def hat_values(knots, xq, L=1.0):
    """psi_k(xq) for every knot k: a dense [K, Q] matrix (small sizes only)."""
    K = len(knots)
    out = np.zeros((K, len(xq)))
    for k in range(K):
        e = np.zeros(K)
        e[k] = 1.0
        out[k] = eval_pl(knots, e, xq, L)
    return out


# ----------------------------------------------------------------------------
# mass matrices
# ----------------------------------------------------------------------------
def mesh_mass(n, L=1.0):
    """Consistent mesh mass matrix of Sec. 2.4 for 1D P1 hats: 2h/3 diagonal, h/6 neighbours."""
    h = L / n
    m = np.zeros((n, n))
    for i in range(n):
        m[i, i] += 2.0 * h / 3.0
        m[i, (i + 1) % n] += h / 6.0
        m[(i + 1) % n, i] += h / 6.0
    return m


def particle_mass(x, L=1.0):
    """Consistent particle mass matrix m_{mu nu} = int psi_mu psi_nu (Sec. 2.4, used by eq. (20))."""
    xw, order = periodic_sort(x, L)
    xs = xw[order]
    N = xs.size
    gap = np.diff(np.concatenate([xs, [xs[0] + L]]))
    ms = np.zeros((N, N))
    for k in range(N):
        ms[k, k] += gap[k] / 3.0
        ms[(k + 1) % N, (k + 1) % N] += gap[k] / 3.0
        ms[k, (k + 1) % N] += gap[k] / 6.0
        ms[(k + 1) % N, k] += gap[k] / 6.0
    m = np.zeros_like(ms)
    m[np.ix_(order, order)] = ms
    return m


# ----------------------------------------------------------------------------
# overlap integrals int f psi_k
# ----------------------------------------------------------------------------
def overlap_exact(f_knots, f_vals, g_knots, L=1.0):
    """c_k = int f(x) psi_k(x) dx over [0, L) for every hat psi_k on g_knots, exactly.

    f is the periodic piecewise-linear function through (f_knots, f_vals).  All
    breakpoints of f and of the hats are merged; on every piece both factors are
    linear, so Simpson's rule integrates the quadratic product exactly.
    """
    gw, order = periodic_sort(g_knots, L)
    gs = gw[order]
    K = gs.size
    fw = np.mod(np.asarray(f_knots, dtype=np.float64), L)
    bps = np.unique(np.concatenate([gs, fw, [0.0]]))
    bps = np.concatenate([bps, [bps[0] + L]])
    a, b = bps[:-1], bps[1:]
    mid = 0.5 * (a + b)
    fa, fm, fb = (eval_pl(f_knots, f_vals, p, L) for p in (a, mid, b))
    c_sorted = np.zeros(K)
    # the piece [a, b] lies inside one gap [gs[k], gs[k+1]] of the hat knots; a
    # piece left of the first knot belongs to the wrap-around gap [gs[-1]-L, gs[0]]
    k = np.searchsorted(gs, mid, side="right") - 1
    wrap_low = k < 0
    k = k % K
    shift = np.where(wrap_low, L, 0.0)
    left = gs[k] - shift
    right = np.where(k + 1 < K, gs[(k + 1) % K], gs[0] + L) - shift
    span = right - left
    psi_l = [(right - p) / span for p in (a, mid, b)]      # hat of knot k on this gap
    psi_r = [1.0 - q for q in psi_l]                       # hat of knot k+1
    h6 = (b - a) / 6.0
    int_left = h6 * (fa * psi_l[0] + 4.0 * fm * psi_l[1] + fb * psi_l[2])
    int_right = h6 * (fa * psi_r[0] + 4.0 * fm * psi_r[1] + fb * psi_r[2])
    np.add.at(c_sorted, k, int_left)
    np.add.at(c_sorted, (k + 1) % K, int_right)
    c = np.empty(K)
    c[order] = c_sorted
    return c


def overlap_appendix_b(f_knots, f_vals, g_knots, L=1.0):
    """Appendix-B quadrature of c_k = int f psi_k over the two gaps adjacent to knot k.

    On each gap e = [g_k, g_{k+1}] of the hat knots, f is sampled at both ends and
    at the midpoint, the parabola Q through the three samples is integrated
    against the two hats of the gap: int_e Q psi_k = |e|/6 (f(g_k) + 2 f(mid)) and
    int_e Q psi_{k+1} = |e|/6 (f(g_{k+1}) + 2 f(mid)).  Exact when f is linear on e
    (no f breakpoint inside e).
    """
    gw, order = periodic_sort(g_knots, L)
    gs = gw[order]
    K = gs.size
    gap = np.diff(np.concatenate([gs, [gs[0] + L]]))
    mid = gs + 0.5 * gap
    f_left = eval_pl(f_knots, f_vals, gs, L)
    f_mid = eval_pl(f_knots, f_vals, mid, L)
    f_right = np.roll(f_left, -1)
    c_sorted = gap / 6.0 * (f_left + 2.0 * f_mid)
    c_sorted += np.roll(gap / 6.0 * (f_right + 2.0 * f_mid), 1)
    c = np.empty(K)
    c[order] = c_sorted
    return c


# ----------------------------------------------------------------------------
# assignments (Table 1)
# ----------------------------------------------------------------------------
def nodes_1d(n, L=1.0):
    return np.arange(n) * (L / n)


def p2m_delta(xp, A, n, L=1.0):
    """delta P2M, eq. (9): the particle interpolant evaluated at the nodes."""
    return eval_pl(xp, A, nodes_1d(n, L), L)


def m2p_delta(xp, Abar, n, L=1.0):
    """delta M2P, eq. (10) read at r_mu: the mesh interpolant evaluated at the particles."""
    return eval_pl(nodes_1d(n, L), Abar, xp, L)


def _mesh_hat_weights(xp, n, L):
    """Element of every particle on the uniform mesh and its two P1 weights (eq. (3))."""
    h = L / n
    t = np.mod(np.asarray(xp, dtype=np.float64), L) / h
    c = np.floor(t)
    frac = t - c
    c = c.astype(np.int64) % n
    return c, (c + 1) % n, 1.0 - frac, frac


def p2m_flip(xp, A, n, L=1.0, vp=None):
    """FLIP P2M, eqs. (11)-(12): sum A v psi_i(x_mu) / sum v psi_i(x_mu), orphans -> 0."""
    vp = particle_volumes(xp, L) if vp is None else vp
    i0, i1, w0, w1 = _mesh_hat_weights(xp, n, L)
    num = np.bincount(i0, vp * A * w0, minlength=n) + np.bincount(i1, vp * A * w1, minlength=n)
    den = np.bincount(i0, vp * w0, minlength=n) + np.bincount(i1, vp * w1, minlength=n)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def p2m_pic(xp, A, n, L=1.0, vp=None):
    """PIC P2M, eq. (11) with eq. (5): sum A v psi_i(x_mu) / h."""
    vp = particle_volumes(xp, L) if vp is None else vp
    i0, i1, w0, w1 = _mesh_hat_weights(xp, n, L)
    num = np.bincount(i0, vp * A * w0, minlength=n) + np.bincount(i1, vp * A * w1, minlength=n)
    return num / (L / n)


def p2m_mass(xp, A, n, L=1.0, quad="appB", m_lu=None):
    """Mass P2M, eqs. (13), (19) / Table 1: Abar = m^{-1} int A psi, m the mesh mass matrix."""
    xn = nodes_1d(n, L)
    c = overlap_exact(xp, A, xn, L) if quad == "exact" else overlap_appendix_b(xp, A, xn, L)
    if m_lu is None:
        m_lu = sla.lu_factor(mesh_mass(n, L))
    return sla.lu_solve(m_lu, c)


def m2p_mass(xp, Abar, n, L=1.0, quad="appB"):
    """Full-mass M2P, eq. (20) / Table 1: Abarbar = m_part^{-1} int Abar psi_nu."""
    xn = nodes_1d(n, L)
    c = overlap_exact(xn, Abar, xp, L) if quad == "exact" else overlap_appendix_b(xn, Abar, xp, L)
    return np.linalg.solve(particle_mass(xp, L), c)


def p2m_lumped(xp, A, n, L=1.0, quad="appB"):
    """Lumped P2M, Table 1 with eq. (17): Abar_i = (1/v_i) int A psi_i, v_i = h."""
    xn = nodes_1d(n, L)
    c = overlap_exact(xp, A, xn, L) if quad == "exact" else overlap_appendix_b(xp, A, xn, L)
    return c / (L / n)


def m2p_lumped(xp, Abar, n, L=1.0, quad="appB"):
    """Lumped M2P, Table 1: Abarbar_mu = (1/v_mu) int Abar psi_mu."""
    xn = nodes_1d(n, L)
    c = overlap_exact(xn, Abar, xp, L) if quad == "exact" else overlap_appendix_b(xn, Abar, xp, L)
    return c / particle_volumes(xp, L)


METHODS = ("delta", "flip", "mass_delta", "full_mass", "mass_lumped", "lumped")


def round_trip(method, xp, A, n, L=1.0, quad="appB", m_lu=None):
    """One P2M followed by one M2P with the pair of Table 1 for ``method``."""
    if method == "delta":
        return m2p_delta(xp, p2m_delta(xp, A, n, L), n, L)
    if method == "flip":
        return m2p_delta(xp, p2m_flip(xp, A, n, L), n, L)
    if method == "mass_delta":
        return m2p_delta(xp, p2m_mass(xp, A, n, L, quad, m_lu), n, L)
    if method == "full_mass":
        return m2p_mass(xp, p2m_mass(xp, A, n, L, quad, m_lu), n, L, quad)
    if method == "mass_lumped":
        return m2p_lumped(xp, p2m_mass(xp, A, n, L, quad, m_lu), n, L, quad)
    if method == "lumped":
        return m2p_lumped(xp, p2m_lumped(xp, A, n, L, quad), n, L, quad)
    raise ValueError(method)


# ----------------------------------------------------------------------------
# Sec. 3.1: moving top-hat
# ----------------------------------------------------------------------------
def tophat_positions(n_particles, distort=0.0, seed=0, L=1.0):
    """Regular particles on the nodes x_mu = mu*dx, optionally moved by U(-distort, distort)*dx."""
    dx = L / n_particles
    x = np.arange(n_particles) * dx
    if distort > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        x = x + rng.uniform(-distort, distort, n_particles) * dx
    return np.mod(x, L)


def tophat_experiment(method, n_nodes=200, n_particles=200, co=0.1, u=1.0, T=1.0,
                      distort=0.0, seed=0, quad="appB", lo=0.25, hi=0.75, L=1.0):
    """Sec. 3.1: advect a top-hat with dx/dt = u, projecting to the mesh and back every step.

    Step order: move the particles, then P2M, then M2P (particle values are
    replaced by the round-trip result).  dt = Co * dx_mesh / u; at T = 1 the
    particles are back where they started.  Returns E1, E2, L2 (metrics module).
    """
    x0 = tophat_positions(n_particles, distort, seed, L)
    A0 = ((x0 > lo) & (x0 < hi)).astype(np.float64)
    dt = co * (L / n_nodes) / u
    steps = int(round(T / dt))
    m_lu = sla.lu_factor(mesh_mass(n_nodes, L))
    A = A0.copy()
    for k in range(1, steps + 1):
        xk = np.mod(x0 + k * u * dt, L)
        A = round_trip(method, xk, A, n_nodes, L, quad, m_lu)
    xT = np.mod(x0 + steps * u * dt, L)
    v0 = particle_volumes(x0, L)
    vT = particle_volumes(xT, L)
    return dict(E1=metrics.e1(v0, A0, vT, A), E2=metrics.e2(v0, A0, vT, A),
                L2=metrics.l2(v0, A0, A), A0=A0, AT=A, x0=x0, steps=steps)
