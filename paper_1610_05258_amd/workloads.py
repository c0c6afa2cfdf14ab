"""Seeded synthetic particle sets for the assignment library.

This module generates inputs only: particle positions, volumes and field values
of the paper's analytic workloads (a top-hat on a periodic segment, Sec. 3.1;
Zalesak's slotted disk under rigid rotation, Sec. 3.2; Taylor-Green vortex
fields, Sec. 3.3 eq. (26)).  It holds none of the assignment arithmetic; the
same arrays are handed to the GPU library and, in tests, to the CPU oracle.

All generation happens in FP64 with numpy's PCG64; arrays meant for the FP32
path are rounded once at the end.  Particle order is the generation order
(cell by cell for stratified sets), followed by any advection.

A problem is a dict with keys dim, nx, ny, lx, ly, x, y, vol (None = uniform
volumes) and the field values live beside it as a [F, N_p] array.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# positions
# ----------------------------------------------------------------------------
def uniform_1d(seed, n_particles, length=1.0):
    """Uniform random positions on [0, length) in FP64."""
    return rng(seed).uniform(0.0, length, n_particles)


def stratified_2d(seed, nx, ny, ppc, lx, ly):
    """``ppc`` particles uniform inside every cell, generated cell by cell (row-major cells)."""
    g = rng(seed)
    hx, hy = lx / nx, ly / ny
    j, i = np.divmod(np.arange(nx * ny, dtype=np.int64), nx)
    i = np.repeat(i, ppc)
    j = np.repeat(j, ppc)
    u = g.random((2, i.size))
    x = (i + u[0]) * hx
    y = (j + u[1]) * hy
    return x, y


def wrap(x, length):
    """Positions wrapped into [0, length) in FP64."""
    return np.mod(x, length)


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------
def tophat(x, lo, hi, closed_left=True):
    """Indicator of [lo, hi) (or of (lo, hi) when closed_left is False)."""
    x = np.asarray(x, dtype=np.float64)
    left = (x >= lo) if closed_left else (x > lo)
    return (left & (x < hi)).astype(np.float64)


# Zalesak's disk (Sec. 3.2 proportions scaled to the unit square): radius 0.15,
# centre (0.5, 0.75), slot width 0.05 (R/3, the paper's 1/6 for R = 0.5) and
# slot length 0.25 (5R/3, the paper's 5/6), vertical, open downward.
ZALESAK = dict(cx=0.5, cy=0.75, r=0.15, slot_w=0.05, slot_len=0.25,
               rot_cx=0.5, rot_cy=0.5, rot_radius=0.5 * 1.4 / 1.5)


def zalesak_disk(x, y, z=ZALESAK):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    inside = (x - z["cx"]) ** 2 + (y - z["cy"]) ** 2 <= z["r"] ** 2
    slot_top = z["cy"] - z["r"] + z["slot_len"]
    in_slot = (np.abs(x - z["cx"]) <= 0.5 * z["slot_w"]) & (y <= slot_top)
    return (inside & ~in_slot).astype(np.float64)


def zalesak_rotate(x, y, angle, z=ZALESAK):
    """Exact rigid rotation about (0.5, 0.5) of the particles within rot_radius.

    The velocity (-(y-0.5), x-0.5) is applied only inside the circle of radius
    0.5*1.4/1.5 (the paper moves only the region within radius 1.4 of its 3x3
    box), so the periodic unit square is never torn.
    """
    dx = np.asarray(x, dtype=np.float64) - z["rot_cx"]
    dy = np.asarray(y, dtype=np.float64) - z["rot_cy"]
    moving = dx * dx + dy * dy <= z["rot_radius"] ** 2
    c, s = math.cos(angle), math.sin(angle)
    xr = z["rot_cx"] + c * dx - s * dy
    yr = z["rot_cy"] + s * dx + c * dy
    return np.where(moving, xr, x), np.where(moving, yr, y)


def taylor_green(x, y):
    """Taylor-Green fields on [0, 2 pi)^2 with k = 1 (Sec. 3.3 eq. (26) at f = 1).

    u = sin x cos y, v = -cos x sin y, p = (cos 2x + cos 2y) / 4.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y),
                     0.25 * (np.cos(2.0 * x) + np.cos(2.0 * y))])


def tg_advect_rk2(x, y, steps, dt, device="cpu"):
    """Midpoint-rule (RK2) advection of positions by the TG velocity, wrapped mod 2 pi each step.

    Runs in FP64 with torch (multi-threaded elementwise maths) on ``device``; the
    CPU is the reproducible default (other devices round sin / cos differently).
    """
    if steps == 0:
        return np.asarray(x, np.float64).copy(), np.asarray(y, np.float64).copy()
    import torch
    X = torch.from_numpy(np.asarray(x, dtype=np.float64).copy()).to(device)
    Y = torch.from_numpy(np.asarray(y, dtype=np.float64).copy()).to(device)
    for _ in range(steps):
        u = torch.sin(X) * torch.cos(Y)
        v = -torch.cos(X) * torch.sin(Y)
        Xm = X + 0.5 * dt * u
        Ym = Y + 0.5 * dt * v
        u = torch.sin(Xm) * torch.cos(Ym)
        v = -torch.cos(Xm) * torch.sin(Ym)
        X = torch.remainder(X + dt * u, TWO_PI)
        Y = torch.remainder(Y + dt * v, TWO_PI)
    return X.cpu().numpy(), Y.cpu().numpy()


def to_f32_positions(x, length):
    """Round FP64 positions to FP32; a value that rounds up to ``length`` stays (it wraps in the locate)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def tophat_1d(seed=0, n=64, n_particles=256, lo=0.25, hi=0.5):
    """1D periodic [0,1): ``n`` P1 elements, uniform random particles, top-hat on [lo, hi), FP64."""
    x = uniform_1d(seed, n_particles)
    prob = dict(dim=1, nx=n, ny=1, lx=1.0, ly=1.0, x=x, y=None, vol=None)
    return prob, tophat(x, lo, hi)[None, :]


def zalesak_2d(seed=1, n=256, ppc=4):
    """2D periodic unit square, ``ppc`` stratified particles per cell, slotted-disk indicator.

    Returns (prob with FP32 positions, values [1, N_p] FP32, x64, y64): the FP64
    master positions drive the rotation; the FP32 copies are what both sides see.
    """
    x, y = stratified_2d(seed, n, n, ppc, 1.0, 1.0)
    a = zalesak_disk(x, y)[None, :]
    prob = dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=to_f32_positions(x, 1.0),
                y=to_f32_positions(y, 1.0), vol=None)
    return prob, a.astype(np.float32), x, y


ZALESAK_DT = TWO_PI / 628.0


def taylor_green_2d(seed=2, n=1024, ppc=8, steps=50, dt=1e-3, noise=1e-3, fields=3):
    """2D periodic [0, 2 pi)^2, ``ppc`` stratified particles per cell, TG fields.

    Values are sampled at the initial positions with N(0, noise^2) added per
    particle and field, then carried while the positions are advected ``steps``
    RK2 steps of ``dt`` by the TG velocity.  Positions and values are FP32.
    """
    x, y = stratified_2d(seed, n, n, ppc, TWO_PI, TWO_PI)
    vals = taylor_green(x, y)[:fields]
    if noise > 0.0:
        vals = vals + rng(seed + 1_000_000).normal(0.0, noise, vals.shape)
    x, y = tg_advect_rk2(x, y, steps, dt)
    prob = dict(dim=2, nx=n, ny=n, lx=TWO_PI, ly=TWO_PI, x=to_f32_positions(x, TWO_PI),
                y=to_f32_positions(y, TWO_PI), vol=None)
    return prob, vals.astype(np.float32)


def tg_fluid_2d(seed=4, n=256, ppc=4):
    """The Taylor-Green vortex sheet set-up of Sec. 3.3: unit periodic box, u0 = 1,
    ``ppc`` stratified particles per cell of an n x n mesh, carrying the exact
    velocity at t = 0 (no noise).  FP32 positions and velocities [2, np]."""
    x, y = stratified_2d(seed, n, n, ppc, 1.0, 1.0)
    vel = tg_fluid_exact(x, y, 0.0)
    prob = dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=to_f32_positions(x, 1.0),
                y=to_f32_positions(y, 1.0), vol=None)
    return prob, vel.astype(np.float32)


def tg_fluid_exact(x, y, t, nu=0.005):
    """Exact Taylor-Green velocity on the unit box at time t (Sec. 3.3): f(t) (sin 2pi x
    cos 2pi y, -cos 2pi x sin 2pi y), f = exp(-8 pi^2 nu t) (u0 = 1, L = 1)."""
    k = TWO_PI
    f = math.exp(-2.0 * nu * k * k * t)
    return np.stack([f * np.sin(k * x) * np.cos(k * y), -f * np.cos(k * x) * np.sin(k * y)])


def tg_disordered(seed, n=1024, ppc=8, steps=200, dt=1e-3, noise=1e-3, fields=3, random_phase=True,
                  device="cpu"):
    """TG-like fields on particles disordered by the flow: ``ppc`` stratified particles
    per cell of an n x n mesh on [0, 2 pi)^2; fields u, v, p of the TG solution with a
    random phase (phi_x, phi_y in [0, 2 pi)) and amplitude in [0.5, 2] (seeded), plus
    N(0, noise^2); the positions are then advected ``steps`` RK2 steps of ``dt`` by the
    TG velocity.  FP32 positions and values."""
    g = rng(seed + 7_000_000)
    phx, phy = (g.uniform(0.0, TWO_PI, 2) if random_phase else (0.0, 0.0))
    amp = g.uniform(0.5, 2.0) if random_phase else 1.0
    x, y = stratified_2d(seed, n, n, ppc, TWO_PI, TWO_PI)
    vals = amp * taylor_green(x + phx, y + phy)[:fields]
    if noise > 0.0:
        vals = vals + g.normal(0.0, noise, vals.shape)
    x, y = tg_advect_rk2(x, y, steps, dt, device)
    prob = dict(dim=2, nx=n, ny=n, lx=TWO_PI, ly=TWO_PI, x=to_f32_positions(x, TWO_PI),
                y=to_f32_positions(y, TWO_PI), vol=None)
    return prob, vals.astype(np.float32)


def uneven_batch(seed=3, count=64, side_lo=32, side_hi=512, ppc_lo=2, ppc_hi=16, fields=2):
    """``count`` independent TG problems with log-uniform mesh side and uniform ppc (no noise, no advection)."""
    g = rng(seed)
    sides = np.rint(np.exp(g.uniform(math.log(side_lo), math.log(side_hi), count))).astype(int)
    ppcs = g.integers(ppc_lo, ppc_hi + 1, count)
    out = []
    for k in range(count):
        x, y = stratified_2d(seed * 1000 + k, sides[k], sides[k], int(ppcs[k]), TWO_PI, TWO_PI)
        vals = taylor_green(x, y)[:fields]
        prob = dict(dim=2, nx=int(sides[k]), ny=int(sides[k]), lx=TWO_PI, ly=TWO_PI,
                    x=to_f32_positions(x, TWO_PI), y=to_f32_positions(y, TWO_PI), vol=None)
        out.append((prob, vals.astype(np.float32)))
    return out
