"""GPU tests of the particle fluid solver step (p2m_ns_step, Sec. 3.3, the
Taylor-Green vortex sheet) against the FP64 oracle ``oracle/ns.py``: one step from
the same FP32 state gives the same mesh velocity, particle velocities and
positions (to the FP32 gate), many steps stay with the oracle and with the exact
solution, and the mass assignment is more accurate than FLIP as in the paper."""
import sys

import numpy as np
import pytest

from oracle import ns

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NU = 0.005     # Re = 200 with u0 = 1, L = 1 (Sec. 3.3)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_05258_amd import binding
    binding.lib()
    return binding


def tg_problem(n, ppc, seed):
    """Stratified particles (ppc per cell), exact Taylor-Green velocities at t = 0."""
    g = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    x = ((i.ravel()[:, None] + g.uniform(0, 1, (n * n, ppc))) * h).ravel().astype(np.float32)
    y = ((j.ravel()[:, None] + g.uniform(0, 1, (n * n, ppc))) * h).ravel().astype(np.float32)
    prob = dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=x, y=y, vol=None)
    a = ns.taylor_green(x.astype(np.float64), y.astype(np.float64), 0.0).astype(np.float32)
    return prob, a


def f64(prob):
    return dict(prob, x=np.asarray(prob["x"], np.float64), y=np.asarray(prob["y"], np.float64))


def torus_dist(a, b):
    d = np.abs(a - b)
    return np.minimum(d, 1.0 - d)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_steps(B, ctx, prob, a, method, dt, steps, tol=1e-8):
    d = B.particles_from(prob, dtype=torch.float32)
    vel = torch.as_tensor(a).cuda().contiguous()
    mv = torch.empty((2, prob["nx"] * prob["ny"]), dtype=torch.float32, device="cuda")
    opts = B.solve_opts(tol=tol, maxit=4000, max_refine=20)
    code = B.NS_MASS if method == "mass" else B.NS_FLIP
    reps = None
    for _ in range(steps):
        _, reps = B.p2m_ns_step(ctx, d, vel, code, dt, NU, opts, mesh_vel=mv)
    torch.cuda.synchronize()
    r = [B.read_report(reps[k], 2) for k in range(3)]
    return (d.x.cpu().numpy(), d.y.cpu().numpy(), vel.cpu().numpy(), mv.cpu().numpy(), r)


@pytest.mark.parametrize("method", ns.ASSIGN)
@pytest.mark.parametrize("n,fft", [(32, True), (48, True), (48, False), (256, True)])
def test_one_step_against_the_oracle(B, method, n, fft):
    """The two mesh systems solved by the 2D FFT (no iteration; 32 and 256 radix 2,
    48 by Bluestein's algorithm), and with P2M_OPT_FFT off by the mass-matrix solver
    (node 0 holding the pressure)."""
    prob, a = tg_problem(n, 2, seed=7)
    dt = 0.5 / n
    say(f"[ns one step] {method} {n}x{n}, fft {fft}, {prob['x'].size} particles")
    ctx = B.Context(0)
    try:
        ctx.set_fft(fft)
        x, y, vel, mv, reps = gpu_steps(B, ctx, prob, a, method, dt, 1)
    finally:
        ctx.close()
    for k, r in enumerate(reps):
        say(f"  report {k}: iters {r.iters[:2].tolist()} refines {r.refines[:2].tolist()} flags {r.flags}")
        assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN | B.FLAG_RANGE | B.FLAG_NONFINITE))
    assert (reps[2].iters[0] == 0) if fft else (reps[2].iters[0] > 0)
    new, a_ref, U_ref = ns.step(f64(prob), a.astype(np.float64), method, dt, NU)
    eU, ea = rel_l2(mv, U_ref), rel_l2(vel, a_ref)
    ex = max(torus_dist(x, new["x"]).max(), torus_dist(y, new["y"]).max())
    say(f"  mesh velocity rel l2 {eU:.2e}, particle velocity {ea:.2e}, positions max {ex:.2e}")
    assert eU <= 5e-6 and ea <= 5e-6 and ex <= 2e-7


@pytest.mark.parametrize("method", ns.ASSIGN)
def test_many_steps_against_the_oracle_and_the_exact_solution(B, method):
    """T = 0.25 at 32 x 32 (16 steps at Courant number 0.5): the GPU run stays with
    the oracle's, and both have the same error against the exact solution."""
    n, steps = 32, 16
    prob, a = tg_problem(n, 2, seed=3)
    dt = 0.5 / n
    ctx = B.Context(0)
    try:
        x, y, vel, _, _ = gpu_steps(B, ctx, prob, a, method, dt, steps)
    finally:
        ctx.close()
    pr, ar = f64(prob), a.astype(np.float64)
    ops = ns.operators(pr)
    for _ in range(steps):
        pr, ar, _ = ns.step(pr, ar, method, dt, NU, ops)
    e_gpu = rel_l2(vel, ns.taylor_green(x.astype(np.float64), y.astype(np.float64), steps * dt))
    e_ref = rel_l2(ar, ns.taylor_green(pr["x"], pr["y"], steps * dt))
    say(f"[ns {steps} steps] {method}: vs oracle {rel_l2(vel, ar):.2e}; L2 vs exact GPU {e_gpu:.4e} "
        f"oracle {e_ref:.4e}")
    assert rel_l2(vel, ar) <= 1e-4
    assert abs(e_gpu - e_ref) <= 1e-3 * e_ref


def test_mass_more_accurate_than_flip(B):
    """Sec. 3.3 (Fig. 4): at the same resolution and time step the mass assignment
    ends much closer to the exact solution than FLIP (128 x 128, T = 0.25).  Four
    particles per cell: the particle mass matrix needs enough particles in every
    node's support as the flow stretches their distribution (with two per cell it
    becomes singular at this resolution and time, and the FP64 oracle's direct
    solve fails)."""
    n = 128
    dt = 0.5 / n
    steps = int(round(0.25 / dt))
    err = {}
    for method in ns.ASSIGN:
        prob, a = tg_problem(n, 4, seed=11)
        ctx = B.Context(0)
        try:
            x, y, vel, _, reps = gpu_steps(B, ctx, prob, a, method, dt, steps)
        finally:
            ctx.close()
        assert not (reps[2].flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN))
        err[method] = rel_l2(vel, ns.taylor_green(x.astype(np.float64), y.astype(np.float64),
                                                  steps * dt))
    say(f"[ns 128x128, T = 0.25] L2 error FLIP {err['flip']:.3e}, mass {err['mass']:.3e}")
    assert err["mass"] < 0.4 * err["flip"]
    assert err["mass"] < 0.025


def test_argument_errors(B):
    prob, a = tg_problem(16, 1, seed=1)
    ctx = B.Context(0)
    try:
        d = B.particles_from(prob, dtype=torch.float32)
        vel = torch.as_tensor(a).cuda()
        with pytest.raises(B.P2MError):
            B.p2m_ns_step(ctx, d, vel, 5, 0.01, NU)
        with pytest.raises(B.P2MError):
            B.p2m_ns_step(ctx, d, vel, B.NS_FLIP, -0.01, NU)
        with pytest.raises(B.P2MError):
            B.p2m_ns_step(ctx, d, vel, B.NS_FLIP, 0.01, NU, B.solve_opts(start=B.START_USER))
        rect = dict(prob, lx=2.0)
        with pytest.raises(B.P2MError):
            B.p2m_ns_step(ctx, B.particles_from(rect, dtype=torch.float32), vel, B.NS_FLIP, 0.01, NU)
    finally:
        ctx.close()


@pytest.mark.parametrize("n,fft", [(2, True), (3, True), (3, False), (4, True), (6, True),
                                   (6, False), (2, False)])
def test_tiny_meshes_against_the_oracle(B, n, fft):
    """Meshes of 2 to 6 nodes a side (a node's periodic neighbours repeat at 2), by the
    FFT (3 and 6 by Bluestein's algorithm) and by the solver, both assignments, one
    step."""
    for method in ns.ASSIGN:
        prob, a = tg_problem(n, 4, seed=40 + n)
        dt = 0.5 / n
        ctx = B.Context(0)
        try:
            ctx.set_fft(fft)
            x, y, vel, mv, reps = gpu_steps(B, ctx, prob, a, method, dt, 1)
        finally:
            ctx.close()
        for r in reps:
            assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN | B.FLAG_RANGE | B.FLAG_NONFINITE))
        new, a_ref, U_ref = ns.step(f64(prob), a.astype(np.float64), method, dt, NU)
        eU = rel_l2(mv, U_ref)
        ex = max(torus_dist(x, new["x"]).max(), torus_dist(y, new["y"]).max())
        say(f"[ns tiny {n}x{n} {method}] mesh velocity rel l2 {eU:.2e}, positions {ex:.2e}")
        assert eU <= 5e-6 and ex <= 2e-7


def test_no_particles_and_invalid_particles(B):
    """No particle: the mesh velocity is 0 and nothing is written to the particles.  A
    particle with a non-finite position is flagged and gets NaN velocity and position;
    the others get the results of the run without it, to rounding (one more particle
    can change the order of the floating-point sums)."""
    prob, a = tg_problem(16, 2, seed=21)
    ctx = B.Context(0)
    try:
        empty = dict(prob, x=np.zeros(0, np.float32), y=np.zeros(0, np.float32))
        d0 = B.particles_from(empty, dtype=torch.float32)
        v0 = torch.zeros((2, 0), dtype=torch.float32, device="cuda")
        mv = torch.full((2, 256), 7.0, dtype=torch.float32, device="cuda")
        _, reps = B.p2m_ns_step(ctx, d0, v0, B.NS_FLIP, 0.01, NU, mesh_vel=mv)
        torch.cuda.synchronize()
        assert torch.count_nonzero(mv).item() == 0
        bad = dict(prob, x=np.concatenate([prob["x"], np.array([np.nan], np.float32)]),
                   y=np.concatenate([prob["y"], np.array([0.5], np.float32)]))
        abad = np.concatenate([a, np.zeros((2, 1), np.float32)], axis=1)
        x1, y1, v1, _, r1 = gpu_steps(B, ctx, bad, abad, "flip", 1.0 / 32, 1)
        x2, y2, v2, _, _ = gpu_steps(B, ctx, prob, a, "flip", 1.0 / 32, 1)
    finally:
        ctx.close()
    assert r1[0].flags & B.FLAG_NONFINITE
    assert np.isnan(v1[:, -1]).all() and np.isnan(x1[-1]) and np.isnan(y1[-1])
    assert np.abs(v1[:, :-1] - v2).max() <= 1e-6
    assert max(torus_dist(x1[:-1], x2).max(), torus_dist(y1[:-1], y2).max()) <= 1e-7
