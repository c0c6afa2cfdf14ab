"""The register-resident solves (diagonal and Chebyshev preconditioners) on the
paths where fields of one call end at different points of the FP64 iterative
refinement: a field with b = 0 (its result is 0 whatever the start), a field the
start already solves (done at the first residual evaluation, before any CG
iteration), fields that need one or many refinements (the correction of each
inner solve is folded into x inside the next residual evaluation, and the
boundary of x alternates between two exchange planes), and a refinement cap of 0.
Every result is checked against the FP64 oracle (Sec. 2.4 under the particle
quadrature) at the FP32 gate, or bit for bit where it is fixed exactly."""
import sys
import zlib

import numpy as np
import pytest

from oracle import metrics
from oracle import p1
from paper_1610_05258_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SOLVERS = ("resident", "chebyshev")


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


def problem(name):
    if name == "tg256":
        return wl.taylor_green_2d(seed=31, n=256, ppc=6, steps=30, dt=2e-3)
    if name == "ragged":
        g = np.random.Generator(np.random.PCG64(zlib.crc32(name.encode())))
        nx, ny = 300, 70
        x = g.uniform(0, 2.0, nx * ny * 4)
        y = g.uniform(0, 0.5, nx * ny * 4)
        prob = dict(dim=2, nx=nx, ny=ny, lx=2.0, ly=0.5, x=x.astype(np.float32),
                    y=y.astype(np.float32), vol=None)
        return prob, g.normal(size=(3, x.size)).astype(np.float32)
    raise KeyError(name)


def oracle(prob, vals):
    pr = dict(prob, x=np.asarray(prob["x"], np.float64), y=np.asarray(prob["y"], np.float64))
    ref, _ = p1.mass_assign(pr, vals.astype(np.float64), solver="direct")
    return ref


def set_solver(B, ctx, solver):
    ctx.set_solver(B.SOLVER_RESIDENT if solver == "resident" else B.SOLVER_RESIDENT_CHEB)


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("name", ["tg256", "ragged"])
def test_fields_ending_at_different_refinements(B, solver, name):
    """Field 0 has b = 0 and a non-zero start: result 0, relative residual 0.
    Field 1 starts at 0.5 everywhere and needs the CG.  Field 2 starts at this
    solver's own result to 1e-9, which meets tol = 1e-7 at the first residual
    evaluation: its result is that start, bit for bit, after 0 iterations."""
    prob, vals = problem(name)
    vals = vals.copy()
    vals[0] = 0.0
    ref = oracle(prob, vals)
    say(f"[{solver}] {name}: nodes {prob['nx']}x{prob['ny']}, particles {vals.shape[1]}")
    ctx = B.Context(0)
    try:
        set_solver(B, ctx, solver)
        d = B.particles_from(prob, dtype=torch.float32)
        v = torch.as_tensor(vals).cuda()
        tight, _ = B.p2m_mass_assign(ctx, d, v, B.solve_opts(tol=1e-9, maxit=2000, max_refine=20))
        x0 = np.empty_like(ref, dtype=np.float32)
        x0[0] = 1.0
        x0[1] = 0.5
        x0[2] = tight[2].cpu().numpy()
        x0t = torch.as_tensor(x0).cuda()
        opts = B.solve_opts(tol=1e-7, maxit=2000, max_refine=20, start=B.START_USER)
        out, rep = B.p2m_mass_assign(ctx, d, v, opts, x0=x0t)
        torch.cuda.synchronize()
        r = B.read_report(rep, 3)
        got = out.cpu().numpy()
        say(f"  iters {r.iters[:3].tolist()} refines {r.refines[:3].tolist()} "
            f"relres {r.rel_residual[:3].tolist()} flags {r.flags}")
        assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN))
        assert np.all(got[0] == 0.0) and r.rel_residual[0] == 0.0 and r.iters[0] == 0
        assert r.iters[1] > 0 and r.refines[1] >= 2
        assert metrics.rel_l2(got[1].astype(np.float64), ref[1]) <= 1e-6
        assert r.iters[2] == 0 and r.refines[2] == 1
        assert np.array_equal(got[2], x0[2])
    finally:
        ctx.close()


@pytest.mark.parametrize("solver", SOLVERS)
def test_many_refinements(B, solver):
    """A loose inner tolerance (1e-2) and a tight outer one (1e-10) take several
    refinements; the FP64 solution keeps improving through them."""
    prob, vals = problem("tg256")
    ref = oracle(prob, vals)
    ctx = B.Context(0)
    try:
        set_solver(B, ctx, solver)
        d = B.particles_from(prob, dtype=torch.float32)
        v = torch.as_tensor(vals).cuda()
        opts = B.solve_opts(tol=1e-10, inner_rtol=1e-2, maxit=5000, max_refine=40)
        out, rep = B.p2m_mass_assign(ctx, d, v, opts)
        out2, _ = B.p2m_mass_assign(ctx, d, v, opts)
        torch.cuda.synchronize()
        r = B.read_report(rep, 3)
        say(f"[{solver}] many refinements: iters {r.iters[:3].tolist()} refines {r.refines[:3].tolist()} "
            f"relres {r.rel_residual[:3].tolist()}")
        assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN))
        assert np.all(r.refines[:3] >= 4)
        assert np.all(r.rel_residual[:3] <= 1e-10)
        assert torch.equal(out, out2)
        for f in range(3):
            e = metrics.rel_l2(out[f].cpu().numpy().astype(np.float64), ref[f])
            assert e <= 1e-6, (f, e)
    finally:
        ctx.close()


@pytest.mark.parametrize("solver", SOLVERS)
def test_refinement_cap_zero(B, solver):
    """max_refine = 0: every field ends at the first residual evaluation with the
    FLIP start b / w as its result (0 at orphan nodes), no CG iteration, and the
    not-converged flag."""
    prob, vals = problem("ragged")
    pr = dict(prob, x=np.asarray(prob["x"], np.float64), y=np.asarray(prob["y"], np.float64))
    st = p1.assemble_stencil(pr, vals.astype(np.float64))
    w = st["w"]
    flip = np.where(w > 0, st["b"] / np.where(w > 0, w, 1.0), 0.0)
    ctx = B.Context(0)
    try:
        set_solver(B, ctx, solver)
        d = B.particles_from(prob, dtype=torch.float32)
        v = torch.as_tensor(vals).cuda()
        opts = B.solve_opts(tol=1e-8, maxit=100, max_refine=0, start=B.START_FLIP)
        out, rep = B.p2m_mass_assign(ctx, d, v, opts)
        torch.cuda.synchronize()
        r = B.read_report(rep, 3)
        assert r.flags & B.FLAG_NOT_CONVERGED
        assert np.all(r.iters[:3] == 0) and np.all(r.refines[:3] == 1)
        got = out.cpu().numpy().astype(np.float64)
        for f in range(3):
            assert metrics.rel_l2(got[f], flip[f]) <= 1e-6
    finally:
        ctx.close()
