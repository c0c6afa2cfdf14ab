"""GPU tests of the solver choices and the autotuner: the tile-streaming solve gives
the resident solve's bits on a mesh both can take, solves a mesh beyond the resident
kernel's capacity to the oracle's gate, and p2m_tune picks, stores, saves and reloads
a plan that later calls apply."""
import sys

import numpy as np
import pytest

from oracle import metrics
from oracle import p1
from paper_1610_05258_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def f64(prob):
    return dict(prob, x=np.asarray(prob["x"], np.float64), y=np.asarray(prob["y"], np.float64))


def tg(n, ny=None, ppc=4, seed=5, F=3):
    ny = ny or n
    x, y = wl.stratified_2d(seed, n, ny, ppc, 2 * np.pi, 2 * np.pi)
    x, y = wl.tg_advect_rk2(x, y, 20, 2e-3)
    vals = wl.taylor_green(x, y)[:F]
    prob = dict(dim=2, nx=n, ny=ny, lx=2 * np.pi, ly=2 * np.pi, x=wl.to_f32_positions(x, 2 * np.pi),
                y=wl.to_f32_positions(y, 2 * np.pi), vol=None)
    return prob, vals.astype(np.float32)


def test_tiles_equal_resident_bitwise(B):
    ctx = B.Context(0)
    prob, vals = tg(200, 150, ppc=3)
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    opts = B.solve_opts(tol=1e-9, maxit=1000, max_refine=10)
    outs, reps = [], []
    for kind in (B.SOLVER_RESIDENT, B.SOLVER_TILES):
        ctx.set_solver(kind)
        o, r = B.p2m_mass_assign(ctx, d, v, opts)
        torch.cuda.synchronize()
        outs.append(o.cpu())
        reps.append(B.read_report(r, 3))
    say(f"[tiles] resident iters {reps[0].iters.tolist()} tiles iters {reps[1].iters.tolist()}")
    assert torch.equal(outs[0], outs[1])
    assert np.array_equal(reps[0].iters, reps[1].iters)
    assert np.array_equal(reps[0].rel_residual, reps[1].rel_residual)


def test_tiles_beyond_resident_capacity(B):
    """1536 x 768 nodes = 288 solver tiles, more than one per compute unit: AUTO takes
    the tile-streaming kernel (workgroups own several tiles)."""
    ctx = B.Context(0)
    prob, vals = tg(1536, 768, ppc=2, seed=8, F=2)
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    opts = B.solve_opts(tol=1e-9, maxit=2000, max_refine=10)
    out, rep = B.p2m_mass_assign(ctx, d, v, opts)
    torch.cuda.synchronize()
    r = B.read_report(rep, 2)
    say(f"[tiles 1536x768] iters {r.iters.tolist()} relres {r.rel_residual.tolist()} flags {r.flags}")
    assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN))
    pr = f64(prob)
    st = p1.assemble_stencil(pr, vals.astype(np.float64))
    M = p1.regularised_matrix(p1.stencil_matrix(pr, st), st["w"])
    got = out.cpu().numpy().astype(np.float64)
    xs = [p1.cg_fp64(M, st["b"][f], rtol=1e-12)[0] for f in range(2)]
    # the grid-synchronised kernel solves the same system to the same gate
    ctx.set_solver(B.SOLVER_STREAMING)
    out2, rep2 = B.p2m_mass_assign(ctx, d, v, opts)
    torch.cuda.synchronize()
    r2 = B.read_report(rep2, 2)
    got2 = out2.cpu().numpy().astype(np.float64)
    for f in range(2):
        e1, e2 = metrics.rel_l2(got[f], xs[f]), metrics.rel_l2(got2[f], xs[f])
        say(f"  field {f}: tiles rel_l2 {e1:.2e}; streaming rel_l2 {e2:.2e} (iters {r2.iters[f]}, "
            f"relres {r2.rel_residual[f]:.1e})")
        assert e1 <= 1e-6 and e2 <= 1e-6


def test_tune_store_save_load(B, tmp_path):
    ctx = B.Context(0)
    prob, vals = tg(192, ppc=4, seed=9)
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    opts = B.solve_opts(tol=1e-8, maxit=1000, max_refine=10)
    assert ctx.plan(d, 3) is None
    plan, tuned, rep = B.p2m_tune(ctx, d, v, opts)
    torch.cuda.synchronize()
    say(f"[tune 192^2 F=3] chosen {plan}")
    assert plan.solver in (B.SOLVER_STREAMING, B.SOLVER_RESIDENT, B.SOLVER_TILES,
                           B.SOLVER_RESIDENT_CHEB)
    assert plan.scatter_tile in (0, 8) and plan.time_ms > 0.0
    got = ctx.plan(d, 3)
    assert got is not None and (got.solver, got.groups, got.scatter_tile, got.inner_rtol) == (
        plan.solver, plan.groups, plan.scatter_tile, plan.inner_rtol)
    # a later call applies the plan: the tuned result again, bit for bit
    again, _ = B.p2m_mass_assign(ctx, d, v, opts)
    torch.cuda.synchronize()
    assert torch.equal(again, tuned)
    ref, _ = p1.mass_assign(f64(prob), vals.astype(np.float64), solver="direct")
    for f in range(3):
        assert metrics.rel_l2(tuned.cpu().numpy()[f].astype(np.float64), ref[f]) <= 1e-6
    # persisted plans: a fresh context applies the same plan
    path = tmp_path / "plans.json"
    ctx.save_plans(path)
    say("  " + path.read_text().strip().replace("\n", " "))
    ctx2 = B.Context(0)
    ctx2.load_plans(path)
    p2 = ctx2.plan(d, 3)
    assert (p2.solver, p2.groups, p2.scatter_tile, p2.inner_rtol) == (plan.solver, plan.groups,
                                                                      plan.scatter_tile, plan.inner_rtol)
    out2, _ = B.p2m_mass_assign(ctx2, d, v, opts)
    torch.cuda.synchronize()
    assert torch.equal(out2, tuned)
    # a different shape class has no plan; clearing forgets
    d_small = B.particles_from(tg(64, ppc=4)[0], dtype=torch.float32)
    assert ctx2.plan(d_small, 3) is None
    ctx2.clear_plans()
    assert ctx2.plan(d, 3) is None
    bad = tmp_path / "bad.json"
    bad.write_text('{\n  "2d-f32-F3-nx8-ny8-ppc2": {"solver": 9, "groups": 0, "scatter_tile": 0, '
                   '"inner_rtol": -1, "time_ms": 1}\n}\n')
    with pytest.raises(B.P2MError):
        ctx2.load_plans(bad)
    assert ctx2.plan(d, 3) is None
