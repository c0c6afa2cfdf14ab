"""GPU tests of the batched mass assignment (p2m_mass_assign_batched): many
independent 2D FP32 problems of uneven size in one graph launch.

Parity bar: every instance's nodal values and report equal, bit for bit, those of
p2m_mass_assign on that instance alone (same binning, same scatter order, same
solver arithmetic and reduction order), and every instance matches the FP64 oracle
at relative l2 <= 1e-6.  Cases: ragged meshes smaller and larger than one solver
tile, F = 1, 2, 3, an instance without particles, an instance with out-of-range
particles, a user start, an iteration cap, the cached graph relaunched on changed
values, and the 64-instance uneven workload (sides log-uniform in [32, 512], 2 to
16 particles per cell, Taylor-Green u, v).
"""
import sys
import time

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


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context(0)


def f64(prob):
    return dict(prob, x=np.asarray(prob["x"], np.float64), y=np.asarray(prob["y"], np.float64))


def tg_instance(seed, nx, ny, ppc, F, lx=2 * np.pi, ly=2 * np.pi):
    x, y = wl.stratified_2d(seed, nx, ny, ppc, lx, ly)
    vals = wl.taylor_green(x * (2 * np.pi / lx), y * (2 * np.pi / ly))
    extra = np.sin(3 * x / lx * 2 * np.pi + 0.3)[None, :]
    vals = np.concatenate([vals, extra])[:F]
    prob = dict(dim=2, nx=nx, ny=ny, lx=lx, ly=ly, x=wl.to_f32_positions(x, lx),
                y=wl.to_f32_positions(y, ly), vol=None)
    return prob, vals.astype(np.float32)


def run_single(B, ctx, prob, vals, opts, x0=None):
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    out, rep = B.p2m_mass_assign(ctx, d, v, opts, x0=x0)
    torch.cuda.synchronize()
    return out.cpu(), B.read_report(rep, vals.shape[0])


def same_report(a, b):
    return (np.array_equal(a.iters, b.iters) and np.array_equal(a.refines, b.refines)
            and np.array_equal(a.rel_residual, b.rel_residual) and a.flags == b.flags
            and a.n_orphan == b.n_orphan and a.n_invalid == b.n_invalid)


def check_batch(B, ctx, insts, opts, oracle=True, x0=None, label=""):
    probs = [B.particles_from(p, dtype=torch.float32) for p, _ in insts]
    vals = [torch.as_tensor(v).cuda() for _, v in insts]
    say(f"[batched {label}] {len(insts)} instances, F={insts[0][1].shape[0]}, sides "
        f"{[p['nx'] for p, _ in insts][:8]}...")
    outs, bt = B.p2m_mass_assign_batched(ctx, probs, vals, opts, x0=x0)
    torch.cuda.synchronize()
    reps = bt.reports()
    worst = 0.0
    for k, (prob, v) in enumerate(insts):
        single, rs = run_single(B, ctx, prob, v, opts,
                                x0=None if x0 is None else x0[k])
        got = outs[k].cpu()
        assert torch.equal(got, single), f"instance {k}: batched != single"
        assert same_report(reps[k], rs), (k, reps[k], rs)
        if oracle and len(prob["x"]) > 0:
            ref, _ = p1.mass_assign(f64(prob), v.astype(np.float64), solver="direct")
            for f in range(v.shape[0]):
                e = metrics.rel_l2(got.numpy()[f].astype(np.float64), ref[f])
                worst = max(worst, e)
                assert e <= 1e-6, (k, f, e)
    say(f"  bitwise equal to single-problem runs; worst rel_l2 vs oracle {worst:.2e}")
    return outs, bt, reps


def test_batched_ragged_f2(B, ctx):
    insts = [tg_instance(40 + i, nx, ny, ppc, 2)
             for i, (nx, ny, ppc) in enumerate([(33, 47, 3), (128, 32, 4), (129, 33, 2),
                                                 (200, 90, 5), (64, 64, 8), (20, 150, 6)])]
    check_batch(B, ctx, insts, B.solve_opts(tol=1e-9, maxit=1000, max_refine=10), label="ragged")


@pytest.mark.parametrize("F", [1, 3])
def test_batched_field_counts(B, ctx, F):
    insts = [tg_instance(60 + F + i, n, n, 4, F) for i, n in enumerate([48, 160, 97])]
    check_batch(B, ctx, insts, B.solve_opts(tol=1e-8, maxit=1000, max_refine=10), label=f"F={F}")


def test_batched_degenerate_instances(B, ctx):
    """An instance without particles (every node an orphan, result 0) and one with
    out-of-range and non-finite positions: each flag lands in its own report only."""
    empty = (dict(dim=2, nx=40, ny=30, lx=1.0, ly=1.0, x=np.zeros(0, np.float32),
                  y=np.zeros(0, np.float32), vol=None), np.zeros((2, 0), np.float32))
    bad_p, bad_v = tg_instance(71, 50, 50, 3, 2)
    bad_p["x"] = bad_p["x"].copy()
    bad_p["x"][5] = np.float32(3 * np.pi)      # beyond L + h
    bad_p["x"][77] = np.float32(np.nan)
    good = tg_instance(72, 70, 40, 4, 2)
    outs, bt, reps = check_batch(B, ctx, [empty, (bad_p, bad_v), good],
                                 B.solve_opts(tol=1e-8, maxit=1000, max_refine=10),
                                 oracle=False, label="degenerate")
    assert torch.count_nonzero(outs[0]) == 0
    assert reps[0].n_orphan == 40 * 30 and reps[0].flags & B.FLAG_ORPHAN
    assert reps[1].n_invalid == 2 and reps[1].flags & B.FLAG_RANGE and reps[1].flags & B.FLAG_NONFINITE
    assert reps[2].n_invalid == 0 and not (reps[2].flags & (B.FLAG_RANGE | B.FLAG_NONFINITE))
    # the valid particles of the bad instance still match the oracle
    ref, _ = p1.mass_assign(f64(bad_p), bad_v.astype(np.float64), solver="direct")
    got = outs[1].cpu().numpy().astype(np.float64)
    for f in range(2):
        assert metrics.rel_l2(got[f], ref[f]) <= 1e-6


def test_batched_user_start_and_iteration_cap(B, ctx):
    insts = [tg_instance(80 + i, n, n, 3, 2) for i, n in enumerate([64, 130])]
    x0 = [torch.full((2, p["nx"] * p["ny"]), 0.25, dtype=torch.float32, device="cuda")
          for p, _ in insts]
    check_batch(B, ctx, insts, B.solve_opts(tol=1e-8, maxit=1000, max_refine=10,
                                            start=B.START_USER), x0=x0, label="user start")
    _, _, reps = check_batch(B, ctx, insts, B.solve_opts(tol=1e-12, maxit=3, max_refine=10),
                             oracle=False, label="maxit 3")
    for r in reps:
        assert r.flags & B.FLAG_NOT_CONVERGED and np.all(r.iters[:2] <= 3)


def test_batched_graph_relaunch(B, ctx):
    """Second and third launches reuse the cached graph: identical results on the
    same inputs, and results that follow values changed in place."""
    insts = [tg_instance(90 + i, n, n, 4, 2) for i, n in enumerate([96, 200, 40])]
    probs = [B.particles_from(p, dtype=torch.float32) for p, _ in insts]
    vals = [torch.as_tensor(v).cuda() for _, v in insts]
    opts = B.solve_opts(tol=1e-8, maxit=1000, max_refine=10)
    bt = B.Batch(ctx, probs, vals, opts)
    first = [o.clone() for o in bt.run()]
    second = [o.clone() for o in bt.run()]
    torch.cuda.synchronize()
    for a, b in zip(first, second):
        assert torch.equal(a, b)
    for v in bt.values:
        v.mul_(-0.5).add_(0.125)
    third = bt.run()
    torch.cuda.synchronize()
    for k, (p, _) in enumerate(insts):
        single, rs = run_single(B, ctx, p, bt.values[k].cpu().numpy(), opts)
        assert torch.equal(third[k].cpu(), single)
        assert same_report(bt.reports()[k], rs)


def test_batched_argument_errors(B, ctx):
    import ctypes
    L = B.lib()
    p, v = tg_instance(99, 32, 32, 2, 2)
    d = B.particles_from(p, dtype=torch.float32)
    n = ctypes.c_size_t()
    one = (B.CProblem * 1)(d.cstruct())
    assert L.p2m_batch_workspace_size(ctx.handle, one, 1, 4, ctypes.byref(n)) == 2     # F > 3
    assert L.p2m_batch_workspace_size(ctx.handle, one, 1, 9, ctypes.byref(n)) == 1
    assert L.p2m_batch_workspace_size(ctx.handle, one, 0, 2, ctypes.byref(n)) == 1
    many = (B.CProblem * 129)(*([d.cstruct()] * 129))
    assert L.p2m_batch_workspace_size(ctx.handle, many, 129, 1, ctypes.byref(n)) == 2
    d64 = B.particles_from(p, dtype=torch.float64)
    assert L.p2m_batch_workspace_size(ctx.handle, (B.CProblem * 1)(d64.cstruct()), 1, 2,
                                      ctypes.byref(n)) == 2
    assert L.p2m_batch_workspace_size(ctx.handle, one, 1, 2, ctypes.byref(n)) == 0
    vals = torch.as_tensor(v).cuda()
    out = torch.empty((2, 32 * 32), dtype=torch.float32, device="cuda")
    reps = torch.zeros((1, 144), dtype=torch.uint8, device="cuda")
    ws = torch.empty(int(n.value), dtype=torch.uint8, device="cuda")
    vp = (ctypes.c_void_p * 1)(vals.data_ptr())
    op = (ctypes.c_void_p * 1)(out.data_ptr())
    opts = B.solve_opts()
    args = lambda nbytes, r: (ctx.handle, one, 1, vp, 2, ctypes.byref(opts), op,
                              ctypes.c_void_p(r), ctypes.c_void_p(ws.data_ptr()),
                              ctypes.c_size_t(nbytes), None)
    assert L.p2m_mass_assign_batched(*args(ws.numel() - 1, reps.data_ptr())) == 3
    assert L.p2m_mass_assign_batched(*args(ws.numel(), 0)) == 1
    bad = B.solve_opts(start=B.START_DELTA1D)
    assert L.p2m_mass_assign_batched(ctx.handle, one, 1, vp, 2, ctypes.byref(bad), op,
                                     ctypes.c_void_p(reps.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), None) == 2
    torch.cuda.synchronize()


# ----------------------------------------------------------------------------
# the uneven workload: 64 instances, sides log-uniform in [32, 512], 2-16 ppc, F = 2
# ----------------------------------------------------------------------------
def test_uneven_batch_64(B, ctx):
    insts = wl.uneven_batch(seed=3, count=64)
    say(f"[config uneven64] {len(insts)} instances, sum nodes "
        f"{sum(p['nx'] * p['ny'] for p, _ in insts)}, sum particles "
        f"{sum(len(p['x']) for p, _ in insts)}")
    probs = [B.particles_from(p, dtype=torch.float32) for p, _ in insts]
    vals = [torch.as_tensor(v).cuda() for _, v in insts]
    # residual target 1e-9: the 2-particles-per-cell instances are ill-conditioned
    # enough that a 1e-8 residual leaves up to ~2e-6 error against the oracle
    opts = B.solve_opts(tol=1e-9, inner_rtol=1e-4, maxit=2000, max_refine=10)
    bt = B.Batch(ctx, probs, vals, opts)
    bt.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps_n = 5
    for _ in range(reps_n):
        bt.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps_n
    say(f"  batched: {dt * 1e3:.3f} ms per batch, {2 * len(insts) / dt:.0f} projections/s")
    reps = bt.reports()
    worst, worst_inf = 0.0, 0.0
    for k, (prob, v) in enumerate(insts):
        got = bt.out[k].cpu()
        single, rs = run_single(B, ctx, prob, v, opts)
        assert torch.equal(got, single), f"instance {k}"
        assert same_report(reps[k], rs), k
        assert np.all(reps[k].rel_residual[:2] <= 1e-9) and not (reps[k].flags & B.FLAG_NOT_CONVERGED)
        pr = f64(prob)
        st = p1.assemble_stencil(pr, v.astype(np.float64))
        M = p1.regularised_matrix(p1.stencil_matrix(pr, st), st["w"])
        for f in range(2):
            x, _ = p1.cg_fp64(M, st["b"][f], rtol=1e-12)
            e = metrics.rel_l2(got.numpy()[f].astype(np.float64), x)
            worst = max(worst, e)
            worst_inf = max(worst_inf, metrics.rel_linf(got.numpy()[f].astype(np.float64), x))
            assert e <= 1e-6, (k, f, e)
    say(f"  all 64 bitwise equal to single runs; worst rel_l2 {worst:.2e}, rel_linf {worst_inf:.2e}")


def test_batched_tune_plan(B, tmp_path):
    """p2m_tune_batched times the inner_rtol candidates on a batch, stores the fastest
    converged plan for the batch's shape class, later runs apply it (the tuned bits
    again), each instance equals the single-problem call with the plan's inner_rtol
    bit for bit, and a saved plan reloads into a fresh context."""
    tctx = B.Context(0)
    insts = [tg_instance(130 + i, n, m, ppc, 3) for i, (n, m, ppc) in
             enumerate([(128, 96, 8), (200, 120, 4), (64, 64, 2), (150, 150, 8)])]
    probs = [B.particles_from(p, dtype=torch.float32) for p, _ in insts]
    vals = [torch.as_tensor(v).cuda() for _, v in insts]
    opts = B.solve_opts(tol=1e-8, inner_rtol=1e-4, maxit=1000, max_refine=10)
    bt = B.Batch(tctx, probs, vals, opts)
    assert bt.plan() is None
    plan = bt.tune()
    tuned = [o.clone() for o in bt.out]
    torch.cuda.synchronize()
    say(f"[batched tune] chosen {plan}")
    assert plan.solver == B.SOLVER_TILES and plan.groups == 0 and plan.scatter_tile == 0
    assert plan.time_ms > 0.0 and plan.inner_rtol < 1.0
    got = bt.plan()
    assert got is not None and got.inner_rtol == plan.inner_rtol
    reps = bt.reports()
    for r in reps:
        assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN))
    again = bt.run()
    torch.cuda.synchronize()
    for a, b in zip(again, tuned):
        assert torch.equal(a, b)
    rt = plan.inner_rtol if plan.inner_rtol >= 0.0 else opts.inner_rtol
    sopts = B.solve_opts(tol=1e-8, inner_rtol=rt, maxit=1000, max_refine=10)
    for k, (prob, v) in enumerate(insts):
        single, rs = run_single(B, tctx, prob, v, sopts)
        assert torch.equal(tuned[k].cpu(), single), k
        assert same_report(reps[k], rs), (k, reps[k], rs)
        ref, _ = p1.mass_assign(f64(prob), v.astype(np.float64), solver="direct")
        for f in range(3):
            assert metrics.rel_l2(single.numpy()[f].astype(np.float64), ref[f]) <= 1e-6
    path = tmp_path / "batch_plans.json"
    tctx.save_plans(path)
    text = path.read_text()
    say("  " + text.strip().replace("\n", " "))
    assert '"batch-f32-F3-n' in text
    ctx2 = B.Context(0)
    ctx2.load_plans(path)
    bt2 = B.Batch(ctx2, probs, vals, opts)
    assert bt2.plan().inner_rtol == plan.inner_rtol
    # another batch (one instance fewer) is another shape class
    assert B.Batch(ctx2, probs[:3], vals[:3], opts).plan() is None
    out2 = bt2.run()
    torch.cuda.synchronize()
    for a, b in zip(out2, tuned):
        assert torch.equal(a, b)
    # plans off: the caller's inner_rtol again
    ctx2.use_plans(False)
    out3 = bt2.run()
    torch.cuda.synchronize()
    for k, (prob, v) in enumerate(insts):
        single, _ = run_single(B, ctx2, prob, v, opts)
        assert torch.equal(out3[k].cpu(), single), k
    # the tuner needs a start it can repeat
    bt_user = B.Batch(tctx, probs, vals, B.solve_opts(tol=1e-6, start=B.START_USER))
    with pytest.raises(B.P2MError):
        bt_user.tune()


def test_batched_at_capacity(B, ctx):
    """128 instances x 2 fields = 256 (instance, field) pairs, the batch limits: every
    instance equals its single-problem run bit for bit; a few against the oracle."""
    g = np.random.Generator(np.random.PCG64(404))
    sides = g.integers(12, 48, size=(128, 2))
    ppcs = g.integers(2, 6, size=128)
    insts = [tg_instance(500 + i, int(nx), int(ny), int(pc), 2)
             for i, ((nx, ny), pc) in enumerate(zip(sides, ppcs))]
    say(f"[batched capacity] 128 instances, sides {int(sides.min())}..{int(sides.max())}")
    probs = [B.particles_from(p, dtype=torch.float32) for p, _ in insts]
    vals = [torch.as_tensor(v).cuda() for _, v in insts]
    opts = B.solve_opts(tol=1e-8, maxit=1000, max_refine=10)
    outs, bt = B.p2m_mass_assign_batched(ctx, probs, vals, opts)
    torch.cuda.synchronize()
    reps = bt.reports()
    for k, (prob, v) in enumerate(insts):
        assert not (reps[k].flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN)), (k, reps[k])
        single, rs = run_single(B, ctx, prob, v, opts)
        assert torch.equal(outs[k].cpu(), single), k
        assert same_report(reps[k], rs), (k, reps[k], rs)
    for k in (0, 63, 127):
        prob, v = insts[k]
        ref, _ = p1.mass_assign(f64(prob), v.astype(np.float64), solver="direct")
        for f in range(2):
            assert metrics.rel_l2(outs[k].cpu().numpy()[f].astype(np.float64), ref[f]) <= 1e-6
    say("  bitwise equal to single-problem runs")
