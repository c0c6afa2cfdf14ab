"""Bounded grid-barrier waits of the mass solves, forced from the host: with
P2M_OPT_SOLVE_SPIN < 0 every wait of a solve's grid barrier gives up at once, so each
solve kernel whose grid has several workgroups stops at its first barrier.  The call
must still end (every kernel runs to its end), raise P2M_FLAG_BREAKDOWN and
P2M_FLAG_NOT_CONVERGED, and return the FP64 solution the solve held, which is the FLIP
start b / w (Sec. 2.3 eqs. (11)-(12)); the next call with the default bound solves to
the FP64 oracle (Sec. 2.4 under the particle quadrature).  The streaming, resident,
Chebyshev and tile-streaming kernels and the batched graph each take this path."""
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


@pytest.fixture(scope="module")
def case():
    prob, vals = wl.taylor_green_2d(seed=17, n=256, ppc=4, steps=10, dt=2e-3)
    pr = dict(prob, x=np.asarray(prob["x"], np.float64), y=np.asarray(prob["y"], np.float64))
    ref, _ = p1.mass_assign(pr, vals.astype(np.float64), solver="direct")
    return prob, vals, ref


def kind_of(B, name):
    return dict(streaming=B.SOLVER_STREAMING, resident=B.SOLVER_RESIDENT,
                chebyshev=B.SOLVER_RESIDENT_CHEB, tiles=B.SOLVER_TILES)[name]


@pytest.mark.parametrize("solver", ["streaming", "resident", "chebyshev", "tiles"])
def test_solve_gives_up_when_forced(B, case, solver):
    prob, vals, ref = case
    say(f"[solve abort] {solver}: 256x256, {vals.shape[1]} particles, F = {vals.shape[0]}")
    ctx = B.Context(0)
    try:
        ctx.set_solver(kind_of(B, solver))
        d = B.particles_from(prob, dtype=torch.float32)
        v = torch.as_tensor(vals).cuda()
        opts = B.solve_opts(tol=1e-8, maxit=2000, max_refine=10)
        flip, _ = B.p2m_assign(ctx, d, B.FLIP, v)
        ctx.set_solve_spin(-1)
        out, rep = B.p2m_mass_assign(ctx, d, v, opts)
        torch.cuda.synchronize()
        r = B.read_report(rep, vals.shape[0])
        got = out.cpu().numpy()
        say(f"  forced: flags {r.flags:#x} iters {r.iters[:3].tolist()}")
        assert r.flags & B.FLAG_BREAKDOWN and r.flags & B.FLAG_NOT_CONVERGED
        assert np.all(np.isfinite(got))
        fl = flip.cpu().numpy().astype(np.float64)
        for f in range(vals.shape[0]):
            assert metrics.rel_l2(got[f].astype(np.float64), fl[f]) <= 1e-6
        ctx.set_solve_spin(0)
        out2, rep2 = B.p2m_mass_assign(ctx, d, v, opts)
        torch.cuda.synchronize()
        r2 = B.read_report(rep2, vals.shape[0])
        say(f"  default: flags {r2.flags:#x} iters {r2.iters[:3].tolist()}")
        assert not (r2.flags & (B.FLAG_BREAKDOWN | B.FLAG_NOT_CONVERGED))
        got2 = out2.cpu().numpy().astype(np.float64)
        for f in range(vals.shape[0]):
            assert metrics.rel_l2(got2[f], ref[f]) <= 1e-6
    finally:
        ctx.close()


def test_batched_solve_gives_up_when_forced(B):
    insts = []
    for k, n in enumerate((64, 160, 96)):
        x, y = wl.stratified_2d(30 + k, n, n, 4, 1.0, 1.0)
        vals = wl.taylor_green(2 * np.pi * x, 2 * np.pi * y)[:2].astype(np.float32)
        prob = dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=wl.to_f32_positions(x, 1.0),
                    y=wl.to_f32_positions(y, 1.0), vol=None)
        insts.append((prob, vals))
    ctx = B.Context(0)
    try:
        probs = [B.particles_from(p, dtype=torch.float32) for p, _ in insts]
        vals = [torch.as_tensor(v).cuda() for _, v in insts]
        opts = B.solve_opts(tol=1e-8, maxit=1000, max_refine=10)
        bt = B.Batch(ctx, probs, vals, opts)
        ctx.set_solve_spin(-1)
        out = [o.clone() for o in bt.run()]
        torch.cuda.synchronize()
        for k, r in enumerate(bt.reports()):
            say(f"[batch abort] instance {k}: flags {r.flags:#x}")
            assert r.flags & B.FLAG_BREAKDOWN and r.flags & B.FLAG_NOT_CONVERGED
            assert torch.isfinite(out[k]).all()
        ctx.set_solve_spin(0)
        bt.run()
        torch.cuda.synchronize()
        for k, r in enumerate(bt.reports()):
            assert not (r.flags & (B.FLAG_BREAKDOWN | B.FLAG_NOT_CONVERGED)), (k, r.flags)
    finally:
        ctx.close()
