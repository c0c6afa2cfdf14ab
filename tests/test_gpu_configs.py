"""GPU parity on the named workloads, at their real sizes:

* the 1D top-hat (64 elements, 256 particles, FP64): delta, FLIP, mass, M2P against
  the oracle at 1e-12, plus the paper's invariants checked on the GPU results;
* Zalesak's slotted disk (256^2, 4 ppc, FP32): 100 steps of rotate -> mass_assign
  -> M2P on the GPU, with per-step parity against the oracle on the same step
  inputs at sampled steps;
* Taylor-Green 1024^2, 8 ppc, F = 3 (the benchmark's configuration and launch
  options): full binning bit-exact, the assembled system and the mass assignment
  against the FP64 oracle, and the preservation property at full size.
"""
import math
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
def ctx(B):
    return B.Context(0)


def f64(prob):
    out = dict(prob)
    for k in ("x", "y", "vol"):
        if out.get(k) is not None:
            out[k] = np.asarray(out[k]).astype(np.float64)
    return out


# ----------------------------------------------------------------------------
# 1D top-hat
# ----------------------------------------------------------------------------
def test_tophat_1d_methods_and_invariants(B, ctx):
    say("[config tophat1d] 64 elements, 256 particles, FP64")
    prob, vals = wl.tophat_1d(seed=0)
    d = B.particles_from(prob, dtype=torch.float64)
    v = torch.as_tensor(vals).cuda()
    vmu = np.full(vals.shape[1], 1.0 / vals.shape[1])
    delta, _ = B.p2m_assign(ctx, d, B.DELTA, v)
    flip, rf = B.p2m_assign(ctx, d, B.FLIP, v)
    mass, rm = B.p2m_mass_assign(ctx, d, v, B.solve_opts(tol=1e-14, maxit=500, max_refine=10, fp64=True))
    back, _ = B.p2m_interpolate(ctx, d, mass)
    b, w, coef, _ = B.p2m_assemble(ctx, d, v)
    torch.cuda.synchronize()
    assert metrics.rel_l2(delta.cpu().numpy()[0], p1.delta_1d(prob, vals)[0]) <= 1e-12
    ref_flip, _ = p1.flip(prob, vals)
    ref_mass, a = p1.mass_assign(prob, vals, solver="direct")
    assert metrics.rel_l2(flip.cpu().numpy()[0], ref_flip[0]) <= 1e-12
    assert metrics.rel_l2(mass.cpu().numpy()[0], ref_mass[0]) <= 1e-12
    m = mass.cpu().numpy()[0]
    wg = w.cpu().numpy()
    A = vals[0]
    # conservativity (FLIP and mass, against w) and stability on the GPU outputs
    assert abs(np.sum(wg * flip.cpu().numpy()[0]) - np.sum(vmu * A)) < 1e-13
    assert abs(np.sum(wg * m) - np.sum(vmu * A)) < 1e-12
    Mg = p1.stencil_matrix(prob, dict(D=coef[0].cpu().numpy(), E=coef[1].cpu().numpy()))
    assert m @ (Mg @ m) <= np.sum(vmu * A * A) * (1 + 1e-12)
    # conservation through M2P: sum v Abarbar = sum w Abar
    assert abs(np.sum(vmu * back.cpu().numpy()[0]) - np.sum(wg * m)) < 1e-13
    # preservation: interpolate a nodal field, mass-assign it back
    nodal = torch.as_tensor(np.cos(2 * np.pi * np.arange(64) / 64)[None, :] + 0.1).cuda()
    part, _ = B.p2m_interpolate(ctx, d, nodal)
    again, _ = B.p2m_mass_assign(ctx, d, part, B.solve_opts(tol=1e-14, maxit=500, max_refine=10, fp64=True))
    torch.cuda.synchronize()
    w_np = wg
    live = w_np > 0
    assert np.max(np.abs(again.cpu().numpy()[0, live] - nodal.cpu().numpy()[0, live])) < 1e-11


# ----------------------------------------------------------------------------
# Zalesak's slotted disk, 100 steps
# ----------------------------------------------------------------------------
def test_zalesak_100_steps(B, ctx):
    say("[config zalesak] 256x256, 4 ppc, 100 steps of rotate -> mass_assign -> M2P (FP32)")
    prob, a0, x64, y64 = wl.zalesak_2d(seed=1, n=256, ppc=4)
    A = torch.as_tensor(a0).cuda()
    opts = B.solve_opts(tol=1e-9, maxit=1000, max_refine=10)
    check_steps = {1, 2, 50, 100}
    worst = 0.0
    for step in range(1, 101):
        x64, y64 = wl.zalesak_rotate(x64, y64, wl.ZALESAK_DT)
        pk = dict(prob, x=x64.astype(np.float32), y=y64.astype(np.float32))
        d = B.particles_from(pk, dtype=torch.float32)
        a_in = A.clone()
        nodal, rep = B.p2m_mass_assign(ctx, d, a_in, opts)
        A, _ = B.p2m_interpolate(ctx, d, nodal)
        if step in check_steps:
            torch.cuda.synchronize()
            r = B.read_report(rep, 1)
            ref, _ = p1.mass_assign(f64(pk), a_in.cpu().numpy().astype(np.float64), solver="direct")
            e = metrics.rel_l2(nodal.cpu().numpy()[0], ref[0])
            ref_back = p1.interpolate(f64(pk), nodal.cpu().numpy().astype(np.float64))
            e2 = metrics.rel_l2(A.cpu().numpy()[0], ref_back[0])
            say(f"  step {step}: iters={r.iters[0]} relres={r.rel_residual[0]:.2e} "
                f"rel_l2(mass)={e:.2e} rel_l2(m2p)={e2:.2e}")
            worst = max(worst, e, e2)
            assert e <= 1e-6 and e2 <= 1e-6
    torch.cuda.synchronize()
    # full mass keeps the plateaus with small over/undershoots (Sec. 3.2)
    fin = A.cpu().numpy()[0]
    say(f"  after 100 steps: min {fin.min():.3f} max {fin.max():.3f}, worst parity {worst:.2e}")
    assert fin.min() > -0.5 and fin.max() < 1.5


# ----------------------------------------------------------------------------
# Taylor-Green 1024^2, 8 ppc, F = 3 (benchmark configuration)
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tg_full():
    say("[config tg1024] generating 1024x1024, 8 ppc, 50 RK2 steps")
    prob, vals = wl.taylor_green_2d(seed=2, n=1024, ppc=8, steps=50, dt=1e-3)
    return prob, vals


def test_tg1024_binning_bit_exact(B, ctx, tg_full):
    prob, vals = tg_full
    say("[config tg1024] p2m_bin vs stable argsort")
    d = B.particles_from(prob, dtype=torch.float32)
    perm, cs, _ = B.p2m_bin(ctx, d)
    torch.cuda.synchronize()
    loc = p1.locate(f64(prob))
    ref_perm, ref_cs = p1.bin_particles(loc["key"], loc["valid"], 1024 * 1024)
    assert np.array_equal(cs.cpu().numpy(), ref_cs)
    assert np.array_equal(perm.cpu().numpy(), ref_perm)


def test_tg1024_assemble_and_mass_assign(B, ctx, tg_full):
    """Same options as the benchmark (tol 1e-8, inner 1e-4)."""
    prob, vals = tg_full
    say("[config tg1024] p2m_assemble + p2m_mass_assign vs FP64 oracle")
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    b, w, coef, _ = B.p2m_assemble(ctx, d, v)
    opts = B.solve_opts(tol=1e-8, inner_rtol=1e-4, maxit=2000, max_refine=10)
    out, rep = B.p2m_mass_assign(ctx, d, v, opts)
    torch.cuda.synchronize()
    r = B.read_report(rep, 3)
    say(f"  iters={r.iters} refines={r.refines} relres={r.rel_residual} flags={r.flags}")
    pr = f64(prob)
    st = p1.assemble_stencil(pr, vals.astype(np.float64))
    for i, k in enumerate(("D", "E", "N", "NE")):
        e = metrics.rel_l2(coef[i].cpu().numpy(), st[k])
        say(f"  {k}: rel_l2 {e:.2e}")
        assert e <= 1e-6
    assert metrics.rel_l2(w.cpu().numpy(), st["w"]) <= 1e-6
    bg = b.cpu().numpy()
    for f in range(3):
        assert metrics.rel_l2(bg[f], st["b"][f]) <= 1e-6
    M = p1.regularised_matrix(p1.stencil_matrix(pr, st), st["w"])
    got = out.cpu().numpy()
    assert np.all(r.rel_residual <= 1e-8) and not (r.flags & B.FLAG_NOT_CONVERGED)
    for f in range(3):
        x, _ = p1.cg_fp64(M, st["b"][f], rtol=1e-12)
        e = metrics.rel_l2(got[f], x)
        say(f"  field {f}: rel_l2 {e:.2e} rel_linf {metrics.rel_linf(got[f], x):.2e}")
        assert e <= 1e-6


def test_tg1024_preservation(B, ctx, tg_full):
    """eq. (18) at full size: interpolate a nodal field, mass-assign it back."""
    prob, _ = tg_full
    say("[config tg1024] preservation: M2P then mass_assign returns the nodal values")
    d = B.particles_from(prob, dtype=torch.float32)
    n = 1024
    xs = np.arange(n) * (2 * math.pi / n)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    nodal = np.stack([np.sin(X) * np.cos(Y), np.cos(3 * X) + 0.5 * np.sin(2 * Y)]).reshape(2, -1)
    nd = torch.as_tensor(nodal.astype(np.float32)).cuda()
    part, _ = B.p2m_interpolate(ctx, d, nd)
    back, rep = B.p2m_mass_assign(ctx, d, part, B.solve_opts(tol=1e-9, inner_rtol=1e-4, maxit=2000,
                                                             max_refine=10))
    torch.cuda.synchronize()
    for f in range(2):
        e = metrics.rel_l2(back.cpu().numpy()[f], nd.cpu().numpy()[f])
        say(f"  field {f}: rel_l2 {e:.2e}")
        assert e <= 1e-6
