"""GPU tests of the learned warm start against the FP64 oracle (oracle/mlp.py):
node features, the network's forward pass, its gradient (relative l2 <= 1e-2 on
the same BF16-rounded weights and inputs), the Adam step, training on solver
targets, and the learned start inside the mass solve, whose answer must still
meet the 1e-6 gate, with the FLIP fallback when the proposal is worse."""
import sys

import numpy as np
import pytest

from oracle import metrics
from oracle import mlp
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


@pytest.fixture(scope="module")
def case(B, ctx):
    """40 x 40 mesh, 6 ppc, disordered by 150 RK2 steps of 5e-3 (about 5 cells)."""
    prob, vals = wl.tg_disordered(11, n=40, ppc=6, steps=150, dt=5e-3)
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    X, base, scale = B.learned_features(ctx, d, v)
    torch.cuda.synchronize()
    pr = f64(prob)
    loc = p1.locate(pr)
    perm, cs = p1.bin_particles(loc["key"], loc["valid"], 40 * 40)
    a = p1.assemble(pr, vals.astype(np.float64), want_matrix=False)
    baseO = mlp.flip_base(a["b"], a["w"])
    XO, scaleO, count = mlp.node_features(pr, vals.astype(np.float64), baseO, a["w"],
                                          np.arange(40 * 40), loc, perm, cs)
    return dict(prob=prob, vals=vals, d=d, v=v, X=X, base=base, scale=scale, XO=XO, scaleO=scaleO,
                baseO=baseO, count=count)


def test_features_match_oracle(case):
    X = case["X"].float().cpu().numpy().astype(np.float64)
    XO = mlp.bf16(case["XO"])
    scale = case["scale"].cpu().numpy()
    scaleO = case["scaleO"]
    say(f"[learned features] usable {np.mean(scale > 0):.3f}, max count {case['count'].max()}")
    # offsets, count and padding: the same FP64 locate and roundings -> equal
    pos = np.ones(mlp.N_IN, bool)
    pos[2:3 * mlp.K_MAX:3] = False
    assert np.array_equal(X[:, :, pos], XO[:, :, pos])
    # value features (A - base) / s: one BF16 step, plus the FP32 rounding of the base
    # (b and w are FP32 sums on the GPU) carried through the division by s
    vg, vo = X[:, :, ~pos], XO[:, :, ~pos]
    amax = np.abs(case["vals"]).max()
    with np.errstate(divide="ignore"):
        carry = np.where(scaleO > 0, 16 * 2.0 ** -24 * (np.abs(case["baseO"].T) + amax) / scaleO, 0.0)
    bound = 2.0 ** -7 * np.maximum(np.abs(vo), np.abs(vg)) + carry[:, :, None] + 1e-30
    worst = np.max(np.abs(vg - vo) / bound)
    say(f"  value features: worst |gpu - oracle| / bound = {worst:.3f}")
    assert worst <= 1.0
    assert np.array_equal(scale > 0, scaleO > 0)
    use = scaleO > 0
    assert np.allclose(scale[use], scaleO[use], rtol=1e-5, atol=0)
    base = case["base"].cpu().numpy()
    assert np.allclose(base.T, case["baseO"], rtol=1e-5, atol=1e-6)


def rand_params(seed):
    g = np.random.default_rng(seed)
    th = mlp.init_params(seed).astype(np.float64)
    p = mlp.unpack(th)
    for k in ("b1", "b2", "b3"):
        p[k][:] = g.normal(0, 0.05, mlp.H)
    p["W4"][:] = g.normal(0, 0.2, mlp.H)
    p["b4"][0] = 0.1
    return th.astype(np.float32)


def usable_rows(case):
    use = (case["scale"].cpu().numpy() > 0).reshape(-1)
    Xr = case["X"].reshape(-1, mlp.N_IN)
    idx = np.flatnonzero(use)
    return Xr, idx


def test_forward_matches_oracle(B, ctx, case):
    th = rand_params(5)
    Xr, idx = usable_rows(case)
    rows = torch.as_tensor(idx[:700]).cuda()
    y = B.learned_forward(ctx, torch.as_tensor(th).cuda(), Xr[rows]).cpu().numpy()
    yo, _ = mlp.forward(th.astype(np.float64), Xr[rows].float().cpu().numpy().astype(np.float64))
    e = metrics.rel_l2(y.astype(np.float64), yo)
    say(f"[learned forward] {len(y)} rows, rel_l2 {e:.2e}")
    assert e <= 5e-3
    assert np.max(np.abs(y - yo)) <= 2e-2 * np.sqrt(np.mean(yo * yo))


def test_gradient_and_adam_match_oracle(B, ctx, case):
    th = rand_params(6)
    Xr, idx = usable_rows(case)
    g = np.random.default_rng(9)
    sel = idx[:300]
    t_all = torch.as_tensor(g.normal(0, 1, Xr.shape[0]).astype(np.float32)).cuda()
    P = torch.as_tensor(th).cuda()
    tr = B.Trainer(ctx, P, batch=300)
    grad = torch.empty(B.LEARNED_NPARAM, dtype=torch.float32, device="cuda")
    rows = torch.as_tensor(sel.astype(np.int32)).cuda()
    loss = tr.run(Xr, t_all, rows, apply=False, grad=grad).item()
    Xo = Xr[torch.as_tensor(sel).cuda()].float().cpu().numpy().astype(np.float64)
    lo, go, _ = mlp.loss_and_grad(th.astype(np.float64), Xo, t_all.cpu().numpy()[sel].astype(np.float64))
    gg = grad.cpu().numpy().astype(np.float64)
    e = metrics.rel_l2(gg, go)
    say(f"[learned grad] loss {loss:.6f} vs {lo:.6f}; grad rel_l2 {e:.2e}")
    assert abs(loss - lo) <= 1e-3 * lo
    assert e <= 1e-2
    for name, (o, n) in mlp.OFFS.items():
        if np.linalg.norm(go[o:o + n]) > 0:
            assert metrics.rel_l2(gg[o:o + n], go[o:o + n]) <= 3e-2, name
    assert np.all(gg[[mlp.OFFS["W1"][0] + r * mlp.N_IN + c for r in range(64)
                      for c in range(mlp.N_FEAT, mlp.N_IN)]] == 0.0)
    # one Adam step from zero moments, against the oracle's step with the GPU gradient
    tr.run(Xr, t_all, rows, lr=1e-3, apply=True)
    th1, _, _ = mlp.adam_step(th.astype(np.float64), np.zeros(mlp.N_PARAM), np.zeros(mlp.N_PARAM),
                              gg, 1, 1e-3)
    assert np.allclose(P.cpu().numpy(), th1, rtol=0, atol=2e-6)
    assert tr.step == 1


def test_determinism(B, ctx, case):
    th = rand_params(7)
    Xr, idx = usable_rows(case)
    t = torch.zeros(Xr.shape[0], dtype=torch.float32, device="cuda")
    rows = torch.as_tensor(idx[:256].astype(np.int32)).cuda()
    out = []
    for _ in range(2):
        P = torch.as_tensor(th).cuda()
        tr = B.Trainer(ctx, P, batch=256)
        for _ in range(3):
            tr.run(Xr, t, rows, lr=1e-3)
        out.append(P.cpu())
    assert torch.equal(out[0], out[1])


@pytest.fixture(scope="module")
def trained(B, ctx, case):
    """A few hundred Adam steps on solver targets of the test case (exact = oracle)."""
    prob, vals = case["prob"], case["vals"]
    ref, _ = p1.mass_assign(f64(prob), vals.astype(np.float64), solver="direct")
    base = case["base"].cpu().numpy()
    scale = case["scale"].cpu().numpy()
    use = scale > 0
    tgt = np.zeros_like(base)
    tgt[use] = (ref.T[use] - base[use]) / scale[use]
    Xr, idx = usable_rows(case)
    target = torch.as_tensor(tgt.reshape(-1).astype(np.float32)).cuda()
    P = torch.as_tensor(mlp.init_params(21)).cuda()
    tr = B.Trainer(ctx, P, batch=512)
    g = np.random.default_rng(3)
    losses = []
    for it in range(400):
        rows = torch.as_tensor(g.choice(idx, 512, replace=False).astype(np.int32)).cuda()
        losses.append(tr.run(Xr, target, rows, lr=2e-3).item())
    say(f"[learned train] loss {np.mean(losses[:10]):.4f} -> {np.mean(losses[-10:]):.4f}, "
        f"target variance {np.var(tgt[use]):.4f}")
    return P, losses, ref


def test_training_reduces_loss(trained):
    _, losses, _ = trained
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:20])


def test_learned_start_in_mass_solve(B, ctx, case, trained):
    P, _, ref = trained
    opts = B.solve_opts(tol=1e-9, maxit=1000, max_refine=10, start=B.START_LEARNED)
    with pytest.raises(B.P2MError):
        B.set_learned(ctx, None)
        B.p2m_mass_assign(ctx, case["d"], case["v"], opts)
    B.set_learned(ctx, P)
    out, rep = B.p2m_mass_assign(ctx, case["d"], case["v"], opts)
    torch.cuda.synchronize()
    r = B.read_report(rep, 3)
    got = out.cpu().numpy().astype(np.float64)
    for f in range(3):
        assert metrics.rel_l2(got[f], ref[f]) <= 1e-6
    flip, rf = B.p2m_mass_assign(ctx, case["d"], case["v"], B.solve_opts(tol=1e-9, maxit=1000,
                                                                        max_refine=10))
    torch.cuda.synchronize()
    rf = B.read_report(rf, 3)
    say(f"[learned solve] iters learned {r.iters.tolist()} vs FLIP {rf.iters.tolist()}, "
        f"flags {r.flags}")
    # a network that proposes nonsense is replaced by the FLIP start, field by field
    bad = P.clone()
    bad[mlp.OFFS["b4"][0]] = 1.0e4
    B.set_learned(ctx, bad)
    out2, rep2 = B.p2m_mass_assign(ctx, case["d"], case["v"], opts)
    torch.cuda.synchronize()
    r2 = B.read_report(rep2, 3)
    assert r2.flags & B.FLAG_LEARNED_FALLBACK
    got2 = out2.cpu().numpy().astype(np.float64)
    for f in range(3):
        assert metrics.rel_l2(got2[f], ref[f]) <= 1e-6
    B.set_learned(ctx, None)


# ----------------------------------------------------------------------------
# the gain of the trained network on a held-out configuration of the learned-start
# workload: 1024^2, 8 ppc, TG fields disordered by 200 RK2 steps (seed 20000, not
# among the training seeds 10000-10015 or the validation seed 19999)
# ----------------------------------------------------------------------------
def test_trained_network_gain(B, ctx):
    import os
    import time
    wpath = os.path.join(os.path.dirname(B.__file__), "learned_tg.npy")
    if not os.path.exists(wpath):
        pytest.skip("no trained parameters (python -m paper_1610_05258_amd.train_learned)")
    say("[learned gain] held-out seed 20000, 1024^2, 8 ppc, 200 disorder steps (GPU advection)")
    prob, vals = wl.tg_disordered(20000, n=1024, ppc=8, steps=200, dt=1e-3, device="cuda")
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    B.set_learned(ctx, torch.as_tensor(np.load(wpath, allow_pickle=False)).cuda())
    out = torch.empty((3, 1024 * 1024), dtype=torch.float32, device="cuda")
    rep = ctx.new_report()

    def run(start, tol, maxit=2000, max_refine=10, reps=5):
        opts = B.solve_opts(tol=tol, inner_rtol=1e-4, maxit=maxit, max_refine=max_refine, start=start)
        B.p2m_mass_assign(ctx, d, v, opts, rep=rep, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            B.p2m_mass_assign(ctx, d, v, opts, rep=rep, out=out)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3, B.read_report(rep, 3)

    # the starts themselves: no iteration, the report holds the start's FP64 residual
    _, r0f = run(B.START_FLIP, 1e-6, maxit=0, max_refine=0, reps=1)
    _, r0l = run(B.START_LEARNED, 1e-6, maxit=0, max_refine=0, reps=1)
    say(f"  start residual FLIP {r0f.rel_residual.tolist()}  learned {r0l.rel_residual.tolist()}")
    assert not (r0l.flags & B.FLAG_LEARNED_FALLBACK)
    assert np.all(r0l.rel_residual < r0f.rel_residual)
    for tol in (1e-6, 1e-8):
        tf, rf = run(B.START_FLIP, tol)
        tl, rl = run(B.START_LEARNED, tol)
        say(f"  tol {tol:g}: FLIP {tf:.3f} ms iters {rf.iters.tolist()} | learned {tl:.3f} ms "
            f"iters {rl.iters.tolist()}")
        assert rl.iters.sum() <= rf.iters.sum()
        assert np.all(rl.rel_residual <= tol)
    # the learned-start answer still meets the gate against the FP64 oracle
    got = out.cpu().numpy().astype(np.float64)
    pr = f64(prob)
    st = p1.assemble_stencil(pr, vals.astype(np.float64))
    M = p1.regularised_matrix(p1.stencil_matrix(pr, st), st["w"])
    for f in range(3):
        x, _ = p1.cg_fp64(M, st["b"][f], rtol=1e-12)
        assert metrics.rel_l2(got[f], x) <= 1e-6
    B.set_learned(ctx, None)
