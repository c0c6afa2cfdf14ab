"""The paper-exact 1D methods on the GPU (Table 1 with the particle hats of Sec. 2;
Sec. 2.4 eq. (20); Appendix B; Sec. 3.1) against the FP64 oracle `oracle/paper1d.py`.

Every operator (delta, FLIP, PIC, mass and lumped P2M; delta, full-mass and lumped
M2P; the particle volumes of eq. (4)) with both quadratures, on random, sparse,
node-aligned, crowded and wrapping particle sets, at relative l2 <= 1e-12 per
field; then the Sec. 3.1 moving top-hat (200 particles, 200 nodes, Co = 0.1,
2000 steps) run on the GPU, which must give the oracle's final profile and
E1 / E2 / L2, and with them Table 2's regular column."""
import os
import sys
import zlib

import numpy as np
import pytest

from oracle import metrics
from oracle import paper1d as px

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2.txt")


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


def case(name):
    g = np.random.Generator(np.random.PCG64(zlib.crc32(name.encode())))
    if name == "random":
        return g.uniform(0, 1, 37), 16
    if name == "sparse":
        return g.uniform(0, 1, 5), 32
    if name == "on_nodes":
        n = 24
        return np.arange(n) / n, n
    if name == "crowded":
        return np.concatenate([g.uniform(0, 1, 200), 0.5 + g.uniform(0, 1, 100) / 20]), 20
    if name == "wrap":
        n = 10
        # 1 (= L) wraps onto node 0 and 1 + 0.03 into the first cell; 1 - 1e-9 leaves a
        # gap of 1e-9 before the wrap (two particles at one position would make the
        # particle interpolant jump there, where the method is not defined)
        x = np.concatenate([g.uniform(0, 1, 30), [1.0 - 1e-9, 1.0, 1.0 + 0.03, 0.05]])
        return x, n
    raise KeyError(name)


CASES = ["random", "sparse", "on_nodes", "crowded", "wrap"]


def dev(B, x, n):
    xt = torch.as_tensor(np.ascontiguousarray(x, np.float64)).cuda()
    return B.Particles(1, n, 1, 1.0, 1.0, xt, None, None)


def check(gpu, ref, tol, what):
    gpu = np.atleast_2d(np.asarray(gpu, np.float64))
    ref = np.atleast_2d(ref)
    for f in range(ref.shape[0]):
        e = metrics.rel_l2(gpu[f], ref[f])
        say(f"  {what}[{f}] rel_l2={e:.3e}")
        assert e <= tol, (what, f, e)


@pytest.mark.parametrize("name", CASES)
def test_volumes(B, ctx, name):
    x, n = case(name)
    say(f"[x1d volumes] {name}")
    v = B.p2m_x1d_volumes(ctx, dev(B, x, n))
    torch.cuda.synchronize()
    check(v.cpu().numpy(), px.particle_volumes(x), 1e-13, "vol")


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("quad", ["exact", "appB"])
def test_p2m_operators(B, ctx, name, quad):
    x, n = case(name)
    say(f"[x1d P2M] {name} {quad}")
    g = np.random.default_rng(5)
    A = g.normal(size=(2, x.size))
    d = dev(B, x, n)
    v = torch.as_tensor(A).cuda()
    q = B.QUAD_EXACT if quad == "exact" else B.QUAD_APPB
    opts = B.solve_opts(tol=1e-14, maxit=5000, max_refine=30, fp64=True)
    ref = dict(delta=lambda a: px.p2m_delta(x, a, n), flip=lambda a: px.p2m_flip(x, a, n),
               pic=lambda a: px.p2m_pic(x, a, n), mass=lambda a: px.p2m_mass(x, a, n, quad=quad),
               lumped=lambda a: px.p2m_lumped(x, a, n, quad=quad))
    kinds = dict(delta=B.X1D_DELTA, flip=B.X1D_FLIP, pic=B.X1D_PIC, mass=B.X1D_MASS, lumped=B.X1D_LUMPED)
    for k, kind in kinds.items():
        out, rep = B.p2m_x1d_assign(ctx, d, kind, q, v, opts=opts)
        torch.cuda.synchronize()
        r = B.read_report(rep, 2)
        assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN)), (k, r.flags)
        check(out.cpu().numpy(), np.stack([ref[k](A[f]) for f in range(2)]), 1e-12, k)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("quad", ["exact", "appB"])
def test_m2p_operators(B, ctx, name, quad):
    x, n = case(name)
    say(f"[x1d M2P] {name} {quad}")
    g = np.random.default_rng(6)
    Ab = g.normal(size=(2, n))
    d = dev(B, x, n)
    nod = torch.as_tensor(Ab).cuda()
    q = B.QUAD_EXACT if quad == "exact" else B.QUAD_APPB
    opts = B.solve_opts(tol=1e-14, maxit=5000, max_refine=30, fp64=True)
    ref = dict(delta=lambda a: px.m2p_delta(x, a, n), mass=lambda a: px.m2p_mass(x, a, n, quad=quad),
               lumped=lambda a: px.m2p_lumped(x, a, n, quad=quad))
    kinds = dict(delta=B.X1D_DELTA, mass=B.X1D_MASS, lumped=B.X1D_LUMPED)
    for k, kind in kinds.items():
        out, rep = B.p2m_x1d_interpolate(ctx, d, kind, q, nod, opts=opts)
        torch.cuda.synchronize()
        r = B.read_report(rep, 2)
        assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN)), (k, r.flags)
        check(out.cpu().numpy(), np.stack([ref[k](Ab[f]) for f in range(2)]), 1e-12, k)


def test_unlocatable_particles_get_nan(B, ctx):
    x = np.array([0.1, 0.35, np.nan, 0.6, 1.7, 0.9])
    n = 8
    d = dev(B, x, n)
    nod = torch.as_tensor(np.random.default_rng(1).normal(size=(1, n))).cuda()
    out, rep = B.p2m_x1d_interpolate(ctx, d, B.X1D_MASS, B.QUAD_EXACT, nod)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    assert np.isnan(got[2]) and np.isnan(got[4]) and np.all(np.isfinite(got[[0, 1, 3, 5]]))
    r = B.read_report(rep, 1)
    assert r.flags & B.FLAG_RANGE and r.flags & B.FLAG_NONFINITE
    ok = np.array([0, 1, 3, 5])
    check(got[ok][None], px.m2p_mass(x[ok], nod.cpu().numpy()[0], n, quad="exact")[None], 1e-12, "mass")


# ----------------------------------------------------------------------------
# Sec. 3.1: the moving top-hat on the GPU
# ----------------------------------------------------------------------------
PAIRS = dict(delta=("X1D_DELTA", "X1D_DELTA"), flip=("X1D_FLIP", "X1D_DELTA"),
             mass_delta=("X1D_MASS", "X1D_DELTA"), full_mass=("X1D_MASS", "X1D_MASS"),
             mass_lumped=("X1D_MASS", "X1D_LUMPED"), lumped=("X1D_LUMPED", "X1D_LUMPED"))


def gpu_tophat(B, ctx, method, n_nodes=200, n_particles=200, co=0.1, u=1.0, T=1.0, distort=0.0,
               seed=0, quad="appB", lo=0.25, hi=0.75, L=1.0):
    """The oracle's tophat_experiment with every P2M and M2P on the GPU: move, P2M,
    M2P per step; positions of each step computed on the host as the oracle does."""
    x0 = px.tophat_positions(n_particles, distort, seed, L)
    A0 = ((x0 > lo) & (x0 < hi)).astype(np.float64)
    dt = co * (L / n_nodes) / u
    steps = int(round(T / dt))
    X = torch.as_tensor(np.stack([np.mod(x0 + k * u * dt, L) for k in range(1, steps + 1)])).cuda()
    q = B.QUAD_EXACT if quad == "exact" else B.QUAD_APPB
    kp, km = (getattr(B, s) for s in PAIRS[method])
    opts = B.solve_opts(tol=1e-15, maxit=5000, max_refine=30, fp64=True)
    A = torch.as_tensor(A0[None, :]).cuda()
    nodal = torch.empty((1, n_nodes), dtype=torch.float64, device="cuda")
    back = torch.empty((1, n_particles), dtype=torch.float64, device="cuda")
    rep = ctx.new_report()
    ws = torch.empty(B.x1d_workspace_size(ctx, B.Particles(1, n_nodes, 1, L, 1.0, X[0], None, None), 1),
                     dtype=torch.uint8, device="cuda")
    for k in range(steps):
        d = B.Particles(1, n_nodes, 1, L, 1.0, X[k], None, None)
        B.p2m_x1d_assign(ctx, d, kp, q, A, opts=opts, ws=ws, rep=rep, out=nodal)
        B.p2m_x1d_interpolate(ctx, d, km, q, nodal, opts=opts, ws=ws, rep=rep, out=back)
        A, back = back, A
    torch.cuda.synchronize()
    AT = A.cpu().numpy()[0]
    xT = np.mod(x0 + steps * u * dt, L)
    v0, vT = px.particle_volumes(x0, L), px.particle_volumes(xT, L)
    return dict(E1=metrics.e1(v0, A0, vT, AT), E2=metrics.e2(v0, A0, vT, AT), L2=metrics.l2(v0, A0, AT),
                AT=AT)


def table2():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            setup, method, e1, e2, l2 = line.split()
            rows[(setup, method)] = tuple(float(v) for v in (e1, e2, l2))
    return rows


@pytest.mark.parametrize("method", ["delta", "flip", "mass_delta", "full_mass"])
def test_table2_regular_column_on_gpu(B, ctx, method):
    say(f"[x1d Table 2] {method}, 200 particles / 200 nodes, Co 0.1, 2000 steps")
    got = gpu_tophat(B, ctx, method)
    ref = px.tophat_experiment(method)
    e = metrics.rel_l2(got["AT"], ref["AT"])
    say(f"  GPU E1 {got['E1']:.6e} E2 {got['E2']:.6e} L2 {got['L2']:.6e}; final profile vs oracle "
        f"rel_l2 {e:.2e}")
    assert e <= 1e-12
    for k in ("E1", "E2", "L2"):
        assert abs(got[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k
    # and the printed table (FLIP is pinned to delta's values: the paper's text says
    # the two coincide for this set-up, its printed E2 for FLIP notwithstanding)
    row = table2()[("regular", "delta" if method == "flip" else method)]
    for val, printed in zip((got["E1"], got["E2"], got["L2"]), row):
        s = f"{printed:g}"
        half = 0.5 * 10.0 ** (-(len(s.split(".")[1]) if "." in s else 0))
        assert abs(100 * val - printed) <= half + 1e-9


@pytest.mark.parametrize("method", ["mass_lumped", "lumped", "full_mass"])
def test_tophat_lumped_and_exact_quadrature_on_gpu(B, ctx, method):
    """The two lumped rows (no printed results) and full mass with exact integrals on
    the distorted set-up: the GPU run equals the oracle's run step for step."""
    say(f"[x1d top-hat] {method}, distorted 0.4, exact quadrature")
    got = gpu_tophat(B, ctx, method, distort=0.4, seed=3, quad="exact", n_nodes=100, n_particles=100)
    ref = px.tophat_experiment(method, distort=0.4, seed=3, quad="exact", n_nodes=100, n_particles=100)
    e = metrics.rel_l2(got["AT"], ref["AT"])
    say(f"  E1 {got['E1']:.3e} E2 {got['E2']:.3e} L2 {got['L2']:.3e}; rel_l2 vs oracle {e:.2e}")
    assert e <= 1e-12
    assert abs(got["E1"] - ref["E1"]) <= 1e-12
