"""Pins of the learned-start oracle (oracle/mlp.py) against things other than itself:
BF16 rounding against hand cases and torch's conversion, the backward against
finite differences, a hand-built network with a closed-form output, Adam's first
step, and the node features against their geometric definition (periodic
minimum-image offsets from the node) on small meshes."""
import numpy as np
import pytest

from oracle import mlp
from oracle import p1
from paper_1610_05258_amd import workloads as wl


def test_bf16_rounding_cases():
    one = 1.0
    ulp = 2.0 ** -7
    cases = [(1.0, 1.0), (1.0 + 2.0 ** -8, 1.0),                 # tie -> even (down)
             (1.0 + 3 * 2.0 ** -8, 1.0 + 2 * ulp),              # tie -> even (up)
             (1.0 + 2.0 ** -8 + 2.0 ** -12, 1.0 + ulp),          # above the tie
             (-2.5, -2.5), (0.0, 0.0), (3.0e38, 2.9979e38)]
    for x, want in cases[:-1]:
        assert mlp.bf16(np.float32(x)) == want, x
    assert np.isnan(mlp.bf16(np.float32("nan")))
    assert one == mlp.bf16(1.0)


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(5)
    x = np.concatenate([g.normal(0, 1, 20000), g.normal(0, 1e-30, 100), g.normal(0, 1e30, 100)])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_backward_matches_finite_differences():
    g = np.random.default_rng(1)
    theta = mlp.init_params(3).astype(np.float64)
    theta[mlp.OFFS["W4"][0]:mlp.OFFS["W4"][0] + 64] = g.normal(0, 0.3, 64)
    theta[mlp.OFFS["b1"][0]:mlp.OFFS["b1"][0] + 64] = g.normal(0, 0.1, 64)
    X = g.normal(0, 1, (12, mlp.N_IN))
    X[:, mlp.N_FEAT:] = 0.0
    t = g.normal(0, 1, 12)
    _, grad, _ = mlp.loss_and_grad(theta, X, t, mirror_gpu=False)
    idx = np.concatenate([g.choice(np.arange(mlp.N_PARAM), 60, replace=False),
                          [mlp.OFFS["b4"][0], mlp.OFFS["W4"][0] + 5, mlp.OFFS["b3"][0] + 7]])
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        lp = mlp.loss_and_grad(tp, X, t, mirror_gpu=False)[0]
        lm = mlp.loss_and_grad(tm, X, t, mirror_gpu=False)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_hand_built_network():
    """y = 2 relu(x_2) + 0.5 through single-path weights (exact in BF16)."""
    theta = np.zeros(mlp.N_PARAM)
    p = mlp.unpack(theta)
    p["W1"][0, 2] = 1.0
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0
    p["W4"][0] = 2.0
    p["b4"][0] = 0.5
    X = np.zeros((3, mlp.N_IN))
    X[:, 2] = [-1.0, 0.25, 3.0]
    y, _ = mlp.forward(theta, X)
    assert np.array_equal(y, [0.5, 1.0, 6.5])


def test_adam_first_step():
    theta = np.array([1.0, -2.0, 0.5])
    grad = np.array([0.3, -4.0, 0.0])
    th, m, v = mlp.adam_step(theta, np.zeros(3), np.zeros(3), grad, 1, 0.01)
    # with zero moments the bias-corrected first step is lr * g / (|g| + eps)
    assert np.allclose(th, theta - 0.01 * grad / (np.abs(grad) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * grad) and np.allclose(v, 0.001 * grad * grad)


def small_problem(n=12, ppc=3, seed=7):
    x, y = wl.stratified_2d(seed, n, n, ppc, 1.0, 1.0)
    x, y = x.copy(), y.copy()
    x[:5] = 0.0                         # particles exactly on node 0 (cell a of node 0)
    y[:5] = 0.0
    prob = dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=x, y=y, vol=None)
    vals = np.stack([np.sin(2 * np.pi * x) + y, np.full_like(x, 0.7)])
    return prob, vals


def test_features_geometry_and_order():
    prob, vals = small_problem()
    n = prob["nx"]
    loc = p1.locate(prob)
    perm, cs = p1.bin_particles(loc["key"], loc["valid"], n * n)
    a = p1.assemble(prob, vals, want_matrix=False)
    base = mlp.flip_base(a["b"], a["w"])
    nodes = np.arange(n * n)
    X, scale, count = mlp.node_features(prob, vals, base, a["w"], nodes, loc, perm, cs)
    h = 1.0 / n
    for node in nodes:
        ix, iy = node % n, node // n
        # the particles of the support of psi_node: minimum-image offsets in (-1, 1)
        ox = (prob["x"] - ix * h + 0.5) % 1.0 - 0.5
        oy = (prob["y"] - iy * h + 0.5) % 1.0 - 0.5
        sup = np.flatnonzero((ox / h >= -1) & (ox / h < 1) & (oy / h >= -1) & (oy / h < 1))
        assert count[node] == sup.size
        k = min(sup.size, mlp.K_MAX)
        if sup.size <= mlp.K_MAX:
            got = np.array(sorted((X[node, 0, 3 * m], X[node, 0, 3 * m + 1]) for m in range(k)))
            want = np.array(sorted((ox[mu] / h, oy[mu] / h) for mu in sup))
            assert got.shape == want.shape and np.allclose(got, want, rtol=0, atol=1e-9), node
        assert X[node, 0, 3 * mlp.K_MAX] == min(sup.size, mlp.K_MAX) / mlp.K_MAX
        assert np.all(X[node, :, mlp.N_FEAT:] == 0.0)
        # cell order a, b, c, d: dx >= 0 first, then dx < 0 ...
        dxs = [X[node, 0, 3 * m] for m in range(k)]
        dys = [X[node, 0, 3 * m + 1] for m in range(k)]
        roles = [(dx < 0, dy < 0) for dx, dy in zip(dxs, dys)]
        order = {(False, False): 0, (True, False): 1, (True, True): 2, (False, True): 3}
        assert [order[r] for r in roles] == sorted(order[r] for r in roles)
    # particles exactly on node 0 have zero offsets; a constant field has s = 0
    assert np.any(np.all(X[0, 0, 0:6].reshape(2, 3)[:, :2] == 0.0, axis=1))
    assert np.all(scale[:, 1] == 0.0)
    # value features have unit RMS over the kept particles where usable
    for node in nodes:
        if scale[node, 0] > 0:
            k = min(count[node], mlp.K_MAX)
            av = X[node, 0, 2:3 * k:3]
            assert abs(np.sqrt(np.mean(av * av)) - 1.0) < 1e-12


def test_features_overflow_and_orphans():
    n = 8
    g = np.random.default_rng(2)
    x = np.concatenate([g.uniform(0.0, 0.01, 60), g.uniform(0.5, 0.6, 40)])
    y = np.concatenate([g.uniform(0.0, 0.01, 60), g.uniform(0.5, 0.6, 40)])
    prob = dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=x, y=y, vol=None)
    vals = (x + 2 * y)[None, :]
    loc = p1.locate(prob)
    perm, cs = p1.bin_particles(loc["key"], loc["valid"], n * n)
    a = p1.assemble(prob, vals, want_matrix=False)
    base = mlp.flip_base(a["b"], a["w"])
    X, scale, count = mlp.node_features(prob, vals, base, a["w"], np.arange(n * n), loc, perm, cs)
    assert count[0] == 60 and scale[0, 0] == 0.0            # overflow: not usable
    assert X[0, 0, 3 * mlp.K_MAX] == 1.0                     # count feature saturates
    empty = np.flatnonzero(count == 0)
    assert empty.size > 0 and np.all(scale[empty] == 0.0) and np.all(X[empty] == 0.0)
