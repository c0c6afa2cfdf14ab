"""GPU binning beyond the common case: crowded cells (the workgroup-cooperative
sort of cells with more than 16 particles, in LDS and in global memory), and the
bounded wait of the scan (its timeout path, forced from the host with the
P2M_OPT_SCAN_SPIN hook: every kernel still exits normally).  Binning is checked
bit for bit against the oracle's stable sort."""
import sys
import zlib

import numpy as np
import pytest

from oracle import metrics
from oracle import p1

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


def crowded(name):
    """Problems with crowded cells (FP32, 2D unless stated)."""
    g = np.random.Generator(np.random.PCG64(zlib.crc32(name.encode())))
    if name == "onecell1d":
        x = g.uniform(0.5, 0.5 + 1.0 / 64, 20000)
        return dict(dim=1, nx=64, ny=1, lx=1.0, ly=1.0, x=x.astype(np.float32), y=None, vol=None)
    if name.startswith("onecell"):
        # every particle in cell (2, 4) of an 8 x 8 mesh on the unit square
        k = int(name[len("onecell"):])
        x = g.uniform(0.25, 0.375, k)
        y = g.uniform(0.5, 0.625, k)
        return dict(dim=2, nx=8, ny=8, lx=1.0, ly=1.0, x=x.astype(np.float32),
                    y=y.astype(np.float32), vol=None)
    if name == "clusters":
        # 300 x 200 mesh: uniform background of 6 per cell plus 40 clusters of
        # 17 .. 3000 particles, each inside one cell, and a band of 30 per cell
        nx, ny = 300, 200
        xs = [g.uniform(0, 1, 6 * nx * ny)]
        ys = [g.uniform(0, 1, 6 * nx * ny)]
        for k in range(40):
            cnt = int(g.integers(17, 3000))
            cx, cy = int(g.integers(0, nx)), int(g.integers(0, ny))
            xs.append((cx + g.uniform(0, 1, cnt)) / nx)
            ys.append((cy + g.uniform(0, 1, cnt)) / ny)
        xs.append(g.uniform(0.5, 0.5 + 40 / nx, 30 * 40 * 3))
        ys.append(g.uniform(0.1, 0.1 + 3 / ny, 30 * 40 * 3))
        x = np.concatenate(xs)
        y = np.concatenate(ys)
        perm = g.permutation(x.size)
        return dict(dim=2, nx=nx, ny=ny, lx=1.0, ly=1.0, x=x[perm].astype(np.float32),
                    y=y[perm].astype(np.float32), vol=None)
    raise KeyError(name)


def f64(prob):
    out = dict(prob)
    for k in ("x", "y", "vol"):
        if out.get(k) is not None:
            out[k] = np.asarray(out[k]).astype(np.float64)
    return out


@pytest.mark.parametrize("name", ["onecell17", "onecell4096", "onecell5000", "onecell100000",
                                  "clusters", "onecell1d"])
def test_crowded_cells_bin_bit_exact(B, ctx, name):
    """Cells of 17 .. 100000 particles: perm and cell_start equal the stable sort.
    4096 particles fit a workgroup's LDS stage, 5000 and more are sorted in
    global memory."""
    say(f"[crowded bin] {name}")
    prob = crowded(name)
    d = B.particles_from(prob, dtype=torch.float32)
    perm, cs, rep = B.p2m_bin(ctx, d)
    torch.cuda.synchronize()
    loc = p1.locate(f64(prob))
    ref_perm, ref_cs = p1.bin_particles(loc["key"], loc["valid"], p1.n_nodes(prob))
    counts = np.diff(ref_cs)
    say(f"  largest cell {counts.max()}, cells > 16: {(counts > 16).sum()}")
    assert np.array_equal(cs.cpu().numpy().astype(np.int64), ref_cs)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), ref_perm)
    assert B.read_report(rep).flags == 0


@pytest.mark.parametrize("name", ["onecell5000", "clusters"])
def test_crowded_cells_mass_assign(B, ctx, name):
    """Mass assignment over crowded cells (many orphan nodes around one cell)
    against the oracle's direct solve; the sum order inside a cell is the binned
    order, so two calls agree bit for bit."""
    say(f"[crowded mass] {name}")
    prob = crowded(name)
    npart = prob["x"].size
    vals = np.random.default_rng(3).normal(size=(2, npart)).astype(np.float32)
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    opts = B.solve_opts(tol=1e-9, maxit=4000, max_refine=20)
    out, rep = B.p2m_mass_assign(ctx, d, v, opts)
    out = out.clone()
    out2, _ = B.p2m_mass_assign(ctx, d, v, opts)
    torch.cuda.synchronize()
    r = B.read_report(rep, 2)
    say(f"  iters={r.iters} flags={r.flags} orphans={r.n_orphan}")
    assert not (r.flags & (B.FLAG_NOT_CONVERGED | B.FLAG_BREAKDOWN | B.FLAG_BIN_TIMEOUT))
    assert torch.equal(out, out2)
    ref, _ = p1.mass_assign(f64(prob), vals.astype(np.float64), solver="direct")
    for f in range(2):
        e = metrics.rel_l2(out[f].cpu().numpy(), ref[f])
        say(f"  field {f} rel_l2={e:.3e}")
        assert e <= 1e-6


def test_scan_timeout_discards_binning(B):
    """With every wait of the scan ended at once (the test hook), a mesh of more
    than one scan tile (128 x 128 = 16384 cells, 2048 per tile) raises
    P2M_FLAG_BIN_TIMEOUT and every cell is left empty: cell_start all 0 and perm
    all -1.  The mass assignment of that call reads the empty binning (every node
    an orphan: result 0).  Back at the default bound the same context bins
    exactly again."""
    from paper_1610_05258_amd import workloads as wl
    say("[scan timeout hook]")
    prob, vals = wl.taylor_green_2d(seed=5, n=128, ppc=2, steps=0)
    c = B.Context(0)
    try:
        d = B.particles_from(prob, dtype=torch.float32)
        v = torch.as_tensor(vals).cuda()
        c.set_scan_spin(-1)
        perm, cs, rep = B.p2m_bin(c, d)
        out, rep_m = B.p2m_mass_assign(c, d, v, B.solve_opts(tol=1e-6))
        torch.cuda.synchronize()
        r = B.read_report(rep)
        rm = B.read_report(rep_m, vals.shape[0])
        say(f"  bin flags={r.flags} mass flags={rm.flags} orphans={rm.n_orphan}")
        assert r.flags & B.FLAG_BIN_TIMEOUT
        assert int(torch.count_nonzero(cs).item()) == 0
        assert bool((perm == -1).all().item())
        assert rm.flags & B.FLAG_BIN_TIMEOUT and rm.flags & B.FLAG_ORPHAN
        assert rm.n_orphan == prob["nx"] * prob["ny"]
        assert int(torch.count_nonzero(out).item()) == 0
        # the batched graph takes the same path: every instance is flagged
        outs, bt = B.p2m_mass_assign_batched(c, [d, d], [v[:2], v[:2]], B.solve_opts(tol=1e-6))
        torch.cuda.synchronize()
        for rb in bt.reports():
            assert rb.flags & B.FLAG_BIN_TIMEOUT
        assert all(int(torch.count_nonzero(o).item()) == 0 for o in outs)
        # default bound again: exact binning, no flag
        c.set_scan_spin(0)
        perm, cs, rep = B.p2m_bin(c, d)
        torch.cuda.synchronize()
        loc = p1.locate(f64(prob))
        ref_perm, ref_cs = p1.bin_particles(loc["key"], loc["valid"], p1.n_nodes(prob))
        assert B.read_report(rep).flags == 0
        assert np.array_equal(perm.cpu().numpy().astype(np.int64), ref_perm)
        assert np.array_equal(cs.cpu().numpy().astype(np.int64), ref_cs)
    finally:
        c.close()
