"""The entry point that allocates nothing (p2m_mass_assign_noalloc): the same
kernels as p2m_mass_assign, with the workspace taken from the library's static
device scratch.  Checked through the C ABI against p2m_mass_assign with a caller
workspace, bit for bit (the same arithmetic in the same order), on two calls in a
row, the second with a smaller input (the scratch keeps the first call's contents,
so everything the second call relies on must be cleared by the call itself), and
both against the FP64 oracle at the FP32 gate (1e-6 relative l2 per field).  A
problem beyond the scratch is rejected before any launch."""
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


def test_noalloc_matches_workspace_entry_point(B):
    ctx = B.Context(0)
    try:
        opts = B.solve_opts(tol=1e-9, maxit=2000, max_refine=20)
        for k, (n, ppc, steps) in enumerate([(192, 6, 30), (64, 4, 10)]):
            prob, vals = wl.taylor_green_2d(seed=40 + k, n=n, ppc=ppc, steps=steps, dt=1e-2)
            d = B.particles_from(prob, dtype=torch.float32)
            v = torch.as_tensor(vals).cuda()
            need = ctx.workspace_size(d, vals.shape[0])
            say(f"[noalloc] call {k + 1}: {n}x{n}, {vals.shape[1]} particles, F={vals.shape[0]}, "
                f"workspace {need} bytes of {B.SCRATCH_BYTES}")
            assert need <= B.SCRATCH_BYTES
            ref, rep_ref = B.p2m_mass_assign(ctx, d, v, opts)
            got, rep = B.p2m_mass_assign_noalloc(ctx, d, v, opts)
            torch.cuda.synchronize()
            r, rr = B.read_report(rep, vals.shape[0]), B.read_report(rep_ref, vals.shape[0])
            say(f"  iters={r.iters} flags={r.flags}")
            assert torch.equal(got, ref)
            assert np.array_equal(r.iters, rr.iters) and r.flags == rr.flags == 0
            pr = dict(prob, x=prob["x"].astype(np.float64), y=prob["y"].astype(np.float64))
            ora, _ = p1.mass_assign(pr, vals.astype(np.float64), solver="direct")
            for f in range(vals.shape[0]):
                e = metrics.rel_l2(got[f].cpu().numpy(), ora[f])
                say(f"  field {f}: rel_l2 vs oracle {e:.2e}")
                assert e <= 1e-6
    finally:
        ctx.close()


def test_noalloc_rejects_problems_beyond_the_scratch(B):
    ctx = B.Context(0)
    try:
        n, ppc = 1024, 8
        npart = n * n * ppc
        x = torch.zeros(npart, dtype=torch.float32, device="cuda")
        d = B.Particles(2, n, n, 1.0, 1.0, x, x, None)
        v = torch.zeros((1, npart), dtype=torch.float32, device="cuda")
        need = ctx.workspace_size(d, 1)
        say(f"[noalloc] 1024x1024 needs {need} bytes > {B.SCRATCH_BYTES}")
        assert need > B.SCRATCH_BYTES
        with pytest.raises(B.P2MError) as ei:
            B.p2m_mass_assign_noalloc(ctx, d, v, B.solve_opts(tol=1e-6))
        assert ei.value.status == B.ERR_SCRATCH
        torch.cuda.synchronize()
    finally:
        ctx.close()
