"""Child process of tests/test_gpu_determinism.py: runs the binning, the assembly,
the mass assignment with each resident solver and a fluid step on fixed seeded
inputs and prints the SHA-256 of every output (one JSON line).  The cooperative
streaming solve is left out: a cooperative launch needs the device's global wave
synchronisation, which another process using the GPU may hold."""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def digests():
    import torch
    from paper_1610_05258_amd import binding as B
    from paper_1610_05258_amd import workloads as wl
    out = {}
    h = lambda t: hashlib.sha256(t.detach().cpu().numpy().tobytes()).hexdigest()
    ctx = B.Context(0)
    try:
        prob, vals = wl.taylor_green_2d(seed=5, n=256, ppc=8, steps=20, dt=1e-3)
        d = B.particles_from(prob, dtype=torch.float32)
        v = torch.as_tensor(vals).cuda()
        perm, cs, _ = B.p2m_bin(ctx, d)
        out["perm"], out["cell_start"] = h(perm), h(cs)
        b, w, coef, _ = B.p2m_assemble(ctx, d, v)
        out["b"], out["w"], out["coef"] = h(b), h(w), h(coef)
        for name, code in (("resident", B.SOLVER_RESIDENT), ("chebyshev", B.SOLVER_RESIDENT_CHEB),
                           ("tiles", B.SOLVER_TILES)):
            ctx.set_solver(code)
            x, _ = B.p2m_mass_assign(ctx, d, v, B.solve_opts(tol=1e-8, maxit=2000, max_refine=10))
            out["mass_" + name] = h(x)
        ctx.set_solver(B.SOLVER_AUTO)
        fp, fv = wl.tg_fluid_2d(seed=6, n=128, ppc=4)
        fd = B.particles_from(fp, dtype=torch.float32)
        vel = torch.as_tensor(fv).cuda()
        for _ in range(3):
            B.p2m_ns_step(ctx, fd, vel, B.NS_MASS, 0.5 / 128, 0.005, B.solve_opts(tol=1e-8))
        out["fluid_vel"], out["fluid_x"] = h(vel), h(fd.x)
        torch.cuda.synchronize()
    finally:
        ctx.close()
    return out


if __name__ == "__main__":
    print(json.dumps(digests()), flush=True)
