"""Throughput of the particle->mesh mass assignment on one MI355X.

Workload (the headline metric's configuration): 2D periodic [0, 2 pi)^2, 1024 x 1024
P1 mesh, 8 stratified particles per cell (8,388,608 particles, seed 2), Taylor-Green
u, v, p with N(0, 1e-3) noise sampled at the initial positions, positions advected
50 RK2 steps of dt = 1e-3; all 3 fields in one call; FP32 scatter / CG with FP64
residuals, refinement and dot products.  Synthetic inputs, resident in HBM before
timing.

One step = one full mass assignment of the 3 fields: binning + scatter-assemble
(p2m_assemble) followed by the solve (p2m_mass_solve) -- together exactly the
kernels of p2m_mass_assign.  value = fields x steps / wall time of the timed steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--tol 1e-8] [--no-cpu]

Prints one JSON line.  Besides the contract keys it carries
  roofline     : HBM roofline of the dominant kernel (the mass solve, one launch
                 per step), algorithmic bytes per launch / its event-timed duration;
  cpu_baseline : the FP64 CPU oracle timed on this host, one thread, on the full input;
  accuracy     : relative l2 error of the GPU result against the FP64 oracle
                 solution of the same input, per field;
  phases       : event-timed milliseconds of the two calls of a step;
  batched      : the uneven batch (64 independent TG problems, sides log-uniform
                 in [32, 512], 2-16 particles per cell, F = 2, seed 3) as one
                 p2m_mass_assign_batched graph launch: aggregate projections/s,
                 the same 64 problems as 64 p2m_mass_assign calls, and the worst
                 per-instance error against the FP64 oracle (--no-batch skips it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle→mesh mass-assignments/sec at 2D 1024² P1, 8 ppc, rel err ≤1e-6"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cg_algorithmic_bytes(k_ref, nn, F, c_m=4):
    """Bytes a CG solve of k_ref iterations must move: per iteration and node the
    c_m stencil coefficients (4 B each) and, per field, a fused read/write of
    x, r and p (24 B)."""
    return float(k_ref) * nn * (4 * c_m + 24 * F)


def mass_assign_algorithmic_bytes(n_part, nn, F, k_ref, d=2, c_m=4, with_vol=False):
    """Bytes one mass assignment must move end to end: the particle stream
    (d coordinates, F values, the volume if given: 4 B each), the F nodal results,
    and k_ref CG iterations of the stencil and the fused x, r, p traffic."""
    return float(n_part * (4 * d + 4 * F + (4 if with_vol else 0)) + nn * 4 * F +
                 k_ref * nn * (4 * c_m + 24 * F))


# committed memory-counter summaries of the resident solve kernels on this workload,
# and the sources each one was taken from
COUNTERS = {2: (os.path.join(ROOT, "profiles", "counters_k_cgr3_tg1024.md"),
                ("k_cgr.hip", "cg_common.hpp", "p2m_internal.hpp")),
            4: (os.path.join(ROOT, "profiles", "counters_k_cgrc3_tg1024.md"),
                ("k_cgrc.hip", "cg_common.hpp", "p2m_internal.hpp"))}


def measured_traffic(solver, inner_rtol):
    """HBM bytes per launch of the resident solve kernel from its committed counter
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a copy of known size), or None
    when there is none for this solver, or the kernel's sources or the solve schedule
    (inner_rtol) differ from those of the counted run."""
    import hashlib
    import re
    if solver not in COUNTERS or not os.path.exists(COUNTERS[solver][0]):
        return None
    path, sources = COUNTERS[solver]
    text = open(path).read()
    m_t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    m_h = re.search(r"^source_sha256: ([0-9a-f]{64})", text, re.M)
    m_r = re.search(r"^inner_rtol: (\S+)", text, re.M)
    if not (m_t and m_h and m_r) or float(m_r.group(1)) != float(inner_rtol):
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1610_05258_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return float(m_t.group(1)) if h.hexdigest() == m_h.group(1) else None


def solver_sources_sha256(solver):
    """sha256 of the sources of a resident solve kernel (recorded in its counter summary)."""
    import hashlib
    h = hashlib.sha256()
    for f in COUNTERS[solver][1]:
        with open(os.path.join(ROOT, "paper_1610_05258_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def oracle_reference(prob, vals, tol):
    """FP64 oracle on the full input: the solution (to 1e-12) and the iteration
    count of FP64 Jacobi-preconditioned CG (the solver's iteration) from the FLIP
    start to ``tol`` (the roofline's K_ref)."""
    from oracle import p1
    pr = dict(prob, x=prob["x"].astype(np.float64), y=prob["y"].astype(np.float64))
    st = p1.assemble_stencil(pr, vals.astype(np.float64))
    M = p1.regularised_matrix(p1.stencil_matrix(pr, st), st["w"])
    w = st["w"]
    xs, k_ref = [], []
    for f in range(vals.shape[0]):
        b = np.where(w > 0, st["b"][f], 0.0)
        x0 = np.where(w > 0, b / np.where(w > 0, w, 1.0), 0.0)
        _, it = p1.pcg_jacobi_fp64(M, b, x0=x0, rtol=tol)
        k_ref.append(it)
        x, _ = p1.cg_fp64(M, b, x0=x0, rtol=1e-12)
        xs.append(x)
    return np.stack(xs), k_ref


def cpu_baseline(prob, vals, min_seconds=10.0):
    """The FP64 oracle's mass assignment (as it stands, p1.mass_assign) on the
    benchmark input itself, repeated until min_seconds have passed, with every
    BLAS / OpenMP pool held to one thread (numpy's bincount and scipy's sparse
    products are single-threaded)."""
    from threadpoolctl import threadpool_limits
    from oracle import p1
    pr = dict(prob, x=prob["x"].astype(np.float64), y=prob["y"].astype(np.float64))
    v = vals.astype(np.float64)
    runs, dt = 0, 0.0
    with threadpool_limits(limits=1):
        while dt < min_seconds or runs == 0:
            t0 = time.perf_counter()
            p1.mass_assign(pr, v)
            dt += time.perf_counter() - t0
            runs += 1
    return dict(value=vals.shape[0] * runs / dt, unit="projections/s", cores=1, kind="oracle",
                sample=f"the full workload (1024x1024, 8 ppc, F=3): {runs} FP64 oracle mass_assign "
                       f"calls (scipy sparse assembly + CG) in {dt:.2f} s on 1 thread of "
                       f"{os.cpu_count()} host cores")


def cpu_baseline_exact2d(n=90, ppc=1, min_seconds=5.0):
    """The FP64 oracle's paper-exact 2D full-mass round trip (oracle/paper2d.py as it
    stands: periodic Delaunay of the particles, Appendix-B right-hand sides, FFT mesh
    solve, sparse LU particle solve) on the first step of the exact2d leg's slotted
    disk, repeated until min_seconds have passed, one thread."""
    import math
    from threadpoolctl import threadpool_limits
    from oracle import paper2d
    from paper_1610_05258_amd import workloads as wl
    x, y = wl.stratified_2d(1, n, n, ppc, 1.0, 1.0)
    a = wl.zalesak_disk(x, y)
    x, y = wl.zalesak_rotate(x, y, 2.0 * math.pi / 100)
    runs, dt = 0, 0.0
    with threadpool_limits(limits=1):
        while dt < min_seconds or runs == 0:
            t0 = time.perf_counter()
            P = paper2d.Paper2D(x, y, n, n, 1.0, 1.0)
            P.m2p_mass(P.p2m_mass(a[None]))
            dt += time.perf_counter() - t0
            runs += 1
    return dict(value=runs / dt, unit="full-mass round trips/s", cores=1, kind="oracle",
                ms_per_step=dt / runs * 1e3,
                sample=f"the exact2d leg's first slotted-disk step ({n}x{n}, {ppc} particle per cell): "
                       f"{runs} FP64 oracle round trips (triangulation, mass P2M, full-mass M2P) in "
                       f"{dt:.2f} s on 1 thread of {os.cpu_count()} host cores")


def batched_leg(B, ctx, check, tune, reps=10, tol=1e-9):
    """The uneven batch as one graph launch, and as one call per problem.  With `tune`
    the batch's inner_rtol is tuned first (unless a loaded plan covers it); the single
    calls then run with the inner_rtol the batch ran with, so they give the same bits."""
    import torch
    from paper_1610_05258_amd import workloads as wl
    insts = wl.uneven_batch(seed=3, count=64)
    probs = [B.particles_from(p, dtype=torch.float32) for p, _ in insts]
    vals = [torch.as_tensor(v).cuda() for _, v in insts]
    F = insts[0][1].shape[0]
    opts = B.solve_opts(tol=tol, inner_rtol=1e-4, maxit=2000, max_refine=10)
    bt = B.Batch(ctx, probs, vals, opts)
    plan = bt.plan()
    if plan is None and tune:
        plan = bt.tune()
        log(f"bench: batch plan {plan}")
    if plan is not None and plan.inner_rtol >= 0.0:
        opts = B.solve_opts(tol=tol, inner_rtol=plan.inner_rtol, maxit=2000, max_refine=10)
    for _ in range(2):
        bt.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bt.run()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    outs = [torch.empty_like(o) for o in bt.out]
    rep_s = [ctx.new_report() for _ in insts]
    ws = ctx.workspace(max(ctx.workspace_size(p, F) for p in probs))

    def singles():
        for k in range(len(insts)):
            B.p2m_mass_assign(ctx, probs[k], vals[k], opts, ws=ws, rep=rep_s[k], out=outs[k])
    singles()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        singles()
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / reps
    r = bt.reports()
    bitwise = all(torch.equal(a, b) for a, b in zip(bt.out, outs))
    res = dict(workload="64 independent taylor-green u,v problems, side log-uniform [32,512], "
                        "2-16 stratified particles per cell, seed 3, F=2, tol=%g" % tol,
               nodes=int(sum(p.n_nodes for p in probs)),
               particles=int(sum(p.n_particles for p in probs)),
               value=len(insts) * F / t_batch, unit="projections/s", ms_per_batch=t_batch * 1e3,
               single_calls_ms=t_single * 1e3, speedup_vs_single_calls=t_single / t_batch,
               bitwise_equal_to_single_calls=bool(bitwise), inner_rtol=opts.inner_rtol,
               max_iters=int(max(int(x.iters[:F].max()) for x in r)),
               max_rel_residual=float(max(float(x.rel_residual[:F].max()) for x in r)),
               flags=int(np.bitwise_or.reduce([x.flags for x in r])))
    log(f"bench: batched {t_batch * 1e3:.3f} ms ({res['value']:.0f} projections/s), "
        f"single calls {t_single * 1e3:.3f} ms, bitwise {bitwise}")
    if check:
        from oracle import metrics
        from oracle import p1
        worst, worst_inf = 0.0, 0.0
        b_alg = 0.0
        for k, (p, v) in enumerate(insts):
            pr = dict(p, x=p["x"].astype(np.float64), y=p["y"].astype(np.float64))
            st = p1.assemble_stencil(pr, v.astype(np.float64))
            M = p1.regularised_matrix(p1.stencil_matrix(pr, st), st["w"])
            got = bt.out[k].cpu().numpy().astype(np.float64)
            w = st["w"]
            k_ref = 0
            for f in range(F):
                x, _ = p1.cg_fp64(M, st["b"][f], rtol=1e-12)
                worst = max(worst, metrics.rel_l2(got[f], x))
                worst_inf = max(worst_inf, metrics.rel_linf(got[f], x))
                bf = np.where(w > 0, st["b"][f], 0.0)
                x0 = np.where(w > 0, bf / np.where(w > 0, w, 1.0), 0.0)
                k_ref = max(k_ref, p1.pcg_jacobi_fp64(M, bf, x0=x0, rtol=tol)[1])
            b_alg += mass_assign_algorithmic_bytes(p["x"].size, p["nx"] * p["ny"], F, k_ref)
        res["max_instance_rel_l2"] = worst
        res["max_instance_rel_linf"] = worst_inf
        gbs = b_alg / t_batch / 1e9
        res["roofline"] = dict(bound="hbm", scope="whole batch graph (binning, scatter, persistent solve)",
                               bytes_per_launch=b_alg, achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=gbs / HBM_PEAK_GBS,
                               k_ref="per instance: FP64 Jacobi-PCG iterations of the oracle from "
                                     "the FLIP start to the batch tol")
        log(f"bench: batched worst instance rel_l2 {worst:.2e}, B_alg {b_alg / 1e9:.3f} GB "
            f"-> {gbs:.0f} GB/s")
    return res


def cold_leg(one_step, stream, samples=5, flush_mib=1024):
    """Steps timed one by one with the device caches flushed first: a 1 GiB buffer
    is written before each sample, evicting the 256 MB MALL and the L2s, so the
    particle stream and the nodal arrays come from HBM."""
    import torch
    flush = torch.empty(flush_mib << 20, dtype=torch.uint8, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for k in range(samples):
        flush.fill_(k & 0xFF)
        torch.cuda.synchronize()
        e0.record(stream)
        one_step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del flush
    return float(np.median(ms)), [float(v) for v in ms]


def tophat_1d_leg(B, ctx, calls=50):
    """The 1D plain-method workload (64 P1 elements, 256 uniform particles, top-hat on
    [0.25, 0.5), FP64): latency of each call, event-timed over `calls` calls, and
    the relative l2 error of each result against the FP64 oracle."""
    import torch
    from oracle import metrics, p1
    from paper_1610_05258_amd import workloads as wl
    prob, vals = wl.tophat_1d(seed=0)
    d = B.particles_from(prob, dtype=torch.float64)
    v = torch.as_tensor(vals).cuda()
    opts = B.solve_opts(tol=1e-13, maxit=500, max_refine=10, fp64=True)
    stream = torch.cuda.current_stream()
    calls_of = dict(
        delta=lambda: B.p2m_assign(ctx, d, B.DELTA, v)[0],
        flip=lambda: B.p2m_assign(ctx, d, B.FLIP, v)[0],
        mass=lambda: B.p2m_mass_assign(ctx, d, v, opts)[0],
    )
    out = {}
    res = {}
    for name, fn in calls_of.items():
        for _ in range(3):
            res[name] = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(calls):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out[f"{name}_us"] = e0.elapsed_time(e1) / calls * 1e3
    nodal = res["mass"]
    m2p = lambda: B.p2m_interpolate(ctx, d, nodal)[0]
    back = m2p()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(calls):
        m2p()
    e1.record(stream)
    torch.cuda.synchronize()
    out["m2p_us"] = e0.elapsed_time(e1) / calls * 1e3
    ref = dict(delta=p1.delta_1d(prob, vals)[0], flip=p1.flip(prob, vals)[0][0],
               mass=p1.mass_assign(prob, vals, solver="direct")[0][0])
    out["rel_l2"] = {k: metrics.rel_l2(res[k].cpu().numpy()[0], ref[k]) for k in ref}
    out["rel_l2"]["m2p"] = metrics.rel_l2(back.cpu().numpy()[0],
                                          p1.interpolate(prob, nodal.cpu().numpy())[0])
    out["workload"] = "1D periodic [0,1), 64 P1 elements, 256 uniform particles (seed 0), top-hat [0.25,0.5), FP64"
    log(f"bench: 1D top-hat latency delta {out['delta_us']:.1f} us, flip {out['flip_us']:.1f} us, "
        f"mass {out['mass_us']:.1f} us, m2p {out['m2p_us']:.1f} us")
    return out


def zalesak_leg(B, ctx, steps=100, tol=1e-8, tune=True):
    """The slotted-disk workload: 256^2, 4 ppc, 100 steps of (mass_assign -> M2P) with
    the particle values carried from step to step.  The rotated FP32 positions of
    every step are computed on the host (exact FP64 rotation) and uploaded before
    timing; the timed loop is the 100 steps on the device, after the solve plan of
    the shape class is tuned on the first step's input (unless a loaded plan covers
    it)."""
    import torch
    from paper_1610_05258_amd import workloads as wl
    prob, a0, x64, y64 = wl.zalesak_2d(seed=1, n=256, ppc=4)
    xs, ys = [], []
    for _ in range(steps):
        x64, y64 = wl.zalesak_rotate(x64, y64, wl.ZALESAK_DT)
        xs.append(x64.astype(np.float32))
        ys.append(y64.astype(np.float32))
    X = torch.as_tensor(np.stack(xs)).cuda()
    Y = torch.as_tensor(np.stack(ys)).cuda()
    ds = [B.Particles(2, 256, 256, 1.0, 1.0, X[k], Y[k], None) for k in range(steps)]
    A0 = torch.as_tensor(a0).cuda()
    opts = B.solve_opts(tol=tol, maxit=1000, max_refine=10)
    ws = ctx.workspace(ctx.workspace_size(ds[0], 1))
    rep = ctx.new_report()
    nodal = torch.empty((1, 256 * 256), dtype=torch.float32, device="cuda")
    vals = [A0.clone(), torch.empty_like(A0)]
    plan = None
    if tune:
        plan = ctx.plan(ds[0], 1)
        if plan is None:
            plan, _, _ = B.p2m_tune(ctx, ds[0], A0, opts)
        torch.cuda.synchronize()

    def run():
        vals[0].copy_(A0)
        for k in range(steps):
            B.p2m_mass_assign(ctx, ds[k], vals[k & 1], opts, ws=ws, rep=rep, out=nodal)
            B.p2m_interpolate(ctx, ds[k], nodal, out=vals[(k + 1) & 1])
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = B.read_report(rep, 1)
    fin = vals[steps & 1].cpu().numpy()[0]
    out = dict(workload="slotted disk, 2D periodic unit square 256x256 P1, 4 stratified ppc (seed 1), "
                        f"100 rotation steps dt=2pi/628, FP32, tol={tol:g}",
               steps=steps, steps_per_s=steps / wall, ms_per_step=wall / steps * 1e3,
               last_iters=int(r.iters[0]), last_rel_residual=float(r.rel_residual[0]),
               final_min=float(fin.min()), final_max=float(fin.max()))
    if plan is not None:
        out["plan"] = dict(solver=int(plan.solver), groups=int(plan.groups),
                           scatter_tile=int(plan.scatter_tile), inner_rtol=float(plan.inner_rtol),
                           tuned_ms=float(plan.time_ms))
    log(f"bench: zalesak {out['steps_per_s']:.0f} steps/s ({out['ms_per_step']:.3f} ms/step)")
    return out


def ns_leg(B, ctx, n=256, ppc=4, t_end=0.25, tol=1e-8, tune=True):
    """The particle fluid solver (Sec. 3.3): Taylor-Green vortex sheet, Re = 200, on an
    n x n mesh with ppc particles per cell, Courant number 0.5 (dt = h / 2), to
    t_end; FLIP and mass assignment (its P2M solve plan tuned first).  Timed: the whole
    run of steps on the device;
    reported with the velocity error of eq. (29) (uniform volumes) against the exact
    solution at t_end."""
    import torch
    from paper_1610_05258_amd import workloads as wl
    nu = 0.005
    dt = 0.5 / n
    steps = int(round(t_end / dt))
    opts = B.solve_opts(tol=tol, maxit=4000, max_refine=20)
    out = dict(workload=f"taylor-green vortex sheet, unit periodic box {n}x{n} P1, {ppc} stratified ppc "
                        f"(seed 4), Re=200, Courant 0.5 (dt={dt:g}), {steps} steps to t={t_end:g}, FP32, "
                        f"tol={tol:g}")
    for name, code in (("flip", B.NS_FLIP), ("mass", B.NS_MASS)):
        prob, vel0 = wl.tg_fluid_2d(seed=4, n=n, ppc=ppc)
        X0, Y0 = torch.as_tensor(prob["x"]).cuda(), torch.as_tensor(prob["y"]).cuda()
        d = B.particles_from(prob, dtype=torch.float32)
        V0 = torch.as_tensor(vel0).cuda()
        vel = V0.clone()
        mv = torch.empty((2, n * n), dtype=torch.float32, device="cuda")
        reps = torch.zeros((3, B.REPORT_BYTES), dtype=torch.uint8, device="cuda")
        ws = ctx.workspace(B.ns_workspace_size(ctx, d))
        if code == B.NS_MASS and tune:
            # the mass P2M's solve plan for this shape class, tuned on the first step's field
            plan, _, _ = B.p2m_tune(ctx, d, V0, opts)
            torch.cuda.synchronize()
            out["mass_plan"] = dict(solver=int(plan.solver), inner_rtol=float(plan.inner_rtol),
                                    tuned_ms=float(plan.time_ms))

        def run(k):
            d.x.copy_(X0)
            d.y.copy_(Y0)
            vel.copy_(V0)
            for _ in range(k):
                B.p2m_ns_step(ctx, d, vel, code, dt, nu, opts, mesh_vel=mv, reps=reps, ws=ws)
        run(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        x, y, v = d.x.cpu().numpy().astype(np.float64), d.y.cpu().numpy().astype(np.float64), \
            vel.cpu().numpy().astype(np.float64)
        ex = wl.tg_fluid_exact(x, y, steps * dt, nu)
        err = float(np.sqrt(((ex - v) ** 2).sum() / (ex ** 2).sum()))
        r = [B.read_report(reps[k], 2) for k in range(3)]
        out[name] = dict(steps_per_s=steps / wall, ms_per_step=wall / steps * 1e3, l2_error=err,
                         last_step_iters=dict(p2m=r[0].iters[:2].tolist(), viscous=r[1].iters[:2].tolist(),
                                              pressure=int(r[2].iters[0])),
                         flags=[int(q.flags) for q in r])
        log(f"bench: fluid {name}: {out[name]['ms_per_step']:.3f} ms/step, L2 error at t={t_end:g} {err:.3e}, "
            f"last step iterations {out[name]['last_step_iters']}")
    out["mass_over_flip_error"] = out["mass"]["l2_error"] / out["flip"]["l2_error"]
    out["side_not_power_of_two"] = ns_fft_vs_solver(B, ctx, tol=tol)
    return out


def ns_fft_vs_solver(B, ctx, n=192, ppc=4, steps=8, tol=1e-8):
    """One mesh side that is not a power of two (192): FLIP steps of the fluid solver
    with its viscous and pressure systems by the 2D FFT (Bluestein's algorithm for
    the rows) and by the iterative mass-matrix solver (P2M_OPT_FFT off), ms per step
    and the largest difference of the mesh velocities after `steps` steps."""
    import torch
    from paper_1610_05258_amd import workloads as wl
    nu, dt = 0.005, 0.5 / n
    opts = B.solve_opts(tol=tol, maxit=4000, max_refine=20)
    res = dict(workload=f"taylor-green vortex sheet, {n}x{n}, {ppc} ppc, FLIP, {steps} steps")
    mvs = {}
    for name, fft in (("fft", True), ("solver", False)):
        prob, vel0 = wl.tg_fluid_2d(seed=4, n=n, ppc=ppc)
        d = B.particles_from(prob, dtype=torch.float32)
        vel = torch.as_tensor(vel0).cuda()
        mv = torch.empty((2, n * n), dtype=torch.float32, device="cuda")
        reps = torch.zeros((3, B.REPORT_BYTES), dtype=torch.uint8, device="cuda")
        ctx.set_fft(fft)
        try:
            ws = ctx.workspace(B.ns_workspace_size(ctx, d))
            B.p2m_ns_step(ctx, d, vel, B.NS_FLIP, dt, nu, opts, mesh_vel=mv, reps=reps, ws=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps - 1):
                B.p2m_ns_step(ctx, d, vel, B.NS_FLIP, dt, nu, opts, mesh_vel=mv, reps=reps, ws=ws)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        finally:
            ctx.set_fft(True)
        r = B.read_report(reps[2], 1)
        mvs[name] = mv.cpu().numpy().astype(np.float64)
        res[name] = dict(ms_per_step=wall / (steps - 1) * 1e3, pressure_iters=int(r.iters[0]))
    res["mesh_velocity_max_diff"] = float(np.abs(mvs["fft"] - mvs["solver"]).max())
    log(f"bench: fluid at {n}^2 (side not a power of two): FFT {res['fft']['ms_per_step']:.3f} ms/step, "
        f"solver {res['solver']['ms_per_step']:.3f} ms/step ({res['solver']['pressure_iters']} pressure "
        f"iterations), max velocity difference {res['mesh_velocity_max_diff']:.1e}")
    return res


def learned_leg(B, ctx, reps=5, tol=1e-6):
    """The learned-start workload (1024^2, 8 ppc, TG fields with random phase and
    amplitude disordered by 200 RK2 steps, held-out seed 20000): iterations and
    wall time of one mass assignment to residual tol from the learned, FLIP and
    zero starts (the plain CG from FLIP is the fallback and the judge)."""
    import torch
    from paper_1610_05258_amd import workloads as wl
    wpath = os.path.join(ROOT, "paper_1610_05258_amd", "learned_tg.npy")
    prob, vals = wl.tg_disordered(20000, n=1024, ppc=8, steps=200, dt=1e-3, device="cuda")
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    B.set_learned(ctx, torch.as_tensor(np.load(wpath, allow_pickle=False)).cuda())
    out_t = torch.empty((3, 1024 * 1024), dtype=torch.float32, device="cuda")
    rep = ctx.new_report()
    ws = ctx.workspace(ctx.workspace_size(d, 3))
    res = {}
    for name, start in (("flip", B.START_FLIP), ("zero", B.START_ZERO), ("learned", B.START_LEARNED)):
        opts = B.solve_opts(tol=tol, inner_rtol=1e-4, maxit=2000, max_refine=10, start=start)
        B.p2m_mass_assign(ctx, d, v, opts, rep=rep, out=out_t, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            B.p2m_mass_assign(ctx, d, v, opts, rep=rep, out=out_t, ws=ws)
        torch.cuda.synchronize()
        r = B.read_report(rep, 3)
        res[name] = dict(ms=(time.perf_counter() - t0) / reps * 1e3, iters=r.iters[:3].tolist(),
                         rel_residual=r.rel_residual[:3].tolist(), flags=int(r.flags))
    B.set_learned(ctx, None)
    res["workload"] = ("taylor-green 1024x1024, 8 ppc, random phase/amplitude, 200 RK2 disorder steps, "
                       f"held-out seed 20000, F=3, tol={tol:g}")
    res["learned_over_flip_time"] = res["learned"]["ms"] / res["flip"]["ms"]
    res["outcome"] = ("the learned start saves no iteration over FLIP and costs its inference: slower"
                      if res["learned"]["ms"] > res["flip"]["ms"] else "the learned start is faster than FLIP")
    log(f"bench: learned start {res['learned']['ms']:.3f} ms {res['learned']['iters']} vs FLIP "
        f"{res['flip']['ms']:.3f} ms {res['flip']['iters']} vs zero {res['zero']['ms']:.3f} ms")
    return res


def plain_vs_combined_leg(B, ctx, prob, vals, reps=5, tol=1e-6):
    """The plain GPU form against the production form on the headline workload, both
    to residual tol.  Plain: the method as configured for the 1D plain case -- FP64
    positions, values and arithmetic, one field per call, the library's default
    launch choices (no tuned plan), the FLIP start.  Production: the three fields in
    one FP32 call with the FP64 residual / refinement split, the tuned plan, and the
    learned start (FLIP where the proposal is worse).  Ratio = plain / production
    wall time for the same three projections."""
    import torch
    wpath = os.path.join(ROOT, "paper_1610_05258_amd", "learned_tg.npy")
    F = vals.shape[0]
    d64 = B.particles_from(prob, dtype=torch.float64)
    v64 = [torch.as_tensor(vals[f:f + 1].astype(np.float64)).cuda() for f in range(F)]
    d32 = B.particles_from(prob, dtype=torch.float32)
    v32 = torch.as_tensor(vals).cuda()
    o64 = B.solve_opts(tol=tol, maxit=4000, max_refine=10, fp64=True)
    ws64 = torch.empty(ctx.workspace_size(d64, 1), dtype=torch.uint8, device="cuda")
    rep = ctx.new_report()
    out64 = torch.empty((1, prob["nx"] * prob["ny"]), dtype=torch.float64, device="cuda")

    def plain():
        for f in range(F):
            B.p2m_mass_assign(ctx, d64, v64[f], o64, ws=ws64, rep=rep, out=out64)
    ctx.use_plans(False)
    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    r_plain = B.read_report(rep, 1)
    ctx.use_plans(True)
    del ws64
    B.set_learned(ctx, torch.as_tensor(np.load(wpath, allow_pickle=False)).cuda())
    o32 = B.solve_opts(tol=tol, inner_rtol=1e-4, maxit=2000, max_refine=10, start=B.START_LEARNED)
    ws32 = ctx.workspace(ctx.workspace_size(d32, F))
    out32 = torch.empty((F, prob["nx"] * prob["ny"]), dtype=torch.float32, device="cuda")

    def combined():
        B.p2m_mass_assign(ctx, d32, v32, o32, ws=ws32, rep=rep, out=out32)
    combined()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        combined()
    torch.cuda.synchronize()
    t_comb = (time.perf_counter() - t0) / reps
    r_comb = B.read_report(rep, F)
    B.set_learned(ctx, None)
    res = dict(tol=tol,
               plain=dict(form="FP64, one field per call, default launch choices, FLIP start",
                          ms=t_plain * 1e3, projections_per_s=F / t_plain,
                          last_iters=int(r_plain.iters[0])),
               production=dict(form="F=3 in one FP32 call, FP64 residual/refinement, tuned plan, "
                                    "learned start with FLIP fallback",
                               ms=t_comb * 1e3, projections_per_s=F / t_comb,
                               iters=r_comb.iters[:F].tolist(),
                               learned_fallback=bool(r_comb.flags & B.FLAG_LEARNED_FALLBACK)),
               ratio=t_plain / t_comb)
    log(f"bench: plain GPU form {t_plain * 1e3:.3f} ms vs production {t_comb * 1e3:.3f} ms "
        f"(ratio {res['ratio']:.2f})")
    return res


def exact2d_leg(B, ctx, n=90, ppc=1, steps=100, big_n=512, big_ppc=4, calls=5):
    """Paper-exact 2D (Sec. 3.2: P1 hats on the periodic Delaunay triangulation of the
    particles; Appendix-B rule; eq. (20)).

    (1) The slotted-disk rotation at the paper's resolution: a 90 x 90 mesh (the paper's
    H / box ratio), one particle per cell (stratified, seed 1), one revolution in 100
    steps (the paper's dt = tau / 100).  Each step rotates the particles exactly (FP64,
    host), then runs P2M and M2P of one Table 1 method on the GPU in one call
    (p2m_x2d_round_trip: one binning and triangulation); the particles carry the M2P
    values.  E1, E2 and L2 after the revolution (the Sec. 3.1 measures with the
    Delaunay volumes), and the event-timed milliseconds per step.
    (2) Throughput at 512 x 512, four particles per cell (1,048,576 particles): the
    triangulation alone and the full-mass round trip (mass P2M, then mass M2P)."""
    import math
    import torch
    from paper_1610_05258_amd import workloads as wl
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def dev(a):
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()

    x0, y0 = wl.stratified_2d(1, n, n, ppc, 1.0, 1.0)
    a0 = wl.zalesak_disk(x0, y0)
    pairs = dict(delta=(B.X1D_DELTA, B.X1D_DELTA), flip=(B.X1D_FLIP, B.X1D_DELTA),
                 mass_delta=(B.X1D_MASS, B.X1D_DELTA), full_mass=(B.X1D_MASS, B.X1D_MASS))
    d0 = B.Particles(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=dev(x0), y=dev(y0))
    v0 = B.p2m_x2d_volumes(ctx, d0)[0].cpu().numpy()
    out = dict(workload=f"slotted disk, {n}x{n} P1 mesh on [0,1)^2, {ppc} stratified particle per cell "
                        f"(seed 1), one revolution in {steps} steps, FP64")
    for name, (kp, km) in pairs.items():
        x, y = x0.copy(), y0.copy()
        vals = dev(a0[None])
        flags = 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = 0.0
        for _ in range(steps):
            x, y = wl.zalesak_rotate(x, y, 2.0 * math.pi / steps)
            d = B.Particles(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, x=dev(x), y=dev(y))
            torch.cuda.synchronize()
            e0.record(stream)
            nodal, vals, reps = B.p2m_x2d_round_trip(ctx, d, kp, km, vals)
            e1.record(stream)
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            flags |= (B.Report.decode(reps[0].cpu().numpy().tobytes(), 1).flags
                      | B.Report.decode(reps[1].cpu().numpy().tobytes(), 1).flags)
        vT = B.p2m_x2d_volumes(ctx, d)[0].cpu().numpy()
        aT = vals.cpu().numpy()[0]
        s1 = float(np.sum(v0 * a0))
        s2 = float(np.sum(v0 * a0 * a0))
        out[name] = dict(E1=(float(np.sum(vT * aT)) - s1) / s1,
                         E2=(float(np.sum(vT * aT * aT)) - s2) / s2,
                         L2=float(np.sqrt(np.sum(v0 * (aT - a0) ** 2) / s2)),
                         ms_per_step=ms / steps, flags=flags)
        log(f"bench: exact 2D {name}: E1 {out[name]['E1']:+.4f} E2 {out[name]['E2']:+.3f} "
            f"L2 {out[name]['L2']:.3f}, {ms / steps:.3f} ms per step")
    out["paper_table3"] = dict(delta=dict(E1=-0.005, E2=-0.29, L2=0.67),
                               flip=dict(E1=0.0014, E2=-0.61, L2=0.67),
                               mass_delta=dict(E2=-0.50, L2=0.61),
                               full_mass=dict(E1=0.005, E2=-0.09, L2=0.30),
                               note="the paper's 3x3 box and disk, particle count not stated: context")

    xb, yb = wl.stratified_2d(7, big_n, big_n, big_ppc, 1.0, 1.0)
    db = B.Particles(dim=2, nx=big_n, ny=big_n, lx=1.0, ly=1.0, x=dev(xb), y=dev(yb))
    ab = dev(wl.zalesak_disk(xb, yb)[None])
    ws = ctx.workspace(B.x2d_workspace_size(ctx, db, 1))
    tri_ms = timed(lambda: B.p2m_x2d_triangulation(ctx, db, ws=ws), calls)
    nb, _ = B.p2m_x2d_assign(ctx, db, B.X1D_MASS, ab, ws=ws)
    p2m_ms = timed(lambda: B.p2m_x2d_assign(ctx, db, B.X1D_MASS, ab, ws=ws), calls)
    m2p_ms = timed(lambda: B.p2m_x2d_interpolate(ctx, db, B.X1D_MASS, nb, ws=ws), calls)
    rt_ms = timed(lambda: B.p2m_x2d_round_trip(ctx, db, B.X1D_MASS, B.X1D_MASS, ab, ws=ws), calls)
    npb = xb.size
    out["throughput"] = dict(
        workload=f"{big_n}x{big_n} mesh, {big_ppc} stratified particles per cell ({npb} particles), FP64",
        triangulation_ms=tri_ms, particles_triangulated_per_s=npb / (tri_ms * 1e-3),
        mass_p2m_ms=p2m_ms, mass_m2p_ms=m2p_ms, full_mass_round_trip_ms=rt_ms)
    log(f"bench: exact 2D at {big_n}^2 x {big_ppc}: triangulation {tri_ms:.3f} ms, mass P2M "
        f"{p2m_ms:.3f} ms, mass M2P {m2p_ms:.3f} ms, full-mass round trip {rt_ms:.3f} ms")
    return out


def m2p_leg(B, ctx, d, nodal, stream, ws, calls=20):
    """M2P interpolation of the solved fields back to the particles (one p2m_interpolate
    call with a workspace: report clear, node-major copy of the nodal values and
    k_gather2d_nm), event-timed over `calls` calls.  Algorithmic bytes:
    positions (8 B) and F outputs (4F B) per particle, the nodal arrays (4F B per node)
    read once."""
    import torch
    F, nn = nodal.shape
    npart = d.n_particles
    g_out = torch.empty((F, npart), dtype=torch.float32, device="cuda")
    g_rep = ctx.new_report()
    for _ in range(3):
        B.p2m_interpolate(ctx, d, nodal, out=g_out, rep=g_rep, ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(calls):
        B.p2m_interpolate(ctx, d, nodal, out=g_out, rep=g_rep, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    nbytes = npart * (8 + 4 * F) + nn * 4 * F
    gbs = nbytes / (ms * 1e-3) / 1e9
    log(f"bench: M2P gather {ms * 1e3:.1f} us per call ({gbs:.0f} GB/s algorithmic)")
    return dict(ms=ms, particles_per_s=npart / (ms * 1e-3), kernel=f"k_gather2d_nm<float, {F}>",
                bytes_per_call=nbytes, achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=gbs / HBM_PEAK_GBS)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the cold-cache, plain-vs-production, learned-start, 1D top-hat "
                         "and slotted-disk legs")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip p2m_tune (the library's default launch choices are timed)")
    ap.add_argument("--save-plans", default=None, metavar="PATH",
                    help="write the tuned plans to PATH (JSON)")
    ap.add_argument("--load-plans", default=None, metavar="PATH",
                    help="apply the plans in PATH instead of tuning (e.g. for profiler runs, "
                         "whose timings would perturb the tuner)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy MIB MiB device-to-device three times "
                         "(a kernel of known traffic for scaling memory counters)")
    ap.add_argument("--leg", default=None,
                    choices=("fluid", "zalesak", "tophat_1d", "learned", "plain_vs_production",
                             "exact2d"),
                    help="run only this leg (no headline) and print its JSON; for profiling one workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the path runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is designed, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1610_05258_amd import binding as B
    from paper_1610_05258_amd import workloads as wl

    if args.leg is not None:
        B.lib()
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        ctx = B.Context(0)
        if args.leg == "plain_vs_production":
            prob, vals = wl.taylor_green_2d(seed=2, n=args.n, ppc=8, steps=50, dt=1e-3)
            res = plain_vs_combined_leg(B, ctx, prob, vals)
        else:
            res = dict(fluid=ns_leg, zalesak=zalesak_leg, tophat_1d=tophat_1d_leg,
                       learned=learned_leg, exact2d=exact2d_leg)[args.leg](B, ctx)
        print(json.dumps({args.leg: res}), flush=True)
        torch.cuda.synchronize()
        ctx.close()
        return

    B.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = args.n
    log(f"bench: generating TG workload {n}x{n}, 8 ppc, 50 RK2 steps")
    prob, vals = wl.taylor_green_2d(seed=2, n=n, ppc=8, steps=50, dt=1e-3)
    F = vals.shape[0]
    ctx = B.Context(0)
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    nn = n * n
    b = torch.empty((F, nn), dtype=torch.float32, device="cuda")
    w = torch.empty(nn, dtype=torch.float32, device="cuda")
    coef = torch.empty((4, nn), dtype=torch.float32, device="cuda")
    out = torch.empty((F, nn), dtype=torch.float32, device="cuda")
    rep_a = ctx.new_report()
    rep_s = ctx.new_report()
    ws = ctx.workspace(ctx.workspace_size(d, F))
    opts = B.solve_opts(tol=args.tol, inner_rtol=1e-4, maxit=2000, max_refine=10)
    stream = torch.cuda.current_stream()

    # fixed output buffers across steps: call the C entry points directly
    import ctypes
    L = B.lib()
    cp = d.cstruct()
    sp = ctypes.c_void_p(stream.cuda_stream)
    wsp, wsn = ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel())

    def one_step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        st = L.p2m_assemble(ctx.handle, ctypes.byref(cp), ctypes.c_void_p(v.data_ptr()), F,
                            ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                            ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(rep_a.data_ptr()),
                            wsp, wsn, sp)
        assert st == 0, B.status_string(st)
        if ev is not None:
            ev[1].record(stream)
        st = L.p2m_mass_solve(ctx.handle, ctypes.byref(cp), F, ctypes.c_void_p(b.data_ptr()),
                              ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(coef.data_ptr()),
                              ctypes.byref(opts), ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(rep_s.data_ptr()), wsp, wsn, sp)
        assert st == 0, B.status_string(st)
        if ev is not None:
            ev[2].record(stream)

    plan = None
    if args.load_plans:
        ctx.load_plans(args.load_plans)
        plan = ctx.plan(d, F)
        assert plan is not None, f"{args.load_plans} holds no plan for this shape"
        log(f"bench: loaded plan {plan}")
    elif not args.no_tune:
        plan, _, _ = B.p2m_tune(ctx, d, v, opts)
        torch.cuda.synchronize()
        log(f"bench: tuned plan {plan}")
    if plan is not None and args.save_plans:
        ctx.save_plans(args.save_plans)
    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    # HIP events on every EV_EVERY-th timed step give the phase split and the solve
    # kernel's duration; an event record adds a queue gap of a few microseconds, so
    # the other steps run without them
    EV_EVERY = 4
    evs = {k: [torch.cuda.Event(enable_timing=True) for _ in range(3)]
           for k in range(0, args.steps, EV_EVERY)}
    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(evs.get(k))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copied {args.calibrate_copy} MiB three times (counter calibration)")
        del src, dst
    asm_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs.values()]))
    cg_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs.values()]))
    r = B.read_report(rep_s, F)
    log(f"bench: {wall / args.steps * 1e3:.3f} ms/step (assemble {asm_ms:.3f} ms, solve {cg_ms:.3f} ms), "
        f"iters {r.iters.tolist()}, refines {r.refines.tolist()}, relres {r.rel_residual.tolist()}")
    result = dict(metric=METRIC, value=F * args.steps / wall, unit="projections/s", n_gpus=1,
                  steps=args.steps, warmup=args.warmup, ms_per_step=wall / args.steps * 1e3,
                  higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32+f64",
                  data="synthetic",
                  config=dict(workload=f"taylor-green 2D periodic {n}x{n} P1, 8 ppc stratified seed 2, "
                                       f"50 RK2 steps dt=1e-3, F=3 (u,v,p + N(0,1e-3)), tol={args.tol:g}",
                              nodes=nn, particles=int(vals.shape[1]), fields=F, tol=args.tol),
                  plan=None if plan is None else dict(solver={1: "streaming (k_cg)", 2: "resident (k_cgr)",
                                                              3: "tile-streaming (k_cgb)",
                                                              4: "resident, Chebyshev (k_cgrc)"}[plan.solver],
                                                      groups=plan.groups, scatter_tile=plan.scatter_tile or 15,
                                                      inner_rtol=(plan.inner_rtol if plan.inner_rtol >= 0
                                                                  else opts.inner_rtol),
                                                      tuned_ms=plan.time_ms),
                  phases=dict(assemble_ms=asm_ms, solve_ms=cg_ms, cg_iters=r.iters.tolist(),
                              refines=r.refines.tolist(), rel_residual=r.rel_residual.tolist(),
                              flags=r.flags))
    result["m2p"] = m2p_leg(B, ctx, d, out, stream, ws)
    if not args.no_extra:
        cold_ms, cold_all = cold_leg(one_step, stream)
        warm_ms = asm_ms + cg_ms
        result["cold"] = dict(ms_per_step=cold_ms, samples_ms=cold_all, warm_ms_per_step=warm_ms,
                              flush="1 GiB written before each sample (MALL 256 MB, L2s evicted)")
        log(f"bench: cold step {cold_ms:.3f} ms (warm {warm_ms:.3f} ms, event-timed)")
    k_ref = None
    if not args.no_cpu:
        log("bench: FP64 oracle on the full input (accuracy and K_ref)")
        x_ref, k_ref = oracle_reference(prob, vals, args.tol)
        got = out.cpu().numpy().astype(np.float64)
        from oracle import metrics
        result["accuracy"] = dict(
            rel_l2=[metrics.rel_l2(got[f], x_ref[f]) for f in range(F)],
            rel_linf=[metrics.rel_linf(got[f], x_ref[f]) for f in range(F)],
            reference="FP64 oracle: particle-quadrature system assembled in FP64 from the same FP32 "
                      "inputs, CG to 1e-12")
        log(f"bench: accuracy {result['accuracy']['rel_l2']}, K_ref {k_ref}")
        log("bench: CPU baseline (oracle on the full input, one thread)")
        result["cpu_baseline"] = cpu_baseline(prob, vals)
        if not args.no_extra:
            result["cpu_baseline"]["exact2d"] = cpu_baseline_exact2d()
            log(f"bench: oracle full-mass round trip (90^2, exact 2D) "
                f"{result['cpu_baseline']['exact2d']['ms_per_step']:.1f} ms on 1 thread")
    if not args.no_batch:
        result["batched"] = batched_leg(B, ctx, check=not args.no_cpu, tune=not args.no_tune)
        if args.save_plans:
            ctx.save_plans(args.save_plans)
    if not args.no_extra:
        result["plain_vs_production"] = plain_vs_combined_leg(B, ctx, prob, vals)
        result["learned"] = learned_leg(B, ctx)
        result["tophat_1d"] = tophat_1d_leg(B, ctx)
        result["zalesak"] = zalesak_leg(B, ctx)
        result["fluid"] = ns_leg(B, ctx)
        result["exact2d"] = exact2d_leg(B, ctx)
    if k_ref is not None:
        kk = max(k_ref)
        b_e2e = mass_assign_algorithmic_bytes(int(vals.shape[1]), nn, F, kk)
        for name, ms in (("warm", wall / args.steps * 1e3),
                         ("cold", result.get("cold", {}).get("ms_per_step"))):
            if ms is None:
                continue
            gbs = b_e2e / (ms * 1e-3) / 1e9
            result.setdefault("roofline_e2e", dict(
                scope="whole mass assignment (binning, scatter, solve) per step", bound="hbm",
                bytes_per_step=b_e2e, peak=HBM_PEAK_GBS, unit="GB/s", k_ref=kk))[name] = dict(
                    ms_per_step=ms, achieved=gbs, frac=gbs / HBM_PEAK_GBS)
    if k_ref is not None:
        kk = max(k_ref)
        achieved = cg_algorithmic_bytes(kk, nn, F) / (cg_ms * 1e-3) / 1e9
        solver = plan.solver if plan is not None else 2
        kernel = {1: f"k_cg<float,2,{F}> (grid-synchronised mass solve)",
                  2: f"k_cgr<{F}> (register-resident mass solve)",
                  3: f"k_cgb<{F}> (tile-streaming mass solve)",
                  4: f"k_cgrc<{F}> (register-resident mass solve, Chebyshev preconditioner)"}[solver]
        traffic = measured_traffic(solver, result["plan"]["inner_rtol"] if plan is not None
                                   else opts.inner_rtol)
        result["roofline"] = dict(bound="hbm", kernel=kernel,
                                  achieved=achieved,
                                  peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                                  traffic=traffic, k_ref=kk,
                                  bytes_per_launch=cg_algorithmic_bytes(kk, nn, F))
        if traffic is not None:
            # the counted HBM bytes of the same launch: well under the algorithmic ones
            # (the CG state stays in registers and LDS), so the kernel is limited by the
            # latency of its grid barriers, not by HBM bandwidth
            counted = traffic / (cg_ms * 1e-3) / 1e9
            result["roofline"]["achieved_counted"] = counted
            result["roofline"]["frac_counted"] = counted / HBM_PEAK_GBS
            result["roofline"]["limiter"] = ("latency (grid barrier per CG iteration)"
                                             if counted < 0.5 * achieved else "hbm")
    print(json.dumps(result), flush=True)
    # release the library context (and the batch graph it caches) while the HIP
    # runtime is fully alive, rather than from a finaliser at interpreter exit
    torch.cuda.synchronize()
    ctx.close()


if __name__ == "__main__":
    main()
