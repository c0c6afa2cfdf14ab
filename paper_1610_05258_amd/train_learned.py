"""Train the learned warm start on solver-generated pairs and save its parameters.

Each training configuration is a disordered Taylor-Green problem (workloads.
tg_disordered: n x n mesh, 8 particles per cell, random phase and amplitude,
0-400 RK2 steps of 1e-3 drawn per seed); its exact nodal values come from the
library's own mass solve refined to an FP64 residual of 1e-10.  For every usable
node and field the network input is the feature row of p2m_learned_features and
the target (exact - base) / s.  Training runs Adam through p2m_learned_train_step
on random minibatches; a held-out configuration measures the validation loss.

    python -m paper_1610_05258_amd.train_learned [--configs 16] [--n 1024] [--steps 6000]

writes learned_tg.npy (FP32 parameters) and learned_tg.json (recipe and losses)
next to this file.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "learned_tg.npy")
META = os.path.join(HERE, "learned_tg.json")
TRAIN_SEED0 = 10000
VAL_SEED = 19999


def init_params(seed):
    """He-normal hidden layers, small output layer, zero biases and padding."""
    from . import binding as B
    g = np.random.Generator(np.random.PCG64(seed))
    H, NIN, NF = B.LEARNED_HIDDEN, B.LEARNED_NIN, 3 * B.LEARNED_KMAX + 1
    th = np.zeros(B.LEARNED_NPARAM, np.float32)
    o = 0
    W1 = th[o:o + H * NIN].reshape(H, NIN)
    W1[:, :NF] = g.normal(0.0, math.sqrt(2.0 / NF), (H, NF))
    o += H * NIN + H
    th[o:o + H * H] = g.normal(0.0, math.sqrt(2.0 / H), H * H)
    o += H * H + H
    th[o:o + H * H] = g.normal(0.0, math.sqrt(2.0 / H), H * H)
    o += H * H + H
    th[o:o + H] = g.normal(0.0, 0.01, H)
    return th


def make_pairs(B, ctx, seed, n, steps, device="cuda"):
    """Feature rows, targets and usable-row indices of one configuration."""
    import torch
    from . import workloads as wl
    prob, vals = wl.tg_disordered(seed, n=n, ppc=8, steps=steps, dt=1e-3, device=device)
    d = B.particles_from(prob, dtype=torch.float32)
    v = torch.as_tensor(vals).cuda()
    exact, rep = B.p2m_mass_assign(ctx, d, v, B.solve_opts(tol=1e-10, inner_rtol=1e-4, maxit=4000,
                                                          max_refine=20))
    X, base, scale = B.learned_features(ctx, d, v)
    use = scale > 0
    target = torch.zeros_like(base)
    target[use] = (exact.t()[use] - base[use]) / scale[use]
    rows = torch.nonzero(use.reshape(-1)).reshape(-1).to(torch.int32)
    return X.reshape(-1, B.LEARNED_NIN), target.reshape(-1), rows, B.read_report(rep, 3)


def main():
    import torch
    from . import binding as B
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--configs", type=int, default=16)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    B.lib()
    ctx = B.Context(0)
    t0 = time.perf_counter()
    data = []
    for c in range(args.configs):
        seed = TRAIN_SEED0 + c
        dis = int(np.random.Generator(np.random.PCG64(seed)).integers(0, 401))
        X, tgt, rows, rep = make_pairs(B, ctx, seed, args.n, dis)
        data.append((X, tgt, rows))
        print(f"config {seed}: {dis} disorder steps, {rows.numel()} usable rows, "
              f"solve iters {rep.iters.tolist()}", flush=True)
    Xv, tv, rv, _ = make_pairs(B, ctx, VAL_SEED, args.n, 200)
    print(f"data in {time.perf_counter() - t0:.1f} s", flush=True)
    params = torch.as_tensor(init_params(args.seed)).cuda()
    tr = B.Trainer(ctx, params, args.batch)
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)

    def val_loss():
        vals = []
        for k in range(0, min(rv.numel(), 65536), args.batch):
            r = rv[k:k + args.batch]
            vals.append(tr.run(Xv, tv, r, apply=False).item())
        return float(np.mean(vals))

    v0 = val_loss()
    log = []
    t1 = time.perf_counter()
    for it in range(args.steps):
        X, tgt, rows = data[it % len(data)]
        pick = torch.randint(0, rows.numel(), (args.batch,), device="cuda", generator=g)
        lr = args.lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * it / args.steps)))
        loss = tr.run(X, tgt, rows[pick], lr=lr)
        if it % 500 == 0 or it == args.steps - 1:
            log.append((it, loss.item()))
            print(f"step {it}: loss {log[-1][1]:.5f} lr {lr:.2e}", flush=True)
    v1 = val_loss()
    print(f"train {time.perf_counter() - t1:.1f} s; validation loss {v0:.5f} -> {v1:.5f}", flush=True)
    np.save(args.out, params.cpu().numpy(), allow_pickle=False)
    meta = dict(configs=args.configs, n=args.n, ppc=8, disorder_steps="uniform 0..400 per seed",
                train_seeds=[TRAIN_SEED0, TRAIN_SEED0 + args.configs - 1], val_seed=VAL_SEED,
                target="exact from the mass solve at FP64 residual 1e-10", steps=args.steps,
                batch=args.batch, lr=args.lr, schedule="cosine to 5%", init_seed=args.seed,
                val_loss_before=v0, val_loss_after=v1, loss_log=log,
                target_variance=float(tv[rv.long()].var().item()))
    with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)


if __name__ == "__main__":
    main()
