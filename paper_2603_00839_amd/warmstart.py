"""Learned warm start for RTG-GMRES.

The network (six 3x3 convolutions, residual output X0 = C + f(C); kernels in
k_cnn.hip) is trained on pairs (C, X) where X is what the plain float32
RTG-GMRES solver of this library returns for C: 128x128x3 synthetic images
(rectangles + Gaussian random field), Gaussian blur sigma ~ U(1,3), noise
1e-3..1e-2, sketch 16x16x3, m = 50, discrepancy-principle mu.  The solver then
corrects from X0, so the plain solver both supplies the labels and removes
whatever error the warm start leaves.

Usage (on a GPU):  python -m paper_2603_00839_amd.warmstart train --count 20000
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import rtg, synth

HERE = os.path.dirname(os.path.abspath(__file__))
DATA_DIR = os.path.join(HERE, "data")
DEFAULT_WEIGHTS = os.path.join(DATA_DIR, "warmstart_cfg5.npy")
SIDE = 128


def _gen(args):
    seed, p = args
    pr = synth.cfg5_problem(seed, p, SIDE)
    return (pr.x_true, pr.a1_band, pr.a2_band, pr.b_band, pr.om1, pr.om2, pr.noise_dir, pr.nu)


def make_pool(workers: int):
    """Fork the generator workers before the GPU is touched in this process."""
    return mp.get_context("fork").Pool(workers)


def observation(op, x_true_dev, noise_dev, nu):
    """C = Phi(X) + N with ||N|| = nu ||Phi(X)|| (eq. (59)); returns (C, delta)."""
    import torch
    chat = rtg.apply_operator(op, x_true_dev)
    delta = nu * float(torch.linalg.vector_norm(chat.double()))
    C = chat + noise_dev * (delta / float(torch.linalg.vector_norm(noise_dev.double())))
    return C.contiguous(), delta


def make_pairs(pool, count: int, seed: int = 0, chunk: int = 512, m: int = 50, device="cuda", log=print):
    """Observations C and plain float32 RTG-GMRES solutions for `count`
    training problems, as device tensors (count, 3, SIDE, SIDE).  `pool` (or
    None for serial generation) must have been created before this process
    touched the GPU."""
    import torch
    C_all = torch.empty((count, 3, SIDE, SIDE), dtype=torch.float32, device=device)
    Y_all = torch.empty_like(C_all)
    t0 = time.time()
    iters = []
    for start in range(0, count, chunk):
        n = min(chunk, count - start)
        jobs = [(seed, p) for p in range(start, start + n)]
        arrs = pool.map(_gen, jobs) if pool is not None else [_gen(j) for j in jobs]
        ops, sks, Cs, prms = [], [], [], []
        for i, (xt, a1, a2, bb, o1, o2, g, nu) in enumerate(arrs):
            op = rtg.setup_operator(SIDE, SIDE, 3, a1, a2, bb)
            sk = rtg.setup_sketch(SIDE, SIDE, 3, o1, o2, None)
            xd = torch.from_numpy(synth.to_device_layout(xt)).to(device)
            gd = torch.from_numpy(synth.to_device_layout(g)).to(device)
            C, delta = observation(op, xd, gd, nu)
            C_all[start + i].copy_(C)
            ops.append(op)
            sks.append(sk)
            Cs.append(C_all[start + i])
            prms.append(rtg.make_params(m, rtg.F32, delta=delta, eta=1.01))
        plan = rtg.BatchPlan(ops, sks, Cs, [None] * n, prms, outs=[Y_all[start + i] for i in range(n)],
                             device=device)
        plan.run()
        iters += [inf.iters for inf in plan.infos()]
        del plan
        log(f"[warmstart] pairs {start + n}/{count} ({time.time() - t0:.1f} s)")
    return C_all, Y_all, iters


def train(net, C_all, Y_all, epochs: int = 20, batch: int = 32, lr0: float = 1e-3, seed: int = 0, log=print):
    """Adam with a cosine learning-rate schedule over `epochs` passes."""
    import torch
    count = C_all.shape[0]
    spe = count // batch
    total = epochs * spe
    gen = torch.Generator().manual_seed(seed)
    history = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(count, generator=gen).to(C_all.device)
        acc = torch.zeros(1, dtype=torch.float64, device=C_all.device)
        for it in range(spe):
            idx = perm[it * batch:(it + 1) * batch]
            Cb = C_all.index_select(0, idx)
            Yb = Y_all.index_select(0, idx)
            lr = lr0 * 0.5 * (1.0 + math.cos(math.pi * step / total))
            loss = net.train_step(Cb, Yb, lr)
            acc += loss.double()
            step += 1
        mse = float(acc.item()) / (spe * batch * 3 * SIDE * SIDE)
        history.append(mse)
        log(f"[warmstart] epoch {ep + 1}/{epochs} mse {mse:.4e}")
    return history


def initial_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, zero last layer (X0 = C at the start);
    flat C-ABI layout."""
    rng = np.random.default_rng(seed)
    chans = [3, 32, 32, 32, 32, 32, 3]
    parts = []
    for l in range(6):
        ci, co = chans[l], chans[l + 1]
        if l == 5:
            w = np.zeros((co, 3, 3, ci))
        else:
            w = rng.standard_normal((co, 3, 3, ci)) * math.sqrt(2.0 / (9 * ci))
        parts += [w.reshape(-1), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def load_default(device="cuda", path: str = DEFAULT_WEIGHTS) -> rtg.WarmStartNet:
    if not os.path.exists(path):
        raise FileNotFoundError(f"no trained warm-start weights at {path}")
    return rtg.WarmStartNet(np.load(path), device=device)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    pool = make_pool(args.workers)           # before any GPU call
    import torch
    log = lambda s: print(s, flush=True)  # noqa: E731
    t0 = time.time()
    C_all, Y_all, iters = make_pairs(pool, args.count, seed=args.seed, log=log)
    pool.close()
    t_pairs = time.time() - t0
    net = rtg.WarmStartNet(initial_params(args.seed))
    with torch.no_grad():
        base = float(torch.mean((C_all - Y_all) ** 2).item())
    log(f"[warmstart] mse of X0 = C against the labels: {base:.4e}")
    t1 = time.time()
    hist = train(net, C_all, Y_all, epochs=args.epochs, batch=args.batch, lr0=args.lr, seed=args.seed, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    params = net.export()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params)
    meta = {"count": args.count, "side": SIDE, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
            "seed": args.seed, "label_solver": "plain float32 RTG-GMRES, m=50, sketch 16x16x3, discrepancy",
            "label_iters_mean": float(np.mean(iters)), "mse_x0_equals_c": base, "mse_per_epoch": hist,
            "seconds_pairs": t_pairs, "seconds_train": t_train}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(json.dumps(meta))


if __name__ == "__main__":
    main()
