"""Training and evaluation of the learned warm start (harness).

Training data are trajectories the solver itself generates on fresh seeded
Cu polycrystals (64^3 with 8 grains, 128^3 with 62 grains; the same
dimensionless time increment and pulse as the 256^3 benchmark).  For every
step the library computes the network features from the state before the
step (nm_ws_features) and the target correction from the converged state
after it (nm_ws_target); training steps (forward, loss, backward, Adam) run
in the library's matrix-core kernels.  This module only orchestrates.

    python -m paper_2211_08263_amd.warmstart --out paper_2211_08263_amd/weights/warmstart_cu.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_cu.npy")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def training_problems(n64: int = 4, n128: int = 2, steps: int = 60):
    from . import workloads as W
    for k in range(n64):
        yield W.make_polycrystal(n=64, n_grains=8, seed=1000 + k, n_steps=steps)
    for k in range(n128):
        yield W.make_polycrystal(n=128, n_grains=62, seed=2000 + k, n_steps=steps)


def collect(pb, net, steps: int, tol: float = 1e-8, skip: int = 2):
    """(grid, features, target) device tensors for steps skip+1 .. steps of one trajectory."""
    import torch
    from . import newmark as nmb
    N = pb.n_vox
    out = []
    with nmb.newmark_init_problem(pb, nmb.Options(tol=tol, max_iter=500, warm_start=nmb.WS_COLD)) as ctx:
        nmb.ws_attach(ctx, net)
        for s in range(steps):
            f = torch.empty(N * 32, dtype=torch.int16, device="cuda")
            t = torch.empty(N * 4, dtype=torch.float32, device="cuda")
            nmb.ws_features(ctx, f)
            nmb.newmark_step(ctx, pb.U(s + 1))
            nmb.ws_target(ctx, t)
            if s >= skip:
                out.append((pb.n, f, t))
    return out


def train(net, samples, epochs: int, lr: float, seed: int = 0, log_every: int = 1):
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(samples))
        tot = 0.0
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))  # cosine decay
        for i in order:
            g, f, t = samples[i]
            tot += net.train_step(g, f, t, lr=float(lr_ep))
        hist.append(tot / len(samples))
        if ep % log_every == 0 or ep == epochs - 1:
            _log(f"[train] epoch {ep} lr {lr_ep:.2e} loss {hist[-1]:.5f}")
    return hist


def target_energy(samples):
    """Mean squared target (the loss of a zero correction, i.e. of the plain predictor)."""
    tot = 0.0
    for _, _, t in samples:
        v = t.view(-1, 4)[:, :3].double()
        tot += float((v * v).mean())
    return tot / len(samples)


def evaluate(pb, net, steps: int, tol: float = 1e-8):
    """Mean PCG iterations and mean initial relative residual per step (steps 3..) for
    each initial iterate on one trajectory."""
    from . import newmark as nmb
    res = {}
    for name, ws in (("cold", nmb.WS_COLD), ("prev", nmb.WS_PREV), ("taylor", nmb.WS_TAYLOR),
                     ("learned", nmb.WS_LEARNED)):
        with nmb.newmark_init_problem(pb, nmb.Options(tol=tol, max_iter=500, warm_start=ws)) as ctx:
            if ws == nmb.WS_LEARNED:
                nmb.ws_attach(ctx, net)
            st = [nmb.newmark_step(ctx, pb.U(s + 1)) for s in range(steps)]
        res[name] = {"iters": float(np.mean([x["iters"][0] for x in st[2:]])),
                     "relres0": float(np.exp(np.mean([np.log(max(x["relres0"], 1e-300)) for x in st[2:]])))}
    return res


def load_weights(net, path: str = DEFAULT_WEIGHTS) -> bool:
    if not os.path.exists(path):
        return False
    w = np.load(path, allow_pickle=False)
    net.set_params(w.astype(np.float32))
    return True


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--n64", type=int, default=4)
    ap.add_argument("--n128", type=int, default=2)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    import torch
    from . import newmark as nmb
    from . import workloads as W
    torch.cuda.set_device(0)
    net = nmb.Net(seed=args.seed)
    t0 = time.time()
    trajs = []
    for pb in training_problems(args.n64, args.n128, args.steps):
        ts = time.time()
        trajs.append(collect(pb, net, args.steps))
        _log(f"[data] {pb.name} trajectory: {len(trajs[-1])} samples, {time.time() - ts:.1f}s")
    # the last 64^3 trajectory is held out for validation
    hold = max(args.n64 - 1, 0)
    val = trajs[hold]
    trn = [s for i, tr in enumerate(trajs) if i != hold for s in tr]
    e_zero = target_energy(val)
    _log(f"[data] {len(trn)} training / {len(val)} validation samples in {time.time() - t0:.1f}s; "
         f"zero-correction loss {e_zero:.4f}")
    t1 = time.time()
    hist = train(net, trn, args.epochs, args.lr, seed=args.seed)
    t_train = time.time() - t1
    # validation loss: forward only via gradients call (no update)
    vl = float(np.mean([net.gradients(g, f, t)[1] for g, f, t in val]))
    evals = {}
    for pb in (W.make_polycrystal(n=64, n_grains=8, seed=1000 + hold, n_steps=args.steps),
               W.make_polycrystal(n=128, n_grains=62, seed=3000, n_steps=args.steps)):
        evals[pb.name] = evaluate(pb, net, args.steps)
        _log(f"[eval] {pb.name}: mean PCG iterations per step {evals[pb.name]}")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, net.get_params().astype(np.float32), allow_pickle=False)
    summary = {"train_samples": len(trn), "val_samples": len(val), "epochs": args.epochs, "lr": args.lr,
               "train_loss_first": hist[0], "train_loss_last": hist[-1], "val_loss": vl,
               "val_zero_correction_loss": e_zero, "val_relative_rms_error": (vl / e_zero) ** 0.5,
               "train_seconds": t_train, "mean_iterations": evals, "weights": os.path.relpath(args.out, os.path.dirname(HERE))}
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
