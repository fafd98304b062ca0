"""Training and evaluation of the learned warm start (harness).

Training data are trajectories the solver itself generates on fresh seeded
Cu polycrystals (64^3 with 8 grains, 128^3 with 62 grains; the same
dimensionless time increment and pulse as the 256^3 benchmark).  Three losses:

  energy (default) and residual: for every step the library stores the
    features and the projected residual rp = P(b - A u~_Gamma) of the predictor
    (nm_ws_residual_sample); a training step minimises a norm of the residual
    r0 = rp - s P A P net(f) of the learned initial iterate, relative to that of
    the reference residual: r0 . (P M P r0) (energy: about the A-norm of the
    initial error, which conjugate gradients reduce) or |r0|^2 (residual: the
    quantity of the stopping test) (nm_ws_train_residual: network forward, FP64
    operator and preconditioner applies, backward, Adam);
  mse: the displacement correction (u_{n+1} - u~)/s from the converged step
    (nm_ws_features / nm_ws_target, nm_net_train_step).

All arithmetic runs in the library's kernels; this module only orchestrates.

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


def collect_residual(pb, net, steps: int, tol: float = 1e-8, skip: int = 2):
    """(context, [(features, rp, s, cref)]) for steps skip+1 .. steps of one trajectory; the
    context stays open because training applies its operator."""
    import torch
    from . import newmark as nmb
    N = pb.n_vox
    ctx = nmb.newmark_init_problem(pb, nmb.Options(tol=tol, max_iter=500, warm_start=nmb.WS_COLD))
    nmb.ws_attach(ctx, net)
    out = []
    for s in range(steps):
        f = torch.empty(N * 32, dtype=torch.int16, device="cuda")
        rp = torch.empty(3 * N, dtype=torch.float64, device="cuda")
        sc, cref, crefm = nmb.ws_residual_sample(ctx, pb.U(s + 1), f, rp)
        nmb.newmark_step(ctx, pb.U(s + 1))
        if s >= skip and sc > 0 and cref > 0 and crefm > 0:
            out.append((f, rp, sc, cref, crefm))
    return ctx, out


def train_residual(data, epochs: int, lr: float, seed: int = 0, metric: int = 1):
    """data: [(context, samples)].  Mean loss per epoch (metric 0: relative residual^2 of the
    learned start; metric 1: its relative preconditioned residual norm r.Mr)."""
    from . import newmark as nmb
    flat = [(ctx, *smp) for ctx, smps in data for smp in smps]
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
        tot = 0.0
        for i in rng.permutation(len(flat)):
            ctx, f, rp, sc, cref, crefm = flat[i]
            tot += nmb.ws_train_residual(ctx, f, rp, sc, crefm if metric == 1 else cref, float(lr_ep), metric=metric)
        hist.append(tot / len(flat))
        _log(f"[train] epoch {ep} lr {lr_ep:.2e} mean loss {hist[-1]:.5f}")
    return hist


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
    ap.add_argument("--loss", choices=["energy", "residual", "mse"], default="energy",
                    help="energy: r.(PMP r) of the learned start; residual: |r|^2; mse: displacement")
    ap.add_argument("--n64", type=int, default=4)
    ap.add_argument("--n128", type=int, default=2)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-steps", type=int, default=40)
    args = ap.parse_args()
    import torch
    from . import newmark as nmb
    from . import workloads as W
    torch.cuda.set_device(0)
    net = nmb.Net(seed=args.seed)
    t0 = time.time()
    probs = list(training_problems(args.n64, args.n128, args.steps))
    # the last 64^3 trajectory is held out for validation
    hold = max(args.n64 - 1, 0)
    summary = {"loss": args.loss, "epochs": args.epochs, "lr": args.lr}
    if args.loss in ("energy", "residual"):
        data = []
        for i, pb in enumerate(probs):
            if i == hold:
                continue
            ts = time.time()
            data.append(collect_residual(pb, net, args.steps))
            _log(f"[data] {pb.name} trajectory: {len(data[-1][1])} samples, {time.time() - ts:.1f}s")
        summary["train_samples"] = sum(len(d[1]) for d in data)
        t1 = time.time()
        hist = train_residual(data, args.epochs, args.lr, seed=args.seed, metric=1 if args.loss == "energy" else 0)
        summary["train_seconds"] = time.time() - t1
        for ctx, _ in data:
            ctx.close()
        del data
    else:
        trajs = []
        for pb in probs:
            ts = time.time()
            trajs.append(collect(pb, net, args.steps))
            _log(f"[data] {pb.name} trajectory: {len(trajs[-1])} samples, {time.time() - ts:.1f}s")
        val = trajs[hold]
        trn = [s for i, tr in enumerate(trajs) if i != hold for s in tr]
        summary["train_samples"] = len(trn)
        e_zero = target_energy(val)
        t1 = time.time()
        hist = train(net, trn, args.epochs, args.lr, seed=args.seed)
        summary["train_seconds"] = time.time() - t1
        vl = float(np.mean([net.gradients(g, f, t)[1] for g, f, t in val]))
        summary.update({"val_loss": vl, "val_zero_correction_loss": e_zero,
                        "val_relative_rms_error": (vl / e_zero) ** 0.5})
        del trajs, val, trn
    summary.update({"data_seconds": t1 - t0, "train_loss_first": hist[0], "train_loss_last": hist[-1]})
    evals = {}
    for pb in (W.make_polycrystal(n=64, n_grains=8, seed=1000 + hold, n_steps=args.steps),
               W.make_polycrystal(n=128, n_grains=62, seed=3000, n_steps=args.steps)):
        evals[pb.name] = evaluate(pb, net, args.eval_steps)
        _log(f"[eval] {pb.name}: {evals[pb.name]}")
    summary["held_out"] = evals
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, net.get_params().astype(np.float32), allow_pickle=False)
    summary["weights"] = os.path.relpath(args.out, os.path.dirname(HERE))
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
