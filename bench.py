#!/usr/bin/env python3
"""Benchmark of the implicit FFT Newmark solver on one MI355X.

Workload: 256^3 Cu polycrystal (500 periodic Voronoi grains, random
orientations), plane longitudinal Ricker pulse prescribed on the x = 0 voxel
slab, Newmark beta = 1/4, gamma = 1/2, dt at CFL 2, PCG to a relative residual
of 1e-8 (projected Gamma route, previous-step initial guess).

A timed "step" is one full Newmark step: predictor and right-hand side,
the constrained Krylov solve (every PCG iteration: one operator apply and one
preconditioner apply), corrector.  Inputs are resident in HBM before timing.
After the timed steps every variant is run again, untimed, reporting the FP64
residual of each solution (true_residual), so that the mixed-precision
variants are checked at the same 1e-8 as the FP64 one.  The explicit
central-difference scheme (section 2.3) is timed on the same grid at its own
stable increment for the implicit-vs-explicit comparison.
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newmark steps/s & operator GVoxel/s at 256^3; learned+mixed vs plain FP64"
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic HBM bytes per voxel of each pass of one operator apply, in units of
# F = one real scalar field (8 B/voxel FP64, 4 B FP32; a half spectrum of one
# component is the same size), plus the 2-byte grain id where a pass reads it.
OPERATOR_PASS_FIELDS = {"x_fwd": 6, "y_deriv": 6, "z_strain": 12, "x_stress": 12, "y_div": 8, "z_div": 9,
                        "x_inv_inertia": 9}
OPERATOR_PASS_ID_BYTES = {"x_stress": 2, "x_inv_inertia": 2}


# HBM bytes per dispatch of the x_stress pass at 256^3 from two rocprofv3 counter runs
# (profiles/hbm_traffic_256cube.md): FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000, the factors a
# 512 MiB device copy reads for those counters.  Valid only for the kernel sources they were
# taken on (hash below); otherwise the traffic is reported as null.
PMC_TRAFFIC = {("x_stress", "fp64"): {"fetch_kib": 410158.5, "write_kib": 786436.8},
               ("x_stress", "fp32"): {"fetch_kib": 213319.0, "write_kib": 393216.5}}
PMC_N = 256
PMC_SCALE = {"fetch": 2.000, "write": 1.000}
PMC_SOURCES_SHA16 = "91438576f595bf0e"
PMC_SOURCES = ("nm_common.h", "nm_fft.h", "nm_passes.h", "nm_passes.hip")


def sources_sha16():
    import hashlib
    h = hashlib.sha256()
    for f in PMC_SOURCES:
        with open(os.path.join(ROOT, "paper_2211_08263_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel, label, n):
    t = PMC_TRAFFIC.get((kernel, label))
    if t is None or n != PMC_N or sources_sha16() != PMC_SOURCES_SHA16:
        return None
    return round(1024 * (t["fetch_kib"] * PMC_SCALE["fetch"] + t["write_kib"] * PMC_SCALE["write"]))


def pass_bytes_per_voxel(name, real_bytes):
    return OPERATOR_PASS_FIELDS[name] * real_bytes + OPERATOR_PASS_ID_BYTES.get(name, 0)


def operator_bytes_per_voxel(real_bytes):
    return sum(pass_bytes_per_voxel(k, real_bytes) for k in OPERATOR_PASS_FIELDS)


def run_variant(pb, opts, steps, warmup, label, net=None):
    import torch
    from paper_2211_08263_amd import newmark as nmb
    t0 = time.time()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = nmb.newmark_init_problem(pb, opts)
    log(f"[{label}] init {time.time() - t0:.1f}s")
    stats = []
    try:
        if net is not None:
            nmb.ws_attach(ctx, net)
        for s in range(warmup):
            nmb.newmark_step(ctx, pb.U(s + 1))
        torch.cuda.synchronize()
        held = (free0 - torch.cuda.mem_get_info()[0]) / 2 ** 30
        t0 = time.perf_counter()
        for s in range(warmup, warmup + steps):
            stats.append(nmb.newmark_step(ctx, pb.U(s + 1)))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        ctx.close()
    its = [st["iters"][0] for st in stats]
    inner = [st["inner_iters"] for st in stats]
    sweeps = [st["sweeps"] for st in stats]
    r0 = [round(st["relres0"], 4) for st in stats]
    log(f"[{label}] {steps} steps in {dt:.3f}s -> {steps / dt:.3f} steps/s; iters {its} inner {inner} "
        f"initial relres {r0}")
    # untimed repeat with the FP64 residual of every solution reported
    opts_true = dataclasses.replace(opts, true_residual=1)
    ctx = nmb.newmark_init_problem(pb, opts_true)
    true_rr = []
    try:
        if net is not None:
            nmb.ws_attach(ctx, net)
        for s in range(warmup + steps):
            st = nmb.newmark_step(ctx, pb.U(s + 1))
            if s >= warmup:
                true_rr.append(st["relres"])
    finally:
        ctx.close()
    log(f"[{label}] FP64 residual of the solutions: max {max(true_rr):.3e}")
    return {"steps_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps, "iters_per_step": its,
            "inner_iters_per_step": inner, "sweeps_per_step": sweeps, "initial_relres_per_step": r0,
            "warm_start_ms_mean": sum(st["t_warm_ms"] for st in stats) / len(stats),
            "relres_max_stopping_test": max(st["relres"] for st in stats),
            "relres_max_fp64_true": max(true_rr), "device_memory_held_GiB": round(held, 2)}


def operator_rates(pb):
    """Operator GVoxel/s (FP64 and FP32) and per-pass times, from HIP events that the
    library records between the passes on its own stream (nm_profile_passes)."""
    import torch
    from paper_2211_08263_amd import newmark as nmb
    N = pb.n_vox
    out = {}
    ctx = nmb.newmark_init_problem(pb, nmb.Options())
    try:
        g = torch.Generator(device="cuda").manual_seed(7)
        for dt, label, rb in ((torch.float64, "fp64", 8), (torch.float32, "fp32", 4)):
            u = torch.randn(3 * N, device="cuda", dtype=torch.float64, generator=g).to(dt)
            Au = torch.empty_like(u)
            torch.cuda.synchronize()
            for _ in range(3):
                nmb.apply_operator(ctx, u, Au)
            runs = [nmb.profile_passes(ctx, 0, u, Au, reps=10) for _ in range(5)]
            totals = sorted(sum(r.values()) for r in runs)
            med = totals[len(totals) // 2]
            passes = {k: sorted(r[k] for r in runs)[len(runs) // 2] for k in runs[0]}
            pre = nmb.profile_passes(ctx, 1, u, Au, reps=10)
            bpv = operator_bytes_per_voxel(rb)
            out[label] = {"apply_ms_median": med, "gvoxel_per_s": N / (med * 1e-3) / 1e9,
                          "model_bytes_per_voxel": bpv, "model_GBps": bpv * N / (med * 1e-3) / 1e9,
                          "passes_ms": passes, "precond_passes_ms": pre}
            log(f"[operator {label}] median {med:.3f} ms -> {N / med / 1e6:.2f} GVoxel/s, "
                f"{bpv * N / med / 1e6:.0f} GB/s model; passes {passes}")
    finally:
        ctx.close()
    return out


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(n_full, grains_full, seed, iters_per_step, n_sample=128):
    """The FP64 oracle (single thread, pinned to one host core) timed on one operator apply
    and one preconditioner apply of a smaller polycrystal with the same grain density; the
    full-grid step time is EXTRAPOLATED from them (N log N scaling, the step's count of
    applies), not measured."""
    import oracle
    from paper_2211_08263_amd import workloads as W
    g = max(1, round(grains_full * (n_sample / n_full) ** 3))
    pb = W.make_polycrystal(n=n_sample, n_grains=g, seed=seed)
    op = oracle.OracleProblem.from_problem(pb)
    u = W.random_field(op.field_shape, seed=7)
    model, ncpu = host_cpu()
    old_aff = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    core = min(old_aff) if old_aff else None
    if core is not None:
        os.sched_setaffinity(0, {core})
    log(f"[cpu] oracle operator and preconditioner apply on {n_sample}^3 (pinned to core {core}) ...")
    try:
        t0 = time.perf_counter()
        op.apply(u)
        t_apply = time.perf_counter() - t0
        t0 = time.perf_counter()
        op.precond(u)
        t_prec = time.perf_counter() - t0
    finally:
        if old_aff:
            os.sched_setaffinity(0, old_aff)
    N_s, N_f = n_sample ** 3, n_full ** 3
    scale = (N_f * math.log2(N_f)) / (N_s * math.log2(N_s))
    applies, precs = iters_per_step + 2, iters_per_step + 1
    step_s = scale * (applies * t_apply + precs * t_prec)
    log(f"[cpu] apply {t_apply:.2f}s precond {t_prec:.2f}s at {n_sample}^3 -> {step_s:.0f}s per {n_full}^3 step")
    return {"value": 1.0 / step_s, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "extrapolated": True,
            "sample": (f"EXTRAPOLATED: one FP64 oracle operator apply ({t_apply:.2f} s) and one preconditioner "
                       f"apply ({t_prec:.2f} s) timed on a {n_sample}^3 polycrystal with {g} grains (same grain "
                       f"density), 1 thread pinned to host core {core}, scaled by N log N (x{scale:.2f}) to "
                       f"{n_full}^3; per step {applies} applies + {precs} preconditioner applies (mean FP64 PCG "
                       f"iterations {iters_per_step}); vector updates excluded"),
            "host_cpu": model, "host_cpus_visible": ncpu, "pinned_core": core,
            "apply_s_sample": t_apply, "precond_s_sample": t_prec,
            "gvoxel_per_s_apply": N_s / t_apply / 1e9}


def network_rates(pb, net, reps=5):
    """The warm-start network (4 layers of 3^3 BF16 convolutions, 31->16->16->16->3) applied
    to 32-channel BF16 features of the full grid, timed with torch events on the stream it
    runs on.  Algorithmic work per voxel: 2 * 27 * (31*16 + 16*16 + 16*16 + 16*3) = 57,024
    FLOP; HBM bytes per voxel: features 64 in, three 16-channel BF16 activations written and
    read (3 * 64), FP32 prediction 16 out and 32 for its copy into the caller's buffer = 304."""
    import torch
    N = pb.n_vox
    feat = torch.randn(N * 32, device="cuda", dtype=torch.float32).to(torch.bfloat16).view(torch.int16)
    pred = torch.empty(N * 4, device="cuda", dtype=torch.float32)
    stream = torch.cuda.current_stream()
    net.forward(pb.n, feat, pred, stream=stream.cuda_stream)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        net.forward(pb.n, feat, pred, stream=stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = sorted(times)[len(times) // 2]
    flop, byts = 57024.0 * N, 304.0 * N
    tf = flop / (ms * 1e-3) / 1e12
    gbs = byts / (ms * 1e-3) / 1e9
    log(f"[network] forward {ms:.3f} ms: {tf:.1f} TFLOP/s ({tf / BF16_MFMA_PEAK_TFLOPS:.3f} of BF16 MFMA), "
        f"{gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.3f} of HBM)")
    return {"forward_ms_median": ms, "flop_per_voxel": 57024, "bytes_per_voxel": 304,
            "achieved_tflops": round(tf, 1), "mfma_peak_tflops": BF16_MFMA_PEAK_TFLOPS,
            "frac_mfma": round(tf / BF16_MFMA_PEAK_TFLOPS, 4), "achieved_GBps": round(gbs, 1),
            "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}


def explicit_rates(pb, steps, warmup):
    """The explicit central-difference scheme (section 2.3) on the same grid and source, at
    0.9 of its stable increment 2 / omega_max (eq. Courant_stable).  omega_max^2 is the larger
    of a power-iteration estimate on the heterogeneous grid and the largest corner-frequency
    eigenvalue of the grains' acoustic tensors over the smallest density."""
    import numpy as np
    import torch
    from paper_2211_08263_amd import newmark as nmb
    from paper_2211_08263_amd import workloads as W
    N = pb.n_vox
    xi = [math.pi * (pb.n[i] - 2) / pb.L[i] for i in range(3)]
    w2_bound = 0.0
    for c21 in pb.C21:
        T = W._voigt66_to_tensor(W.voigt_from21(c21))
        for s1 in (1, -1):
            for s2 in (1, -1):
                v = np.array([xi[0], s1 * xi[1], s2 * xi[2]])
                w2_bound = max(w2_bound, float(np.linalg.eigvalsh(np.einsum("ijkl,j,l->ik", T, v, v)).max()))
    w2_bound /= float(np.min(pb.rho))
    ctx = nmb.newmark_init_problem(pb, nmb.Options())
    try:
        x = torch.randn(3 * N, device="cuda", dtype=torch.float64)
        w2_est = nmb.omega2_max(ctx, x, 100)
    finally:
        ctx.close()
    w2 = max(w2_est, w2_bound)
    dt = 0.9 * 2.0 / math.sqrt(w2)
    pe = dataclasses.replace(pb, dt=dt, beta=0.0, gamma_nm=0.5)
    rows = np.stack([pe.Udot(s + 1) for s in range(warmup + steps)])
    ctx = nmb.newmark_init_problem(pe, nmb.Options())
    try:
        nmb.explicit_step(ctx, rows[:warmup], n_steps=warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nmb.explicit_step(ctx, rows[warmup:], n_steps=steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        u = nmb.get_state(ctx)["u"]
    finally:
        ctx.close()
    assert np.isfinite(u).all()
    bpv = 77 * 8 + 4  # x-forward with the displacement update 15F, operator passes 47F + 2 B, last pass 15F + 2 B
    log(f"[explicit] omega_max^2 {w2:.4f} (power iteration {w2_est:.4f}, grain bound {w2_bound:.4f}); "
        f"dt {dt:.4f} vs implicit {pb.dt:.4f}; {steps} steps in {el:.3f}s -> {steps / el:.1f} steps/s")
    return {"steps_per_s": steps / el, "ms_per_step": 1e3 * el / steps, "dt": dt, "omega2_max_power_iter": w2_est,
            "omega2_max_grain_bound": w2_bound, "simulated_time_per_s": dt * steps / el,
            "model_bytes_per_voxel": bpv, "model_GBps": bpv * N * steps / el / 1e9}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--grains", type=int, default=500)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--variants", default="fp64,fp64_cold,mixed,mixed_cold,mixed_learned",
                    help="precision (fp64|mixed) _ initial iterate (prev|cold|taylor|learned; default prev)")
    ap.add_argument("--inner-tol", type=float, default=1e-5, help="floor of the FP32 inner-solve tolerance")
    ap.add_argument("--cpu-sample", choices=["apply", "none"], default="apply")
    ap.add_argument("--skip-operator", action="store_true")
    ap.add_argument("--skip-network", action="store_true")
    ap.add_argument("--skip-explicit", action="store_true")
    ap.add_argument("--explicit-steps", type=int, default=50)
    ap.add_argument("--gamma", choices=["slab", "sphere"], default="slab",
                    help="prescribed-displacement set: x = 0 slab, or the centred sphere of radius 6")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no multi-GPU "
              "path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2211_08263_amd import newmark as nmb
    from paper_2211_08263_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        x = torch.empty(args.copy_probe_mib * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    t0 = time.time()
    pb = W.make_polycrystal(n=args.n, n_grains=args.grains, seed=args.seed, gamma=args.gamma, sphere_radius=6.0)
    log(f"[setup] polycrystal {args.n}^3 with {args.grains} grains in {time.time() - t0:.1f}s; "
        f"dt {pb.dt:.4f}, fc {pb.pulse_fc:.4f}, |Gamma| {pb.gamma_idx.size}")

    variants = {}
    starts = {"prev": nmb.WS_PREV, "cold": nmb.WS_COLD, "taylor": nmb.WS_TAYLOR, "learned": nmb.WS_LEARNED}
    names = args.variants.split(",")
    for v in names:
        prec, _, start = v.partition("_")
        if prec not in ("fp64", "mixed") or (start and start not in starts):
            raise SystemExit(f"unknown variant {v}")
    net = None
    if any(v.endswith("_learned") for v in names):
        from paper_2211_08263_amd import warmstart
        net = nmb.Net()
        if not warmstart.load_weights(net):
            raise SystemExit(f"no trained warm-start weights at {warmstart.DEFAULT_WEIGHTS}")
    for v in names:
        prec, _, start = v.partition("_")
        o = nmb.Options(tol=1e-8, max_iter=500, warm_start=starts[start or "prev"],
                        precision=nmb.PREC_MIXED if prec == "mixed" else nmb.PREC_FP64, inner_tol=args.inner_tol)
        variants[v] = run_variant(pb, o, args.steps, args.warmup, v, net if start == "learned" else None)

    op = {} if args.skip_operator else operator_rates(pb)
    head = next((h for h in ("mixed_learned", "mixed") if h in variants), names[0])
    hv = variants[head]
    roof = None
    if op:
        # dominant kernel of the headline (mixed-precision) path: the slowest FP32 operator pass;
        # the FP64 one of the baseline path beside it
        rl = {}
        for label, rb in (("fp32", 4), ("fp64", 8)):
            passes = op[label]["passes_ms"]
            dom = max(passes, key=passes.get)
            bpv = pass_bytes_per_voxel(dom, rb)
            achieved = bpv * pb.n_vox / (passes[dom] * 1e-3) / 1e9
            rl[label] = {"bound": "hbm", "kernel": f"{dom} ({label} operator pass)", "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": pmc_traffic(dom, label, args.n), "traffic_unit": "bytes per launch",
                         "algorithmic_bytes": bpv * pb.n_vox, "bytes_per_voxel": bpv, "avg_ms": passes[dom],
                         "operator_chain_GBps": round(op[label]["model_GBps"], 1),
                         "operator_chain_frac": round(op[label]["model_GBps"] / HBM_PEAK_GBS, 4)}
        roof = dict(rl["fp32" if head.startswith("mixed") else "fp64"])
        roof["other_precision"] = rl["fp64" if head.startswith("mixed") else "fp32"]
    netr = network_rates(pb, net) if (net is not None and not args.skip_network) else None
    expl = None if args.skip_explicit else explicit_rates(pb, args.explicit_steps, 5)
    if net is not None:
        net.close()
    cpu = None
    if args.cpu_sample == "apply":
        fp = variants.get("fp64", hv)
        cpu = cpu_baseline(args.n, args.grains, args.seed, int(round(float(np.mean(fp["iters_per_step"])))))

    def ratio(a, b):
        return round(variants[a]["steps_per_s"] / variants[b]["steps_per_s"], 3) if a in variants and b in variants \
            else None

    impl_sim = {k: v["steps_per_s"] * pb.dt for k, v in variants.items()}
    line = {
        "metric": METRIC, "value": round(hv["steps_per_s"], 4), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(hv["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("bf16+f32+f64" if head.endswith("learned") else "f32+f64") if head.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.n}^3 Cu polycrystal, {args.grains} Voronoi grains (seed {args.seed}), "
                               f"{'x=0 slab' if args.gamma == 'slab' else 'centred sphere r=6'} Ricker, tol 1e-8, "
                               "projected Gamma route",
                   "baseline_variant": "fp64 (FP64 PCG, previous-step initial iterate)",
                   "headline_variant": head,
                   "speedup_vs_fp64": ratio(head, "fp64"),
                   "speedup_vs_fp64_cold": ratio(head, "fp64_cold"),
                   "learned_vs_mixed_cold": ratio("mixed_learned", "mixed_cold"),
                   "mixed_cold_vs_fp64": ratio("mixed_cold", "fp64"),
                   "grid": [args.n] * 3, "dt": pb.dt, "tol": 1e-8,
                   "inner_tol_floor": args.inner_tol,
                   "variants": variants,
                   "operator": op,
                   "network": netr,
                   "explicit": expl,
                   "simulated_time_per_s": {**{k: round(v, 4) for k, v in impl_sim.items()},
                                            **({"explicit": round(expl["simulated_time_per_s"], 4)} if expl else {})}},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
