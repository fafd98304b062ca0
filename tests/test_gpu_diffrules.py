"""GPU parity of the finite-difference differentiation rules (section 5 suggests discrete
difference rules against the noise of large contrast) against the FP64 oracle: the
second-order (CENTRED2, symbol i sin(xi h)/h) and fourth-order (CENTRED4) centred differences
in place of the spectral derivative.

* Operator and preconditioner, element by element (FP64 <= 1e-12, FP32 <= 1e-5 max relative),
  on grids with several tiles and on a padded 2^20-voxel grid with a 256-long axis.
* Implicit Newmark, projected route, FP64 with the oracle replaying the GPU's iteration counts
  (<= 1e-10), and mixed precision (<= 1e-5 of the FP64 oracle).
* The explicit central-difference scheme (<= 1e-10; no Krylov solve).
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

from gpu_common import dev, field3, random_problem, rel_l2, rel_max

pytestmark = pytest.mark.gpu

CASES = [(1, 3, (16, 8, 8)), (2, 3, (64, 32, 16)), (1, 2, (64, 64)), (2, 3, (128, 16, 64)), (1, 3, (256, 64, 64)),
         (2, 3, (64, 64, 256))]
IDS = [f"rule{r}-{d}d-" + "x".join(map(str, n)) for r, d, n in CASES]


@pytest.mark.parametrize("rule,dim,n", CASES, ids=IDS)
def test_operator_and_preconditioner_match_oracle(rule, dim, n):
    import torch
    pb = dataclasses.replace(random_problem(dim, n, seed=5 + sum(n)), diff_rule=rule)
    op = oracle.OracleProblem.from_problem(pb)
    u = W.random_field(op.field_shape, seed=7)
    want_a = field3(op.apply(u), dim)
    want_m = field3(op.precond(u), dim)
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10)) as ctx:
        for dtype, bar in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
            ud = dev(field3(u, dim), dtype)
            out = torch.empty_like(ud)
            nmb.apply_operator(ctx, ud, out)
            torch.cuda.synchronize()
            ea = rel_max(out.double().cpu().numpy(), want_a)
            nmb.precond_apply(ctx, ud, out)
            torch.cuda.synchronize()
            em = rel_max(out.double().cpu().numpy(), want_m)
            print(f"rule {rule} dim={dim} n={n} {dtype}: apply {ea:.2e} precond {em:.2e}", flush=True)
            assert ea <= bar and em <= bar


@pytest.mark.parametrize("rule", [1, 2])
def test_newmark_fp64_with_difference_rule_matches_oracle(rule):
    pb = dataclasses.replace(W.make_spheres3d(n=32, seed=2), diff_rule=rule)
    steps = 6
    us, its = [], []
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500, compute_reaction=1)) as ctx:
        for s in range(steps):
            st = nmb.newmark_step(ctx, pb.U(s + 1))
            its.append([st["iters"][0], -1])
            us.append(nmb.get_state(ctx)["u"].copy())
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    ref = oracle.OracleProblem.from_problem(pb).newmark(pb.gamma_idx, U, steps, replay=np.array(its))
    e = max(rel_l2(us[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0)
    spec = oracle.OracleProblem.from_problem(dataclasses.replace(pb, diff_rule=0)).newmark(pb.gamma_idx, U, steps,
                                                                                          tol=1e-12)
    d = rel_l2(spec["u"][-1], ref["u"][-1])
    print(f"rule {rule} Newmark FP64: iters {[i[0] for i in its]}, rel L2 {e:.2e}; vs spectral {d:.2e}", flush=True)
    assert e <= 1e-10
    assert d > 1e-3  # the rule is in effect


def test_mixed_precision_with_fourth_order_rule():
    pb = dataclasses.replace(W.make_polycrystal(n=32, n_grains=20, seed=3), diff_rule=2)
    steps = 6
    us = []
    opts = nmb.Options(tol=1e-8, max_iter=500, precision=nmb.PREC_MIXED, inner_tol=1e-4)
    with nmb.newmark_init_problem(pb, opts) as ctx:
        for s in range(steps):
            nmb.newmark_step(ctx, pb.U(s + 1))
            us.append(nmb.get_state(ctx)["u"].copy())
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    ref = oracle.OracleProblem.from_problem(pb).newmark(pb.gamma_idx, U, steps, tol=1e-12, max_iter=1000)
    e = max(rel_l2(us[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0)
    print(f"rule 2 mixed: rel L2 {e:.2e}", flush=True)
    assert e <= 1e-5


def test_explicit_with_centred_rule_matches_oracle():
    base = W.make_disc2d()
    # base.dt is CFL 2 on the fastest speed; a fifth of it is below the explicit bound of the
    # spectral and of the centred derivative (whose largest frequency is 1/h per axis)
    dt = 0.2 * base.dt
    pb = dataclasses.replace(base, dt=dt, beta=0.0, gamma_nm=0.5, diff_rule=1)
    steps = 120
    rows = np.stack([pb.Udot(s + 1) for s in range(steps)])
    with nmb.newmark_init_problem(pb, nmb.Options()) as ctx:
        nmb.explicit_step(ctx, rows[:20], n_steps=20)
        u20 = nmb.get_state(ctx)["u"].copy()
        nmb.explicit_step(ctx, rows[20:], n_steps=steps - 20)
        st = nmb.get_state(ctx)
    ref = oracle.OracleProblem.from_problem(pb).explicit(pb.gamma_idx, rows, steps, want_v=True)
    eu = max(rel_l2(u20, ref["u"][19]), rel_l2(st["u"], ref["u"][-1]))
    ev = rel_l2(st["v"], ref["v"][-1])
    print(f"rule 1 explicit: dt {dt:.4f}, rel L2 u {eu:.2e} v {ev:.2e}, |u| {np.abs(st['u']).max():.3e}", flush=True)
    assert eu <= 1e-10 and ev <= 1e-10
    assert np.abs(st["u"]).max() < 10.0
