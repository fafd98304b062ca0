"""GPU parity of the Krylov solve and the Newmark loop against the FP64 oracle.

FP64 runs are compared with the oracle replaying the GPU's iteration counts
(both stop on a tolerance otherwise, and two correct solvers may differ by
about kappa * tol); bar 1e-10 relative L2 per step.  Mixed precision is
compared with the FP64 oracle run to tolerance; bar 1e-5."""
import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

from gpu_common import dev, field3, random_problem, rel_l2

pytestmark = pytest.mark.gpu


def test_pcg_solve_matches_oracle_replay():
    import torch
    pb = random_problem(3, (32, 16, 16), seed=5, dt=1.2)
    op = oracle.OracleProblem.from_problem(pb)
    b = W.random_field(op.field_shape, seed=1)
    with nmb.newmark_init_problem(pb) as ctx:
        bd = dev(b.reshape(3, -1))
        x = torch.zeros_like(bd)
        it, rel = nmb.pcg_solve(ctx, bd, x, tol=1e-10)
        got = x.cpu().numpy()
    print("pcg iterations", it, "rel", rel, flush=True)
    assert 1 < it < 200
    want, it2, _ = op.pcg(b, fixed_iters=it)
    err = rel_l2(got, want.reshape(3, -1))
    assert err <= 1e-10, err


def _run_gpu(pb, steps, opts, per_step=None):
    u_hist, stats = [], []
    with nmb.newmark_init_problem(pb, opts) as ctx:
        for s in range(steps):
            st = nmb.newmark_step(ctx, pb.U(s + 1))
            stats.append(st)
            u_hist.append(nmb.get_state(ctx)["u"].copy())
    return np.stack(u_hist), stats


def test_disc2d_projected_full_run_matches_oracle():
    """2D plane strain 64x64 disc (inclusion E=10, rho=3), Ricker on the left 2-voxel strip,
    100 steps at CFL 2, tol 1e-10, projected route."""
    pb = W.make_disc2d()
    steps = pb.n_steps
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    u_gpu, stats = _run_gpu(pb, steps, nmb.Options(tol=pb.tol, max_iter=500))
    its = np.array([[s["iters"][0], -1] for s in stats])
    op = oracle.OracleProblem.from_problem(pb)
    ref = op.newmark(pb.gamma_idx, U, steps, route=oracle.ROUTE_PROJECTED, replay=its)
    errs = [rel_l2(u_gpu[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0]
    print("disc2d projected: iters", its[:, 0].min(), its[:, 0].max(), "max rel L2", max(errs), flush=True)
    assert max(errs) <= 1e-10


def test_disc2d_green_route_matches_oracle():
    """The paper's route: Green matrix of the 128 Gamma voxels (256 x 256), LU, two solves per step."""
    pb = W.make_disc2d()
    steps = 30
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    opts = nmb.Options(tol=1e-10, max_iter=500, route=nmb.ROUTE_GREEN, green_tol=1e-13)
    u_gpu, stats = _run_gpu(pb, steps, opts)
    its = np.array([s["iters"] for s in stats])
    op = oracle.OracleProblem.from_problem(pb)
    ref = op.newmark(pb.gamma_idx, U, steps, route=oracle.ROUTE_GREEN, replay=its, green_tol=1e-13)
    errs = [rel_l2(u_gpu[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0]
    print("disc2d green: max rel L2", max(errs), flush=True)
    assert max(errs) <= 1e-10
    # Gamma holds the prescribed displacement
    ug = u_gpu.reshape(steps, 2, -1)[:, 0, pb.gamma_idx]
    np.testing.assert_allclose(ug, U[:, :1].repeat(pb.gamma_idx.size, 1), atol=1e-9)


def test_spheres3d_projected_prefix_matches_oracle():
    """3D two-phase composite (RSA spheres, contrast 10x/3x) on a 32^3 grid, first 6 steps."""
    pb = W.make_spheres3d(n=32, seed=2)
    steps = 6
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    u_gpu, stats = _run_gpu(pb, steps, nmb.Options(tol=1e-8, max_iter=500))
    its = np.array([[s["iters"][0], -1] for s in stats])
    ref = oracle.OracleProblem.from_problem(pb).newmark(pb.gamma_idx, U, steps, replay=its)
    errs = [rel_l2(u_gpu[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0]
    print("spheres3d: iters", its[:, 0], "max rel L2", max(errs), flush=True)
    assert max(errs) <= 1e-10


def test_polycrystal_mixed_precision_within_1e5_of_fp64_oracle():
    pb = W.make_polycrystal(n=32, n_grains=20, seed=3)
    steps = 6
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    opts = nmb.Options(tol=1e-8, max_iter=500, precision=nmb.PREC_MIXED, inner_tol=1e-4)
    u_gpu, stats = _run_gpu(pb, steps, opts)
    ref = oracle.OracleProblem.from_problem(pb).newmark(pb.gamma_idx, U, steps, tol=1e-12, max_iter=1000)
    errs = [rel_l2(u_gpu[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0]
    print("mixed: sweeps", [s["sweeps"] for s in stats], "inner", [s["inner_iters"] for s in stats],
          "max rel L2", max(errs), flush=True)
    assert max(errs) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_start_with_lifting_responses_matches_oracle(precision):
    """Projected route, zero initial iterate: the reference residual comes from the
    precomputed responses A e_c of the Gamma lifting and doubles as the initial residual
    (no operator apply).  Compared with the oracle run to a tighter tolerance."""
    pb = W.make_polycrystal(n=16, n_grains=6, seed=7)
    steps = 5
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    prec = nmb.PREC_MIXED if precision == "mixed" else nmb.PREC_FP64
    u_gpu, stats = _run_gpu(pb, steps, nmb.Options(tol=1e-12 if precision == "fp64" else 1e-10, max_iter=800,
                                                   precision=prec, warm_start=nmb.WS_COLD, inner_tol=1e-5))
    ref = oracle.OracleProblem.from_problem(pb).newmark(pb.gamma_idx, U, steps, tol=1e-13, max_iter=2000)
    errs = [rel_l2(u_gpu[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0]
    print(precision, "zero start: iters", [s["iters"][0] for s in stats], "inner", [s["inner_iters"] for s in stats],
          "initial relres", [round(s["relres0"], 6) for s in stats], "max rel L2", max(errs), flush=True)
    assert all(abs(s["relres0"] - 1.0) < 1e-12 for s in stats if s["relres0"] > 0)
    assert max(errs) <= (1e-10 if precision == "fp64" else 1e-8)
