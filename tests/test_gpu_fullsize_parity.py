"""Element-wise oracle parity at the benchmark's full grid size (256^3), in the launch
configuration the benchmark times.

The oracle cannot apply the operator to a general 256^3 field in test time, but it can
when the microstructure and the field do not vary along one axis: then only the zero
frequency is present along that axis, every derivative along it vanishes, and the image
under the discretized operator (and under the preconditioner, whose reference medium is
the same volume average) does not vary along it either.  The 256^3 result therefore
equals the oracle's result on the grid with one voxel along that axis, at every voxel.
The grains are columns of a periodic 2D Voronoi tessellation (Cu, random orientations, so
the stiffness is fully anisotropic); the inputs are i.i.d. normal fields constant along
the column axis.

* operator and preconditioner, FP64 (max relative error <= 1e-12) and FP32 (<= 1e-5),
  columns along each of the three axes;
* Newmark steps of the projected route (x = 0 slab, Ricker pulse, CFL 2, tol 1e-8) on the
  column-along-z polycrystal: FP64 with the GPU's iteration counts replayed by the oracle
  (relative L2 <= 1e-10 per step, reaction on Gamma <= 1e-9), then mixed precision and mixed
  precision with the learned start against the same oracle trajectory (<= 1e-5).
"""
import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

from gpu_common import dev, rel_l2, rel_max

pytestmark = pytest.mark.gpu

N = 256


@pytest.fixture(scope="module", params=[2, 1, 0], ids=["z-columns", "y-columns", "x-columns"])
def columnar(request):
    axis = request.param
    full, red = W.make_columnar_polycrystal(n=N, n_grains=500, seed=3 + axis, axis=axis)
    return axis, full, red


def test_operator_and_preconditioner_at_256cube(columnar):
    import torch
    axis, full, red = columnar
    op = oracle.OracleProblem.from_problem(red)
    u = W.random_field(op.field_shape, seed=11 + axis)
    want_A = W.extrude_field(op.apply(u), N, axis).reshape(3, -1)
    want_M = W.extrude_field(op.precond(u), N, axis).reshape(3, -1)
    uf = W.extrude_field(u, N, axis).reshape(3, -1)
    with nmb.newmark_init_problem(full, nmb.Options(tol=1e-8)) as ctx:
        for dtype, bar in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
            print(f"256^3 columns along axis {axis}, {dtype}: operator and preconditioner", flush=True)
            ud = dev(uf, dtype)
            out = torch.empty_like(ud)
            nmb.apply_operator(ctx, ud, out)
            torch.cuda.synchronize()
            ea = rel_max(out.double().cpu().numpy(), want_A)
            nmb.precond_apply(ctx, ud, out)
            torch.cuda.synchronize()
            em = rel_max(out.double().cpu().numpy(), want_M)
            print(f"  apply rel err {ea:.3e}, precond rel err {em:.3e}", flush=True)
            assert ea <= bar, ea
            assert em <= bar, em


@pytest.fixture(scope="module")
def zcolumns():
    full, red = W.make_columnar_polycrystal(n=N, n_grains=500, seed=3, axis=2)
    return full, red


STEPS = 8


def _gpu_run(pb, opts, steps, net=None):
    us, Fs, stats = [], [], []
    with nmb.newmark_init_problem(pb, opts) as ctx:
        if net is not None:
            nmb.ws_attach(ctx, net)
        for s in range(steps):
            print(f"  GPU step {s + 1} of {pb.name}", flush=True)
            stats.append(nmb.newmark_step(ctx, pb.U(s + 1)))
            st = nmb.get_state(ctx)
            # the field is constant along z: keep one plane (and check that it is)
            u = st["u"]
            for k in (1, N // 2, N - 1):
                assert rel_max(u[:, k], u[:, 0]) <= 1e-12
            us.append(u[:, :1].copy())
            Fs.append(st["F"].copy())
    return us, Fs, stats


@pytest.fixture(scope="module")
def fp64_and_oracle(zcolumns):
    full, red = zcolumns
    print("FP64 Newmark steps at 256^3 (z columns)", flush=True)
    us, Fs, stats = _gpu_run(full, nmb.Options(tol=1e-8, max_iter=500, compute_reaction=1), STEPS)
    its = np.array([[s["iters"][0], -1] for s in stats])
    print(f"  GPU iterations {its[:, 0].tolist()}; oracle replay on {red.n}", flush=True)
    U = np.stack([red.U(s + 1) for s in range(STEPS)])
    ref = oracle.OracleProblem.from_problem(red).newmark(red.gamma_idx, U, STEPS, replay=its, want_F=True)
    return us, Fs, stats, ref


def test_fp64_newmark_prefix_at_256cube(fp64_and_oracle, zcolumns):
    full, red = zcolumns
    us, Fs, stats, ref = fp64_and_oracle
    errs = [rel_l2(us[s], ref["u"][s]) for s in range(STEPS)]
    # reaction on Gamma: the GPU lists the points of the full slab (x = 0, every y and z),
    # the oracle those of its single plane; on the column grid they repeat along z
    ng_red = red.gamma_idx.size
    Ferr = []
    for s in range(STEPS):
        Fg = Fs[s].reshape(-1, 3)  # point major, 3 components (full slab: n2 * n3 points, z slowest)
        Fr = ref["F"][s].reshape(-1, 3)
        Fg0 = Fg[:ng_red]  # the points with z index 0
        assert rel_max(Fg[(N - 1) * ng_red:N * ng_red], Fg0) <= 1e-12
        Ferr.append(rel_l2(Fg0, Fr))
    print(f"FP64 256^3: per-step rel L2 {['%.2e' % e for e in errs]}, reaction {['%.2e' % e for e in Ferr]}",
          flush=True)
    assert max(errs) <= 1e-10
    assert max(Ferr) <= 1e-9


def test_mixed_newmark_prefix_at_256cube(fp64_and_oracle, zcolumns):
    full, red = zcolumns
    ref = fp64_and_oracle[3]
    print("mixed-precision Newmark steps at 256^3 (z columns)", flush=True)
    us, _, stats = _gpu_run(full, nmb.Options(tol=1e-8, max_iter=500, precision=nmb.PREC_MIXED, true_residual=1),
                            STEPS)
    errs = [rel_l2(us[s], ref["u"][s]) for s in range(STEPS)]
    print(f"mixed 256^3: per-step rel L2 {['%.2e' % e for e in errs]}, true relres "
          f"{['%.1e' % s['relres'] for s in stats]}", flush=True)
    assert max(errs) <= 1e-5
    assert max(s["relres"] for s in stats) <= 1e-8


def test_mixed_learned_newmark_prefix_at_256cube(fp64_and_oracle, zcolumns):
    """The benchmark's headline configuration (mixed precision with the learned start) at
    its full size, against the FP64 oracle."""
    from paper_2211_08263_amd import warmstart
    full, red = zcolumns
    ref = fp64_and_oracle[3]
    net = nmb.Net()
    assert warmstart.load_weights(net)
    print("mixed precision + learned start at 256^3 (z columns)", flush=True)
    try:
        us, _, stats = _gpu_run(full, nmb.Options(tol=1e-8, max_iter=500, precision=nmb.PREC_MIXED,
                                                  warm_start=nmb.WS_LEARNED, true_residual=1), STEPS, net=net)
    finally:
        net.close()
    errs = [rel_l2(us[s], ref["u"][s]) for s in range(STEPS)]
    print(f"mixed+learned 256^3: per-step rel L2 {['%.2e' % e for e in errs]}, true relres "
          f"{['%.1e' % s['relres'] for s in stats]}", flush=True)
    assert max(errs) <= 1e-5
    assert max(s["relres"] for s in stats) <= 1e-8
