"""The C ABI's error convention and state calls on the GPU.

* a step that fails (Krylov limit reached: NM_ENOTCONV; non-finite prescribed
  displacement: NM_ENAN) leaves the state (u, v, a, step count) as it was, bit for bit;
* nm_set_state followed by nm_get_state returns the same arrays, and a run resumed from a
  checkpoint continues bit for bit as the uninterrupted run (the reductions are
  deterministic: fixed shuffle trees and fixed-order second passes);
* two identical runs give identical results;
* a context created on a caller's non-default stream with a non-zero initial state holds
  that state (nm_newmark_init queues its zero fills on that stream before the copies);
* the reaction on Gamma (projected route with compute_reaction, and the Green route's
  G^-1 V / (beta dt^2)) and the Taylor initial iterate against the oracle;
* an empty Gamma (free vibration from a random initial state) against the oracle.
The error paths that fail before any device work are in test_abi.py (CPU).
"""
import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

from gpu_common import rel_l2

pytestmark = pytest.mark.gpu


def _state(ctx):
    st = nmb.get_state(ctx)
    return st["u"].copy(), st["v"].copy(), st["a"].copy(), st["step"]


def _same(s1, s2):
    return all(np.array_equal(a, b) for a, b in zip(s1[:3], s2[:3])) and s1[3] == s2[3]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_failed_step_leaves_the_state(precision):
    pb = W.make_spheres3d(n=16, seed=2)
    prec = nmb.PREC_MIXED if precision == "mixed" else nmb.PREC_FP64
    rng = np.random.default_rng(4)
    shp = (3,) + pb.phase_id.shape
    u, v, a = rng.standard_normal(shp), rng.standard_normal(shp), rng.standard_normal(shp)
    # two iterations (and, in mixed precision, one refinement sweep) cannot reach 1e-14
    opts = nmb.Options(tol=1e-14, max_iter=2, max_sweeps=1, precision=prec)
    with nmb.newmark_init_problem(pb, opts) as ctx:
        nmb.set_state(ctx, u, v, a, 7)
        before = _state(ctx)
        assert _same(before, (u, v, a, 7))
        with pytest.raises(nmb.NewmarkError) as e:
            nmb.newmark_step(ctx, pb.U(8))
        assert e.value.code == nmb.NM_ENOTCONV, e.value
        assert _same(_state(ctx), before)
        bad = pb.U(8).copy()
        bad[1] = np.nan
        with pytest.raises(nmb.NewmarkError) as e:
            nmb.newmark_step(ctx, bad)
        assert e.value.code == nmb.NM_ENAN, e.value
        assert _same(_state(ctx), before)


def _run(pb, opts, steps, start=0, state=None):
    with nmb.newmark_init_problem(pb, opts) as ctx:
        if state is not None:
            nmb.set_state(ctx, *state)
        for s in range(start, start + steps):
            nmb.newmark_step(ctx, pb.U(s + 1))
        return _state(ctx)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_resume_and_repeat_are_bitwise(precision):
    pb = W.make_polycrystal(n=32, n_grains=20, seed=3)
    prec = nmb.PREC_MIXED if precision == "mixed" else nmb.PREC_FP64
    opts = nmb.Options(tol=1e-8, max_iter=500, precision=prec)
    full = _run(pb, opts, 8)
    again = _run(pb, opts, 8)
    assert _same(full, again), "two identical runs differ"
    half = _run(pb, opts, 4)
    resumed = _run(pb, opts, 4, start=4, state=half)
    print(f"{precision}: resumed vs uninterrupted max |du| {np.abs(resumed[0] - full[0]).max():.3e}", flush=True)
    assert _same(resumed, full), "a resumed run differs from the uninterrupted one"


def test_initial_state_on_a_caller_stream():
    import torch
    pb = W.make_polycrystal(n=32, n_grains=20, seed=5)
    rng = np.random.default_rng(9)
    u0 = rng.standard_normal((3,) + pb.phase_id.shape)
    v0 = rng.standard_normal((3,) + pb.phase_id.shape)
    side = torch.cuda.Stream()
    with nmb.newmark_init_problem(pb, nmb.Options(), u0=u0, v0=v0, stream=side.cuda_stream) as ctx:
        assert nmb.get_stream(ctx) == side.cuda_stream
        st = nmb.get_state(ctx)
        assert np.array_equal(st["u"], u0) and np.array_equal(st["v"], v0)
    # the initial acceleration a0 = div(C : grad^s u0) / rho against the oracle
    op = oracle.OracleProblem.from_problem(pb)
    a0 = op.div_stress(u0) / pb.rho[pb.phase_id][None]
    assert rel_l2(st["a"], a0) <= 1e-11


def test_projected_reaction_matches_oracle():
    """F = (A u - b)|Gamma / (beta dt^2) of the projected route, over the first steps of the
    3D two-phase composite, with replayed iteration counts."""
    pb = W.make_spheres3d(n=32, seed=2)
    steps = 5
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    us, Fs, its = [], [], []
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500, compute_reaction=1)) as ctx:
        for s in range(steps):
            st = nmb.newmark_step(ctx, pb.U(s + 1))
            its.append([st["iters"][0], -1])
            g = nmb.get_state(ctx)
            us.append(g["u"].copy())
            Fs.append(g["F"].copy())
    ref = oracle.OracleProblem.from_problem(pb).newmark(pb.gamma_idx, U, steps, replay=np.array(its), want_F=True)
    eu = max(rel_l2(us[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0)
    eF = max(rel_l2(Fs[s], ref["F"][s]) for s in range(steps) if np.abs(ref["F"][s]).max() > 0)
    print(f"projected reaction: u rel L2 {eu:.2e}, F rel L2 {eF:.2e}", flush=True)
    assert eu <= 1e-10
    assert eF <= 1e-9


def test_green_route_3d_matches_oracle():
    """The paper's Green-matrix route in 3D: a 16^3 Cu polycrystal driven through the voxels
    of a small sphere (Gamma); G from the unit-force solves, its LU factors, two solves per
    step, and the Gamma force F = G^-1 V / (beta dt^2) (Algorithm 2), against the oracle's
    Green route with replayed iteration counts."""
    pb = W.make_polycrystal(n=16, n_grains=6, seed=7, gamma="sphere", sphere_radius=1.5)
    assert 4 <= pb.gamma_idx.size <= 40
    steps = 6
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    opts = nmb.Options(tol=1e-10, max_iter=500, route=nmb.ROUTE_GREEN, green_tol=1e-13)
    us, Fs, its = [], [], []
    with nmb.newmark_init_problem(pb, opts) as ctx:
        G = nmb.green_matrix(ctx)
        for s in range(steps):
            st = nmb.newmark_step(ctx, pb.U(s + 1))
            its.append(st["iters"])
            g = nmb.get_state(ctx)
            us.append(g["u"].copy())
            Fs.append(g["F"].copy())
    op = oracle.OracleProblem.from_problem(pb)
    Gref, _ = op.green_matrix(pb.gamma_idx, tol=1e-13)
    eG = float(np.abs(G - Gref).max() / np.abs(Gref).max())
    ref = op.newmark(pb.gamma_idx, U, steps, route=oracle.ROUTE_GREEN, replay=np.array(its), green_tol=1e-13,
                     want_F=True)
    eu = max(rel_l2(us[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0)
    eF = max(rel_l2(Fs[s], ref["F"][s]) for s in range(steps) if np.abs(ref["F"][s]).max() > 0)
    print(f"green 3d: |Gamma| {pb.gamma_idx.size}, G rel {eG:.2e}, u rel L2 {eu:.2e}, F rel L2 {eF:.2e}", flush=True)
    assert eG <= 1e-10
    assert eu <= 1e-10
    assert eF <= 1e-8
    # Gamma carries the prescribed displacement
    for s in range(steps):
        ug = us[s].reshape(3, -1)[:, pb.gamma_idx]
        np.testing.assert_allclose(ug, np.repeat(U[s][:, None], pb.gamma_idx.size, 1), atol=1e-9 * max(
            1.0, np.abs(U).max()))


def test_taylor_start_matches_oracle():
    """The second-order Taylor initial iterate changes only the iteration count: the solution
    matches the oracle run to a tighter tolerance."""
    pb = W.make_polycrystal(n=16, n_grains=6, seed=7)
    steps = 5
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    u_gpu, its = [], []
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-12, max_iter=800, warm_start=nmb.WS_TAYLOR)) as ctx:
        for s in range(steps):
            st = nmb.newmark_step(ctx, pb.U(s + 1))
            its.append(st["iters"][0])
            u_gpu.append(nmb.get_state(ctx)["u"].copy())
    ref = oracle.OracleProblem.from_problem(pb).newmark(pb.gamma_idx, U, steps, tol=1e-13, max_iter=2000)
    errs = [rel_l2(u_gpu[s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0]
    print(f"taylor start: iters {its}, max rel L2 {max(errs):.2e}", flush=True)
    assert max(errs) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_free_vibration_without_gamma_matches_oracle(precision):
    """Empty Gamma (n_gamma = 0): free vibration of a heterogeneous anisotropic medium from a
    random initial state (projected route with nothing to project; the reference residual is
    then ||b||) against the oracle, FP64 with the oracle replaying the GPU's iterations (1e-10)
    and mixed precision (1e-5 of the FP64 oracle)."""
    import dataclasses
    rng = np.random.default_rng(21)
    pb = dataclasses.replace(W.make_polycrystal(n=16, n_grains=6, seed=21), gamma_idx=np.zeros(0, np.int64))
    u0 = rng.standard_normal((3,) + pb.phase_id.shape)
    v0 = rng.standard_normal((3,) + pb.phase_id.shape)
    steps = 6
    prec = nmb.PREC_MIXED if precision == "mixed" else nmb.PREC_FP64
    us, its = [], []
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500, precision=prec), u0=u0, v0=v0) as ctx:
        for s in range(steps):
            st = nmb.newmark_step(ctx, np.zeros(3))
            its.append([st["iters"][0], -1])
            us.append(nmb.get_state(ctx)["u"].copy())
    op = oracle.OracleProblem.from_problem(pb)
    U = np.zeros((steps, 3))
    if precision == "fp64":
        ref = op.newmark(pb.gamma_idx, U, steps, replay=np.array(its), u0=u0, v0=v0)
        bar = 1e-10
    else:
        ref = op.newmark(pb.gamma_idx, U, steps, tol=1e-13, u0=u0, v0=v0)
        bar = 1e-5
    e = max(rel_l2(us[s], ref["u"][s]) for s in range(steps))
    print(f"no Gamma, {precision}: iterations {[i[0] for i in its]}, max rel L2 {e:.2e}", flush=True)
    assert e <= bar
