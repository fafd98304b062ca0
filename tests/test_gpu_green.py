"""The Green-matrix route's device kernels and its reuse (Algorithm 2's preprocessing; G can
be stored and reused, section 3.2).

* The device LU with partial pivoting (blocked, 64-column panels) and its solves against
  numpy's dense solve, on matrices that span several panels and need row swaps; a zero
  matrix reports NM_ESINGULAR.
* A stored G passed back through options.green_in replaces the unit-force solves and gives
  the same trajectory bit for bit.
* Mixed precision on the Green route (unit-force solves and the two solves per step as FP64
  iterative refinement of FP32 PCG corrections) within 1e-5 of the FP64 oracle's Green
  route, and the two routes agree (the constrained solution is unique).
"""
import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

from gpu_common import rel_l2

pytestmark = pytest.mark.gpu


def _slab16():
    return W.make_polycrystal(n=16, n_grains=6, seed=7)  # x = 0 slab: 256 points, 768 dofs


@pytest.mark.parametrize("kind", ["random", "zero-diagonal"])
def test_device_lu_matches_numpy(kind):
    pb = _slab16()
    nd = 3 * pb.gamma_idx.size
    rng = np.random.default_rng(3)
    G = rng.standard_normal((nd, nd))
    if kind == "zero-diagonal":
        np.fill_diagonal(G, 0.0)  # every step needs a row swap
    else:
        G += 4 * np.sqrt(nd) * np.eye(nd)
    opts = nmb.Options(route=nmb.ROUTE_GREEN, tol=1e-10, green_in=G)
    with nmb.newmark_init_problem(pb, opts) as ctx:
        assert np.array_equal(nmb.green_matrix(ctx), G)
        for k in range(3):
            V = rng.standard_normal(nd)
            X = nmb.green_solve(ctx, V)
            want = np.linalg.solve(G, V)
            err = float(np.linalg.norm(X - want) / np.linalg.norm(want))
            print(f"device LU ({kind}, n = {nd}): rel err {err:.2e}, cond {np.linalg.cond(G):.1e}", flush=True)
            assert err <= 1e-10 * max(1.0, np.linalg.cond(G) / 1e3)


def test_singular_green_matrix_is_reported():
    pb = _slab16()
    nd = 3 * pb.gamma_idx.size
    with pytest.raises(nmb.NewmarkError) as e:
        nmb.newmark_init_problem(pb, nmb.Options(route=nmb.ROUTE_GREEN, green_in=np.zeros((nd, nd))))
    assert e.value.code == nmb.NM_ESINGULAR


def test_stored_green_matrix_gives_the_same_trajectory():
    pb = W.make_disc2d()
    steps = 12
    opts = nmb.Options(tol=1e-10, max_iter=500, route=nmb.ROUTE_GREEN, green_tol=1e-13)
    with nmb.newmark_init_problem(pb, opts) as ctx:
        G = nmb.green_matrix(ctx)
        for s in range(steps):
            nmb.newmark_step(ctx, pb.U(s + 1))
        a = nmb.get_state(ctx)
    opts.green_in = G
    with nmb.newmark_init_problem(pb, opts) as ctx:
        for s in range(steps):
            nmb.newmark_step(ctx, pb.U(s + 1))
        b = nmb.get_state(ctx)
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["F"], b["F"])


def test_mixed_precision_green_route():
    pb = W.make_polycrystal(n=16, n_grains=6, seed=7, gamma="sphere", sphere_radius=1.5)
    steps = 6
    U = np.stack([pb.U(s + 1) for s in range(steps)])
    res = {}
    for name, prec, route in (("green-mixed", nmb.PREC_MIXED, nmb.ROUTE_GREEN),
                              ("projected-fp64", nmb.PREC_FP64, nmb.ROUTE_PROJECTED)):
        opts = nmb.Options(tol=1e-10, max_iter=500, route=route, precision=prec, green_tol=1e-11, inner_tol=1e-5)
        us, st = [], []
        with nmb.newmark_init_problem(pb, opts) as ctx:
            for s in range(steps):
                st.append(nmb.newmark_step(ctx, pb.U(s + 1)))
                us.append(nmb.get_state(ctx)["u"].copy())
        res[name] = (us, st)
    ref = oracle.OracleProblem.from_problem(pb).newmark(pb.gamma_idx, U, steps, route=oracle.ROUTE_GREEN, tol=1e-13,
                                                        green_tol=1e-13)
    e_or = max(rel_l2(res["green-mixed"][0][s], ref["u"][s]) for s in range(steps) if np.abs(ref["u"][s]).max() > 0)
    e_rt = max(rel_l2(res["green-mixed"][0][s], res["projected-fp64"][0][s]) for s in range(steps)
               if np.abs(ref["u"][s]).max() > 0)
    st = res["green-mixed"][1]
    print(f"mixed Green route: vs FP64 oracle {e_or:.2e}, vs projected FP64 {e_rt:.2e}; sweeps "
          f"{[x['sweeps'] for x in st]}, FP32 iterations {[x['inner_iters'] for x in st]}", flush=True)
    assert e_or <= 1e-5
    assert e_rt <= 1e-5
    assert all(x["sweeps"] >= 2 for x in st)
    # the FP64 residual of the u_b solve (zero at the first step, whose right-hand side is zero)
    assert all(x["relres"] <= 1e-10 and x["relres0"] >= x["relres"] for x in st)
    assert all(x["relres"] > 0 for x in st[1:])


@pytest.mark.parametrize("case", ["polycrystal-16-sphere", "disc2d", "spheres-32-slab", "spheres-32-slab-mixed"])
def test_unit_force_solves_run_together(case):
    """Several unit-force solves through one chain of kernels (fields side by side, each loop
    with its own scalars, frozen once converged) give the Green matrix the one-at-a-time solves
    give: bit for bit in FP64; in mixed precision (FP64 refinement of FP32 corrections, fields
    whose FP64 residual has converged frozen in later corrections) to the unit-force tolerance."""
    import time
    if case == "disc2d":
        pb = W.make_disc2d()
    elif case.startswith("spheres-32-slab"):
        pb = W.make_spheres3d(n=32, seed=2)
    else:
        pb = W.make_polycrystal(n=16, n_grains=6, seed=7, gamma="sphere", sphere_radius=1.5)
    nd = pb.dim * pb.gamma_idx.size
    res = {}
    for batch in (1, 0, 5):
        prec = nmb.PREC_MIXED if case.endswith("mixed") else nmb.PREC_FP64
        opts = nmb.Options(tol=1e-10, max_iter=800, route=nmb.ROUTE_GREEN, green_tol=1e-12, green_batch=batch,
                           precision=prec)
        t0 = time.perf_counter()
        with nmb.newmark_init_problem(pb, opts) as ctx:
            t_init = time.perf_counter() - t0
            G = nmb.green_matrix(ctx)
            for s in range(4):
                nmb.newmark_step(ctx, pb.U(s + 1))
            u = nmb.get_state(ctx)["u"].copy()
        res[batch] = (G, u, t_init)
    G1, u1, t1 = res[1]
    for batch in (0, 5):
        G, u, t = res[batch]
        eg = float(np.abs(G - G1).max() / np.abs(G1).max())
        eu = float(np.abs(u - u1).max() / np.abs(u1).max())
        print(f"{case}: {nd} unit-force solves, one at a time {t1:.2f} s, batch {batch or 'auto'} {t:.2f} s; "
              f"G max rel diff {eg:.1e}, u {eu:.1e}", flush=True)
        if case.endswith("mixed"):
            assert eg <= 1e-10 and eu <= 1e-9
        else:
            assert eg <= 1e-13 and eu <= 1e-12
