"""GPU parity of the explicit central-difference scheme (section 2.3) and of the power
iteration for omega_max (section 2.3.3) against the FP64 oracle.

There is no Krylov solve, so both sides compute the same sequence of operations up to
rounding: bar 1e-10 relative L2 per compared step (displacement, velocity and the Gamma
force).  Time increments: a fraction of 2 / omega_max with omega_max^2 bounded by the stiffest
phase over the lightest density at the corner frequencies of the grid (eq. Courant_stable)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

from gpu_common import dev, rel_l2

pytestmark = pytest.mark.gpu


def _omega2_bound(pb):
    """max over phases of lambda_max(C_ijkl xi_j xi_l) / min rho over the corner frequencies."""
    n = pb.n
    xs = [np.pi * (n[i] - 2) / pb.L[i] if n[i] > 1 else 0.0 for i in range(3)]
    corners = [np.array([s0 * xs[0], s1 * xs[1], s2 * xs[2]]) for s0 in (1, -1) for s1 in (1, -1) for s2 in (1, -1)]
    best = 0.0
    for c21 in pb.C21:
        T = W._voigt66_to_tensor(W.voigt_from21(c21))
        for xi in corners:
            Q = np.einsum("ijkl,j,l->ik", T, xi, xi)
            best = max(best, float(np.linalg.eigvalsh(Q).max()))
    return best / float(np.min(pb.rho))


def _explicit_problem(pb, factor=0.8):
    dt = factor * 2.0 / np.sqrt(_omega2_bound(pb))
    return dataclasses.replace(pb, dt=dt, beta=0.0, gamma_nm=0.5)


def _udot_rows(pb, steps, amp=1.0):
    return np.stack([pb.Udot(s + 1) for s in range(steps)]) * amp


def _run_gpu(pb, rows, batches, per_point=False):
    """Run the explicit scheme in the given batch sizes; state and Gamma force after each."""
    out = []
    with nmb.newmark_init_problem(pb, nmb.Options()) as ctx:
        k = 0
        for nb in batches:
            nmb.explicit_step(ctx, rows[k:k + nb], per_point=per_point, n_steps=nb)
            k += nb
            st = nmb.get_state(ctx)
            out.append((k, st["u"].copy(), st["v"].copy(), st["F"].copy()))
    return out


def _compare(pb, rows, batches, per_point=False, bar=1e-10):
    steps = sum(batches)
    got = _run_gpu(pb, rows, batches, per_point)
    ref = oracle.OracleProblem.from_problem(pb).explicit(pb.gamma_idx, rows, steps, per_point=per_point,
                                                         want_v=True, want_F=True)
    eu = ev = eF = 0.0
    for k, u, v, F in got:
        eu = max(eu, rel_l2(u, ref["u"][k - 1]))
        ev = max(ev, rel_l2(v, ref["v"][k - 1]))
        if pb.gamma_idx.size and np.abs(ref["F"][k - 1]).max() > 0:
            eF = max(eF, rel_l2(F, ref["F"][k - 1]))
    print(f"{pb.name}: dt {pb.dt:.4f}, {steps} explicit steps, rel L2 u {eu:.2e} v {ev:.2e} F {eF:.2e}", flush=True)
    assert eu <= bar and ev <= bar and eF <= bar
    return got, ref


def test_disc2d_explicit_matches_oracle():
    pb = _explicit_problem(W.make_disc2d())
    steps = 240
    _compare(pb, _udot_rows(pb, steps), [1, 7, 32, 200])


def test_spheres3d_explicit_matches_oracle():
    pb = _explicit_problem(W.make_spheres3d(n=32, seed=2))
    steps = 120
    _compare(pb, _udot_rows(pb, steps), [10, 50, 60])


def test_sphere_source_per_point_velocities_match_oracle():
    """A spherical source in a polycrystal with a different velocity history at every Gamma
    point (per-point rows)."""
    base = W.make_polycrystal(n=32, n_grains=12, seed=8, gamma="sphere", sphere_radius=3.0)
    pb = _explicit_problem(base)
    steps = 60
    ng = pb.gamma_idx.size
    w = 1.0 + 0.5 * np.sin(np.arange(ng))  # per-point amplitude
    rows = np.stack([(pb.Udot(s + 1)[None, :] * w[:, None]).reshape(-1) for s in range(steps)])
    _compare(pb, rows, [20, 40], per_point=True)


def test_explicit_at_256cube_matches_oracle():
    """Full size, in the benchmark's launch configuration: 256^3 polycrystal with grains as z
    columns (see test_gpu_fullsize_parity.py) against the oracle on one z plane."""
    full, red = W.make_columnar_polycrystal(n=256, n_grains=500, seed=3, axis=2)
    full = _explicit_problem(full)
    red = dataclasses.replace(red, dt=full.dt, beta=0.0)
    steps = 40
    rows = _udot_rows(full, steps)
    got = []
    with nmb.newmark_init_problem(full, nmb.Options()) as ctx:
        for k in (10, 30):
            print(f"  256^3 explicit batch of {k} steps", flush=True)
            nmb.explicit_step(ctx, rows[sum(g[0] for g in got):sum(g[0] for g in got) + k], n_steps=k)
            u = nmb.get_state(ctx)["u"]
            got.append((k, u[:, :1].copy(), float(np.abs(u[:, -1] - u[:, 0]).max())))
    ref = oracle.OracleProblem.from_problem(red).explicit(red.gamma_idx, rows, steps)
    kk = 0
    for k, u, zdev in got:
        kk += k
        e = rel_l2(u, ref["u"][kk - 1])
        print(f"256^3 explicit after {kk} steps: rel L2 {e:.2e}, z variation {zdev:.1e}", flush=True)
        assert e <= 1e-10
        assert zdev <= 1e-12 * np.abs(u).max()


def test_omega2_max_matches_oracle_and_closed_form():
    import torch
    # heterogeneous: same start vector and iteration count as the oracle
    pb = W.make_spheres3d(n=16, seed=2)
    x0 = W.random_field((3, 16, 16, 16), seed=4)
    with nmb.newmark_init_problem(pb, nmb.Options()) as ctx:
        xd = dev(x0.reshape(3, -1))
        lam = nmb.omega2_max(ctx, xd, 60)
        xg = xd.cpu().numpy()
    lam_o, xo = oracle.OracleProblem.from_problem(pb).omega2_max(x0, 60)
    print(f"omega2_max: GPU {lam:.12e} oracle {lam_o:.12e}", flush=True)
    assert abs(lam - lam_o) <= 1e-10 * lam_o
    assert rel_l2(xg, xo.reshape(3, -1)) <= 1e-8
    # homogeneous anisotropic medium: the closed form of eq. Eigenvalues_1D_homogeneo
    n = 32
    C21 = W.voigt_to21(W.rotate_voigt66(W.copper_scaled66(), W.random_rotations(np.random.default_rng(3), 1)[0]))
    hom = W.Problem("hom", 3, (n, n, n), (float(n),) * 3, np.zeros((n, n, n), np.uint16), C21[None], np.array([1.0]),
                    np.zeros(0, np.int64), 0.1)
    w2 = _omega2_bound(hom)
    with nmb.newmark_init_problem(hom, nmb.Options()) as ctx:
        x = torch.randn(3 * n ** 3, dtype=torch.float64, device="cuda")
        lam = nmb.omega2_max(ctx, x, 300)
    print(f"homogeneous: power iteration {lam:.6f} vs closed form {w2:.6f}", flush=True)
    assert lam <= w2 * (1 + 1e-10)
    assert lam >= 0.97 * w2


def test_explicit_context_errors():
    pb = _explicit_problem(W.make_spheres3d(n=16, seed=2))
    rows = _udot_rows(pb, 3)
    with nmb.newmark_init_problem(pb, nmb.Options()) as ctx:
        nmb.explicit_step(ctx, rows[:1])
        before = nmb.get_state(ctx)
        with pytest.raises(nmb.NewmarkError) as e:
            nmb.newmark_step(ctx, pb.U(2))
        assert e.value.code == nmb.NM_EINVAL
        bad = rows[1:3].copy()
        bad[1, 0] = np.inf
        with pytest.raises(nmb.NewmarkError) as e:
            nmb.explicit_step(ctx, bad, n_steps=2)
        assert e.value.code == nmb.NM_ENAN
        after = nmb.get_state(ctx)
        assert all(np.array_equal(before[k], after[k]) for k in ("u", "v", "a")) and after["step"] == 1
    with nmb.newmark_init_problem(W.make_spheres3d(n=16, seed=2), nmb.Options()) as ctx:
        with pytest.raises(nmb.NewmarkError) as e:
            nmb.explicit_step(ctx, rows[:1])
        assert e.value.code == nmb.NM_EINVAL
