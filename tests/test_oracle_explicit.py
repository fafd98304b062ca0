"""Pins of the oracle's explicit central-difference scheme (section 2.3: Newmark with
beta = 0, gamma = 1/2, the velocity prescribed on Gamma) and of its eigenvalue iteration
for the stable increment.

* One Fourier mode in a homogeneous anisotropic medium follows the exact central-difference
  map u_n = cos(n theta) u_0, cos theta = 1 - omega^2 dt^2 / 2, with omega^2 an eigenvalue of
  the acoustic tensor Q(xi) (eq. Eigenvalues_1D_homogeneo; numpy's eigh).
* The stable increment 2 / omega_max (eq. Courant_stable), omega_max^2 the largest eigenvalue
  of Q over the discrete frequencies (brute force over every frequency, numpy): 2% below it a
  random field stays bounded, 2% above it the run blows up.
* Free vibration of a heterogeneous medium conserves the discrete energy of the central
  difference scheme, |u_{n+1} - u_n|^2_rho / (2 dt^2) + u_{n+1} . K u_n / 2 (exactly, up to
  rounding: it follows from the recurrence alone).
* The velocity on Gamma equals the prescribed one after every step; the Gamma force
  balances rho a_n - div sigma(u_n) there.
* A 3D x-layered medium driven on a full plane equals the 1D run with modulus lambda + 2 mu.
* d'Alembert (appendix C): a velocity-driven 1D bar reproduces U(t - |x - x0| / c).
* The power iteration reaches omega_max^2 of a homogeneous medium (the closed form above) and
  stays below it (a Rayleigh quotient) on a heterogeneous one.
"""
import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import workloads as W


def _tensor(c21):
    return W._voigt66_to_tensor(W.voigt_from21(c21))


def _xi_axis(n, L):
    k = np.arange(n)
    kk = np.where(2 * k < n, k, k - n).astype(float)
    kk[n // 2] = 0.0  # Nyquist bin: zero frequency
    return 2 * np.pi * kk / L


def _omega2_max_homogeneous(c21, rho, n, L):
    """Largest eigenvalue of Q(xi) = C_ijkl xi_j xi_l / rho over every discrete frequency."""
    T = _tensor(c21)
    x1, x2, x3 = (_xi_axis(n[i], L[i]) for i in range(3))
    X = np.stack(np.meshgrid(x1, x2, x3, indexing="ij"), -1).reshape(-1, 3)
    Q = np.einsum("ijkl,pj,pl->pik", T, X, X) / rho
    return float(np.linalg.eigvalsh(Q).max())


def _homogeneous(n, c21, rho, dt):
    phase = np.zeros((n[2], n[1], n[0]), np.uint16)
    return oracle.OracleProblem(3, n, tuple(float(x) for x in n), phase, c21[None], [rho], dt)


def _cu21(seed):
    R = W.random_rotations(np.random.default_rng(seed), 1)[0]
    return W.voigt_to21(W.rotate_voigt66(W.copper_scaled66(), R))


def test_free_vibration_follows_the_central_difference_map():
    n = (8, 8, 8)
    c21, rho = _cu21(1), 1.3
    m = np.array([1, -2, 3])
    xi = 2 * np.pi * m / 8.0
    lam, vec = np.linalg.eigh(np.einsum("ijkl,j,l->ik", _tensor(c21), xi, xi) / rho)
    z, y, x = np.meshgrid(*(np.arange(8) + 0.5,) * 3, indexing="ij")
    wave = np.cos(xi[0] * x + xi[1] * y + xi[2] * z)
    # below the stable increment of the whole grid (rounding excites every frequency)
    dt = 0.9 * 2.0 / np.sqrt(_omega2_max_homogeneous(c21, rho, n, (8.0,) * 3))
    p = _homogeneous(n, c21, rho, dt)
    steps = 40
    for k in range(3):
        u0 = vec[:, k][:, None, None, None] * wave[None]
        r = p.explicit(np.zeros(0, np.int64), np.zeros((steps, 3)), steps, u0=u0)
        theta = np.arccos(1 - lam[k] * dt * dt / 2)
        want = np.cos(theta * np.arange(1, steps + 1))[:, None, None, None, None] * u0[None]
        err = np.abs(r["u"] - want).max() / np.abs(u0).max()
        assert err < 1e-12, (k, err)


@pytest.mark.parametrize("factor,bounded", [(0.98, True), (1.02, False)])
def test_stable_increment_is_two_over_omega_max(factor, bounded):
    n = (8, 8, 8)
    c21, rho = _cu21(2), 1.0
    w2 = _omega2_max_homogeneous(c21, rho, n, (8.0, 8.0, 8.0))
    dt = factor * 2.0 / np.sqrt(w2)
    p = _homogeneous(n, c21, rho, dt)
    u0 = W.random_field((3, 8, 8, 8), seed=3)
    steps = 300
    r = p.explicit(np.zeros(0, np.int64), np.zeros((steps, 3)), steps, u0=u0)
    growth = np.abs(r["u"][-1]).max() / np.abs(u0).max()
    if bounded:
        assert np.abs(r["u"]).max() / np.abs(u0).max() < 20.0, growth
    else:
        assert growth > 1e6, growth


def test_heterogeneous_free_vibration_conserves_the_discrete_energy():
    rng = np.random.default_rng(5)
    n = (8, 4, 8)
    C21 = W.random_anisotropic21(rng, 3)
    rho = np.array([1.0, 2.0, 0.7])
    phase = W.random_phase_map(rng, n, 3)
    p = oracle.OracleProblem(3, n, tuple(float(x) for x in n), phase, C21, rho, 0.05)
    u0 = W.random_field(p.field_shape, seed=6)
    v0 = W.random_field(p.field_shape, seed=7)
    steps = 60
    r = p.explicit(np.zeros(0, np.int64), np.zeros((steps, 3)), steps, u0=u0, v0=v0)
    us = np.concatenate([u0[None], r["u"]])
    rv = rho[phase][None]

    def K(u):
        return -p.div_stress(u)

    E = [0.5 * np.sum(rv * (us[k + 1] - us[k]) ** 2) / p.dt ** 2 + 0.5 * np.sum(us[k + 1] * K(us[k]))
         for k in range(steps)]
    E = np.array(E)
    dev = np.abs(E - E[0]).max() / abs(E[0])
    assert dev < 1e-11, dev


def test_prescribed_velocity_on_gamma_and_force_balance():
    pb = W.make_polycrystal(n=16, n_grains=5, seed=9, gamma="sphere", sphere_radius=3.0)
    p = oracle.OracleProblem.from_problem(pb)
    dt = 0.3
    steps = 25
    Ud = np.stack([pb.Udot(s + 1, dt) for s in range(steps)]) * 5.0
    p.dt = dt
    p.s.dt = dt
    r = p.explicit(pb.gamma_idx, Ud, steps, want_v=True, want_F=True)
    for s in range(steps):
        vg = r["v"][s].reshape(3, -1)[:, pb.gamma_idx]
        np.testing.assert_allclose(vg, np.repeat(Ud[s][:, None], pb.gamma_idx.size, 1), rtol=0,
                                   atol=1e-13 * max(1.0, np.abs(Ud).max()))
    # rho a_n - div sigma(u_n) is the Gamma force on Gamma and zero elsewhere
    rho = pb.rho[pb.phase_id][None]
    bal = (rho * r["a_last"] - p.div_stress(r["u"][-1])).reshape(3, -1)
    F = r["F"][-1].reshape(-1, 3).T
    scale = np.abs(F).max()
    np.testing.assert_allclose(bal[:, pb.gamma_idx], F, rtol=0, atol=1e-10 * scale)
    off = np.ones(pb.n_vox, bool)
    off[pb.gamma_idx] = False
    assert np.abs(bal[:, off]).max() <= 1e-10 * scale


def test_3d_layered_plane_source_equals_1d():
    n1 = 32
    Es, nu, rhos = (1.0, 4.0), 0.3, (1.0, 2.0)
    layer = ((np.arange(n1) // 8) % 2).astype(np.uint16)
    C21 = np.stack([W.voigt_to21(W.isotropic_voigt66(E, nu)) for E in Es])
    ph3 = np.broadcast_to(layer[None, None, :], (4, 4, n1)).copy()
    dt = 0.2
    p3 = oracle.OracleProblem(3, (n1, 4, 4), (32.0, 4.0, 4.0), ph3, C21, rhos, dt)
    M = np.array([W.isotropic_voigt66(E, nu)[0, 0] for E in Es])
    C1 = np.zeros((2, 21))
    C1[:, 0] = M
    p1 = oracle.OracleProblem(1, (n1,), (32.0,), layer, C1, rhos, dt)
    steps = 80
    Ud = np.array([W.ricker_rate((s + 1) * dt, 0.1) for s in range(steps)])
    r1 = p1.explicit(np.array([0], np.int64), Ud[:, None], steps)
    r3 = p3.explicit(W.gamma_x_slab((n1, 4, 4)), np.stack([Ud, 0 * Ud, 0 * Ud], 1), steps)
    np.testing.assert_allclose(r3["u"][:, 0], np.broadcast_to(r1["u"][:, 0], r3["u"][:, 0].shape), atol=1e-11)
    np.testing.assert_allclose(r3["u"][:, 1:], 0.0, atol=1e-12)


def test_dalembert_velocity_driven_bar():
    """Homogeneous bar whose point x0 moves with velocity U'(t): the displacement is
    U(t - |x - x0| / c) (two counter-propagating pulses, appendix C).  Both schemes share the
    spatial error of the single-voxel source (a few per cent here); at the explicit stable
    increments the time error is far below it, and the explicit run agrees with the implicit
    run at a small time increment to a fraction of that error (both are second order in
    time and converge to the same semi-discrete solution)."""
    n, L, c = 2048, 512.0, 1.0
    h = L / n
    fc = 1.0 / 32
    x = (np.arange(n) + 0.5) * h
    d = np.minimum(np.abs(x - 0.5 * h), L - np.abs(x - 0.5 * h))
    T = 200.0
    C1 = np.zeros((1, 21))
    C1[0, 0] = c * c
    exact = W.ricker(T - d / c, fc)
    dt_c = 2.0 / (c * 2 * np.pi * (n // 2 - 1) / L)
    steps = int(np.ceil(T / (0.4 * dt_c)))
    dt = T / steps
    p = oracle.OracleProblem(1, (n,), (L,), np.zeros(n, np.uint16), C1, [1.0], dt)
    Ud = np.array([W.ricker_rate((s + 1) * dt, fc) for s in range(steps)])
    ue = p.explicit(np.array([0], np.int64), Ud[:, None], steps)["u"][-1, 0, 0, 0]
    pi = oracle.OracleProblem(1, (n,), (L,), np.zeros(n, np.uint16), C1, [1.0], T / 3200)
    Ui = np.array([W.ricker((s + 1) * T / 3200, fc) for s in range(3200)])
    ui = pi.newmark(np.array([0], np.int64), Ui[:, None], 3200, tol=1e-12)["u"][-1, 0, 0, 0]
    e_exact = np.linalg.norm(ue - exact) / np.linalg.norm(exact)
    e_impl = np.linalg.norm(ue - ui) / np.linalg.norm(exact)
    print(f"explicit vs analytic {e_exact:.3e}, vs implicit at dt = T/3200 {e_impl:.3e}")
    assert e_exact < 5e-2
    assert e_impl < 3e-3


def test_power_iteration_reaches_the_largest_eigenvalue():
    n = (8, 8, 8)
    c21, rho = _cu21(4), 1.0
    w2 = _omega2_max_homogeneous(c21, rho, n, (8.0,) * 3)
    p = _homogeneous(n, c21, rho, 0.1)
    lam, _ = p.omega2_max(W.random_field(p.field_shape, seed=1), 400)
    assert lam <= w2 * (1 + 1e-12)
    assert lam >= 0.97 * w2, (lam, w2)
    # heterogeneous: a Rayleigh quotient below the largest single-phase bound
    rng = np.random.default_rng(2)
    C21 = np.stack([_cu21(5), 3.0 * _cu21(6)])
    rho2 = np.array([1.0, 1.5])
    phase = W.random_phase_map(rng, n, 2)
    ph = oracle.OracleProblem(3, n, (8.0,) * 3, phase, C21, rho2, 0.1)
    lam_h, x = ph.omega2_max(W.random_field(ph.field_shape, seed=2), 300)
    bound = max(_omega2_max_homogeneous(C21[g], rho2.min(), n, (8.0,) * 3) for g in range(2))
    assert 0 < lam_h <= bound
    # the returned vector is normalised in the rho-weighted norm
    assert abs(np.sum(rho2[phase][None] * x * x) - 1.0) < 1e-12
