"""Pins of the oracle's viscous buffer (section 5 proposes a viscous or compliant buffer to
suppress the second wave that periodicity creates): M a + C v + K u = f with C = diag(c(x))
per phase, integrated by the same Newmark rule, so that the implicit operator's density is
rho + gamma dt c and the right-hand side (rho + gamma dt c) u~ - beta dt^2 c v~.

* Zero coefficients reproduce the undamped run bit for bit.
* Free vibration of a heterogeneous damped medium obeys the exact discrete dissipation
  identity of the trapezoidal rule (beta = 1/4, gamma = 1/2):
      E_{n+1} - E_n = -dt vbar . C vbar,   vbar = (v_n + v_{n+1}) / 2,
      E = v.M v / 2 + u.K u / 2  (M = diag(rho), K = -div(C : grad^s .)),
  the velocities following from the displacements alone (u_{n+1} - u_n = dt vbar).
* A viscous ramp absorbs the pulse that runs into it, while a pulse elsewhere equals the
  undamped run.
"""
import numpy as np

import oracle
from paper_2211_08263_amd import workloads as W


def test_zero_damping_is_the_undamped_run():
    rng = np.random.default_rng(1)
    n = (8, 8, 4)
    C21 = W.random_anisotropic21(rng, 2)
    phase = W.random_phase_map(rng, n, 2)
    g = W.gamma_x_slab(n)
    U = np.array([[W.ricker((s + 1) * 0.7, 0.1), 0.0, 0.0] for s in range(6)])
    a = oracle.OracleProblem(3, n, (8.0, 8.0, 4.0), phase, C21, [1.0, 2.0], 0.7).newmark(g, U, 6, tol=1e-12)
    b = oracle.OracleProblem(3, n, (8.0, 8.0, 4.0), phase, C21, [1.0, 2.0], 0.7, damping=[0.0, 0.0]).newmark(
        g, U, 6, tol=1e-12)
    assert np.array_equal(a["u"], b["u"])


def test_damped_free_vibration_obeys_the_discrete_dissipation_identity():
    rng = np.random.default_rng(2)
    n = (8, 4, 8)
    C21 = W.random_anisotropic21(rng, 3)
    rho = np.array([1.0, 2.0, 0.7])
    damp = np.array([0.0, 0.3, 1.5])
    phase = W.random_phase_map(rng, n, 3)
    dt = 0.9
    p = oracle.OracleProblem(3, n, tuple(float(x) for x in n), phase, C21, rho, dt, damping=damp)
    u0 = W.random_field(p.field_shape, seed=3)
    v0 = W.random_field(p.field_shape, seed=4)
    steps = 25
    r = p.newmark(np.zeros(0, np.int64), np.zeros((steps, 3)), steps, tol=1e-14, max_iter=3000, u0=u0, v0=v0)
    us = np.concatenate([u0[None], r["u"]])
    rv = rho[phase][None]
    cv = damp[phase][None]
    vs = [v0]
    for k in range(steps):
        vbar = (us[k + 1] - us[k]) / dt
        vs.append(2 * vbar - vs[-1])
    np.testing.assert_allclose(vs[-1], r["v"], rtol=0, atol=1e-9 * np.abs(r["v"]).max())

    def E(u, v):
        return 0.5 * np.sum(rv * v * v) - 0.5 * np.sum(u * p.div_stress(u))

    Es = [E(us[k], vs[k]) for k in range(steps + 1)]
    worst, lost = 0.0, 0.0
    for k in range(steps):
        vbar = 0.5 * (vs[k] + vs[k + 1])
        diss = dt * np.sum(cv * vbar * vbar)
        lost += diss
        worst = max(worst, abs(Es[k + 1] - Es[k] + diss))
    assert lost > 0.2 * Es[0]  # the damping does something
    assert worst <= 1e-9 * Es[0], worst / Es[0]


def test_viscous_ramp_absorbs_a_pulse_and_leaves_the_rest_alone():
    """Two smooth pulses on a periodic bar of 2048 voxels (no Gamma; initial data u0 = f(x - x0),
    v0 = -/+ f'): A runs right into a viscous layer whose coefficient rises as a quadratic
    ramp over 400 voxels (one phase per voxel, so c(x) has no jump), B runs left, away from it.
    After 400 steps A has spent 200 steps in the ramp and B has not come near it: B equals the
    undamped run to solver tolerance (the implicit solve is local: its kernel decays over a
    fraction of a voxel at dt = h / c), A's amplitude has fallen below a quarter of the
    undamped one and what the ramp sent back is below a tenth.  (A sharp-edged layer couples
    to the zero-stiffness checkerboard of even grids, the Nyquist bin being zero, and changes
    the far field by about 1e-5 here; with a point source on Gamma the change reaches 1e-3.)"""
    n = 2048
    x = np.arange(n) + 0.5
    w = 24.0

    def f(x0):
        return np.exp(-((x - x0) / w) ** 2)

    def fp(x0):
        return -2.0 * (x - x0) / w ** 2 * f(x0)

    layer = (x > 1200) & (x < 1900)
    phase = np.zeros(n, np.uint16)
    phase[layer] = np.arange(1, layer.sum() + 1)
    n_ph = int(layer.sum()) + 1
    ramp = np.clip((x[layer] - 1200) / 400, 0, 1)
    damp = np.concatenate([[0.0], 0.2 * ramp ** 2])
    C1 = np.zeros((n_ph, 21))
    C1[:, 0] = 1.0
    u0 = (f(1000) + f(500))[None]
    v0 = (-fp(1000) + fp(500))[None]
    steps = 400
    runs = {}
    for name, dmp in (("free", None), ("buffer", damp)):
        p = oracle.OracleProblem(1, (n,), (float(n),), phase, C1, np.ones(n_ph), 1.0, damping=dmp)
        runs[name] = p.newmark(np.zeros(0, np.int64), np.zeros((steps, 1)), steps, tol=1e-13, u0=u0, v0=v0)["u"][:, 0, 0, 0]
    uf, ub = runs["free"][-1], runs["buffer"][-1]
    B = x < 800
    back = (x > 800) & (x < 1200)
    e_B = np.abs(ub[B] - uf[B]).max() / np.abs(uf[B]).max()
    att = np.abs(ub[layer]).max() / np.abs(uf[layer]).max()
    refl = np.abs(ub[back]).max()
    assert np.abs(uf[back]).max() < 1e-10  # nothing there without the buffer
    assert e_B < 1e-8, e_B
    assert att < 0.25, att
    assert refl < 0.1, refl
