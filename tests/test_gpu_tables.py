"""Implicit against explicit on the GPU, as Tables 2 and 3 compare them (sections 2.3 and 3):
the same plane-wave bar (512 x 8 x 8 voxels, Gamma the x = 0 plane, P-wave Ricker pulse of 64
voxels per wavelength, Table 1 metals) integrated by the implicit Newmark method at 1, 2, 5 and
10 CFL and by the explicit central-difference scheme at 0.9 of its stable increment
(2 / omega_max, eq. Courant_stable, omega_max from the corner frequencies of the grid), with the
error e_r (relative L2 at the final time) and the wall time of each run.

e_r is taken against the time-converged solution on the same grid (the 1D oracle run of the bar
at 0.25 CFL; the 3D GPU run of a plane wave equals the 1D run), so that it isolates the time
integration; for the homogeneous bar the error against d'Alembert's U(t - |x - x0| / c), which
adds the spatial error of the point source, is printed beside it.
* Homogeneous aluminium (Table 2) and Al/Fe/Al layers (Table 3): the explicit run is converged in
  time (e_r below 1e-2), the implicit error grows with the increment, by about 4 from 1 to 2 CFL
  (second order), and the explicit run takes more than ten times the steps of the implicit run at
  10 CFL.  With 64 voxels per wavelength, 10 CFL leaves 6.4 steps per period, so the implicit
  error there is of order one: the paper's pulses span far more voxels than this bar allows.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

pytestmark = pytest.mark.gpu


def _omega_max(pb):
    """Largest frequency of the spectral operator for isotropic phases: max c_L |xi| over the
    corner frequencies (every axis at (n_i - 2) pi / L_i, the Nyquist bin being zero)."""
    xi2 = sum((np.pi * (n - 2) / L) ** 2 for n, L in zip(pb.n, pb.L) if n > 1)
    c_max = max(W.iso_speeds(pb.C21[g], pb.rho[g])[0] for g in range(len(pb.rho)))
    return c_max * np.sqrt(xi2)


def _implicit(pb, t_end):
    steps = int(round(t_end / pb.dt))
    pb.dt = t_end / steps
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=800)) as ctx:
        t0 = time.perf_counter()
        its = 0
        for s in range(steps):
            its += nmb.newmark_step(ctx, pb.U(s + 1))["iters"][0]
        ms = (time.perf_counter() - t0) * 1e3
        u = nmb.get_state(ctx)["u"][0, 0, 0].copy()
    return u, steps, its, ms


def _explicit(pb, t_end, frac=0.9):
    import dataclasses
    dt = frac * 2.0 / _omega_max(pb)
    steps = int(np.ceil(t_end / dt))
    dt = t_end / steps
    pe = dataclasses.replace(pb, dt=dt, beta=0.0, gamma_nm=0.5)
    rows = np.stack([pe.Udot(s + 1) for s in range(steps)])
    with nmb.newmark_init_problem(pe, nmb.Options()) as ctx:
        t0 = time.perf_counter()
        k = 0
        while k < steps:
            nb = min(200, steps - k)
            nmb.explicit_step(ctx, rows[k:k + nb], n_steps=nb)
            k += nb
        ms = (time.perf_counter() - t0) * 1e3
        u = nmb.get_state(ctx)["u"][0, 0, 0].copy()
    return u, steps, ms, dt


def _table(runs):
    for name, (e, ex, steps, extra, ms) in runs.items():
        tail = "" if ex is None else f", vs d'Alembert {ex:.3e}"
        print(f"  {name:>14}: e_r {e:.3e}{tail}, {steps:5d} steps{extra}, {ms:8.1f} ms", flush=True)


def _reference(base, t_end):
    """The 1D oracle run of the same bar at 0.25 CFL (the time-converged solution on this grid)."""
    n1 = base.n[0]
    C1 = np.zeros((len(base.rho), 21))
    for g in range(len(base.rho)):
        C1[g, 0] = W.voigt_from21(base.C21[g])[0, 0]
    c_max = max(W.iso_speeds(base.C21[g], base.rho[g])[0] for g in range(len(base.rho)))
    steps = int(round(t_end / (0.25 / c_max)))
    dt = t_end / steps
    U = np.array([W.ricker((s + 1) * dt, base.pulse_fc) for s in range(steps)])[:, None]
    return oracle.OracleProblem(1, (n1,), (float(n1),), base.phase_id[0, 0], C1, base.rho, dt).newmark(
        np.array([0], np.int64), U, steps, tol=1e-12)["u"][-1, 0, 0, 0]


def _compare(layers, travel, exact=None):
    base = W.make_planar_bar(layers=layers)
    c0 = W.iso_speeds(base.C21[0], base.rho[0])[0]
    c_max = max(W.iso_speeds(base.C21[g], base.rho[g])[0] for g in range(len(base.rho)))
    t_end = 2.0 / base.pulse_fc + travel * base.n[0] / c0
    ref = _reference(base, t_end)
    ex = None if exact is None else exact(base, c0, t_end)

    def err(u, r):
        return float(np.linalg.norm(u - r) / np.linalg.norm(r))

    runs = {}
    for cfl in (1.0, 2.0, 5.0, 10.0):
        u, steps, its, ms = _implicit(W.make_planar_bar(layers=layers, cfl=cfl), t_end)
        runs[f"implicit {cfl:g} CFL"] = (err(u, ref), None if ex is None else err(u, ex), steps,
                                         f" ({its} PCG iterations)", ms)
    u, steps, ms, dt = _explicit(base, t_end)
    runs[f"explicit {dt * c_max:.2f} CFL"] = (err(u, ref), None if ex is None else err(u, ex), steps, "", ms)
    _table(runs)
    return runs


def _check(runs):
    e = {k: v[0] for k, v in runs.items()}
    s = {k: v[2] for k, v in runs.items()}
    ex = [k for k in runs if k.startswith("explicit")][0]
    assert e[ex] <= 1e-2
    assert e["implicit 1 CFL"] < e["implicit 2 CFL"] < e["implicit 5 CFL"] < e["implicit 10 CFL"]
    assert 3.0 <= e["implicit 2 CFL"] / e["implicit 1 CFL"] <= 5.0  # second order in time
    assert s[ex] >= 10 * s["implicit 10 CFL"]


def _dalembert(base, c, t_end):
    x = np.arange(base.n[0]) + 0.5
    d = np.minimum(np.abs(x - 0.5), base.n[0] - np.abs(x - 0.5))
    return W.ricker(t_end - d / c, base.pulse_fc)


def test_table2_homogeneous_bar_implicit_vs_explicit():
    print("Table 2 analogue (homogeneous Al bar, P wave; e_r against the time-converged run):", flush=True)
    _check(_compare((("Al", 1.0),), 0.3, exact=_dalembert))


def test_table3_layered_bar_implicit_vs_explicit():
    print("Table 3 analogue (Al/Fe/Al bar, P wave; e_r against the time-converged run):", flush=True)
    _check(_compare((("Al", 0.3), ("Fe", 0.3), ("Al", 0.4)), 0.5))
