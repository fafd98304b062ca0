"""Seeded synthetic problem inputs for the implicit FFT Newmark solver.

This module only builds *inputs*: voxel phase maps, per-phase stiffness and
density tables, the prescribed-displacement set Gamma, the prescribed time
history U(t) and the time increment.  It holds none of the solver's
arithmetic (no transforms, no operator, no Krylov, no time integration), so
that both the CPU oracle and the GPU library can consume the same arrays.

Conventions shared by every consumer
------------------------------------
* Voxel (i, j, k) has centre ((i + 1/2) h1, (j + 1/2) h2, (k + 1/2) h3)
  (paper, section 2.2.3, voxel discretization).  Its linear index is
  ``i + n1 * (j + n2 * k)``: x is the fastest axis.  numpy arrays are shaped
  ``(n3, n2, n1)``.
* Vector fields are SoA: shape ``(dim, n3, n2, n1)``.
* Stiffness tables hold, per phase, the 21 upper-triangle entries (row
  major) of the 6x6 Voigt matrix in the order 11, 22, 33, 23, 13, 12, with
  engineering shear strains, so that ``sigma_v = C_v @ eps_v`` with
  ``eps_v = (e11, e22, e33, 2 e23, 2 e13, 2 e12)``.
* Units are scaled so that the voxel size is 1 and densities and moduli are
  O(1); the problem is linear, so relative errors do not depend on units.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
N_VOIGT21 = 21


# ----------------------------------------------------------------------------
# Stiffness tables
# ----------------------------------------------------------------------------
def voigt_to21(C66: np.ndarray) -> np.ndarray:
    """Upper triangle (row major) of a symmetric 6x6 Voigt matrix."""
    C66 = np.asarray(C66, dtype=np.float64)
    iu = np.triu_indices(6)
    return C66[iu].copy()


def voigt_from21(c21: np.ndarray) -> np.ndarray:
    c21 = np.asarray(c21, dtype=np.float64)
    C = np.zeros((6, 6))
    iu = np.triu_indices(6)
    C[iu] = c21
    C = C + C.T - np.diag(np.diag(C))
    return C


def isotropic_voigt66(E: float, nu: float) -> np.ndarray:
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def cubic_voigt66(C11: float, C12: float, C44: float) -> np.ndarray:
    C = np.zeros((6, 6))
    C[:3, :3] = C12
    C[0, 0] = C[1, 1] = C[2, 2] = C11
    C[3, 3] = C[4, 4] = C[5, 5] = C44
    return C


def _voigt66_to_tensor(C66: np.ndarray) -> np.ndarray:
    T = np.zeros((3, 3, 3, 3))
    for a, (i, j) in enumerate(VOIGT_PAIRS):
        for b, (k, l) in enumerate(VOIGT_PAIRS):
            v = C66[a, b]
            for (p, q) in ((i, j), (j, i)):
                for (r, s) in ((k, l), (l, k)):
                    T[p, q, r, s] = v
    return T


def _tensor_to_voigt66(T: np.ndarray) -> np.ndarray:
    C = np.zeros((6, 6))
    for a, (i, j) in enumerate(VOIGT_PAIRS):
        for b, (k, l) in enumerate(VOIGT_PAIRS):
            C[a, b] = T[i, j, k, l]
    return C


def rotate_voigt66(C66: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Stiffness of a crystal whose axes are rotated by R: C'_ijkl = R_ip R_jq R_kr R_ls C_pqrs."""
    T = _voigt66_to_tensor(C66)
    Tr = np.einsum("ip,jq,kr,ls,pqrs->ijkl", R, R, R, R, T, optimize=True)
    return _tensor_to_voigt66(Tr)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed rotations (Shoemake's subgroup algorithm on unit quaternions)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1 - u1)
    b = np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    w, x, y, z = q[:, 3], q[:, 0], q[:, 1], q[:, 2]
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


# Copper, cubic (GPa, kg/m^3).  Scaled so that C11 -> 1 and rho -> 1.
CU_C11, CU_C12, CU_C44, CU_RHO = 168.4, 121.4, 75.4, 8960.0


def copper_scaled66() -> np.ndarray:
    return cubic_voigt66(1.0, CU_C12 / CU_C11, CU_C44 / CU_C11)


def longitudinal_speed_max(C66: np.ndarray, rho: float, n_dirs: int = 0) -> float:
    """Largest quasi-longitudinal phase speed over propagation directions.

    Input preparation only (it fixes the time increment): the eigenvalues of
    the Christoffel matrix n.C.n / rho over a fixed set of directions that
    contains the cubic axes, face and body diagonals.
    """
    T = _voigt66_to_tensor(C66)
    dirs = [np.array(v, dtype=float) for v in
            ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1),
             (1, -1, 0), (1, 0, -1), (0, 1, -1),
             (1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1))]
    if n_dirs:
        g = np.random.default_rng(0).normal(size=(n_dirs, 3))
        dirs += list(g)
    best = 0.0
    for n in dirs:
        n = n / np.linalg.norm(n)
        Q = np.einsum("ijkl,j,l->ik", T, n, n) / rho
        best = max(best, float(np.sqrt(np.linalg.eigvalsh(Q).max())))
    return best


def voigt_average66(C66: np.ndarray) -> np.ndarray:
    """Orientation (Voigt) average of a stiffness: the isotropic part."""
    T = _voigt66_to_tensor(C66)
    I = np.eye(3)
    a = np.einsum("iijj->", T)  # C_iijj
    b = np.einsum("ijij->", T)  # C_ijij
    # isotropic tensor lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)
    # C_iijj = 9 lam + 6 mu ; C_ijij = 3 lam + 12 mu
    mu = (3 * b - a) / 30.0
    lam = (a - 6 * mu) / 9.0
    Tiso = lam * np.einsum("ij,kl->ijkl", I, I) + mu * (
        np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I))
    return _tensor_to_voigt66(Tiso)


# ----------------------------------------------------------------------------
# Microstructures
# ----------------------------------------------------------------------------
def voxel_centres(n: Tuple[int, ...]) -> Tuple[np.ndarray, ...]:
    return tuple(np.arange(m) + 0.5 for m in n)


def disc_2d(n1: int, n2: int, radius: float, centre=None) -> np.ndarray:
    """Phase map (1, n2, n1): 1 inside the disc (voxel centres within radius, ties in)."""
    c = (n1 / 2.0, n2 / 2.0) if centre is None else centre
    x = np.arange(n1) + 0.5
    y = np.arange(n2) + 0.5
    d2 = (x[None, :] - c[0]) ** 2 + (y[:, None] - c[1]) ** 2
    return (d2 <= radius * radius).astype(np.uint16)[None]


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def rsa_spheres(n: int, rng: np.random.Generator, rmin: float = 4.0, rmax: float = 10.0,
                target_fraction: float = 0.3, max_tries: int = 200000) -> Tuple[np.ndarray, np.ndarray]:
    """Periodic random sequential adsorption of non-overlapping spheres.

    Radii ~ U[rmin, rmax], centres ~ U[0, n)^3; a candidate is rejected if it
    overlaps an accepted sphere under the minimum-image convention.  Stops
    once the voxel volume fraction of the inclusion phase reaches the target.
    Returns (phase map (n, n, n) uint16 with 1 = inclusion, sphere array).
    """
    phase = np.zeros((n, n, n), dtype=np.uint16)
    spheres = []
    c1 = np.arange(n) + 0.5
    count = 0
    for _ in range(max_tries):
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0, n, size=3)
        ok = True
        for (cs, rs) in spheres:
            d = _min_image(c - cs, n)
            if np.dot(d, d) < (r + rs) ** 2:
                ok = False
                break
        if not ok:
            continue
        spheres.append((c, r))
        # paint voxels of this sphere (periodic)
        lo = np.floor(c - r - 1).astype(int)
        hi = np.ceil(c + r + 1).astype(int)
        ii = np.arange(lo[0], hi[0])
        jj = np.arange(lo[1], hi[1])
        kk = np.arange(lo[2], hi[2])
        dx = (ii + 0.5 - c[0])
        dy = (jj + 0.5 - c[1])
        dz = (kk + 0.5 - c[2])
        inside = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2) <= r * r
        K, J, I = np.nonzero(inside)
        kz, jy, ix = kk[K] % n, jj[J] % n, ii[I] % n
        new = phase[kz, jy, ix] == 0
        count += int(new.sum())
        phase[kz, jy, ix] = 1
        if count >= target_fraction * n ** 3:
            break
    sph = np.array([[*c, r] for (c, r) in spheres])
    return phase, sph


def voronoi_periodic(n: Tuple[int, int, int], n_seeds: int, rng: np.random.Generator) -> np.ndarray:
    """Periodic Voronoi tessellation: phase id = index of the nearest seed
    (minimum-image distance) to each voxel centre.  Seeds ~ U[0, n_i)."""
    from scipy.spatial import cKDTree
    n1, n2, n3 = n
    seeds = np.stack([rng.uniform(0, n1, n_seeds), rng.uniform(0, n2, n_seeds),
                      rng.uniform(0, n3, n_seeds)], axis=1)
    tree = cKDTree(seeds, boxsize=(n1, n2, n3))
    out = np.empty((n3, n2, n1), dtype=np.uint16)
    x = np.arange(n1) + 0.5
    y = np.arange(n2) + 0.5
    X, Y = np.meshgrid(x, y, indexing="xy")
    pts = np.empty((n2 * n1, 3))
    pts[:, 0] = X.ravel()
    pts[:, 1] = Y.ravel()
    for k in range(n3):
        pts[:, 2] = k + 0.5
        _, idx = tree.query(pts, k=1, workers=-1)
        out[k] = idx.reshape(n2, n1).astype(np.uint16)
    return out


# ----------------------------------------------------------------------------
# Gamma sets (prescribed-displacement voxels) and pulses
# ----------------------------------------------------------------------------
def gamma_x_slab(n: Tuple[int, int, int], width: int = 1) -> np.ndarray:
    """Linear indices of the voxels with x index < width (sorted, int64)."""
    n1, n2, n3 = n
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(width), indexing="ij")
    idx = (i + n1 * (j + n2 * k)).ravel()
    return np.sort(idx).astype(np.int64)


def gamma_sphere(n: Tuple[int, int, int], centre, radius: float) -> np.ndarray:
    n1, n2, n3 = n
    x = np.arange(n1) + 0.5
    y = np.arange(n2) + 0.5
    z = np.arange(n3) + 0.5
    d2 = ((z[:, None, None] - centre[2]) ** 2 + (y[None, :, None] - centre[1]) ** 2
          + (x[None, None, :] - centre[0]) ** 2)
    idx = np.flatnonzero(d2.ravel() <= radius * radius)
    return idx.astype(np.int64)


def ricker(t, fc: float, t0: Optional[float] = None, amp: float = 1.0):
    """Ricker wavelet A (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0, t0 = 2/f."""
    if t0 is None:
        t0 = 2.0 / fc
    tau = np.asarray(t, dtype=np.float64) - t0
    a = (np.pi * fc * tau) ** 2
    return amp * (1 - 2 * a) * np.exp(-a)


def ricker_rate(t, fc: float, t0: Optional[float] = None, amp: float = 1.0):
    """Time derivative of ricker(): the prescribed velocity of the explicit scheme's source.
    With a = (pi fc tau)^2: d/dt [(1 - 2a) e^-a] = 2 pi^2 fc^2 tau (2a - 3) e^-a."""
    if t0 is None:
        t0 = 2.0 / fc
    tau = np.asarray(t, dtype=np.float64) - t0
    a = (np.pi * fc * tau) ** 2
    return amp * 2.0 * (np.pi * fc) ** 2 * tau * (2 * a - 3) * np.exp(-a)


def bell_pulse(t, A: float, omega: float, alpha: float = 4.0):
    """Bell pulse of the paper's 1D tests (section 3.1): A (t (T - t))^alpha / (T^2/4)^alpha on [0, T], T = pi/omega."""
    T = math.pi / omega
    t = np.asarray(t, dtype=np.float64)
    v = A * (t * (T - t)) ** alpha / ((T * T / 4.0) ** alpha)
    return np.where((t >= 0) & (t <= T), v, 0.0)


# ----------------------------------------------------------------------------
# Problems
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """Everything the solver needs (the paper's Algorithm 2 inputs)."""
    name: str
    dim: int
    n: Tuple[int, int, int]          # (n1, n2, n3), n3 == 1 for dim == 2
    L: Tuple[float, float, float]
    phase_id: np.ndarray             # (n3, n2, n1) uint16
    C21: np.ndarray                  # (n_phases, 21) float64
    rho: np.ndarray                  # (n_phases,) float64
    gamma_idx: np.ndarray            # (n_gamma,) int64 sorted unique
    dt: float
    beta: float = 0.25
    gamma_nm: float = 0.5
    pulse_fc: float = 0.0
    pulse_dir: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    n_steps: int = 0
    tol: float = 1e-8
    damping: Optional[np.ndarray] = None  # (n_phases,) viscous coefficients (force -c v), or None
    diff_rule: int = 0                     # 0 spectral derivative, 1 / 2 centred differences of order 2 / 4

    @property
    def n_vox(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def U(self, step: int) -> np.ndarray:
        """Prescribed displacement vector (dim values, uniform on Gamma) at t_step = step * dt."""
        a = float(ricker(step * self.dt, self.pulse_fc)) if self.pulse_fc > 0 else 0.0
        return np.array(self.pulse_dir[: self.dim], dtype=np.float64) * a

    def Udot(self, step: int, dt: Optional[float] = None) -> np.ndarray:
        """Prescribed velocity (the rate of U) at t_step = step * dt (dt defaults to the
        problem's; the explicit scheme runs at its own stable increment)."""
        h = self.dt if dt is None else dt
        a = float(ricker_rate(step * h, self.pulse_fc)) if self.pulse_fc > 0 else 0.0
        return np.array(self.pulse_dir[: self.dim], dtype=np.float64) * a


def _iso_pair(E_m=1.0, nu=0.3, rho_m=1.0, E_i=10.0, rho_i=3.0):
    C = np.stack([voigt_to21(isotropic_voigt66(E_m, nu)), voigt_to21(isotropic_voigt66(E_i, nu))])
    rho = np.array([rho_m, rho_i])
    return C, rho


def plane_strain_cL(E, nu, rho):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return math.sqrt((lam + 2 * mu) / rho)


def make_disc2d(n: int = 64, radius: float = 12.0, cfl: float = 2.0, n_steps: int = 100,
                tol: float = 1e-10) -> Problem:
    """2D plane strain: matrix E=1, nu=0.3, rho=1 with a centred disc E=10, rho=3;
    Gamma = the left 2-voxel strip, Ricker pulse along x1 (~8 voxels per wavelength)."""
    phase = disc_2d(n, n, radius)
    C, rho = _iso_pair()
    c_max = max(plane_strain_cL(1.0, 0.3, 1.0), plane_strain_cL(10.0, 0.3, 3.0))
    dt = cfl / c_max
    fc = plane_strain_cL(1.0, 0.3, 1.0) / 8.0
    gam = gamma_x_slab((n, n, 1), width=2)
    return Problem("disc2d", 2, (n, n, 1), (float(n), float(n), 1.0), phase, C, rho, gam, dt,
                   pulse_fc=fc, n_steps=n_steps, tol=tol)


def make_spheres3d(n: int = 128, seed: int = 2, cfl: float = 2.0, n_steps: int = 200,
                   tol: float = 1e-8, fraction: float = 0.3) -> Problem:
    """3D two-phase composite: RSA spheres r ~ U[4,10] to volume fraction 0.3,
    contrast 10x stiffness / 3x density, nu = 0.3; Gamma = x=0 face slab."""
    rng = np.random.default_rng(seed)
    phase, _ = rsa_spheres(n, rng, target_fraction=fraction)
    C, rho = _iso_pair()
    cL = lambda E, r: math.sqrt(E * (1 - 0.3) / ((1 + 0.3) * (1 - 0.6)) / r)
    dt = cfl / max(cL(1.0, 1.0), cL(10.0, 3.0))
    fc = cL(1.0, 1.0) / 8.0
    gam = gamma_x_slab((n, n, n))
    return Problem("spheres3d", 3, (n, n, n), (float(n),) * 3, phase, C, rho, gam, dt,
                   pulse_fc=fc, n_steps=n_steps, tol=tol)


def make_polycrystal(n: int = 256, n_grains: int = 500, seed: int = 3, cfl: float = 2.0,
                     n_steps: int = 300, tol: float = 1e-8, gamma: str = "slab",
                     sphere_radius: float = 6.0) -> Problem:
    """Cu polycrystal: periodic Voronoi grains with uniformly random orientations.

    Moduli scaled by C11 and density by rho_Cu.  dt = cfl / c_L[111] (the
    largest longitudinal speed of the crystal); Ricker centre frequency
    c_ref / 8 with c_ref the orientation-averaged longitudinal speed."""
    rng = np.random.default_rng(seed)
    phase = voronoi_periodic((n, n, n), n_grains, rng)
    Rs = random_rotations(rng, n_grains)
    C0 = copper_scaled66()
    C = np.stack([voigt_to21(rotate_voigt66(C0, R)) for R in Rs])
    rho = np.ones(n_grains)
    c_max = longitudinal_speed_max(C0, 1.0)
    dt = cfl / c_max
    c_ref = math.sqrt(voigt_average66(C0)[0, 0])
    fc = c_ref / 8.0
    if gamma == "slab":
        gam = gamma_x_slab((n, n, n))
    else:
        gam = gamma_sphere((n, n, n), (n / 2.0, n / 2.0, n / 2.0), sphere_radius)
    return Problem(f"polycrystal{n}", 3, (n, n, n), (float(n),) * 3, phase, C, rho, gam, dt,
                   pulse_fc=fc, n_steps=n_steps, tol=tol)


def make_columnar_polycrystal(n: int = 256, n_grains: int = 500, seed: int = 3, cfl: float = 2.0,
                              n_steps: int = 300, tol: float = 1e-8, axis: int = 2):
    """Cu polycrystal whose grains are columns along one axis (a periodic 2D Voronoi
    tessellation of the other two axes, extruded), on an n^3 grid.

    Returns ``(full, reduced)``: the n^3 problem and the same problem on a grid with
    one voxel along ``axis`` (dim 3; the transverse Voronoi map and the grain table are
    shared).  Every field that does not vary along ``axis`` has the same image under the
    discretized operator on both grids, so the reduced problem is a small stand-in for
    the full one.  With axis == 2 the prescribed-displacement set is the x = 0 slab on
    both grids; otherwise it is empty.  Time increment and pulse as in
    make_polycrystal."""
    rng = np.random.default_rng(seed)
    red_n = [n, n, n]
    red_n[axis] = 1
    red_n = tuple(red_n)
    phase_red = voronoi_periodic(red_n, n_grains, rng)  # shape (n3, n2, n1) with a 1 along axis
    Rs = random_rotations(rng, n_grains)
    C0 = copper_scaled66()
    C = np.stack([voigt_to21(rotate_voigt66(C0, R)) for R in Rs])
    rho = np.ones(n_grains)
    dt = cfl / longitudinal_speed_max(C0, 1.0)
    fc = math.sqrt(voigt_average66(C0)[0, 0]) / 8.0
    np_axis = 2 - axis  # numpy axis of the grid axis
    phase_full = np.ascontiguousarray(np.repeat(phase_red, n, axis=np_axis))
    if axis == 2:
        g_full, g_red = gamma_x_slab((n, n, n)), gamma_x_slab(red_n)
    else:
        g_full = g_red = np.zeros(0, np.int64)
    full = Problem(f"columnar{n}", 3, (n, n, n), (float(n),) * 3, phase_full, C, rho, g_full, dt,
                   pulse_fc=fc, n_steps=n_steps, tol=tol)
    Lr = [float(n)] * 3
    Lr[axis] = 1.0
    red = Problem(f"columnar{n}-reduced", 3, red_n, tuple(Lr), phase_red, C, rho, g_red, dt,
                  pulse_fc=fc, n_steps=n_steps, tol=tol)
    return full, red


def extrude_field(f: np.ndarray, n: int, axis: int) -> np.ndarray:
    """Repeat a (dim, n3, n2, n1) field that has length 1 along grid axis ``axis`` n times."""
    return np.ascontiguousarray(np.repeat(f, n, axis=3 - axis))


# Table 1 of the paper (E in GPa, rho in kg/m^3, Poisson ratio); scaled below so that
# aluminium has E = 1 and rho = 1.
TABLE1 = {"Al": (70.3, 2700.0, 0.345), "Fe": (211.4, 7850.0, 0.293), "U": (172.0, 18950.0, 0.3)}


def table1_scaled(name: str):
    """(21 Voigt constants, density) of a Table 1 metal, isotropic, scaled by aluminium."""
    E, rho, nu = TABLE1[name]
    E0, rho0, _ = TABLE1["Al"]
    return voigt_to21(isotropic_voigt66(E / E0, nu)), rho / rho0


def iso_speeds(c21: np.ndarray, rho: float):
    """Longitudinal and shear speeds of an isotropic stiffness."""
    C = voigt_from21(c21)
    return math.sqrt(C[0, 0] / rho), math.sqrt(C[5, 5] / rho)


def make_planar_bar(n1: int = 512, n2: int = 8, n3: int = 8, layers=(("Al", 1.0),), wave: str = "P",
                    wavelength_vox: float = 64.0, cfl: float = 2.0, tol: float = 1e-10) -> Problem:
    """Plane-wave bar of section 3.2: x-layered Table 1 metals (consecutive fractions of n1),
    Gamma = the x = 0 plane, Ricker pulse along x (P wave) or y (S wave) with the given
    wavelength in voxels at the first layer's speed; dt = cfl / (largest longitudinal speed)."""
    mats = [table1_scaled(m) for m, _ in layers]
    C = np.stack([m[0] for m in mats])
    rho = np.array([m[1] for m in mats])
    ends = np.cumsum([f for _, f in layers])
    ends = ends / ends[-1]
    xc = (np.arange(n1) + 0.5) / n1
    lay = np.searchsorted(ends, xc, side="right").clip(0, len(layers) - 1).astype(np.uint16)
    phase = np.ascontiguousarray(np.broadcast_to(lay[None, None, :], (n3, n2, n1)))
    cL0, cS0 = iso_speeds(C[0], rho[0])
    c_max = max(iso_speeds(C[g], rho[g])[0] for g in range(len(layers)))
    dt = cfl / c_max
    fc = (cL0 if wave == "P" else cS0) / wavelength_vox
    pb = Problem(f"bar-{wave}", 3, (n1, n2, n3), (float(n1), float(n2), float(n3)), phase, C, rho,
                 gamma_x_slab((n1, n2, n3)), dt, pulse_fc=fc, tol=tol,
                 pulse_dir=(1.0, 0.0, 0.0) if wave == "P" else (0.0, 1.0, 0.0))
    return pb


def gamma_cylinder_x(n: Tuple[int, int, int], centre, radius: float) -> np.ndarray:
    """Voxels whose (y, z) centre lies within radius of centre (every x): a source line
    through an x-periodic plate."""
    n1, n2, n3 = n
    y = np.arange(n2) + 0.5
    z = np.arange(n3) + 0.5
    disc = ((y[None, :] - centre[0]) ** 2 + (z[:, None] - centre[1]) ** 2) <= radius * radius  # (n3, n2)
    full = np.broadcast_to(disc[:, :, None], (n3, n2, n1))
    return np.flatnonzero(full.ravel()).astype(np.int64)


def make_plate(n: int = 512, n1: int = 8, radius: float = 2.5, framed: bool = False, wavelength_vox: float = 32.0,
               cfl: float = 2.0, tol: float = 1e-8) -> Problem:
    """Circular waves of section 4.1.1 (homogeneous Al plate) and 4.1.2 (Al core framed by Fe,
    core side 0.39 of the plate): the plate is x-periodic and constant along x (n1 voxels, the
    paper's one-voxel thickness), the source a cylinder of the given radius through the centre
    of the (y, z) plane, prescribed along x (transverse to the plate: antiplane shear waves),
    Ricker pulse with the given wavelength at aluminium's shear speed."""
    al, fe = table1_scaled("Al"), table1_scaled("Fe")
    C = np.stack([al[0], fe[0]])
    rho = np.array([al[1], fe[1]])
    phase = np.zeros((n, n, n1), np.uint16)
    if framed:
        yz = (np.arange(n) + 0.5) / n
        core = np.abs(yz - 0.5) <= 0.39 / 2
        inside = core[:, None] & core[None, :]  # (z, y)
        phase[:] = np.where(inside, 0, 1).astype(np.uint16)[:, :, None]
    c_max = max(iso_speeds(C[g], rho[g])[0] for g in range(2))
    dt = cfl / c_max
    fc = iso_speeds(al[0], al[1])[1] / wavelength_vox
    g = gamma_cylinder_x((n1, n, n), (n / 2.0, n / 2.0), radius)
    return Problem("plate-framed" if framed else "plate", 3, (n1, n, n), (float(n1), float(n), float(n)), phase, C, rho,
                   g, dt, pulse_fc=fc, tol=tol)


def make_sphere_source(n: int = 128, radius: float = 2.0, framed: bool = False, wavelength_vox: float = 16.0,
                       cfl: float = 2.0, tol: float = 1e-8) -> Problem:
    """Spherical waves of section 4.1.3 (homogeneous Al cube) and 4.2 (Al cube of side 0.62
    framed by Fe): Gamma = the voxels within radius of the centre, displacement along x,
    Ricker pulse with the given wavelength at aluminium's shear speed."""
    al, fe = table1_scaled("Al"), table1_scaled("Fe")
    C = np.stack([al[0], fe[0]])
    rho = np.array([al[1], fe[1]])
    phase = np.zeros((n, n, n), np.uint16)
    if framed:
        c1 = np.abs((np.arange(n) + 0.5) / n - 0.5) <= 0.62 / 2
        inside = c1[:, None, None] & c1[None, :, None] & c1[None, None, :]
        phase = np.where(inside, 0, 1).astype(np.uint16)
    c_max = max(iso_speeds(C[g], rho[g])[0] for g in range(2))
    dt = cfl / c_max
    fc = iso_speeds(al[0], al[1])[1] / wavelength_vox
    g = gamma_sphere((n, n, n), (n / 2.0, n / 2.0, n / 2.0), radius)
    return Problem("sphere-framed" if framed else "sphere", 3, (n, n, n), (float(n),) * 3, phase, C, rho, g, dt,
                   pulse_fc=fc, tol=tol)


def random_field(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. N(0,1) field (operator micro-benchmark and parity input)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def random_anisotropic21(rng: np.random.Generator, n_phases: int, scale: float = 1.0) -> np.ndarray:
    """Random positive-definite 6x6 Voigt stiffnesses (general anisotropy), for tests."""
    out = []
    for _ in range(n_phases):
        A = rng.standard_normal((6, 6))
        C = A @ A.T / 6.0 + np.eye(6) * 0.5
        out.append(voigt_to21(C * scale))
    return np.stack(out)


def random_phase_map(rng: np.random.Generator, n: Tuple[int, int, int], n_phases: int) -> np.ndarray:
    n1, n2, n3 = n
    return rng.integers(0, n_phases, size=(n3, n2, n1)).astype(np.uint16)
