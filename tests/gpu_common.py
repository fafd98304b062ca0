"""Helpers shared by the GPU tests (device buffers via torch, inputs from workloads)."""
import numpy as np

from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def field3(u, dim):
    """Pad a (dim, ...) field with zero components to 3 x N."""
    u = np.asarray(u, dtype=np.float64)
    if dim == 3:
        return u.reshape(3, -1)
    out = np.zeros((3, u[0].size))
    out[:dim] = u.reshape(dim, -1)
    return out


def rel_max(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_problem(dim, n, n_phases=3, seed=0, dt=0.7, aniso=True):
    rng = np.random.default_rng(seed)
    nn = tuple(n) + (1,) * (3 - len(n))
    L = tuple(float(x) * 0.5 for x in nn)
    if aniso:
        C21 = W.random_anisotropic21(rng, n_phases)
    else:
        C21 = np.stack([W.voigt_to21(W.isotropic_voigt66(1.0 + 2 * i, 0.3)) for i in range(n_phases)])
    rho = 0.5 + rng.random(n_phases)
    phase = W.random_phase_map(rng, nn, n_phases)
    return W.Problem("rand", dim, nn, L, phase, C21, rho, np.zeros(0, np.int64), dt)
