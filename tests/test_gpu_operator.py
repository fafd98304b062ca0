"""GPU parity of the operator A and the preconditioner M against the FP64 oracle.

Sizes span several blocks and a partial last block of x lines; the inputs are
i.i.d. normal fields (every frequency bin including the Nyquist ones).  The
last six grids hold 2^20 voxels, so the spectra use the padded component
stride of the large grids, and each puts a 256- or 512-long axis in x, y and z
in turn: every axis length the benchmark grids compile to is compared with the
oracle element by element.
Bars: FP64 max relative error <= 1e-12, FP32 <= 1e-5 (relative to the
largest output entry)."""
import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

from gpu_common import dev, field3, random_problem, rel_max

pytestmark = pytest.mark.gpu

# the last two grids give the column passes full tiles of kx columns (the launch shape of
# the large grids): (128, 16, 64) the z passes and the preconditioner z pass, (128, 64, 16)
# the y passes; the others have fewer kx columns than one tile
CASES = [(3, (16, 8, 8)), (3, (64, 32, 16)), (3, (8, 16, 32)), (2, (64, 64)), (2, (16, 128)), (3, (32, 32, 32)),
         (3, (128, 16, 64)), (3, (128, 64, 16)),
         (3, (256, 64, 64)), (3, (64, 256, 64)), (3, (64, 64, 256)),
         (3, (512, 64, 32)), (3, (32, 512, 64)), (3, (32, 64, 512))]
IDS = [f"{d}d-" + "x".join(map(str, n)) for d, n in CASES]


def _ctx(pb):
    return nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10))


@pytest.mark.parametrize("dim,n", CASES, ids=IDS)
def test_apply_operator_matches_oracle(dim, n):
    import torch
    pb = random_problem(dim, n, seed=sum(n))
    op = oracle.OracleProblem.from_problem(pb)
    u = W.random_field(op.field_shape, seed=7)
    want = field3(op.apply(u), dim)
    with _ctx(pb) as ctx:
        for dtype, bar in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
            ud = dev(field3(u, dim), dtype)
            out = torch.empty_like(ud)
            nmb.apply_operator(ctx, ud, out)
            torch.cuda.synchronize()
            got = out.double().cpu().numpy()
            err = rel_max(got, want)
            print(f"apply dim={dim} n={n} {dtype}: rel err {err:.3e}", flush=True)
            assert err <= bar, err


@pytest.mark.parametrize("dim,n", CASES, ids=IDS)
def test_precond_matches_oracle(dim, n):
    import torch
    pb = random_problem(dim, n, seed=3 + sum(n))
    op = oracle.OracleProblem.from_problem(pb)
    r = W.random_field(op.field_shape, seed=8)
    want = field3(op.precond(r), dim)
    with _ctx(pb) as ctx:
        for dtype, bar in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
            rd = dev(field3(r, dim), dtype)
            out = torch.empty_like(rd)
            nmb.precond_apply(ctx, rd, out)
            torch.cuda.synchronize()
            err = rel_max(out.double().cpu().numpy(), want)
            print(f"precond dim={dim} n={n} {dtype}: rel err {err:.3e}", flush=True)
            assert err <= bar, err


def test_operator_properties_at_full_size():
    """At 256^3 (the benchmark grid): symmetry <v, A u> = <A v, u>, the homogeneous
    plane-wave closed form, and M A = I for a homogeneous medium."""
    import torch
    n = 256
    pb = W.make_polycrystal(n=n, n_grains=500, seed=3)
    with _ctx(pb) as ctx:
        g = torch.Generator(device="cuda").manual_seed(0)
        u = torch.randn(3 * n ** 3, device="cuda", dtype=torch.float64, generator=g)
        v = torch.randn(3 * n ** 3, device="cuda", dtype=torch.float64, generator=g)
        Au, Av = torch.empty_like(u), torch.empty_like(v)
        nmb.apply_operator(ctx, u, Au)
        nmb.apply_operator(ctx, v, Av)
        torch.cuda.synchronize()
        a, b = float(torch.dot(v, Au)), float(torch.dot(Av, u))
        assert abs(a - b) <= 1e-12 * abs(a) * 10, (a, b)
    # homogeneous anisotropic medium: closed form and exact preconditioner
    C21 = W.voigt_to21(W.rotate_voigt66(W.copper_scaled66(), W.random_rotations(np.random.default_rng(1), 1)[0]))
    hom = W.Problem("hom", 3, (n, n, n), (float(n),) * 3, np.zeros((n, n, n), np.uint16), C21[None], np.array([1.0]),
                    np.zeros(0, np.int64), 1.6)
    with _ctx(hom) as ctx:
        m = np.array([3, -5, 17])
        xi = 2 * np.pi * m / n
        z, y, x = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
        ph = torch.from_numpy(xi[0] * x + xi[1] * y + xi[2] * z).cuda()
        amp = np.array([0.3, -1.0, 0.7])
        u = torch.cat([float(c) * torch.cos(ph).reshape(-1) for c in amp]).contiguous()
        Au = torch.empty_like(u)
        nmb.apply_operator(ctx, u, Au)
        T = W._voigt66_to_tensor(W.voigt_from21(C21))
        K = np.einsum("ikjm,k,m->ij", T, xi, xi)
        Mat = 0.25 * 1.6 ** 2 * K + np.eye(3)
        want = torch.cat([float(c) * torch.cos(ph).reshape(-1) for c in Mat @ amp])
        torch.cuda.synchronize()
        err = float((Au - want).abs().max() / want.abs().max())
        assert err <= 1e-12, err
        z_ = torch.empty_like(u)
        r = torch.randn(3 * n ** 3, device="cuda", dtype=torch.float64)
        Ar = torch.empty_like(r)
        nmb.apply_operator(ctx, r, Ar)
        nmb.precond_apply(ctx, Ar, z_)
        torch.cuda.synchronize()
        err = float((z_ - r).abs().max() / r.abs().max())
        assert err <= 1e-11, err
