"""nm_conv3d_bf16_noalloc (device buffers from the library's file-scope scratch array)
against nm_conv3d_bf16 (buffers allocated per call), two calls in a row, the second on a
smaller grid (the scratch keeps the first call's contents; a stale bias or partial sum
would show).  Forward and backward-data results must be identical; the weight gradient
groups its FP32 partial sums differently above 256 tiles of 16 voxels (bar 1e-5 relative)
and identically below."""
import numpy as np
import pytest

from paper_2211_08263_amd import newmark as nmb

pytestmark = pytest.mark.gpu


def _bits(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


def _dev(bits):
    import torch
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).cuda()


def _case(n, cinp, cin, cout, seed, with_bias):
    import torch
    rng = np.random.default_rng(seed)
    N = n[0] * n[1] * n[2]
    x = _dev(_bits(rng.standard_normal((N, cinp))))
    dyv = np.zeros((N, 16))
    dyv[:, :cout] = rng.standard_normal((N, cout))
    dy = _dev(_bits(dyv))
    w = (rng.standard_normal((cout, cin, 27)) * 0.3).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32) if with_bias else None
    out = {}
    for noalloc in (False, True):
        o0 = torch.full((N * 16,), -1.0, dtype=torch.float32, device="cuda")
        nmb.conv3d_bf16(0, n, cinp, cin, cout, x=x, w=w, bias=b, out=o0, noalloc=noalloc)
        o1 = None
        if cinp == 16:
            o1 = torch.full((N * 16,), -1.0, dtype=torch.float32, device="cuda")
            nmb.conv3d_bf16(1, n, cinp, cin, cout, w=w, dy=dy, out=o1, noalloc=noalloc)
        dw, db = nmb.conv3d_bf16(2, n, cinp, cin, cout, x=x, dy=dy, noalloc=noalloc)
        torch.cuda.synchronize()
        out[noalloc] = (o0.cpu().numpy(), None if o1 is None else o1.cpu().numpy(), dw, db)
    a, z = out[False], out[True]
    assert np.array_equal(a[0], z[0]), "forward differs"
    if cinp == 16:
        assert np.array_equal(a[1], z[1]), "backward-data differs"
    ew = float(np.abs(a[2] - z[2]).max() / np.abs(a[2]).max())
    eb = float(np.abs(a[3] - z[3]).max() / np.abs(a[3]).max())
    print(f"no-alloc n={n} cinp={cinp}: forward/backward-data identical, weight grad {ew:.2e} bias {eb:.2e}",
          flush=True)
    if N // 16 <= 256:
        assert ew == 0.0 and eb == 0.0
    assert ew <= 1e-5 and eb <= 1e-5


@pytest.mark.parametrize("cinp,cin,cout", [(32, 31, 16), (16, 16, 3)])
def test_noalloc_conv_matches_the_allocating_entry(cinp, cin, cout):
    # first a grid whose weight gradient uses more partial-sum slots than the scratch
    # holds, then a smaller one without a bias (the first call's bias is still there)
    _case((32, 16, 32), cinp, cin, cout, seed=1, with_bias=True)
    _case((16, 8, 16), cinp, cin, cout, seed=2, with_bias=False)


def test_noalloc_rejects_bad_arguments():
    with pytest.raises(nmb.NewmarkError):
        nmb.conv3d_bf16(0, (16, 8, 8), 24, 16, 16, noalloc=True)
    with pytest.raises(nmb.NewmarkError):
        nmb.conv3d_bf16(3, (16, 8, 8), 16, 16, 16, noalloc=True)
