"""Host-side checks of the seeded input generators (no solver arithmetic)."""
import numpy as np

from paper_2211_08263_amd import workloads as W


def test_isotropic_and_cubic_voigt_tables():
    C = W.isotropic_voigt66(1.0, 0.3)
    lam, mu = 0.3 / (1.3 * 0.4), 1.0 / 2.6
    assert abs(C[0, 0] - (lam + 2 * mu)) < 1e-15 and abs(C[3, 3] - mu) < 1e-15
    c21 = W.voigt_to21(C)
    np.testing.assert_array_equal(W.voigt_from21(c21), C)


def test_rotation_preserves_invariants_and_rotations_are_orthonormal():
    rng = np.random.default_rng(0)
    R = W.random_rotations(rng, 20)
    np.testing.assert_allclose(np.einsum("nij,nkj->nik", R, R), np.broadcast_to(np.eye(3), R.shape), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    C0 = W.copper_scaled66()
    for r in R[:5]:
        Cr = W.rotate_voigt66(C0, r)
        np.testing.assert_allclose(Cr, Cr.T, atol=1e-14)
        # bulk-like invariants C_iijj and C_ijij are rotation invariant
        T0, Tr = W._voigt66_to_tensor(C0), W._voigt66_to_tensor(Cr)
        assert abs(np.einsum("iijj->", T0) - np.einsum("iijj->", Tr)) < 1e-12
        assert abs(np.einsum("ijij->", T0) - np.einsum("ijij->", Tr)) < 1e-12
    # identity rotation leaves the crystal unchanged
    np.testing.assert_allclose(W.rotate_voigt66(C0, np.eye(3)), C0, atol=1e-15)


def test_copper_speeds():
    C0 = W.copper_scaled66()
    # c_L[111] / c_L[100] for Cu: sqrt((C11 + 2 C12 + 4 C44) / 3 / C11)
    want = np.sqrt((168.4 + 2 * 121.4 + 4 * 75.4) / 3 / 168.4)
    assert abs(W.longitudinal_speed_max(C0, 1.0) - want) < 1e-12


def test_disc_and_gamma_sets():
    ph = W.disc_2d(64, 64, 12.0)
    assert ph.shape == (1, 64, 64) and int(ph.sum()) == 448
    g = W.gamma_x_slab((64, 64, 1), width=2)
    assert g.size == 128 and np.all(g % 64 < 2) and np.all(np.diff(g) > 0)
    s = W.gamma_sphere((512, 512, 512), (256.0, 256.0, 256.0), 6.0)
    assert s.size == 912


def test_voronoi_and_spheres_deterministic():
    a = W.voronoi_periodic((16, 16, 16), 10, np.random.default_rng(5))
    b = W.voronoi_periodic((16, 16, 16), 10, np.random.default_rng(5))
    np.testing.assert_array_equal(a, b)
    assert a.max() < 10
    ph, sph = W.rsa_spheres(32, np.random.default_rng(1), target_fraction=0.2)
    assert abs(ph.mean() - 0.2) < 0.05
    # no two spheres overlap (minimum image)
    for i in range(len(sph)):
        for j in range(i):
            d = sph[i, :3] - sph[j, :3]
            d -= 32 * np.round(d / 32)
            assert np.linalg.norm(d) >= sph[i, 3] + sph[j, 3]


def test_ricker_starts_at_rest():
    assert abs(W.ricker(0.0, 0.145)) < 1e-15
    assert abs(W.ricker(2 / 0.145, 0.145) - 1.0) < 1e-15
