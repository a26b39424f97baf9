"""Seeded input generators: geometry pins (no device needed)."""
import numpy as np

from paper_1402_6297_amd import media


def test_spheres_cylinders_geometry():
    r, s = 0.345, 0.11
    eps, gam = media.spheres_cylinders_chiral(128, radius=r, cyl_radius=s, eps_in=13.0, gamma=0.5)
    inside = eps > 1.0
    # sphere plus the three cylinders outside it: a cylinder leaves the sphere
    # completely at |x| = h = sqrt(r^2 - s^2), and for h < |x| < r the sphere covers
    # the disc of radius sqrt(r^2 - x^2) of its cross-section (the cylinders' mutual
    # overlaps lie within s sqrt(2) < r of the lattice point, inside the sphere)
    h = np.sqrt(r * r - s * s)
    cap = 6 * np.pi * (2 * r ** 3 / 3 - r * r * h + h ** 3 / 3)
    v = 4.0 / 3.0 * np.pi * r ** 3 + 3 * np.pi * s * s * (1.0 - 2.0 * h) - cap
    assert abs(inside.mean() - v) < 0.01 * v
    # the structure is symmetric under permutations and reflections of the axes
    assert np.array_equal(inside, np.transpose(inside, (1, 0, 2)))
    assert np.array_equal(inside, np.transpose(inside, (2, 1, 0)))
    assert np.array_equal(inside, inside[::-1, ::-1, ::-1])
    # voxel next to the lattice point (corner) is inside; the cell centre is outside;
    # the middle of an x-directed cylinder is inside, off-axis points near it are not
    assert inside[0, 0, 0] and not inside[64, 64, 64]
    assert inside[0, 0, 64] and not inside[20, 20, 64]
    assert np.all(gam[inside] == 0.5) and np.all(gam[~inside] == 0.0)


def test_random_general_is_hermitian_positive():
    eps, mu, xi, zeta = media.random_general(4, seed=3)
    adj = lambda t: np.conj(np.transpose(t, (0, 2, 1)))
    assert np.abs(eps - adj(eps)).max() == 0 and np.abs(mu - adj(mu)).max() == 0
    assert np.array_equal(zeta, adj(xi))
    assert np.linalg.eigvalsh(mu).min() >= 0.6 - 1e-12
    phi = eps - xi @ np.linalg.inv(mu) @ zeta
    assert np.linalg.eigvalsh(0.5 * (phi + adj(phi))).min() > 0.3


def test_band_path_gxmrg():
    ks = media.kpath_gxmrg(10)
    assert ks.shape == (40, 3)
    assert np.all(np.linalg.norm(ks, axis=1) > 0)  # Gamma never sampled
    assert np.allclose(ks[0], [0.025, 0, 0]) and np.allclose(ks[10], [0.5, 0.025, 0])
    assert np.allclose(ks[20], [0.5, 0.5, 0.025]) and np.allclose(ks[39], [0.025, 0.025, 0.025])
    assert np.all((ks >= 0) & (ks <= 0.5))
