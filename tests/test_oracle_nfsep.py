"""Pins for the oracle's NFSEP (CPU only).

The checks use facts the NFSEP formulas do not restate: the nonzero spectrum
of the plain 6n GEP (dense QZ on diag(C, C^*) x = omega B x, built from the
Kronecker form of C and no SVD basis), the closed form of a homogeneous lossy
dielectric, the reduction to the pinned HHPD pencil when the assumption holds,
LAPACK solves for GMRES, and dense eigenvectors for the residual.
"""
import numpy as np
import pytest

from oracle import basis, medium, nfgep, nfsep, yee
from paper_1402_6297_amd import media

K0 = (0.1, 0.2, 0.3)


def _tens(t):
    eps, mu, xi, zeta = t
    return dict(eps=eps, mu=mu, xi=xi, zeta=zeta)


def match(a, b):
    """Greedy nearest matching of two complex spectra; max relative distance."""
    b = list(np.asarray(b))
    worst = 0.0
    for x in np.asarray(a):
        j = int(np.argmin([abs(x - y) for y in b]))
        worst = max(worst, abs(x - b[j]) / max(abs(x), 1e-300))
        b.pop(j)
    return worst


@pytest.mark.parametrize("grid", [(4, 4, 4), (3, 4, 5)])
@pytest.mark.parametrize("which", ["random", "lossy"])
def test_nonzero_spectrum_equals_gep(grid, which):
    """Thm 3.2: K carries exactly the 4n nonzero eigenvalues of the 6n GEP, and
    the GEP's other 2n eigenvalues are zero; the medium is outside the HHPD
    assumption."""
    t = _tens(media.random_nonhhpd(*grid, seed=3) if which == "random"
              else media.lossy_sphere_tensors(*grid, radius=0.4))
    assert not medium.check_assumption(t)
    n = grid[0] * grid[1] * grid[2]
    gep = nfgep.gep_dense(grid, K0, t)
    gep = gep[np.isfinite(gep)]
    scale = np.abs(gep).max()
    zeros = gep[np.abs(gep) <= 1e-9 * scale]
    nonzero = gep[np.abs(gep) > 1e-9 * scale]
    assert len(zeros) == 2 * n and len(nonzero) == 4 * n
    w = nfsep.eigs_dense(grid, K0, t)
    assert np.abs(w).min() > 1e-6 * scale        # no zero eigenvalue left
    assert match(w, nonzero) < 1e-9
    if which == "lossy":
        assert np.abs(w.imag).max() > 1e-3 * scale  # genuinely complex spectrum


def test_homogeneous_lossy_dielectric_closed_form():
    """xi = zeta = 0, mu = 1, constant complex eps: per frequency the curl-curl
    relation gives omega^2 = sigma^2 / eps, sigma^2 = sum_l |lambda_l|^2, so K
    has +-sigma/sqrt(eps), each twice."""
    grid, eps0 = (4, 3, 5), 9.0 + 1.5j
    t = _tens(media.homogeneous_tensors(*grid, eps=eps0))
    L1, L2, L3 = yee.lambdas(grid, K0)
    s = np.sqrt(np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2)
    w0 = s / np.sqrt(eps0)
    ref = np.concatenate([w0, w0, -w0, -w0])
    assert match(nfsep.eigs_dense(grid, K0, t), ref) < 1e-10
    sel = nfsep.smallest_positive(ref, 6)
    assert np.all(sel.real > 0) and np.all(np.diff(np.abs(sel)) >= 0)
    assert np.abs(np.abs(sel) - np.sort(np.abs(np.concatenate([w0, w0])))[:6]).max() < 1e-12


def test_hhpd_medium_reduces_to_pencil():
    """Under the assumption, K's eigenvalues are the omega of the pinned HHPD
    pencil B_r y = omega^{-1} A_r y (Thm 3.2 against Thm 4.2): real, same set."""
    grid = (4, 4, 4)
    t = _tens(media.random_general(*grid, seed=5))
    assert medium.check_assumption(t)
    w = nfsep.eigs_dense(grid, K0, t)
    ref = nfgep.nfgep_dense(grid, K0, t)
    assert np.abs(w.imag).max() < 1e-9 * np.abs(w).max()
    assert match(w, ref) < 1e-10


@pytest.mark.parametrize("grid", [(4, 4, 4), (3, 4, 5)])
def test_matrix_free_K_equals_dense(grid):
    t = _tens(media.random_nonhhpd(*grid, seed=7))
    n = grid[0] * grid[1] * grid[2]
    y = media.random_vector(4 * n, seed=2)
    ref = nfsep.K_dense(grid, K0, t) @ y
    for route in ("fft", "separable"):
        out = nfsep.apply_K(y, grid, K0, t, route=route)
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_gmres_solves_K():
    grid = (4, 4, 4)
    t = _tens(media.random_nonhhpd(*grid, seed=1))
    n = grid[0] * grid[1] * grid[2]
    b = media.random_vector(4 * n, seed=4)
    Kd = nfsep.K_dense(grid, K0, t)
    x, it, res = nfsep.gmres(lambda v: nfsep.apply_K(v, grid, K0, t), b, rtol=1e-12)
    ref = np.linalg.solve(Kd, b)
    assert res <= 1e-12 and it <= 4 * n
    assert np.linalg.norm(Kd @ x - b) <= 2e-12 * np.linalg.norm(b)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


def test_shift_invert_arnoldi_matches_dense_4():
    grid = (4, 4, 4)
    t = _tens(media.lossy_sphere_tensors(*grid, radius=0.4))
    ref = nfsep.smallest_positive(nfsep.eigs_dense(grid, K0, t), 4)
    w = nfsep.si_arnoldi(grid, K0, t, nev=4)
    assert np.abs(w - ref).max() <= 1e-9 * np.abs(ref).max()


def test_residual_and_rayleigh_of_dense_eigenvector():
    """For an eigenpair (omega, y) of the dense K and z = Sigma^{1/2} y, the
    residual is at rounding level and the Rayleigh quotient returns omega; a
    perturbed omega gives the residual |d omega| / |omega|."""
    grid = (4, 4, 4)
    t = _tens(media.random_nonhhpd(*grid, seed=2))
    w, Y = np.linalg.eig(nfsep.K_dense(grid, K0, t))
    j = int(np.argmin(np.where(w.real > 0, np.abs(w), np.inf)))
    sh = np.sqrt(nfgep.sigma_r(grid, K0))
    z = np.concatenate([sh, sh]) * Y[:, j]
    assert nfsep.residual(z, w[j], grid, K0, t) < 1e-12
    assert abs(nfsep.rayleigh(z, grid, K0, t) - w[j]) < 1e-12 * abs(w[j])
    d = 1e-6 * abs(w[j])
    assert abs(nfsep.residual(z, w[j] + d, grid, K0, t) - 1e-6) < 1e-9


@pytest.mark.parametrize("grid", [(4, 4, 4), (6, 6, 6)])
def test_sparse_gep_shift_invert_matches_dense(grid):
    """The FFT-free route on the 6n GEP (the independent reference at 16^3)."""
    t = _tens(media.lossy_sphere_tensors(*grid, radius=0.4))
    ref = nfsep.smallest_positive(nfsep.eigs_dense(grid, K0, t), 5)
    w = nfsep.gep_shift_invert(grid, K0, t, nev=5)
    assert np.abs(w - ref).max() <= 1e-10 * np.abs(ref).max()
