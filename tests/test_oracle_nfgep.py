"""Pins for the oracle's pencil, GEP and solvers (CPU only).

The checks use facts the oracle's formulas do not restate: Hermitian
definiteness, the GEP's null-space dimension, closed forms for air and for a
homogeneous chiral medium (derived per frequency, not via A_r), the gamma = 0
reduction to a Hermitian-definite problem solved by LAPACK, conjugation
symmetry, independence of alpha/beta, and three independent eigenvalue routes
(dense QZ on the 6n GEP, dense eigh on the 4n pencil, ARPACK on the pencil,
sparse shift-invert on the GEP without any FFT).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis, medium, nfgep, yee
from paper_1402_6297_amd import media

K0 = np.array([0.1, 0.2, 0.3])


def _sphere(n, **kw):
    eps, gam = media.sphere_chiral(n, **kw)
    return medium.tensors_chiral(eps, gam)


def _homog_closed_form(grid, k, eps0, g0):
    """Four nonzero omega per frequency for a homogeneous chiral medium.

    Per frequency C acts as the cross product with lambda; eliminating H from
    the 6x6 pencil gives [M^*M - gamma omega (M + M^*) - Phi omega^2] e = 0,
    whose nonzero roots are
      omega^2 = [eps s2 - g^2 Re c +- g sqrt(eps (s2 - Re c)^2 + Phi (Im c)^2)] / Phi^2
    with s2 = sum |lambda_l|^2, c = sum lambda_l^2, Phi = eps - g^2.
    """
    L1, L2, L3 = yee.lambdas(grid, k)
    s2 = np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2
    c = L1 ** 2 + L2 ** 2 + L3 ** 2
    Phi = eps0 - g0 ** 2
    disc = np.sqrt(eps0 * (s2 - c.real) ** 2 + Phi * c.imag ** 2)
    w2 = np.concatenate([(eps0 * s2 - g0 ** 2 * c.real + g0 * disc),
                         (eps0 * s2 - g0 ** 2 * c.real - g0 * disc)]) / Phi ** 2
    return np.sort(np.sqrt(w2))


def test_Ar_hermitian_positive_definite_and_matrix_free():
    grid = (4, 4, 4)
    t = _sphere(4)
    A = nfgep.Ar_dense(grid, K0, t)
    assert np.abs(A - A.conj().T).max() < 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0
    rng = np.random.default_rng(1)
    u = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    for route in ("fft", "sep"):
        assert np.abs(nfgep.apply_Ar(u, grid, K0, t, route=route) - A @ u).max() < 1e-12 * np.abs(A @ u).max()


def test_Ar_matrix_free_pseudochiral_odd_grid():
    grid = (3, 4, 5)
    eps, gam = media.rods_pseudochiral(3, 4, 5, radius=0.3)
    for pair in ((0, 1), (0, 2), (1, 2)):
        t = medium.tensors_pseudochiral(eps, gam, pair)
        A = nfgep.Ar_dense(grid, K0, t)
        assert np.linalg.eigvalsh(A).min() > 0
        u = np.random.default_rng(2).standard_normal(A.shape[0]) + 0j
        assert np.abs(nfgep.apply_Ar(u, grid, K0, t) - A @ u).max() < 1e-12 * np.abs(A @ u).max()


def test_air_Ar_is_identity_and_spectrum_is_sigma():
    """eps = mu = 1, xi = zeta = 0: A_r = I and omega = +-sigma_f, each twice (Sec. 5,
    second validation problem)."""
    grid = (4, 4, 4)
    eps, gam = media.homogeneous(4, eps=1.0, gamma=0.0)
    t = medium.tensors_chiral(eps, gam)
    A = nfgep.Ar_dense(grid, K0, t)
    assert np.abs(A - np.eye(A.shape[0])).max() < 1e-13
    w = nfgep.gep_dense(grid, K0, t)
    sigma = np.sqrt(sum(np.abs(L) ** 2 for L in yee.lambdas(grid, K0)))
    pos = np.sort(w.real[w.real > 1e-8])
    neg = np.sort(-w.real[w.real < -1e-8])
    expect = np.sort(np.concatenate([sigma, sigma]))
    assert np.abs(pos - expect).max() < 1e-12 * expect.max()
    assert np.abs(neg - expect).max() < 1e-12 * expect.max()


@pytest.mark.parametrize("eps0,g0", [(13.0, 0.5), (1.0, 0.8), (4.0, 1.9)])
def test_homogeneous_chiral_closed_form(eps0, g0):
    grid = (4, 4, 4)
    eps, gam = media.homogeneous(4, eps=eps0, gamma=g0)
    t = medium.tensors_chiral(eps, gam)
    cf = _homog_closed_form(grid, K0, eps0, g0)
    w = nfgep.gep_dense(grid, K0, t)
    pos = np.sort(w.real[w.real > 1e-8])
    assert np.abs(pos - cf).max() < 1e-12 * cf.max()
    wn = nfgep.nfgep_dense(grid, K0, t)
    assert np.abs(np.sort(wn[wn > 0]) - cf).max() < 1e-12 * cf.max()


def test_gep_null_space_real_spectrum_and_nfgep_equivalence():
    """Sec. 3: 2n zero eigenvalues; Thm 4.1: all real; Thm 3.2/4.2: the 4n nonzero ones
    are the pencil's."""
    grid = (4, 4, 4)
    n = 64
    t = _sphere(4)
    w = nfgep.gep_dense(grid, K0, t)
    mag = np.sort(np.abs(w))
    assert mag[2 * n - 1] < 1e-10 * mag.max() and mag[2 * n] > 1e-3 * mag.max()
    nz = w[np.abs(w) > 1e-8 * mag.max()]
    assert np.abs(nz.imag).max() < 1e-10 * mag.max()
    wn = np.sort(nfgep.nfgep_dense(grid, K0, t))
    assert wn.size == 4 * n
    assert np.abs(np.sort(nz.real) - wn).max() < 1e-11 * mag.max()


def test_gamma_zero_reduces_to_eps_eigenproblem():
    """gamma = 0: omega^2 are the nonzero eigenvalues of C^*C e = omega^2 eps_d e (Sec. 5)."""
    grid = (4, 4, 4)
    eps, _ = media.sphere_chiral(4, gamma_in=0.0)
    t = medium.tensors_chiral(eps, np.zeros_like(eps))
    C = yee.C_matrix(grid, K0).toarray()
    epsd = np.diag(np.tile(eps.ravel(), 3))
    w2 = sla.eigh(C.conj().T @ C, epsd, eigvals_only=True)
    w2 = np.sort(w2[w2 > 1e-8 * w2.max()])
    w = nfgep.nfgep_dense(grid, K0, t)
    pos = np.sort(w[w > 0])
    assert np.abs(pos ** 2 - w2).max() < 1e-11 * w2.max()


def test_conjugation_symmetry():
    """conj(C(k)) = C(1-k) and conj(B_gamma) = -B_{-gamma}: spec(k, g) = -spec(1-k, -g)."""
    grid = (4, 4, 4)
    eps, gam = media.sphere_chiral(4)
    w1 = nfgep.gep_dense(grid, K0, medium.tensors_chiral(eps, gam))
    w2 = nfgep.gep_dense(grid, 1.0 - K0, medium.tensors_chiral(eps, -gam))
    pos1 = np.sort(w1.real[w1.real > 1e-8])
    neg2 = np.sort(-w2.real[w2.real < -1e-8])
    assert np.abs(pos1 - neg2).max() < 1e-11 * pos1.max()


def test_alpha_beta_invariance():
    grid = (4, 4, 4)
    t = _sphere(4)
    w1 = np.sort(nfgep.nfgep_dense(grid, K0, t, alpha=-1.0, beta=2.0))
    w2 = np.sort(nfgep.nfgep_dense(grid, K0, t, alpha=2.0, beta=-3.0))
    assert np.abs(w1 - w2).max() < 1e-11 * np.abs(w1).max()


def test_cg_solves_and_air_in_one_iteration():
    grid = (4, 4, 4)
    t = _sphere(4)
    A = nfgep.Ar_dense(grid, K0, t)
    b = media.random_vector(A.shape[0], 5)
    x, it, rel = nfgep.cg(lambda v: A @ v, b, rtol=1e-12)
    assert rel <= 1e-12
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-10 * np.abs(x).max()
    x, it, rel = nfgep.cg(lambda v: v, b, rtol=1e-12)
    assert it == 1 and rel == 0.0


def test_eigsh_and_shift_invert_routes_match_dense():
    grid = (4, 4, 4)
    t = _sphere(4)
    ref = nfgep.positive_smallest(nfgep.gep_dense(grid, K0, t), 6, 1e-8)
    w_si = nfgep.gep_shift_invert(grid, K0, t, nev=6)
    assert np.abs(w_si - ref).max() < 1e-11 * ref.max()
    w_l, Y = nfgep.nfgep_eigsh(grid, K0, t, nev=6, cg_rtol=1e-13)
    assert np.abs(np.sort(w_l) - ref).max() < 1e-10 * ref.max()
    for j in range(3):
        eta = nfgep.pencil_residual(Y[:, j], 1.0 / w_l[j], grid, K0, t)
        assert eta < 1e-8
        assert abs(nfgep.rayleigh_omega(Y[:, j], grid, K0, t) - w_l[j]) < 1e-12 * w_l[j]
