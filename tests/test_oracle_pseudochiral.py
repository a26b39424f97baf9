"""Pins for the oracle's pseudochiral medium (CPU only).

``oracle.medium.tensors_pseudochiral`` builds xi = i gamma (e_a e_b^T + e_b e_a^T)
and zeta = -i gamma (...) per voxel.  It is pinned here by what Sec. 4.3 states
and by routes that never form the SVD basis or A_r:

* the paper prints xi_d and zeta_d for the x-z coupling as 3x3 arrays of
  diagonal blocks (i gamma I~ at block positions (x, z) and (z, x), and
  -i gamma I~ for zeta_d); the oracle's sparse matrices must be exactly those;
* Sec. 4.3 states that Phi = eps_d - xi_d zeta_d is diagonal with entries eps_o,
  eps_i and eps_i - gamma^2: the coupled axes carry eps - gamma^2, the third eps;
* the assumption of Sec. 4.1 then holds and A_r (Thm 4.2) is Hermitian on the
  whole matrix and positive definite;
* for a homogeneous medium the GEP of Sec. 3 splits per frequency into 6x6
  pencils built from the curl's symbol (Thm 2.1) alone: the pencil's spectrum
  must be their union (this fixes the coupled axes and the sign of zeta);
* gamma = 0 gives the plain dielectric problem.

The last tests plant mistakes in copies of the tensors (zeta with the wrong sign,
the wrong axis pair) and check that the pins above reject them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import medium, nfgep, yee
from paper_1402_6297_amd import media

K0 = np.array([0.1, 0.2, 0.3])
PAIRS = ((0, 1), (0, 2), (1, 2))


def _rods(grid, radius=0.3):
    return media.rods_pseudochiral(*grid, radius=radius)


def _curl_symbol(l1, l2, l3):
    """Per-frequency 3x3 symbol of C = [[0,-C3,C2],[C3,0,-C1],[-C2,C1,0]] (C_l T = T Lambda_l)."""
    return np.array([[0, -l3, l2], [l3, 0, -l1], [-l2, l1, 0]], dtype=np.complex128)


def _per_frequency_spectrum(grid, k, eps0, g0, pair):
    """Nonzero omega of the homogeneous GEP, one 6x6 pencil per frequency.

    diag(C, C^*) x = omega i [[zeta, mu], [-eps, -xi]] x with constant tensors
    commutes with T, so each frequency f gives diag(C_f, C_f^*) x_f =
    omega i [[zeta, I], [-eps I, -xi]] x_f with the 3x3 xi, zeta of Sec. 4.3
    written out here for the coupled axes ``pair``.
    """
    a, b = pair
    xi = np.zeros((3, 3), dtype=np.complex128)
    xi[a, b] = xi[b, a] = 1j * g0
    zeta = np.zeros((3, 3), dtype=np.complex128)
    zeta[a, b] = zeta[b, a] = -1j * g0
    I3 = np.eye(3)
    Bf = 1j * np.block([[zeta, I3], [-eps0 * I3, -xi]])
    out = []
    for l1, l2, l3 in zip(*yee.lambdas(grid, k)):
        Cf = _curl_symbol(l1, l2, l3)
        Z = np.zeros((3, 3))
        w = sla.eig(np.block([[Cf, Z], [Z, Cf.conj().T]]), Bf, right=False)
        out.append(w[np.abs(w) > 1e-9 * np.abs(w).max()])
    w = np.concatenate(out)
    assert np.abs(w.imag).max() < 1e-9 * np.abs(w).max()
    return np.sort(w.real)


@pytest.mark.parametrize("pair", PAIRS)
def test_tensors_are_the_printed_block_matrices(pair):
    """Sec. 4.3: xi_d has i gamma I~ at blocks (a, b) and (b, a), zeta_d -i gamma I~ there,
    eps_d = diag(eps, eps, eps), mu_d = I; every other block is zero."""
    grid = (3, 4, 5)
    eps, gam = _rods(grid)
    n = eps.size
    m = {key: v.toarray() for key, v in medium.material_matrices(
        medium.tensors_pseudochiral(eps, gam, pair)).items()}
    Itil_g = np.diag(gam.ravel())
    Z = np.zeros((n, n))
    a, b = pair
    xi_blocks = [[Z, Z, Z], [Z, Z, Z], [Z, Z, Z]]
    xi_blocks[a][b] = xi_blocks[b][a] = 1j * Itil_g
    zeta_blocks = [[Z, Z, Z], [Z, Z, Z], [Z, Z, Z]]
    zeta_blocks[a][b] = zeta_blocks[b][a] = -1j * Itil_g
    assert np.array_equal(m["xi"], np.block(xi_blocks))
    assert np.array_equal(m["zeta"], np.block(zeta_blocks))
    E = np.diag(eps.ravel())
    assert np.array_equal(m["eps"], np.block([[E, Z, Z], [Z, E, Z], [Z, Z, E]]))
    assert np.array_equal(m["mu"], np.eye(3 * n))


@pytest.mark.parametrize("pair", PAIRS)
def test_phi_is_diagonal_with_the_stated_entries(pair):
    """Sec. 4.3: Phi = eps_d - xi_d zeta_d is diagonal, eps - gamma^2 on the coupled axes
    and eps on the third; positive for gamma < sqrt(eps_i), so the assumption holds."""
    grid = (3, 4, 5)
    eps, gam = _rods(grid)
    t = medium.tensors_pseudochiral(eps, gam, pair)
    _, Phi, _ = medium.voxel_blocks(t)
    e, g = eps.ravel(), gam.ravel()
    expect = np.zeros((e.size, 3, 3))
    o = 3 - pair[0] - pair[1]
    expect[:, pair[0], pair[0]] = e - g ** 2
    expect[:, pair[1], pair[1]] = e - g ** 2
    expect[:, o, o] = e
    assert np.abs(Phi - expect).max() < 1e-14 * e.max()
    vals = set(np.round(np.concatenate([e - g ** 2, e]), 12))
    assert vals <= {1.0, 13.0, round(13.0 - 0.4 ** 2, 12)}  # eps_o, eps_i, eps_i - gamma^2
    assert medium.check_assumption(t)


@pytest.mark.parametrize("pair", PAIRS)
def test_Ar_hermitian_on_the_full_matrix(pair):
    grid = (3, 4, 5)
    eps, gam = _rods(grid)
    A = nfgep.Ar_dense(grid, K0, medium.tensors_pseudochiral(eps, gam, pair))
    assert np.abs(A - A.conj().T).max() <= 1e-14 * np.abs(A).max()
    w = np.linalg.eigvals(A)  # general solver: no Hermitian symmetry assumed
    assert np.abs(w.imag).max() < 1e-12 * np.abs(w).max()
    assert w.real.min() > 0


@pytest.mark.parametrize("pair", PAIRS)
@pytest.mark.parametrize("eps0,g0", [(13.0, 0.4), (1.0, 0.8), (4.0, 1.9)])
def test_homogeneous_pencil_equals_per_frequency_gep(pair, eps0, g0):
    grid = (4, 4, 4)
    eps = np.full(grid[::-1], eps0)
    gam = np.full(grid[::-1], g0)
    t = medium.tensors_pseudochiral(eps, gam, pair)
    ref = _per_frequency_spectrum(grid, K0, eps0, g0, pair)
    w = np.sort(nfgep.nfgep_dense(grid, K0, t))
    assert w.size == ref.size
    assert np.abs(w - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("pair", PAIRS)
def test_rods_gep_equals_pencil(pair):
    """Sec. 3 / Thm 4.2: the plain 6n GEP and the pencil share the nonzero spectrum."""
    grid = (4, 4, 4)
    eps, gam = _rods(grid)
    t = medium.tensors_pseudochiral(eps, gam, pair)
    w = nfgep.gep_dense(grid, K0, t)
    mag = np.abs(w).max()
    nz = w[np.abs(w) > 1e-8 * mag]
    assert nz.size == 4 * eps.size
    assert np.abs(nz.imag).max() < 1e-10 * mag
    wn = np.sort(nfgep.nfgep_dense(grid, K0, t))
    assert np.abs(np.sort(nz.real) - wn).max() < 1e-11 * mag


def test_gamma_zero_is_the_dielectric_problem():
    grid = (3, 4, 5)
    eps, _ = _rods(grid)
    zero = np.zeros_like(eps)
    for pair in PAIRS:
        tp = medium.tensors_pseudochiral(eps, zero, pair)
        tc = medium.tensors_chiral(eps, zero)
        for key in ("eps", "mu", "xi", "zeta"):
            assert np.array_equal(tp[key], tc[key])
    C = yee.C_matrix(grid, K0).toarray()
    w2 = sla.eigh(C.conj().T @ C, np.diag(np.tile(eps.ravel(), 3)), eigvals_only=True)
    w2 = np.sort(w2[w2 > 1e-8 * w2.max()])
    w = nfgep.nfgep_dense(grid, K0, medium.tensors_pseudochiral(eps, zero, (0, 1)))
    assert np.abs(np.sort(w[w > 0]) ** 2 - w2).max() < 1e-11 * w2.max()


# ----------------------------------------------------------- planted mistakes

def test_planted_zeta_sign_flip_is_rejected():
    grid = (3, 4, 5)
    eps, gam = _rods(grid)
    t = medium.tensors_pseudochiral(eps, gam, (0, 1))
    bad = dict(t, zeta=-t["zeta"])  # zeta = +i gamma S
    assert not medium.check_assumption(bad)
    A = nfgep.Ar_dense(grid, K0, bad)
    assert np.abs(A - A.conj().T).max() > 1e-3 * np.abs(A).max()
    hg = (4, 4, 4)
    e, g = np.full(hg[::-1], 13.0), np.full(hg[::-1], 0.4)
    th = medium.tensors_pseudochiral(e, g, (0, 1))
    w = nfgep.gep_dense(hg, K0, dict(th, zeta=-th["zeta"]))
    w = w[np.abs(w) > 1e-8 * np.abs(w).max()]
    ref = _per_frequency_spectrum(hg, K0, 13.0, 0.4, (0, 1))
    assert w.size != ref.size or np.abs(np.sort(w.real) - ref).max() > 1e-6 * np.abs(ref).max()


def test_planted_axis_swap_is_rejected():
    grid = (4, 4, 4)
    eps0, g0 = 13.0, 0.4
    eps = np.full(grid[::-1], eps0)
    gam = np.full(grid[::-1], g0)
    ref = _per_frequency_spectrum(grid, K0, eps0, g0, (0, 2))
    w = np.sort(nfgep.nfgep_dense(grid, K0, medium.tensors_pseudochiral(eps, gam, (0, 1))))
    assert np.abs(w - ref).max() > 1e-6 * np.abs(ref).max()
    _, Phi, _ = medium.voxel_blocks(medium.tensors_pseudochiral(eps, gam, (0, 1)))
    assert abs(Phi[0, 2, 2].real - (eps0 - g0 ** 2)) > 0.1  # z is not coupled in (x, y)
