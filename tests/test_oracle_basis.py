"""Pins for the oracle's Yee operator, twisted DFT and SVD basis (CPU only).

Each check ties the oracle to a fact other than its own formulas: unitarity,
a library FFT or SVD, the eigen-relations of Thm 2.1/2.3/2.4 and the SVD of
Thm 2.5 checked by matrix products against the explicitly built sparse C.
"""
import numpy as np
import pytest

from oracle import basis, yee

GRIDS = [(4, 4, 4), (3, 4, 5), (6, 2, 4)]
KS = [np.array([0.1, 0.2, 0.3]), np.array([0.5, 0.0, 0.0]), np.array([0.25, 0.5, 0.5])]


@pytest.mark.parametrize("grid", GRIDS)
def test_T_unitary_and_matches_library_fft(grid):
    k = KS[0]
    T = yee.T_dense(grid, k)
    n = T.shape[0]
    assert np.abs(T.conj().T @ T - np.eye(n)).max() < 1e-13
    rng = np.random.default_rng(3)
    q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    D = np.exp(2j * np.pi * sum(
        k[l] * np.indices(grid[::-1])[2 - l] / grid[l] for l in range(3))).ravel()
    # numpy's ifftn is the textbook inverse DFT (e^{+}, 1/n).
    ref = D * np.fft.ifftn(q.reshape(grid[::-1])).ravel() * np.sqrt(n)
    assert np.abs(T @ q - ref).max() < 1e-12
    for route in (yee.T_apply_fft, yee.T_apply_separable):
        assert np.abs(route(q, grid, k) - T @ q).max() < 1e-12
        assert np.abs(route(q, grid, k, adjoint=True) - T.conj().T @ q).max() < 1e-12


@pytest.mark.parametrize("m,kl", [(4, 0.1), (5, 0.5), (7, 0.0)])
def test_K_eigendecomposition(m, kl):
    """K (D U) = (D U) Lambda_{a,m} (eq. before Thm 2.1), Lambda from lambda_axis with delta=1."""
    K = yee.K_matrix(m, kl).toarray()
    DU = np.diag(yee.D_diag(m, kl)) @ yee.U_matrix(m)
    lam = yee.lambda_axis(m, kl, 1.0)
    assert np.abs(K @ DU - DU @ np.diag(lam)).max() < 1e-12


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("k", KS)
def test_C_l_diagonalised_by_T(grid, k):
    """Thm 2.1: C_l T = T Lambda_l."""
    T = yee.T_dense(grid, k)
    for C_l, L_l in zip(yee.C_parts(grid, k), yee.lambdas(grid, k)):
        assert np.abs(C_l @ T - T * L_l[None, :]).max() < 1e-11 * max(1, np.abs(L_l).max())


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("k", KS)
def test_svd_of_C(grid, k):
    """Thm 2.3-2.5: Q, P unitary, C Q0 = 0, P0^* C = 0, C = P_r Sigma_r Q_r^*, C^* = Q_r Sigma_r P_r^*."""
    b = basis.basis_dense(grid, k)
    n = b["T"].shape[0]
    C = b["C"]
    scale = np.abs(C).max()
    assert np.abs(b["Q"].conj().T @ b["Q"] - np.eye(3 * n)).max() < 1e-12
    assert np.abs(b["P"].conj().T @ b["P"] - np.eye(3 * n)).max() < 1e-12
    assert np.abs(C @ b["Q0"]).max() < 1e-12 * scale
    assert np.abs(b["P0"].conj().T @ C).max() < 1e-12 * scale
    S = np.concatenate([b["sigma"], b["sigma"]])
    assert np.abs((b["Pr"] * S[None, :]) @ b["Qr"].conj().T - C).max() < 1e-12 * scale
    assert np.abs((b["Qr"] * S[None, :]) @ b["Pr"].conj().T - C.conj().T).max() < 1e-12 * scale
    # Thm 2.4: C^*C = Q diag(Lq, Lq, 0) Q^*
    Lq = b["sigma"] ** 2
    d = np.concatenate([Lq, Lq, np.zeros(n)])
    assert np.abs((b["Q"] * d[None, :]) @ b["Q"].conj().T - C.conj().T @ C).max() < 1e-11 * scale ** 2
    assert np.abs((b["P"] * d[None, :]) @ b["P"].conj().T - C @ C.conj().T).max() < 1e-11 * scale ** 2


@pytest.mark.parametrize("grid", [(4, 4, 4), (3, 4, 5)])
def test_singular_values_match_library_svd(grid):
    """Dense LAPACK SVD of C: n zeros and each sigma_f twice."""
    k = KS[0]
    b = basis.basis_dense(grid, k)
    n = b["T"].shape[0]
    sv = np.sort(np.linalg.svd(b["C"], compute_uv=False))
    expect = np.sort(np.concatenate([np.zeros(n), b["sigma"], b["sigma"]]))
    assert np.abs(sv - expect).max() < 1e-12 * sv.max()
    assert np.sum(sv < 1e-10 * sv.max()) == n   # null-space dimension n


@pytest.mark.parametrize("alpha,beta", [(-1.0, 2.0), (2.0, -3.0)])
def test_pi_vectors_match_dense_basis(alpha, beta):
    """Per-frequency Pi's give the same Q_r, P_r as the dense construction."""
    grid, k = (3, 4, 5), KS[0]
    b = basis.basis_dense(grid, k, alpha=alpha, beta=beta)
    _, pi1, pi2, sigma = basis.pi_vectors(grid, k, alpha=alpha, beta=beta)
    I3T = np.kron(np.eye(3), b["T"])
    blk = lambda v: np.vstack([np.diag(v[c]) for c in range(3)])
    assert np.abs(I3T @ blk(pi1) - b["Q1"]).max() < 1e-12
    assert np.abs(I3T @ blk(pi2) - b["Q2"]).max() < 1e-12
    assert np.abs(I3T @ blk(-np.conj(pi2)) - b["P2"]).max() < 1e-12
    assert np.abs(I3T @ blk(np.conj(pi1)) - b["P1"]).max() < 1e-12
    assert np.abs(sigma - b["sigma"]).max() < 1e-13 * sigma.max()


@pytest.mark.parametrize("route", ["fft", "sep"])
def test_matrix_free_Pr_Qr_match_dense(route):
    grid, k = (4, 3, 5), KS[2]
    b = basis.basis_dense(grid, k)
    n = b["T"].shape[0]
    rng = np.random.default_rng(7)
    y = rng.standard_normal(2 * n) + 1j * rng.standard_normal(2 * n)
    x = rng.standard_normal(3 * n) + 1j * rng.standard_normal(3 * n)
    assert np.abs(basis.apply_Pr(y, grid, k, route=route) - b["Pr"] @ y).max() < 1e-12
    assert np.abs(basis.apply_Qr(y, grid, k, route=route) - b["Qr"] @ y).max() < 1e-12
    assert np.abs(basis.apply_PrH(x, grid, k, route=route) - b["Pr"].conj().T @ x).max() < 1e-12
    assert np.abs(basis.apply_QrH(x, grid, k, route=route) - b["Qr"].conj().T @ x).max() < 1e-12


def test_lemma_full_rank_mixed_sign_a():
    """Lemma 2.2 with alpha=-1, beta=2: Lambda_q > 0 and every Lambda_p column nonzero,
    including k on the Brillouin-zone boundary and a k with two zero components."""
    for grid in [(8, 8, 8), (16, 16, 16), (5, 6, 7)]:
        for k in (np.array([0.5, 0.0, 0.0]), np.array([0.5, 0.5, 0.5]), np.array([1e-3, 0, 0])):
            Lq, Lp = basis.lambda_q_p(grid, k, alpha=-1.0, beta=2.0)
            assert Lq.min() > 0
            assert np.sqrt((np.abs(Lp) ** 2).sum(axis=0)).min() > 1e-6 * np.sqrt(Lq).min()


def test_gamma_point_is_singular():
    """k = 0 makes Lambda_q singular (Lemma 2.2 needs k != 0)."""
    Lq, _ = basis.lambda_q_p((4, 4, 4), np.zeros(3))
    assert Lq.min() == 0.0
