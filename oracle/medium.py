"""Material matrices eps_d, mu_d, xi_d, zeta_d of the discrete GEP (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A medium is given per voxel as four 3x3 complex tensors (arrays of shape
(n, 3, 3)).  The 3n x 3n matrices use the component-major block layout of the
paper: entry (c*n + g, c'*n + g) holds tensor[g, c, c'] (Sec. 3; Sec. 4.3
writes xi_d for pseudochiral media in exactly this 3x3-of-diagonal-blocks form).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def tensors_chiral(eps, gamma, mu=None):
    """Chiral (Pasteur) medium: eps I_3, mu I_3, xi = i gamma I_3, zeta = -i gamma I_3 (Sec. 4.3)."""
    eps = np.asarray(eps, dtype=np.float64).ravel()
    gamma = np.asarray(gamma, dtype=np.float64).ravel()
    n = eps.size
    I = np.eye(3)[None, :, :]
    mu_v = np.ones(n) if mu is None else np.asarray(mu, dtype=np.float64).ravel()
    return dict(eps=eps[:, None, None] * I + 0j,
                mu=mu_v[:, None, None] * I + 0j,
                xi=1j * gamma[:, None, None] * I,
                zeta=-1j * gamma[:, None, None] * I)


def tensors_pseudochiral(eps, gamma, pair=(0, 1)):
    """Pseudochiral medium: xi = i gamma (e_a e_b^T + e_b e_a^T), zeta = xi^* (Sec. 4.3).

    The paper's example couples x and z, pair=(0, 2); the 128^3 rod workload
    couples x and y, pair=(0, 1).  Pinned by the block matrices Sec. 4.3 prints,
    its diagonal Phi (eps - gamma^2 on the coupled axes, eps on the third) and a
    per-frequency GEP of the homogeneous medium (tests/test_oracle_pseudochiral.py).
    """
    eps = np.asarray(eps, dtype=np.float64).ravel()
    gamma = np.asarray(gamma, dtype=np.float64).ravel()
    n = eps.size
    ia, ib = pair
    S = np.zeros((3, 3))
    S[ia, ib] = S[ib, ia] = 1.0
    I = np.eye(3)[None, :, :]
    return dict(eps=eps[:, None, None] * I + 0j,
                mu=np.ones(n)[:, None, None] * I + 0j,
                xi=1j * gamma[:, None, None] * S[None],
                zeta=-1j * gamma[:, None, None] * S[None])


def block_matrix(t):
    """(n,3,3) tensor field -> sparse 3n x 3n matrix with diagonal n x n blocks."""
    n = t.shape[0]
    rows = [[sp.diags(t[:, c, cp]) for cp in range(3)] for c in range(3)]
    return sp.bmat(rows, format="csr").astype(np.complex128)


def material_matrices(tens):
    """eps_d, mu_d, xi_d, zeta_d as sparse 3n x 3n matrices."""
    return {key: block_matrix(tens[key]) for key in ("eps", "mu", "xi", "zeta")}


def B_matrix(tens):
    """B = i [[zeta_d, mu_d], [-eps_d, -xi_d]] (Sec. 3, eq. for B)."""
    m = material_matrices(tens)
    return (1j * sp.bmat([[m["zeta"], m["mu"]], [-m["eps"], -m["xi"]]])).tocsr()


def voxel_blocks(tens):
    """Per-voxel 3x3 blocks of mu^{-1}, Phi = eps - xi mu^{-1} zeta and Phi^{-1} (Sec. 4.1)."""
    mu_inv = np.linalg.inv(tens["mu"])
    Phi = tens["eps"] - tens["xi"] @ mu_inv @ tens["zeta"]
    return mu_inv, Phi, np.linalg.inv(Phi)


def check_assumption(tens, tol=1e-12):
    """True when mu_d > 0, Phi > 0 and xi_d^* = zeta_d (the HHPD assumption, Sec. 4.1)."""
    mu_inv, Phi, _ = voxel_blocks(tens)
    herm = lambda X: np.allclose(X, np.conj(np.swapaxes(X, 1, 2)), atol=tol)
    if not (herm(tens["mu"]) and herm(Phi)):
        return False
    if not np.allclose(np.conj(np.swapaxes(tens["xi"], 1, 2)), tens["zeta"], atol=tol):
        return False
    return bool(np.all(np.linalg.eigvalsh(tens["mu"]) > 0) and
                np.all(np.linalg.eigvalsh(0.5 * (Phi + np.conj(np.swapaxes(Phi, 1, 2)))) > 0))
