"""Derivatives of eigenvalues w.r.t. per-voxel eps and gamma (oracle, tiny grids).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Route: first-order perturbation of the non-Hermitian GEP G x = omega B(p) x of
Sec. 3, with G = diag(C, C^*) fixed.  With right and left eigenvectors x, w
(G x = omega B x, w^* G = omega w^* B):

    d omega = -omega (w^* dB x) / (w^* B x).

For the chiral medium (Sec. 4.3) B = i [[zeta_d, mu_d], [-eps_d, -xi_d]] with
xi = i gamma, zeta = -i gamma, so dB/d eps_g = i [[0,0],[-E_g,0]] and
dB/d gamma_g = i [[-i E_g, 0], [0, -i E_g]] = [[E_g,0],[0,E_g]], E_g the
3n x 3n indicator of voxel g in all three components.

This route does not use A_r, P_r, Q_r or the pencil at all; it needs simple
eigenvalues.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import medium, yee


def chiral_eigs_and_grads(grid, k, eps, gamma, nev, a=1.0, zero_tol=1e-8):
    """nev smallest positive omega and their gradients (nev, n) w.r.t. eps and gamma."""
    tens = medium.tensors_chiral(eps, gamma)
    C = yee.C_matrix(grid, k, a).toarray()
    Z = np.zeros_like(C)
    G = np.block([[C, Z], [Z, C.conj().T]])
    B = medium.B_matrix(tens).toarray()
    w, VL, VR = sla.eig(G, B, left=True, right=True)
    scale = np.abs(w).max()
    idx = [i for i in np.argsort(w.real) if w[i].real > zero_tol * scale][:nev]
    n = grid[0] * grid[1] * grid[2]
    d_eps = np.zeros((nev, n))
    d_gam = np.zeros((nev, n))
    omegas = np.array([w[i].real for i in idx])
    for j, i in enumerate(idx):
        x = VR[:, i]
        wl = VL[:, i]
        denom = np.vdot(wl, B @ x)
        # w^* dB x for each voxel g, summed over the 3 components of that voxel.
        xE, xH = x[:3 * n].reshape(3, n), x[3 * n:].reshape(3, n)
        wE, wH = wl[:3 * n].reshape(3, n), wl[3 * n:].reshape(3, n)
        # d eps_g: i * [[0,0],[-E_g,0]] -> w_H^* (-i) x_E
        num_eps = (np.conj(wH) * (-1j) * xE).sum(axis=0)
        # d gamma_g: [[E_g,0],[0,E_g]] -> w_E^* x_E + w_H^* x_H
        num_gam = (np.conj(wE) * xE).sum(axis=0) + (np.conj(wH) * xH).sum(axis=0)
        d_eps[j] = (-w[i] * num_eps / denom).real
        d_gam[j] = (-w[i] * num_gam / denom).real
    return omegas, d_eps, d_gam
