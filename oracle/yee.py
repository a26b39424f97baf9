"""Yee single-curl operator, twisted DFT and the diagonal Lambda's (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Index convention: flat g = i1 + n1*i2 + n1*n2*i3 (x fastest), the Kronecker
order I_{n3} (x) I_{n2} (x) K_{a1,n1} used by C1 (Sec. 2).  A numpy array of
shape (n3, n2, n1) raveled in C order follows it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def mesh(grid, a=1.0):
    """Mesh lengths delta_l = a / n_l on the simple cubic lattice a_l = a e_l."""
    n1, n2, n3 = grid
    return a / n1, a / n2, a / n3


def bloch_phase(k_l, a=1.0):
    """exp(i 2 pi k . a_l) for a_l = a e_l (the wrap entry of K, Sec. 2)."""
    return np.exp(2j * np.pi * k_l * a)


def K_matrix(m, k_l, a=1.0):
    """K_{a,m}: -1 on the diagonal, +1 above it, exp(i2pi k.a) in the corner.

    Forward difference with the Bloch wrap x_m := exp(i2pi k.a) x_0 (Sec. 2,
    definition of K_{a,m}).
    """
    K = sp.lil_matrix((m, m), dtype=np.complex128)
    for j in range(m):
        K[j, j] = -1.0
        if j + 1 < m:
            K[j, j + 1] = 1.0
    K[m - 1, 0] += bloch_phase(k_l, a)
    return K.tocsr()


def C_parts(grid, k, a=1.0):
    """C1, C2, C3 as Kronecker products (Sec. 2, equations for C_l)."""
    n1, n2, n3 = grid
    dx, dy, dz = mesh(grid, a)
    I1, I2, I3 = (sp.identity(m, dtype=np.complex128, format="csr") for m in (n1, n2, n3))
    C1 = sp.kron(I3, sp.kron(I2, K_matrix(n1, k[0], a))) / dx
    C2 = sp.kron(I3, sp.kron(K_matrix(n2, k[1], a), I1)) / dy
    C3 = sp.kron(K_matrix(n3, k[2], a), sp.kron(I2, I1)) / dz
    return C1.tocsr(), C2.tocsr(), C3.tocsr()


def C_matrix(grid, k, a=1.0):
    """The 3n x 3n discrete single curl C = [[0,-C3,C2],[C3,0,-C1],[-C2,C1,0]] (Sec. 2)."""
    C1, C2, C3 = C_parts(grid, k, a)
    return sp.bmat([[None, -C3, C2], [C3, None, -C1], [-C2, C1, None]], format="csr")


def D_diag(m, k_l, a=1.0):
    """Diagonal of D_{a,m} = diag(1, e^{theta}, ..., e^{(m-1) theta}), theta = i2pi k.a/m."""
    return np.exp(2j * np.pi * k_l * a * np.arange(m) / m)


def U_matrix(m):
    """U_m = [u_{m,0} ... u_{m,m-1}], (u_{m,i})_j = exp(i 2 pi i j / m)."""
    j = np.arange(m)
    return np.exp(2j * np.pi * np.outer(j, j) / m)


def lambda_axis(m, k_l, delta, a=1.0):
    """Diagonal of Lambda_{a,m} / delta: (exp(i2pi (i + k.a)/m) - 1)/delta, i = 0..m-1.

    Eigenvalues of K_{a,m} scaled by the mesh (eq. K(DU) = (DU) Lambda and
    Thm 2.1).
    """
    i = np.arange(m)
    return (np.exp(2j * np.pi * (i + k_l * a) / m) - 1.0) / delta


def lambdas(grid, k, a=1.0):
    """Per-frequency diagonals of Lambda_1, Lambda_2, Lambda_3 (Thm 2.1), each of length n.

    Lambda_1 = delta_x^{-1} (I (x) I (x) Lambda_{a1,n1}) etc., so at frequency
    f = (i1, i2, i3) the entries are lambda_1(i1), lambda_2(i2), lambda_3(i3).
    """
    n1, n2, n3 = grid
    dx, dy, dz = mesh(grid, a)
    l1 = lambda_axis(n1, k[0], dx, a)
    l2 = lambda_axis(n2, k[1], dy, a)
    l3 = lambda_axis(n3, k[2], dz, a)
    L1 = np.kron(np.ones(n3), np.kron(np.ones(n2), l1))
    L2 = np.kron(np.ones(n3), np.kron(l2, np.ones(n1)))
    L3 = np.kron(l3, np.kron(np.ones(n2), np.ones(n1)))
    return L1, L2, L3


def T_dense(grid, k, a=1.0):
    """T = n^{-1/2} (D3 (x) D2 (x) D1)(U3 (x) U2 (x) U1) as a dense n x n matrix (Sec. 2)."""
    n1, n2, n3 = grid
    n = n1 * n2 * n3
    D = np.kron(D_diag(n3, k[2], a), np.kron(D_diag(n2, k[1], a), D_diag(n1, k[0], a)))
    U = np.kron(U_matrix(n3), np.kron(U_matrix(n2), U_matrix(n1)))
    return (D[:, None] * U) / np.sqrt(n)


def twist(grid, k, a=1.0):
    """Diagonal of D3 (x) D2 (x) D1 as a flat length-n array."""
    n1, n2, n3 = grid
    return np.kron(D_diag(n3, k[2], a), np.kron(D_diag(n2, k[1], a), D_diag(n1, k[0], a)))


# --- T applied without forming it -------------------------------------------------
# Two routes that must agree: separable dense 1-D DFT factors (the Kronecker
# structure of T, applied axis by axis) and numpy's FFT (T q = D * sqrt(n) *
# ifftn(q); T^* p = fftn(conj(D) * p) / sqrt(n), the fftn/ifftn use stated in
# Sec. 5).

def _apply_axis(mat, arr, axis):
    return np.moveaxis(np.tensordot(mat, np.moveaxis(arr, axis, 0), axes=(1, 0)), 0, axis)


def T_apply_separable(q, grid, k, a=1.0, adjoint=False):
    """T q (or T^* q) for q of length n, applying U_l along each axis."""
    n1, n2, n3 = grid
    n = n1 * n2 * n3
    D = twist(grid, k, a)
    x = np.asarray(q, dtype=np.complex128).reshape(n3, n2, n1)
    if not adjoint:
        for m, axis in ((n1, 2), (n2, 1), (n3, 0)):
            x = _apply_axis(U_matrix(m), x, axis)
        return D * x.reshape(n) / np.sqrt(n)
    x = (np.conj(D) * x.reshape(n)).reshape(n3, n2, n1)
    for m, axis in ((n1, 2), (n2, 1), (n3, 0)):
        x = _apply_axis(np.conj(U_matrix(m)).T, x, axis)
    return x.reshape(n) / np.sqrt(n)


def T_apply_fft(q, grid, k, a=1.0, adjoint=False):
    """T q = D * sqrt(n) * ifftn(q);  T^* p = fftn(conj(D) p)/sqrt(n)."""
    n1, n2, n3 = grid
    n = n1 * n2 * n3
    D = twist(grid, k, a)
    if not adjoint:
        x = np.fft.ifftn(np.asarray(q, dtype=np.complex128).reshape(n3, n2, n1))
        return D * x.reshape(n) * np.sqrt(n)
    x = np.fft.fftn((np.conj(D) * np.asarray(q, dtype=np.complex128)).reshape(n3, n2, n1))
    return x.reshape(n) / np.sqrt(n)
