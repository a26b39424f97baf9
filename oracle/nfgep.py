"""The HHPD null-space-free pencil B_r y = omega^{-1} A_r y and its solvers (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* A_r = diag(P_r^*, Q_r^*) [[mu^{-1} zeta, -I], [I, 0]] diag(Phi^{-1}, mu^{-1})
        [[xi mu^{-1}, I], [-I, 0]] diag(P_r, Q_r)         (Thm 4.2, eq. for A_r)
* B_r = i [[0, Sigma_r^{-1}], [-Sigma_r^{-1}, 0]]          (Thm 4.2)
* the discrete GEP diag(C, C^*) x = omega B x, B = i[[zeta_d, mu_d],[-eps_d, -xi_d]]
  (Sec. 3), whose nonzero eigenvalues equal those of the pencil (Thm 3.2, Thm 4.2).

The vector y in C^{4n} is [y_a; y_b; y_c; y_d] with [y_a; y_b] multiplying
P_r = [P_2, P_1] and [y_c; y_d] multiplying Q_r = [Q_1, Q_2].
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis, medium, yee


# --- dense (tiny grids) -----------------------------------------------------------

def Ar_dense(grid, k, tens, a=1.0, alpha=-1.0, beta=2.0, bas=None):
    """A_r as the literal product of its five factors (Thm 4.2)."""
    bas = basis.basis_dense(grid, k, a, alpha, beta) if bas is None else bas
    Pr, Qr = bas["Pr"], bas["Qr"]
    m = {key: val.toarray() for key, val in medium.material_matrices(tens).items()}
    n3 = Pr.shape[0]
    I = np.eye(n3)
    Z = np.zeros((n3, n3))
    mu_inv = np.linalg.inv(m["mu"])
    Phi = m["eps"] - m["xi"] @ mu_inv @ m["zeta"]
    left = np.block([[mu_inv @ m["zeta"], -I], [I, Z]])
    mid = np.block([[np.linalg.inv(Phi), Z], [Z, mu_inv]])
    right = np.block([[m["xi"] @ mu_inv, I], [-I, Z]])
    Zr = np.zeros_like(Pr)
    outer = np.block([[Pr, Zr], [Zr, Qr]])
    return outer.conj().T @ left @ mid @ right @ outer


def sigma_r(grid, k, a=1.0):
    """Diagonal of Sigma_r = diag(Lambda_q^{1/2}, Lambda_q^{1/2}) (Thm 2.5), length 2n."""
    L1, L2, L3 = yee.lambdas(grid, k, a)
    s = np.sqrt((np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2))
    return np.concatenate([s, s])


def Br_dense(grid, k, a=1.0):
    """B_r = i [[0, Sigma_r^{-1}], [-Sigma_r^{-1}, 0]] (Thm 4.2)."""
    s = sigma_r(grid, k, a)
    Si = np.diag(1.0 / s)
    Z = np.zeros_like(Si)
    return 1j * np.block([[Z, Si], [-Si, Z]])


def gep_dense(grid, k, tens, a=1.0):
    """All 6n eigenvalues of diag(C, C^*) x = omega B x by dense QZ (Sec. 3)."""
    C = yee.C_matrix(grid, k, a).toarray()
    Z = np.zeros_like(C)
    G = np.block([[C, Z], [Z, C.conj().T]])
    B = medium.B_matrix(tens).toarray()
    return sla.eig(G, B, right=False)


def positive_smallest(omegas, nev, zero_tol):
    """nev smallest eigenvalues with real part above zero_tol (real parts, ascending)."""
    w = np.real(np.asarray(omegas))
    w = np.sort(w[w > zero_tol])
    return w[:nev]


def nfgep_dense(grid, k, tens, a=1.0, alpha=-1.0, beta=2.0):
    """All 4n eigenvalues omega = 1/theta of B_r y = theta A_r y (dense, Hermitian-definite)."""
    A = Ar_dense(grid, k, tens, a, alpha, beta)
    B = Br_dense(grid, k, a)
    theta = sla.eigh(B, A, eigvals_only=True)
    return 1.0 / theta


# --- matrix-free (any grid) --------------------------------------------------------

def apply_Ar(u, grid, k, tens, a=1.0, alpha=-1.0, beta=2.0, route="fft"):
    """A_r u without forming A_r: P_r/Q_r, the per-voxel middle factors, P_r^*/Q_r^*."""
    n = grid[0] * grid[1] * grid[2]
    u = np.asarray(u, dtype=np.complex128)
    E = basis.apply_Pr(u[:2 * n], grid, k, a, alpha, beta, route).reshape(3, n).T
    H = basis.apply_Qr(u[2 * n:], grid, k, a, alpha, beta, route).reshape(3, n).T
    mu_inv, _, Phi_inv = medium.voxel_blocks(tens)
    mv = lambda M, v: np.einsum("gij,gj->gi", M, v)
    s1 = mv(tens["xi"], mv(mu_inv, E)) + H          # [[xi mu^-1, I],[-I,0]] [E; H]
    s2 = -E
    t1 = mv(Phi_inv, s1)                             # diag(Phi^-1, mu^-1)
    t2 = mv(mu_inv, s2)
    o1 = mv(mu_inv, mv(tens["zeta"], t1)) - t2       # [[mu^-1 zeta, -I],[I,0]]
    o2 = t1
    return np.concatenate([basis.apply_PrH(o1.T.ravel(), grid, k, a, alpha, beta, route),
                           basis.apply_QrH(o2.T.ravel(), grid, k, a, alpha, beta, route)])


def apply_Br(y, grid, k, a=1.0):
    """B_r y: [i Sigma^{-1} y_Q; -i Sigma^{-1} y_P] (Thm 4.2)."""
    n2 = len(y) // 2
    s = sigma_r(grid, k, a)
    y = np.asarray(y, dtype=np.complex128)
    return np.concatenate([1j * y[n2:] / s, -1j * y[:n2] / s])


def cg(apply_A, b, rtol=1e-10, maxit=10000):
    """Unpreconditioned conjugate gradients from x0 = 0 (Sec. 4.2).

    Stops when ||r||_2 <= rtol ||b||_2.  Returns (x, iterations, relres).
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    bnorm = np.sqrt(np.vdot(b, b).real)
    if bnorm == 0.0:
        return x, 0, 0.0
    it = 0
    while np.sqrt(rr) > rtol * bnorm and it < maxit:
        q = apply_A(p)
        alpha = rr / np.vdot(p, q).real
        x += alpha * p
        r -= alpha * q
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, np.sqrt(rr) / bnorm


def nfgep_eigsh(grid, k, tens, nev=10, a=1.0, alpha=-1.0, beta=2.0,
                cg_rtol=1e-12, tol=1e-12, ncv=None, route="fft", seed=0):
    """nev smallest positive omega via ARPACK on B_r y = theta A_r y, largest theta.

    Generalized regular mode with M = A_r and M^{-1} applied by CG: the invert
    Lanczos approach of Sec. 4.2 with a library Lanczos.  Returns
    (omega ascending, Y) with Y the A_r-orthonormal eigenvectors (4n x nev).
    """
    n4 = 4 * grid[0] * grid[1] * grid[2]
    Aop = lambda v: apply_Ar(v, grid, k, tens, a, alpha, beta, route)
    A = spla.LinearOperator((n4, n4), matvec=Aop, dtype=np.complex128)
    B = spla.LinearOperator((n4, n4), matvec=lambda v: apply_Br(v, grid, k, a),
                            dtype=np.complex128)
    Minv = spla.LinearOperator((n4, n4), matvec=lambda v: cg(Aop, v, cg_rtol)[0],
                               dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n4) + 1j * rng.standard_normal(n4)
    theta, Y = spla.eigsh(B, k=nev, M=A, Minv=Minv, which="LA",
                          ncv=ncv or 3 * nev, tol=tol, v0=v0)
    order = np.argsort(-theta)
    theta, Y = theta[order], Y[:, order]
    return 1.0 / theta, Y


def gep_shift_invert(grid, k, tens, nev=10, shift=None, a=1.0):
    """nev smallest positive omega of the sparse 6n GEP by shift-invert, no FFT at all.

    (G - s B)^{-1} B x = x/(omega - s) with 0 < s < omega_1: the largest
    positive values of 1/(omega - s) belong to the smallest omega above s; the
    2n zero eigenvalues map to -1/s and drop out.
    """
    C = yee.C_matrix(grid, k, a)
    G = sp.bmat([[C, None], [None, C.conj().T]], format="csc")
    B = medium.B_matrix(tens).tocsc()
    if shift is None:
        shift = 0.05 * sigma_r(grid, k, a).min()
    lu = spla.splu((G - shift * B).tocsc())
    n6 = G.shape[0]
    op = spla.LinearOperator((n6, n6), matvec=lambda v: lu.solve(B @ v), dtype=np.complex128)
    nu = spla.eigs(op, k=nev, which="LR", tol=1e-13, ncv=max(4 * nev, 40),
                   return_eigenvectors=False)
    omega = shift + 1.0 / nu
    return np.sort(np.real(omega))


# --- Rayleigh quotient and residual ------------------------------------------------

def pencil_residual(y, theta, grid, k, tens, a=1.0, alpha=-1.0, beta=2.0):
    """eta = ||B_r y - theta A_r y|| / (|theta| ||A_r y||) with exact applies."""
    Ay = apply_Ar(y, grid, k, tens, a, alpha, beta)
    By = apply_Br(y, grid, k, a)
    return np.linalg.norm(By - theta * Ay) / (abs(theta) * np.linalg.norm(Ay))


def rayleigh_omega(y, grid, k, tens, a=1.0, alpha=-1.0, beta=2.0):
    """omega = (y^* A_r y) / (y^* B_r y), the pencil Rayleigh quotient."""
    Ay = apply_Ar(y, grid, k, tens, a, alpha, beta)
    By = apply_Br(y, grid, k, a)
    return (np.vdot(y, Ay) / np.vdot(y, By)).real
