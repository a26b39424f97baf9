"""The null space free eigenvalue problem (NFSEP) for any medium with a nonsingular B (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* K = diag(Sigma_r^{1/2} Q_r^*, Sigma_r^{1/2} P_r^*) B^{-1} diag(P_r Sigma_r^{1/2}, Q_r Sigma_r^{1/2})
  (Thm 3.2), a 4n x 4n matrix with no Hermitian structure in general.
* K y = omega y has exactly the nonzero eigenvalues of the discrete GEP
  diag(C, C^*) x = omega B x (Thm 3.1, Thm 3.2) and no zero eigenvalue.
* The paper solves it with a shift-and-invert Arnoldi method at zero shift and
  a GMRES inner solve when the medium lies outside the HHPD assumption
  (opening of Sec. 4, the NFSEP column of the summary table, the else-branch
  of Algorithm 1).  Algorithm 1 then scales the eigenvector by
  diag(Sigma_r^{1/2}, Sigma_r^{1/2}) before recovering the fields.

"Smallest positive" is read here as: the eigenvalues with positive real part,
in ascending modulus (what a zero shift delivers first).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import basis, medium, nfgep


def voxel_Binv(tens):
    """Per-voxel inverse of the 6 x 6 block i [[zeta, mu], [-eps, -xi]] (Sec. 3, eq. for B)."""
    Bv = 1j * np.block([[tens["zeta"], tens["mu"]], [-tens["eps"], -tens["xi"]]])
    return np.linalg.inv(Bv)


def K_dense(grid, k, tens, a=1.0, alpha=-1.0, beta=2.0, bas=None):
    """K as the literal product of its three factors (Thm 3.2)."""
    bas = basis.basis_dense(grid, k, a, alpha, beta) if bas is None else bas
    Pr, Qr = bas["Pr"], bas["Qr"]
    sh = np.sqrt(nfgep.sigma_r(grid, k, a))          # Sigma_r^{1/2}, length 2n
    Binv = np.linalg.inv(medium.B_matrix(tens).toarray())
    left = sla.block_diag(sh[:, None] * Qr.conj().T, sh[:, None] * Pr.conj().T)
    right = sla.block_diag(Pr * sh[None, :], Qr * sh[None, :])
    return left @ Binv @ right


def eigs_dense(grid, k, tens, a=1.0, alpha=-1.0, beta=2.0):
    """All 4n eigenvalues of K (dense LAPACK)."""
    return np.linalg.eigvals(K_dense(grid, k, tens, a, alpha, beta))


def apply_W(x, grid, k, tens, a=1.0, alpha=-1.0, beta=2.0, route="fft"):
    """W x = diag(Q_r^*, P_r^*) B^{-1} diag(P_r, Q_r) x, the unscaled middle of K (Thm 3.2)."""
    n = grid[0] * grid[1] * grid[2]
    x = np.asarray(x, dtype=np.complex128)
    E = basis.apply_Pr(x[:2 * n], grid, k, a, alpha, beta, route).reshape(3, n).T
    H = basis.apply_Qr(x[2 * n:], grid, k, a, alpha, beta, route).reshape(3, n).T
    o = np.einsum("gij,gj->gi", voxel_Binv(tens), np.concatenate([E, H], axis=1))
    top = basis.apply_QrH(o[:, :3].T.ravel(), grid, k, a, alpha, beta, route)
    bot = basis.apply_PrH(o[:, 3:].T.ravel(), grid, k, a, alpha, beta, route)
    return np.concatenate([top, bot])


def _s_half(grid, k, a):
    """diag(Sigma_r^{1/2}, Sigma_r^{1/2}) as a length-4n vector."""
    sh = np.sqrt(nfgep.sigma_r(grid, k, a))
    return np.concatenate([sh, sh])


def apply_K(y, grid, k, tens, a=1.0, alpha=-1.0, beta=2.0, route="fft"):
    """K y = S W S y with S = diag(Sigma_r^{1/2}, Sigma_r^{1/2}), without forming K."""
    s = _s_half(grid, k, a)
    return s * apply_W(s * np.asarray(y, dtype=np.complex128), grid, k, tens, a, alpha, beta, route)


def smallest_positive(omegas, nev, rel_zero=1e-8):
    """The nev eigenvalues with Re omega > rel_zero max|omega|, in ascending modulus."""
    w = np.asarray(omegas, dtype=np.complex128)
    w = w[np.real(w) > rel_zero * np.abs(w).max()]
    return w[np.argsort(np.abs(w), kind="stable")][:nev]


def gmres(apply_A, b, rtol=1e-12, maxit=2000):
    """Minimal-residual solve of A x = b over the Krylov space of b (no restart).

    Arnoldi with modified Gram-Schmidt builds V and the Hessenberg H; the
    small least-squares problem min ||beta e1 - H c|| is solved by LAPACK.
    Stops when the minimal residual is <= rtol ||b||.  Returns (x, iterations, relres).
    """
    b = np.asarray(b, dtype=np.complex128)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros_like(b), 0, 0.0
    V = [b / beta]
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    c = np.zeros(0, dtype=np.complex128)
    res = 1.0
    j = 0
    for j in range(maxit):
        w = apply_A(V[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        rhs = np.zeros(j + 2, dtype=np.complex128)
        rhs[0] = beta
        c, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], rhs, rcond=None)
        res = np.linalg.norm(rhs - H[:j + 2, :j + 1] @ c) / beta
        if res <= rtol or H[j + 1, j] == 0.0:
            break
        V.append(w / H[j + 1, j])
    x = sum(ci * vi for ci, vi in zip(c, V))
    return x, j + 1, res


def si_arnoldi(grid, k, tens, nev=6, a=1.0, alpha=-1.0, beta=2.0, inner_rtol=1e-13, tol=1e-12,
               ncv=None, route="fft", seed=0):
    """Shift-and-invert Arnoldi at zero shift on K with GMRES inner solves (Sec. 4 opening).

    ARPACK (library Arnoldi, shift-invert mode) with OPinv = K^{-1} = S^{-1}
    W^{-1} S^{-1}, W^{-1} by ``gmres`` (W lacks the Sigma_r scaling that makes
    K ill-conditioned), returns the 2 nev + 4 eigenvalues of K of smallest
    modulus; the nev with positive real part are kept, ascending in modulus.
    """
    n4 = 4 * grid[0] * grid[1] * grid[2]
    s = _s_half(grid, k, a)
    Kop = lambda v: apply_K(v, grid, k, tens, a, alpha, beta, route)
    Wop = lambda v: apply_W(v, grid, k, tens, a, alpha, beta, route)
    K = spla.LinearOperator((n4, n4), matvec=Kop, dtype=np.complex128)
    Kinv = spla.LinearOperator((n4, n4), matvec=lambda v: gmres(Wop, v / s, inner_rtol)[0] / s,
                               dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n4) + 1j * rng.standard_normal(n4)
    kk = 2 * nev + 4
    w = spla.eigs(K, k=kk, sigma=0.0, OPinv=Kinv, which="LM", ncv=ncv or max(3 * kk, 40), tol=tol,
                  v0=v0, return_eigenvectors=False)
    return smallest_positive(w, nev)


def residual(z, omega, grid, k, tens, a=1.0, alpha=-1.0, beta=2.0):
    """eta = ||K y - omega y|| / (|omega| ||y||) for y = Sigma^{-1/2} z (z the scaled vector of Alg. 1)."""
    y = np.asarray(z, dtype=np.complex128) / _s_half(grid, k, a)
    r = apply_K(y, grid, k, tens, a, alpha, beta) - omega * y
    return np.linalg.norm(r) / (abs(omega) * np.linalg.norm(y))


def rayleigh(z, grid, k, tens, a=1.0, alpha=-1.0, beta=2.0):
    """omega = y^* K y / y^* y for y = Sigma^{-1/2} z (the least-squares eigenvalue estimate)."""
    y = np.asarray(z, dtype=np.complex128) / _s_half(grid, k, a)
    return np.vdot(y, apply_K(y, grid, k, tens, a, alpha, beta)) / np.vdot(y, y)


def gep_shift_invert(grid, k, tens, nev=6, shift=None, a=1.0, extra=6):
    """nev eigenvalues with positive real part and smallest modulus, from the sparse 6n GEP.

    No FFT and no SVD basis: (G - s B)^{-1} B x = x / (omega - s) with
    G = diag(C, C^*) (Sec. 3) and a real shift 0 < s below the wanted
    eigenvalues; the 2n zero eigenvalues map to -1/s and are never among the
    largest real parts.  ARPACK returns nev + extra values of largest real part
    of 1/(omega - s); they are mapped back and the smallest_positive nev kept.
    """
    import scipy.sparse as sp
    from . import yee
    Cm = yee.C_matrix(grid, k, a)
    G = sp.bmat([[Cm, None], [None, Cm.conj().T]], format="csc")
    B = medium.B_matrix(tens).tocsc()
    if shift is None:
        shift = 0.05 * nfgep.sigma_r(grid, k, a).min()
    lu = spla.splu((G - shift * B).tocsc())
    n6 = G.shape[0]
    op = spla.LinearOperator((n6, n6), matvec=lambda v: lu.solve(B @ v), dtype=np.complex128)
    nu = spla.eigs(op, k=nev + extra, which="LR", tol=1e-14, ncv=max(4 * (nev + extra), 40),
                   return_eigenvectors=False)
    return smallest_positive(shift + 1.0 / nu, nev)
