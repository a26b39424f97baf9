"""Null-space and range bases of C and the SVD C = P_r Sigma_r Q_r^* (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Two routes:

* ``basis_dense``: dense 3n x n matrices built exactly as the paper writes them:
  Q_0 = (I_3 (x) T) Pi_0 (Thm 2.3); Q_1 = (I - Q_0 Q_0^*) T_1 (Lp^* Lp Lq^{-1})^{-1/2},
  P_1 likewise with P_0 (the projection construction); Q_2 = C^* T_1
  (Lp^* Lp)^{-1/2}, P_2 = C T_1 (Lp^* Lp)^{-1/2} (the curl construction);
  Q = [Q1 Q2 Q0], P = [P2 P1 P0] (ordering before Thm 2.4), Q_r = [Q1 Q2],
  P_r = [P2 P1] (Thm 2.5).  Only the first (projection) line of the Q_1
  definition is used; its displayed right-hand side has a different scale.
* ``pi_vectors``: the same Pi's per frequency (3-vectors), for the
  matrix-free oracle at larger grids: the projection of a = (alpha, beta, 1)
  off pi_0, scaled by (||p||^2/sigma^2)^{-1/2}, and pi_2 = conj(p)/||p|| with p
  the Lambda_p column (Lemma 2.2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import yee


def lambda_q_p(grid, k, a=1.0, alpha=-1.0, beta=2.0):
    """Lambda_q (length n, real) and Lambda_p (3 x n) of Lemma 2.2."""
    L1, L2, L3 = yee.lambdas(grid, k, a)
    Lq = (np.conj(L1) * L1 + np.conj(L2) * L2 + np.conj(L3) * L3).real
    Lp = np.stack([beta * L3 - L2, L1 - alpha * L3, alpha * L2 - beta * L1])
    return Lq, Lp


def _stack_diag(cols):
    """3 x n per-frequency columns -> dense 3n x n block matrix [diag(c0); diag(c1); diag(c2)]."""
    return np.vstack([np.diag(c) for c in cols])


def basis_dense(grid, k, a=1.0, alpha=-1.0, beta=2.0):
    """Dense Q_0, Q_1, Q_2, P_0, P_1, P_2 (each 3n x n), Sigma_r diagonal, and C.

    Returns a dict with those keys plus 'Q', 'P', 'Qr', 'Pr', 'sigma' (length n,
    Lambda_q^{1/2}), 'T' and 'C' (dense).
    """
    n1, n2, n3 = grid
    n = n1 * n2 * n3
    T = yee.T_dense(grid, k, a)
    C = yee.C_matrix(grid, k, a).toarray()
    L1, L2, L3 = yee.lambdas(grid, k, a)
    Lq, Lp = lambda_q_p(grid, k, a, alpha, beta)
    I3T = np.kron(np.eye(3), T)
    Pi0 = _stack_diag([L1, L2, L3]) * (Lq ** -0.5)[None, :]
    Q0 = I3T @ Pi0
    P0 = I3T @ np.conj(Pi0)
    T1 = np.vstack([alpha * T, beta * T, T])
    LpLp = (np.conj(Lp) * Lp).sum(axis=0).real
    s1 = (LpLp / Lq) ** -0.5
    s2 = LpLp ** -0.5
    I = np.eye(3 * n)
    Q1 = ((I - Q0 @ Q0.conj().T) @ T1) * s1[None, :]
    P1 = ((I - P0 @ P0.conj().T) @ T1) * s1[None, :]
    Q2 = (C.conj().T @ T1) * s2[None, :]
    P2 = (C @ T1) * s2[None, :]
    sigma = np.sqrt(Lq)
    return dict(T=T, C=C, Q0=Q0, Q1=Q1, Q2=Q2, P0=P0, P1=P1, P2=P2,
                Q=np.hstack([Q1, Q2, Q0]), P=np.hstack([P2, P1, P0]),
                Qr=np.hstack([Q1, Q2]), Pr=np.hstack([P2, P1]), sigma=sigma,
                Pi0=Pi0)


def pi_vectors(grid, k, a=1.0, alpha=-1.0, beta=2.0):
    """Per-frequency pi_0, pi_1, pi_2 (each 3 x n) and sigma (length n).

    pi_0 = lambda / sigma (Thm 2.3).  pi_1 is the orthogonal projection of the
    T_1 column (alpha, beta, 1) off pi_0, times (Lp^*Lp Lq^{-1})^{-1/2}
    (projection construction of Q_1).  pi_2 = conj(Lp column)(Lp^*Lp)^{-1/2}
    (curl construction of Q_2).
    """
    L1, L2, L3 = yee.lambdas(grid, k, a)
    Lq, Lp = lambda_q_p(grid, k, a, alpha, beta)
    n = Lq.size
    sigma = np.sqrt(Lq)
    pi0 = np.stack([L1, L2, L3]) / sigma[None, :]
    avec = np.array([alpha, beta, 1.0], dtype=np.complex128)[:, None] * np.ones((1, n))
    proj = avec - pi0 * (np.conj(pi0) * avec).sum(axis=0)[None, :]
    LpLp = (np.conj(Lp) * Lp).sum(axis=0).real
    pi1 = proj * ((LpLp / Lq) ** -0.5)[None, :]
    pi2 = np.conj(Lp) * (LpLp ** -0.5)[None, :]
    return pi0, pi1, pi2, sigma


# --- matrix-free P_r, Q_r and their adjoints --------------------------------------
# P_r = (I_3 (x) T)[-conj(Pi_2), conj(Pi_1)],  Q_r = (I_3 (x) T)[Pi_1, Pi_2]  (Thm 2.5).

def _T(q, grid, k, a, adjoint, route):
    f = yee.T_apply_fft if route == "fft" else yee.T_apply_separable
    return f(q, grid, k, a, adjoint=adjoint)


def apply_Pr(yP, grid, k, a=1.0, alpha=-1.0, beta=2.0, route="fft"):
    """P_r y for y of length 2n -> length 3n (component-major E_x, E_y, E_z)."""
    _, pi1, pi2, _ = pi_vectors(grid, k, a, alpha, beta)
    n = pi1.shape[1]
    ya, yb = yP[:n], yP[n:]
    e = -np.conj(pi2) * ya[None, :] + np.conj(pi1) * yb[None, :]
    return np.concatenate([_T(e[c], grid, k, a, False, route) for c in range(3)])


def apply_Qr(yQ, grid, k, a=1.0, alpha=-1.0, beta=2.0, route="fft"):
    """Q_r y for y of length 2n -> length 3n."""
    _, pi1, pi2, _ = pi_vectors(grid, k, a, alpha, beta)
    n = pi1.shape[1]
    yc, yd = yQ[:n], yQ[n:]
    h = pi1 * yc[None, :] + pi2 * yd[None, :]
    return np.concatenate([_T(h[c], grid, k, a, False, route) for c in range(3)])


def apply_PrH(x, grid, k, a=1.0, alpha=-1.0, beta=2.0, route="fft"):
    """P_r^* x for x of length 3n -> length 2n."""
    _, pi1, pi2, _ = pi_vectors(grid, k, a, alpha, beta)
    n = pi1.shape[1]
    xh = np.stack([_T(x[c * n:(c + 1) * n], grid, k, a, True, route) for c in range(3)])
    return np.concatenate([(-pi2 * xh).sum(axis=0), (pi1 * xh).sum(axis=0)])


def apply_QrH(x, grid, k, a=1.0, alpha=-1.0, beta=2.0, route="fft"):
    """Q_r^* x for x of length 3n -> length 2n."""
    _, pi1, pi2, _ = pi_vectors(grid, k, a, alpha, beta)
    n = pi1.shape[1]
    xh = np.stack([_T(x[c * n:(c + 1) * n], grid, k, a, True, route) for c in range(3)])
    return np.concatenate([(np.conj(pi1) * xh).sum(axis=0), (np.conj(pi2) * xh).sum(axis=0)])


def sparse_blockdiag3(cols):
    """Helper: 3n x n sparse matrix from three length-n diagonals."""
    return sp.vstack([sp.diags(c) for c in cols], format="csr")
