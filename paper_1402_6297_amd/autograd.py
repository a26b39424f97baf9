"""Differentiable smallest eigenvalues of a chiral medium.

``eigenvalues(eps, gamma, grid, k, nev)`` returns the nev smallest positive
omega of the null-space free GEP (Sec. 3) as a torch tensor that carries a
gradient back to the per-voxel ``eps`` and ``gamma`` fields.  The forward pass
is ``nsf_eigs``; the backward pass is ``nsf_eig_grad``, the HIP kernel that
evaluates the Hellmann-Feynman derivative of the Hermitian positive definite
pencil (Thm 4.2): for an A_r-normalised eigenvector y, d omega = omega y^* dA_r y,
which reduces to per-voxel sums over the real-space fields E' = P_r y_P and
H' = Q_r y_Q.

An eigenvalue that belongs to a numerically degenerate cluster has no
derivative of its own; only symmetric functions of the cluster do.  The
backward pass therefore replaces the incoming weights dS/d omega_j by their
mean over each cluster (a no-op when the weights are already equal there, as
for a sum of eigenvalues), and warns when they were not.  That needs every
copy of a multiple eigenvalue, so the forward pass runs the solver's
multiplicity checks (fresh starts A_r-orthogonal to the converged pairs, until one changes nothing),
and it solves for one pair more than it returns: when omega_nev and
omega_{nev+1} form one cluster, a function of the first nev alone is not
differentiable there, and the forward pass warns.

No plan is held between the passes: the backward pass builds one for the saved
medium, so the graph may be differentiated more than once (retain_graph=True).
"""
from __future__ import annotations

import warnings

import numpy as np
import torch

from . import nsf


def clusters(omega: np.ndarray, rtol: float) -> list[list[int]]:
    """Index groups of ascending omega whose neighbours differ by <= rtol*|omega|."""
    groups: list[list[int]] = []
    for j, w in enumerate(omega):
        if groups and abs(w - omega[groups[-1][-1]]) <= rtol * max(abs(w), 1e-300):
            groups[-1].append(j)
        else:
            groups.append([j])
    return groups


def cut_in_cluster(omega: np.ndarray, nev: int, rtol: float) -> bool:
    """Whether omega[nev - 1] and omega[nev] (ascending) belong to one cluster."""
    if len(omega) <= nev:
        return False
    a, b = omega[nev - 1], omega[nev]
    return abs(b - a) <= rtol * max(abs(b), 1e-300)


def cluster_weights(omega: np.ndarray, weights: np.ndarray, rtol: float) -> np.ndarray:
    """Average the weights over degenerate clusters (see the module docstring)."""
    w = np.array(weights, dtype=np.float64)
    for g in clusters(omega, rtol):
        if len(g) > 1:
            m = w[g].mean()
            if np.abs(w[g] - m).max() > 1e-12 * max(np.abs(w[g]).max(), 1e-300):
                warnings.warn(f"eigenvalues {g} are degenerate to rtol {rtol:g}: their gradients "
                              "are not separately defined; using the mean weight over the cluster",
                              RuntimeWarning, stacklevel=3)
            w[g] = m
    return w


class NSFEig(torch.autograd.Function):
    """omega = NSFEig.apply(eps, gamma, grid, k, nev, res_tol, cg_rtol, seed, cluster_rtol).

    eps, gamma: float64 tensors on a HIP device, shape (n3, n2, n1) (x fastest).
    Returns float64 omega (nev,) on the same device, ascending.
    """

    @staticmethod
    def forward(ctx, eps, gamma, grid, k, nev, res_tol, cg_rtol, seed, cluster_rtol):
        if not (eps.is_cuda and gamma.is_cuda):
            raise TypeError("eps and gamma must be HIP device tensors")
        eps_c = eps.detach().contiguous()
        gam_c = gamma.detach().contiguous()
        with nsf.Plan(grid, k) as plan:
            plan.set_chiral(eps_c, gam_c)
            plan.set_option(nsf.NSF_OPT_VERIFY, 16)  # stops at the first check that changes nothing
            n = plan.n
            Y = torch.empty((nev + 1, 4 * n), dtype=torch.complex128, device=eps.device)
            st, om, res, stats = plan.eigs(nev + 1, res_tol=res_tol, cg_rtol=cg_rtol, seed=seed, Y=Y)
        if st != nsf.NSF_OK:
            raise nsf.NsfError(st, f"eigensolve did not converge (residuals {res})")
        if cut_in_cluster(om, nev, cluster_rtol):
            warnings.warn(f"omega_{nev} and omega_{nev + 1} are degenerate to rtol {cluster_rtol:g}: the "
                          f"{nev} smallest eigenvalues are not differentiable functions of the medium there",
                          RuntimeWarning, stacklevel=2)
        ctx.grid, ctx.k = grid, k
        ctx.omega = om[:nev]
        ctx.cluster_rtol = cluster_rtol
        ctx.save_for_backward(eps_c, gam_c, Y[:nev])
        ctx.stats = stats
        return torch.as_tensor(om[:nev], dtype=torch.float64, device=eps.device)

    @staticmethod
    def backward(ctx, grad_omega):
        eps_c, gam_c, Y = ctx.saved_tensors
        w = cluster_weights(ctx.omega, grad_omega.detach().double().cpu().numpy(), ctx.cluster_rtol)
        d_eps = torch.empty(eps_c.shape, dtype=torch.float64, device=Y.device)
        d_gamma = torch.empty_like(d_eps)
        with nsf.Plan(ctx.grid, ctx.k) as plan:
            plan.set_chiral(eps_c, gam_c)
            plan.eig_grad(ctx.omega, Y, w, d_eps, d_gamma)
        return d_eps, d_gamma, None, None, None, None, None, None, None


def eigenvalues(eps, gamma, grid, k, nev, res_tol=1e-10, cg_rtol=1e-11, seed=0, cluster_rtol=1e-8):
    """The nev smallest positive omega, differentiable w.r.t. eps and gamma."""
    return NSFEig.apply(eps, gamma, tuple(grid), tuple(k), int(nev), float(res_tol), float(cg_rtol),
                        int(seed), float(cluster_rtol))
