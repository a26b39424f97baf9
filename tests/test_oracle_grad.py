"""Pins for the oracle's eigenvalue gradients (CPU only).

Checked against central finite differences of dense LAPACK eigenvalues and,
for a homogeneous medium, against the derivative of the closed form.
"""
import numpy as np

from oracle import grad, medium, nfgep, yee
from paper_1402_6297_amd import media

K0 = np.array([0.1, 0.2, 0.3])


def _smallest(eps, gam, nev, grid=(4, 4, 4)):
    w = nfgep.gep_dense(grid, K0, medium.tensors_chiral(eps, gam))
    return nfgep.positive_smallest(w, nev, 1e-8)


def test_gradient_matches_central_differences():
    grid = (4, 4, 4)
    eps, gam = media.noise_chiral(4, sigma_vox=1.0, seed=4)
    om, de, dg = grad.chiral_eigs_and_grads(grid, K0, eps, gam, 3)
    h = 1e-6
    for g in (0, 17, 42, 63):
        for field, ref in (("eps", de), ("gam", dg)):
            e1, g1 = eps.copy().ravel(), gam.copy().ravel()
            e2, g2 = eps.copy().ravel(), gam.copy().ravel()
            if field == "eps":
                e1[g] += h
                e2[g] -= h
            else:
                g1[g] += h
                g2[g] -= h
            fd = (_smallest(e1, g1, 3) - _smallest(e2, g2, 3)) / (2 * h)
            assert np.abs(fd - ref[:, g]).max() < 1e-6 * np.abs(ref).max() + 1e-9


def test_gradient_sum_matches_closed_form_derivative():
    """Homogeneous chiral: sum_g d omega / d eps_g equals d omega/d eps of the closed form."""
    grid = (4, 4, 4)
    eps0, g0 = 13.0, 0.5
    eps, gam = media.homogeneous(4, eps=eps0, gamma=g0)
    om, de, dg = grad.chiral_eigs_and_grads(grid, K0, eps, gam, 2)
    L1, L2, L3 = yee.lambdas(grid, K0)
    s2 = np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2
    c = L1 ** 2 + L2 ** 2 + L3 ** 2

    def branch(e, gg):
        Phi = e - gg ** 2
        disc = np.sqrt(e * (s2 - c.real) ** 2 + Phi * c.imag ** 2)
        return np.sqrt(np.concatenate([e * s2 - gg ** 2 * c.real + gg * disc,
                                       e * s2 - gg ** 2 * c.real - gg * disc]) / Phi ** 2)

    w0 = branch(eps0, g0)
    h = 1e-6
    for j in range(2):
        i = np.argmin(np.abs(w0 - om[j]))
        d_eps = (branch(eps0 + h, g0)[i] - branch(eps0 - h, g0)[i]) / (2 * h)
        d_gam = (branch(eps0, g0 + h)[i] - branch(eps0, g0 - h)[i]) / (2 * h)
        assert abs(de[j].sum() - d_eps) < 1e-7 * abs(d_eps)
        assert abs(dg[j].sum() - d_gam) < 1e-7 * max(abs(d_gam), 1e-3)
