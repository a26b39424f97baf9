"""Seeded synthetic inputs: media, Bloch vectors and start vectors.

This module only lays out input data (per-voxel material fields, k-points,
random vectors).  It holds none of the eigensolver's arithmetic, so both the
HIP path and the CPU oracle may consume what it produces.

Conventions shared with the rest of the package:

* A voxel field is a float64 array of shape ``(n3, n2, n1)``; raveled in C
  order it gives the flat index ``g = i1 + n1*i2 + n1*n2*i3`` (x fastest),
  the Kronecker order of the Yee operator (Sec. 2, definition of C1..C3).
* The lattice is simple cubic with constant ``a`` and mesh ``delta_l = a/n_l``.
* The inclusion test is a voxel-centre indicator: voxel ``(i1,i2,i3)`` is
  inside when its centre ``((i+1/2) delta)`` lies strictly inside the shape.
  One indicator serves every material tensor (Sec. 4.3 uses a 0/1 indicator
  matrix for the chiral and pseudochiral parameters).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "voxel_centres",
    "sphere_chiral",
    "rods_pseudochiral",
    "noise_chiral",
    "kpath_gxmgr",
    "uneven_batch",
    "random_vector",
    "homogeneous",
    "lossy_sphere_tensors",
    "random_nonhhpd",
    "homogeneous_tensors",
]


def voxel_centres(n1: int, n2: int, n3: int, a: float = 1.0):
    """Coordinates of voxel centres, each of shape (n3, n2, n1)."""
    x = (np.arange(n1) + 0.5) * (a / n1)
    y = (np.arange(n2) + 0.5) * (a / n2)
    z = (np.arange(n3) + 0.5) * (a / n3)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def sphere_chiral(n1, n2=None, n3=None, radius=0.3, centre=(0.5, 0.5, 0.5),
                  eps_in=13.0, gamma_in=0.5, eps_out=1.0, gamma_out=0.0,
                  a=1.0):
    """One sphere per cell: (eps, gamma) voxel fields for a chiral medium.

    Inside the sphere eps = eps_in and the chirality is gamma_in, outside
    eps_out and gamma_out (Sec. 4.3, chiral parameters xi = i*gamma,
    zeta = -i*gamma; Sec. 5 describes spheres in a simple cubic cell).
    """
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    X, Y, Z = voxel_centres(n1, n2, n3, a)
    cx, cy, cz = (c * a for c in centre)
    inside = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2 < (radius * a) ** 2
    eps = np.where(inside, eps_in, eps_out).astype(np.float64)
    gamma = np.where(inside, gamma_in, gamma_out).astype(np.float64)
    return eps, gamma


def spheres_cylinders_chiral(n1, n2=None, n3=None, radius=0.345, cyl_radius=0.11,
                             eps_in=13.0, eps_out=1.0, gamma=0.5, a=1.0):
    """The paper's simple cubic structure (Sec. 5): a sphere of radius r at every
    lattice point, joined to its neighbours by circular cylinders of radius s along
    the three lattice directions; inside the structure eps_in and chirality gamma,
    outside eps_out and no chirality (the triplet (eps_i, eps_o, gamma)).
    Voxel-centre indicator; the lattice point sits at the cell corner."""
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    X, Y, Z = voxel_centres(n1, n2, n3, a)
    # offsets from the nearest lattice point (periodic images)
    dx = X / a - np.round(X / a)
    dy = Y / a - np.round(Y / a)
    dz = Z / a - np.round(Z / a)
    inside = dx ** 2 + dy ** 2 + dz ** 2 < radius ** 2
    s2 = cyl_radius ** 2
    inside |= (dy ** 2 + dz ** 2 < s2) | (dx ** 2 + dz ** 2 < s2) | (dx ** 2 + dy ** 2 < s2)
    eps = np.where(inside, eps_in, eps_out).astype(np.float64)
    gam = np.where(inside, gamma, 0.0).astype(np.float64)
    return eps, gam


def rods_pseudochiral(n1, n2=None, n3=None, radius=0.2, axis_xy=(0.5, 0.5),
                      eps_in=13.0, gamma_in=0.4, eps_out=1.0, gamma_out=0.0,
                      a=1.0):
    """Rods along z through ``axis_xy``: (eps, gamma) voxel fields.

    The coupling pattern (which two axes xi couples) is not a property of the
    voxel fields; it is passed separately to the solver.
    """
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    X, Y, _ = voxel_centres(n1, n2, n3, a)
    cx, cy = (c * a for c in axis_xy)
    inside = (X - cx) ** 2 + (Y - cy) ** 2 < (radius * a) ** 2
    eps = np.where(inside, eps_in, eps_out).astype(np.float64)
    gamma = np.where(inside, gamma_in, gamma_out).astype(np.float64)
    return eps, gamma


def noise_chiral(n1, n2=None, n3=None, sigma_vox=2.0, seed=0,
                 eps_lo=1.0, eps_hi=13.0, gamma_scale=0.3):
    """Smooth random permittivity and a chirality that follows it.

    u ~ U[0,1) i.i.d. per voxel (``default_rng(seed)``), a periodic Gaussian
    filter of width ``sigma_vox`` voxels (truncate 4), min-max mapped to
    [eps_lo, eps_hi]; gamma = gamma_scale*(eps-eps_lo)/(eps_hi-eps_lo), which
    keeps eps*mu > gamma^2 for mu = 1.
    """
    from scipy.ndimage import gaussian_filter

    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    rng = np.random.default_rng(seed)
    u = rng.random((n3, n2, n1))
    s = gaussian_filter(u, sigma=sigma_vox, mode="wrap", truncate=4.0)
    s = (s - s.min()) / (s.max() - s.min())
    eps = eps_lo + (eps_hi - eps_lo) * s
    gamma = gamma_scale * (eps - eps_lo) / (eps_hi - eps_lo)
    return eps.astype(np.float64), gamma.astype(np.float64)


def random_general(n1, n2=None, n3=None, seed=0, xi_norm=0.6):
    """Random bianisotropic voxel tensors (eps, mu, xi, zeta), each (n, 3, 3) complex.

    mu = Q diag(d) Q^* with d ~ U[0.6, 1.6], eps = R diag(e) R^* with e ~ U[1, 13]
    (Q, R random unitary), xi a complex normal matrix scaled to spectral norm
    xi_norm * U[0, 1), zeta = xi^*.  With xi_norm <= 0.6 the bounds give
    eps - xi mu^-1 zeta >= (1 - 0.36 / 0.6) I > 0, so every voxel meets the
    Hermitian positive definite assumption by construction.
    """
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    n = n1 * n2 * n3
    rng = np.random.default_rng(seed)

    def unitary():
        a = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
        q, _ = np.linalg.qr(a)
        return q

    def herm(vals, q):
        return np.einsum("gij,gj,gkj->gik", q, vals, q.conj())

    mu = herm(rng.uniform(0.6, 1.6, (n, 3)), unitary())
    eps = herm(rng.uniform(1.0, 13.0, (n, 3)), unitary())
    a = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    a /= np.linalg.norm(a, ord=2, axis=(1, 2))[:, None, None]
    xi = a * (xi_norm * rng.random(n))[:, None, None]
    zeta = np.conj(np.transpose(xi, (0, 2, 1)))
    # exact Hermitian symmetry of eps and mu
    eps = 0.5 * (eps + np.conj(np.transpose(eps, (0, 2, 1))))
    mu = 0.5 * (mu + np.conj(np.transpose(mu, (0, 2, 1))))
    return eps, mu, xi, np.ascontiguousarray(zeta)


def _iso(values, n):
    """(n,) complex scalars -> (n, 3, 3) isotropic tensors value * I."""
    return np.asarray(values, dtype=np.complex128).reshape(n)[:, None, None] * np.eye(3)[None]


def lossy_sphere_tensors(n1, n2=None, n3=None, radius=0.3, eps_in=13.0 + 0.5j, gamma_in=0.5,
                         eps_out=1.0, a=1.0):
    """Lossy chiral sphere as per-voxel tensors (eps, mu, xi, zeta), each (n, 3, 3) complex.

    Inside: eps = eps_in I with a positive imaginary part (absorption), xi =
    i gamma_in I, zeta = -i gamma_in I; outside: eps_out I, no chirality; mu = I.
    The complex permittivity makes eps_d, and hence Phi, non-Hermitian, so the
    medium lies outside the Hermitian positive definite assumption (Sec. 4.1)
    while B stays nonsingular (Sec. 3).
    """
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    n = n1 * n2 * n3
    X, Y, Z = voxel_centres(n1, n2, n3, a)
    inside = ((X - 0.5 * a) ** 2 + (Y - 0.5 * a) ** 2 + (Z - 0.5 * a) ** 2 < (radius * a) ** 2).ravel()
    eps = np.where(inside, eps_in, eps_out)
    gam = np.where(inside, gamma_in, 0.0)
    return _iso(eps, n), _iso(np.ones(n), n), _iso(1j * gam, n), _iso(-1j * gam, n)


def random_nonhhpd(n1, n2=None, n3=None, seed=0, loss=0.4, coupling=0.4):
    """Random bianisotropic voxel tensors with no Hermitian structure, each (n, 3, 3).

    eps = R diag(e) R^* + i loss G_e G_e^* (e ~ U[2, 12], G_e complex normal /
    sqrt 3), mu = Q diag(d) Q^* with d ~ U[0.8, 1.4] (Q, R random unitary), and
    xi, zeta two independent complex normal matrices of spectral norm coupling,
    so zeta != xi^* (a non-reciprocal lossy medium, Sec. 3: the NFSEP needs only
    a nonsingular B).
    """
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    n = n1 * n2 * n3
    rng = np.random.default_rng(seed)

    def cnormal():
        return rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))

    def unitary():
        q, _ = np.linalg.qr(cnormal())
        return q

    def herm(vals, q):
        return np.einsum("gij,gj,gkj->gik", q, vals, q.conj())

    ge = cnormal() / np.sqrt(3.0)
    eps = herm(rng.uniform(2.0, 12.0, (n, 3)), unitary()) + 1j * loss * np.einsum("gij,gkj->gik", ge, ge.conj())
    mu = herm(rng.uniform(0.8, 1.4, (n, 3)), unitary())
    mu = 0.5 * (mu + np.conj(np.transpose(mu, (0, 2, 1))))

    def scaled():
        a = cnormal()
        return a * (coupling / np.linalg.norm(a, ord=2, axis=(1, 2)))[:, None, None]

    xi = scaled()
    zeta = scaled()
    return eps, mu, xi, zeta


def homogeneous_tensors(n1, n2=None, n3=None, *, eps=1.0, mu=1.0, xi=0.0, zeta=0.0):
    """Constant isotropic tensors eps I, mu I, xi I, zeta I (complex scalars allowed)."""
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    n = n1 * n2 * n3
    return tuple(_iso(np.full(n, v, dtype=np.complex128), n) for v in (eps, mu, xi, zeta))


def homogeneous(n1, n2=None, n3=None, *, eps=1.0, gamma=0.0):
    """Constant (eps, gamma) fields."""
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    return (np.full((n3, n2, n1), float(eps)),
            np.full((n3, n2, n1), float(gamma)))


def kpath_gxmgr(per_segment: int = 10):
    """Bloch vectors on Gamma-X-M-Gamma-R, in reciprocal units (k_l in [0,1/2]).

    Each segment is sampled at its midpoints t = (j+1/2)/per_segment, so no
    vertex is taken twice and Gamma (k = 0, where the curl basis does not
    exist) is never sampled.
    """
    G = np.array([0.0, 0.0, 0.0])
    X = np.array([0.5, 0.0, 0.0])
    M = np.array([0.5, 0.5, 0.0])
    R = np.array([0.5, 0.5, 0.5])
    ks = []
    for p, q in ((G, X), (X, M), (M, G), (G, R)):
        for j in range(per_segment):
            t = (j + 0.5) / per_segment
            ks.append(p + t * (q - p))
    return np.array(ks)


def kpath_gxmrg(per_segment: int = 10):
    """Bloch vectors on G-X-M-R-G (the band-structure path of the paper's Sec. 5),
    sampled at segment midpoints as in ``kpath_gxmgr``."""
    G = np.array([0.0, 0.0, 0.0])
    X = np.array([0.5, 0.0, 0.0])
    M = np.array([0.5, 0.5, 0.0])
    R = np.array([0.5, 0.5, 0.5])
    ks = []
    for p, q in ((G, X), (X, M), (M, R), (R, G)):
        for j in range(per_segment):
            t = (j + 0.5) / per_segment
            ks.append(p + t * (q - p))
    return np.array(ks)


def uneven_batch(count: int = 32, seed: int = 0, grids=(48, 64, 96, 128)):
    """Mixed-size batch of chiral-sphere instances.

    Returns a list of dicts with keys ``grid`` (n, n, n), ``k`` (3,),
    ``radius``, ``eps_in``, ``gamma_in``.  Sizes drawn from ``grids``; sphere
    radius ~ U[0.15,0.35], eps_in ~ U[4,13], gamma_in ~ U[0,0.5],
    k ~ U[0,1/2]^3.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(grids))
        out.append(dict(grid=(n, n, n),
                        k=rng.uniform(0.0, 0.5, size=3),
                        radius=float(rng.uniform(0.15, 0.35)),
                        eps_in=float(rng.uniform(4.0, 13.0)),
                        gamma_in=float(rng.uniform(0.0, 0.5))))
    return out


def random_vector(size: int, seed: int = 0) -> np.ndarray:
    """Complex normal vector (real and imaginary parts N(0,1)), complex128."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(size) + 1j * rng.standard_normal(size)).astype(np.complex128)
