"""Write the stored expected eigenvalues used by the GPU parity tests.

Only the CPU oracle (``oracle/``) computes these values; nothing here touches
the HIP library.  Inputs come from the seeded generators in
``paper_1402_6297_amd.media``.  Usage:

    python tests/golden/make_golden.py config1_16      # ~2 min
    python tests/golden/make_golden.py config2_64      # ~80 min (ARPACK + CG in numpy)
    python tests/golden/make_golden.py nfsep_lossy16   # NFSEP, lossy chiral sphere

Each entry records the workload, the oracle route and its tolerances.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import medium, nfgep, nfsep  # noqa: E402
from paper_1402_6297_amd import media  # noqa: E402


def config1_16():
    """Chiral sphere r=0.3, eps 13, gamma 0.5 on 16^3, k=(0.1,0.2,0.3), 10 smallest omega."""
    grid, k = (16, 16, 16), (0.1, 0.2, 0.3)
    eps, gam = media.sphere_chiral(16)
    t = medium.tensors_chiral(eps, gam)
    t0 = time.time()
    w_si = nfgep.gep_shift_invert(grid, k, t, nev=10)
    t1 = time.time()
    w_l, _ = nfgep.nfgep_eigsh(grid, k, t, nev=10, cg_rtol=1e-13, tol=1e-13)
    t2 = time.time()
    w_l = np.sort(w_l)
    assert np.abs(w_si - w_l).max() < 1e-10 * w_si.max(), (w_si, w_l)
    return dict(grid=grid, k=k, medium="sphere_chiral(r=0.3, eps_in=13, gamma_in=0.5)",
                omega=w_si.tolist(), omega_arpack=w_l.tolist(),
                route="sparse shift-invert on the 6n GEP (no FFT); cross-checked by ARPACK on the pencil",
                seconds=[t1 - t0, t2 - t1])


def config2_64():
    """Same medium on 64^3, k=(0.25,0,0), 10 smallest omega (ARPACK on the pencil, CG 1e-12)."""
    grid, k = (64, 64, 64), (0.25, 0.0, 0.0)
    eps, gam = media.sphere_chiral(64)
    t = medium.tensors_chiral(eps, gam)
    t0 = time.time()
    w, Y = nfgep.nfgep_eigsh(grid, k, t, nev=10, cg_rtol=1e-12, tol=1e-12)
    order = np.argsort(w)
    w, Y = w[order], Y[:, order]
    eta = [float(nfgep.pencil_residual(Y[:, j], 1.0 / w[j], grid, k, t)) for j in range(10)]
    return dict(grid=grid, k=k, medium="sphere_chiral(r=0.3, eps_in=13, gamma_in=0.5)",
                omega=w.tolist(), residual=eta,
                route="ARPACK (eigsh, which='LA') on B_r y = theta A_r y with CG (rtol 1e-12) inner solves",
                seconds=time.time() - t0)


def nfsep_lossy16():
    """Lossy chiral sphere r=0.3, eps 13+0.5i, gamma 0.5 on 16^3 (outside the HHPD
    assumption), k=(0.1,0.2,0.3): the 8 eigenvalues of positive real part and
    smallest modulus of the NFSEP (Thm 3.2), by sparse shift-invert on the 6n
    GEP, cross-checked by zero-shift shift-invert Arnoldi on K with GMRES."""
    grid, k = (16, 16, 16), (0.1, 0.2, 0.3)
    eps, mu, xi, zeta = media.lossy_sphere_tensors(16)
    t = dict(eps=eps, mu=mu, xi=xi, zeta=zeta)
    t0 = time.time()
    w = nfsep.gep_shift_invert(grid, k, t, nev=8)
    t1 = time.time()
    w2 = nfsep.si_arnoldi(grid, k, t, nev=8, inner_rtol=1e-13, tol=1e-12)
    t2 = time.time()
    assert np.abs(w - w2).max() < 1e-10 * np.abs(w).max(), (w, w2)
    return dict(grid=grid, k=k, medium="lossy_sphere_tensors(r=0.3, eps_in=13+0.5i, gamma_in=0.5)",
                omega_re=w.real.tolist(), omega_im=w.imag.tolist(),
                omega2_re=w2.real.tolist(), omega2_im=w2.imag.tolist(),
                route="sparse shift-invert on the 6n GEP (no FFT); cross-checked by shift-invert "
                      "Arnoldi on K with GMRES inner solves",
                seconds=[t1 - t0, t2 - t1])


if __name__ == "__main__":
    for name in sys.argv[1:]:
        res = globals()[name]()
        path = os.path.join(HERE, f"{name}.json")
        with open(path, "w") as f:
            json.dump(res, f, indent=1)
        print(f"wrote {path}")
