"""GPU parity of the NFSEP path (Thm 3.2; the else-branch of Algorithm 1) against
the CPU oracle: media outside the HHPD assumption (lossy, non-reciprocal).

Bars: the K matvec <= 1e-12 relative (max-abs error over max-abs value, as
every matvec here); eigenvalues <= 1e-10 relative to the largest returned
modulus with residuals eta <= res_tol; fields that solve the 6n GEP to the
eigenpair residual.
"""
import json
import os

import numpy as np
import pytest

from oracle import basis, medium, nfgep, nfsep, yee
from paper_1402_6297_amd import media, nsf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(x, ref):
    return np.abs(x - ref).max() / np.abs(ref).max()


def tens_of(t):
    eps, mu, xi, zeta = t
    return dict(eps=eps, mu=mu, xi=xi, zeta=zeta)


def medium_for(kind, grid, seed=3):
    if kind == "random":
        return media.random_nonhhpd(*grid, seed=seed)
    if kind == "lossy":
        return media.lossy_sphere_tensors(*grid, radius=0.4 if max(grid) <= 6 else 0.3)
    raise ValueError(kind)


def match(a, b):
    b = list(np.asarray(b))
    worst = 0.0
    for x in np.asarray(a):
        j = int(np.argmin([abs(x - y) for y in b]))
        worst = max(worst, abs(x - b[j]))
        b.pop(j)
    return worst


K_CASES = [((4, 4, 4), (0.1, 0.2, 0.3)), ((3, 4, 5), (0.25, 0.5, 0.1)),
           ((16, 12, 10), (0.3, 0.1, 0.2)), ((32, 32, 32), (0.1, 0.2, 0.3)),
           ((64, 16, 48), (0.3, 0.0, 0.2))]


@pytest.mark.parametrize("path", [0, 1, 2], ids=["auto", "generic", "twolevel"])
@pytest.mark.parametrize("kind", ["random", "lossy"])
@pytest.mark.parametrize("grid,k", K_CASES)
def test_K_matches_oracle(grid, k, kind, path):
    n = grid[0] * grid[1] * grid[2]
    t = medium_for(kind, grid)
    y = media.random_vector(4 * n, 5)
    ref = nfsep.apply_K(y, grid, k, tens_of(t))
    with nsf.Plan(grid, k) as P:
        P.set_option(nsf.NSF_OPT_FFT_PATH, path)
        P.set_nfsep(*t)
        assert P.query()["medium_kind"] == nsf.NSF_MEDIUM_NFSEP
        out = torch.empty(4 * n, dtype=torch.complex128, device="cuda")
        P.K(dev(y), out)
        got = host(out)
        yd = dev(y)
        P.K(yd, yd)  # in place
        got2 = host(yd)
    assert rel(got, ref) < 1e-12
    assert np.array_equal(got, got2)


@pytest.mark.parametrize("which", ["nfsep", "general"])
def test_palette_matches_per_voxel_storage(which):
    """A piecewise-constant medium stored as a palette of its distinct voxel
    factors plus a 16-bit index gives bitwise the same applies as the factors
    stored per voxel; a medium with all voxels distinct falls back to per voxel."""
    grid, k = (32, 24, 16), (0.1, 0.2, 0.3)
    n = grid[0] * grid[1] * grid[2]
    if which == "nfsep":
        t = media.lossy_sphere_tensors(*grid)
    else:
        tt = medium.tensors_chiral(*media.sphere_chiral(*grid))
        t = (tt["eps"], tt["mu"], tt["xi"], tt["zeta"])
    u = dev(media.random_vector(4 * n, 3))
    outs, infos = [], []
    for pal in (1, 0):
        with nsf.Plan(grid, k) as P:
            P.set_option(nsf.NSF_OPT_MEDIUM_PALETTE, pal)
            (P.set_nfsep if which == "nfsep" else P.set_tensor)(*t)
            infos.append(P.medium_info())
            o = torch.empty_like(u)
            (P.K if which == "nfsep" else P.Ar)(u, o)
            outs.append(host(o))
    full = 576 if which == "nfsep" else 336
    assert infos[0] == {"palette": 2, "voxel_bytes": 2} and infos[1] == {"palette": 0, "voxel_bytes": full}
    assert np.array_equal(outs[0], outs[1])
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*media.random_nonhhpd(*grid, seed=2))
        assert P.medium_info() == {"palette": 0, "voxel_bytes": 576}


@pytest.mark.parametrize("grid,k", [((16, 16, 16), (0.1, 0.2, 0.3)), ((8, 12, 6), (0.3, 0.1, 0.2))])
def test_nfsep_factor_is_Ar_middle_for_hhpd_media(grid, k):
    """Under the assumption N = i J B^{-1} equals A_r's middle factor, so the
    NFSEP plan's A_r apply equals the chiral plan's (<= 1e-12)."""
    n = grid[0] * grid[1] * grid[2]
    eps, gam = media.sphere_chiral(*grid)
    t = medium.tensors_chiral(eps, gam)
    u = dev(media.random_vector(4 * n, 9))
    a = torch.empty_like(u)
    b = torch.empty_like(u)
    with nsf.Plan(grid, k) as P, nsf.Plan(grid, k) as Q:
        P.set_chiral(eps, gam)
        Q.set_nfsep(t["eps"], t["mu"], t["xi"], t["zeta"])
        P.Ar(u, a)
        Q.Ar(u, b)
        assert rel(host(b), host(a)) < 1e-12


def test_solve_matches_dense_4():
    grid, k = (4, 4, 4), (0.1, 0.2, 0.3)
    n = 64
    t = media.random_nonhhpd(*grid, seed=1)
    b = media.random_vector(4 * n, 4)
    ref = np.linalg.solve(nfsep.K_dense(grid, k, tens_of(t)), b)
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*t)
        x = torch.empty(4 * n, dtype=torch.complex128, device="cuda")
        st, it, rr = P.nfsep_solve(dev(b), x, rtol=1e-13)
        got = host(x)
    assert st == nsf.NSF_OK and rr <= 1e-13 and it > 0
    assert rel(got, ref) < 1e-10


@pytest.mark.parametrize("restart", [5, 40])
def test_solve_residual_32(restart):
    """K x = b at 32^3 for a lossy sphere: the oracle's matrix-free K applied to
    the GPU solution reproduces b (restarted and unrestarted GMRES)."""
    grid, k = (32, 32, 32), (0.1, 0.2, 0.3)
    n = 32 ** 3
    t = media.lossy_sphere_tensors(*grid)
    b = media.random_vector(4 * n, 6)
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*t)
        x = torch.empty(4 * n, dtype=torch.complex128, device="cuda")
        st, it, rr = P.nfsep_solve(dev(b), x, rtol=1e-11, restart=restart, maxit=5000)
        got = host(x)
    assert st == nsf.NSF_OK and rr <= 1e-11
    r = nfsep.apply_K(got, grid, k, tens_of(t)) - b
    s = np.sqrt(nfgep.sigma_r(grid, k))
    bound = 1e-11 * np.sqrt(s.max() / s.min())  # K = S'(iJ4) Kern S'
    assert np.linalg.norm(r) <= 2 * bound * np.linalg.norm(b)


@pytest.mark.parametrize("grid", [(4, 4, 4), (3, 4, 5)])
@pytest.mark.parametrize("kind", ["random", "lossy"])
def test_eigs_match_dense(grid, kind):
    k = (0.1, 0.2, 0.3)
    n = grid[0] * grid[1] * grid[2]
    t = medium_for(kind, grid)
    nev = 5
    ref = nfsep.smallest_positive(nfsep.eigs_dense(grid, k, tens_of(t)), nev)
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*t)
        Y = torch.empty(nev * 4 * n, dtype=torch.complex128, device="cuda")
        st, om, res, stats = P.eigs_nfsep(nev, res_tol=1e-11, inner_rtol=1e-13, max_basis=20, Y=Y)
        Yh = host(Y).reshape(nev, 4 * n)
    assert st == nsf.NSF_OK and res.max() <= 1e-11
    assert (np.abs(om - ref) <= 1e-10 * np.abs(ref)).all()
    for j in range(nev):  # the oracle's residual and Rayleigh quotient of the GPU pairs
        assert abs(np.linalg.norm(Yh[j]) - 1.0) < 1e-12
        assert nfsep.residual(Yh[j], om[j], grid, k, tens_of(t)) <= 1e-11
        assert abs(nfsep.rayleigh(Yh[j], grid, k, tens_of(t)) - om[j]) <= 1e-12 * abs(om[j])


def test_eigs_lossy_sphere_golden_16():
    g = json.load(open(os.path.join(HERE, "golden", "nfsep_lossy16.json")))
    grid, k = tuple(g["grid"]), tuple(g["k"])
    ref = np.array(g["omega_re"]) + 1j * np.array(g["omega_im"])
    nev = len(ref)
    t = media.lossy_sphere_tensors(*grid)
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*t)
        st, om, res, stats = P.eigs_nfsep(nev, res_tol=1e-10, inner_rtol=1e-12)
    assert st == nsf.NSF_OK and res.max() <= 1e-10
    assert (np.abs(om - ref) <= 1e-10 * np.abs(ref)).all()
    assert stats["cg_solves"] > 0 and stats["lanczos_steps"] >= nev


def test_eigs_hhpd_medium_agree_with_lanczos_16():
    """For a chiral medium the NFSEP operator is the invert Lanczos operator:
    the Arnoldi path and nsf_eigs give the same (real) eigenvalues."""
    grid, k = (16, 16, 16), (0.1, 0.2, 0.3)
    eps, gam = media.sphere_chiral(16)
    t = medium.tensors_chiral(eps, gam)
    nev = 6
    with nsf.Plan(grid, k) as P, nsf.Plan(grid, k) as Q:
        P.set_chiral(eps, gam)
        st, om, res, _ = P.eigs(nev, res_tol=1e-10, cg_rtol=1e-12)
        assert st == nsf.NSF_OK
        Q.set_nfsep(t["eps"], t["mu"], t["xi"], t["zeta"])
        st2, om2, res2, _ = Q.eigs_nfsep(nev, res_tol=1e-10, inner_rtol=1e-12)
    assert st2 == nsf.NSF_OK and res2.max() <= 1e-10
    assert (np.abs(om2.imag) <= 1e-10 * np.abs(om)).all()
    assert (np.abs(om2.real - om) <= 1e-10 * np.abs(om)).all()


def test_eigs_homogeneous_lossy_dielectric_closed_form_16():
    """Constant eps = 9 + 1.5i, mu = 1, no coupling: every eigenvalue is
    sigma_f / sqrt(eps) (twice, one per polarisation).  A single-vector Krylov
    method finds one direction of each double eigenvalue, so the returned values
    are closed-form values in ascending modulus, starting at the smallest."""
    grid, k = (16, 16, 16), (0.1, 0.2, 0.3)
    eps0 = 9.0 + 1.5j
    t = media.homogeneous_tensors(*grid, eps=eps0)
    L1, L2, L3 = yee.lambdas(grid, k)
    cf = np.sort_complex(np.sqrt(np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2) / np.sqrt(eps0))
    cf = cf[np.argsort(np.abs(cf))]
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*t)
        st, om, res, _ = P.eigs_nfsep(4, res_tol=1e-10, inner_rtol=1e-12)
    assert st == nsf.NSF_OK
    for w in om:
        assert np.abs(cf - w).min() <= 1e-10 * np.abs(cf).max()
    assert abs(om[0] - cf[0]) <= 1e-10 * abs(cf[0])
    assert np.all(np.diff(np.abs(om)) >= -1e-12)


def test_fields_of_nfsep_eigenpairs_solve_the_gep_6():
    """Algorithm 1, last step, for a medium outside the assumption: the fields
    B^{-1} diag(P_r, Q_r) x of the scaled eigenvectors solve diag(C, C^*) x =
    omega B x."""
    grid, k = (6, 6, 6), (0.1, 0.2, 0.3)
    n = 216
    t = media.lossy_sphere_tensors(*grid)
    nev = 4
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*t)
        Y = torch.empty(nev * 4 * n, dtype=torch.complex128, device="cuda")
        st, om, res, _ = P.eigs_nfsep(nev, res_tol=1e-11, inner_rtol=1e-13, Y=Y)
        assert st == nsf.NSF_OK
        eh = torch.empty(6 * n, dtype=torch.complex128, device="cuda")
        C = yee.C_matrix(grid, k)
        Bm = medium.B_matrix(tens_of(t))
        for j in range(nev):
            P.fields(Y[j * 4 * n:(j + 1) * 4 * n], eh)
            x = host(eh)
            lhs = np.concatenate([C @ x[:3 * n], C.conj().T @ x[3 * n:]])
            rhs = om[j] * (Bm @ x)
            assert np.linalg.norm(lhs - rhs) <= 1e-9 * np.linalg.norm(rhs)


def test_eigs_residuals_by_oracle_32():
    """32^3 non-reciprocal random medium: each returned pair checked one by one
    with the oracle's matrix-free K (residual and Rayleigh quotient)."""
    grid, k = (32, 32, 32), (0.3, 0.1, 0.2)
    n = 32 ** 3
    t = media.random_nonhhpd(*grid, seed=11)
    nev = 4
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*t)
        Y = torch.empty(nev * 4 * n, dtype=torch.complex128, device="cuda")
        st, om, res, stats = P.eigs_nfsep(nev, res_tol=1e-9, inner_rtol=1e-11, Y=Y)
        Yh = host(Y).reshape(nev, 4 * n)
    assert st == nsf.NSF_OK and res.max() <= 1e-9
    for j in range(nev):
        assert nfsep.residual(Yh[j], om[j], grid, k, tens_of(t)) <= 1.5e-9
        assert abs(nfsep.rayleigh(Yh[j], grid, k, tens_of(t)) - om[j]) <= 1e-12 * abs(om[j])
    assert np.all(om.real > 0) and np.all(np.diff(np.abs(om)) >= -1e-12)


def test_hhpd_solvers_reject_an_nfsep_medium():
    grid, k = (4, 4, 4), (0.1, 0.2, 0.3)
    t = media.random_nonhhpd(*grid, seed=1)
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*t)
        with pytest.raises(nsf.NsfError) as e:
            P.eigs(2)
        assert e.value.status == nsf.NSF_E_STATE
        b = torch.ones(256, dtype=torch.complex128, device="cuda")
        x = torch.empty_like(b)
        with pytest.raises(nsf.NsfError) as e:
            nsf.nsf_cg_solve(P.handle, b, x)
        assert e.value.status == nsf.NSF_E_STATE
    with nsf.Plan(grid, k) as P:
        P.set_chiral(*media.sphere_chiral(4))
        with pytest.raises(nsf.NsfError) as e:
            P.eigs_nfsep(2)
        assert e.value.status == nsf.NSF_E_STATE
