"""CPU-only checks of the C ABI: the library loads, exports every declared
symbol, and its host-only paths (plan validation, the dense Hermitian
eigensolver) behave.  No call here touches a GPU."""
import os
import re

import numpy as np
import pytest

from paper_1402_6297_amd import nsf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nsf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nsf_[a-zA-Z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = nsf.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert sorted(nsf.EXPORTED) == names


def test_plan_create_valid_and_query():
    p = nsf.nsf_plan_create(16, 16, 16, 1.0, (0.1, 0.2, 0.3), stream=0)
    q = nsf.nsf_plan_query(p)
    assert q["n"] == 4096 and q["medium_kind"] == 0
    # sigma_f = ||lambda_f||, per-axis minima add up
    lam = [np.abs((np.exp(2j * np.pi * (np.arange(16) + k) / 16) - 1) * 16) for k in (0.1, 0.2, 0.3)]
    assert abs(q["sigma_min"] - np.sqrt(sum(l.min() ** 2 for l in lam))) < 1e-12 * q["sigma_max"]
    assert abs(q["sigma_max"] - np.sqrt(sum(l.max() ** 2 for l in lam))) < 1e-12 * q["sigma_max"]
    nsf.nsf_plan_destroy(p)


@pytest.mark.parametrize("args,code", [
    ((16, 16, 16, 1.0, (0.0, 0.0, 0.0)), nsf.NSF_E_KPOINT),        # Gamma point
    ((16, 16, 16, 1.0, (1.0, 2.0, -1.0)), nsf.NSF_E_KPOINT),       # integer k is Gamma too
    ((7, 16, 16, 1.0, (0.1, 0.2, 0.3)), nsf.NSF_E_ARG),            # prime factor 7
    ((1024, 2, 2, 1.0, (0.1, 0.2, 0.3)), nsf.NSF_E_ARG),           # too long an axis
    ((1, 16, 16, 1.0, (0.1, 0.2, 0.3)), nsf.NSF_E_ARG),
    ((0, 16, 16, 1.0, (0.1, 0.2, 0.3)), nsf.NSF_E_ARG),            # empty grid
    ((16, -4, 16, 1.0, (0.1, 0.2, 0.3)), nsf.NSF_E_ARG),
    ((16, 16, 16, -1.0, (0.1, 0.2, 0.3)), nsf.NSF_E_ARG),
    ((16, 16, 16, 1.0, (float("nan"), 0.2, 0.3)), nsf.NSF_E_ARG),
])
def test_plan_create_rejects(args, code):
    with pytest.raises(nsf.NsfError) as e:
        nsf.nsf_plan_create(*args, stream=0)
    assert e.value.status == code


def test_plan_create_rejects_rank_deficient_basis():
    # a = (1, 1, 1) with k = (t, t, t) on a cube: lambda is parallel to a at f = 0.
    with pytest.raises(nsf.NsfError) as e:
        nsf.nsf_plan_create(8, 8, 8, 1.0, (0.1, 0.1, 0.1), alpha=1.0, beta=1.0, stream=0)
    assert e.value.status == nsf.NSF_E_BASIS
    with pytest.raises(nsf.NsfError):
        nsf.nsf_plan_create(8, 8, 8, 1.0, (0.1, 0.1, 0.1), alpha=0.0, beta=1.0, stream=0)


def test_medium_validation_on_host():
    p = nsf.nsf_plan_create(4, 4, 4, 1.0, (0.1, 0.2, 0.3), stream=0)
    eps = np.full(64, 13.0)
    gam = np.full(64, 0.5)
    gam[5] = 4.0  # gamma^2 > eps: Phi not positive
    with pytest.raises(nsf.NsfError) as e:
        nsf.nsf_set_medium_chiral(p, eps, gam)
    assert e.value.status == nsf.NSF_E_NOT_HHPD
    assert "voxel 5" in nsf.nsf_last_error(p)
    gam[5] = np.nan
    with pytest.raises(nsf.NsfError) as e:
        nsf.nsf_set_medium_pseudochiral(p, 0, 1, eps, gam)
    assert e.value.status == nsf.NSF_E_ARG
    with pytest.raises(nsf.NsfError) as e:
        nsf.nsf_set_medium_pseudochiral(p, 1, 1, eps, np.zeros(64))
    assert e.value.status == nsf.NSF_E_ARG
    nsf.nsf_plan_destroy(p)


def test_binding_rejects_wrong_medium_sizes_before_the_call():
    """Host media must hold exactly n voxels (the C call reads n of each)."""
    p = nsf.nsf_plan_create(4, 4, 4, 1.0, (0.1, 0.2, 0.3), stream=0)
    eps, gam = np.full(64, 13.0), np.full(64, 0.5)
    for bad in ((eps[:63], gam), (eps, np.zeros(65))):
        with pytest.raises(ValueError):
            nsf.nsf_set_medium_chiral(p, *bad)
        with pytest.raises(ValueError):
            nsf.nsf_set_medium_pseudochiral(p, 0, 1, *bad)
    t = [np.zeros((63, 3, 3), np.complex128)] * 4
    with pytest.raises(ValueError):
        nsf.nsf_set_medium_tensor(p, *t)
    with pytest.raises(ValueError):
        nsf.nsf_set_medium_nfsep(p, *t)
    try:  # the right sizes pass the binding and reach the library (which needs a device)
        nsf.nsf_set_medium_chiral(p, eps, gam)
    except nsf.NsfError as e:
        assert e.status == nsf.NSF_E_HIP
    nsf.nsf_plan_destroy(p)


@pytest.mark.parametrize("m", [1, 2, 7, 30])
def test_hermitian_eig_matches_lapack(m):
    rng = np.random.default_rng(m)
    X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    H = X + X.conj().T
    w, V = nsf.nsf_hermitian_eig(H)
    ref = np.linalg.eigvalsh(H)
    assert np.abs(w - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(V.conj().T @ V - np.eye(m)).max() < 1e-12
    assert np.abs(H @ V - V * w[None, :]).max() < 1e-11 * np.abs(ref).max()


def test_status_strings():
    assert nsf.nsf_status_string(0) == "ok"
    assert "CG" in nsf.nsf_status_string(nsf.NSF_E_BREAKDOWN)


@pytest.mark.parametrize("option,good,bad", [
    (nsf.NSF_OPT_FFT_PATH, [0, 1, 2], [-1, 3]),
    (nsf.NSF_OPT_MID_COLS, [1, 2, 4, 8, 16], [0, 3, 32]),
    (nsf.NSF_OPT_CG_GRAPH, [0, 1], [-1, 2]),
    (nsf.NSF_OPT_X_ROWS, [1, 2, 4], [0, 3, 8]),
    (nsf.NSF_OPT_YZ_COLS, [1, 2, 4, 8, 16], [0, 6, 32]),
    (nsf.NSF_OPT_MID_PAIRS, [0, 1], [-1, 2]),
    (nsf.NSF_OPT_CG_START, [0, 1], [-1, 2]),
    (nsf.NSF_OPT_VERIFY, [0, 1, 16], [-1, 17]),
    (nsf.NSF_OPT_ORTHO_GATE, [0, 1], [-1, 2]),
    (nsf.NSF_OPT_GMRES_RESTART, [4, 40, 500], [3, 501]),
    (nsf.NSF_OPT_CG_RELAX, [0, 1], [-1, 2]),
    (nsf.NSF_OPT_WARM_CHAIN, [0, 1], [-1, 2]),
    (nsf.NSF_OPT_CG_RING, [0, 1], [-1, 2]),
    (nsf.NSF_OPT_VACUUM, [0, 1], [-1, 2]),
    (nsf.NSF_OPT_MEDIUM_PALETTE, [0, 1], [-1, 2]),
])
def test_plan_options_validate(option, good, bad):
    p = nsf.nsf_plan_create(8, 8, 8, 1.0, (0.1, 0.2, 0.3), stream=0)
    try:
        for v in good:
            assert nsf.nsf_plan_set_option(p, option, v) == nsf.NSF_OK
        for v in bad:
            with pytest.raises(nsf.NsfError) as e:
                nsf.nsf_plan_set_option(p, option, v)
            assert e.value.status == nsf.NSF_E_ARG
        with pytest.raises(nsf.NsfError):
            nsf.nsf_plan_set_option(p, 99, 0)
    finally:
        nsf.nsf_plan_destroy(p)


def test_autotune_needs_a_medium():
    p = nsf.nsf_plan_create(8, 8, 8, 1.0, (0.1, 0.2, 0.3), stream=0)
    try:
        with pytest.raises(nsf.NsfError) as e:
            nsf.nsf_plan_autotune(p, 3)
        assert e.value.status == nsf.NSF_E_STATE
        with pytest.raises(nsf.NsfError) as e:
            nsf.nsf_plan_autotune(p, 0)
        assert e.value.status == nsf.NSF_E_ARG
    finally:
        nsf.nsf_plan_destroy(p)


@pytest.mark.parametrize("breaker,msg", [
    ("mu_indefinite", "mu is not positive definite"),
    ("zeta_not_adjoint", "zeta differs from xi"),
    ("phi_indefinite", "Phi = eps - xi mu^-1 zeta is not positive definite"),
    ("eps_not_hermitian", "eps is not Hermitian"),
])
def test_general_medium_validation(breaker, msg):
    from paper_1402_6297_amd import media

    eps, mu, xi, zeta = media.random_general(4, seed=1)
    g = 13
    if breaker == "mu_indefinite":
        mu[g] = -np.eye(3)
    elif breaker == "zeta_not_adjoint":
        zeta[g, 0, 1] += 1e-6
    elif breaker == "phi_indefinite":
        xi[g] = 3.0 * np.eye(3)
        zeta[g] = 3.0 * np.eye(3)
    else:
        eps[g, 0, 1] += 0.5j
    p = nsf.nsf_plan_create(4, 4, 4, 1.0, (0.1, 0.2, 0.3), stream=0)
    try:
        with pytest.raises(nsf.NsfError) as e:
            nsf.nsf_set_medium_tensor(p, eps, mu, xi, zeta)
        assert e.value.status == nsf.NSF_E_NOT_HHPD
        assert msg in str(e.value) and f"voxel {g}" in str(e.value)
    finally:
        nsf.nsf_plan_destroy(p)


def test_workspace_size_and_validation():
    import ctypes

    p = nsf.nsf_plan_create(8, 8, 8, 1.0, (0.1, 0.2, 0.3), stream=0)
    try:
        n = 512
        b4 = nsf.nsf_plan_workspace_size(p, 4)
        b10 = nsf.nsf_plan_workspace_size(p, 10)
        b10m = nsf.nsf_plan_workspace_size(p, 10, max_basis=60)
        # fields 6n + CG 24n + basis 2 (m+1) 4n complex values, m = max(3 nev, nev + 8)
        assert b4 >= 16 * n * (6 + 24 + 2 * 13 * 4) and b10 > b4 and b10m > b10
        # too small for fields + CG + a 2-vector basis: refused before any device use
        assert nsf.lib().nsf_plan_set_workspace(p, ctypes.c_void_p(0x100000), 1024) == nsf.NSF_E_ARG
        with pytest.raises(nsf.NsfError):
            nsf.nsf_plan_workspace_size(p, 0)
    finally:
        nsf.nsf_plan_destroy(p)


def _key_order_ok(d):
    """Positive real part first, then descending modulus."""
    for a, b in zip(d[:-1], d[1:]):
        pa, pb = a.real > 0, b.real > 0
        if pa != pb:
            if not pa:
                return False
        elif abs(a) < abs(b) * (1 - 1e-12):
            return False
    return True


@pytest.mark.parametrize("m,kind", [(1, "random"), (2, "random"), (9, "random"), (30, "random"),
                                    (24, "hermitian"), (16, "normal_pairs"), (40, "hessenberg_plus_row")])
def test_schur_sorted_matches_lapack(m, kind):
    """The host Schur form of the NFSEP eigensolver: A = Z T Z^*, Z unitary, T
    upper triangular with LAPACK's eigenvalues on its diagonal, in the wanted
    order; the shapes include the restarted Krylov-Schur matrix (triangular
    block plus one full row) and a spectrum of +- pairs."""
    rng = np.random.default_rng(m)
    X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    if kind == "hermitian":
        A = X + X.conj().T
    elif kind == "normal_pairs":
        w = rng.standard_normal(m // 2) + 0.1j * rng.standard_normal(m // 2)
        Q, _ = np.linalg.qr(X)
        A = Q @ np.diag(np.concatenate([w, -w])) @ Q.conj().T
    elif kind == "hessenberg_plus_row":
        A = np.triu(X, -1)
        k = m // 2
        A[:k, :k] = np.triu(A[:k, :k])
        A[k, :k] = rng.standard_normal(k)
    else:
        A = X
    T, Z = nsf.nsf_schur_sorted(A)
    scale = np.abs(A).max()
    assert np.abs(np.tril(T, -1)).max(initial=0.0) == 0.0
    assert np.abs(Z.conj().T @ Z - np.eye(m)).max() < 1e-12
    assert np.abs(Z @ T @ Z.conj().T - A).max() < 1e-12 * m * scale
    d = np.diag(T)
    ref = list(np.linalg.eigvals(A))
    for x in d:
        j = int(np.argmin([abs(x - y) for y in ref]))
        assert abs(x - ref[j]) < 1e-9 * scale
        ref.pop(j)
    assert _key_order_ok(d)


@pytest.mark.parametrize("breaker,msg", [("singular", "is singular at voxel"),
                                         ("nonfinite", "non-finite value at voxel")])
def test_nfsep_medium_validation(breaker, msg):
    from paper_1402_6297_amd import media

    eps, mu, xi, zeta = media.random_nonhhpd(4, seed=2)
    g = 21
    if breaker == "singular":  # B = i [[0, 0], [-eps, 0]]
        mu[g] = 0.0
        xi[g] = 0.0
        zeta[g] = 0.0
    else:
        xi[g, 1, 2] = np.nan
    p = nsf.nsf_plan_create(4, 4, 4, 1.0, (0.1, 0.2, 0.3), stream=0)
    try:
        with pytest.raises(nsf.NsfError) as e:
            nsf.nsf_set_medium_nfsep(p, eps, mu, xi, zeta)
        assert e.value.status == nsf.NSF_E_ARG
        assert msg in str(e.value) and f"voxel {g}" in str(e.value)
        with pytest.raises(nsf.NsfError) as e:
            nsf.nsf_eigs_nfsep(p, 4)
        assert e.value.status == nsf.NSF_E_STATE
    finally:
        nsf.nsf_plan_destroy(p)


def test_cg_noalloc_rejects_grids_above_its_scratch_before_any_device_call():
    import ctypes as C

    p = nsf.nsf_plan_create(64, 64, 32, 1.0, (0.1, 0.2, 0.3), stream=0)  # 131072 voxels
    try:
        it, rel = C.c_int(), C.c_double()
        st = nsf.lib().nsf_cg_solve_noalloc(p, C.c_void_p(256), C.c_void_p(512), 1e-10, 100,
                                            C.byref(it), C.byref(rel))
        assert st == nsf.NSF_E_ARG
        assert "65536" in nsf.nsf_last_error(p)
    finally:
        nsf.nsf_plan_destroy(p)
