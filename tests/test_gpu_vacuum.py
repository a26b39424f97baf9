"""Vacuum skipping (NSF_OPT_VACUUM = 1, the default).

In a pencil column where every voxel is vacuum (eps 1, gamma 0) the middle factor
is the identity, so the z pass leaves such columns out, and the y passes leave
out groups of x with no other voxel.  Checked here: the apply
with and without skipping on chiral and pseudochiral media at every z-pass
tiling, against the oracle; air (every column skipped: A_r = I); a medium
without vacuum; CG, eigensolves and a shared batch whose instances list
different numbers of tiles.
"""
import numpy as np
import pytest

from oracle import medium, nfgep, yee
from paper_1402_6297_amd import media, nsf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _plan(grid, k, kind, eps, gam, vac, mid=None, yz=None):
    P = nsf.Plan(grid, k)
    if kind == "chiral":
        P.set_chiral(eps, gam)
    else:
        P.set_pseudochiral(*kind, eps, gam)
    P.set_option(nsf.NSF_OPT_VACUUM, vac)
    if mid:
        P.set_option(nsf.NSF_OPT_MID_COLS, mid)
    if yz:
        P.set_option(nsf.NSF_OPT_YZ_COLS, yz)
    return P


@pytest.mark.parametrize("kind", ["chiral", (0, 1), (0, 2), (1, 2)])
@pytest.mark.parametrize("mid,yz", [(1, 16), (4, 2), (16, 8), (16, 16), (2, 1)])
def test_apply_with_and_without_skipping_32(kind, mid, yz):
    grid, k = (32, 32, 32), (0.1, 0.2, 0.3)
    n = 32 ** 3
    if kind == "chiral":
        eps, gam = media.sphere_chiral(32)
        tens = medium.tensors_chiral(eps, gam)
    else:
        eps, gam = media.rods_pseudochiral(32, radius=0.3)
        tens = medium.tensors_pseudochiral(eps, gam, kind)
    u = torch.from_numpy(media.random_vector(4 * n, 11)).to("cuda")
    outs = []
    for vac in (1, 0):
        with _plan(grid, k, kind, eps, gam, vac, mid, yz) as P:
            out = torch.empty_like(u)
            P.Ar(u, out)
            outs.append(host(out))
    assert rel(outs[0], outs[1]) <= 1e-14
    ref = nfgep.apply_Ar(host(u), grid, k, tens)
    assert rel(outs[0], ref) <= 1e-12


def test_air_is_identity_and_no_vacuum_is_unchanged_16():
    grid, k = (16, 16, 16), (0.1, 0.2, 0.3)
    n = 16 ** 3
    u = torch.from_numpy(media.random_vector(4 * n, 2)).to("cuda")
    eps, gam = media.homogeneous(16, eps=1.0, gamma=0.0)
    with _plan(grid, k, "chiral", eps, gam, 1) as P:
        out = torch.empty_like(u)
        P.Ar(u, out)
        assert rel(host(out), host(u)) <= 1e-14
    eps, gam = media.homogeneous(16, eps=2.0, gamma=0.5)
    outs = []
    for vac in (1, 0):
        with _plan(grid, k, "chiral", eps, gam, vac) as P:
            out = torch.empty_like(u)
            P.Ar(u, out)
            outs.append(host(out))
    assert rel(outs[0], outs[1]) <= 1e-14


def test_cg_and_eigs_with_and_without_skipping_32():
    grid, k = (32, 32, 32), (0.1, 0.2, 0.3)
    n = 32 ** 3
    eps, gam = media.sphere_chiral(32)
    b = torch.from_numpy(media.random_vector(4 * n, 4)).to("cuda")
    res = {}
    for vac in (1, 0):
        with _plan(grid, k, "chiral", eps, gam, vac) as P:
            x = torch.empty_like(b)
            st, it, relres = P.cg(b, x, rtol=1e-12, maxit=2000)
            assert st == nsf.NSF_OK and relres <= 1e-12
            st, om, rs, stats = P.eigs(10, res_tol=1e-10, cg_rtol=1e-12)
            assert st == nsf.NSF_OK and rs.max() <= 1e-10
            res[vac] = (host(x), it, om)
    assert abs(res[1][1] - res[0][1]) <= 1
    assert rel(res[1][0], res[0][0]) <= 1e-10
    assert np.all(np.abs(res[1][2] - res[0][2]) <= 1e-10 * res[0][2])
    tens = medium.tensors_chiral(eps, gam)
    r = host(b) - nfgep.apply_Ar(res[1][0], grid, k, tens)
    assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(host(b))


def test_shared_batch_with_air_and_spheres_16():
    """One shared wave of 16^3 instances listing 0 (air) to many tiles."""
    grid = (16, 16, 16)
    ks = [(0.1, 0.2, 0.3), (0.3, 0.1, 0.2), (0.2, 0.2, 0.1)]
    meds = [media.homogeneous(16, eps=1.0, gamma=0.0), media.sphere_chiral(16), media.sphere_chiral(16, radius=0.45)]
    kw = dict(res_tol=1e-10, cg_rtol=1e-12)
    with nsf.Batch([grid] * 3, ks) as B:
        for i, (e, g) in enumerate(meds):
            B.set_chiral(i, e, g)
        st, om, res, stats, wave = B.eigs(6, **kw)
    assert st == nsf.NSF_OK and res.max() <= 1e-10 and wave == 3
    L1, L2, L3 = yee.lambdas(grid, ks[0])  # air: omega = |lambda| of some frequency
    sig = np.sqrt(np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2).ravel()
    assert np.all(np.min(np.abs(om[0][:, None] - sig[None, :]), axis=1) <= 1e-10 * om[0])
    for i in (1, 2):
        with _plan(grid, ks[i], "chiral", *meds[i], 0) as P:
            st1, om1, _, _ = P.eigs(6, **kw)
        assert st1 == nsf.NSF_OK
        assert np.all(np.abs(om[i] - om1) <= 1e-10 * om1)


def test_shared_batch_pseudochiral_rods_16():
    """Pseudochiral rods of different radii sharing launches, against plain solves
    without skipping."""
    grid = (16, 16, 16)
    ks = [(0.1, 0.2, 0.3), (0.3, 0.1, 0.2), (0.2, 0.05, 0.1)]
    meds = [media.rods_pseudochiral(16, radius=r) for r in (0.15, 0.25, 0.35)]
    kw = dict(res_tol=1e-10, cg_rtol=1e-12)
    with nsf.Batch([grid] * 3, ks) as B:
        for i, (e, g) in enumerate(meds):
            B.set_pseudochiral(i, 0, 1, e, g)
        st, om, res, stats, wave = B.eigs(6, **kw)
    assert st == nsf.NSF_OK and res.max() <= 1e-10 and wave == 3
    for i in range(3):
        with _plan(grid, ks[i], (0, 1), *meds[i], 0) as P:
            st1, om1, _, _ = P.eigs(6, **kw)
        assert st1 == nsf.NSF_OK
        assert np.all(np.abs(om[i] - om1) <= 1e-10 * om1)
