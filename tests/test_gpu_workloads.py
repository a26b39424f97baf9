"""GPU parity of the paper's own workloads and of the solver options around them.

* the chirality sweep of Sec. 5 (spheres joined by cylinders, k = (1/2, 0, 0),
  eps_i = 13 with gamma up to 3 and eps_i = 1 with gamma up to 0.9, where
  Phi = eps_i - gamma^2 approaches 0 and CG slows down) against the dense pencil;
* the band-structure media of Sec. 5, (eps_i, eps_o, gamma) = (13, 1, 0.5) and
  (1, 1, 0.8), at a generic k and at k-points of the G-X-M-R-G path;
* the relaxed inner CG tolerance (NSF_OPT_CG_RELAX) against fixed-tolerance solves;
* batch instances chained along a k-path (NSF_OPT_WARM_CHAIN) against cold solves;
* multiple eigenvalues (air at a k on a lattice axis): every copy from the batch
  path and from the differentiable wrapper, and with default options only true
  eigenvalues.

Eigenvalues are compared one by one, relative to each eigenvalue.
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


def close(om, ref, tol=1e-10):
    om, ref = np.asarray(om), np.asarray(ref)
    return om.shape == ref.shape and bool((np.abs(om - ref) <= tol * np.abs(ref)).all())


def dense_smallest(grid, k, eps, gam, nev):
    w = nfgep.nfgep_dense(grid, k, medium.tensors_chiral(eps, gam))
    return np.sort(w[w > 0])[:nev]


@pytest.mark.parametrize("eps_i,gamma", [(13.0, 3.0), (1.0, 0.9), (13.0, 0.25), (1.0, 0.05)])
def test_gamma_sweep_matches_dense_8(eps_i, gamma):
    grid, k = (8, 8, 8), (0.5, 0.0, 0.0)
    eps, gam = media.spheres_cylinders_chiral(8, eps_in=eps_i, eps_out=1.0, gamma=gamma)
    ref = dense_smallest(grid, k, eps, gam, 10)
    with nsf.Plan(grid, k) as P:
        P.set_chiral(eps, gam)
        P.set_option(nsf.NSF_OPT_VERIFY, 16)  # k on a lattice axis of a cubic structure
        st, om, res, stats = P.eigs(10, res_tol=1e-10, cg_rtol=1e-12)
    assert st == nsf.NSF_OK and res.max() <= 1e-10
    assert close(om, ref), (om, ref)


def test_gamma_sweep_cg_slows_as_phi_vanishes_16():
    """Sec. 5: the condition number of the linear systems grows without bound as gamma
    approaches sqrt(eps_i); the average CG iterations per solve grow with gamma."""
    grid, k = (16, 16, 16), (0.5, 0.0, 0.0)
    its = []
    for gamma in (0.05, 0.6, 0.9):
        eps, gam = media.spheres_cylinders_chiral(16, eps_in=1.0, eps_out=1.0, gamma=gamma)
        with nsf.Plan(grid, k) as P:
            P.set_chiral(eps, gam)
            st, om, res, stats = P.eigs(10, res_tol=1e-8, cg_rtol=1e-10)
        assert st == nsf.NSF_OK and res.max() <= 1e-8
        its.append(stats["cg_iters_avg"])
    assert its[0] < its[1] < its[2], its


@pytest.mark.parametrize("eps_i,eps_o,gamma", [(13.0, 1.0, 0.5), (1.0, 1.0, 0.8)])
@pytest.mark.parametrize("k", [(0.1, 0.2, 0.3), (0.25, 0.0, 0.0), (0.5, 0.25, 0.0), (0.5, 0.5, 0.35)],
                         ids=["generic", "G-X", "X-M", "M-R"])
def test_band_structure_media_match_dense_8(eps_i, eps_o, gamma, k):
    grid = (8, 8, 8)
    eps, gam = media.spheres_cylinders_chiral(8, eps_in=eps_i, eps_out=eps_o, gamma=gamma)
    ref = dense_smallest(grid, k, eps, gam, 10)
    with nsf.Plan(grid, k) as P:
        P.set_chiral(eps, gam)
        P.set_option(nsf.NSF_OPT_VERIFY, 16)
        st, om, res, stats = P.eigs(10, res_tol=1e-10, cg_rtol=1e-12)
    assert st == nsf.NSF_OK and res.max() <= 1e-10
    assert close(om, ref), (om, ref)


@pytest.mark.parametrize("case", ["sphere16", "rods16", "scsc16_eps1_g09", "rods16_next_to_gamma"])
def test_relaxed_inner_tolerance_same_eigenpairs(case):
    grid = (16, 16, 16)
    if case == "sphere16":
        k, (eps, gam), pair = (0.1, 0.2, 0.3), media.sphere_chiral(16), None
    elif case.startswith("rods16"):
        k = (0.1, 0.2, 0.3) if case == "rods16" else (0.025, 0.0, 0.0)
        (eps, gam), pair = media.rods_pseudochiral(16, radius=0.3), (0, 1)
    else:
        k, pair = (0.5, 0.0, 0.0), None
        eps, gam = media.spheres_cylinders_chiral(16, eps_in=1.0, eps_out=1.0, gamma=0.9)
    out = {}
    for relax in (0, 1):
        with nsf.Plan(grid, k) as P:
            if pair:
                P.set_pseudochiral(*pair, eps, gam)
            else:
                P.set_chiral(eps, gam)
            P.set_option(nsf.NSF_OPT_CG_RELAX, relax)
            out[relax] = P.eigs(10, res_tol=1e-8, cg_rtol=1e-10)
    (st0, om0, r0, s0), (st1, om1, r1, s1) = out[0], out[1]
    assert st0 == st1 == nsf.NSF_OK
    assert r0.max() <= 1e-8 and r1.max() <= 1e-8
    assert close(om1, om0)
    assert s1["cg_iters_total"] <= s0["cg_iters_total"]


def test_relaxed_inner_tolerance_batch_matches_plain():
    grids = [(16, 16, 16), (16, 16, 16), (12, 12, 12)]
    ks = [(0.1, 0.2, 0.3), (0.3, 0.1, 0.0), (0.2, 0.2, 0.2)]
    meds = [media.sphere_chiral(g[0]) for g in grids]
    with nsf.Batch(grids, ks) as B:
        for i, (e, g) in enumerate(meds):
            B.set_chiral(i, e, g)
            nsf.nsf_plan_set_option(B.plan(i), nsf.NSF_OPT_CG_RELAX, 1)
        st, om, res, stats, _ = B.eigs(8, res_tol=1e-8, cg_rtol=1e-10)
    assert st == nsf.NSF_OK and res.max() <= 1e-8
    for i, (g, k, (e, gm)) in enumerate(zip(grids, ks, meds)):
        with nsf.Plan(g, k) as P:
            P.set_chiral(e, gm)
            P.set_option(nsf.NSF_OPT_CG_RELAX, 0)
            st1, om1, _, _ = P.eigs(8, res_tol=1e-8, cg_rtol=1e-10)
        assert st1 == nsf.NSF_OK and close(om[i], om1)


def test_warm_chain_batch_matches_cold_solves():
    """Three consecutive k-points of the 128^3 rods path (each 128^3 instance runs
    in a wave of its own): with NSF_OPT_WARM_CHAIN the second and third start from
    their predecessor's Ritz vectors, reach the same eigenvalues as cold plain
    solves and take fewer Lanczos steps."""
    g, nev = (128, 128, 128), 10
    ks = [tuple(k) for k in media.kpath_gxmgr(10)[14:17]]
    eps, gam = media.rods_pseudochiral(128)
    kw = dict(res_tol=1e-8, cg_rtol=1e-10, seed=0)
    with nsf.Batch([g] * 3, ks) as B:
        for i in range(3):
            B.set_pseudochiral(i, 0, 1, eps, gam)
            nsf.nsf_plan_set_option(B.plan(i), nsf.NSF_OPT_WARM_CHAIN, int(i > 0))
        st, om, res, stats, wave = B.eigs(nev, **kw)
    assert st == nsf.NSF_OK and res.max() <= 1e-8 and wave == 1
    for i, k in enumerate(ks):
        with nsf.Plan(g, k) as P:
            P.set_pseudochiral(0, 1, eps, gam)
            st1, om1, _, s1 = P.eigs(nev, **kw)
        assert st1 == nsf.NSF_OK and close(om[i], om1, 1e-9), (i, om[i], om1)
        if i == 0:
            assert stats[0]["lanczos_steps"] == s1["lanczos_steps"]  # same cold start
        else:
            assert stats[i]["lanczos_steps"] < s1["lanczos_steps"], (stats[i], s1)


# ------------------------------------------------------- multiple eigenvalues

def _air_reference(grid, k, count):
    L1, L2, L3 = yee.lambdas(grid, k)
    sig = np.sqrt(np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2)
    return np.sort(np.concatenate([sig, sig]))[:count]


def test_air_default_options_return_true_eigenvalues():
    """Without the multiplicity check a multiple eigenvalue may appear fewer times than
    it occurs; every returned value is still a converged, true eigenvalue."""
    grid, k = (8, 8, 8), (0.1, 0.0, 0.0)
    eps, gam = media.homogeneous(8, eps=1.0, gamma=0.0)
    L1, L2, L3 = yee.lambdas(grid, k)
    sig = np.unique(np.round(np.sqrt(np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2), 12))
    with nsf.Plan(grid, k) as P:
        P.set_chiral(eps, gam)
        st, om, res, _ = P.eigs(12, res_tol=1e-10, cg_rtol=1e-12)
    assert st == nsf.NSF_OK and res.max() <= 1e-10
    for w in om:
        assert np.abs(sig - w).min() <= 1e-10 * w


def test_air_batch_with_checks_returns_every_copy():
    grid = (8, 8, 8)
    ks = [(0.1, 0.0, 0.0), (0.0, 0.2, 0.0)]
    eps, gam = media.homogeneous(8, eps=1.0, gamma=0.0)
    with nsf.Batch([grid] * 2, ks) as B:
        for i in range(2):
            B.set_chiral(i, eps, gam)
            nsf.nsf_plan_set_option(B.plan(i), nsf.NSF_OPT_VERIFY, 16)
        st, om, res, stats, _ = B.eigs(12, res_tol=1e-10, cg_rtol=1e-12)
    assert st == nsf.NSF_OK and res.max() <= 1e-10
    for i, k in enumerate(ks):
        ref = _air_reference(grid, k, 12)
        assert np.sum(np.isclose(ref, ref[0], rtol=1e-12)) >= 2
        assert close(om[i], ref), (om[i], ref)


def test_autograd_forward_returns_every_copy():
    from paper_1402_6297_amd import autograd

    grid, k = (8, 8, 8), (0.1, 0.0, 0.0)
    eps, gam = media.homogeneous(8, eps=1.0, gamma=0.0)
    ref = _air_reference(grid, k, 14)
    assert ref[12] == ref[13]  # a double eigenvalue straddles the cut at 13
    e = torch.from_numpy(eps).to("cuda").requires_grad_(True)
    g = torch.from_numpy(gam).to("cuda").requires_grad_(True)
    om = autograd.eigenvalues(e, g, grid, k, 12, res_tol=1e-10, cg_rtol=1e-12)
    assert close(om.detach().cpu().numpy(), ref[:12])
    with pytest.warns(RuntimeWarning, match="not differentiable"):
        om = autograd.eigenvalues(e, g, grid, k, 13, res_tol=1e-10, cg_rtol=1e-12)
    assert close(om.detach().cpu().numpy(), ref[:13])


def test_autograd_backward_twice_with_retained_graph():
    from paper_1402_6297_amd import autograd

    grid, k = (6, 6, 6), (0.1, 0.2, 0.3)
    eps, gam = media.noise_chiral(6, sigma_vox=1.0, seed=7)
    e = torch.from_numpy(eps).to("cuda").requires_grad_(True)
    g = torch.from_numpy(gam).to("cuda").requires_grad_(True)
    om = autograd.eigenvalues(e, g, grid, k, 3, res_tol=1e-11, cg_rtol=1e-13)
    om.sum().backward(retain_graph=True)
    g1 = e.grad.clone()
    e.grad = None
    om.sum().backward()
    assert torch.equal(e.grad, g1)
