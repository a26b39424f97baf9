"""nsf_cg_solve_noalloc (CG vectors in the library's static device array) against
nsf_cg_solve on two calls in a row, the second on a smaller grid: same iteration
count and the same solution (bit for bit: the same kernels run in the same order),
and a true residual checked by the oracle's A_r."""
import numpy as np
import pytest

from oracle import medium, nfgep
from paper_1402_6297_amd import media, nsf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _solve_both(grid, k, kind, seed):
    n = grid[0] * grid[1] * grid[2]
    b = media.random_vector(4 * n, seed)
    if kind == "chiral":
        eps, gam = media.sphere_chiral(*grid)
        tens = medium.tensors_chiral(eps, gam)
    else:
        eps, gam = media.rods_pseudochiral(*grid, radius=0.3)
        tens = medium.tensors_pseudochiral(eps, gam, (0, 1))
    bd = torch.from_numpy(b).to("cuda")
    with nsf.Plan(grid, k) as P:
        if kind == "chiral":
            P.set_chiral(eps, gam)
        else:
            P.set_pseudochiral(0, 1, eps, gam)
        x0 = torch.full((4 * n,), 7.0 + 1j, dtype=torch.complex128, device="cuda")  # overwritten
        st0, it0, rel0 = P.cg_noalloc(bd, x0, rtol=1e-10)
        x1 = torch.empty_like(x0)
        st1, it1, rel1 = P.cg(bd, x1, rtol=1e-10)
        torch.cuda.synchronize()
    assert st0 == st1 == nsf.NSF_OK
    assert it0 == it1 and rel0 == rel1
    xa, xb = x0.cpu().numpy(), x1.cpu().numpy()
    assert np.array_equal(xa, xb)
    r = b - nfgep.apply_Ar(xa, grid, k, tens)
    assert np.linalg.norm(r) <= 10 * 1e-10 * np.linalg.norm(b)
    return it0


def test_noalloc_cg_matches_cg_on_two_calls_second_smaller():
    it_big = _solve_both((64, 32, 32), (0.1, 0.2, 0.3), "chiral", 21)  # the largest grid it takes
    it_small = _solve_both((16, 16, 12), (0.3, 0.1, 0.2), "pseudo", 22)
    assert it_big > 0 and it_small > 0


def test_noalloc_cg_rejects_larger_grids_and_missing_media():
    with nsf.Plan((64, 64, 32), (0.1, 0.2, 0.3)) as P:
        P.set_chiral(*media.sphere_chiral(64, 64, 32))
        b = torch.ones(4 * P.n, dtype=torch.complex128, device="cuda")
        x = torch.empty_like(b)
        with pytest.raises(nsf.NsfError) as e:
            P.cg_noalloc(b, x)
        assert e.value.status == nsf.NSF_E_ARG
    with nsf.Plan((16, 16, 16), (0.1, 0.2, 0.3)) as P:
        b = torch.ones(4 * P.n, dtype=torch.complex128, device="cuda")
        with pytest.raises(nsf.NsfError) as e:
            P.cg_noalloc(b, torch.empty_like(b))
        assert e.value.status == nsf.NSF_E_STATE
