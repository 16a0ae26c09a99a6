"""The paper's accuracy experiment on the GPU path (Sec. 5.2, Experiment III): 2D
unit square, absorption 0.2, scattering 2, grids h = 1/(24 (2k - 1)) whose cell
centres at k = 1 are shared by every grid, errors against the finest grid's
solution on those points.  The paper finds (M-iii) first order and (M-ii) close to
second order on such grids (eq. EQ: ERROR gives O(h) and O(h^2 (1 + log h))); its
source is a figure only, a smooth ring stands in.  Checked here on k = 1..3 against
k = 6 (a reference this close inflates both observed orders, by about the same
amount): the (M-iii) error falls at least at order 0.8, the (M-ii) error at an
order at least 0.3 higher, and it is at least 5 times smaller."""
import numpy as np
import pytest

from paper_1610_00835_amd import inputs
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _coarse_solution(ertvie, torch, k, scheme, mus=2.0):
    nn = 24 * (2 * k - 1)
    n = (nn, nn)
    N = nn * nn
    h = 1.0 / nn
    x = inputs.centres(n, h)
    rr = np.sqrt(np.sum((x - 0.5) ** 2, axis=1))
    f = torch.from_numpy(np.exp(-(rr - 0.25) ** 2 / (2 * 0.05 ** 2))).cuda()
    case = {"dim": 2, "n": n, "h": h, "kernel": ertvie.K_HOMOGENEOUS, "sigma_t": np.full(N, mus + 0.2),
            "sigma_s": np.full(N, mus)}
    with ertvie.plan_from_case(case, method="fmm" if nn > 72 else "direct", prec="fp64", cheb_n=8,
                               scheme=scheme) as plan:
        U = torch.empty_like(f)
        info = plan.solve(f, U, tol=1e-12, max_iter=400)
    assert info["converged"] == 1
    sel = np.arange(24) * (2 * k - 1) + k - 1
    return U.cpu().numpy().reshape(nn, nn)[np.ix_(sel, sel)].reshape(-1)


def test_mii_second_order_miii_first_order():
    import torch
    from paper_1610_00835_amd import ertvie
    ertvie.load()
    hs = np.array([1.0 / (24 * (2 * k - 1)) for k in (1, 2, 3)])
    err = {}
    for scheme in (0, 1):
        ref = _coarse_solution(ertvie, torch, 6, scheme)
        err[scheme] = np.array([np.linalg.norm(_coarse_solution(ertvie, torch, k, scheme) - ref) / np.linalg.norm(ref)
                                for k in (1, 2, 3)])
    order = {s: np.log(err[s][:-1] / err[s][1:]) / np.log(hs[:-1] / hs[1:]) for s in (0, 1)}
    log("(M-iii) errors", err[0], "orders", order[0])
    log("(M-ii)  errors", err[1], "orders", order[1])
    assert np.all(order[0] > 0.8)
    assert np.all(order[1] > order[0] + 0.3)
    assert np.all(err[1] * 5 < err[0])
