"""GPU parity of the diffusion preconditioner (Sec. 4.4, eq. EQ:DA) against its
reference (oracle/diffusion.py): the same finite differences and the same V-cycles
in FP64 on both sides (sums in the same order), bar relative L2 <= 1e-12; and the
paper's preconditioning experiment with it (Experiment V)."""
import os

import numpy as np
import pytest

from oracle import diffusion as Dm
from paper_1610_00835_amd import inputs
from tests.gpu_util import log, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ev():
    from paper_1610_00835_amd import ertvie
    ertvie.load()
    return ertvie


@pytest.mark.parametrize("name,n", [("c1", (20, 16)), ("c3", (12, 10, 9)), ("c5", (16, 16, 16)), ("c1", (37, 5)),
                                    ("c1", (4, 3)), ("c5", (40, 36, 33))])
def test_diff_precond_matches_reference(ev, name, n):
    case = inputs.make_case(name, n=n, seed=1)
    N = int(np.prod(n))
    R = np.random.default_rng(2).standard_normal((N, 2))
    with ev.plan_from_case(case, method="direct", prec="fp64", nrhs_max=2) as plan:
        Z = to_host(plan.diff_precond(to_dev(R), to_dev(np.zeros((N, 2)))))
        r1 = to_dev(R[:, 1])
        z1 = to_host(plan.diff_precond(r1, r1))
    lv = Dm.hierarchy(case["n"], case["h"], case["sigma_t"], case["sigma_s"])
    for k in range(2):
        ref = Dm.apply(R[:, k], case["dim"], case["n"], case["h"], case["sigma_t"], case["sigma_s"], levels=lv)
        e = rel_l2(Z[:, k], ref)
        log("diffusion preconditioner", name, n, "column", k, "rel L2", e, "levels", len(lv))
        assert e <= 1e-12
    assert np.array_equal(z1, Z[:, 1])


def test_diff_precond_full_size(ev):
    case = inputs.make_case("c5", n=(128, 128, 128), seed=0)
    N = 128 ** 3
    r = np.random.default_rng(3).standard_normal(N)
    with ev.plan_from_case(case, method="direct", prec="fp64") as plan:
        z = to_host(plan.diff_precond(to_dev(r), to_dev(np.zeros(N))))
    ref = Dm.apply(r, 3, case["n"], case["h"], case["sigma_t"], case["sigma_s"])
    e = rel_l2(z, ref)
    log("diffusion preconditioner 128^3 rel L2", e)
    assert e <= 1e-12


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_exp6_iterations.txt")


def test_diffusion_preconditioned_solve_thin_cells(ev):
    """2D 256^2, absorption 0.2, scattering 40 (sigma_t h = 0.16): GMRES with the
    diffusion preconditioner reaches the unpreconditioned solution (1e-10) in
    fewer iterations; as flexible right preconditioner and in the mixed solve."""
    import torch
    n = (256, 256)
    N = 256 * 256
    x = inputs.centres(n, 1.0 / 256)
    f = torch.from_numpy(np.exp(-np.sum((x - 0.5) ** 2, axis=1) / (2 * 0.1 ** 2))).cuda()
    case = {"dim": 2, "n": n, "h": 1.0 / 256, "kernel": ev.K_HOMOGENEOUS, "sigma_t": np.full(N, 40.2),
            "sigma_s": np.full(N, 40.0)}
    with ev.plan_from_case(case, method="fmm", prec="fp64", cheb_n=6) as plan:
        U0 = torch.empty_like(f)
        r0 = plan.solve(f, U0, tol=1e-12, max_iter=300)
        U1 = torch.empty_like(f)
        r1 = plan.solve(f, U1, tol=1e-12, max_iter=300, precond_diffusion=True)
        U2 = torch.empty_like(f)
        r2 = plan.solve(f, U2, tol=1e-12, max_iter=300, precond_diffusion=True, mixed=True, inner_tol=1e-4)
        d1 = float(torch.linalg.norm(U1 - U0) / torch.linalg.norm(U0))
        d2 = float(torch.linalg.norm(U2 - U0) / torch.linalg.norm(U0))
    log("plain", r0, "\ndiffusion", r1, "\nmixed + diffusion", r2, "\ndifferences", d1, d2)
    assert r1["converged"] == 1 and r2["converged"] == 1
    assert d1 <= 1e-10 and d2 <= 1e-10
    assert r1["iters"] < r0["iters"]
