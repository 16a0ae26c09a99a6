"""Heterogeneous 64^3 workload (blob medium, ray-quadrature kernel): FP32 FMM apply on
sampled rows against the oracle, and the FP64-refined solve's true residual."""
import numpy as np
import pytest

from paper_1610_00835_amd import inputs
from tests.gpu_util import gpu_apply, log, oracle_problem, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    from paper_1610_00835_amd import ertvie
    ertvie.load()
    case = inputs.make_case("c3", seed=0)
    return ertvie, case


def test_c3_fmm_apply_rows(c3, oracle_mod):
    ev, case = c3
    P = oracle_problem(oracle_mod, case)
    x = inputs.random_vector(P.N, 11)
    rows = np.random.default_rng(7).choice(P.N, size=128, replace=False)
    ref = P.apply_rows(x, rows, op=2)
    with ev.plan_from_case(case, method="fmm", prec="fp32") as plan:
        info = plan.fmm_info()
        y = gpu_apply(plan, x, ev.OP_A)
    err = rel_l2(y[rows], ref)
    log("c3 fmm fp32 apply rows rel L2", err, info)
    assert err <= 2e-5
