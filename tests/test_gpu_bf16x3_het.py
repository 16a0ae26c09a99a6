"""Split-BF16x3 far-field translations in a heterogeneous medium (Sec. 3.3 eq. EQ: M2L over
the cached per-pair matrices of the ray-quadrature kernel): the 64^3 blob medium with 64
right-hand sides, BF16x3 against FP32 and both against the oracle, element by element on
sampled rows.

Bars.  FP32 applies: the FMM bar 1e-6.  A split-BF16x3 product a w = hi_a hi_w + hi_a lo_w +
lo_a hi_w differs from the FP32 product by the dropped lo_a lo_w (<= 2^-16 |a w|) and the
rounding of the two lo parts (<= 2^-17 |a w| each), i.e. <= 2^-15 |a w| per term; only the
far-field terms take this path.  BF16x3 against FP32: 2^-15 of the magnitude of the far
field, which is below the norm of y here, so relative to y the bound is 2^-15 (checked per
column and in L2); against the oracle: 1e-6 + 2^-15."""
import numpy as np
import pytest

from paper_1610_00835_amd import inputs
from tests.gpu_util import gpu_apply, log, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

BF16X3_TERM = 2.0 ** -15


@pytest.fixture(scope="module")
def ev():
    from paper_1610_00835_amd import ertvie
    ertvie.load()
    return ertvie


def test_c4_bf16x3_vs_fp32_64_rhs(ev, oracle_mod):
    case = inputs.make_case("c4", seed=0, nrhs=64)
    P = oracle_problem(oracle_mod, case)
    X = inputs.random_vector(P.N, 5, nrhs=64)
    rows = np.random.default_rng(31).choice(P.N, size=32, replace=False)
    ref = P.apply_rows(X, rows, op=2)
    with ev.plan_from_case(case, method="fmm", prec="fp32", nrhs_max=64) as plan:
        info = plan.fmm_info("bf16x3")
        Y32 = gpu_apply(plan, X, ev.OP_A)
        Y16 = gpu_apply(plan, X, ev.OP_A, prec="bf16x3")
        Y16b = gpu_apply(plan, X, ev.OP_A, prec="bf16x3")
        Y16c = gpu_apply(plan, X, ev.OP_A, prec="bf16x3")     # graph replay
        y1 = gpu_apply(plan, X[:, 7], ev.OP_A, prec="bf16x3")
        y1_32 = gpu_apply(plan, X[:, 7], ev.OP_A)
    e32 = rel_l2(Y32[rows], ref)
    e16 = rel_l2(Y16[rows], ref)
    d = rel_l2(Y16, Y32)
    dcol = max(rel_l2(Y16[:, b], Y32[:, b]) for b in range(64))
    log("64^3 blob medium, 64 rhs: FP32 vs oracle %.3e, BF16x3 vs oracle %.3e, BF16x3 vs FP32 %.3e "
        "(worst column %.3e)" % (e32, e16, d, dcol), info)
    assert info["cheb_n"] == 8 and info["levels"] == 3
    assert np.array_equal(Y16, Y16b) and np.array_equal(Y16, Y16c)
    assert e32 <= 1e-6
    assert d <= BF16X3_TERM and dcol <= BF16X3_TERM
    assert e16 <= 1e-6 + BF16X3_TERM
    # one column through the same split products: its far field equals the batched
    # column's; the near field of one column is summed by the streaming kernel instead
    # of the matrix cores (FP32 rounding apart)
    assert rel_l2(y1, Y16[:, 7]) <= 1e-6
    assert rel_l2(y1, y1_32) <= BF16X3_TERM
