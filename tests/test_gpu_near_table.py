"""Near-field products read from the offset table (homogeneous medium on a uniform grid,
leaf a power of two >= 4; Sec. 3.3's near field with the translation invariance of the
kernel): every execution form, fixed through the plan's `form` option, against the oracle and
against each other.

The offset-stationary forms 1-3 read the same FP32/FP64 values as the explicit blocks
and reduce each output in the same order, so they agree bit for bit; the target-tile
form 0 (explicit blocks, another summation order) and, in FP32, forms 4 and 5 (source
columns staged in LDS; one wave per 16 rows, or 64 columns per wave over every fourth
block of 16 rows) agree to rounding.  Repeated
calls (the second captures a graph, the third replays it) return the same bits.
Bars against the oracle: the FMM bar of 1e-6 at n = 8 for both precisions.
"""
import numpy as np
import pytest

from paper_1610_00835_amd import inputs
from tests.gpu_util import gpu_apply, log, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ev():
    from paper_1610_00835_amd import ertvie
    ertvie.load()
    return ertvie


@pytest.mark.parametrize("recipe,n,leaf", [("c2", (16, 16, 16), 4), ("c2", (32, 32, 32), 8),
                                           ("c1", (64, 64), 8), ("c1", (72, 40), 8)])
def test_near_table_forms(ev, oracle_mod, recipe, n, leaf):
    case = inputs.make_case(recipe, n=n, seed=5)
    P = oracle_problem(oracle_mod, case)
    dim = case["dim"]
    x = inputs.random_vector(P.N, 6)
    rows = np.random.default_rng(7).choice(P.N, size=min(P.N, 400), replace=False)
    ref = P.apply_rows(x, rows, op=2)
    for prec, agree in (("fp64", 1e-13), ("fp32", 1e-6)):
        out = {}
        lds64 = prec == "fp32" and leaf ** dim <= 252       # form 5 stages 64 columns of leaf^dim values
        for form in ("0", "1", "2", "3") + (("4",) if prec == "fp32" else ()) + (("5",) if lds64 else ()):
            with ev.plan_from_case(case, method="fmm", prec=prec, leaf=leaf, form=int(form)) as plan:
                ys = [gpu_apply(plan, x, ev.OP_A) for _ in range(3)]
                info = plan.fmm_info()
            assert info["near_table"] == (4 * leaf - 1) ** dim
            assert info["form_near"] == int(form)
            assert np.array_equal(ys[0], ys[1]) and np.array_equal(ys[0], ys[2]), form
            out[form] = ys[0]
        err = rel_l2(out["1"][rows], ref)
        log("near table", recipe, n, leaf, prec, "vs oracle", err, "form 0 vs 1", rel_l2(out["0"], out["1"]))
        assert np.array_equal(out["1"], out["2"]) and np.array_equal(out["1"], out["3"])
        assert rel_l2(out["0"], out["1"]) <= agree
        for f in ("4", "5"):
            if f in out:
                log("near table", recipe, n, leaf, "form", f, "vs 1", rel_l2(out[f], out["1"]))
                assert rel_l2(out[f], out["1"]) <= agree
        assert err <= 1e-6
