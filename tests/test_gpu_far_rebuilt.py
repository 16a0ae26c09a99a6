"""Heterogeneous translation levels over the plan's cache budget (ert_vie_opts.far_cache_gb)
keep the pairs that fit stored; every apply rebuilds the others chunk by chunk, by the same
ray march (Sec. 4.2's kernel evaluations), and streams each chunk through the same pair
products, with the per-target sums after all chunks.  Such a plan gives the fully stored
plan's results bit for bit: the streaming (1 and 3 right-hand sides), matrix-core (16) and
split-BF16x3 products, eager applies and graph replays, and a mixed-precision solve whose two
operators are both rebuilt.  The stored plans are the ones the oracle parity tests check."""
import numpy as np
import pytest

from paper_1610_00835_amd import inputs
from tests.gpu_util import gpu_apply, log, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ev():
    from paper_1610_00835_amd import ertvie
    ertvie.load()
    return ertvie


def _vectors(N, nrhs, seed):
    X = inputs.random_vector(N, seed, nrhs=nrhs)
    return X if nrhs > 1 else np.asarray(X).reshape(-1)


@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("fp32", 3), ("fp32", 16), ("fp64", 16), ("bf16x3", 1)])
def test_rebuilt_level_equals_stored(ev, prec, nrhs):
    """32^3 blob medium, leaf 4^3, order 4 (far field on levels 2 and 3): a budget that holds
    level 2 and 100 more blocks keeps 94 pairs of level 3 stored (a sixteenth of the room goes
    to the scratch buffer) and rebuilds the others in chunks of 6 box pairs."""
    case = inputs.make_case("c3", n=(32, 32, 32), seed=5)
    N = int(np.prod(case["n"]))
    X = _vectors(N, nrhs, 31)
    kw = dict(method="fmm", prec=prec, leaf=4, cheb_n=4, nrhs_max=nrhs)
    with ev.plan_from_case(case, **kw) as a:
        ia = a.fmm_info()
        ya = gpu_apply(a, X, ev.OP_A)
    assert ia["levels"] == 3 and ia["far_rebuilt"] == [0, 0, 0, 0]
    block = ia["nodes_padded"] ** 2 * 4
    level2 = ia["far_pairs"][2] // 2 * block
    with ev.plan_from_case(case, far_cache_gb=(level2 + 100 * block) / 1e9, **kw) as b:
        ib = b.fmm_info()
        ys = [gpu_apply(b, X, ev.OP_A) for _ in range(3)]   # eager, captured, replayed
    log("rebuilt level 3", prec, nrhs, "rebuilt", ib["far_rebuilt"], "cache bytes", ib["cache_bytes"],
        "stored plan", ia["cache_bytes"])
    assert ib["far_rebuilt"] == [0, 0, 0, 1]
    assert ib["cache_bytes"] < ia["cache_bytes"]
    for y in ys:
        assert np.array_equal(y, ya)


def test_all_levels_rebuilt_mixed_solve(ev):
    """16^3, leaf 4^3 (far field on level 2 only), a budget of nothing: every translation
    matrix is rebuilt one box pair at a time in each apply, for the FP64 outer operator
    (order 6) and the FP32 inner operator (order 4) of a mixed solve to 1e-8.  The solve
    takes the same steps and returns the same solution as with the stored caches."""
    import torch
    case = inputs.make_case("c3", n=(16, 16, 16), seed=6)
    fd = to_dev(case["f"])
    out = []
    for budget in (0.0, 1e-12):
        with ev.plan_from_case(case, method="fmm", prec="fp64", leaf=4, cheb_n=6, inner_cheb_n=4,
                               far_cache_gb=budget) as plan:
            i64 = plan.fmm_info("fp64")
            i32 = plan.fmm_info("fp32")
            Ud = torch.empty_like(fd)
            info = plan.solve(fd, Ud, tol=1e-8, mixed=True, inner_tol=1e-4)
            y = gpu_apply(plan, case["f"], ev.OP_A)
            out.append((i64["far_rebuilt"], i32["far_rebuilt"], info, to_host(Ud), y))
    (r64a, r32a, ia, Ua, ya), (r64b, r32b, ib, Ub, yb) = out
    log("all rebuilt, mixed solve", ib)
    assert r64a == [0, 0, 0] and r32a == [0, 0, 0]
    assert r64b == [0, 0, 1] and r32b == [0, 0, 1]
    assert ia["converged"] == 1 and ib["converged"] == 1
    assert ib["iters"] == ia["iters"] and ib["matvecs"] == ia["matvecs"]
    assert ib["rel_resid_true"] <= 1e-8
    assert np.array_equal(Ub, Ua)
    assert np.array_equal(yb, ya)
