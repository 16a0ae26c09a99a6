"""The allocation-free variant of Algorithm 1 step S.3 (ert_vie_transport_noalloc: the
library's static device scratch instead of a hipMalloc per call) against
ert_vie_transport through the C ABI.  Both run the same kernels on the same inputs, so the
bar is bit-for-bit equality.  Two calls in a row, the second with a smaller input (the
shared scratch keeps the first call's contents), then the largest accepted size and the
first rejected one (ERT_EINVAL before any device work: the output keeps its contents)."""
import ctypes

import numpy as np
import pytest

from paper_1610_00835_amd import inputs
from tests.gpu_util import log, to_dev

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = (1 << 22) + (1 << 16)


@pytest.fixture(scope="module")
def ev():
    from paper_1610_00835_amd import ertvie
    ertvie.load()
    return ertvie


def _dirs(dim, k, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((k, dim))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _both(ev, plan, U, f, dirs):
    import torch
    a = torch.full((len(dirs), plan.N), np.nan, dtype=torch.float64, device="cuda")
    b = torch.full_like(a, -1.0)
    plan.transport(U, f, dirs, a)
    plan.transport(U, f, dirs, b, noalloc=True)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_transport_noalloc_equals_transport(ev):
    import torch
    # first call: the 32^3 many-scattering medium, 26 directions
    case = inputs.make_case("c5", n=(32, 32, 32), seed=4)
    U = np.random.default_rng(1).uniform(0, 1, 32 ** 3)
    with ev.plan_from_case(case, method="direct", prec="fp64") as plan:
        a, b = _both(ev, plan, to_dev(U), to_dev(case["f"]), _dirs(3, 26, 2))
    log("noalloc 32^3 x 26: equal", np.array_equal(a, b), "finite", bool(np.all(np.isfinite(a))))
    assert np.all(np.isfinite(a)) and np.array_equal(a, b)
    # second call, smaller: a 2D 24 x 20 grid, 5 directions, the source alone
    case2 = inputs.make_case("c1", n=(24, 20))
    with ev.plan_from_case(case2, method="direct", prec="fp64") as plan:
        a2, b2 = _both(ev, plan, None, to_dev(case2["f"]), _dirs(2, 5, 3))
    assert np.all(np.isfinite(a2)) and np.array_equal(a2, b2)
    # the largest accepted 2D grid for one direction (2 N + 2 <= SCRATCH_DOUBLES), then one
    # row more (rejected)
    for n1, ok in ((1039, True), (1040, False)):
        n = (2048, n1)
        N = n[0] * n[1]
        st = np.full(N, 3.0)
        with ev.Plan(2, n, 1.0 / 2048, st, 0.9 * st) as plan:
            f = to_dev(np.ones(N))
            dirs = _dirs(2, 1, 5)
            if ok:
                assert 2 * N + 2 <= SCRATCH_DOUBLES
                a3, b3 = _both(ev, plan, None, f, dirs)
                assert np.all(np.isfinite(a3)) and np.array_equal(a3, b3)
            else:
                assert 2 * N + 2 > SCRATCH_DOUBLES
                phi = torch.full((1, N), 7.0, dtype=torch.float64, device="cuda")
                d = np.ascontiguousarray(dirs)
                st_ = ev.load().ert_vie_transport_noalloc(plan.handle, None, ctypes.c_void_p(f.data_ptr()),
                                                          d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1,
                                                          ctypes.c_void_p(phi.data_ptr()))
                torch.cuda.synchronize()
                assert st_ == ev.EINVAL
                assert bool(torch.all(phi == 7.0))
                log("rejected:", ev.load().ert_vie_last_error().decode())
