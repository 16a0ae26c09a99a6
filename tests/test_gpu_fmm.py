"""GPU parity of the FMM apply (Sec. 3.3) against the FP64 oracle.

Bar (relative L2 over all outputs, or over sampled rows at full size): 1e-6 for the
FMM apply with the default n = 8 Chebyshev nodes per axis on homogeneous media, FP64
and FP32 (n = 6 measures ~3e-6 in 3D, above the bar; the order test reports it).
A tree without far field reproduces the dense sum to rounding.  Heterogeneous media
and split-BF16x3 report their measured error against a looser bar stated per test.
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


@pytest.mark.parametrize("n,leaf", [((8, 8, 8), 4), ((16, 16, 16), 8), ((10, 7, 12), 8)])
def test_no_far_field_equals_dense(ev, oracle_mod, n, leaf):
    """Every leaf is a neighbour of every other: the FMM is the dense sum (near-field GEMM)."""
    case = inputs.make_case("c2", n=n, seed=1)
    P = oracle_problem(oracle_mod, case)
    x = inputs.random_vector(P.N, 2)
    yo = P.apply(x, op=2)
    for prec, bar in (("fp64", 1e-13), ("fp32", 1e-6)):
        with ev.plan_from_case(case, method="fmm", prec=prec, leaf=leaf) as plan:
            err = rel_l2(gpu_apply(plan, x, ev.OP_A), yo)
        log("no far field", n, leaf, prec, "rel L2", err)
        assert err <= bar


@pytest.mark.parametrize("prec,svd_tol", [("fp64", -1.0), ("fp64", 0.0), ("fp32", -1.0), ("fp32", 0.0)])
def test_fmm_homogeneous_16cubed(ev, oracle_mod, prec, svd_tol):
    """16^3 with 4^3-cell leaves (far field on level 2), translations plain and compressed."""
    bar = 1e-6
    case = inputs.make_case("c2", n=(16, 16, 16), seed=0)
    P = oracle_problem(oracle_mod, case)
    x = inputs.random_vector(P.N, 3)
    with ev.plan_from_case(case, method="fmm", prec=prec, leaf=4, svd_tol=svd_tol) as plan:
        for op in (ev.OP_G, ev.OP_A):
            err = rel_l2(gpu_apply(plan, x, op), P.apply(x, op=op))
            log("16^3 fmm", prec, "svd_tol", svd_tol, "op", op, "rel L2", err)
            assert err <= bar


@pytest.mark.parametrize("prec,leaf", [("fp64", 8), ("fp32", 8), ("fp32", 4), ("bf16x3", 8)])
def test_fmm_c2_full_size_rows(ev, oracle_mod, prec, leaf):
    """32^3, sigma_t = 5, sigma_s = 4, n = 8: sampled rows vs the oracle, all rows vs the dense GPU sum."""
    case = inputs.make_case("c2", seed=0)
    P = oracle_problem(oracle_mod, case)
    x = case["f"]
    rows = np.random.default_rng(1).choice(P.N, size=800, replace=False)
    with ev.plan_from_case(case, method="fmm", prec=prec, leaf=leaf) as plan:
        for op in (ev.OP_G, ev.OP_A):
            yg = gpu_apply(plan, x, op)
            err = rel_l2(yg[rows], P.apply_rows(x, rows, op=op))
            log("c2 fmm", prec, "leaf", leaf, "op", op, "rows rel L2", err)
            assert err <= 1e-6
        # and the whole vector against the (oracle-pinned) FP64 dense apply on the GPU
        yd = gpu_apply(plan, x, ev.OP_A, method="direct", prec="fp64")
        yf = gpu_apply(plan, x, ev.OP_A)
        err = rel_l2(yf, yd)
        log("c2 fmm", prec, "leaf", leaf, "vs dense, all rows", err)
        assert err <= 1e-6


def test_fmm_error_decreases_with_order(ev, oracle_mod):
    """Table 1 trend: the far-field error falls with the interpolation order n."""
    case = inputs.make_case("c2", n=(16, 16, 16), seed=5)
    P = oracle_problem(oracle_mod, case)
    x = inputs.random_vector(P.N, 6)
    ref = P.apply(x, op=1)
    errs = []
    for n in (3, 4, 6, 8):
        with ev.plan_from_case(case, method="fmm", prec="fp64", cheb_n=n, leaf=4, svd_tol=-1) as plan:
            errs.append(rel_l2(gpu_apply(plan, x, ev.OP_GS), ref))
    log("error vs n (3,4,6,8):", errs)
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 2e-7


def test_fmm_2d(ev, oracle_mod):
    """2D 64^2 (sigma_t = 2) with 8^2-cell leaves, three levels."""
    case = inputs.make_case("c1")
    P = oracle_problem(oracle_mod, case)
    x = case["f"]
    with ev.plan_from_case(case, method="fmm", prec="fp64") as plan:
        err = rel_l2(gpu_apply(plan, x, ev.OP_A), P.apply(x, op=2))
    log("2D fmm rel L2", err)
    assert err <= 1e-6


@pytest.mark.parametrize("n,leaf", [((20, 13, 9), 4), ((37, 5, 17), 4), ((41, 23, 30), 8)])
def test_fmm_ragged(ev, oracle_mod, n, leaf):
    case = inputs.make_case("c2", n=n, seed=2)
    P = oracle_problem(oracle_mod, case)
    x = inputs.random_vector(P.N, 7)
    with ev.plan_from_case(case, method="fmm", prec="fp64", leaf=leaf) as plan:
        err = rel_l2(gpu_apply(plan, x, ev.OP_A), P.apply(x, op=2))
    log("ragged", n, err)
    assert err <= 1e-6


@pytest.mark.parametrize("forms", [None, (1, 1), (4, 4), (5, 4)])
def test_fmm_multi_rhs_and_determinism(ev, oracle_mod, forms):
    """Repeated applies return the same bits.  Each right-hand-side count tunes its own
    execution forms, which may sum in different orders: the columns of a 5-column apply
    agree with single-column applies to FP32 rounding, and bit for bit once the forms are
    fixed (the plan's `form` option, (near field, translations)), since every form reduces
    each column on its own.  A form that does not apply to a product leaves it to the timing
    (form 5 takes reduction lengths up to 240, shorter than this plan's compressed
    translations at order 8), so the forms in use are checked to be the requested ones."""
    case = inputs.make_case("c2", n=(16, 16, 16), seed=3)
    X = inputs.random_vector(4096, 9, nrhs=5)
    with ev.plan_from_case(case, method="fmm", prec="fp32", nrhs_max=5, leaf=4, form=forms) as plan:
        Y = gpu_apply(plan, X, ev.OP_A)
        Y2 = gpu_apply(plan, X, ev.OP_A)
        Y3 = gpu_apply(plan, X, ev.OP_A)
        assert np.array_equal(Y, Y2) and np.array_equal(Y, Y3)
        if forms:
            gpu_apply(plan, X[:, 0], ev.OP_A)
            info = plan.fmm_info()
            log("fixed forms", forms, "in use: near", info["form_near"], "far", info["form_far"])
            assert info["form_near"] == forms[0]
            assert all(f == forms[1] for f in info["form_far"][2:])
        bar = 1e-12 if forms else 1e-6
        for b in range(5):
            yb = gpu_apply(plan, X[:, b], ev.OP_A)
            assert np.max(np.abs(yb - Y[:, b])) <= bar * np.max(np.abs(yb))


def test_fmm_bf16x3_vs_fp32(ev, oracle_mod):
    """Split-BF16x3 translations against plain FP32 (both vs the oracle)."""
    case = inputs.make_case("c2", n=(32, 32, 32), seed=0)
    P = oracle_problem(oracle_mod, case)
    x = case["f"]
    rows = np.random.default_rng(2).choice(P.N, size=600, replace=False)
    ref = P.apply_rows(x, rows, op=1)
    with ev.plan_from_case(case, method="fmm", prec="fp32") as plan:
        y32 = gpu_apply(plan, x, ev.OP_GS)
        y16 = gpu_apply(plan, x, ev.OP_GS, prec="bf16x3")
    e32 = rel_l2(y32[rows], ref)
    e16 = rel_l2(y16[rows], ref)
    d = rel_l2(y16, y32)
    log("bf16x3 vs oracle", e16, "fp32 vs oracle", e32, "bf16x3 vs fp32", d)
    assert e16 <= 1e-5 and d <= 1e-5


def test_fmm_heterogeneous(ev, oracle_mod):
    """Ray-quadrature kernel through a seeded blob medium (16^3).  Bar 1e-5: the step count of
    the midpoint rule jumps with the segment length, so the kernel is not smooth across far
    boxes and the Chebyshev interpolant has an error floor (measured 8.3e-6 at n = 8)."""
    case = inputs.make_case("c3", n=(16, 16, 16), seed=0)
    P = oracle_problem(oracle_mod, case)
    x = inputs.random_vector(P.N, 4)
    ref = P.apply(x, op=2)
    for prec in ("fp64", "fp32"):
        with ev.plan_from_case(case, method="fmm", prec=prec, leaf=4) as plan:
            err = rel_l2(gpu_apply(plan, x, ev.OP_A), ref)
        log("heterogeneous fmm", prec, "rel L2", err)
        assert err <= 1e-5


def test_fmm_graph_replays_match_eager(ev, oracle_mod):
    """Applies after the second call of a rhs count replay a captured graph; every replay
    (with other work and synchronisations in between) equals the eager apply bit for bit."""
    import torch
    from tests.gpu_util import to_dev, to_host
    case = inputs.make_case("c2", n=(32, 32, 32), seed=4)
    with ev.plan_from_case(case, method="fmm", prec="fp32", nrhs_max=2) as plan:
        xs = [inputs.random_vector(case["f"].size, 20 + i) for i in range(5)]
        plan.profile(True)            # eager path (no graph) while profiling
        eager = [gpu_apply(plan, x, ev.OP_A) for x in xs]
        plan.profile(False)
        for rep in range(3):
            for i, x in enumerate(xs):
                y = gpu_apply(plan, x, ev.OP_A if i % 2 == 0 else ev.OP_A)
                assert np.array_equal(y, eager[i]), (rep, i)
                # unrelated device work between replays
                t = torch.randn(1000, device="cuda").sum()
                torch.cuda.synchronize()
        # two right-hand sides use their own graph, and their own tuned forms (which may sum
        # in another order than the single-column forms): FP32 rounding apart
        X = np.stack([xs[0], xs[1]], axis=1)
        Ys = [gpu_apply(plan, X, ev.OP_A) for _ in range(3)]
        assert np.array_equal(Ys[0], Ys[1]) and np.array_equal(Ys[0], Ys[2])
        assert np.max(np.abs(Ys[2][:, 0] - eager[0])) <= 1e-6 * np.max(np.abs(eager[0]))


@pytest.mark.parametrize("recipe,n,leaf", [("c2", (32, 32, 32), 8), ("c3", (16, 16, 16), 4)])
def test_fmm_graph_back_to_back_applies(ev, oracle_mod, recipe, n, leaf):
    """Replays of the captured apply queued back to back behind other work on the plan's
    stream, each with its own vectors (a replay replaces the root kernel node's arguments,
    the rest of the apply reads them from device memory): every result equals the eager
    apply of its vector bit for bit.  The one-level homogeneous tree and a heterogeneous
    tree have different root kernels."""
    import torch
    from tests.gpu_util import to_dev, to_host
    case = inputs.make_case(recipe, n=n, seed=8)
    N = case["f"].size
    xs = [to_dev(inputs.random_vector(N, 40 + i)) for i in range(4)]
    with ev.plan_from_case(case, method="fmm", prec="fp32", leaf=leaf) as plan:
        plan.profile(True)                # eager applies while profiling
        eager = []
        for x in xs:
            y = torch.empty_like(x)
            plan.apply(x, y, op=ev.OP_A)
            eager.append(to_host(y))
        plan.profile(False)
        ys = [torch.empty_like(x) for x in xs]
        for _ in range(2):                # capture, then replay
            for x, y in zip(xs, ys):
                plan.apply(x, y, op=ev.OP_A)
            torch.cuda.synchronize()
        for rep in range(3):
            for y in ys:
                y.zero_()
            a = torch.randn(4096, 4096, device="cuda")
            b = a @ a                     # keeps the stream busy while the applies are queued
            for x, y in zip(xs, ys):
                plan.apply(x, y, op=ev.OP_A)
            torch.cuda.synchronize()
            del a, b
            for i, y in enumerate(ys):
                assert np.array_equal(to_host(y), eager[i]), (rep, i)


@pytest.mark.parametrize("svd_tol", [1e-6, 1e-5])
def test_fmm_compression_tolerance(ev, oracle_mod, svd_tol):
    """Looser singular-value cutoffs keep the 32^3 apply within the 1e-6 bar."""
    case = inputs.make_case("c2", seed=0)
    P = oracle_problem(oracle_mod, case)
    x = case["f"]
    rows = np.random.default_rng(3).choice(P.N, size=600, replace=False)
    ref = P.apply_rows(x, rows, op=1)
    with ev.plan_from_case(case, method="fmm", prec="fp64", svd_tol=svd_tol) as plan:
        err = rel_l2(gpu_apply(plan, x, ev.OP_GS)[rows], ref)
        info = plan.fmm_info()
    log("svd_tol", svd_tol, "rank", info["rank"], "rel L2", err)
    assert err <= 1e-6


@pytest.mark.parametrize("n,leaf,prec", [((12, 10, 9), 3, "fp32"), ((12, 10, 9), 3, "fp64"),
                                         ((20, 17, 6), 5, "fp32")])
def test_fmm_heterogeneous_odd_leaf(ev, oracle_mod, n, leaf, prec):
    """Cached near blocks and per-pair translations with leaf sizes whose cell count is not a
    multiple of the 16-byte row group (27 and 125 cells per leaf): scalar row loads, the
    reduction split between thread groups, ragged box lattices.  Bar 2e-5: on grids this small
    the far pairs take as few as 12 ray steps and the jumps of the step count with the segment
    length set the interpolation floor (1.49e-5 measured at 12 x 10 x 9, the same in FP64 and
    FP32); it falls as the grid grows (2.6e-7 at 64^3)."""
    case = inputs.make_case("c3", n=n, seed=5)
    P = oracle_problem(oracle_mod, case)
    x = inputs.random_vector(P.N, 12)
    ref = P.apply(x, op=2)
    with ev.plan_from_case(case, method="fmm", prec=prec, leaf=leaf) as plan:
        info = plan.fmm_info()
        err = rel_l2(gpu_apply(plan, x, ev.OP_A), ref)
    log("heterogeneous odd leaf", n, leaf, prec, "rel L2", err, info)
    assert sum(info["far_pairs"]) > 0
    assert err <= 2e-5


def test_fmm_heterogeneous_2d(ev, oracle_mod):
    """2D ray-quadrature kernel through a smooth medium (varying sigma_t), 40 x 33 cells."""
    n = (40, 33)
    h = 1.0 / 40
    x = inputs.centres(n, h)
    st = 1.5 + 6.0 * np.exp(-((x[:, 0] - 0.4) ** 2 + (x[:, 1] - 0.55) ** 2) / (2 * 0.15 ** 2))
    case = {"name": "het2d", "dim": 2, "n": n, "h": h, "kernel": inputs.KERNEL_RAY,
            "sigma_t": st, "sigma_s": 0.8 * st, "f": np.zeros(len(st))}
    P = oracle_problem(oracle_mod, case)
    v = inputs.random_vector(P.N, 13)
    ref = P.apply(v, op=2)
    for prec in ("fp64", "fp32"):
        with ev.plan_from_case(case, method="fmm", prec=prec, leaf=4) as plan:
            err = rel_l2(gpu_apply(plan, v, ev.OP_A), ref)
        log("heterogeneous 2d", prec, "rel L2", err)
        assert err <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fmm_heterogeneous_many_rhs(ev, oracle_mod, prec):
    """11 right-hand sides (passes of 4, 4, 2 and 1 in the streaming products): every column
    equals its single-column apply, and the batch equals the oracle (bar 2e-5 as for the other
    small heterogeneous grids; 1.01e-5 measured)."""
    case = inputs.make_case("c3", n=(16, 16, 16), seed=6)
    P = oracle_problem(oracle_mod, case)
    X = inputs.random_vector(P.N, 14, nrhs=11)
    with ev.plan_from_case(case, method="fmm", prec=prec, leaf=4, nrhs_max=11) as plan:
        Y = gpu_apply(plan, X, ev.OP_A)
        for b in (0, 7, 8, 10):
            yb = gpu_apply(plan, X[:, b], ev.OP_A)
            assert np.max(np.abs(yb - Y[:, b])) <= 1e-12 * np.max(np.abs(yb))
    for b in (0, 9):
        assert rel_l2(Y[:, b], P.apply(X[:, b], op=2)) <= 2e-5


@pytest.mark.parametrize("prec,nrhs", [("fp32", 20), ("fp64", 20), ("fp32", 70)])
def test_fmm_heterogeneous_many_rhs_matrix_cores(ev, oracle_mod, prec, nrhs):
    """From 16 right-hand sides on, the cached-pair products run on the matrix cores, 64
    right-hand sides per pass (70 = 64 + 6).  Every column equals its single-column apply
    (streaming form) to accumulation order, and the oracle to the heterogeneous bar."""
    case = inputs.make_case("c3", n=(16, 16, 16), seed=7)
    P = oracle_problem(oracle_mod, case)
    X = inputs.random_vector(P.N, 16, nrhs=nrhs)
    tol = 1e-12 if prec == "fp64" else 2e-6
    with ev.plan_from_case(case, method="fmm", prec=prec, leaf=4, nrhs_max=nrhs) as plan:
        Y = gpu_apply(plan, X, ev.OP_A)
        for b in (0, 15, nrhs - 1):
            yb = gpu_apply(plan, X[:, b], ev.OP_A)
            d = np.max(np.abs(yb - Y[:, b])) / np.max(np.abs(yb))
            log("many rhs", prec, nrhs, "column", b, "max rel diff vs single column", d)
            assert d <= tol
    assert rel_l2(Y[:, 3], P.apply(X[:, 3], op=2)) <= 2e-5


@pytest.mark.parametrize("n,leaf", [((6, 6, 6), 3), ((10, 9, 7), 5), ((9, 9, 9), 8), ((5, 7, 3), 4)])
def test_fmm_heterogeneous_odd_leaves_near_only(ev, oracle_mod, n, leaf):
    """At most two leaves per axis, so every pair of leaves is a near pair and the FMM is
    the dense sum over FP32-stored kernel values: blocks of 27, 125 and 512 points
    (element-wise loads in the streaming products), and grids whose last leaf holds one
    cell along an axis (rays between cells of that layer interpolate from the cell below,
    outside the leaf); FP64 and FP32 applies of 3 right-hand sides against the oracle
    within the FP32 rounding of the stored values (bar 1e-6)."""
    case = inputs.make_case("c3", n=n, seed=8)
    P = oracle_problem(oracle_mod, case)
    X = inputs.random_vector(P.N, 18, nrhs=3)
    for prec in ("fp64", "fp32"):
        with ev.plan_from_case(case, method="fmm", prec=prec, leaf=leaf, nrhs_max=3) as plan:
            Y = gpu_apply(plan, X, ev.OP_A)
        err = max(rel_l2(Y[:, b], P.apply(X[:, b], op=2)) for b in range(3))
        log("odd leaves, near field only", n, leaf, prec, "rel L2", err)
        assert err <= 1e-6


@pytest.mark.parametrize("n,leaf", [((12, 12, 12), 3), ((20, 20, 20), 5), ((24, 24, 24), 6)])
def test_fmm_heterogeneous_odd_leaves(ev, oracle_mod, n, leaf):
    """Leaves of 3^3, 5^3 and 6^3 cells with a far field: the streaming products (3
    right-hand sides; element-wise loads for 27 and 125 points) equal the matrix-core
    products of the same plan (16 right-hand sides) to accumulation order, and the oracle
    to the FMM error of these small boxes (bar 5e-5; 2.6e-5 measured at 12^3 with 3^3
    leaves, where the far pairs take as few as 12 ray steps)."""
    case = inputs.make_case("c3", n=n, seed=8)
    P = oracle_problem(oracle_mod, case)
    X = inputs.random_vector(P.N, 18, nrhs=3)
    X16 = np.asfortranarray(np.tile(X, (1, 6))[:, :16])
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-6)):
        with ev.plan_from_case(case, method="fmm", prec=prec, leaf=leaf, nrhs_max=16) as plan:
            Y = gpu_apply(plan, X, ev.OP_A)
            Y16 = gpu_apply(plan, X16, ev.OP_A)
        d = max(np.max(np.abs(Y16[:, b] - Y[:, b])) / np.max(np.abs(Y[:, b])) for b in range(3))
        err = max(rel_l2(Y[:, b], P.apply(X[:, b], op=2)) for b in (0, 2))
        log("odd leaves", n, leaf, prec, "streaming vs matrix cores", d, "rel L2 vs oracle", err)
        assert d <= tol
        assert err <= 5e-5


def test_read_rate_diagnostic(ev):
    """ert_vie_read_rate streams a buffer (whole pieces only) and reports a positive time;
    the rate it implies stays below the 8 TB/s peak."""
    import torch
    a = torch.zeros(1 << 26, dtype=torch.float32, device="cuda")   # 256 MiB
    nbytes, ms = ev.read_rate(a, 224 * 224 * 4, reps=3)
    assert nbytes == (a.numel() * 4) // (224 * 224 * 4) * (224 * 224 * 4)
    assert ms > 0 and nbytes / (ms * 1e-3) < 8.0e12
    log("read rate, 256 MiB in 200704-byte pieces:", nbytes / (ms * 1e-3) / 1e9, "GB/s")


def test_fmm_homogeneous_64cubed_lds64_form(ev, oracle_mod):
    """The 64^3 homogeneous recipe (two far-field levels, translations compressed at 1e-6 to
    ranks 256 and 224): execution form 5 (64-column tiles over all rows, source columns in
    LDS) where it applies (rank 224 <= 252) against form 1, to FP32 rounding (bar 1e-6), and
    the oracle on sampled rows (the FMM bar 1e-6); repeated applies return the same bits."""
    case = inputs.make_case("c2", n=(64, 64, 64), seed=0)
    P = oracle_problem(oracle_mod, case)
    x = inputs.random_vector(P.N, 13)
    rows = np.random.default_rng(2).choice(P.N, size=64, replace=False)
    out = {}
    for form in (1, 5):
        with ev.plan_from_case(case, method="fmm", prec="fp32", form=(1, form)) as plan:
            ys = [gpu_apply(plan, x, ev.OP_A) for _ in range(3)]
            info = plan.fmm_info()
        assert np.array_equal(ys[0], ys[1]) and np.array_equal(ys[0], ys[2])
        out[form] = (ys[0], info)
    info5 = out[5][1]
    log("64^3 forms", info5["rank"], info5["form_far"])
    assert info5["form_far"][3] == 5 and info5["rank"][3] <= 252
    d = rel_l2(out[5][0], out[1][0])
    err = rel_l2(out[5][0][rows], P.apply_rows(x, rows, op=2))
    log("64^3 form 5 vs form 1", d, "vs oracle rows", err)
    assert d <= 1e-6 and err <= 1e-6
