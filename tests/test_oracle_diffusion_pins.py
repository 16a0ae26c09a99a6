"""Pins of the diffusion preconditioner's reference (oracle/diffusion.py, Sec. 4.4,
eq. EQ:DA): the operator against a face-by-face dense assembly, exactness for
quadratic profiles in the interior and for Robin-compatible linear profiles at
the boundary, symmetry and positivity, multigrid convergence to a dense LAPACK
solve, and the preconditioner's effect in the diffusive regime."""
import numpy as np
import pytest

from oracle import diffusion as Dm


def _medium(n, seed, lo=2.0, hi=8.0):
    rng = np.random.default_rng(seed)
    N = int(np.prod(n))
    st = rng.uniform(lo, hi, N)
    return st, st * rng.uniform(0.5, 0.99, N)


@pytest.mark.parametrize("n", [(7, 6), (5, 4, 3)])
def test_operator_matches_dense_assembly(n):
    st, ss = _medium(n, 1)
    h = 1.0 / max(n)
    lv = Dm.Level(n, h, st, ss)
    L = Dm.matrix(n, h, st, ss)
    U = np.random.default_rng(2).standard_normal(int(np.prod(n)))
    assert np.allclose(lv.apply(U.reshape(n[::-1])).reshape(-1), L @ U, rtol=0, atol=1e-11 * np.abs(L).max())
    assert np.allclose(L, L.T, rtol=0, atol=1e-12 * np.abs(L).max())
    assert np.linalg.eigvalsh(L).min() > 0


def test_quadratic_profile_exact_in_the_interior():
    """Constant coefficients: the 5-point operator is exact for quadratics, so
    -D Lap(x^2 + 3 y^2) + mu_a U = -8 D + mu_a U in every interior cell."""
    n = (9, 8)
    h = 0.1
    N = 72
    st, ss = np.full(N, 4.0), np.full(N, 3.0)
    lv = Dm.Level(n, h, st, ss)
    y, x = np.indices(n[::-1]) * h + h / 2
    U = x ** 2 + 3 * y ** 2
    LU = lv.apply(U)
    D = 1 / (2 * 4.0)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(LU[inner], (-8 * D + 1.0 * U)[inner], rtol=1e-12, atol=1e-12)


def test_robin_boundary_exact_for_compatible_linear_profile():
    """U = l + x with l = 2 D satisfies U + l dU/dn = 0 at x = 0 (n = -e_x); the
    boundary term reproduces the flux exactly, so L U = 0 on the first column
    (mu_a = 0, away from the y boundary rows)."""
    n = (8, 9)
    h = 0.125
    N = 72
    st = np.full(N, 5.0)
    lv = Dm.Level(n, h, st, st)                  # mu_a = 0
    D = 1 / (2 * 5.0)
    y, x = np.indices(n[::-1]) * h + h / 2
    U = 2 * D + x
    LU = lv.apply(U)
    assert np.max(np.abs(LU[1:-1, 0])) <= 1e-12
    assert np.max(np.abs(LU[1:-1, 1:-1])) <= 1e-12


@pytest.mark.parametrize("n", [(16, 12), (8, 7, 6)])
def test_vcycles_converge_to_dense_solve(n):
    st, ss = _medium(n, 3, 5.0, 50.0)
    h = 1.0 / max(n)
    lv = Dm.hierarchy(n, h, st, ss)
    b = np.random.default_rng(4).standard_normal(int(np.prod(n)))
    exact = np.linalg.solve(Dm.matrix(n, h, st, ss), b)
    e1 = np.linalg.norm(Dm.solve_approx(lv, b, 1) - exact) / np.linalg.norm(exact)
    e40 = np.linalg.norm(Dm.solve_approx(lv, b, 40) - exact) / np.linalg.norm(exact)
    assert e1 < 0.5 and e40 < 1e-10


def test_preconditioner_in_diffusive_regime(oracle_mod):
    """Optically thin cells in a thick domain (2D 64^2, sigma_t = 10.2, sigma_s = 10,
    sigma_t h = 0.16), a smooth interior residual: two V-cycles leave 12 % of the
    residual where the identity leaves 75 % (on cells of optical thickness near 1 the
    diffusion model stops matching the discrete operator's absorption and the gain
    goes away)."""
    n = (64, 64)
    h = 1.0 / 64
    N = 64 * 64
    st, ss = np.full(N, 10.2), np.full(N, 10.0)
    P = oracle_mod.Problem(2, n, h, 0, st, ss)
    from paper_1610_00835_amd import inputs
    x = inputs.centres(n, h)
    r = np.exp(-np.sum((x - 0.5) ** 2, axis=1) / (2 * 0.1 ** 2))
    z = Dm.apply(r, 2, n, h, st, ss, cycles=2)
    res_pc = np.linalg.norm(r - P.apply(z, op=2)) / np.linalg.norm(r)
    res_id = np.linalg.norm(r - P.apply(r, op=2)) / np.linalg.norm(r)
    assert res_pc < 0.25 * res_id


@pytest.mark.parametrize("n", [(8, 6), (7, 5), (6, 4, 5), (5, 5, 3)])
def test_transfers_against_their_definition(n):
    """The V-cycle's grid transfers, cell by cell: restriction = the average over the (up to
    2^d) fine cells whose indices halve to the coarse cell (ragged grids: fewer children at
    the far edge), prolongation = the coarse parent's value; so restricting a prolonged
    field returns it (to the rounding of the sum of its copies), constants stay constant, and
    on even grids the total is kept up to the factor 2^d."""
    st, ss = _medium(n, 5)
    lv = Dm.Level(n, 1.0 / max(n), st, ss)
    shp = n[::-1]
    rng = np.random.default_rng(6)
    x = rng.standard_normal(shp)
    nc = tuple((v + 1) // 2 for v in n)
    ref = np.zeros(nc[::-1])
    cnt = np.zeros(nc[::-1])
    for idx in np.ndindex(*shp):
        c = tuple(i // 2 for i in idx)
        ref[c] += x[idx]
        cnt[c] += 1
    ref /= cnt
    r = Dm._restrict(lv, x)
    assert r.shape == ref.shape and np.allclose(r, ref, rtol=0, atol=1e-14)
    e = rng.standard_normal(nc[::-1])
    p = Dm._prolong(lv, e)
    for idx in np.ndindex(*shp):
        assert p[idx] == e[tuple(i // 2 for i in idx)]
    assert np.allclose(Dm._restrict(lv, Dm._prolong(lv, e)), e, rtol=1e-15, atol=0)
    assert np.allclose(Dm._restrict(lv, np.full(shp, 2.5)), 2.5, rtol=0, atol=1e-15)
    if all(v % 2 == 0 for v in n):
        assert abs(r.sum() * 2 ** len(n) - x.sum()) <= 1e-12 * np.abs(x).sum()
