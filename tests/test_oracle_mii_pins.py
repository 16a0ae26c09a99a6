"""Pins of the oracle's approach (M-ii) (Sec. 3.2 and Remark 3.1): the cell
integral I(t) of |z|^{1-d} against independent numerical integration, its value
at t = 0 in closed form, the exact additivity over a tiling, and its far-field
Taylor expansion; the assembled matrix against the same additivity (row sums of
the free-space operator), symmetry, and a dense LU solve."""
import itertools
import os

import numpy as np
import pytest
from scipy import integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "selfcell_sigma0.txt")


def _golden():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


@pytest.mark.parametrize("t", [(0.1, 0.0), (0.13, -0.07), (0.25, 0.31), (-0.6, 0.05), (1.3, 2.2)])
def test_cell_integral_2d_closed_form_vs_quadrature(oracle_mod, t):
    h = 0.1
    v, _ = integrate.dblquad(lambda y, x: 1.0 / np.hypot(x, y), t[0] - h / 2, t[0] + h / 2, t[1] - h / 2,
                             t[1] + h / 2, epsabs=1e-15, epsrel=1e-13)
    assert oracle_mod.cell_integral(2, h, t) == pytest.approx(v, rel=1e-11)


@pytest.mark.parametrize("t", [(0.1, 0.0, 0.0), (0.13, -0.07, 0.21), (0.1, 0.1, 0.1), (-0.35, 0.05, 0.2),
                               (0.9, -0.4, 1.7)])
def test_cell_integral_3d_vs_quadrature(oracle_mod, t):
    h = 0.1
    v, _ = integrate.tplquad(lambda z, y, x: 1.0 / (x * x + y * y + z * z), t[0] - h / 2, t[0] + h / 2,
                             t[1] - h / 2, t[1] + h / 2, t[2] - h / 2, t[2] + h / 2, epsabs=1e-15, epsrel=1e-12)
    assert oracle_mod.cell_integral(3, h, t) == pytest.approx(v, rel=1e-10)


@pytest.mark.parametrize("dim", [2, 3])
def test_cell_integral_at_zero_is_the_self_cell_limit(oracle_mod, dim):
    """I(0) / |S^{d-1}| is the sigma -> 0 limit of the (M-iii) diagonal (golden file)."""
    g = _golden()
    h = 0.37
    area = 2 * np.pi if dim == 2 else 4 * np.pi
    key = "d2_per_h" if dim == 2 else "d3_per_h"
    assert oracle_mod.cell_integral(dim, h, (0.0,) * dim) / area == pytest.approx(g[key] * h, rel=1e-13)


@pytest.mark.parametrize("dim,m", [(2, 4), (3, 2)])
def test_cell_integral_additivity(oracle_mod, dim, m):
    """The cells at offsets -m..m tile the cube of side (2m+1) h, and the integral
    of |z|^{1-d} over a cube centred at 0 scales with its side: the sum is (2m+1) I(0)."""
    h = 0.05
    tot = sum(oracle_mod.cell_integral(dim, h, [h * v for v in o])
              for o in itertools.product(range(-m, m + 1), repeat=dim))
    assert tot == pytest.approx((2 * m + 1) * oracle_mod.cell_integral(dim, h, (0.0,) * dim), rel=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_cell_integral_far_field_expansion(oracle_mod, dim):
    """Cell average of f = |z|^{1-d}: f + h^2/24 Lap f + O(h^4);
    Lap |z|^{-1} = |z|^{-3} in 2D, Lap |z|^{-2} = 2 |z|^{-4} in 3D."""
    h = 1.0
    for r in (8.0, 16.0, 32.0):
        e = np.ones(dim) / np.sqrt(dim)
        t = r * np.array([0.8, 0.6, 0.0][:dim] if dim == 2 else [0.48, 0.6, 0.64])
        f = r ** (1 - dim)
        lap = r ** -3 if dim == 2 else 2 * r ** -4
        I = oracle_mod.cell_integral(dim, h, t)
        assert abs(I - h ** dim * (f + lap * h * h / 24)) <= 0.05 * lap * h ** (dim + 2) / 24 * (8.0 / r) ** 2
        del e


def _matrix(O, dim, n, sigma, kernel=0, scheme=1):
    N = int(np.prod(n))
    P = O.Problem(dim, n, 1.0 / max(n), kernel, np.full(N, sigma), np.full(N, 0.5 * sigma), scheme=scheme)
    return P, P.matrix()


@pytest.mark.parametrize("dim,n", [(2, (9, 9)), (3, (5, 5, 5))])
def test_free_space_row_sum_of_centre_cell(oracle_mod, dim, n):
    """sigma_t = 0 (E = 1): the centre row of the (M-ii) matrix sums the cell
    integrals over the whole grid, i.e. the integral of |z|^{1-d} over the
    domain (side n h, centred on the cell) divided by |S^{d-1}|."""
    N = int(np.prod(n))
    h = 1.0 / n[0]
    P = oracle_mod.Problem(dim, n, h, 0, np.zeros(N), np.zeros(N), scheme=1)
    A = P.matrix()
    j = N // 2
    area = 2 * np.pi if dim == 2 else 4 * np.pi
    assert A[j].sum() == pytest.approx(n[0] * oracle_mod.cell_integral(dim, h, (0.0,) * dim) / area, rel=1e-13)


@pytest.mark.parametrize("dim,n,kernel", [(2, (7, 6), 0), (2, (7, 6), 1), (3, (4, 4, 3), 0), (3, (4, 3, 3), 1)])
def test_mii_matrix_symmetric_and_close_to_miii(oracle_mod, dim, n, kernel):
    N = int(np.prod(n))
    rng = np.random.default_rng(2)
    st = np.full(N, 3.0) if kernel == 0 else rng.uniform(1.0, 5.0, N)
    h = 1.0 / max(n)
    P2 = oracle_mod.Problem(dim, n, h, kernel, st, 0.5 * st, scheme=1)
    P3 = oracle_mod.Problem(dim, n, h, kernel, st, 0.5 * st, scheme=0)
    A2, A3 = P2.matrix(), P3.matrix()
    assert np.array_equal(A2, A2.T)
    off = ~np.eye(N, dtype=bool)
    ratio = A2[off] / A3[off]
    # I(t) / (h^d |t|^{1-d}) = 1 + h^2 / (24 |t|^2) (2D), 1 + h^2 / (12 |t|^2) (3D) + O(h^4 / |t|^4)
    assert np.all(ratio > 1.0) and np.max(ratio) < 1.1
    # the apply uses the same entries as the matrix
    x = rng.uniform(-1, 1, N)
    assert np.allclose(P2.apply(x, op=2), x - A2 @ (0.5 * st * x), rtol=0, atol=1e-14)


def test_mii_gmres_equals_dense_solve(oracle_mod):
    n = (12, 12)
    N = 144
    h = 1.0 / 12
    st = np.full(N, 4.0)
    ss = np.full(N, 3.0)
    P = oracle_mod.Problem(2, n, h, 0, st, ss, scheme=1)
    A = P.matrix()
    f = np.random.default_rng(5).uniform(0, 1, N)
    U, phi, info = P.gmres(f, tol=1e-13)
    Ud = np.linalg.solve(np.eye(N) - A * ss[None, :], A @ f)
    assert info["converged"] == 1
    assert np.linalg.norm(U - Ud) <= 1e-11 * np.linalg.norm(Ud)
