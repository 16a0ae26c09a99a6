"""Pins of the transport-sweep reference (oracle/transport.py, Algorithm 1 S.3)
against closed forms and the C oracle: constant medium and source (exact solution
Q (1 - exp(-sigma s)) / sigma), the source Q = sigma_t (exact solution
1 - exp(-optical depth to the boundary), with the depth from the C oracle's ray
rule), mirror symmetry, and the interpolation against scipy."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from oracle import transport as T


def _dirs(dim, k, seed=0):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((k, dim))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    axes = np.eye(dim)
    return np.concatenate([d, axes, -axes])


@pytest.mark.parametrize("dim,n", [(2, (9, 7)), (3, (6, 5, 4))])
def test_constant_medium_and_source_exact(dim, n):
    h = 1.0 / max(n)
    N = int(np.prod(n))
    sig, q = 3.7, 1.3
    cells = np.arange(N)
    idx = np.stack(np.unravel_index(cells, n[::-1])[::-1], axis=1)
    x = h * (idx + 0.5)
    for v in _dirs(dim, 5):
        phi = T.sweep(np.full(N, q), np.full(N, sig), n, h, v)
        sb = T.boundary_distance(x, v, n, h)
        exact = q * -np.expm1(-sig * sb) / sig
        assert np.max(np.abs(phi - exact)) <= 1e-14 * q / sig


@pytest.mark.parametrize("dim,n", [(2, (8, 6)), (3, (5, 6, 4))])
def test_source_equal_to_attenuation_telescopes(oracle_mod, dim, n):
    """Q = sigma_t: every step contributes exp(-tau_{k-1}) - exp(-tau_k), so
    Phi = 1 - exp(-tau) with tau the midpoint-rule optical depth of the C oracle
    (same segment, same number of steps)."""
    h = 1.0 / max(n)
    N = int(np.prod(n))
    st = np.random.default_rng(4).uniform(1.0, 9.0, N)
    P = oracle_mod.Problem(dim, n, h, 1, st)
    cells = np.arange(0, N, 3)
    idx = np.stack(np.unravel_index(cells, n[::-1])[::-1], axis=1)
    x = h * (idx + 0.5)
    for v in _dirs(dim, 3, seed=1):
        phi = T.sweep(st, st, n, h, v, cells)
        sb = T.boundary_distance(x, v, n, h)
        m = np.maximum(1, np.ceil(sb / (0.5 * h) * (1.0 - 1e-12))).astype(int)
        for i in range(len(cells)):
            xa = np.zeros(3)
            xb = np.zeros(3)
            xa[:dim] = x[i]
            xb[:dim] = x[i] - sb[i] * v
            tau = P.tau(xa, xb, int(m[i]))
            assert phi[i] == pytest.approx(-np.expm1(-tau), rel=1e-12, abs=1e-15)


def test_mirror_symmetry():
    """A medium and source symmetric under x -> L - x give Phi(x, v) = Phi(L - x, -v)."""
    n = (8, 6, 5)
    h = 1.0 / 8
    rng = np.random.default_rng(7)
    a = rng.uniform(1, 5, n[::-1])
    st = (a + a[::-1, ::-1, ::-1]).reshape(-1)
    b = rng.uniform(0, 2, n[::-1])
    q = (b + b[::-1, ::-1, ::-1]).reshape(-1)
    N = st.size
    mirror = np.arange(N)[::-1]
    for v in _dirs(3, 4, seed=3):
        p1 = T.sweep(q, st, n, h, v)
        p2 = T.sweep(q, st, n, h, -v)
        assert np.max(np.abs(p1 - p2[mirror])) <= 1e-13 * np.max(np.abs(p1))


def test_interpolation_matches_scipy():
    n = (7, 5, 4)
    h = 0.1
    rng = np.random.default_rng(2)
    F = rng.uniform(-1, 1, n[::-1])
    axes = [h * (np.arange(v) + 0.5) for v in n[::-1]]
    ref = RegularGridInterpolator(axes, F, method="linear")
    p = rng.uniform(0, 1, (200, 3)) * np.array(n) * h
    pc = np.clip(p, h / 2, np.array(n) * h - h / 2)
    assert np.allclose(T._interp(F.reshape(-1), n, h, p), ref(pc[:, ::-1]), rtol=0, atol=1e-14)


def test_recover_forms_the_source():
    n = (6, 6)
    h = 1 / 6
    N = 36
    rng = np.random.default_rng(1)
    st = rng.uniform(1, 3, N)
    ss = 0.5 * st
    U = rng.uniform(0, 1, N)
    f = rng.uniform(0, 1, N)
    d = _dirs(2, 2)
    out = T.recover(U, f, st, ss, n, h, d)
    assert out.shape == (N, len(d))
    assert np.allclose(out[:, 0], T.sweep(ss * U + f, st, n, h, d[0]), rtol=0, atol=0)
    assert np.all(T.recover(np.zeros(N), np.zeros(N), st, ss, n, h, d) == 0.0)


def test_angular_average_converges_to_U(oracle_mod):
    """Algorithm 1 is consistent: U solves the integral equation (S.2) and is the
    angular average of the Phi that S.3 recovers from it.  On the 2D recipe (64^2 at
    h = 1/64, approach (M-ii), 256 directions) the average differs from U by
    under 1e-3 and the difference falls by more than 3x from 32^2 to 64^2."""
    from paper_1610_00835_amd import inputs
    errs = []
    for n0 in (32, 64):
        case = inputs.make_case("c1", n=(n0, n0))
        P = oracle_mod.Problem(2, case["n"], case["h"], 0, case["sigma_t"], case["sigma_s"], scheme=1)
        U, _, info = P.gmres(case["f"], tol=1e-12)
        th = 2 * np.pi * (np.arange(256) + 0.5) / 256
        dirs = np.stack([np.cos(th), np.sin(th)], 1)
        avg = T.recover(U, case["f"], case["sigma_t"], case["sigma_s"], case["n"], case["h"], dirs).mean(1)
        errs.append(np.linalg.norm(avg - U) / np.linalg.norm(U))
    assert errs[1] < 1e-3 and errs[0] > 3 * errs[1]
