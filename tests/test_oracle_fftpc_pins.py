"""Pins of the FFT-based preconditioner's reference (oracle/fftpc.py, Sec. 4.4)
against things other than itself: the dense C oracle's operator (for a constant
medium the periodic operator restricted to the grid is exactly I - K S), a
brute-force circulant matrix solved by LAPACK, and closed-form special cases."""
import numpy as np
import pytest

from oracle import fftpc as F
from paper_1610_00835_amd import inputs


def _const(dim, n, st, ss):
    N = int(np.prod(n))
    return np.full(N, st), np.full(N, ss)


@pytest.mark.parametrize("n", [7, 8, 9, 11, 12, 13, 16, 23, 64, 100, 128])
def test_smooth_period(n):
    m = F.smooth_period(n)
    assert m >= 2 * n
    k = m
    for p in (2, 3, 5, 7):
        while k % p == 0:
            k //= p
    assert k == 1
    for q in range(2 * n, m):                  # nothing smaller qualifies
        k = q
        for p in (2, 3, 5, 7):
            while k % p == 0:
                k //= p
        assert k != 1
    if n in (8, 9, 12, 16, 64, 100, 128):
        assert m == 2 * n


@pytest.mark.parametrize("dim,n,kernel", [(2, (7, 6), 0), (3, (5, 4, 3), 0), (3, (6, 5, 4), 1), (2, (11, 9), 1)])
def test_periodic_operator_is_solver_operator_for_constant_medium(oracle_mod, dim, n, kernel):
    """P C E x = x - A (sigma_s x) with A the dense M-iii matrix of the C oracle:
    pins the kernel array (h^d, omega_d, r^(d-1), decay), its wrap-around, the
    self-cell entry and the sign and scale of the symbol."""
    h = 1.0 / max(n)
    st, ss = _const(dim, n, 3.5, 2.75)
    P = oracle_mod.Problem(dim, n, h, kernel, st, ss)
    x = np.random.default_rng(3).uniform(-1, 1, P.N)
    ref = P.apply(x, op=2)
    got = F.periodic_operator(x, dim, n, h, st, ss)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("dim,n,kernel", [(2, (7, 6), 0), (3, (5, 4, 3), 1)])
def test_periodic_operator_is_solver_operator_mii(oracle_mod, dim, n, kernel):
    """The same identity with the (M-ii) entries (Sec. 3.2, Remark 3.1)."""
    h = 1.0 / max(n)
    st, ss = _const(dim, n, 3.5, 2.75)
    P = oracle_mod.Problem(dim, n, h, kernel, st, ss, scheme=1)
    x = np.random.default_rng(4).uniform(-1, 1, P.N)
    ref = P.apply(x, op=2)
    got = F.periodic_operator(x, dim, n, h, st, ss, scheme=1)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def _circulant(w, m, sbar_s):
    """Dense matrix of the periodic operator I - sbar_s (w * .) by brute force."""
    idx = np.stack(np.meshgrid(*[np.arange(v) for v in m[::-1]], indexing="ij"), -1).reshape(-1, len(m))
    M = idx.shape[0]
    C = np.eye(M)
    for a in range(M):
        d = (idx[a][None, :] - idx) % np.array(m[::-1])
        C[a] -= sbar_s * w[tuple(d.T)]
    return C, idx


@pytest.mark.parametrize("dim,n", [(3, (3, 2, 2)), (2, (3, 5)), (3, (2, 3, 3))])
def test_apply_is_restricted_inverse_of_periodic_operator(oracle_mod, dim, n):
    """z = P C^{-1} E r, with C built entry by entry and solved by LAPACK; a
    heterogeneous medium enters through its means."""
    h = 1.0 / max(n)
    rng = np.random.default_rng(11)
    N = int(np.prod(n))
    st = rng.uniform(2.0, 6.0, N)
    ss = st * rng.uniform(0.5, 0.95, N)
    sbar_t, sbar_s = F.mean_medium(st, ss)
    assert sbar_t == pytest.approx(st.sum() / N, rel=1e-15)
    m = F.periods(n)
    w = F.kernel_array(dim, n, h, sbar_t, F.self_cell(dim, n, h, sbar_t))
    C, idx = _circulant(w, m, sbar_s)
    r = rng.uniform(-1, 1, N)
    inside = np.all(idx < np.array(n[::-1]), axis=1)
    e = np.zeros(C.shape[0])
    e[inside] = r.reshape(n[::-1]).reshape(-1)
    ref = np.linalg.solve(C, e)[inside]
    got = F.apply(r, dim, n, h, st, ss)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    R = np.stack([r, 2 * r[::-1]], axis=1)                     # columns one by one
    G = F.apply(R, dim, n, h, st, ss)
    assert np.allclose(G[:, 0], got, rtol=0, atol=1e-15) and np.allclose(G[:, 1], F.apply(2 * r[::-1], dim, n, h, st, ss), rtol=0, atol=1e-15)


def test_no_scattering_is_identity():
    n = (6, 5, 4)
    st, ss = _const(3, n, 4.0, 0.0)
    r = np.random.default_rng(2).uniform(-1, 1, int(np.prod(n)))
    assert np.max(np.abs(F.apply(r, 3, n, 1 / 6, st, ss) - r)) <= 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_symbol_real_positive_minimum_at_zero_frequency(dim):
    """The kernel array is positive and even, so its DFT is real with the largest
    value at zero frequency: c >= c[0] = 1 - sbar_s sum(w) > 0 for albedo < 1."""
    n = (12,) * dim
    h = 1.0 / 12
    st, ss = _const(dim, n, 8.0, 0.99 * 8.0)
    sbar_t, sbar_s = F.mean_medium(st, ss)
    w = F.kernel_array(dim, n, h, sbar_t, F.self_cell(dim, n, h, sbar_t))
    assert np.all(w > 0)
    spec = np.fft.fftn(w)
    assert np.max(np.abs(spec.imag)) <= 1e-12 * abs(spec[(0,) * dim])
    c = F.symbol(dim, n, h, st, ss)
    assert c[(0,) * dim] == pytest.approx(1 - sbar_s * w.sum(), rel=1e-12)
    assert c.min() >= c[(0,) * dim] - 1e-12 and c[(0,) * dim] > 0


def test_interior_residual_nearly_inverted_for_constant_medium(oracle_mod):
    """For a constant medium and a residual far from the boundary (the paper's
    assumption), z nearly solves (I - K S) z = r; the identity does not."""
    n = (12, 12, 12)
    h = 1.0 / 12
    st, ss = _const(3, n, 20.0, 0.99 * 20.0)
    P = oracle_mod.Problem(3, n, h, 0, st, ss)
    x = inputs.centres(n, h)
    r = np.exp(-np.sum((x - 0.5) ** 2, axis=1) / (2 * 0.08 ** 2))
    z = F.apply(r, 3, n, h, st, ss)
    res_pc = np.linalg.norm(r - P.apply(z, op=2)) / np.linalg.norm(r)
    res_id = np.linalg.norm(r - P.apply(r, op=2)) / np.linalg.norm(r)
    assert res_pc < 0.05 * res_id and res_pc < 0.05
