"""FP64 CPU reference of the FFT-based preconditioner of Sec. 4.4 ("FFT-based
Preconditioner", eqs. EQ: FFT and EQ:SOL FFT).

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the CPU-baseline leg of
bench.py.  The product library never imports it.

The idea of the paper: when sigma_t varies little, the equation with the medium
replaced by its mean is a good approximation of the true one, and on a regular
grid that equation is a convolution, so it can be inverted with FFTs on a
periodic box of twice the size with zero extension of the residual and
restriction of the result.  Here it is written out for the discrete operator of
the solver, (I - K S) with K the collocation matrix (M-iii, Sec. 3.2) and S =
diag(sigma_s):

  mean medium   sbar_t = mean of sigma_t over the cells, sbar_s = mean of sigma_s;
  kernel array  w on a periodic grid of m_i cells per axis, w[i] = h^d G(h o(i))
                with o(i)_a = i_a if i_a <= m_a / 2 else i_a - m_a, G the
                homogeneous kernel exp(-sbar_t r) / (omega_d r^(d-1)), and
                w[0] = the self-cell integral of the medium sbar_t (the
                diagonal of the M-iii matrix);
  symbol        c = 1 - sbar_s DFT(w)   (real: w is even in every axis);
  apply         z = P IDFT( DFT(E r) / c ),
                E the zero extension of a grid field to the periodic grid and P
                the restriction back to the grid.

With approach (M-ii) (scheme=1; Sec. 3.2, Remark 3.1) the kernel array holds that
discretisation's entries instead: w[i] = E(h o(i)) I(h o(i)) / |S^{d-1}| with I the
integral of |z|^{1-d} over the cell of side h centred at the offset (the oracle's
cell_integral), including i = 0 (E = 1 there).

Period.  The paper extends [0, 1]^d to [0, 2]^d, i.e. m_i = 2 n_i.  Any
m_i >= 2 n_i - 1 keeps every pair offset of the grid distinct modulo m_i, so
that P C E = I - K_bar S_bar exactly for the mean medium (C the periodic
operator with symbol c).  m_i is the smallest integer >= 2 n_i whose prime
factors are all <= 7; it equals 2 n_i unless 2 n_i has a larger prime factor.

The discrete FFTs are numpy's (a library primitive standing for the DFT).
Fields are flat float64 arrays in the solver's cell order (x fastest).
"""
import numpy as np

from . import oracle as O


def smooth_period(n):
    """Smallest integer >= 2 n whose prime factors are all <= 7."""
    m = 2 * int(n)
    while True:
        k = m
        for p in (2, 3, 5, 7):
            while k % p == 0:
                k //= p
        if k == 1:
            return m
        m += 1


def periods(n):
    return tuple(smooth_period(v) for v in n)


def mean_medium(sigma_t, sigma_s):
    """The constant medium the preconditioner inverts (Sec. 4.4: the mean of the
    coefficient over the domain)."""
    return float(np.mean(sigma_t)), float(np.mean(sigma_s))


def self_cell(dim, n, h, sbar_t, scheme=0):
    """Diagonal of the matrix for the constant medium sbar_t (the oracle's
    singular self-cell quadrature for M-iii, I(0) / |S^{d-1}| for M-ii)."""
    N = int(np.prod(n))
    return O.Problem(dim, n, h, 0, np.full(N, sbar_t), scheme=scheme).self_cell(0)


def kernel_array(dim, n, h, sbar_t, dself, scheme=0):
    """w on the periodic grid, array shape (m_{d-1}, ..., m_0) (x fastest)."""
    m = periods(n)
    omega = 2.0 * np.pi if dim == 2 else 4.0 * np.pi
    axes, iaxes = [], []
    for a in range(dim):
        i = np.arange(m[a])
        o = np.where(i <= m[a] // 2, i, i - m[a])
        iaxes.append(np.abs(o))
        axes.append(o.astype(np.float64) * h)
    grids = np.meshgrid(*axes[::-1], indexing="ij")        # slowest axis first
    r = np.sqrt(sum(g * g for g in grids))
    w = np.empty_like(r)
    nz = r > 0
    if scheme == 1:
        # the cell integral depends on |o_a| only: evaluate each distinct offset once
        ig = np.meshgrid(*iaxes[::-1], indexing="ij")
        cache = {}
        it = np.nditer(ig, flags=["multi_index"])
        Ivals = np.empty_like(r)
        for _ in it:
            key = tuple(int(g[it.multi_index]) for g in ig)[::-1]      # x first
            if key not in cache:
                cache[key] = O.cell_integral(dim, h, [h * v for v in key])
            Ivals[it.multi_index] = cache[key]
        w[nz] = np.exp(-sbar_t * r[nz]) * Ivals[nz] / omega
    else:
        w[nz] = h ** dim * np.exp(-sbar_t * r[nz]) / (omega * r[nz] ** (dim - 1))
    w[~nz] = dself
    return w


def symbol(dim, n, h, sigma_t, sigma_s, scheme=0):
    """c = 1 - sbar_s DFT(w) (real array of the periodic grid's shape)."""
    sbar_t, sbar_s = mean_medium(sigma_t, sigma_s)
    w = kernel_array(dim, n, h, sbar_t, self_cell(dim, n, h, sbar_t, scheme), scheme)
    return 1.0 - sbar_s * np.fft.fftn(w).real


def _extend(x, n, m):
    e = np.zeros(m[::-1])
    e[tuple(slice(0, v) for v in n[::-1])] = np.asarray(x, dtype=np.float64).reshape(n[::-1])
    return e


def _restrict(e, n):
    return np.ascontiguousarray(e[tuple(slice(0, v) for v in n[::-1])]).reshape(-1)


def apply(r, dim, n, h, sigma_t, sigma_s, c=None, scheme=0):
    """z = P IDFT(DFT(E r) / c) for a flat residual r (or columns r[:, k])."""
    n = tuple(n)
    m = periods(n)
    if c is None:
        c = symbol(dim, n, h, sigma_t, sigma_s, scheme)
    r = np.asarray(r, dtype=np.float64)
    if r.ndim == 2:
        return np.stack([apply(r[:, k], dim, n, h, sigma_t, sigma_s, c, scheme) for k in range(r.shape[1])], axis=1)
    return _restrict(np.fft.ifftn(np.fft.fftn(_extend(r, n, m)) / c).real, n)


def periodic_operator(x, dim, n, h, sigma_t, sigma_s, c=None, scheme=0):
    """P C E x: the periodic operator the preconditioner inverts, restricted to
    the grid.  For a constant medium it is the solver's I - K S."""
    n = tuple(n)
    m = periods(n)
    if c is None:
        c = symbol(dim, n, h, sigma_t, sigma_s, scheme)
    return _restrict(np.fft.ifftn(np.fft.fftn(_extend(x, n, m)) * c).real, n)
