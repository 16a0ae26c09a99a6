"""FP64 CPU reference of the diffusion preconditioner of Sec. 4.4 ("Diffusion
Preconditioner", eq. EQ:DA).

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the CPU-baseline leg of
bench.py.  The product library never imports it.

The diffusion approximation of the transport problem for the angular average U,

    -div( D grad U ) + mu_a U = f  in the domain,   U + l dU/dn = 0  on its boundary,
    D = 1 / (d sigma_t),  mu_a = sigma_t - sigma_s,  l = 2 / (d sigma_t) = 2 D,

models the map f -> U of the integral equation, U = (I - K)^{-1} A f with K = A S,
S = diag(sigma_s).  Since (I - K)^{-1} = I + (I - K)^{-1} A S, the preconditioner is

    M r = r + L^{-1} (sigma_s r),

with L^{-1} replaced by `cycles` multigrid V-cycles from a zero start (the paper
uses a second-order finite-difference discretisation and a standard V-cycle; the
grid of the diffusion problem is the solver's grid, so no transfer is needed).

Discretisation (cell-centred, per unit volume): for cell j
    (L U)_j = sum over interior faces (j,k) of Dface (U_j - U_k) / h^2
            + sum over boundary faces of j of 2 D_j / (h (h + 2 l_j)) U_j
            + mu_a_j U_j,
    Dface = 2 D_j D_k / (D_j + D_k)  (harmonic mean),
the boundary term from the Robin condition with the boundary value extrapolated
from the cell centre (U_b + l (U_b - U_j) / (h/2) = 0).

Multigrid (the reading of "standard V-cycle"): levels by halving each axis
(ceil(n/2); an odd last coarse cell holds one fine cell) down to at most 4 cells
per axis; on each coarse level sigma_t and sigma_s are the averages of the
children and the operator is rediscretised with 2h; smoother: red-black
Gauss-Seidel (colour (i0+i1+i2) mod 2, red first), 2 sweeps before and after the
coarse correction; restriction: average of the children; prolongation:
constant (each child receives its parent's correction); coarsest level: 60
red-black sweeps.
"""
import numpy as np

PRE, POST, COARSE_SWEEPS, COARSEST = 2, 2, 60, 4


class Level:
    def __init__(self, n, h, st, ss):
        self.n = tuple(n)
        self.dim = len(n)
        self.h = h
        self.st = np.asarray(st, dtype=np.float64).reshape(self.n[::-1])
        self.ss = np.asarray(ss, dtype=np.float64).reshape(self.n[::-1])
        d = self.dim
        self.D = 1.0 / (d * self.st)
        self.mua = self.st - self.ss
        self.l = 2.0 * self.D
        # face coefficients along each array axis (axis 0 is the slowest grid axis)
        self.Df = []
        for ax in range(d):
            a = np.moveaxis(self.D, ax, 0)
            hm = 2.0 * a[:-1] * a[1:] / (a[:-1] + a[1:])
            self.Df.append(np.moveaxis(hm, 0, ax))
        # diagonal
        diag = self.mua.copy()
        for ax in range(d):
            df = np.moveaxis(self.Df[ax], ax, 0)
            dg = np.moveaxis(diag, ax, 0)
            dg[:-1] += df / h ** 2
            dg[1:] += df / h ** 2
            rob = np.moveaxis(2.0 * self.D / (h * (h + 2.0 * self.l)), ax, 0)
            dg[0] += rob[0]
            dg[-1] += rob[-1]
        self.diag = diag
        shape = self.n[::-1]
        idx = np.indices(shape).sum(axis=0)
        self.red = (idx % 2) == 0

    def offdiag(self, U):
        """sum over interior faces of Dface U_k / h^2 (the off-diagonal part, negated)."""
        out = np.zeros_like(U)
        for ax in range(self.dim):
            df = np.moveaxis(self.Df[ax], ax, 0)
            u = np.moveaxis(U, ax, 0)
            o = np.moveaxis(out, ax, 0)
            o[:-1] += df * u[1:] / self.h ** 2
            o[1:] += df * u[:-1] / self.h ** 2
        return out

    def apply(self, U):
        return self.diag * U - self.offdiag(U)

    def rbgs(self, U, b, sweeps):
        for _ in range(sweeps):
            for colour in (self.red, ~self.red):
                U = np.where(colour, (b + self.offdiag(U)) / self.diag, U)
        return U


def _coarsen(lv):
    nc = tuple((v + 1) // 2 for v in lv.n)

    def avg(F):
        out = np.zeros(nc[::-1])
        cnt = np.zeros(nc[::-1])
        for off in np.ndindex(*(2,) * lv.dim):
            sl = tuple(slice(o, None, 2) for o in off)
            part = F[sl]
            tgt = tuple(slice(0, s) for s in part.shape)
            out[tgt] += part
            cnt[tgt] += 1
        return out / cnt

    return Level(nc, 2 * lv.h, avg(lv.st), avg(lv.ss)), avg


def hierarchy(n, h, sigma_t, sigma_s):
    levels = [Level(n, h, sigma_t, sigma_s)]
    while max(levels[-1].n) > COARSEST:
        lv, _ = _coarsen(levels[-1])
        levels.append(lv)
    return levels


def _restrict(fine, r):
    _, avg = _coarsen(fine)
    return avg(r)


def _prolong(fine, e):
    out = np.zeros(fine.n[::-1])
    for off in np.ndindex(*(2,) * fine.dim):
        sl = tuple(slice(o, None, 2) for o in off)
        tgt = out[sl]
        tgt[...] = e[tuple(slice(0, s) for s in tgt.shape)]
    return out


def vcycle(levels, k, U, b):
    lv = levels[k]
    if k == len(levels) - 1:
        return lv.rbgs(U, b, COARSE_SWEEPS)
    U = lv.rbgs(U, b, PRE)
    rc = _restrict(lv, b - lv.apply(U))
    ec = vcycle(levels, k + 1, np.zeros(levels[k + 1].n[::-1]), rc)
    U = U + _prolong(lv, ec)
    return lv.rbgs(U, b, POST)


def solve_approx(levels, b, cycles):
    """`cycles` V-cycles for L U = b from U = 0 (b flat, cell order x fastest)."""
    lv = levels[0]
    B = np.asarray(b, dtype=np.float64).reshape(lv.n[::-1])
    U = np.zeros_like(B)
    for _ in range(cycles):
        U = vcycle(levels, 0, U, B)
    return U.reshape(-1)


def apply(r, dim, n, h, sigma_t, sigma_s, cycles=2, levels=None):
    """z = r + (cycles V-cycles for L e = sigma_s r)."""
    if levels is None:
        levels = hierarchy(tuple(n), h, sigma_t, sigma_s)
    r = np.asarray(r, dtype=np.float64)
    return r + solve_approx(levels, np.asarray(sigma_s) * r, cycles)


def matrix(n, h, sigma_t, sigma_s):
    """L as a dense matrix assembled face by face (small grids; for the pins)."""
    n = tuple(n)
    dim = len(n)
    N = int(np.prod(n))
    st = np.asarray(sigma_t, dtype=np.float64)
    ss = np.asarray(sigma_s, dtype=np.float64)
    D = 1.0 / (dim * st)
    L = np.diag(st - ss)
    strides = [int(np.prod(n[:a])) for a in range(dim)]
    for j in range(N):
        i = [(j // strides[a]) % n[a] for a in range(dim)]
        for a in range(dim):
            for s in (-1, 1):
                ia = i[a] + s
                if 0 <= ia < n[a]:
                    k = j + s * strides[a]
                    df = 2 * D[j] * D[k] / (D[j] + D[k])
                    L[j, j] += df / h ** 2
                    L[j, k] -= df / h ** 2
                else:
                    L[j, j] += 2 * D[j] / (h * (h + 4 * D[j]))
    return L
