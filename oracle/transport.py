"""FP64 CPU reference of Algorithm 1 step S.3: recovering the angular solution
Phi(x, v) from U by the scattering-free transport equation

    v . grad Phi + sigma_t Phi = Q,   Phi = 0 on the inflow boundary,
    Q = sigma_s U + f                       (S.3 (i)),

solved along characteristics (S.3 (ii)): Phi(x, v) is the integral over the ray
from x backwards to the domain boundary of exp(-optical depth) Q.

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the CPU-baseline leg of
bench.py.  The product library never imports it.

Discretisation (the paper leaves the transport solver open; this is the reading):
the ray x - t v, 0 <= t <= s_b (s_b = distance to the boundary of the box
[0, n_a h]^d) is cut into m = max(1, ceil(s_b / (h/2) (1 - 1e-12))) equal steps
(the relative margin keeps the count of an exact multiple of h/2, as on every
axis-parallel ray, independent of the last bit of s_b) of length
D; on step k sigma_t and Q take their values at the step midpoint t_k = (k - 1/2) D
(d-linear interpolation of the cell values, clamped to the cell-centre box, as
the kernel's ray rule does), and the step is integrated exactly for those
constants (step characteristics):

    Phi = sum_k exp(-tau_{k-1}) Q_k (1 - exp(-sigma_k D)) / sigma_k,
    tau_k = tau_{k-1} + sigma_k D,  tau_0 = 0.

For constant sigma_t and Q this is the exact solution Q (1 - exp(-sigma s_b)) / sigma.
"""
import numpy as np


def _interp(field, n, h, p):
    """d-linear interpolation of a cell-centred field at points p (M x d), each
    coordinate clamped to [h/2, n_a h - h/2] (constant extension)."""
    dim = len(n)
    F = np.asarray(field, dtype=np.float64).reshape(n[::-1])
    i0, t = [], []
    for a in range(dim):
        u = np.clip(p[:, a] / h - 0.5, 0.0, n[a] - 1.0)
        k = np.minimum(np.floor(u).astype(np.int64), max(n[a] - 2, 0))
        i0.append(k)
        t.append(u - k if n[a] > 1 else np.zeros_like(u))
    acc = np.zeros(p.shape[0])
    for corner in range(1 << dim):
        w = np.ones(p.shape[0])
        idx = []
        for a in range(dim):
            bit = (corner >> a) & 1
            ia = np.minimum(i0[a] + bit, n[a] - 1)
            idx.append(ia)
            w = w * (t[a] if bit else 1.0 - t[a])
        acc += w * F[tuple(idx[::-1])]
    return acc


def boundary_distance(x, v, n, h):
    """Distance from points x (M x d) backwards along -v to the box boundary."""
    s = np.full(x.shape[0], np.inf)
    for a in range(len(n)):
        if v[a] > 0:
            s = np.minimum(s, x[:, a] / v[a])
        elif v[a] < 0:
            s = np.minimum(s, (n[a] * h - x[:, a]) / (-v[a]))
    return s


def sweep(q, sigma_t, n, h, v, cells=None):
    """Phi(x_j, v) for the cells j (default all), for source q and one unit direction v."""
    n = tuple(n)
    dim = len(n)
    N = int(np.prod(n))
    cells = np.arange(N) if cells is None else np.asarray(cells)
    idx = np.stack(np.unravel_index(cells, n[::-1])[::-1], axis=1)
    x = h * (idx + 0.5)
    v = np.asarray(v, dtype=np.float64)
    sb = boundary_distance(x, v, n, h)
    m = np.maximum(1, np.ceil(sb / (0.5 * h) * (1.0 - 1e-12))).astype(np.int64)
    D = sb / m
    phi = np.zeros(len(cells))
    tau = np.zeros(len(cells))
    for k in range(1, int(m.max()) + 1):
        live = k <= m
        tk = (k - 0.5) * D
        p = x - tk[:, None] * v[None, :]
        sg = _interp(sigma_t, n, h, p)
        qk = _interp(q, n, h, p)
        sd = sg * D
        step = np.where(sd > 1e-300, -np.expm1(-sd) / np.where(sg > 0, sg, 1.0), D)
        phi += np.where(live, np.exp(-tau) * qk * step, 0.0)
        tau += np.where(live, sd, 0.0)
    return phi


def recover(U, f, sigma_t, sigma_s, n, h, dirs, cells=None):
    """Step S.3: Q = sigma_s U + f, then one sweep per direction; returns (cells x ndir)."""
    q = np.asarray(sigma_s) * np.asarray(U) + np.asarray(f)
    return np.stack([sweep(q, sigma_t, n, h, d, cells) for d in np.atleast_2d(dirs)], axis=1)
