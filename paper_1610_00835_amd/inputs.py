"""Seeded synthetic inputs: media (sigma_t, sigma_s) and sources f on a cell-centred grid.

This module holds no arithmetic of the method: it only draws coefficient
fields and source terms.  Both the oracle side (tests) and the GPU side
(tests, bench) take their inputs from here, so they consume identical bits.

The paper's own sources exist only as a figure (Sec. 5, Fig. 1), so smooth
Gaussian sources of the sizes below stand in for them.  Grid convention:
cell (i0,i1,i2) has centre h (i + 1/2) per axis, arrays are flat and
x-fastest (j = i0 + n0 (i1 + n1 i2)).  Random draws use numpy's PCG64
``default_rng(seed)`` in the order stated in each recipe.
"""
import numpy as np

KERNEL_HOMOGENEOUS = 0
KERNEL_RAY = 1


def centres(n, h):
    """Cell centres, shape (N, d), x-fastest."""
    axes = [h * (np.arange(m) + 0.5) for m in n]
    mesh = np.meshgrid(*axes, indexing="ij")          # mesh[a][i0, i1, ...]
    pts = np.stack([m.transpose(tuple(reversed(range(len(n))))).reshape(-1) for m in mesh], axis=1)
    return pts


def _gauss(x, c, w):
    d2 = np.sum((x - np.asarray(c)[None, :]) ** 2, axis=1)
    return np.exp(-d2 / (2.0 * w * w))


def _bumps(x, rng, k=4, width=0.05):
    """k Gaussian bumps: centres U[0.2,0.8]^d drawn first, then amplitudes U[0.5,1]."""
    d = x.shape[1]
    c = rng.uniform(0.2, 0.8, size=(k, d))
    a = rng.uniform(0.5, 1.0, size=k)
    f = np.zeros(x.shape[0])
    for i in range(k):
        f += a[i] * _gauss(x, c[i], width)
    return f


def _blob_medium(x, rng, base, k=8):
    """base + sum_k a_k exp(-|x-c_k|^2/(2 w_k^2)); draw order a (U[2,10]), c (U[0.2,0.8]^d), w (U[0.05,0.15])."""
    d = x.shape[1]
    a = rng.uniform(2.0, 10.0, size=k)
    c = rng.uniform(0.2, 0.8, size=(k, d))
    w = rng.uniform(0.05, 0.15, size=k)
    s = np.full(x.shape[0], float(base))
    for i in range(k):
        s += a[i] * _gauss(x, c[i], w[i])
    return s


def _face_sources(x, n, h, rng, nrhs, width=0.03):
    """nrhs Gaussians centred 2h inside a random face of the unit cube.

    Per source: face = rng.integers(2 d) (axis = face // 2, high side if odd),
    then the in-face coordinates U[0.2,0.8]^(d-1).
    """
    d = x.shape[1]
    F = np.zeros((x.shape[0], nrhs))
    for b in range(nrhs):
        face = int(rng.integers(2 * d))
        axis, high = face // 2, face % 2
        c = np.empty(d)
        other = rng.uniform(0.2, 0.8, size=d - 1)
        c[[a for a in range(d) if a != axis]] = other
        ext = n[axis] * h
        c[axis] = ext - 2.0 * h if high else 2.0 * h
        F[:, b] = _gauss(x, c, width)
    return F


def make_case(name, n=None, seed=0, nrhs=None):
    """Return a dict with dim, n, h, kernel, sigma_t, sigma_s, f (N or N x nrhs), name.

    Recipes (unit square / cube, h = 1 / max(n)):
      c1: 2D 64^2, sigma_t = 2, sigma_s = 1, f = exp(-|x-(.5,.5)|^2 / (2 0.1^2)), homogeneous kernel.
      c2: 3D 32^3, sigma_t = 5, sigma_s = 4, f = 4 bumps of width 0.05 (seeded), homogeneous kernel.
      c3: 3D 64^3, sigma_t = 1 + 8 blobs (seeded), sigma_s = 0.9 sigma_t, f = 4 bumps drawn after
          the medium from the same stream, ray-quadrature kernel.
      c4: the c3 medium of `seed` and `nrhs` (64) face sources from default_rng(seed + 100).
      c5: 3D 128^3, sigma_t = U[5,50] (one draw) + 8 blobs, sigma_s = 0.99 sigma_t, f = one face source.
    `n` overrides the grid (parity tests use small grids with the same recipe).
    """
    name = name.lower()
    if name == "c1":
        n = tuple(n or (64, 64))
        h = 1.0 / max(n)
        x = centres(n, h)
        N = x.shape[0]
        st = np.full(N, 2.0)
        ss = np.full(N, 1.0)
        f = _gauss(x, (0.5, 0.5), 0.1)
        kern = KERNEL_HOMOGENEOUS
    elif name == "c2":
        n = tuple(n or (32, 32, 32))
        h = 1.0 / max(n)
        x = centres(n, h)
        N = x.shape[0]
        rng = np.random.default_rng(seed)
        st = np.full(N, 5.0)
        ss = np.full(N, 4.0)
        f = _bumps(x, rng)
        kern = KERNEL_HOMOGENEOUS
    elif name == "c3":
        n = tuple(n or (64, 64, 64))
        h = 1.0 / max(n)
        x = centres(n, h)
        rng = np.random.default_rng(seed)
        st = _blob_medium(x, rng, 1.0)
        ss = 0.9 * st
        f = _bumps(x, rng)
        kern = KERNEL_RAY
    elif name == "c4":
        n = tuple(n or (64, 64, 64))
        h = 1.0 / max(n)
        x = centres(n, h)
        rng = np.random.default_rng(seed)
        st = _blob_medium(x, rng, 1.0)
        ss = 0.9 * st
        f = _face_sources(x, n, h, np.random.default_rng(seed + 100), nrhs or 64)
        kern = KERNEL_RAY
    elif name == "c5":
        n = tuple(n or (128, 128, 128))
        h = 1.0 / max(n)
        x = centres(n, h)
        rng = np.random.default_rng(seed)
        base = rng.uniform(5.0, 50.0)
        st = _blob_medium(x, rng, base)
        ss = 0.99 * st
        f = _face_sources(x, n, h, rng, nrhs or 1)
        if (nrhs or 1) == 1:
            f = f[:, 0]
        kern = KERNEL_RAY
    else:
        raise ValueError("unknown case %r" % name)
    return {"name": name, "dim": len(n), "n": n, "h": h, "kernel": kern,
            "sigma_t": np.ascontiguousarray(st), "sigma_s": np.ascontiguousarray(ss),
            "f": np.ascontiguousarray(f) if f.ndim == 1 else np.asfortranarray(f)}


def random_vector(N, seed, nrhs=None):
    """Seeded test vector(s) U[-1,1] for parity of the apply."""
    rng = np.random.default_rng(seed)
    if nrhs is None:
        return rng.uniform(-1.0, 1.0, size=N)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(N, nrhs)))
