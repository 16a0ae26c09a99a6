"""Pins of the U-Net reference (oracle/unet.py) against library routines, adjoint
identities and finite differences, so that a flipped tap, a transposed operand, a
dropped skip connection or a wrong pooling factor fails here."""
import numpy as np
import pytest
from scipy import signal

from oracle import unet as U

W_SMALL = (2, 3, 4)


def _rng(seed):
    return np.random.default_rng(seed)


def test_conv3_matches_scipy_correlate():
    rng = _rng(0)
    x = rng.standard_normal((3, 4, 5, 6))
    W = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    y = U.conv3(x, W, b)
    for o in range(2):
        ref = b[o] + sum(signal.correlate(x[i], W[o, i], mode="same", method="direct") for i in range(3))
        np.testing.assert_allclose(y[o], ref, rtol=1e-12, atol=1e-12)


def test_conv3_adjoints():
    rng = _rng(1)
    x = rng.standard_normal((3, 4, 4, 6))
    W = rng.standard_normal((5, 3, 3, 3, 3))
    g = rng.standard_normal((5, 4, 4, 6))
    lhs = np.sum(U.conv3(x, W, np.zeros(5)) * g)
    assert np.isclose(lhs, np.sum(x * U.conv3_input_grad(g, W)), rtol=1e-12)
    dW, db = U.conv3_weight_grad(x, g)
    assert np.isclose(lhs, np.sum(W * dW), rtol=1e-12)
    np.testing.assert_allclose(db, g.sum(axis=(1, 2, 3)), rtol=1e-12)


def test_pool_upsample():
    rng = _rng(2)
    x = rng.standard_normal((2, 4, 6, 8))
    y = rng.standard_normal((2, 2, 3, 4))
    assert np.isclose(np.sum(U.pool2(x) * y), np.sum(x * U.pool2_grad(y)), rtol=1e-12)
    assert np.isclose(np.sum(U.up2(y) * x), np.sum(y * U.up2_grad(x)), rtol=1e-12)
    np.testing.assert_allclose(U.pool2(U.up2(y)), y, rtol=0, atol=0)
    # block average at one output cell, written out
    assert np.isclose(U.pool2(x)[1, 1, 2, 3], x[1, 2:4, 4:6, 6:8].mean(), rtol=1e-14)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = _rng(3)
    a = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, -2.5e-39, 3.3e38]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(U.bf16_round(a), ref)


def _fd(fun, p, d, L0):
    """Central difference of fun along d, over the largest step (1e-6, 1e-7 or 1e-8) whose
    two one-sided differences agree (no ReLU kink inside the interval)."""
    for eps in (1e-6, 1e-7, 1e-8):
        Lp, Lm = fun(p + eps * d), fun(p - eps * d)
        fp, fm = (Lp - L0) / eps, (L0 - Lm) / eps
        if abs(fp - fm) <= 1e-5 * max(1.0, abs(fp)):
            return (Lp - Lm) / (2 * eps)
    raise AssertionError("no kink-free difference interval")


def _problem(seed, n=(8, 8, 8), B=2, widths=W_SMALL):
    rng = _rng(seed)
    X = rng.standard_normal((B, U.CIN, n[2], n[1], n[0]))
    T = rng.standard_normal((B, n[2], n[1], n[0]))
    p = rng.standard_normal(U.param_count(widths)) * 0.3
    return p, X, T


def test_param_layout():
    assert U.param_count() == sum(co * ci * k ** 3 + co for co, ci, k in U.layer_shapes())
    p = np.arange(U.param_count(W_SMALL), dtype=np.float64)
    np.testing.assert_array_equal(U.pack(U.unpack(p, W_SMALL)), p)


@pytest.mark.parametrize("layer", list(range(11)))
def test_gradient_matches_finite_differences(layer):
    """Directional derivative along a random direction inside one layer's parameters
    (central differences over a kink-free step) equals the analytic gradient."""
    p, X, T = _problem(10 + layer)
    L, g = U.loss_and_grad(p, X, T, W_SMALL)
    shapes = U.layer_shapes(W_SMALL)
    o = sum(co * ci * k ** 3 + co for co, ci, k in shapes[:layer])
    co, ci, k = shapes[layer]
    d = np.zeros_like(p)
    d[o:o + co * ci * k ** 3 + co] = _rng(100 + layer).standard_normal(co * ci * k ** 3 + co)
    fd = _fd(lambda q: U.loss_and_grad(q, X, T, W_SMALL)[0], p, d, L)
    an = float(np.dot(g, d))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (layer, fd, an)


def test_gradient_with_respect_to_skip_paths():
    """Zeroing the decoder's weights on the upsampled channels leaves only the skip paths;
    the gradient still matches finite differences in the encoder's first layers."""
    p, X, T = _problem(30)
    layers = U.unpack(p.copy(), W_SMALL)
    w1, w2, w3 = W_SMALL
    layers[6][0][:, :w3] = 0.0
    layers[8][0][:, :w2] = 0.0
    q = U.pack(layers)
    L, g = U.loss_and_grad(q, X, T, W_SMALL)
    d = np.zeros_like(q)
    d[:w1 * U.CIN * 27] = _rng(31).standard_normal(w1 * U.CIN * 27)
    fd = _fd(lambda r: U.loss_and_grad(r, X, T, W_SMALL)[0], q, d, L)
    assert abs(fd - np.dot(g, d)) <= 1e-6 * max(1.0, abs(fd))


def test_loss_is_relative_squared_error():
    p, X, T = _problem(40, B=3)
    Y = U.forward(p, X, W_SMALL)
    L, _ = U.loss_and_grad(p, X, T, W_SMALL)
    ref = np.mean([np.sum((y - t) ** 2) / np.sum(t * t) for y, t in zip(Y, T)])
    assert np.isclose(L, ref, rtol=1e-13)
    # a perfect prediction has zero loss and zero gradient in the last bias
    L0, g0 = U.loss_and_grad(p, X, Y, W_SMALL)
    assert L0 == 0.0 and g0[-1] == 0.0


def test_bf16_mode_changes_only_by_rounding():
    """BF16 weights with split (hi + lo) activations: a perturbation at the level of the
    weights' rounding (2^-9 relative), well above the activations' (2^-17)."""
    p, X, T = _problem(50)
    Y = U.forward(p, X, W_SMALL)
    Yb = U.forward(p, X, W_SMALL, bf16=True)
    d = np.linalg.norm(Yb - Y) / np.linalg.norm(Y)
    assert 1e-5 < d < 3e-2
    a = np.random.default_rng(51).standard_normal(1000)
    assert np.max(np.abs(U.bf16_split(a) - a.astype(np.float32)) / np.abs(a)) <= 2.0 ** -16


def test_preconditioner_identity_part():
    """With zero parameters the network outputs zero and z = r; the target of the exact
    correction of r = e - K e is K e / s."""
    n = (8, 8, 8)
    rng = np.random.default_rng(52)
    r = rng.standard_normal(512)
    st = rng.uniform(1, 5, 512)
    z = U.precondition(np.zeros(U.param_count(W_SMALL)), r, st, 0.5 * st, n, W_SMALL)
    np.testing.assert_array_equal(z, r)
    e = rng.standard_normal(512)
    s = np.sqrt(np.mean(r ** 2))
    np.testing.assert_allclose(U.target(r, e), (e - r) / s, rtol=1e-15)


def test_adam_first_step_is_signed_learning_rate():
    rng = _rng(60)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    q, m, v = U.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(q, p - 1e-3 * np.sign(g), rtol=0, atol=1e-9)


def test_features():
    n = (4, 8, 4)
    rng = _rng(70)
    r = rng.standard_normal(128)
    st = rng.uniform(1, 5, 128)
    F, s = U.features(r, st, 0.9 * st, n)
    assert F.shape == (3, 4, 8, 4)
    assert np.isclose(np.mean(F[0] ** 2), 1.0)
    assert np.isclose(F[1].ravel()[17], np.log(st[17])) and np.allclose(F[2], 0.9)


def test_restriction_and_extension_invariants():
    """Cell averages: a constant stays constant, the total (times f^3) is kept, averaging a
    piecewise-constant extension gives the coarse field back, and the averages of a
    linear field are its values at the block centres."""
    rng = np.random.default_rng(3)
    n, f = (8, 12, 4), 2
    nc = (4, 6, 2)
    x = rng.standard_normal(int(np.prod(n)))
    assert np.allclose(U.restrict(np.full(x.size, 3.5), n, f), 3.5, rtol=0, atol=1e-15)
    assert abs(U.restrict(x, n, f).sum() * f ** 3 - x.sum()) <= 1e-12 * np.abs(x).sum()
    y = rng.standard_normal(int(np.prod(nc)))
    assert np.allclose(U.restrict(U.prolong(y, nc, f), n, f), y, rtol=1e-15, atol=0)
    # linear field a + b.x at cell centres (i + 1/2): block averages sit at the block centres
    i2, i1, i0 = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    lin = (1.0 + 0.5 * (i0 + 0.5) - 0.25 * (i1 + 0.5) + 2.0 * (i2 + 0.5)).ravel()
    c2, c1, c0 = np.meshgrid(np.arange(nc[2]), np.arange(nc[1]), np.arange(nc[0]), indexing="ij")
    ctr = (1.0 + 0.5 * f * (c0 + 0.5) - 0.25 * f * (c1 + 0.5) + 2.0 * f * (c2 + 0.5)).ravel()
    assert np.allclose(U.restrict(lin, n, f), ctr, rtol=0, atol=1e-12)


def test_coarse_preconditioner_reduces_to_the_network_when_f_is_one():
    """With f = 1 the coarse-grid composition is the network itself; with zero parameters it
    is the identity for any f."""
    rng = np.random.default_rng(5)
    n = (8, 8, 8)
    N = 512
    p = rng.standard_normal(U.param_count()) * 0.05
    r = rng.standard_normal(N)
    st = rng.uniform(1.0, 20.0, N)
    ss = st * 0.9
    assert np.allclose(U.precondition_coarse(p, r, st, ss, n, 1), U.precondition(p, r, st, ss, n), rtol=0, atol=1e-13)
    z0 = U.precondition_coarse(np.zeros(U.param_count()), r, st, ss, n, 2)
    assert np.array_equal(z0, r)
