"""FP64 CPU reference of the learned right preconditioner: a three-level 3D
convolutional U-Net, its loss and its gradient.

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the CPU-baseline leg of
bench.py.  The product library never imports it.

The preconditioner is not part of the paper's method; it maps a residual r of
(I - K) U = phi (Sec. 2, Eq. (2.4) and Algorithm 1, step S.2) plus the medium to
an approximate correction e with (I - K) e ~ r, and is used as a right
preconditioner of flexible GMRES.  Everything here is plain numpy in float64.

Grid and tensors.  A field on an n0 x n1 x n2 cell grid is an array [n2][n1][n0]
(x fastest, the cell order of the solver).  Activations are [C][n2][n1][n0];
a batch is [B][C][n2][n1][n0].  Every n_i must be a multiple of 4 (two 2x
poolings).

Network (widths w1, w2, w3; 3 input channels; one output channel):
  L1  3x3x3 conv  cin      -> w1, ReLU      (full grid)
  L2  3x3x3 conv  w1       -> w1, ReLU      = skip s1
      2x2x2 average pool
  L3  3x3x3 conv  w1       -> w2, ReLU      (half grid)
  L4  3x3x3 conv  w2       -> w2, ReLU      = skip s2
      2x2x2 average pool
  L5  3x3x3 conv  w2       -> w3, ReLU      (quarter grid)
  L6  3x3x3 conv  w3       -> w3, ReLU
      nearest 2x upsampling, concatenation [upsampled, s2]
  L7  3x3x3 conv  w3 + w2  -> w2, ReLU      (half grid)
  L8  3x3x3 conv  w2       -> w2, ReLU
      nearest 2x upsampling, concatenation [upsampled, s1]
  L9  3x3x3 conv  w2 + w1  -> w1, ReLU      (full grid)
  L10 3x3x3 conv  w1       -> w1, ReLU
  L11 1x1x1 conv  w1       -> 1             (no activation)
A 3x3x3 convolution is a cross-correlation with zero padding:
  out[o][z][y][x] = b[o] + sum_{i, a, c, d in {-1,0,1}} W[o][i][a+1][c+1][d+1] in[i][z+a][y+c][x+d].

Parameters.  One flat float vector, layer by layer: W (shape [cout][cin][k][k][k])
then b ([cout]).

Preconditioner.  For a residual r (scale s = rms(r)) the network output y on the
features gives z = r + s y: the identity part of the correction passes through
exactly and the network supplies the rest.  For a correction e with
(I - K) e = r, e - r = K e is the part the (smoothing) transport operator
produces, so the training target is t = (e - r) / s.

Loss.  Mean over the batch of the relative squared error
  L = (1/B) sum_b ||y_b - t_b||^2 / ||t_b||^2.

Rounding mode.  With bf16=True the 3x3x3 convolutions of the forward pass and
the input-gradient convolutions of the backward pass take their weights rounded
to bfloat16 and their activations (resp. output gradients) as the sum of two
bfloat16 parts, hi = bf16(x) and lo = bf16(x - hi) (round to nearest even); sums
stay in float64.  Weight gradients, biases, the 1x1 layer, pooling and
upsampling use unrounded values.  This is where a BF16-operand, FP32-accumulate
implementation rounds, so the two agree to accumulation order.
"""
import numpy as np

CIN = 3


def layer_shapes(widths=(16, 32, 64), cin=CIN):
    """(cout, cin, k) of L1..L11."""
    w1, w2, w3 = widths
    return [(w1, cin, 3), (w1, w1, 3), (w2, w1, 3), (w2, w2, 3), (w3, w2, 3), (w3, w3, 3),
            (w2, w3 + w2, 3), (w2, w2, 3), (w1, w2 + w1, 3), (w1, w1, 3), (1, w1, 1)]


def param_count(widths=(16, 32, 64), cin=CIN):
    return sum(co * ci * k ** 3 + co for co, ci, k in layer_shapes(widths, cin))


def unpack(params, widths=(16, 32, 64), cin=CIN):
    """Flat vector -> list of (W, b) views, float64."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for co, ci, k in layer_shapes(widths, cin):
        nw = co * ci * k ** 3
        W = p[o:o + nw].reshape(co, ci, k, k, k)
        o += nw
        b = p[o:o + co]
        o += co
        out.append((W, b))
    assert o == p.size, "parameter vector has the wrong length"
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16_split(a):
    """hi + lo with hi = bf16(a) and lo = bf16(a - hi), a taken as float32."""
    f = np.asarray(a, dtype=np.float32).astype(np.float64)
    hi = bf16_round(f)
    return hi + bf16_round(f - hi)


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even), via float32.

    float64 -> float32 rounds to nearest even first; bfloat16 keeps the top 16
    bits of the float32 pattern, rounding the dropped 16 bits to nearest even."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------ primitives ----

def conv3(x, W, b):
    """3x3x3 cross-correlation with zero padding; x [ci][Z][Y][X] -> [co][Z][Y][X]."""
    ci, Z, Y, X = x.shape
    co = W.shape[0]
    xp = np.zeros((ci, Z + 2, Y + 2, X + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((co, Z, Y, X))
    for a in range(3):
        for c in range(3):
            for d in range(3):
                out += np.einsum("oi,izyx->ozyx", W[:, :, a, c, d], xp[:, a:a + Z, c:c + Y, d:d + X])
    return out + b[:, None, None, None]


def conv3_input_grad(g, W):
    """Adjoint of conv3 with respect to its input: g [co][Z][Y][X] -> [ci][Z][Y][X]."""
    co, Z, Y, X = g.shape
    ci = W.shape[1]
    gp = np.zeros((co, Z + 2, Y + 2, X + 2))
    gp[:, 1:-1, 1:-1, 1:-1] = g
    out = np.zeros((ci, Z, Y, X))
    # out[i][p] = sum_o sum_tap W[o][i][tap] g[o][p - tap]
    for a in range(3):
        for c in range(3):
            for d in range(3):
                sh = gp[:, 2 - a:2 - a + Z, 2 - c:2 - c + Y, 2 - d:2 - d + X]
                out += np.einsum("oi,ozyx->izyx", W[:, :, a, c, d], sh)
    return out


def conv3_weight_grad(x, g):
    """dW[o][i][tap] = sum_p g[o][p] x[i][p + tap], db[o] = sum_p g[o][p]."""
    ci, Z, Y, X = x.shape
    xp = np.zeros((ci, Z + 2, Y + 2, X + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    co = g.shape[0]
    dW = np.zeros((co, ci, 3, 3, 3))
    for a in range(3):
        for c in range(3):
            for d in range(3):
                dW[:, :, a, c, d] = np.einsum("ozyx,izyx->oi", g, xp[:, a:a + Z, c:c + Y, d:d + X])
    return dW, g.sum(axis=(1, 2, 3))


def pool2(x):
    C, Z, Y, X = x.shape
    return x.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).mean(axis=(2, 4, 6))


def pool2_grad(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_grad(g):
    C, Z, Y, X = g.shape
    return g.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).sum(axis=(2, 4, 6))


# --------------------------------------------------------------- network ----

def _conv_fwd(x, W, b, bf16):
    if bf16:
        return conv3(bf16_split(x), bf16_round(W), b)
    return conv3(x, W, b)


def forward_one(layers, x, bf16=False):
    """x [cin][Z][Y][X] -> (y [Z][Y][X], cache)."""
    cache = {}

    def block(name, inp, li):
        W, b = layers[li]
        pre = _conv_fwd(inp, W, b, bf16)
        out = np.maximum(pre, 0.0)
        cache[name] = (inp, out, li)
        return out

    e1 = block("L1", x, 0)
    s1 = block("L2", e1, 1)
    e2 = block("L3", pool2(s1), 2)
    s2 = block("L4", e2, 3)
    e3 = block("L5", pool2(s2), 4)
    e3b = block("L6", e3, 5)
    d2 = block("L7", np.concatenate([up2(e3b), s2]), 6)
    d2b = block("L8", d2, 7)
    d1 = block("L9", np.concatenate([up2(d2b), s1]), 8)
    d1b = block("L10", d1, 9)
    W, b = layers[10]
    y = np.einsum("i,izyx->zyx", W[0, :, 0, 0, 0], d1b) + b[0]
    cache["L11"] = d1b
    return y, cache


def backward_one(layers, cache, gy, bf16=False):
    """Gradient of a scalar with dL/dy = gy through one sample: list of (dW, db)."""
    grads = [None] * 11
    W11, _ = layers[10]
    d1b = cache["L11"]
    grads[10] = (np.einsum("zyx,izyx->i", gy, d1b).reshape(1, -1, 1, 1, 1), np.array([gy.sum()]))
    g = W11[0, :, 0, 0, 0][:, None, None, None] * gy[None]

    def back(name, gout):
        inp, out, li = cache[name]
        W, _ = layers[li]
        gpre = gout * (out > 0.0)
        grads[li] = conv3_weight_grad(inp, gpre)
        if bf16:
            return conv3_input_grad(bf16_split(gpre), bf16_round(W))
        return conv3_input_grad(gpre, W)

    w1 = layers[0][0].shape[0]
    w2 = layers[2][0].shape[0]
    w3 = layers[4][0].shape[0]
    g = back("L10", g)
    g = back("L9", g)                 # [w2 + w1]
    g_s1 = g[w2:].copy()
    g = back("L8", up2_grad(g[:w2]))
    g = back("L7", g)                 # [w3 + w2]
    g_s2 = g[w3:].copy()
    g = back("L6", up2_grad(g[:w3]))
    g = back("L5", g)
    g = back("L4", pool2_grad(g) + g_s2)
    g = back("L3", g)
    g = back("L2", pool2_grad(g) + g_s1)
    back("L1", g)
    assert w1 == layers[1][0].shape[0]
    return grads


def forward(params, X, widths=(16, 32, 64), bf16=False):
    """X [B][cin][Z][Y][X] -> Y [B][Z][Y][X]."""
    layers = unpack(params, widths, X.shape[1])
    return np.stack([forward_one(layers, x, bf16)[0] for x in X])


def loss_and_grad(params, X, T, widths=(16, 32, 64), bf16=False):
    """Relative squared-error loss over the batch and its gradient (flat, float64)."""
    layers = unpack(params, widths, X.shape[1])
    B = X.shape[0]
    total = 0.0
    acc = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    for x, t in zip(X, T):
        y, cache = forward_one(layers, x, bf16)
        tt = float(np.sum(t * t))
        total += float(np.sum((y - t) ** 2)) / tt / B
        gy = 2.0 * (y - t) / tt / B
        for i, (dW, db) in enumerate(backward_one(layers, cache, gy, bf16)):
            acc[i][0][...] += dW
            acc[i][1][...] += db
    return total, pack(acc)


def precondition(params, r, sigma_t, sigma_s, n, widths=(16, 32, 64), bf16=False):
    """z = r + s * net(features(r)) for one residual (flat, solver cell order)."""
    F, s = features(r, sigma_t, sigma_s, n)
    if bf16:
        F = F.astype(np.float32).astype(np.float64)
    y = forward(params, F[None], widths, bf16)[0]
    return np.asarray(r, dtype=np.float64) + s * y.ravel()


def restrict(x, n, f):
    """Cell averages of a flat field on an n0 x n1 x n2 grid (x fastest) over f x f x f blocks."""
    X = np.asarray(x, dtype=np.float64).reshape(n[2] // f, f, n[1] // f, f, n[0] // f, f)
    return X.mean(axis=(1, 3, 5)).ravel()


def prolong(y, nc, f):
    """A coarse field (nc0 x nc1 x nc2) extended piecewise constant to the grid refined by f."""
    Y = np.asarray(y, dtype=np.float64).reshape(nc[2], nc[1], nc[0])
    return np.repeat(np.repeat(np.repeat(Y, f, axis=0), f, axis=1), f, axis=2).ravel()


def precondition_coarse(params, r, sigma_t, sigma_s, n, f, widths=(16, 32, 64), bf16=False):
    """The network on the grid coarsened by f: z = r + P(s_c net(features(R r, R sigma_t,
    R sigma_s))), R the cell averages over f^3 blocks, P the piecewise-constant extension."""
    nc = tuple(v // f for v in n)
    rc = restrict(r, n, f)
    F, s = features(rc, restrict(sigma_t, n, f), restrict(sigma_s, n, f), nc)
    if bf16:
        F = F.astype(np.float32).astype(np.float64)
    y = forward(params, F[None], widths, bf16)[0]
    return np.asarray(r, dtype=np.float64) + prolong(s * y.ravel(), nc, f)


def target(r, e):
    """Training target (e - r) / rms(r) for a pair (r, e), flat."""
    s = float(np.sqrt(np.mean(np.asarray(r) ** 2)))
    s = s if s > 0.0 else 1.0
    return (np.asarray(e, dtype=np.float64) - np.asarray(r, dtype=np.float64)) / s


def features(r, sigma_t, sigma_s, n):
    """Input channels of the preconditioner for a residual r on an n0 x n1 x n2 grid:
    r / rms(r), log sigma_t, sigma_s / sigma_t (returned [3][n2][n1][n0]) and rms(r)."""
    shp = (n[2], n[1], n[0])
    s = float(np.sqrt(np.mean(np.asarray(r) ** 2)))
    s = s if s > 0.0 else 1.0
    st = np.asarray(sigma_t, dtype=np.float64)
    return np.stack([np.asarray(r).reshape(shp) / s, np.log(st).reshape(shp),
                     (np.asarray(sigma_s) / st).reshape(shp)]), s


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) in float64; returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
