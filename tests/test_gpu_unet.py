"""GPU parity of the learned preconditioner's kernels against the U-Net reference
(oracle/unet.py, float64 with the same BF16 operand rounding), its training step,
and what it gains inside the solver.

Bars: the GPU rounds the same operands (BF16 weights, activations split into two BF16
parts) and accumulates in FP32 where the reference accumulates in float64, so results
differ by accumulation order (~1e-6 relative per sum) plus rare rounding flips of an
operand part whose FP32 value sits next to a rounding boundary (a 2^-16 relative change
of one term, which the split keeps from compounding).  Network output and loss:
rel L2 <= 1e-4; parameter gradients per layer: rel L2 <= 1e-3."""
import numpy as np
import pytest

from oracle import unet as U
from paper_1610_00835_amd import inputs
from tests.gpu_util import log, rel_l2

pytestmark = pytest.mark.gpu

WIDTHS = (16, 32, 64)


@pytest.fixture(scope="module")
def ev():
    from paper_1610_00835_amd import ertvie
    ertvie.load()
    return ertvie


def _rand(n, B, seed):
    rng = np.random.default_rng(seed)
    N = int(np.prod(n))
    r = rng.standard_normal((B, N))
    e = rng.standard_normal((B, N)) * 3.0
    st = rng.uniform(1.0, 50.0, (B, N))
    ss = st * rng.uniform(0.5, 0.99, (B, N))
    return r, e, st, ss


def _params(seed, widths=WIDTHS):
    from paper_1610_00835_amd import learn
    p = learn.init_params(widths, seed)
    rng = np.random.default_rng(seed + 1)
    layers = U.unpack(p.astype(np.float64), widths)
    for W, b in layers:
        b[...] = rng.uniform(-0.05, 0.05, b.shape)
    return U.pack(layers).astype(np.float32)


def _oracle_inputs(r, st, ss, n):
    X, S = [], []
    for b in range(r.shape[0]):
        F, s = U.features(r[b], st[b], ss[b], n)
        X.append(F.astype(np.float32).astype(np.float64))
        S.append(s)
    return np.stack(X), np.array(S)


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,B", [((8, 8, 8), 2), ((16, 8, 12), 1), ((32, 32, 32), 1)])
def test_forward_matches_reference(ev, n, B):
    import torch
    r, e, st, ss = _rand(n, B, 1)
    p = _params(3)
    with ev.Net(n, batch_max=B) as net:
        net.set_params(p)
        z = torch.empty((B, int(np.prod(n))), dtype=torch.float64, device="cuda")
        net.forward(_dev(r), _dev(st), _dev(ss), z)
        zg = _host(z)
        z2 = torch.empty_like(z)
        net.forward(_dev(r), _dev(st), _dev(ss), z2)
        assert np.array_equal(zg, _host(z2))            # deterministic
        if B > 1:                                       # batch = columns one by one
            z1 = torch.empty((1, z.shape[1]), dtype=torch.float64, device="cuda")
            net.forward(_dev(r[1:2]), _dev(st[1:2]), _dev(ss[1:2]), z1)
            assert np.array_equal(_host(z1)[0], zg[1])
    X, S = _oracle_inputs(r, st, ss, n)
    Y = U.forward(p.astype(np.float64), X, WIDTHS, bf16=True)
    ref = Y.reshape(B, -1) * S[:, None]
    # z = r + s y: compare the network part
    err = rel_l2(zg - r, ref)
    log("unet forward", n, B, "rel L2 vs reference", err)
    assert err <= 1e-4
    z0 = U.precondition(p.astype(np.float64), r[0], st[0], ss[0], n, WIDTHS, bf16=True)
    assert rel_l2(zg[0], z0) <= 1e-4


@pytest.mark.parametrize("n,f", [((16, 16, 16), 2), ((32, 32, 16), 4), ((8, 8, 8), 1)])
def test_coarse_grid_preconditioner_matches_reference(ev, n, f):
    """The network on the plan's grid coarsened by f (cell averages in, piecewise-constant
    correction out) against oracle/unet.py's composition; the restriction alone against the
    oracle's cell averages (FP64, bar 1e-14)."""
    import torch
    N = int(np.prod(n))
    nc = tuple(v // f for v in n)
    r, _, st, ss = _rand(n, 1, 11)
    p = _params(13)
    case = {"dim": 3, "n": n, "h": 1.0 / max(n), "kernel": 1, "sigma_t": st[0], "sigma_s": ss[0]}
    with ev.plan_from_case(case, method="direct", prec="fp64") as plan, ev.Net(nc, batch_max=1) as net:
        net.set_params(p)
        z = torch.empty(N, dtype=torch.float64, device="cuda")
        plan.net_apply(net, _dev(r[0]), z)
        zg = _host(z)
        yc = torch.empty(N // f ** 3, dtype=torch.float64, device="cuda")
        plan.restrict(_dev(r[0]), yc, f)
        rc = _host(yc)
    ref = U.precondition_coarse(p.astype(np.float64), r[0], st[0], ss[0], n, f, WIDTHS, bf16=True)
    err = rel_l2(zg - r[0], ref - r[0])
    log("coarse-grid preconditioner", n, "f", f, "rel L2 of the correction vs reference", err)
    assert rel_l2(rc, U.restrict(r[0], n, f)) <= 1e-14
    assert err <= 1e-4


@pytest.mark.parametrize("n,B", [((8, 8, 8), 2), ((16, 16, 16), 2), ((32, 16, 16), 1)])
def test_gradient_matches_reference(ev, n, B):
    """The weight gradients sum over voxels in slabs of 1024 per batch column: 8^3 is one
    slab per column, 16^3 four and 32 x 16 x 16 eight on the finest level, so the
    in-column slab offsets are exercised on the larger grids."""
    r, e, st, ss = _rand(n, B, 4)
    p = _params(5)
    with ev.Net(n, batch_max=B) as net:
        net.set_params(p)
        loss, g = net.grad(_dev(r), _dev(e), _dev(st), _dev(ss))
    X, S = _oracle_inputs(r, st, ss, n)
    T = np.stack([U.target(r[b], e[b]).astype(np.float32).astype(np.float64).reshape(n[2], n[1], n[0])
                  for b in range(B)])
    Lr, gr = U.loss_and_grad(p.astype(np.float64), X, T, WIDTHS, bf16=True)
    log("unet loss gpu", loss, "reference", Lr)
    assert abs(loss - Lr) <= 1e-4 * abs(Lr)
    o = 0
    for li, (co, ci, k) in enumerate(U.layer_shapes(WIDTHS)):
        nw = co * ci * k ** 3
        for name, a, b in (("W", o, o + nw), ("b", o + nw, o + nw + co)):
            e_ = rel_l2(g[a:b].astype(np.float64), gr[a:b])
            log("  layer", li + 1, name, "rel L2", e_)
            assert e_ <= 1e-3, (li + 1, name, e_)
        o += nw + co
    assert o == g.size


def test_adam_step_matches_reference(ev):
    n, B = (8, 8, 8), 2
    r, e, st, ss = _rand(n, B, 6)
    p = _params(7)
    with ev.Net(n, batch_max=B) as net:
        net.set_params(p)
        _, g = net.grad(_dev(r), _dev(e), _dev(st), _dev(ss))
        net.train_step(_dev(r), _dev(e), _dev(st), _dev(ss), lr=2e-3)
        q = net.get_params()
    ref, _, _ = U.adam_step(p.astype(np.float64), g.astype(np.float64), np.zeros(p.size), np.zeros(p.size), 1,
                            lr=2e-3)
    assert np.max(np.abs(q - ref)) <= 1e-6


def test_training_reduces_loss(ev):
    from paper_1610_00835_amd import learn
    n, B = (8, 8, 8), 4
    r, e, st, ss = _rand(n, B, 8)
    e = r * 3.0 + 0.5 * np.roll(r, 1, axis=1)      # a learnable map
    with ev.Net(n, batch_max=B) as net:
        net.set_params(learn.init_params(WIDTHS, 9))
        args = (_dev(r), _dev(e), _dev(st), _dev(ss))
        L0 = net.train_step(*args, lr=1e-3)
        for _ in range(60):
            L = net.train_step(*args, lr=1e-3)
    log("training loss", L0, "->", L)
    assert L < 0.5 * L0


def _c5_case(n, seed):
    return inputs.make_case("c5", n=n, seed=seed)


def test_learned_preconditioner_gain_and_judge(ev):
    """16^3 media from the 128^3 recipe (base sigma_t in [5, 50] plus blobs, albedo 0.99).
    Train on the pairs of plain solves of 6 media.  On the residuals of a held-out
    medium's solve, one application of the trained preconditioner leaves a smaller
    residual ||r - (I - K) M(r)|| than the method without the network (M = identity,
    z = r); the preconditioned solve reaches the plain solve's solution at a 1e-8 true
    residual.  A network whose output is not finite has every preconditioned step
    rejected by the residual check, and the plain fallback still converges."""
    import torch
    from paper_1610_00835_amd import learn
    n = (16, 16, 16)
    pairs = learn.PairSet()
    for s in range(1000, 1006):
        case = _c5_case(n, s)
        with ev.plan_from_case(case, method="direct", prec="fp64") as plan:
            R, E, info = learn.collect_pairs(plan, case["f"], restart=3, tol=1e-10, max_pairs=60)
        log("medium", s, "plain solve", info["iters"], "iters,", R.shape[0], "pairs")
        pairs.add(R, E, case["sigma_t"], case["sigma_s"])
    pairs.finalize()
    with ev.Net(n, batch_max=4) as net:
        net.set_params(learn.init_params(WIDTHS, 0))
        losses = learn.train(net, pairs, steps=400, batch=4, lr=2e-3, seed=1, log_every=100, log=log)
        case = _c5_case(n, 0)
        fd = _dev(case["f"])
        st = _dev(case["sigma_t"][None])
        ss = _dev(case["sigma_s"][None])
        with ev.plan_from_case(case, method="direct", prec="fp64") as plan:
            R, E, _ = learn.collect_pairs(plan, case["f"], restart=3, tol=1e-10, max_pairs=60)
            gain = []
            for k in range(R.shape[0]):
                r = R[k:k + 1].contiguous()
                z = torch.empty_like(r)
                net.forward(r, st, ss, z)
                az = torch.empty_like(r)
                plan.apply(z, az, op=ev.OP_A)
                ar = torch.empty_like(r)
                plan.apply(r, ar, op=ev.OP_A)
                torch.cuda.synchronize()
                gain.append((float(torch.linalg.norm(r - az) / torch.linalg.norm(r)),
                             float(torch.linalg.norm(r - ar) / torch.linalg.norm(r))))
            U0 = torch.empty_like(fd)
            plain = plan.solve(fd, U0, tol=1e-8, max_iter=2000)
            U1 = torch.empty_like(fd)
            pre = plan.solve(fd, U1, tol=1e-8, max_iter=2000, precond=net, precond_steps=10)
            d = rel_l2(_host(U1), _host(U0))
        g = np.array(gain)
        log("one application, residual left: network", g[:, 0].mean(), "identity", g[:, 1].mean())
        log("plain", plain)
        log("learned", pre, "difference of solutions", d)
        assert losses[-1][1] < losses[0][1]
        assert g[:, 0].mean() < 0.8 * g[:, 1].mean()
        assert plain["converged"] == 1 and pre["converged"] == 1 and pre["rel_resid_true"] <= 1e-8
        assert d <= 1e-6
        p = net.get_params()
        p[-1] = np.nan
        net.set_params(p)
        with ev.plan_from_case(case, method="direct", prec="fp64") as plan:
            U2 = torch.empty_like(fd)
            bad = plan.solve(fd, U2, tol=1e-8, max_iter=2000, precond=net, precond_steps=10)
            assert np.all(np.isfinite(_host(U2)))
        log("non-finite network", bad)
        assert bad["converged"] == 1 and bad["rejected"] >= 1 and bad["rejected"] == bad["restarts"]


def test_network_after_fft_preconditioner_gain(ev):
    """The network trained on the FFT-based preconditioner's output (the committed
    64^3 weights, trained on media 1000-1023): on the residuals of a held-out medium's
    solve (seed 0), one application of net(M r) leaves a smaller residual
    ||r - (I - K) z|| than M r alone, and is closer to the exact correction."""
    import os
    import torch
    from paper_1610_00835_amd import learn
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1610_00835_amd",
                        "weights", "precond_c5_64_fft.npz")
    w = np.load(path)
    n = (64, 64, 64)
    case = _c5_case(n, 0)
    st = _dev(case["sigma_t"][None])
    ss = _dev(case["sigma_s"][None])
    with ev.plan_from_case(case, method="fmm", prec="fp64") as plan, ev.Net(n, batch_max=1) as net:
        net.set_params(w["params"])
        R, E, _ = learn.collect_pairs(plan, case["f"], restart=4, tol=1e-9, max_pairs=40)
        res = []
        for k in range(R.shape[0]):
            r = R[k:k + 1].contiguous()
            q = torch.empty_like(r)
            plan.fft_precond(r, q)
            z = torch.empty_like(r)
            net.forward(q, st, ss, z)
            aq = torch.empty_like(r)
            plan.apply(q, aq, op=ev.OP_A)
            az = torch.empty_like(r)
            plan.apply(z, az, op=ev.OP_A)
            torch.cuda.synchronize()
            nr = float(torch.linalg.norm(r))
            e = E[k:k + 1]
            res.append((float(torch.linalg.norm(r - aq)) / nr, float(torch.linalg.norm(r - az)) / nr,
                        float(torch.linalg.norm(e - q) / torch.linalg.norm(e)),
                        float(torch.linalg.norm(e - z) / torch.linalg.norm(e))))
    g = np.array(res)
    log("residual left: FFT-based %.3f, network after it %.3f; error left: %.3f vs %.3f" % tuple(g.mean(0)))
    assert g[:, 1].mean() < 0.8 * g[:, 0].mean()
    assert g[:, 3].mean() < g[:, 2].mean()


def test_coarse_network_fewer_iterations(ev):
    """The committed coarse-grid network (32^3, trained on the 1927 cell-averaged pairs of
    64^3 solves of media 1000-1119) on a held-out 64^3 medium (seed 0) of the many-scattering
    recipe: the FP64-refined solve with FP32 inner flexible GMRES on the order-4 operator
    takes fewer inner iterations with the network (applied to the cell averages over 2^3
    blocks) than the same solve without it, and reaches the plain FP64 GMRES solution at a
    1e-8 true residual.  Wall time is logged, not asserted: each network application
    (about 0.5 ms of small convolution launches on the 32^3 grid) costs about what the
    saved iterations save at this size (measured 0.074 s against 0.073 s)."""
    import json
    import os
    import torch
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1610_00835_amd",
                        "weights", "precond_c5_32c.npz")
    w = np.load(path)
    meta = json.loads(str(w["meta"]))
    case = _c5_case((64, 64, 64), 0)
    fd = _dev(case["f"])
    with ev.plan_from_case(case, method="fmm", prec="fp64", inner_cheb_n=4, inner_near16=True) as plan, \
            ev.Net(tuple(meta["n"]), batch_max=1) as net:
        net.set_params(w["params"])
        U0 = torch.empty_like(fd)
        plain = plan.solve(fd, U0, tol=1e-8)
        kw = dict(tol=1e-8, mixed=True, inner_tol=float(meta["inner_tol"]))
        U1 = torch.empty_like(fd)
        runs = {}
        for name, extra in (("mixed", {}), ("learned", dict(precond=net, precond_steps=int(meta["precond_steps"])))):
            plan.solve(fd, U1, **kw, **extra)                     # graphs and tuning
            best = None
            for _ in range(3):
                r = plan.solve(fd, U1, **kw, **extra)
                best = r if best is None or r["t_solve"] < best["t_solve"] else best
            runs[name] = best
            runs[name]["vs_plain"] = rel_l2(_host(U1), _host(U0))
    log("held-out 64^3 medium: plain", plain, "\nmixed", runs["mixed"], "\nmixed + coarse network", runs["learned"])
    m, l = runs["mixed"], runs["learned"]
    assert plain["converged"] == 1 and m["converged"] == 1 and l["converged"] == 1
    assert l["rel_resid_true"] <= 1e-8 and l["vs_plain"] <= 1e-6
    assert l["iters"] < m["iters"]
