"""Train the learned right preconditioner on the seeded random media of the
heterogeneous many-scattering recipe (base sigma_t ~ U[5, 50] plus 8 Gaussian
blobs, albedo 0.99, one face source), then compare, on held-out media, plain FP64
GMRES with the FP64-refined solve whose inner flexible GMRES runs on the FP32
operator with the network as right preconditioner.

    python -m paper_1610_00835_amd.train_precond --n 64 --media 24 --steps 1500 --fft \
        --inner-tol 1e-3 --out paper_1610_00835_amd/weights/precond_c5_64_fft.npz
    python -m paper_1610_00835_amd.train_precond --n 128 --coarsen 4 --media 80 --restart 2 \
        --max-pairs 26 --pair-prec fp32 --pair-cheb-n 4 --pair-tol 1e-6 --steps 4000 --batch 8 \
        --cheb-n 6 --inner-cheb-n 4 --inner-near16 --inner-tol 1e-2 --test 1 \
        --out paper_1610_00835_amd/weights/precond_c5_32c.npz

With --coarsen f the network lives on the grid coarsened by f: it is trained on the cell
averages of the pairs over f^3 blocks and the solver applies it to the cell averages of
its vectors, extending the correction piecewise constant (the same coarse grid serves
finer plans: a 32^3 network trained from 64^3 solves acts on 128^3 with f = 4).

Training pairs come from the method's own solves (learn.collect_pairs).  The output
file holds the FP32 parameters, the widths, the grid, the media seeds, the loss
history and the held-out comparison.
"""
import argparse
import json
import os
import time

import numpy as np

from . import ertvie, inputs, learn


def log(*a):
    print(*a, flush=True)


def plan_for(case, args, prec="fp64"):
    return ertvie.plan_from_case(case, method="fmm", prec=prec, leaf=args.leaf, cheb_n=args.cheb_n,
                                 inner_cheb_n=args.inner_cheb_n, inner_near16=args.inner_near16)


def compare(net, case, args):
    """Plain FP64 GMRES vs the FP64-refined solve with FP32 inner GMRES on the lower-order
    operator, with and without the network as right preconditioner (with --fft, all inner
    solves use the FFT-based preconditioner and the network acts on its output)."""
    import torch
    fd = torch.as_tensor(np.ascontiguousarray(case["f"])).cuda()
    out = {}
    pre = dict(tol=1e-8, max_iter=args.max_iter, mixed=True, inner_tol=args.inner_tol, allow_noconv=True,
               precond_fft=args.fft)
    with plan_for(case, args) as plan:
        t0 = time.perf_counter()
        plan.fmm_info("fp64")
        plan.fmm_info("fp32")
        out["plan_s"] = time.perf_counter() - t0
        U0 = torch.empty_like(fd)
        plan.solve(fd, U0, tol=1e-8, max_iter=args.max_iter, allow_noconv=True)   # warm (graphs, tuning)
        plain = plan.solve(fd, U0, tol=1e-8, max_iter=args.max_iter, allow_noconv=True)
        U1 = torch.empty_like(fd)
        plan.solve(fd, U1, precond=net, precond_steps=args.precond_steps, **pre)
        learned = plan.solve(fd, U1, precond=net, precond_steps=args.precond_steps, **pre)
        U2 = torch.empty_like(fd)
        mixed = plan.solve(fd, U2, **pre)
        torch.cuda.synchronize()
        d = float(torch.linalg.norm(U1 - U0) / torch.linalg.norm(U0))
    out.update(plain=plain, learned=learned, mixed_plain=mixed, rel_diff_solutions=d,
               speedup=plain["t_solve"] / learned["t_solve"] if learned["converged"] else None)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--media", type=int, default=24, help="training media (seeds 1000, 1001, ...)")
    ap.add_argument("--test", type=int, default=2, help="held-out media (seeds 0, 1, ...)")
    ap.add_argument("--restart", type=int, default=4, help="GMRES cycle length of the pair-generating solves")
    ap.add_argument("--max-pairs", type=int, default=80)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--leaf", type=int, default=8)
    ap.add_argument("--cheb-n", type=int, default=0)
    ap.add_argument("--inner-cheb-n", type=int, default=4, help="Chebyshev order of the FP32 inner operator")
    ap.add_argument("--precond-steps", type=int, default=10)
    ap.add_argument("--inner-tol", type=float, default=1e-3)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--fft", action="store_true",
                    help="train the network to act on the FFT-based preconditioner's output")
    ap.add_argument("--inner-near16", action="store_true",
                    help="the FP32 inner operator reads the near-field cache rounded to BF16")
    ap.add_argument("--pair-prec", default="fp64", choices=["fp64", "fp32"],
                    help="operator of the pair-generating solves")
    ap.add_argument("--pair-cheb-n", type=int, default=0, help="its Chebyshev order (default --cheb-n)")
    ap.add_argument("--pair-tol", type=float, default=1e-9, help="its GMRES tolerance")
    ap.add_argument("--coarsen", type=int, default=1,
                    help="the network's grid is the training grid coarsened by this factor")
    ap.add_argument("--test-n", type=int, default=0, help="grid of the held-out comparison (default --n)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    ertvie.load()
    n = (args.n,) * 3
    f = args.coarsen
    nnet = tuple(v // f for v in n)
    widths = (16, 32, 64)
    pairs = learn.PairSet()
    t0 = time.perf_counter()
    for s in range(1000, 1000 + args.media):
        case = inputs.make_case("c5", n=n, seed=s)
        pplan = ertvie.plan_from_case(case, method="fmm", prec=args.pair_prec, leaf=args.leaf,
                                      cheb_n=args.pair_cheb_n or args.cheb_n, inner_near16=args.inner_near16)
        with pplan as plan:
            R, E, info = learn.collect_pairs(plan, case["f"], restart=args.restart, tol=args.pair_tol,
                                             max_pairs=args.max_pairs, max_iter=args.max_iter, fft=args.fft)
            if f > 1:
                R, E, stc, ssc = learn.restrict_pairs(plan, R, E, case["sigma_t"], case["sigma_s"], f)
            else:
                stc, ssc = case["sigma_t"], case["sigma_s"]
        pairs.add(R, E, stc, ssc)
        log("medium %d: %d iterations, %d pairs, %.1f s" % (s, info["iters"], R.shape[0], time.perf_counter() - t0))
        torch.cuda.empty_cache()
    pairs.finalize()
    t_pairs = time.perf_counter() - t0
    npairs = len(pairs)
    log("pairs: %d in %.1f s" % (npairs, t_pairs))
    net = ertvie.Net(nnet, batch_max=args.batch, widths=widths)
    net.set_params(learn.init_params(widths, args.seed))
    t0 = time.perf_counter()
    losses = learn.train(net, pairs, steps=args.steps, batch=args.batch, lr=args.lr, seed=args.seed + 1,
                         log_every=max(1, args.steps // 10), log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log("training: %d steps in %.1f s" % (args.steps, t_train))
    del pairs
    torch.cuda.empty_cache()
    results = []
    nt = (args.test_n,) * 3 if args.test_n else n
    for s in range(args.test):
        r = compare(net, inputs.make_case("c5", n=nt, seed=s), args)
        log("held-out medium %d: %s" % (s, json.dumps(r)))
        results.append(r)
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        meta = {"n": nnet, "train_n": n, "coarsen": f, "widths": widths, "pair_prec": args.pair_prec,
                "pair_cheb_n": args.pair_cheb_n or args.cheb_n, "pair_tol": args.pair_tol,
                "train_media": list(range(1000, 1000 + args.media)), "pairs": npairs,
                "restart": args.restart, "steps": args.steps, "batch": args.batch, "lr": args.lr,
                "pairs_s": t_pairs, "train_s": t_train, "losses": losses, "held_out": results,
                "precond_steps": args.precond_steps, "inner_tol": args.inner_tol, "fft": args.fft}
        np.savez(args.out, params=net.get_params(), meta=json.dumps(meta))
        log("wrote", args.out)
    net.close()


if __name__ == "__main__":
    main()
