"""Benchmark: FMM matvec throughput of the isotropic-ERT volume-integral operator
on one MI355X, plus time-to-solution, roofline fraction and the CPU oracle baseline.

One step = one application of (I - K) u = u - A (sigma_s u) through the whole FMM
(gather, near field, P2M, M2M, M2L, L2L, L2P, assembly) on the 3D unit cube
32^3 workload (sigma_t = 5, sigma_s = 4, leaf 4^3 cells, n = 6 Chebyshev nodes per
axis), inputs resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--prec fp32|fp64|bf16x3]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "bf16_mfma": 2.5e15, "hbm": 8.0e12}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def m2l_flops_per_apply(tree_counts, K):
    """Algorithmic M2L work: 2 K^2 multiply-adds per (target box, source box) pair."""
    return 2.0 * K * K * sum(tree_counts)


def interaction_pairs(nb, D):
    """Far-field (M2L) pair count per level for a full 2^L tree over nb^D leaves."""
    L = int(np.ceil(np.log2(nb)))
    out = []
    for l in range(2, L + 1):
        n = int(np.ceil(nb / 2 ** (L - l)))
        idx = np.arange(n)
        cnt = 0
        # per axis: targets t, sources s with |t//2 - s//2| <= 1 and |t - s| > 1 in some axis
        near1 = np.abs(idx[:, None] - idx[None, :]) <= 1
        par1 = np.abs(idx[:, None] // 2 - idx[None, :] // 2) <= 1
        pa = par1.sum()
        nr = (near1 & par1).sum()
        cnt = pa ** D - nr ** D
        out.append(int(cnt))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the work would shard by right-hand sides or Morton leaf ranges; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1610_00835_amd import ertvie, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    case = inputs.make_case("c2", seed=0)
    N = int(np.prod(case["n"]))
    f = torch.from_numpy(case["f"]).to(dev)
    y = torch.empty_like(f)

    stream = torch.cuda.current_stream()
    t_plan0 = time.perf_counter()
    plan = ertvie.plan_from_case(case, method="fmm", prec=args.prec, stream=stream)
    plan.apply(f, y, op=ertvie.OP_A)          # builds the FMM operators on first use
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t_plan0
    log("plan + first apply: %.3f s" % t_plan)

    for _ in range(args.warmup):
        plan.apply(f, y, op=ertvie.OP_A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(f, y, op=ertvie.OP_A)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    value = N / (ms * 1e-3) / 1e6
    log("FMM apply (%s): %.4f ms/step, %.1f Mpts/s" % (args.prec, ms, value))

    # per-stage device time (events on the plan's stream), separate pass
    plan.profile(True)
    for _ in range(args.steps):
        plan.apply(f, y, op=ertvie.OP_A)
    prof = plan.profile(False)
    stage_ms = {k: v[0] / args.steps for k, v in prof.items() if v[1]}
    launches = {k: v[1] / args.steps for k, v in prof.items() if v[1]}
    log("per-apply stage ms:", json.dumps({k: round(v, 5) for k, v in stage_ms.items()}))

    info = plan.fmm_info()
    log("fmm:", json.dumps(info))
    # algorithmic work of the box-offset GEMMs: 2 R^2 per far pair (R = stored translation rank, or the
    # padded node count when uncompressed); 2 per near point pair
    L = info["levels"]
    m2l_flops = sum(2.0 * (info["rank"][l] or info["nodes_padded"]) ** 2 * info["far_pairs"][l]
                    for l in range(2, L + 1))
    near_flops = 2.0 * info["near_pairs"]
    peak = {"fp32": PEAK["fp32_mfma"], "fp64": PEAK["fp64_mfma"], "bf16x3": PEAK["bf16_mfma"]}[args.prec]
    # the dominant kernel of the apply
    cand = {"m2l": (m2l_flops, stage_ms.get("m2l", 0.0), launches.get("m2l", 1)),
            "near": (near_flops, stage_ms.get("near", 0.0), launches.get("near", 1))}
    dom = max(cand, key=lambda k: cand[k][1])
    flops, tms, nl = cand[dom]
    dpeak = peak if dom == "m2l" else {"fp64": PEAK["fp64_mfma"]}.get(args.prec, PEAK["fp32_mfma"])
    achieved = (flops / nl) / (tms / nl * 1e-3) if tms > 0 else 0.0
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved / 1e12, "peak": dpeak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / dpeak, "traffic": None,
                "flops_per_launch": flops / nl, "launch_ms": tms / nl, "launches_per_apply": nl,
                "m2l_tflops": (m2l_flops / (stage_ms["m2l"] * 1e-3) / 1e12) if stage_ms.get("m2l") else None,
                "near_tflops": (near_flops / (stage_ms["near"] * 1e-3) / 1e12) if stage_ms.get("near") else None}

    # accuracy of this apply against the oracle on sampled rows
    extra = {"plan_s": t_plan, "stage_ms": stage_ms}
    from oracle import oracle as O
    P = O.Problem(3, case["n"], case["h"], 0, case["sigma_t"], case["sigma_s"])
    rows = np.random.default_rng(0).choice(N, size=256, replace=False)
    yo = P.apply_rows(case["f"], rows, op=2)
    yg = y.cpu().numpy()
    extra["rel_l2_vs_oracle_rows"] = float(np.linalg.norm(yg[rows] - yo) / np.linalg.norm(yo))

    if not args.no_solve:
        # time to 1e-8: plain FP64 GMRES on the FP64 FMM operator vs FP32-inner refinement
        U = torch.empty_like(f)
        with ertvie.plan_from_case(case, method="fmm", prec="fp64", stream=stream) as p64:
            p64.apply(f, y, op=ertvie.OP_A)
            torch.cuda.synchronize()
            t = time.perf_counter()
            i64 = p64.solve(f, U, tol=1e-8)
            t_fp64 = time.perf_counter() - t
            U64 = U.cpu().numpy()
            plan_f = p64
            p64.apply(f, y, op=ertvie.OP_A, prec="fp32")
            torch.cuda.synchronize()
            t = time.perf_counter()
            imx = plan_f.solve(f, U, tol=1e-8, mixed=True, inner_tol=1e-4)
            t_mixed = time.perf_counter() - t
            Umx = U.cpu().numpy()
        extra["solve"] = {"tol": 1e-8, "fp64_gmres_s": t_fp64, "fp64_iters": i64["iters"],
                          "mixed_s": t_mixed, "mixed_inner_iters": imx["iters"], "mixed_refinements": imx["restarts"],
                          "mixed_rel_resid_true": imx["rel_resid_true"],
                          "mixed_vs_fp64_rel_l2": float(np.linalg.norm(Umx - U64) / np.linalg.norm(U64))}
        log("solve:", json.dumps(extra["solve"]))

    cpu = None
    if not args.no_cpu_baseline:
        cores = len(os.sched_getaffinity(0))
        reps = 2
        t = time.perf_counter()
        for _ in range(reps):
            P.apply(case["f"], op=2, nthreads=cores)
        dt = (time.perf_counter() - t) / reps
        cpu = {"value": N / dt / 1e6, "unit": "Mpts/s", "cores": cores, "kind": "oracle",
               "sample": "%d full dense FP64 applies of (I - K) on the 32^3 workload, %.2f s each" % (reps, dt)}
        log("cpu oracle:", json.dumps(cpu))

    out = {"metric": "FMM matvec Mpts/s", "value": value, "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3+f32"}[args.prec],
           "data": "synthetic",
           "config": {"workload": "3D unit cube 32^3 (N=32768), homogeneous sigma_t=5 sigma_s=4, "
                                  "4 seeded Gaussian sources; FMM leaf 8^3 cells, n=8, compressed translations",
                      "op": "u - K(sigma_s u)", "prec": args.prec, "nrhs": 1},
           "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
