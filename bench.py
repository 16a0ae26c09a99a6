"""Benchmark: FMM matvec throughput of the isotropic-ERT volume-integral operator and time to
a 1e-8 solve on one MI355X, with the dominant kernel's roofline fraction and the CPU oracle.

Headline workload: the many-scattering medium at 128^3 (N = 2,097,152; base sigma_t ~ U[5,50]
plus 8 seeded blobs, sigma_s = 0.99 sigma_t, one face source; ray-quadrature kernel).  One
step = one application of (I - K) u = u - A (sigma_s u) through the whole FMM in FP64 (gather,
near field over the cached kernel blocks, P2M, M2M, M2L over the cached per-pair translations,
L2L, L2P, assembly with the FP64 self term), inputs resident in HBM, replayed from a captured
graph.  Beside it: time to a 1e-8 true residual for plain FP64 GMRES, the mixed-precision
refinement, and both with the learned and the FFT-based right preconditioners.  Other
workloads (32^3 homogeneous, 64^3 blob medium, 64 right-hand sides) go to "extra".
Prints one JSON line on stdout (progress on stderr).

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-solve]
                  [--headline-only] [--form F]
"""
import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FLOPS = {"fp32": 157.3e12, "fp64": 78.6e12, "bf16x3": 2.5e15 / 3.0}   # bf16x3: three bf16 MFMA products
HBM = 8.0e12
SZ = {"fp32": 4, "fp64": 8, "bf16x3": 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_applies(torch, plan, x, y, op, steps, warmup, **kw):
    """Wall time per apply (ms) of `steps` applies after `warmup` untimed ones, bracketed by
    device synchronisations."""
    for _ in range(warmup):
        plan.apply(x, y, op=op, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply(x, y, op=op, **kw)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def stage_profile(plan, x, y, op, steps):
    plan.profile(True)
    for _ in range(steps):
        plan.apply(x, y, op=op)
    prof = plan.profile(False)
    ms = {k: v[0] / steps for k, v in prof.items() if v[1]}
    n = {k: v[1] / steps for k, v in prof.items() if v[1]}
    return ms, n


# Singular-value cutoff of the compressed translations on the 32^3 workload (one far-field
# level): rank 160 of 512, apply error 1.5e-7 against the oracle.
SVD_TOL = 1e-5

# HBM bytes per launch of the dominant kernel from the FETCH_SIZE / WRITE_SIZE counter runs,
# scaled by the readings of a 256 MiB device copy (profiles/near_m2l_c2_32cubed_fp32_hbm_traffic.md).
# Keyed by (workload, precision, kernel, execution forms "near,far" the autotuner chose); a
# combination without counters, or a kernel changed since they were taken, reports null.
MEASURED_TRAFFIC = {("c2", "fp32", "near+m2l", "1,1"): 39.20e6}


def roofline_of(info, stage_ms, launches, prec, dim=3, workload=None, forms=None):
    """Roofline of the dominant box-offset product (M2L or near field) from its algorithmic work:
    M2L: 2 R^2 flops per far pair, bytes = translation matrices (one per box offset) + multipoles in
    + locals out; near: 2 flops per point pair, bytes = the 3^d near blocks (or the offset table the
    offset-stationary forms read in a homogeneous medium) + charges in + potentials out."""
    sz = SZ[prec]
    L = info["levels"]
    noff = 7 ** dim - 3 ** dim
    m2l_flops = m2l_bytes = 0.0
    for l in range(2, L + 1):
        R = info["rank"][l] or info["nodes_padded"]
        pairs = info["far_pairs"][l]
        nbox = (info["leaf_boxes"] / 2 ** (dim * (L - l)))
        m2l_flops += 2.0 * R * R * pairs
        m2l_bytes += (min(noff, pairs) * R * R + 2.0 * nbox * R) * sz
    S = info["leaf"] ** dim
    near_flops = 2.0 * info["near_pairs"]
    # the offset-stationary forms of a homogeneous near field read one table over cell
    # offsets instead of the 3^d explicit S x S blocks
    near_ops = info["near_table"] if (info.get("near_table") and info.get("form_near", 0) >= 1) else 3 ** dim * S * S
    near_bytes = (near_ops + 2.0 * info["leaf_boxes"] * S) * (8 if prec == "fp64" else 4)
    cand = {"m2l": (m2l_flops, m2l_bytes, stage_ms.get("m2l", 0.0), launches.get("m2l", 1.0), prec),
            "near": (near_flops, near_bytes, stage_ms.get("near", 0.0), launches.get("near", 1.0),
                     "fp64" if prec == "fp64" else "fp32")}
    if not stage_ms.get("m2l") and m2l_flops > 0 and prec != "bf16x3":
        # one-level tree after tuning: near field and translations share one launch
        cand = {"near+m2l": (near_flops + m2l_flops, near_bytes + m2l_bytes, stage_ms.get("near", 0.0),
                             launches.get("near", 1.0), "fp64" if prec == "fp64" else "fp32")}
    dom = max(cand, key=lambda k: cand[k][2])
    flops, nbytes, tms, nl, kprec = cand[dom]
    ai = flops / nbytes
    ridge = PEAK_FLOPS[kprec] / HBM
    t = tms / nl * 1e-3
    if ai < ridge:
        achieved, peak, unit, bound, per = nbytes / nl / t / 1e9, HBM / 1e9, "GB/s", "hbm", nbytes / nl
    else:
        achieved, peak, unit, bound, per = flops / nl / t / 1e12, PEAK_FLOPS[kprec] / 1e12, "TFLOP/s", "mfma", flops / nl
    return {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": MEASURED_TRAFFIC.get((workload, prec, dom, forms)), "forms": forms, "per_launch": per, "launch_ms": tms / nl, "launches_per_apply": nl,
            "arith_intensity_flop_per_byte": ai, "ridge_flop_per_byte": ridge,
            "kernel_flops_per_launch": flops / nl,
            "m2l_tflops": m2l_flops / (stage_ms["m2l"] * 1e-3) / 1e12 if stage_ms.get("m2l") else None,
            "near_tflops": near_flops / (stage_ms["near"] * 1e-3) / 1e12 if stage_ms.get("near") else None}


# Sec. 5.3, Experiments V and VI: GMRES iterations to 1e-12 without and with the
# FFT-based preconditioner (Table TAB:EXP VI, the paper's MATLAB code on one laptop core).
PAPER_EXP6_ITERS = {10.0: (21, 9), 20.0: (34, 11), 40.0: (78, 13), 80.0: (110, 15)}
# Experiment V: the same setting with the diffusion preconditioner (plain, preconditioned)
PAPER_EXP5_ITERS = {10.0: (21, 36), 20.0: (34, 38), 40.0: (78, 42), 80.0: (110, 52)}


def paper_experiment_vi(torch, ertvie, inputs, stream):
    """The paper's preconditioning experiments (V and VI): 2D unit square, h = 1/512
    (N = 262,144), Chebyshev order 6, absorption 0.2 and scattering 10, 20, 40, 80
    (homogeneous), GMRES to 1e-12, unpreconditioned, with the FFT-based preconditioner and
    with the diffusion preconditioner.  The paper's source exists
    only as a figure; a Gaussian of width 0.1 at the centre stands in for it (far from the
    boundary, the preconditioner's assumption)."""
    n = (512, 512)
    N = 512 * 512
    x = inputs.centres(n, 1.0 / 512)
    f = np.exp(-np.sum((x - 0.5) ** 2, axis=1) / (2 * 0.1 ** 2))
    fd = torch.from_numpy(f).cuda()
    out = {"workload": "2D 512^2, mu_a = 0.2, homogeneous, Gaussian source (width 0.1), tol 1e-12, FMM n = 6, FP64",
           "paper_iters_plain_fft": {str(k): v for k, v in PAPER_EXP6_ITERS.items()},
           "paper_iters_plain_diffusion": {str(k): v for k, v in PAPER_EXP5_ITERS.items()}, "runs": {}}
    keys = ("iters", "matvecs", "t_solve", "rel_resid_true")
    for mus in sorted(PAPER_EXP6_ITERS):
        case = {"dim": 2, "n": n, "h": 1.0 / 512, "kernel": ertvie.K_HOMOGENEOUS,
                "sigma_t": np.full(N, mus + 0.2), "sigma_s": np.full(N, mus)}
        with ertvie.plan_from_case(case, method="fmm", prec="fp64", stream=stream, cheb_n=6) as plan:
            U = torch.empty_like(fd)
            plan.solve(fd, U, tol=1e-12, max_iter=300)                       # graphs, tuning
            r0 = plan.solve(fd, U, tol=1e-12, max_iter=300)
            U0 = U.clone()
            plan.solve(fd, U, tol=1e-12, max_iter=300, precond_fft=True)
            r1 = plan.solve(fd, U, tol=1e-12, max_iter=300, precond_fft=True)
            d = float(torch.linalg.norm(U - U0) / torch.linalg.norm(U0))
            plan.solve(fd, U, tol=1e-12, max_iter=300, precond_diffusion=True)
            r2 = plan.solve(fd, U, tol=1e-12, max_iter=300, precond_diffusion=True)
            d2 = float(torch.linalg.norm(U - U0) / torch.linalg.norm(U0))
        run = {"plain": {k: r0[k] for k in keys}, "fft": {k: r1[k] for k in keys}, "fft_vs_plain_rel_l2": d,
               "speedup": r0["t_solve"] / r1["t_solve"], "diffusion": {k: r2[k] for k in keys},
               "diffusion_vs_plain_rel_l2": d2, "diffusion_speedup": r0["t_solve"] / r2["t_solve"]}
        for k in ("plain", "fft", "diffusion"):
            run[k]["ms_per_iter"] = 1e3 * run[k]["t_solve"] / max(1, run[k]["matvecs"])
        out["runs"][str(mus)] = run
        log("experiments V/VI mu_s = %g: plain %d iterations (paper %d), FFT-preconditioned %d (paper %d), "
            "diffusion-preconditioned %d (paper %d); %.3f s / %.3f s / %.3f s"
            % (mus, r0["iters"], PAPER_EXP6_ITERS[mus][0], r1["iters"], PAPER_EXP6_ITERS[mus][1], r2["iters"],
               PAPER_EXP5_ITERS[mus][1], r0["t_solve"], r1["t_solve"], r2["t_solve"]))
    return out


def fft_pass_bytes(n, m):
    """Bytes each pass of one FFT-based preconditioner apply reads and writes (3D; FP64
    vectors, complex FP32 work grids, FP32 folded 1/c)."""
    n0, n1, n2 = n
    m0, m1, m2 = m
    H0, H1, H2 = m0 // 2 + 1, m1 // 2 + 1, m2 // 2 + 1
    t1 = n2 * n1 * H0 * 8
    t2 = n2 * m1 * H0 * 8
    N = n0 * n1 * n2
    return {"x_forward": N * 8 + t1, "y_forward": t1 + t2, "z_mid": 2 * t2 + H2 * H1 * H0 * 4,
            "y_inverse": t2 + t1, "x_inverse": t1 + N * 8}


def fft_only(torch, ertvie, inputs, stream, steps=50):
    """The FFT-based preconditioner alone on the many-scattering media at 64^3 and 128^3:
    device time per apply (events) and the bytes its five passes move."""
    out = {}
    for n in (64, 128):
        case = inputs.make_case("c5", n=(n, n, n), seed=0)
        with ertvie.plan_from_case(case, method="fmm", prec="fp64", stream=stream) as plan:
            info = plan.fft_info()
            x = torch.from_numpy(inputs.random_vector(plan.N, 21)).cuda()
            z = torch.empty_like(x)
            ms = timed_fft(torch, plan, x, z, steps)
        pb = fft_pass_bytes((n, n, n), info["m"])
        tot = sum(pb.values())
        out["%d^3" % n] = {"apply_ms": ms, "periods": info["m"], "pass_bytes": pb, "bytes_per_apply": tot,
                           "gb_per_s": tot / (ms * 1e-3) / 1e9}
        log("FFT-based preconditioner %d^3: %.4f ms per apply, %.1f MB moved, %.0f GB/s" %
            (n, ms, tot / 1e6, tot / (ms * 1e-3) / 1e9))
    return out


def paper_experiment_iii(torch, ertvie, inputs, stream, kmax=12, mus_list=(2.0, 5.0, 10.0)):
    """The paper's accuracy experiment (Sec. 5.2, Experiments III/IV): 2D unit square with
    absorption 0.2 and scattering 2, 5, 10 (homogeneous), grids h = 1/(24 (2k - 1)),
    k = 1..kmax, the k = kmax solution as reference, errors on the k = 1 collocation points
    (shared by every grid: the refinement factors are odd), for approaches (M-ii) and (M-iii).
    The paper's sources exist only as figures; a smooth ring (radius 0.25, width 0.05, centred)
    stands in.  FMM of order 8 (the paper used 6) so that the interpolation error stays below
    the discretisation error of the finest grids; GMRES to 1e-12."""
    out = {"workload": "2D, mu_a = 0.2, h = 1/(24(2k-1)), k = 1..%d, ring source, FMM n = 8, FP64, tol 1e-12" % kmax,
           "runs": {}}
    for mus in mus_list:
        for scheme, name in ((1, "M-ii"), (0, "M-iii")):
            sols = {}
            t0 = time.perf_counter()
            for k in range(1, kmax + 1):
                nn = 24 * (2 * k - 1)
                n = (nn, nn)
                N = nn * nn
                h = 1.0 / nn
                x = inputs.centres(n, h)
                rr = np.sqrt(np.sum((x - 0.5) ** 2, axis=1))
                f = torch.from_numpy(np.exp(-(rr - 0.25) ** 2 / (2 * 0.05 ** 2))).cuda()
                case = {"dim": 2, "n": n, "h": h, "kernel": ertvie.K_HOMOGENEOUS,
                        "sigma_t": np.full(N, mus + 0.2), "sigma_s": np.full(N, mus)}
                with ertvie.plan_from_case(case, method="fmm" if nn > 72 else "direct", prec="fp64", stream=stream,
                                           cheb_n=8, scheme=scheme) as plan:
                    U = torch.empty_like(f)
                    info = plan.solve(f, U, tol=1e-12, max_iter=400)
                idx = np.arange(24)
                sel = (idx * (2 * k - 1) + k - 1)
                sols[k] = U.cpu().numpy().reshape(nn, nn)[np.ix_(sel, sel)].reshape(-1)
                if info["converged"] != 1:
                    log("experiment III: %s mu_s %g k %d did not converge" % (name, mus, k))
            ref = sols[kmax]
            errs = [float(np.linalg.norm(sols[k] - ref) / np.linalg.norm(ref)) for k in range(1, kmax)]
            hs = [1.0 / (24 * (2 * k - 1)) for k in range(1, kmax)]
            orders = [float(np.log(errs[i] / errs[i + 1]) / np.log(hs[i] / hs[i + 1])) for i in range(len(errs) - 1)]
            out["runs"]["%s_mu_s_%g" % (name, mus)] = {"h": hs, "rel_l2_err": errs, "observed_order": orders,
                                                       "seconds": time.perf_counter() - t0}
            log("experiment III %s mu_s %g: errors %s" % (name, mus, " ".join("%.2e" % e for e in errs)))
    return out


def homogeneous_64(torch, ertvie, inputs, O, stream):
    """The 32^3 workload's medium on a 64^3 grid (N = 262,144; two far-field levels): FP32
    FMM apply time, the box-offset products' throughput at this size, and the error on
    sampled rows against the oracle."""
    case = inputs.make_case("c2", n=(64, 64, 64), seed=0)
    N = int(np.prod(case["n"]))
    x = torch.from_numpy(inputs.random_vector(N, 13)).cuda()
    y = torch.empty_like(x)
    with ertvie.plan_from_case(case, method="fmm", prec="fp32", stream=stream) as plan:
        plan.apply(x, y, op=ertvie.OP_A)
        plan.apply(x, y, op=ertvie.OP_A)
        ms = timed_applies(torch, plan, x, y, ertvie.OP_A, 20, 3)
        yh = y.cpu().numpy()
        st, ln = stage_profile(plan, x, y, ertvie.OP_A, 10)
        info = plan.fmm_info()
    info["leaf_boxes"] = int(np.prod([-(-n // info["leaf"]) for n in case["n"]]))
    rf = roofline_of(info, st, ln, "fp32")
    P = O.Problem(3, case["n"], case["h"], 0, case["sigma_t"], case["sigma_s"])
    rows = np.random.default_rng(2).choice(N, size=24, replace=False)
    yo = P.apply_rows(inputs.random_vector(N, 13), rows, op=2)
    out = {"workload": "64^3 homogeneous sigma_t = 5, sigma_s = 4, FP32 FMM (leaf 8^3, n = 8, compression 1e-6)",
           "apply_ms": ms, "mpts_per_s": N / (ms * 1e-3) / 1e6, "stage_ms": st, "fmm": info,
           "near_tflops": rf["near_tflops"], "m2l_tflops": rf["m2l_tflops"], "dominant": rf["kernel"],
           "dominant_frac": rf["frac"], "dominant_bound": rf["bound"],
           "rel_l2_vs_oracle_rows": float(np.linalg.norm(yh[rows] - yo) / np.linalg.norm(yo))}
    log("64^3 homogeneous:", json.dumps({k: v for k, v in out.items() if k not in ("fmm",)}))
    return out


def timed_fft(torch, plan, x, z, steps):
    """Mean device time of the FFT-based preconditioner on the plan's stream (events)."""
    for _ in range(3):
        plan.fft_precond(x, z)
    s = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(steps):
        plan.fft_precond(x, z)
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def many_rhs_64(torch, ertvie, inputs, stream):
    """64 face sources on the 64^3 blob medium: the batched apply of all 64 columns (the
    cached-pair products on the matrix cores) and block GMRES to 1e-8, against column-by-
    column GMRES timed on 4 columns."""
    case = inputs.make_case("c4", seed=0, nrhs=64)
    F = torch.from_numpy(np.ascontiguousarray(case["f"].T)).cuda()
    out = {"workload": "64^3 blob medium, 64 face sources, tol 1e-8"}
    with ertvie.plan_from_case(case, method="fmm", prec="fp64", stream=stream, nrhs_max=64, inner_cheb_n=4) as plan:
        plan.fmm_info("fp64")
        plan.fmm_info("fp32")
        X = torch.from_numpy(np.ascontiguousarray(inputs.random_vector(plan.N, 5, nrhs=64).T)).cuda()
        Y = torch.empty_like(X)
        for prec in ("fp64", "fp32"):
            out["apply_64rhs_ms_" + prec] = timed_applies(torch, plan, X, Y, ertvie.OP_A, 3, 2, prec=prec)
        keys = ("iters", "matvecs", "restarts", "t_solve", "rel_resid_true")
        U = torch.empty_like(F)
        plan.solve(F, U, tol=1e-8, block=True)
        r = plan.solve(F, U, tol=1e-8, block=True)
        out["block_fp64"] = {k: r[k] for k in keys}
        r = plan.solve(F, U, tol=1e-8, block=True, mixed=True, inner_tol=1e-2)
        out["block_mixed"] = {k: r[k] for k in keys}
        U4 = torch.empty_like(F[:4])
        r = plan.solve(F[:4].contiguous(), U4, tol=1e-8)
        out["columns_fp64_4_of_64"] = {k: r[k] for k in keys}
        out["columns_fp64_64_extrapolated_s"] = r["t_solve"] * 16
    # the far-field translations as split-BF16x3 against FP32, both at order 8 on 64 columns
    with ertvie.plan_from_case(case, method="fmm", prec="fp32", stream=stream, nrhs_max=64) as plan:
        X = torch.from_numpy(np.ascontiguousarray(inputs.random_vector(plan.N, 5, nrhs=64).T)).cuda()
        Y = torch.empty_like(X)
        res = {}
        for prec in ("fp32", "bf16x3"):
            ms = timed_applies(torch, plan, X, Y, ertvie.OP_A, 3, 2, prec=prec)
            res[prec] = Y.clone()
            plan.apply(X, Y, op=ertvie.OP_A, prec=prec)
            plan.profile(True)
            plan.apply(X, Y, op=ertvie.OP_A, prec=prec)
            st = {k: v[0] for k, v in plan.profile(False).items() if v[1]}
            out["apply_64rhs_order8_" + prec] = {"apply_ms": ms, "m2l_ms": st.get("m2l"), "near_ms": st.get("near")}
        out["bf16x3_vs_fp32_rel_l2"] = float(torch.linalg.norm(res["bf16x3"] - res["fp32"]) /
                                             torch.linalg.norm(res["fp32"]))
    log("64 right-hand sides:", json.dumps(out))
    return out


# network on the 32^3 coarse grid (trained on the cell averages of 64^3 solves' pairs); the
# solver applies it to the cell averages of its vectors over 4^3 blocks at 128^3
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1610_00835_amd", "weights",
                       "precond_c5_32c.npz")
# network trained on the FFT-based preconditioner's output (it acts after that preconditioner)
WEIGHTS_FFT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1610_00835_amd", "weights",
                           "precond_c5_64_fft.npz")




# The headline's kernel caches: FMM of Chebyshev order 6 for the FP64 operator (order 8 would
# need 640 GB for the far field alone), order 4 for the FP32 inner operator of mixed solves,
# whose near field reads the BF16-rounded plane of the shared near-field cache.
C5_N = 128
C5_CHEB, C5_INNER_CHEB = 6, 4
# HBM bytes per launch of the dominant kernel from the FETCH_SIZE / WRITE_SIZE counter runs,
# scaled by the readings of a 256 MiB device copy (profiles/*_hbm_traffic.md).  Keyed by
# (workload, precision, stage of the kernel, execution forms); a combination without counters,
# or a kernel changed since they were taken, reports null.
MEASURED_TRAFFIC = dict(MEASURED_TRAFFIC)
# 128^3 FP64 operator (k_pair_sym over the symmetric caches): far field 66.13 GB per apply in
# 3 launches, near field 53.95 GB in one (profiles/pair_sym_c5_128cubed_hbm_traffic.md)
MEASURED_TRAFFIC[("c5_128", "fp64", "m2l")] = 22.044e9
MEASURED_TRAFFIC[("c5_128", "fp64", "near")] = 53.948e9


def hbm_read_reference(torch, ertvie, dev, stream, gib=16, reps=5):
    """The attainable streaming read rate of this GPU in the access pattern of the cached-pair
    products (ert_vie_read_rate over a zero-filled 16 GiB buffer, one workgroup per piece of a
    stored block's size: 224^2 and 512^2 FP32 values), reported beside the 8 TB/s peak."""
    a = torch.zeros(gib * (1 << 28), dtype=torch.float32, device=dev)
    out = {}
    for name, piece in (("pieces_200704_B", 224 * 224 * 4), ("pieces_1048576_B", 512 * 512 * 4)):
        nbytes, ms = ertvie.read_rate(a, piece, reps, stream)
        out[name] = {"bytes": nbytes, "ms": ms, "gb_per_s": nbytes / (ms * 1e-3) / 1e9}
    del a
    torch.cuda.empty_cache()
    out["gb_per_s"] = max(v["gb_per_s"] for v in out.values())
    return out


def het_roofline(info, stage_ms, launches, n, near_plane_bytes=4, workload=None):
    """Roofline of the cached-pair products of a heterogeneous plan (HBM-bound: every cached
    kernel value is read once per apply for one right-hand side).  The kernel is symmetric,
    so one block is stored per unordered pair of boxes and serves both directions.
    Algorithmic bytes: near field, the S x S block of every leaf with itself and one block per
    unordered pair of neighbouring leaves (grid of whole leaves), near_plane_bytes per value;
    far field, one Kp x Kp FP32 matrix per unordered interaction-list pair of every level.  The
    dominant stage (near or m2l) by time is the reported kernel; time per launch from the stage
    events."""
    Kp = info["nodes_padded"]
    S = info["leaf"] ** len(n)
    nb = [-(-v // info["leaf"]) for v in n]
    nleaf = int(np.prod(nb))
    directed = int(np.prod([3 * v - 2 for v in nb]))           # leaf pairs at offsets in [-1, 1]^d
    near_blocks = nleaf + (directed - nleaf) // 2
    near_bytes = near_blocks * S * S * near_plane_bytes
    far_bytes = sum(info["far_pairs"][l] // 2 * Kp * Kp * 4.0 for l in range(2, info["levels"] + 1))
    cand = {"near": (near_bytes, stage_ms.get("near", 0.0), launches.get("near", 1.0)),
            "m2l": (far_bytes, stage_ms.get("m2l", 0.0), launches.get("m2l", 1.0))}
    dom = max(cand, key=lambda k: cand[k][1])
    nbytes, tms, nl = cand[dom]
    per = nbytes / nl
    t = tms / nl * 1e-3
    achieved = per / t / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM / 1e9, "unit": "GB/s",
            "frac": achieved / (HBM / 1e9), "traffic": MEASURED_TRAFFIC.get((workload, "fp64", dom)),
            "per_launch": per, "launch_ms": tms / nl, "launches_per_apply": nl,
            "near_gb_per_s": near_bytes / (stage_ms["near"] * 1e-3) / 1e9 if stage_ms.get("near") else None,
            "m2l_gb_per_s": far_bytes / (stage_ms["m2l"] * 1e-3) / 1e9 if stage_ms.get("m2l") else None,
            "near_bytes_per_apply": near_bytes, "far_bytes_per_apply": far_bytes, "near_blocks": near_blocks,
            "far_blocks": [info["far_pairs"][l] // 2 for l in range(info["levels"] + 1)]}


def c5_headline(torch, ertvie, inputs, O, stream, args):
    """The many-scattering medium at 128^3: FP64 FMM apply throughput (the metric), its stage
    profile and roofline, time to 1e-8 for plain FP64 GMRES and the mixed and preconditioned
    solves, and the oracle on sampled rows (its time is the CPU baseline, its values the
    parity check of the timed apply)."""
    n = (C5_N,) * 3
    case = inputs.make_case("c5", n=n, seed=0)
    N = int(np.prod(n))
    fd = torch.from_numpy(case["f"]).cuda()
    res = {"workload": "3D unit cube 128^3 (N=2,097,152), many-scattering medium seed 0: sigma_t = U[5,50] + 8 "
                       "seeded blobs, sigma_s = 0.99 sigma_t, one face source; midpoint ray-quadrature kernel; FMM "
                       "leaf 8^3, Chebyshev order %d (FP64 operator), %d (FP32 inner operator, near field read "
                       "as BF16)" % (C5_CHEB, C5_INNER_CHEB)}
    torch.cuda.empty_cache()
    t = time.perf_counter()
    plan = ertvie.plan_from_case(case, method="fmm", prec="fp64", stream=stream, cheb_n=C5_CHEB,
                                 inner_cheb_n=C5_INNER_CHEB, inner_near16=True)
    try:
        info = plan.fmm_info("fp64")
        log("128^3: FP64 operator built, %.1f s" % (time.perf_counter() - t))
        plan.fmm_info("fp32")
        torch.cuda.synchronize()
        res["plan_s"] = time.perf_counter() - t
        log("128^3: plan %.1f s" % res["plan_s"])
        x = torch.from_numpy(inputs.random_vector(N, 21)).cuda()
        y = torch.empty_like(x)
        plan.apply(x, y, op=ertvie.OP_A)          # first call
        plan.apply(x, y, op=ertvie.OP_A)          # captures the apply graph
        ms = timed_applies(torch, plan, x, y, ertvie.OP_A, args.steps, args.warmup)
        res["apply_ms_fp64"] = ms
        yh = y.cpu().numpy()
        log("128^3 FP64 apply: %.3f ms, %.1f Mpts/s" % (ms, N / (ms * 1e-3) / 1e6))
        st_ms, st_n = stage_profile(plan, x, y, ertvie.OP_A, max(3, min(args.steps, 10)))
        res["stage_ms_fp64"] = st_ms
        log("128^3 FP64 stage ms:", json.dumps({k: round(v, 3) for k, v in st_ms.items()}))
        roof = het_roofline(info, st_ms, st_n, n, workload="c5_128")
        log("128^3 roofline:", json.dumps(roof))
        plan.apply(x, y, op=ertvie.OP_A, prec="fp32")
        plan.apply(x, y, op=ertvie.OP_A, prec="fp32")
        res["apply_ms_fp32_inner"] = timed_applies(torch, plan, x, y, ertvie.OP_A, max(3, args.steps // 2), 1,
                                                   prec="fp32")
        res["fmm_fp64"] = info
        if not args.no_solve:
            res.update(c5_solves(torch, ertvie, plan, fd, N))
        if not args.no_solve and not args.headline_only:
            res["recover_phi"] = transport_s3(torch, inputs, plan, fd, res.get("_U0"), N)
        res.pop("_U0", None)
    finally:
        plan.close()
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on sampled rows of the same apply: ~20 s of CPU on 16 cores
        cores = len(os.sched_getaffinity(0))
        nrows = max(4, min(cores, 16))
        rows = np.random.default_rng(3).choice(N, size=nrows, replace=False)
        P = O.Problem(3, case["n"], case["h"], 1, case["sigma_t"], case["sigma_s"])
        t = time.perf_counter()
        yo = P.apply_rows(inputs.random_vector(N, 21), rows, op=2, nthreads=cores)
        dt = time.perf_counter() - t
        res["fp64_apply_rel_l2_vs_oracle_rows"] = float(np.linalg.norm(yh[rows] - yo) / np.linalg.norm(yo))
        res["oracle_rows"] = nrows
        full_s = dt * N / nrows
        cpu = {"value": N / full_s / 1e6, "unit": "Mpts/s", "cores": cores, "kind": "oracle",
               "sample": "%d sampled rows of the dense FP64 apply of (I - K) on the 128^3 workload (ray-quadrature "
                         "kernel), %.1f s on %d threads, extrapolated by N/rows to %.3g s per apply"
                         % (nrows, dt, cores, full_s)}
        log("128^3 apply error on %d rows: %.3e; cpu oracle: %s" % (nrows, res["fp64_apply_rel_l2_vs_oracle_rows"],
                                                                    json.dumps(cpu)))
    return ms, roof, res, cpu


def c5_order8_rebuilt(torch, ertvie, inputs, O, stream):
    """The 128^3 many-scattering medium with the FP64 operator at Chebyshev order 8: its
    translation matrices (about 330 GB) exceed the device, so the plan stores what fits and
    every apply rebuilds the leaf-level matrices by the ray march (far_cache_gb default).
    Reports the plan, the apply time and the error on sampled rows against the oracle."""
    n = (C5_N,) * 3
    case = inputs.make_case("c5", n=n, seed=0)
    N = int(np.prod(n))
    torch.cuda.empty_cache()
    t = time.perf_counter()
    plan = ertvie.plan_from_case(case, method="fmm", prec="fp64", stream=stream, cheb_n=8)
    try:
        info = plan.fmm_info("fp64")
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t
        log("128^3 order 8: plan %.1f s, rebuilt levels %s, caches %.1f GB"
            % (plan_s, info["far_rebuilt"], info["cache_bytes"] / 1e9))
        x = torch.from_numpy(inputs.random_vector(N, 21)).cuda()
        y = torch.empty_like(x)
        times = []
        for _ in range(3):          # eager, captured, replayed
            torch.cuda.synchronize()
            t = time.perf_counter()
            plan.apply(x, y, op=ertvie.OP_A)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            log("128^3 order 8 apply: %.3f s" % times[-1])
        yh = y.cpu().numpy()
    finally:
        plan.close()
        torch.cuda.empty_cache()
    cores = len(os.sched_getaffinity(0))
    nrows = max(4, min(cores, 16))
    rows = np.random.default_rng(3).choice(N, size=nrows, replace=False)
    P = O.Problem(3, case["n"], case["h"], 1, case["sigma_t"], case["sigma_s"])
    yo = P.apply_rows(inputs.random_vector(N, 21), rows, op=2, nthreads=cores)
    err = float(np.linalg.norm(yh[rows] - yo) / np.linalg.norm(yo))
    log("128^3 order 8: error on %d rows %.3e" % (nrows, err))
    return {"workload": "128^3 many-scattering medium seed 0, FP64 FMM apply of I - K, leaf 8^3, Chebyshev order 8",
            "plan_s": plan_s, "apply_s": times, "far_rebuilt": info["far_rebuilt"],
            "cache_gb": info["cache_bytes"] / 1e9, "far_pairs": info["far_pairs"],
            "rel_l2_vs_oracle_rows": err, "oracle_rows": nrows}


def c5_solves(torch, ertvie, plan, fd, N):
    """Time to a 1e-8 true residual at 128^3 (each solve once untimed for graph capture and
    tuning, then timed): plain FP64 GMRES; the FP64-refined solve with FP32 inner GMRES on the
    order-4 operator (mixed); mixed with the learned preconditioner; mixed with the FFT-based
    preconditioner on the inner solves; and that with the network after it."""
    out = {}
    keys = ("iters", "matvecs", "restarts", "t_solve", "rel_resid_true", "rejected", "precond_applies")
    U = torch.empty_like(fd)
    # the Krylov basis is allocated for max_iter vectors (16.8 MB each at this size)
    plan.solve(fd, U, tol=1e-8, max_iter=150)
    r = plan.solve(fd, U, tol=1e-8, max_iter=150)
    out["plain_fp64_gmres"] = {k: r[k] for k in keys}
    U0 = U.clone()
    out["_U0"] = U0
    log("128^3 plain:", json.dumps(out["plain_fp64_gmres"]))
    runs = [("mixed", dict(mixed=True, inner_tol=1e-2), None, None),
            ("mixed_fft", dict(mixed=True, inner_tol=1e-3, precond_fft=True), None, None)]
    for name, path in (("mixed_learned", WEIGHTS), ("mixed_fft_learned", WEIGHTS_FFT)):
        if os.path.exists(path):
            w = np.load(path)
            meta = json.loads(str(w["meta"]))
            kw = dict(mixed=True, inner_tol=float(meta.get("inner_tol", 1e-2)),
                      precond_steps=int(meta.get("precond_steps", 0)))
            if "fft" in name:
                kw["precond_fft"] = True
            # a coarse-grid network keeps its grid; a full-grid one takes the plan's
            f = int(meta.get("coarsen", 1))
            ngrid = tuple(int(v) for v in meta["n"]) if f > 1 else (C5_N,) * 3
            runs.append((name, kw, w["params"], ngrid))
    for name, kw, params, ngrid in runs:
        net = None
        if params is not None:
            net = ertvie.Net(ngrid, stream=plan.stream)
            net.set_params(params)
            kw = dict(kw, precond=net)
        try:
            plan.solve(fd, U, tol=1e-8, max_iter=150, **kw)
            r = plan.solve(fd, U, tol=1e-8, max_iter=150, **kw)
        finally:
            if net is not None:
                net.close()
        out[name] = {k: r[k] for k in keys}
        out[name]["vs_plain_rel_l2"] = float(torch.linalg.norm(U - U0) / torch.linalg.norm(U0))
        out[name]["speedup_vs_plain"] = out["plain_fp64_gmres"]["t_solve"] / r["t_solve"]
        log("128^3 %s:" % name, json.dumps(out[name]))
    return out


def transport_s3(torch, inputs, plan, fd, U0, N):
    """Algorithm 1 S.3 from the solution: Phi for 26 directions (cube faces, edges, corners)."""
    if U0 is None:
        return None
    n = int(round(N ** (1.0 / 3.0)))
    dirs = np.array([d for d in itertools.product((-1, 0, 1), repeat=3) if any(d)], dtype=np.float64)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    phi = torch.empty((len(dirs), N), dtype=torch.float64, device="cuda")
    plan.transport(U0, fd, dirs, phi)                    # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.transport(U0, fd, dirs, phi)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    # ray steps of the sweep (the same count rule as the kernel), for the per-step rate
    xc = inputs.centres((n, n, n), 1.0 / n)
    steps = 0
    for v in dirs:
        sb = np.full(N, np.inf)
        for a in range(3):
            if v[a] > 0:
                sb = np.minimum(sb, xc[:, a] / v[a])
            elif v[a] < 0:
                sb = np.minimum(sb, (1.0 - xc[:, a]) / (-v[a]))
        steps += int(np.maximum(1, np.ceil(sb / (0.5 / n) * (1 - 1e-12))).sum())
    out = {"directions": len(dirs), "seconds": ts, "cell_directions_per_s": N * len(dirs) / ts,
           "ray_steps": steps, "steps_per_s": steps / ts,
           # eight interpolation corners of one (sigma_t, Q) pair, 16 bytes each
           "l2_gather_bytes_per_s": steps * 8 * 16 / ts}
    log("128^3 S.3:", json.dumps(out))
    return out


def c2_32(torch, ertvie, inputs, O, stream, args):
    """32^3 homogeneous workload (sigma_t = 5, sigma_s = 4, four Gaussian sources): FP32 FMM
    apply with compressed translations, its stage profile and the roofline of the grouped
    near-field + translation launch, the FP64 and BF16x3 applies, the dense FP64 apply, and
    time to 1e-8 (FP64 GMRES and the mixed solve)."""
    case = inputs.make_case("c2", seed=0)
    N = int(np.prod(case["n"]))
    f = torch.from_numpy(case["f"]).cuda()
    y = torch.empty_like(f)
    out = {"workload": "3D unit cube 32^3 (N=32768), homogeneous sigma_t=5 sigma_s=4, four seeded Gaussian "
                       "sources; FMM leaf 8^3 cells, n=8, translations compressed at 1e-5; FP32 apply of I - K"}
    t = time.perf_counter()
    with ertvie.plan_from_case(case, method="fmm", prec="fp32", stream=stream, svd_tol=SVD_TOL, form=args.form) as plan:
        plan.apply(f, y, op=ertvie.OP_A)          # builds the FMM operators, tunes the execution forms
        plan.apply(f, y, op=ertvie.OP_A)          # captures the apply graph
        torch.cuda.synchronize()
        out["plan_s"] = time.perf_counter() - t
        ms = timed_applies(torch, plan, f, y, ertvie.OP_A, 50, 5)
        yg = y.cpu().numpy()
        st_ms, st_n = stage_profile(plan, f, y, ertvie.OP_A, 20)
        info = plan.fmm_info()
    info["leaf_boxes"] = int(np.prod([-(-n // info["leaf"]) for n in case["n"]]))
    forms = "%d,%d" % (info["form_near"], info["form_far"][info["levels"]])
    out.update({"apply_ms": ms, "mpts_per_s": N / (ms * 1e-3) / 1e6, "stage_ms": st_ms, "fmm": info,
                "roofline": roofline_of(info, st_ms, st_n, "fp32", workload="c2", forms=forms)})
    P = O.Problem(3, case["n"], case["h"], 0, case["sigma_t"], case["sigma_s"])
    rows = np.random.default_rng(0).choice(N, size=256, replace=False)
    yo = P.apply_rows(case["f"], rows, op=2)
    out["rel_l2_vs_oracle_rows"] = float(np.linalg.norm(yg[rows] - yo) / np.linalg.norm(yo))
    log("32^3 FP32 apply %.4f ms (%.1f Mpts/s), error on 256 rows %.2e, roofline %s"
        % (ms, out["mpts_per_s"], out["rel_l2_vs_oracle_rows"], json.dumps(out["roofline"])))
    with ertvie.plan_from_case(case, method="fmm", prec="fp64", stream=stream, svd_tol=SVD_TOL) as p64:
        p64.apply(f, y, op=ertvie.OP_A)
        p64.apply(f, y, op=ertvie.OP_A)
        out["fp64_apply_ms"] = timed_applies(torch, p64, f, y, ertvie.OP_A, 20, 2)
        y64 = y.cpu().numpy()
        out["fp64_rel_l2_vs_oracle_rows"] = float(np.linalg.norm(y64[rows] - yo) / np.linalg.norm(yo))
        p64.apply(f, y, op=ertvie.OP_A, prec="bf16x3")
        out["bf16x3_apply_ms"] = timed_applies(torch, p64, f, y, ertvie.OP_A, 20, 2, prec="bf16x3")
        y16 = y.cpu().numpy()
        out["bf16x3_rel_l2_vs_oracle_rows"] = float(np.linalg.norm(y16[rows] - yo) / np.linalg.norm(yo))
        out["direct_fp64_apply_ms"] = timed_applies(torch, p64, f, y, ertvie.OP_A, 2, 1, method="direct")
        if not args.no_solve:
            U = torch.empty_like(f)
            p64.solve(f, U, tol=1e-8)                               # warm: FP64 graphs
            p64.solve(f, U, tol=1e-8, mixed=True, inner_tol=1e-4)   # warm: builds the FP32 operator
            i64 = p64.solve(f, U, tol=1e-8)
            U64 = U.clone()
            imx = p64.solve(f, U, tol=1e-8, mixed=True, inner_tol=1e-4)
            out["solve"] = {"tol": 1e-8, "fp64_gmres_s": i64["t_solve"], "fp64_iters": i64["iters"],
                            "fp64_rel_resid_true": i64["rel_resid_true"], "mixed_s": imx["t_solve"],
                            "mixed_inner_iters": imx["iters"], "mixed_refinements": imx["restarts"],
                            "mixed_rel_resid_true": imx["rel_resid_true"],
                            "mixed_vs_fp64_rel_l2": float(torch.linalg.norm(U - U64) / torch.linalg.norm(U64))}
    log("32^3:", json.dumps({k: v for k, v in out.items() if k not in ("fmm", "roofline")}))
    return out, P, case


def c3_64(torch, ertvie, inputs, O, stream):
    """64^3 heterogeneous blob medium with the ray-quadrature kernel (cached pair
    translations): FP32 FMM apply, stage profile, error on sampled rows."""
    c3 = inputs.make_case("c3", seed=0)
    N3 = int(np.prod(c3["n"]))
    x3 = inputs.random_vector(N3, 11)
    xd = torch.from_numpy(x3).cuda()
    yd = torch.empty_like(xd)
    t = time.perf_counter()
    with ertvie.plan_from_case(c3, method="fmm", prec="fp32", stream=stream) as p3:
        p3.apply(xd, yd, op=ertvie.OP_A)
        p3.apply(xd, yd, op=ertvie.OP_A)
        torch.cuda.synchronize()
        t3plan = time.perf_counter() - t
        ms3 = timed_applies(torch, p3, xd, yd, ertvie.OP_A, 5, 1)
        y3 = yd.cpu().numpy()
        st3, _ = stage_profile(p3, xd, yd, ertvie.OP_A, 3)
    P3 = O.Problem(3, c3["n"], c3["h"], 1, c3["sigma_t"], c3["sigma_s"])
    r3 = np.random.default_rng(7).choice(N3, size=24, replace=False)
    y3o = P3.apply_rows(x3, r3, op=2)
    out = {"workload": "64^3 blob medium seed 0, FP32 FMM (leaf 8^3, n = 8)", "plan_s": t3plan, "apply_ms": ms3,
           "mpts_per_s": N3 / (ms3 * 1e-3) / 1e6, "stage_ms": st3,
           "rel_l2_vs_oracle_rows": float(np.linalg.norm(y3[r3] - y3o) / np.linalg.norm(y3o))}
    log("c3:", json.dumps(out))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 128^3 workload (applies, stage profile, solves)")
    ap.add_argument("--form", type=int, default=None,
                    help="fix the execution form of the 32^3 box-offset products (0..5) instead of timing them")
    ap.add_argument("--many-rhs-only", action="store_true",
                    help="only the 64-right-hand-side section on the 64^3 blob medium (one JSON line)")
    ap.add_argument("--homogeneous-only", action="store_true",
                    help="only the homogeneous 32^3 and 64^3 sections (one JSON line of their results)")
    ap.add_argument("--fft-only", action="store_true",
                    help="time only the FFT-based preconditioner (64^3 and 128^3) and exit")
    ap.add_argument("--paper-exp3", action="store_true",
                    help="also run the paper's accuracy experiment ((M-ii) vs (M-iii), 2D, 12 grids, three media)")
    ap.add_argument("--paper-exp6", action="store_true",
                    help="also run the paper's preconditioning experiment (2D 512^2, four media)")
    ap.add_argument("--rebuilt-only", action="store_true",
                    help="only the 128^3 order-8 FP64 apply whose leaf-level translation matrices do not fit "
                         "and are rebuilt by every apply (one JSON line)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run three 256 MiB device copies (reference for memory-traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the work would shard by "
              "right-hand sides or by Morton-contiguous leaf ranges).", file=sys.stderr)
        sys.exit(2)

    import torch
    from oracle import oracle as O
    from paper_1610_00835_amd import ertvie, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.fft_only:
        print(json.dumps({"fft_precond": fft_only(torch, ertvie, inputs, stream, args.steps)}), flush=True)
        return
    if args.many_rhs_only:
        print(json.dumps({"many_rhs_64cubed": many_rhs_64(torch, ertvie, inputs, stream)}), flush=True)
        return
    if args.rebuilt_only:
        print(json.dumps({"order8_128cubed_rebuilt": c5_order8_rebuilt(torch, ertvie, inputs, O, stream)}),
              flush=True)
        return
    if args.homogeneous_only:
        out = {}
        out["c2_32cubed_homogeneous"], _, _ = c2_32(torch, ertvie, inputs, O, stream, args)
        out["c2_recipe_64cubed_homogeneous"] = homogeneous_64(torch, ertvie, inputs, O, stream)
        print(json.dumps(out), flush=True)
        return

    ertvie.load()
    read_ref = hbm_read_reference(torch, ertvie, dev, stream)
    log("HBM read reference:", json.dumps(read_ref))
    N = C5_N ** 3
    ms, roofline, c5, cpu = c5_headline(torch, ertvie, inputs, O, stream, args)
    roofline["attainable_read_gb_per_s"] = read_ref["gb_per_s"]
    roofline["frac_of_attainable_read"] = roofline["achieved"] / read_ref["gb_per_s"]
    value = N / (ms * 1e-3) / 1e6
    extra = {"many_scattering_128cubed": c5, "hbm_read_reference": read_ref}
    if not args.headline_only:
        extra["c2_32cubed_homogeneous"], _, _ = c2_32(torch, ertvie, inputs, O, stream, args)
        extra["c2_recipe_64cubed_homogeneous"] = homogeneous_64(torch, ertvie, inputs, O, stream)
        extra["c3_64cubed_heterogeneous"] = c3_64(torch, ertvie, inputs, O, stream)
        if not args.no_solve:
            extra["many_rhs_64cubed"] = many_rhs_64(torch, ertvie, inputs, stream)
    if args.paper_exp6:
        extra["paper_experiment_vi"] = paper_experiment_vi(torch, ertvie, inputs, stream)
    if args.paper_exp3:
        extra["paper_experiment_iii"] = paper_experiment_iii(torch, ertvie, inputs, stream)

    out = {"metric": "FMM matvec Mpts/s; time to 1e-8 solve, plain FP64 GMRES vs mixed+learned (1 GPU)",
           "value": value, "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": c5["workload"], "op": "u - K(sigma_s u)", "prec": "fp64", "nrhs": 1},
           "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
