#!/usr/bin/env python3
"""Throughput of the NNCA H2 matvec on one MI355X.

Workload: 3D 1/|x-y| (zero on the diagonal), N = 2^20 points uniform in
[-1,1]^3, leaf <= 64, ACA tolerance 1e-6, one right-hand side x ~ N(0,1)
(seeded, synthetic).  A step is one mixed-precision matvec y = A~ x through
the whole apply path (gather/split, P2M/M2M, M2L, L2L/L2P, near field and
FP64 combine) with the H2 representation resident in HBM; the FP64 GPU build
(tree, ACA pivots, transfer operators) is timed separately.

Prints one JSON line.  The per-launch durations of the dominant kernel (M2L)
come from HIP events the library records on its launch stream during the
timed steps.  The CPU baseline is the plain FP64 oracle timed on a smaller
sample of the same distribution and scaled by interaction count.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H2 matvecs/s at N=1M 3D 1/r, mixed vs FP64 at rel.err≤1e-6; % roofline"
# Roofline of the dominant kernel, the symmetric FP32 transverse pass (M2L)
# of the two finest levels (1/r).  Its bound is plain VALU arithmetic.  Peak FP32
# vector rate of the chip: 157.3 TFLOP/s = 256 CU x 128 lanes/clock x
# 2.4 GHz x 2 (FMA), i.e. 7.864e13 lane-instructions/s.  One unordered pair
# of pivots costs 1 addition and 3 FMA for r^2 = |t|^2 + |s|^2 - 2 t.s, one
# v_rsq_f32 (quarter rate: 4 issue slots) and 2 FMA (its row and its column
# term): 10 slots.
VALU_LANE_SLOTS = 256 * 128 * 2.4e9
SLOTS_PER_PAIR = 10.0
PEAK_PAIRS = VALU_LANE_SLOTS / SLOTS_PER_PAIR
# HBM bytes per launch of that kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs of `bench.py --probe` (profiles/h2_matvec_c2_hbm_bytes.md), scaled by
# the counters' reading of a 256 MiB copy: fetch + write MiB at kappa and
# kappa-1.  Valid for one version of k_m2l_sym; None once the kernel changes.
M2L_SYM_HBM_MIB = ((387.7, 343.8), (30.9, 120.3))
# Dense FP32 matrix-core peak of MI355X (the many-column transverse pass and
# near field multiply FP32 kernel tiles by weight tiles on the matrix cores)
FP32_MFMA_PEAK = 157.3e12


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_full_inter: int, sample_n: int = 1 << 16, reps: int = 3, points=None, x=None, yd_gpu=None,
                 direct_rows: int = 16384):
    """Oracle (plain FP64 C, OpenMP over cells) on a sample of the workload,
    on all host threads and on one; with the full problem's points, its
    compensated direct sum on `direct_rows` sampled rows, which also checks
    the GPU direct sum `yd_gpu` behind the error figures."""
    import oracle
    from paper_2203_14832_amd.workloads import workload
    p, xs = workload("c2", n=sample_n)
    T = oracle.Tree(p, 64)
    H = oracle.H2(T, "inv_r", 1e-6)
    H.matvec(xs[:, 0])
    t0 = time.perf_counter()
    for _ in range(reps):
        H.matvec(xs[:, 0])
    dt = (time.perf_counter() - t0) / reps
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        H.matvec(xs[:, 0])
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    far, near = H.interactions()
    rate = (far + near) / dt
    out = {
        "value": rate / n_full_inter, "unit": "matvecs/s", "cores": threads, "kind": "oracle",
        "sample": f"oracle FP64 matvec on N={sample_n} points of the same distribution (leaf 64, tol 1e-6), "
                  f"{reps} timed matvecs, {far + near} interactions each, scaled by interaction count to "
                  f"the N=2^20 problem ({n_full_inter} interactions)",
        "sample_seconds_per_matvec": dt, "one_thread_seconds_per_matvec": dt1,
        "one_thread_matvecs_per_s": (far + near) / dt1 / n_full_inter, "cpu_model": cpu_model(),
    }
    if points is not None and yd_gpu is not None:
        n = points.shape[0]
        rows = np.sort(np.random.default_rng(2024).choice(n, min(direct_rows, n), replace=False))
        t0 = time.perf_counter()
        yo = oracle.direct(points, x, "inv_r", rows=rows)
        dtd = time.perf_counter() - t0
        out["direct_sample"] = {
            "rows": int(rows.size), "seconds": dtd,
            "gpu_direct_rel_err": float(np.linalg.norm(yd_gpu[rows] - yo) / np.linalg.norm(yo)),
            "gpu_direct_max_abs_err_over_max": float(np.abs(yd_gpu[rows] - yo).max() / np.abs(yo).max()),
        }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--probe", action="store_true",
                    help="counter runs: one 256 MiB device copy (calibration of byte counters) and --steps "
                         "mixed matvecs of the workload, no timing")
    ap.add_argument("--rates", action="store_true",
                    help="print the device's attainable rates (copy, FMA, rsq, the symmetric pass's inner loop)")
    ap.add_argument("--config", default="c2", choices=["c2", "c3", "c4", "c5", "ie", "exp", "general", "svm"],
                    help="c2: the metric (N=2^20 cube, 1 RHS); c3: 64 RHS on the sphere, block vs column loop; "
                         "c4: Gaussian forward + backward (x and length scale); c5: uneven batch of 32 problems")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_14832_amd import nnca
    from paper_2203_14832_amd.workloads import workload

    if args.probe:
        return probe(args)
    if args.rates:
        print(json.dumps({"attainable": nnca.probe_rates(torch.device("cuda:0")),
                          "peaks": {"hbm_bytes_per_s": 8e12, "fp32_lane_ops_per_s": VALU_LANE_SLOTS,
                                    "yardstick_pairs_per_s": PEAK_PAIRS}}), flush=True)
        return
    if args.config == "c3":
        return bench_many_rhs(args)
    if args.config == "c4":
        return bench_backward(args)
    if args.config == "c5":
        return bench_batch(args)
    if args.config == "ie":
        return bench_integral_equation(args)
    if args.config == "exp":
        return bench_experiments(args)
    if args.config == "general":
        return bench_general(args)
    if args.config == "svm":
        return bench_svm(args)
    dev = torch.device("cuda:0")
    p, x = workload("c2", n=args.n)
    n = p.shape[0]
    t0 = time.perf_counter()
    H = nnca.H2Matrix(p, "inv_r", 1e-6, 64, device=dev)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = H.info()
    bst = H.build_stats()
    inter = info["m2l_interactions"] + info["p2p_interactions"]
    print(f"[bench] built N={n} kappa={info['kappa']} in {build_s:.2f}s, "
          f"M2L {info['m2l_interactions']:.3e} + P2P {info['p2p_interactions']:.3e} interactions",
          file=sys.stderr, flush=True)

    X = torch.tensor(x[:, 0], device=dev).reshape(1, n).contiguous()
    Ym = torch.empty_like(X)
    Y64 = torch.empty_like(X)

    def run(prec, Y, k):
        for _ in range(k):
            H.matvec_raw(X, Y, 1, prec)

    # FP64 matvec (reference arithmetic on the same pivots), with the same
    # schedule as the mixed one (symmetric transverse pass) and with the plain
    # (every ordered pair) pass
    def time_fp64(sym):
        H.set_symmetric(sym)
        run("fp64", Y64, 2)
        torch.cuda.synchronize()
        k64 = max(3, args.steps // 4)
        t0 = time.perf_counter()
        run("fp64", Y64, k64)
        torch.cuda.synchronize()
        H.set_symmetric(True)
        return (time.perf_counter() - t0) / k64 * 1e3

    fp64_plain_ms = time_fp64(False)
    fp64_ms = time_fp64(True)
    run("fp64", Y64, 1)

    # timed mixed-precision steps; HIP events on the library stream bracket
    # the launches of the transverse-pass kernel only
    run("mixed", Ym, args.warmup)
    torch.cuda.synchronize()
    H.profile(True, passes=[2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run("mixed", Ym, args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    passes, levels, ms = H.profile_read()
    H.profile(False)
    ms_step = dt / args.steps * 1e3
    value = args.steps / dt

    # the same steps without any event, for reference
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run("mixed", Ym, args.steps)
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t0) / args.steps * 1e3

    # the mixed form with the plain (every ordered pair) transverse pass, to
    # separate the gain of FP32 arithmetic from that of the symmetric pass
    H.set_symmetric(False)
    run("mixed", Ym, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run("mixed", Ym, args.steps)
    torch.cuda.synchronize()
    ms_nosym = (time.perf_counter() - t0) / args.steps * 1e3
    H.set_symmetric(True)
    run("mixed", Ym, 1)

    # per-pass breakdown from separate (untimed) steps with every launch bracketed
    H.profile(True)
    run("mixed", Ym, 5)
    torch.cuda.synchronize()
    bp, bl, bm = H.profile_read()
    H.profile(False)
    breakdown = {name: float(bm[bp == i].sum() / 5)
                 for i, name in enumerate(["gather", "up", "m2l", "down", "p2p", "m2l_combine"])}

    # dominant kernel: the symmetric FP32 transverse pass of the two finest
    # levels (coarser levels run the FP64-refined form)
    kap = info["kappa"]
    fine = (passes == 2) & (levels >= kap - 1)
    m2l_ms = ms[fine]
    m2l_per_step = m2l_ms.sum() / args.steps
    launches_per_step = m2l_ms.size / args.steps
    fine_inter = sum(info["m2l_level"][l] for l in range(max(kap - 1, 0), kap + 1))
    pairs = fine_inter / 2
    pair_rate = pairs / (m2l_per_step * 1e-3)
    coarse_ms = float(ms[(passes == 2) & (levels < kap - 1)].sum() / args.steps)

    err_mixed = float(torch.linalg.norm(Ym - Y64) / torch.linalg.norm(Y64))
    out = {
        "metric": METRIC, "value": value, "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"3D 1/r, N={n} uniform in [-1,1]^3, leaf 64, tol 1e-6, 1 RHS N(0,1), "
                               f"mixed FP32 apply with FP64 pivots/operators and FP64 near-field refinement",
                   "n": n, "kappa": info["kappa"], "leaf_size": 64, "tol": 1e-6, "nrhs": 1},
        "roofline": {"bound": "alu", "achieved": pair_rate / 1e9, "peak": PEAK_PAIRS / 1e9,
                     "unit": "G pairs/s", "frac": pair_rate / PEAK_PAIRS,
                     "traffic": (sum(f + w for f, w in M2L_SYM_HBM_MIB) / len(M2L_SYM_HBM_MIB) * 2 ** 20
                                 if M2L_SYM_HBM_MIB else None),
                     "traffic_unit": "bytes per launch (HBM, counters)",
                     "kernel": "k_m2l_sym<1/r, FP32> (levels kappa-1, kappa)",
                     "launches_per_step": launches_per_step,
                     "avg_launch_ms": float(m2l_ms.mean()) if m2l_ms.size else None,
                     "pairs_per_launch": pairs / max(launches_per_step, 1),
                     "directed_interactions_per_s": 2 * pair_rate,
                     "peak_derivation": "7.864e13 FP32 lane-instr/s / 10 slots per pair "
                                        "(r^2: add + 3 fma; 1/r: v_rsq_f32 = 4; 2 fma)"},
        "m2l_fine_ms_per_launch_by_level": {int(l): float(ms[(passes == 2) & (levels == l)].mean())
                                            for l in range(max(kap - 1, 0), kap + 1)},
        "m2l_coarse_fp64_ms_per_step": coarse_ms, "m2l_level_interactions": info["m2l_level"],
        # both forms with the symmetric transverse pass (the same schedule)
        "fp64_ms_per_step": fp64_ms, "fp64_matvecs_per_s": 1e3 / fp64_ms, "speedup_vs_fp64": fp64_ms / ms_step,
        # both forms with the plain pass, and the mixed default against it
        "fp64_plain_pass_ms_per_step": fp64_plain_ms, "mixed_plain_pass_ms_per_step": ms_nosym,
        "speedup_vs_fp64_plain_pass": fp64_plain_ms / ms_nosym,
        "speedup_mixed_vs_fp64_plain_pass": fp64_plain_ms / ms_step,
        "err_mixed_vs_fp64": err_mixed, "build_seconds": build_s, "pass_ms_per_step": breakdown,
        # the build's pivot traversal against HBM: its algorithmic panel reads
        # (step k of a cell's ACA reads the k previous panel rows twice) over
        # its time
        "build_roofline": {"bound": "hbm", "kernel": "k_aca / k_acm_* (pivot traversal, FP64)",
                           "achieved": bst["aca_panel_bytes"] / bst["aca_seconds"] / 1e9, "peak": 8000.0,
                           "unit": "GB/s", "frac": bst["aca_panel_bytes"] / bst["aca_seconds"] / 8e12,
                           "aca_seconds": bst["aca_seconds"], "panel_bytes": bst["aca_panel_bytes"],
                           "build_seconds_library": bst["build_seconds"]},
        "interactions_per_step": inter, "ms_per_step_without_events": ms_plain,
    }
    # attainable rates measured on this device (copy, FMA, rsq, and the
    # kernel's inner loop with its operands in registers)
    att = nnca.probe_rates(dev)
    out["attainable"] = att
    out["roofline"]["frac_of_attainable_inner_loop"] = pair_rate / att["sym_pairs_per_s_valu"]
    yd = None
    if not args.no_direct:
        yd = nnca.direct(p, X.reshape(n), "inv_r", device=dev)
        torch.cuda.synchronize()
        out["err_fp64_vs_direct"] = float(torch.linalg.norm(Y64.reshape(n) - yd) / torch.linalg.norm(yd))
        out["err_mixed_vs_direct"] = float(torch.linalg.norm(Ym.reshape(n) - yd) / torch.linalg.norm(yd))
        yd = yd.cpu().numpy()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inter, points=p, x=x[:, 0], yd_gpu=yd)
    print(json.dumps(out), flush=True)


def bench_experiments(args):
    """The trends of Exp. 1-4 (Sec. 5) with the regularised kernels (a = 1e-4):
    assembly time, FP64 and mixed matvec times and the relative error against
    the FP64 direct sum, (i) against the ACA tolerance at N = 102400 in 2D
    (uniform points with both kernels, Exp. 1; the 320^2 Chebyshev grid with
    the log kernel, Exp. 2), (ii) against N at tol 1e-7 in 3D (uniform points,
    Exp. 3; Chebyshev grids, Exp. 4) with the 1/r kernel."""
    import torch
    from paper_2203_14832_amd import nnca
    from paper_2203_14832_amd.workloads import chebyshev_grid
    dev = torch.device("cuda:0")
    a = 1e-4
    rows = []

    def one(exp, dist, kind, p, tol, leaf=64):
        n = p.shape[0]
        x = torch.tensor(np.random.default_rng(1010).standard_normal(n), device=dev)
        t0 = time.perf_counter()
        H = nnca.H2Matrix(p, kind, tol, leaf, length_scale=a, device=dev)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        yd = nnca.direct(p, x, kind, a, device=dev)
        out = {"exp": exp, "dist": dist, "kernel": kind, "n": n, "tol": tol, "assembly_s": ta,
               "kappa": H.info()["kappa"]}
        for prec in ("fp64", "mixed"):
            y = H.matvec(x, prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                y = H.matvec(x, prec)
            torch.cuda.synchronize()
            out[f"matvec_ms_{prec}"] = (time.perf_counter() - t0) / 5 * 1e3
            out[f"eps_m_{prec}"] = float(torch.linalg.norm(y - yd) / torch.linalg.norm(yd))
        rows.append(out)
        print(json.dumps(out), file=sys.stderr, flush=True)
        H.close()
        torch.cuda.empty_cache()

    rng = np.random.default_rng(1011)
    p2u = rng.uniform(-1, 1, (102400, 2))
    p2c = chebyshev_grid(320, 2)
    for tol in (1e-3, 1e-5, 1e-7, 1e-9, 1e-11):
        one(1, "uniform 2D", "log_reg", p2u, tol)
        one(1, "uniform 2D", "inv_reg", p2u, tol)
        one(2, "Chebyshev 2D", "log_reg", p2c, tol)
    for m in (15, 16, 17, 18, 19, 20):
        one(3, "uniform 3D", "inv_reg", rng.uniform(-1, 1, (1 << m, 3)), 1e-7)
    for na in (32, 40, 50, 64, 80, 100):
        one(4, "Chebyshev 3D", "inv_reg", chebyshev_grid(na, 3), 1e-7)
    print(json.dumps({"config": "exp", "a": a, "rows": rows}), flush=True)


def bench_general(args):
    """The general case P != Q (Sec. 2.3): 3D 1/r, tol 1e-6, leaf 64, sources
    Q = 2^20 points uniform in [-1,1]^3, targets P either 2^20 other points
    uniform in the same cube (evaluation at new points) or 2^19 points in the
    shifted cube 0.3 + 0.8 [-1,1]^3.  Build time, the forward (Q -> P) and
    transposed (P -> Q) products in FP64 and mixed precision, interactions
    per second, and the error against the FP64 direct sum on 16384 sampled
    targets (nnca_direct over the sampled targets and the sources with zero
    weights on the targets: K is 0 only at r = 0, as in the method)."""
    import torch
    from paper_2203_14832_amd import nnca
    dev = torch.device("cuda:0")
    rows = []
    steps = max(1, args.steps // 4)
    for name in ("same_cube", "shifted"):
        rng = np.random.default_rng(1012)
        Q = rng.uniform(-1, 1, (1 << 20, 3))
        if name == "same_cube":
            P = rng.uniform(-1, 1, (1 << 20, 3))
        else:
            P = rng.uniform(-1, 1, (1 << 19, 3)) * 0.8 + 0.3
        x = torch.tensor(rng.standard_normal(Q.shape[0]), device=dev)
        g = torch.tensor(rng.standard_normal(P.shape[0]), device=dev)
        t0 = time.perf_counter()
        G = nnca.H2General(P, Q, "inv_r", 1e-6, 64, device=dev)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        inf = G.info()
        inter = inf["m2l_interactions"] + inf["p2p_interactions"]
        out = {"layout": name, "np": int(P.shape[0]), "nq": int(Q.shape[0]), "kappa": inf["kappa"],
               "assembly_s": ta, "m2l_interactions": inf["m2l_interactions"],
               "p2p_interactions": inf["p2p_interactions"]}
        sample = np.sort(rng.choice(P.shape[0], 16384, replace=False))
        Z = np.vstack([P[sample], Q])
        xz = torch.cat([torch.zeros(len(sample), dtype=torch.float64, device=dev), x])
        yd = nnca.direct(Z, xz, "inv_r", device=dev)[: len(sample)]
        sd = torch.tensor(sample, device=dev)
        for prec in ("fp64", "mixed"):
            for tr, fn, v in (("forward", G.matvec, x), ("transposed", G.rmatvec, g)):
                y = fn(v, prec)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    y = fn(v, prec)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / steps * 1e3
                out[f"{tr}_ms_{prec}"] = ms
                if tr == "forward":
                    out[f"interactions_per_s_{prec}"] = inter / (ms * 1e-3)
                    out[f"eps_m_{prec}"] = float(torch.linalg.norm(y[sd] - yd) / torch.linalg.norm(yd))
        rows.append(out)
        print(json.dumps(out), file=sys.stderr, flush=True)
        G.close()
        del G
        torch.cuda.empty_cache()
    print(json.dumps({"config": "general", "workload": "3D 1/r, tol 1e-6, leaf 64, 2^20 uniform sources; targets "
                                                       "2^20 uniform in the same cube, or 2^19 in a shifted cube",
                      "rows": rows}), flush=True)


def bench_svm(args):
    """Exp. 6 in 2D: kernel SVM trained by projected gradient ascent with
    the H2 matvec (FSVM).  The two datasets (M points uniform in
    [-1.4,1.4]^2, 85 % for training): exp(-r) with the
    disk labels and exp(-r^2) with the wave labels; lambda = 1, beta = 1,
    the step 1 / (||K~|| + beta n), tol 1e-8 for the ACA, training until the
    relative step is below 1e-4.  Per dataset: assembly (build) seconds,
    training steps and seconds, seconds per step with the H2 product and
    with the GPU direct sum in its place (NSVM), and the per-class and
    overall accuracy on the held-out points.  Then seconds per step at M =
    2^16, 2^18, 2^20 (100 steps at tol 0)."""
    import torch
    from paper_2203_14832_amd import nnca
    from paper_2203_14832_amd.workloads import svm_dataset
    dev = torch.device("cuda:0")
    rows = []
    for kind, rule in (("exp_r", "disk"), ("gauss", "wave")):
        for m in (5625, 1 << 16, 1 << 18, 1 << 20):
            P, y, Q, yq = svm_dataset(m, 2, rule)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            G = nnca.H2Matrix(P, kind, 1e-8, 64, device=dev)
            torch.cuda.synchronize()
            ta = time.perf_counter() - t0
            row = {"kernel": kind, "labels": rule, "M": m, "train": [int((y > 0).sum()), int((y < 0).sum())],
                   "test": [int((yq > 0).sum()), int((yq < 0).sum())], "assembly_s": ta}
            if m == 5625:
                t0 = time.perf_counter()
                a, b, it, eta = G.svm_train(y, 1.0, 1.0, tol=1e-4, max_iter=50000)
                torch.cuda.synchronize()
                tt = time.perf_counter() - t0
                GG = nnca.H2General(Q, P, kind, 1e-8, 64, device=dev)
                f = GG.svm_decision(y, a, b).cpu().numpy()
                GG.close()
                acc = [float(np.mean(np.sign(f[yq == c]) == c)) for c in (1.0, -1.0)]
                row.update({"steps": it, "train_s": tt, "s_per_step": tt / max(it, 1), "eta": eta, "bias": b,
                            "accuracy_per_class": acc, "accuracy": float(np.mean(np.sign(f) == yq))})
                # NSVM: the same step with the GPU direct sum for K v
                v = torch.tensor(y, device=dev)
                nnca.direct(P, v, kind, device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(20):
                    nnca.direct(P, v, kind, device=dev)
                torch.cuda.synchronize()
                row["direct_matvec_s"] = (time.perf_counter() - t0) / 20
            else:
                G.svm_train(y, 1.0, 1.0, tol=0.0, max_iter=3)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, it, _ = G.svm_train(y, 1.0, 1.0, tol=0.0, max_iter=100)
                torch.cuda.synchronize()
                tt = time.perf_counter() - t0
                row.update({"steps": it, "train_s": tt, "s_per_step": tt / it})
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
            G.close()
            del G
            torch.cuda.empty_cache()
    print(json.dumps({"config": "svm", "workload": "kernel SVM by projected gradient ascent (Exp. 6, 2D): "
                                                   "exp(-r) disk / exp(-r^2) wave labels, [-1.4,1.4]^2, 85/15 "
                                                   "split, lambda 1, beta 1, ACA tol 1e-8, leaf 64",
                      "rows": rows}), flush=True)


def bench_integral_equation(args):
    """Exp. 5: (I + w A~) sigma = f on the cell centres of uniform grids of
    20^3 ... 90^3 points in [-1,1]^3, 1/r, tol 1e-7, leaf 64, f = (I + w A~)
    sigma for a seeded sigma, GMRES to a relative residual of 1e-10 with the
    FP64 matvec (and, with --steps > 0, with the mixed one to 1e-6)."""
    import torch
    from paper_2203_14832_amd import nnca
    from paper_2203_14832_amd.workloads import nystrom_grid
    dev = torch.device("cuda:0")
    rows = []
    for na in (20, 30, 40, 50, 60, 70, 80, 90):
        p, w, sigma = nystrom_grid(na)
        t0 = time.perf_counter()
        H = nnca.H2Matrix(p, "inv_r", 1e-7, 64, device=dev)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        s = torch.tensor(sigma, device=dev)
        f = s + w * H.matvec(s, "fp64")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, rr = H.solve(f, 1.0, w, tol=1e-10, restart=50, max_iter=200)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        es = float(torch.linalg.norm(x - s) / torch.linalg.norm(s))
        row = {"n": int(p.shape[0]), "iters": it, "relres": rr, "eps_s": es, "assembly_s": ta, "solve_s": ts}
        f32 = s + w * H.matvec(s, "mixed")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xm, itm, rrm = H.solve(f32, 1.0, w, tol=1e-6, restart=50, max_iter=200, precision="mixed")
        torch.cuda.synchronize()
        row.update({"iters_mixed_1e-6": itm, "solve_s_mixed_1e-6": time.perf_counter() - t0,
                    "eps_s_mixed": float(torch.linalg.norm(xm - s) / torch.linalg.norm(s))})
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        H.close()
        del H
        torch.cuda.empty_cache()
    print(json.dumps({"config": "ie", "workload": "Nystrom (I + w A) sigma = f, 3D 1/r, uniform grid cell centres "
                                                  "in [-1,1]^3, tol 1e-7, leaf 64, GMRES(50) to 1e-10",
                      "rows": rows}), flush=True)


def probe(args):
    """For hardware-counter runs (rocprofv3 --pmc): a plain device-to-device
    copy of 256 MiB (known bytes read and written, to scale the byte
    counters) and `steps` mixed matvecs of the default workload."""
    import torch
    from paper_2203_14832_amd import nnca
    from paper_2203_14832_amd.workloads import workload
    dev = torch.device("cuda:0")
    a = torch.ones(32 << 20, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    p, x = workload("c2", n=args.n)
    n = p.shape[0]
    H = nnca.H2Matrix(p, "inv_r", 1e-6, 64, device=dev)
    X = torch.tensor(x[:, 0], device=dev).reshape(1, n).contiguous()
    Y = torch.empty_like(X)
    for _ in range(args.steps):
        H.matvec_raw(X, Y, 1, "mixed")
    torch.cuda.synchronize()
    print(json.dumps({"probe": "copy 268435456 bytes + mixed matvecs", "n": n, "steps": args.steps}), flush=True)


def bench_many_rhs(args):
    """64 right-hand sides on N=262144 points on the unit sphere (1/r, tol 1e-7):
    one block matvec (FP32 transverse pass on MFMA) against 64 one-column
    matvecs, both mixed precision."""
    import torch
    from paper_2203_14832_amd import nnca
    from paper_2203_14832_amd.workloads import CONFIGS, workload
    dev = torch.device("cuda:0")
    c = CONFIGS["c3"]
    p, x = workload("c3")
    n, R = p.shape[0], x.shape[1]
    t0 = time.perf_counter()
    H = nnca.H2Matrix(p, c["kernel"], c["tol"], c["leaf"], device=dev, max_rhs=R)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = H.info()
    X = torch.tensor(x.T.copy(), device=dev)           # (R, n): column-major n x R
    Yb = torch.empty_like(X)
    Yl = torch.empty_like(X)
    Y64 = torch.empty_like(X)
    H.matvec_raw(X, Y64, R, "fp64")
    for _ in range(args.warmup):
        H.matvec_raw(X, Yb, R, "mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        H.matvec_raw(X, Yb, R, "mixed")
    torch.cuda.synchronize()
    block_ms = (time.perf_counter() - t0) / args.steps * 1e3
    for col in range(R):
        H.matvec_raw(X[col:col + 1], Yl[col:col + 1], 1, "mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, args.steps // 4)
    for _ in range(reps):
        for col in range(R):
            H.matvec_raw(X[col:col + 1], Yl[col:col + 1], 1, "mixed")
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) / reps * 1e3
    # per-pass event timing of a few block matvecs: the transverse pass per
    # level and the near field, for the matrix-core roofline of the block
    H.profile(True)
    for _ in range(3):
        H.matvec_raw(X, Yb, R, "mixed")
    torch.cuda.synchronize()
    ps, lv, pm = H.profile_read()
    H.profile(False)
    kap = info["kappa"]
    fl = max(info["lmin"], kap - info["mixed_fp32_levels"] + 1)
    f32_levels = list(range(fl, kap + 1))
    m2l32_ms = float(pm[(ps == 2) & (lv >= fl)].sum() / 3)
    m2l64_ms = float(pm[(ps == 2) & (lv < fl)].sum() / 3)
    p2p_ms = float(pm[ps == 4].sum() / 3)
    f32_inter = sum(info["m2l_level"][l] for l in f32_levels)
    # one FMA per column and interaction; the mixed near field multiplies
    # x_hi and x_lo (two FMAs)
    m2l_flops = 2.0 * R * f32_inter
    p2p_flops = 4.0 * R * info["p2p_interactions"]
    roof = {"bound": "mfma", "kernel": "k_m2l_mfma<1/r> (FP32 kernel tiles x weight tiles, levels %s)" % f32_levels,
            "achieved": m2l_flops / (m2l32_ms * 1e-3) / 1e12, "peak": FP32_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": m2l_flops / (m2l32_ms * 1e-3) / FP32_MFMA_PEAK, "traffic": None,
            "ms_per_block": m2l32_ms, "flops_per_block": m2l_flops,
            "near_field": {"kernel": "k_p2p_mfma<1/r> (+ combine)", "ms_per_block": p2p_ms,
                           "achieved": p2p_flops / (p2p_ms * 1e-3) / 1e12,
                           "frac": p2p_flops / (p2p_ms * 1e-3) / FP32_MFMA_PEAK},
            "coarse_fp64_refined_m2l_ms_per_block": m2l64_ms,
            "pass_ms_per_block": {name: float(pm[ps == i].sum() / 3)
                                  for i, name in enumerate(["gather", "up", "m2l", "down", "p2p"])}}
    err_block = float((torch.linalg.norm(Yb - Y64, dim=1) / torch.linalg.norm(Y64, dim=1)).max())
    err_loop = float((torch.linalg.norm(Yl - Y64, dim=1) / torch.linalg.norm(Y64, dim=1)).max())
    inter = info["m2l_interactions"] + info["p2p_interactions"]
    out = {"metric": "matvec columns/s, 64 RHS block vs one-column loop", "value": R / (block_ms * 1e-3),
           "unit": "columns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": block_ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"3D 1/r, N={n} uniform on the unit sphere, leaf {c['leaf']}, tol {c['tol']}, "
                                  f"{R} RHS N(0,1), mixed precision", "n": n, "nrhs": R, "kappa": info["kappa"]},
           "loop_ms_per_64_columns": loop_ms, "block_speedup": loop_ms / block_ms,
           "err_block_vs_fp64_max": err_block, "err_loop_vs_fp64_max": err_loop, "build_seconds": build_s,
           "interactions_per_column": inter,
           "block_interaction_columns_per_s": inter * R / (block_ms * 1e-3), "roofline": roof}
    print(json.dumps(out), flush=True)


def bench_backward(args):
    """Gaussian kernel, N=200000 points of the two-component mixture (h=0.5,
    leaf 128, tol 1e-6): one step is the mixed forward y = A~ x plus the
    backward (A~^T g and dL/dh with the pivots frozen)."""
    import torch
    from paper_2203_14832_amd import nnca
    from paper_2203_14832_amd.workloads import CONFIGS, cotangent, workload
    dev = torch.device("cuda:0")
    c = CONFIGS["c4"]
    p, x = workload("c4")
    n = p.shape[0]
    g = cotangent("c4", n)
    t0 = time.perf_counter()
    H = nnca.H2Matrix(p, c["kernel"], c["tol"], c["leaf"], length_scale=c["h"], device=dev)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    X = torch.tensor(x[:, 0], device=dev)
    G = torch.tensor(g, device=dev)
    t0 = time.perf_counter()
    dx64, dh64 = H.backward(X, G, "fp64")          # first call factors K(I, J) of every ACA cell
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    y64 = H.matvec(X, "fp64")

    def step():
        y = H.matvec(X, "mixed")
        dx, dh = H.backward(X, G, "mixed")
        return y, dx, dh

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y, dx, dh = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    fwd = []
    for prec in ("mixed", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            H.matvec(X, prec)
        torch.cuda.synchronize()
        fwd.append((time.perf_counter() - t0) / args.steps * 1e3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        H.backward(X, G, "fp64")
    torch.cuda.synchronize()
    bwd64 = (time.perf_counter() - t0) / args.steps * 1e3
    relerr = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    out = {"metric": "forward+backward steps/s (Gaussian H2 matvec, x- and h-gradient)", "value": 1e3 / ms,
           "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"3D exp(-r^2/h^2), h={c['h']}, N={n} two-component Gaussian mixture, "
                                  f"leaf {c['leaf']}, tol {c['tol']}, 1 RHS, mixed precision passes", "n": n},
           "forward_ms_mixed": fwd[0], "forward_ms_fp64": fwd[1], "step_ms_fp64": fwd[1] + bwd64,
           "dldh_mixed": float(dh), "dldh_fp64": float(dh64),
           "dldh_rel_diff_mixed_vs_fp64": abs(float(dh) - float(dh64)) / abs(float(dh64)),
           "y_rel_err_mixed_vs_fp64": relerr(y, y64), "dx_rel_err_mixed_vs_fp64": relerr(dx, dx64),
           "backward_setup_seconds": setup_s, "build_seconds": build_s}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """32 independent 3D 1/r problems, N_b log-uniform in [1e4, 2e5] points
    uniform in [-1,1]^3 (leaf 64, tol 1e-6), 8 RHS each, mixed precision:
    the batch (one graph of merged launches, autotuned transverse-pass
    splits) against the 32 problems applied one after another."""
    import torch
    from paper_2203_14832_amd import nnca
    from paper_2203_14832_amd.workloads import batch_problem, batch_sizes
    dev = torch.device("cuda:0")
    sizes = batch_sizes()
    R = 8
    t0 = time.perf_counter()
    hs, xs = [], []
    for b, nb in enumerate(sizes):
        p, x = batch_problem(b, nb, R)
        hs.append(nnca.H2Matrix(p, "inv_r", 1e-6, 64, device=dev))
        xs.append(x)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    B = nnca.H2Batch(hs, graph=True, autotune=True)
    torch.cuda.synchronize()
    merge_s = time.perf_counter() - t0
    rows = B.rows
    X = torch.tensor(np.concatenate(xs, axis=0).T.copy(), device=dev)     # (R, rows)
    Y = torch.empty_like(X)
    t0 = time.perf_counter()
    B.matvec_raw(X, Y, R, "mixed")              # eager run, autotune, capture
    torch.cuda.synchronize()
    capture_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        B.matvec_raw(X, Y, R, "mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.matvec_raw(X, Y, R, "mixed")
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) / args.steps * 1e3
    Xs = [X[:, B.offsets[b]:B.offsets[b + 1]].contiguous() for b in range(len(hs))]
    Ys = [torch.empty_like(v) for v in Xs]
    Y64 = [torch.empty_like(v) for v in Xs]
    for h, xb, yb in zip(hs, Xs, Y64):
        h.matvec_raw(xb, yb, R, "fp64")

    def separate():
        for h, xb, yb in zip(hs, Xs, Ys):
            h.matvec_raw(xb, yb, R, "mixed")

    for _ in range(args.warmup):
        separate()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        separate()
    torch.cuda.synchronize()
    sep_ms = (time.perf_counter() - t0) / args.steps * 1e3
    err_b = max(float((torch.linalg.norm(Y[:, B.offsets[b]:B.offsets[b + 1]] - Y64[b], dim=1)
                       / torch.linalg.norm(Y64[b], dim=1)).max()) for b in range(len(hs)))
    err_s = max(float((torch.linalg.norm(Ys[b] - Y64[b], dim=1) / torch.linalg.norm(Y64[b], dim=1)).max())
                for b in range(len(hs)))
    out = {"metric": "batched matvec columns/s, 32 uneven problems x 8 RHS", "value": len(hs) * R / (batch_ms * 1e-3),
           "unit": "columns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": batch_ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(hs)} independent 3D 1/r problems, N_b log-uniform in [1e4, 2e5] "
                                  f"(sum {rows}), uniform in [-1,1]^3, leaf 64, tol 1e-6, {R} RHS each, mixed",
                      "rows": rows, "sizes": sizes},
           "separate_ms": sep_ms, "batch_speedup": sep_ms / batch_ms, "err_batch_vs_fp64_max": err_b,
           "err_separate_vs_fp64_max": err_s, "build_seconds": build_s, "merge_seconds": merge_s,
           "first_call_seconds": capture_s}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
