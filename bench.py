#!/usr/bin/env python3
"""Throughput of the batched DALM solver on one MI355X.

One step = one pass of the solver over one batch of synthetic instances
already resident in HBM: the per-instance penalties and constant term, the
iterations (z-, y-, w-steps fused in one MFMA GEMM launch per iteration, the
convergence test and active-set compaction), the output extraction and the
FP64 optimality certificate of every instance.  The dictionary's one-time
FP64 factorisation (the plan) is built before the timed region and reported
separately as ``plan_ms``.

Prints ONE JSON line on stdout; everything else goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense): HBM3E 8 TB/s; MFMA BF16 2.5 PFLOP/s, FP32 157.3 TFLOP/s.
# A split-BF16 product issues three BF16 MFMAs per algorithmic multiply-add
# (hi*hi + hi*lo + lo*hi), so its algorithmic flops run at a third of the peak.
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "split": 2500.0 / 3.0}
ELEM_BYTES = {"fp32": 4, "bf16": 2, "split": 4}


def dalm_work_model(m, n_dict, structure):
    """Algorithmic work of one DALM iteration of one instance (the method's
    own: two products with the dictionary and the two triangular solves with
    the Cholesky factor of the y-step, Algorithm 2), and the matrix bytes one
    batched iteration reads once:
        flops   F = 4 m n_B + 2 m^2
        matrix  2 m n_B s (the dictionary twice, s bytes per element in the
                product's arithmetic) + 4 m^2 (the FP32 factor, both solves)
        state   4 (4 n + 5 m + 2 n_B) bytes per instance (FP32 state, fused
                updates; n = n_B + m for the cross-and-bouquet form)."""
    n = n_dict + (m if structure == "cab" else 0)
    return {"flops": 4.0 * m * n_dict + 2.0 * m * m,
            "matrix": lambda s: 2.0 * m * n_dict * s + 4.0 * m * m,
            "state": 4.0 * (4 * n + 5 * m + 2 * n_dict)}


def dalm_structured_model(m, n_dict):
    """The same for the structured (Woodbury) y-step of the cross-and-bouquet
    form with n_B < m: B and B^T once each and the n_B x n_B inverse of
    K = I + B^T B, all in the product's arithmetic:
        flops   F = 4 m n_B + 2 n_B^2
        matrix  (2 m n_B + n_B^2) s."""
    return {"flops": 4.0 * m * n_dict + 2.0 * n_dict * n_dict,
            "matrix": lambda s: (2.0 * m * n_dict + 1.0 * n_dict * n_dict) * s}


def dalm_roofline(m, n_dict, structure, agg, kern_s, launches):
    """Roofline of the DALM iteration over a timed run: instance-iterations
    by arithmetic (agg cols_*), iterations of the slowest instance (one
    batched iteration each: the matrices are read once per iteration), and
    the kernel time from HIP events.  The bound is the larger of the MFMA
    time (each arithmetic at its peak) and the HBM time."""
    wm = dalm_work_model(m, n_dict, structure)
    cols = {"fp32": agg["cols_fp32"], "bf16": agg["cols_bf16"], "split": agg["cols_split"]}
    tot_cols = max(sum(cols.values()), 1.0)
    # instance-iterations of the structured form (FP32 or BF16 tiles only):
    # counted at its own flops and matrix bytes
    c_st = min(agg.get("cols_structured", 0.0), cols["fp32"] + cols["bf16"])
    f_st = c_st / tot_cols
    ws = dalm_structured_model(m, n_dict)
    flops = {k: wm["flops"] * c for k, c in cols.items()}
    if c_st > 0:
        # split the structured share between FP32 and BF16 in proportion
        nb = cols["fp32"] + cols["bf16"]
        for k in ("fp32", "bf16"):
            share = c_st * cols[k] / nb
            flops[k] += (ws["flops"] - wm["flops"]) * share
    s_avg = sum(ELEM_BYTES[k] * c for k, c in cols.items()) / tot_cols
    bytes_total = (agg["iterations"] * ((1.0 - f_st) * wm["matrix"](s_avg) + f_st * ws["matrix"](s_avg))
                   + wm["state"] * tot_cols)
    tot_flops = sum(flops.values())
    t_mfma = sum(flops[k] / (PEAK_TFLOPS[k] * 1e12) for k in flops)
    t_hbm = bytes_total / (PEAK_HBM_GBS * 1e9)
    nl = max(launches, 1.0)
    if t_mfma >= t_hbm:
        eff_peak = tot_flops / t_mfma / 1e12
        achieved = tot_flops / kern_s / 1e12 if kern_s > 0 else 0.0
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": round(eff_peak, 1),
                "unit": "TFLOP/s", "frac": round(achieved / eff_peak, 4)}
    else:
        achieved = bytes_total / kern_s / 1e9 if kern_s > 0 else 0.0
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4)}
    roof.update({"avg_launch_us": round(1e6 * kern_s / nl, 3), "launches_timed": int(launches),
                 "algorithmic_flops_per_launch": round(tot_flops / nl),
                 "algorithmic_bytes_per_launch": round(bytes_total / nl),
                 "flops_per_instance_iteration": wm["flops"],
                 "state_bytes_per_instance": wm["state"],
                 "t_mfma_s": t_mfma, "t_hbm_s": t_hbm})
    return roof, tot_flops, bytes_total

WORKLOADS = {
    # B 1200 x 700 (100 classes x 7), A = [B, I]; 512 test vectors, 30 % corrupted
    "cab-1200x700-n512": dict(m=1200, classes=100, per_class=7, N=512, frac=0.3, cfg=3, precision="bf16_refine"),
    # B 4800 x 2100 (300 classes x 7); 2048 test vectors, corruption U[0, 0.5] each
    "cab-4800x2100-n2048": dict(m=4800, classes=300, per_class=7, N=2048, frac="uneven", cfg=4, precision="bf16_refine"),
}
DEFAULT_WORKLOAD = "cab-1200x700-n512"
# The paper's noise-free synthetic benchmark (Sec. VI-A): m = 800, Gaussian A with
# unit columns, x0 d-sparse with U[-10, 10] nonzeros, b = A x0.  The paper averages
# 20 trials; here they are 20 planted x0 solved as one batch against one A.
E1_WORKLOADS = {
    "e1-800x1000-d100": dict(m=800, n=1000, k=100),
    "e1-800x1000-d200": dict(m=800, n=1000, k=200),
    "e1-800x2000-d100": dict(m=800, n=2000, k=100),
}

# The l1 problem of the alignment step (Sec. II-B, Sec. VI-C): per instance its own
# B = [A_i, -J] of 7 training images and a similarity transform's 4 Jacobian
# columns, on a 40 x 30 grid (1200 x 11); 1000 (subject, query) instances with a
# 10 % occluding block.  Tolerances as in the paper's alignment table.
ALIGN_WORKLOADS = {
    "align-1200x11-n1000": dict(h=40, wd=30, n_img=7, N=1000, cfg=6, tols=(1e-2, 1e-3, 1e-4), tol=1e-3),
}

# The (QP_lambda) compressive-sensing sweep: Gaussian 2000 x 8000 with unit
# columns, 200 +-1 spikes, noise 0.01, lambda = 1e-3, 64 instances sharing A;
# batched against one instance per launch.
QP_WORKLOADS = {"qp-2000x8000-n64": dict(tol=3e-6, max_iter=30000, plain=2)}
# Plain single-instance (P1): Gaussian 200 x 1000 with unit columns, 20 N(0,1)
# nonzeros at random positions, b = A x0, one instance per solve, FP32,
# stopping at relative change 1e-6 (Sec. VI-A shape); 8 planted x0 share A.
PLAIN_WORKLOADS = {"plain-200x1000": dict(m=200, n=1000, k=20, N=8, tol=1e-6, max_iter=20000)}
# The differentiable unrolled DALM: the 1200 x 700 cross-and-bouquet
# dictionary, 256 corrupted test vectors, 50 iterations, checkpoints every 10,
# forward and backward to b and B.
UNROLLED_WORKLOADS = {"unrolled-1200x700-n256": dict(N=256, iters=50, every=10, cfg=5)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS) + sorted(E1_WORKLOADS) + sorted(ALIGN_WORKLOADS)
                    + sorted(QP_WORKLOADS) + sorted(UNROLLED_WORKLOADS) + sorted(PLAIN_WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16_refine", "bf16x3"],
                    help="default: bf16_refine for the cross-and-bouquet workloads, fp32 for e1-*")
    ap.add_argument("--form", default="auto", choices=["auto", "dense", "structured"],
                    help="DALM iteration form of the cross-and-bouquet workloads (include/l1_alm.h)")
    ap.add_argument("--method", default="dalm", choices=["dalm", "palm", "adm", "dalm_cg1"],
                    help="e1-* workloads only (the cross-and-bouquet benchmark is DALM)")
    ap.add_argument("--e1-instances", type=int, default=20)
    ap.add_argument("--tol", type=float, default=4e-6)
    ap.add_argument("--max-iter", type=int, default=40000)
    ap.add_argument("--check-instances", type=int, default=4,
                    help="instances whose x is compared with the exact LP optimum")
    ap.add_argument("--plain-instances", type=int, default=8,
                    help="instances solved one per launch with FP32 for the plain-path figure")
    ap.add_argument("--cpu-instances", type=int, default=8,
                    help="instances the FP64 CPU oracle solves for the cpu_baseline figure")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="run the split-K autotuner on the plan before timing and record it in the cache")
    ap.add_argument("--tune-out", default=None, help="cache file written by --tune (default: the package's)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration under rocprofv3)")
    return ap.parse_args()


def traffic_record(src_hash, name="dalm_iteration_traffic.json"):
    """HBM bytes per launch of a kernel from the committed PMC summary, if
    it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != src_hash:
        return None
    return rec


def kernel_source_hash(files=("iter.hip", "internal.h", "tail.hip", "tail.h", "dalm_test.h")):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1007_3753_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); instances are "
              "independent, so N GPUs would each run this same per-GPU workload.", file=sys.stderr)
        sys.exit(2)
    if args.workload in E1_WORKLOADS:
        return e1_main(args)
    if args.workload in ALIGN_WORKLOADS:
        return align_main(args)
    if args.workload in QP_WORKLOADS:
        return qp_main(args)
    if args.workload in UNROLLED_WORKLOADS:
        return unrolled_main(args)
    if args.workload in PLAIN_WORKLOADS:
        return plain_main(args)
    if args.precision is None:
        args.precision = WORKLOADS[args.workload]["precision"]
    if args.method != "dalm":
        print("the cross-and-bouquet benchmark runs DALM", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1007_3753_amd import Plan
    from workloads import cab_problem

    wl = WORKLOADS[args.workload]
    t0 = time.time()
    P = cab_problem(m=wl["m"], classes=wl["classes"], per_class=wl["per_class"], N=wl["N"],
                    frac=wl["frac"], cfg=wl["cfg"])
    log(f"workload {args.workload}: B {P.A.shape}, N {P.N}, generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    A = torch.as_tensor(P.A, device=dev)
    b = torch.as_tensor(P.b, device=dev)
    m, nd, N = P.m, P.n_dict, P.N
    n_full = nd + m
    plan = Plan(A, structure="cab", precision=args.precision, max_batch=N, time_kernels=True,
                iteration_form=args.form)
    plan_ms = plan.last_stats()["plan_ms"]
    log(f"plan ({args.precision}) built in {plan_ms:.1f} ms")
    # launch shape: the split-K table from the autotuner (run here with
    # --tune, before the timed region), else the cached one, else the heuristic
    from paper_1007_3753_amd import tuning
    if args.tune:
        t0 = time.perf_counter()
        table = tuning.tune(plan, path=args.tune_out or tuning.CACHE)
        ks_info = {"source": "tuned in this run", "table": table,
                   "tune_s": round(time.perf_counter() - t0, 2)}
    else:
        table = tuning.apply(plan)
        ks_info = {"source": "cache" if table is not None else "heuristic", "table": table}
    log(f"split-K table: {ks_info}")

    def step():
        r = plan.solve(b, tol=args.tol, max_iter=args.max_iter)
        rep = plan.kkt(b, r.x, e=r.e, y=r.y)
        return r, rep

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    agg = dict(timed_ms=0.0, timed_launches=0.0, launch_fp32=0.0, launch_bf16=0.0, launch_split=0.0,
               cols_fp32=0.0, cols_bf16=0.0, cols_split=0.0, iterations=0.0, cols_structured=0.0)
    t_start = time.perf_counter()
    for i in range(args.steps):
        r, rep = step()
        st = plan.last_stats()
        for k in agg:
            agg[k] += st[k]
        log(f"step {i + 1}/{args.steps}: solve {st['solve_ms']:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    value = N / (ms_per_step / 1e3)
    iters = r.iters.cpu().numpy()
    status = r.status.cpu().numpy()
    rep = rep.cpu().numpy()
    log(f"{args.steps} steps: {ms_per_step:.2f} ms/step -> {value:.1f} solves/s; iterations "
        f"mean {iters.mean():.0f} max {iters.max()}; status counts {np.bincount(status, minlength=4).tolist()}")

    # ---- roofline of the iteration kernel (gemm_kernel<EPI_DALM>) -----------
    kern_s = agg["timed_ms"] / 1e3
    nl = max(agg["timed_launches"], 1.0)
    roof, tot_flops, bytes_total = dalm_roofline(m, nd, "cab", agg, kern_s, nl)
    trec = traffic_record(kernel_source_hash())
    roof["traffic"] = None if trec is None else trec.get("hbm_bytes_per_launch_at_workload", {}).get(args.workload)
    roof.update({
        "kernel": "DALM iteration: gemm_kernel<EPI_DALM> (+ its split-K gemm_kernel<EPI_PARTIAL> "
                  "launch when few column tiles are active, + 1/16 of a compaction; two "
                  "gemm_kernel<EPI_DALM> launches in the structured form), or one "
                  "iteration of dalm_tail_kernel once few instances are left",
        "structured_share": round(agg["cols_structured"] / max(agg["cols_fp32"] + agg["cols_bf16"]
                                                                + agg["cols_split"], 1.0), 3),
        "kernel_share_of_step": round(agg["timed_ms"] / (ms_per_step * args.steps), 3),
    })
    log(f"iteration kernel: {nl:.0f} launches, avg {1e6 * kern_s / nl:.2f} us; "
        f"{tot_flops / kern_s / 1e12:.1f} algorithmic TFLOP/s, {bytes_total / kern_s / 1e9:.0f} GB/s "
        f"({roof['bound']}-bound, {100 * roof['frac']:.1f} % of the roofline)")

    out = {
        "metric": "solves/sec at rel. err <=1e-4 vs FP64 oracle (batched DALM, cross-and-bouquet)",
        "value": round(value, 2), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16_refine": "bf16+split-bf16 (f32 accumulate)",
                  "bf16x3": "split-bf16 (f32 accumulate)"}[args.precision],
        "data": "synthetic (seeded cross-and-bouquet stand-in for face images; no dataset)",
        "config": {"workload": args.workload, "m": m, "n_dict": nd, "n_full": n_full, "N": N,
                   "problem": "P1", "structure": "cab", "method": "dalm",
                   "precision": args.precision, "tol": args.tol, "max_iter": args.max_iter,
                   "iteration_form": args.form},
        "plan_ms": round(plan_ms, 2),
        "ksplit": ks_info,
        "iterations": {"mean": float(iters.mean()), "max": int(iters.max())},
        "status_counts": np.bincount(status, minlength=4).tolist(),
        "kkt_max": {"primal": float(rep[:, 0].max()), "dual_inf": float(rep[:, 1].max()),
                    "gap": float(rep[:, 3].max())},
        "roofline": roof,
    }

    # ---- accuracy -------------------------------------------------------------
    # every instance against its planted solution (at this corruption level the
    # l1 optimum is the planted one: checked below by the exact LP on samples)
    X = r.x.cpu().numpy().astype(np.float64)
    err_pl = np.linalg.norm(X - P.x0, axis=0) / np.linalg.norm(P.x0.astype(np.float64), axis=0)
    out["rel_err_vs_planted"] = {"instances": int(N), "max": float(err_pl.max()),
                                 "p99": float(np.quantile(err_pl, 0.99)),
                                 "median": float(np.median(err_pl))}
    out["rel_err_vs_planted"]["within_1e-4"] = int((err_pl <= 1e-4).sum())
    out["rel_err_vs_planted"]["within_1e-3"] = int((err_pl <= 1e-3).sum())
    log(f"rel. err of x vs planted solution, all {N} instances: max {err_pl.max():.2e}; "
        f"{int((err_pl <= 1e-4).sum())} within 1e-4, {int((err_pl <= 1e-3).sum())} within 1e-3")
    gpath = os.path.join(ROOT, "tests", "golden", "c4_reference.npz")
    if args.workload == "cab-4800x2100-n2048" and os.path.exists(gpath):
        # the exact LP optima (oracle, certified) of the golden sample
        g = np.load(gpath)
        ge = [float(np.linalg.norm(X[:, j] - g["w"][:nd, k]) / np.linalg.norm(g["w"][:nd, k]))
              for k, j in enumerate(g["idx"])]
        out["rel_err_vs_lp"] = {"instances": [int(j) for j in g["idx"]], "max": max(ge), "all": ge,
                                "corruption": [round(float(f), 3) for f in g["frac"]]}
        log(f"rel. err of x vs the LP optima of the golden sample: max {max(ge):.2e}")
    # the recognition criterion of the face experiments (Sec. VI-B) on the
    # solved batch: every test vector is drawn from one subject's columns
    from paper_1007_3753_amd import classify
    ptr = np.arange(0, nd + 1, P.per_class)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, label, score = classify(r.x, ptr)
    torch.cuda.synchronize()
    cls_ms = 1e3 * (time.perf_counter() - t)
    rate = float((label.cpu().numpy() == P.labels).mean())
    out["recognition"] = {"rate": rate, "ms": round(cls_ms, 3), "subjects": int(len(ptr) - 1),
                          "score_median": float(score.median())}
    log(f"recognition (Sec. VI-B criterion): {100 * rate:.1f} % of {N} in {cls_ms:.2f} ms")
    # the residual rule of the classifier the paper builds on, on the same batch
    from paper_1007_3753_amd import class_residuals
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, rlabel = class_residuals(A, r.x, b, ptr, e=r.e)
    torch.cuda.synchronize()
    res_ms = 1e3 * (time.perf_counter() - t)
    rrate = float((rlabel.cpu().numpy() == P.labels).mean())
    out["recognition"]["residual_rule"] = {"rate": rrate, "ms": round(res_ms, 3)}
    log(f"recognition (residual rule): {100 * rrate:.1f} % of {N} in {res_ms:.2f} ms")
    if not args.no_check and args.check_instances > 0 and m <= 2000:
        from oracle import p1_lp, full_matrix
        Af = full_matrix(P.A, "cab")
        idx = np.unique(np.linspace(0, N - 1, args.check_instances).astype(int))
        errs, lp_vs_planted = [], []
        for j in idx:
            w_lp, _ = p1_lp(Af, P.b[:, j])
            errs.append(float(np.linalg.norm(X[:, j] - w_lp[:nd]) / np.linalg.norm(w_lp[:nd])))
            lp_vs_planted.append(float(np.linalg.norm(w_lp[:nd] - P.x0[:, j]) / np.linalg.norm(w_lp[:nd])))
        out["rel_err_vs_lp"] = {"instances": idx.tolist(), "max": max(errs), "all": errs,
                                "lp_vs_planted_max": max(lp_vs_planted)}
        log(f"rel. err of x vs LP optimum on {len(idx)} instances: max {max(errs):.2e} "
            f"(LP vs planted {max(lp_vs_planted):.1e})")

    # ---- plain path: one instance per launch, FP32 ----------------------------
    if not args.no_plain and args.plain_instances > 0:
        plain = Plan(A, structure="cab", precision="fp32", max_batch=1)
        k = min(args.plain_instances, N)
        plain.solve(b[:, :1], tol=args.tol, max_iter=args.max_iter)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for j in range(k):
            plain.solve(b[:, j:j + 1], tol=args.tol, max_iter=args.max_iter)
        torch.cuda.synchronize()
        ps = k / (time.perf_counter() - t)
        out["plain"] = {"solves_per_s": round(ps, 3), "instances": k, "precision": "fp32",
                        "batched_over_plain": round(value / ps, 1)}
        log(f"plain one-instance-per-launch FP32: {ps:.2f} solves/s -> batched is {value / ps:.0f}x")
        plain.close()

    # ---- CPU baseline: the FP64 oracle on this host's cores ------------------
    if not args.no_cpu_baseline and args.cpu_instances > 0:
        from oracle import dalm as oracle_dalm, kkt_report, full_matrix
        threads = _threads()
        k = min(args.cpu_instances, N)
        if m <= 2000:
            # like for like: the first k instances solved to the same tolerance
            t = time.perf_counter()
            o = oracle_dalm(P.A, P.b[:, :k], structure="cab", tol=args.tol, max_iter=args.max_iter)
            dt = time.perf_counter() - t
            out["cpu_baseline"] = {
                "value": round(k / dt, 5), "unit": "solves/s", "cores": int(threads), "kind": "oracle",
                "sample": f"first {k} of the {N} instances, FP64 NumPy/SciPy Algorithm 2 with a "
                          f"Cholesky y-step, same tol ({args.tol:g}); {dt:.1f} s, iterations "
                          f"{o.iters.tolist()}; the rate extrapolates to the batch"}
            log(f"CPU oracle: {k} instances in {dt:.1f} s on {threads} threads")
            # ground truth (not timed for ranking): the exact LP optimum of
            # instance 0 (oracle, simplex/interior point in FP64) with its FP64
            # certificate, and the GPU result against it
            from oracle import p1_lp
            t = time.perf_counter()
            Af = full_matrix(P.A, "cab")
            wg, yg = p1_lp(Af, P.b[:, 0])
            gdt = time.perf_counter() - t
            rep0 = kkt_report(Af, P.b[:, 0], wg, yg)
            xg = wg[:nd]
            out["cpu_ground_truth"] = {
                "instance": 0, "solver": "exact LP (oracle.p1_lp)", "s": round(gdt, 2),
                "kkt": rep0, "gpu_rel_err": float(np.linalg.norm(X[:, 0] - xg) / np.linalg.norm(xg))}
            log(f"CPU ground truth (instance 0, exact LP): {gdt:.1f} s, KKT {rep0}; "
                f"GPU rel. err {out['cpu_ground_truth']['gpu_rel_err']:.2e}")
        else:
            # a solve of this size takes minutes on the host: 100 iterations of
            # instance 0, extrapolated to the batch's mean iteration count
            K = 100
            t = time.perf_counter()
            oracle_dalm(P.A, P.b[:, :1], structure="cab", fixed_iters=K)
            dt = time.perf_counter() - t
            per_solve = dt / K * float(iters.mean())
            out["cpu_baseline"] = {
                "value": round(1.0 / per_solve, 6), "unit": "solves/s", "cores": int(threads), "kind": "oracle",
                "sample": f"{K} iterations of instance 0 ({dt:.1f} s, FP64 Algorithm 2 with a Cholesky "
                          f"y-step), extrapolated to the batch's mean iteration count "
                          f"({float(iters.mean()):.0f})"}
            log(f"CPU oracle: {K} iterations in {dt:.1f} s -> {per_solve:.0f} s per solve (extrapolated)")

    plan.close()
    if args.copy_calibration:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = x.numel() * 4

    print(json.dumps(out), flush=True)


def plain_main(args):
    """One instance per solve: the plain path of (P1) by DALM or PALM in FP32
    on the 200 x 1000 Gaussian workload.  A step solves the 8 instances one
    after another (each to relative change 1e-6); accuracy against the exact
    LP optimum of each instance; the FP64 oracle on the same instances is the
    CPU baseline."""
    import numpy as np
    import torch

    from paper_1007_3753_amd import Plan
    from workloads import dense_p1
    from oracle import p1_lp

    wl = PLAIN_WORKLOADS[args.workload]
    method = args.method if args.method in ("dalm", "palm") else "dalm"
    P = dense_p1(m=wl["m"], n=wl["n"], k=wl["k"], N=wl["N"])
    dev = torch.device("cuda:0")
    A = torch.as_tensor(P.A, device=dev)
    b = torch.as_tensor(P.b, device=dev)
    N, m, n = wl["N"], wl["m"], wl["n"]
    plan = Plan(A, method=method, precision="fp32", max_batch=1, time_kernels=True)
    plan_ms = plan.last_stats()["plan_ms"]

    def step():
        out = []
        for j in range(N):
            out.append(plan.solve(b[:, j:j + 1], tol=wl["tol"], max_iter=wl["max_iter"]))
        return out

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    kern_ms, iters_tot, launches = 0.0, 0, 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        rs = step()
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = N / (ms_per_step / 1e3)
    # per-iteration kernel time of the last instance's solve (HIP events)
    st = plan.last_stats()
    X = np.stack([r.x.cpu().numpy()[:, 0].astype(np.float64) for r in rs], axis=1)
    its = [int(r.iters[0]) for r in rs]
    sts = [int(r.status[0]) for r in rs]
    errs = []
    for j in range(N):
        x_lp, _ = p1_lp(P.A, P.b[:, j])
        errs.append(float(np.linalg.norm(X[:, j] - x_lp) / np.linalg.norm(x_lp)))
    out = {
        "metric": f"solves/sec at rel. err <=1e-4 vs FP64 oracle (plain single-instance {method.upper()})",
        "value": round(value, 2), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (the paper's noise-free Gaussian recipe with N(0,1) nonzeros, seeded)",
        "config": {"workload": args.workload, "m": m, "n": n, "d": wl["k"], "N": 1, "instances_per_step": N,
                   "problem": "P1", "structure": "dense", "method": method, "precision": "fp32",
                   "tol": wl["tol"]},
        "plan_ms": round(plan_ms, 2),
        "iterations": its, "status": sts,
        "rel_err_vs_lp": {"max": max(errs), "all": errs},
    }
    if method == "dalm" and st["timed_launches"] > 0:
        # HBM roofline of the iteration launch (N = 1): the method's own bytes,
        # the dictionary twice and the FP32 factor (both solves) plus the state
        wm = dalm_work_model(m, n, "dense")
        per_launch = wm["matrix"](4) + wm["state"]
        us = 1e3 * st["timed_ms"] / st["timed_launches"]
        ach = per_launch / (us * 1e-6) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(ach / PEAK_HBM_GBS, 4), "avg_launch_us": round(us, 3),
                           "launches_timed": int(st["timed_launches"]),
                           "algorithmic_bytes_per_launch": round(per_launch), "traffic": None,
                           "kernel": "DALM iteration: gemm_kernel<EPI_DALM> of one instance (with its split-K "
                                     "part), HIP events around the blocks of the last solve"}
    elif method == "palm":
        # wall clock per FISTA step of the last solve: the Gram matrix (n x n
        # FP32) once + per instance n * 24 bytes
        inner = max(st["inner_iterations"], 1.0)
        us = 1e3 * st["solve_ms"] / inner
        per_launch = 4.0 * n * n + 24.0 * n
        ach = per_launch / (us * 1e-6) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(ach / PEAK_HBM_GBS, 4), "avg_launch_us": round(us, 3),
                           "launches_timed": int(inner), "algorithmic_bytes_per_launch": round(per_launch),
                           "traffic": None,
                           "kernel": "PALM FISTA step: gemm_kernel<EPI_FISTA> with the Gram matrix, wall clock of "
                                     "the last solve over its FISTA launches (e-step and multiplier launches included)"}
    if not args.no_cpu_baseline:
        from oracle import dalm as oracle_dalm, palm as oracle_palm
        t = time.perf_counter()
        if method == "dalm":
            o = oracle_dalm(P.A, P.b, tol=wl["tol"], max_iter=wl["max_iter"])
        else:
            o = oracle_palm(P.A, P.b, tol=wl["tol"], max_iter=wl["max_iter"])
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(N / dt, 3), "unit": "solves/s", "cores": int(_threads()),
                               "kind": "oracle",
                               "sample": f"the same {N} instances, FP64 NumPy/SciPy {method.upper()} to the same "
                                         f"tolerance, {dt:.2f} s"}
        log(f"CPU oracle: {N} instances in {dt:.2f} s")
    plan.close()
    log(f"{method} plain: {value:.1f} solves/s, rel. err vs LP max {max(errs):.2e}, iterations {its}")
    print(json.dumps(out), flush=True)


def e1_main(args):
    """Relative error of x against the planted x0 as a function of GPU time
    (the paper's Fig. on synthetic data, Sec. VI-A) for one method, and the
    time to a mean relative error of 1e-5.  Each point of the curve is a
    fixed-count solve of the whole batch (median of ``--steps`` runs)."""
    import numpy as np
    import torch

    from paper_1007_3753_amd import Plan
    from workloads import dense_p1

    prec = args.precision or "fp32"
    wl = E1_WORKLOADS[args.workload]
    N = args.e1_instances
    P = dense_p1(m=wl["m"], n=wl["n"], k=wl["k"], N=N, cfg=5, values="uniform10")
    dev = torch.device("cuda:0")
    A = torch.as_tensor(P.A, device=dev)
    b = torch.as_tensor(P.b, device=dev)
    X0 = P.x0.astype(np.float64)
    nx0 = np.linalg.norm(X0, axis=0)
    # ADM: PALM with one FISTA step per outer step (the inexact form the paper compares with, Sec. V-A)
    inner = 1 if args.method == "adm" else 100
    plan = Plan(A, structure="dense", method={"adm": "palm"}.get(args.method, args.method), precision=prec,
                max_batch=N, max_inner=inner, time_kernels=True)
    plan_ms = plan.last_stats()["plan_ms"]
    ks = {"dalm": [5, 10, 20, 30, 50, 70, 100, 150, 200, 300, 500, 1000, 2000],
          "dalm_cg1": [5, 10, 20, 30, 50, 70, 100, 150, 200, 300, 500, 1000, 2000],
          "palm": [1, 2, 3, 5, 7, 10, 15, 20, 30, 50, 70, 100, 150, 200, 300, 500],
          "adm": [10, 20, 50, 70, 100, 150, 200, 300, 500, 700, 1000, 2000, 5000]}[args.method]
    target = 1e-5
    plan.solve(b, max_iter=-ks[0])
    torch.cuda.synchronize()
    curve, hit, agg = [], None, None
    for K in ks:
        for _ in range(args.warmup):
            plan.solve(b, max_iter=-K)
        times = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = plan.solve(b, max_iter=-K)
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t))
        err = np.linalg.norm(r.x.cpu().numpy().astype(np.float64) - X0, axis=0) / nx0
        ms = float(np.median(times))
        curve.append([K, round(ms, 4), float(err.mean()), float(err.max())])
        log(f"{args.method} {prec} {K:5d} iterations: {ms:9.3f} ms  mean rel. err {err.mean():.2e}")
        if hit is None and err.mean() <= target:
            hit = (K, ms)
            agg = plan.last_stats()
        if err.mean() <= 1e-6 or (hit is not None and len(curve) > 1 and err.mean() > 0.5 * curve[-2][2]):
            break   # at the arithmetic's floor
    # a converged solve of the batch (stop on the relative change, 1e-6)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rc = plan.solve(b, tol=1e-6, max_iter=20000)
    torch.cuda.synchronize()
    conv_ms = 1e3 * (time.perf_counter() - t)
    errc = np.linalg.norm(rc.x.cpu().numpy().astype(np.float64) - X0, axis=0) / nx0
    out = {
        "metric": f"ms to mean rel. err <= 1e-5 vs planted x0 ({N} instances, batched {args.method.upper()})",
        "value": round(hit[1], 4) if hit else None, "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(hit[1], 4) if hit else None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16_refine": "bf16+split-bf16 (f32 accumulate)",
                  "bf16x3": "split-bf16 (f32 accumulate)"}[prec],
        "data": "synthetic (the paper's noise-free Gaussian recipe, seeded)",
        "config": {"workload": args.workload, "m": wl["m"], "n": wl["n"], "d": wl["k"], "N": N,
                   "problem": "P1", "structure": "dense", "method": args.method, "precision": prec},
        "plan_ms": round(plan_ms, 2),
        "iterations_to_target": hit[0] if hit else None,
        "curve": {"columns": ["iterations", "ms", "mean_rel_err", "max_rel_err"], "points": curve},
        "converged": {"tol": 1e-6, "ms": round(conv_ms, 3), "iterations_max": int(rc.iters.max()),
                      "mean_rel_err": float(errc.mean()), "max_rel_err": float(errc.max()),
                      "status_counts": np.bincount(rc.status.cpu().numpy(), minlength=4).tolist()},
    }
    n = wl["n"]
    if args.method == "dalm" and agg is not None and agg["timed_launches"] > 0:
        # HIP events around the iteration launches; per launch the operator
        # (n x n FP32) once + per instance n * (4 + 24) bytes
        kern_s = agg["timed_ms"] / 1e3
        nl = agg["timed_launches"]
        bytes_total = nl * n * n * 4 + n * N * nl * 28
        what = "DALM iteration: gemm_kernel<EPI_DALM> (+ split-K part), HIP events"
    elif args.method == "dalm_cg1" and hit is not None:
        # wall clock of the fixed-count solve: per iteration A is read twice
        # (A u and A^T g, FP32) and per instance the model of the three
        # elementwise launches, n (36) + m (28) bytes
        kern_s = hit[1] / 1e3
        nl = hit[0]
        m_ = wl["m"]
        bytes_total = nl * (8 * m_ * n + N * (36 * n + 28 * m_))
        what = ("DALM with one CG step: two FP32 products (A u, A^T g) and three elementwise launches per "
                "iteration, wall clock of the whole solve")
    elif args.method in ("palm", "adm") and hit is not None:
        # wall clock of the fixed-count solve (no per-launch events on this
        # path): K outer steps of `inner` FISTA steps, each the Gram matrix
        # (n x n FP32) once + per instance n * 24 bytes
        kern_s = hit[1] / 1e3
        nl = hit[0] * inner
        bytes_total = nl * n * n * 4 + n * N * nl * 24
        what = (f"PALM FISTA step: gemm_kernel<EPI_FISTA>, wall clock of the whole solve "
                f"({inner} FISTA step(s) per outer step, with the outer steps' e-step, A x and A^T c)")
    else:
        kern_s = 0.0
    if kern_s > 0:
        achieved = bytes_total / kern_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                           "kernel": what, "avg_launch_us": round(1e6 * kern_s / nl, 3),
                           "launches_timed": int(nl)}
    else:
        out["roofline"] = None
    if not args.no_cpu_baseline and hit is not None:
        from oracle import dalm as oracle_dalm, palm as oracle_palm
        t = time.perf_counter()
        if args.method == "dalm":
            oracle_dalm(P.A, P.b[:, :1], structure="dense", fixed_iters=hit[0])
        elif args.method == "dalm_cg1":
            oracle_dalm(P.A, P.b[:, :1], structure="dense", fixed_iters=hit[0], y_step="cg1")
        else:
            oracle_palm(P.A, P.b[:, :1], structure="dense", fixed_outer=hit[0], fixed_inner=inner)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(1e3 * dt, 2), "unit": "ms", "cores": os.cpu_count(),
                               "kind": "oracle",
                               "sample": f"instance 0 alone, FP64, the same {hit[0]} iterations"}
    print(json.dumps(out), flush=True)


def align_main(args):
    """Alignment l1 problems solved per second: the whole batch, each instance
    with its own dictionary, solved to the relative-change tolerance in one
    launch of the alignment kernel (timed with HIP events on its stream)."""
    import numpy as np
    import torch

    from paper_1007_3753_amd import align
    from workloads import align_problem

    wl = ALIGN_WORKLOADS[args.workload]
    t0 = time.time()
    P = align_problem(N=wl["N"], h=wl["h"], wd=wl["wd"], n_img=wl["n_img"], cfg=wl["cfg"])
    N, m, k = P.B.shape
    log(f"workload {args.workload}: B_j {m} x {k}, N {N}, generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    # the library's layout, made once: each B_j column-major and b column-major
    # (views whose transposes are contiguous, so the binding copies nothing)
    B = torch.as_tensor(np.ascontiguousarray(P.B.transpose(0, 2, 1)), device=dev).transpose(1, 2)
    b = torch.as_tensor(np.ascontiguousarray(P.b.T), device=dev).t()
    w0 = P.w0.astype(np.float64)
    per_tol = {}
    for tol in wl["tols"]:
        for _ in range(max(1, args.warmup)):
            align(B, b, tol=tol, max_iter=1000)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t = time.perf_counter()
        for e0, e1 in ev:
            e0.record()
            w, e, it, st = align(B, b, tol=tol, max_iter=1000)
            e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / args.steps
        ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
        wn = w.cpu().numpy().astype(np.float64)
        err = np.linalg.norm(wn - w0, axis=0) / np.linalg.norm(w0, axis=0)
        its = it.cpu().numpy()
        per_tol[tol] = dict(ms=ms, wall_ms=1e3 * wall, iters_mean=float(its.mean()), iters_max=int(its.max()),
                            iters_total=int(its.sum()), err_mean=float(err.mean()), err_max=float(err.max()),
                            status=np.bincount(st.cpu().numpy(), minlength=4).tolist())
        log(f"tol {tol:g}: {ms:.3f} ms ({N / ms * 1e3:.0f} solves/s), iterations mean "
            f"{its.mean():.2f}, rel. err of w vs planted: mean {err.mean():.2e}")
    main_tol = wl["tol"]
    r = per_tol[main_tol]
    value = N / (r["ms"] / 1e3)
    out = {
        "metric": f"alignment l1 problems solved per second ({m} x {k} per-instance B, tol {main_tol:g})",
        "value": round(value, 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["ms"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (normal equations f64)",
        "data": "synthetic (alignment-shaped dictionaries and occluded queries, seeded)",
        "config": {"workload": args.workload, "m": m, "k": k, "N": N, "problem": "align",
                   "method": "palm", "tol": main_tol},
        "per_tol": {f"{t:g}": {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in d.items()}
                    for t, d in per_tol.items()},
    }
    # Algorithmic work per instance and iteration: B w in FP32 and B^T s in
    # FP64 (2mk flops each) and the row-wise steps (e, s, theta: 10 flops a
    # row).  The bound for that mix is the time the two vector pipes need one
    # after the other: F32 / 157.3 + F64 / 78.6 TFLOP/s.
    f32 = (2 * m * k + 10 * m) * r["iters_total"]
    f64 = 2 * m * k * r["iters_total"]
    t_s = r["ms"] / 1e3
    peak = (f32 + f64) / (f32 / 157.3e12 + f64 / 78.6e12) / 1e12
    achieved = (f32 + f64) / t_s / 1e12
    trec = traffic_record(kernel_source_hash(("align.hip", "internal.h")), "align_traffic.json")
    traffic = None if trec is None else trec.get("hbm_bytes_per_launch_at_workload", {}).get(args.workload)
    out["roofline"] = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 1), "unit": "TFLOP/s",
                       "frac": round(achieved / peak, 4), "traffic": traffic,
                       "kernel": "align_kernel (one launch per batch), HIP events",
                       "avg_launch_us": round(1e3 * r["ms"], 2), "launches_timed": args.steps,
                       "hbm_bytes_per_launch": N * (m * k + 2 * m + k + 2) * 4,
                       "lds_bytes_per_launch": 2 * m * k * 4 * r["iters_total"]}
    if not args.no_cpu_baseline:
        from oracle import align_palm
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        t = time.perf_counter()
        o = align_palm(P.B, P.b, tol=main_tol, max_iter=1000)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": round(N / dt, 2), "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"all {N} instances, FP64 NumPy PALM, same tol; {dt:.1f} s, "
                      f"iterations mean {o.iters.mean():.2f}"}
    if args.copy_calibration:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = x.numel() * 4
    print(json.dumps(out), flush=True)


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count()


def qp_main(args):
    """(QP_lambda) sweep: batched DALM solves/s against one instance per
    launch, accuracy against the oracle's FP64 optimum of instance 0."""
    import numpy as np
    import torch

    from paper_1007_3753_amd import Plan
    from workloads import dense_qp

    wl = QP_WORKLOADS[args.workload]
    P = dense_qp()
    N, m, n = P.N, P.m, P.n_dict
    dev = torch.device("cuda:0")
    A = torch.as_tensor(P.A, device=dev)
    b = torch.as_tensor(P.b, device=dev)
    # one beta for the batch (it enters the factor A A^T + (lambda/beta) I):
    # beta0/3 with beta0 the mean ||b||_1 / m.  Swept at tol 3e-6: beta0 75,
    # beta0/2 224, beta0/3 324, beta0/4 359 solves/s; below beta0/5 the FP32
    # stopping test of this one-tile batch (no refresh of the operand's
    # reference point) no longer reaches the tolerance, and beta0/4 already
    # fails at 2e-6 where beta0/3 converges
    beta = float(np.mean(np.abs(P.b.astype(np.float64)).sum(0) / m)) / 3.0
    plan = Plan(A, problem="qp", lam=P.lam, beta=beta, precision="fp32", max_batch=N, time_kernels=True)
    plan_ms = plan.last_stats()["plan_ms"]
    from paper_1007_3753_amd import tuning
    if args.tune:
        t0 = time.perf_counter()
        table = tuning.tune(plan, path=args.tune_out or tuning.CACHE)
        ks_info = {"source": "tuned in this run", "table": table, "tune_s": round(time.perf_counter() - t0, 2)}
    else:
        table = tuning.apply(plan)
        ks_info = {"source": "cache" if table is not None else "heuristic", "table": table}
    log(f"split-K table: {ks_info}")
    for _ in range(args.warmup):
        plan.solve(b, tol=wl["tol"], max_iter=wl["max_iter"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    timed_ms = timed_n = 0.0
    for _ in range(args.steps):
        r = plan.solve(b, tol=wl["tol"], max_iter=wl["max_iter"])
        st = plan.last_stats()
        timed_ms += st["timed_ms"]
        timed_n += st["timed_launches"]
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / args.steps
    its = r.iters.cpu().numpy()
    X = r.x.cpu().numpy().astype(np.float64)
    rep = plan.kkt(b, r.x).cpu().numpy()
    x_ref = np.load(os.path.join(ROOT, "tests", "golden", "qp_sweep_instance0.npy"))
    err0 = float(np.linalg.norm(X[:, 0] - x_ref) / np.linalg.norm(x_ref))
    log(f"batched: {ms:.1f} ms for {N} instances, iterations mean {its.mean():.0f} max {its.max()}; "
        f"instance 0 vs the FP64 optimum {err0:.2e}")
    # one instance per launch (the plain path), on the first instances
    k = wl["plain"]
    plain = Plan(A, problem="qp", lam=P.lam, beta=beta, precision="fp32", max_batch=1)
    plain.solve(b[:, :1], tol=wl["tol"], max_iter=wl["max_iter"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for j in range(k):
        plain.solve(b[:, j:j + 1], tol=wl["tol"], max_iter=wl["max_iter"])
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t) / k
    value = N / (ms / 1e3)
    out = {
        "metric": "solves/s, QP_lambda sweep (batched DALM, FP32)", "value": round(value, 2), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Gaussian compressive-sensing sweep)",
        "config": {"workload": args.workload, "m": m, "n": n, "N": N, "problem": "QP_lambda", "lambda": P.lam,
                   "beta": beta, "method": "dalm", "precision": "fp32", "tol": wl["tol"]},
        "plan_ms": round(plan_ms, 1),
        "ksplit": ks_info,
        "iterations": {"mean": float(its.mean()), "max": int(its.max())},
        "status_counts": np.bincount(r.status.cpu().numpy(), minlength=4).tolist(),
        "rel_err_instance0_vs_fp64_optimum": err0,
        "kkt_max": {"dual_inf": float(rep[:, 1].max()), "gap": float(rep[:, 3].max())},
        "plain": {"solves_per_s": round(1.0 / plain_s, 3), "instances": k, "batched_over_plain": round(value * plain_s, 1)},
    }
    # roofline of the iteration launch: FP32 products, P (n x n) read once per launch
    if timed_n > 0:
        launch_s = timed_ms / 1e3 / timed_n
        n_pad = -(-n // 64) * 64
        cols = float(its.mean()) * N / float(its.max())    # average active instances per launch
        flops = 2.0 * n * n * cols
        bytes_ = 4.0 * n_pad * n_pad + cols * n * 28
        t_mfma, t_hbm = flops / 157.3e12, bytes_ / (PEAK_HBM_GBS * 1e9)
        if t_mfma >= t_hbm:
            out["roofline"] = {"bound": "mfma", "achieved": round(flops / launch_s / 1e12, 2), "peak": 157.3,
                               "unit": "TFLOP/s", "frac": round(flops / launch_s / 1e12 / 157.3, 4)}
        else:
            out["roofline"] = {"bound": "hbm", "achieved": round(bytes_ / launch_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                               "unit": "GB/s", "frac": round(bytes_ / launch_s / 1e9 / PEAK_HBM_GBS, 4)}
        out["roofline"].update({"traffic": None, "avg_launch_us": round(1e6 * launch_s, 2),
                                "kernel": "DALM iteration launch (FP32), HIP events",
                                "avg_active_instances": round(cols, 1)})
    if not args.no_cpu_baseline:
        from oracle import dalm as oracle_dalm
        K = 100
        t = time.perf_counter()
        oracle_dalm(P.A, P.b[:, :1], problem="qp", lam=P.lam, beta=beta, fixed_iters=K)
        dt = time.perf_counter() - t
        per_solve = dt / K * float(its.mean())
        out["cpu_baseline"] = {"value": round(1.0 / per_solve, 4), "unit": "solves/s", "cores": _threads(),
                               "kind": "oracle",
                               "sample": f"{K} iterations of instance 0 ({dt:.1f} s, FP64 with a Cholesky "
                                         f"y-step), extrapolated to the batch's mean iteration count"}
    print(json.dumps(out), flush=True)


def unrolled_main(args):
    """Differentiable unrolled DALM: time of one forward (fixed iteration
    count, checkpointed) and backward (gradients to b and B) over the batch;
    the gradients against the oracle's reverse mode."""
    import numpy as np
    import torch

    from paper_1007_3753_amd import Plan
    from workloads import cab_problem

    wl = UNROLLED_WORKLOADS[args.workload]
    P = cab_problem(m=1200, classes=100, per_class=7, N=wl["N"], cfg=wl["cfg"])
    N, K = wl["N"], wl["iters"]
    dev = torch.device("cuda:0")
    A = torch.as_tensor(P.A, device=dev)
    b = torch.as_tensor(P.b, device=dev)
    plan = Plan(A, structure="cab", precision="fp32", max_batch=N, record_tape=True, checkpoint_every=wl["every"])
    r = np.random.default_rng([10073753, 77, 1])
    gx_np, ge_np = r.standard_normal((P.n_dict, N)), r.standard_normal((P.m, N))
    gx = torch.as_tensor(gx_np, dtype=torch.float32, device=dev)
    ge = torch.as_tensor(ge_np, dtype=torch.float32, device=dev)
    # the penalty is an input of the differentiated map, passed explicitly and
    # held constant: ||b||_1 / m per instance
    beta = np.abs(P.b.astype(np.float64)).sum(axis=0) / P.m
    pen = torch.as_tensor(beta, dtype=torch.float32, device=dev)

    def step():
        plan.solve(b, max_iter=-K, want_y=False, pen=pen)
        return plan.backward(gx, ge)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        gb, gB = step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / args.steps
    # forward alone
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.solve(b, max_iter=-K, want_y=False, pen=pen)
    torch.cuda.synchronize()
    fwd_ms = 1e3 * (time.perf_counter() - t)
    n = P.n_dict + P.m
    # forward K products, backward K recomputed + K reverse products (2 n^2 each per instance)
    flops = 3.0 * K * 2.0 * n * n * N
    out = {
        "metric": "ms per forward + backward, unrolled DALM (gradients to b and B)", "value": round(ms, 3),
        "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded cross-and-bouquet stand-in, 30 % corruption; random output adjoints)",
        "config": {"workload": args.workload, "m": P.m, "n_dict": P.n_dict, "N": N, "iterations": K,
                   "checkpoint_every": wl["every"]},
        "forward_ms": round(fwd_ms, 3),
        "roofline": {"bound": "mfma", "achieved": round(flops / (ms / 1e3) / 1e12, 3), "peak": 157.3,
                     "unit": "TFLOP/s", "frac": round(flops / (ms / 1e3) / 1e12 / 157.3, 4), "traffic": None,
                     "kernel": "whole forward + backward (FP32 products; 3 products of P per iteration), wall clock"},
    }
    if not args.no_check or not args.no_cpu_baseline:
        from oracle import unrolled_vjp
        t = time.perf_counter()
        gb_o, gB_o = unrolled_vjp(P.A, P.b, beta.astype(np.float32).astype(np.float64), K, gx_np, ge_np)
        dt = time.perf_counter() - t
        gbn, gBn = gb.cpu().numpy().astype(np.float64), gB.cpu().numpy().astype(np.float64)
        out["grad_rel_err_vs_oracle"] = {
            "b": float(np.linalg.norm(gbn - gb_o) / np.linalg.norm(gb_o)),
            "B": float(np.linalg.norm(gBn - gB_o) / np.linalg.norm(gB_o))}
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {"value": round(1e3 * dt, 1), "unit": "ms", "cores": _threads(), "kind": "oracle",
                                   "sample": f"the whole batch ({N} instances), FP64 forward and reverse mode"}
    log(f"forward + backward {ms:.1f} ms (forward {fwd_ms:.1f} ms); {out.get('grad_rel_err_vs_oracle')}")
    print(json.dumps(out), flush=True)


def run():
    """main() with a deterministic teardown: every plan is destroyed and the
    device drained before the interpreter starts to shut down."""
    try:
        main()
    finally:
        if "paper_1007_3753_amd._lib" in sys.modules:
            sys.modules["paper_1007_3753_amd._lib"].close_all()


if __name__ == "__main__":
    run()
