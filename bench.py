"""Benchmark: ALS iterations per second of CPRAND-MIX on a 400x400x400 FP32
tensor (rank 10, column congruence 0.5, 1% noise, S = 10 R ceil(ln R) = 300,
P-hat = 2^14), each decomposition run to the paper's fit target F-hat >=
1 - 1.2 eta = 0.988 (200 iterations at most).

One step = one whole decomposition on the GPU: ||X||, random signs, the
mixing pass along every mode, the factor mixes, then the ALS loop (sample,
sampled Khatri-Rao rows, fiber gather, MTTKRP on MFMA, FP64 solve,
normalisation, factor remix, sampled fit estimate, stop test) and the final
unmix.  `value` is outer iterations per second of the whole step.

Also reported (not part of `value`):
  - the result's exact fit (the library's full-MTTKRP fit check) and factor
    match score, loop-only rate and one-time setup time,
  - CPRAND-MIX, plain CPRAND and CPRAND-PREMIX (DCT) over five sampling
    seeds, to the fit target and with the paper's |dF| <= 1e-4 stop rule
    (medians and every run),
  - the roofline of the dominant kernel (the mixing pass), from HIP events
    recorded around each pass inside the timed steps,
  - a gather/MTTKRP throughput leg: one cprand_mttkrp_sampled launch over
    many samples of the mixed tensor, timed with HIP events,
  - the dense comparison: full MTTKRP, exact against sampled fit check,
    CP-ALS against CPRAND iterations,
  - the CPU oracle (numpy FP64) on a bounded sample of the same work,
  - precision form: 150^4 tensor (R=20, S=1000), BF16 MFMA gathers with one
    FP32 refinement against the FP32 path,
  - learned proposal: 1000^3 spiky tensor (R=50, congruence 0.9, S=2000),
    the network trained on the GPU, against uniform, CPRAND-MIX and
    exact-marginal sampling,
  - combined form: 60^5 spiky tensor (R=25), learned proposal with BF16
    products against FP32 CPRAND-MIX.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs main,dense,precision,learned,combined]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the mixing pass on the 400^3 workload (average of
# the three passes of the main leg, the last one also writing its mode-major
# copy), from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE, scaled by what the
# same counters read for a 1 GiB device copy (FETCH_SIZE x 2, WRITE_SIZE x 1).
# Valid for the kernel as measured; None when the mixing kernel has changed
# since the counters were taken.
MIX_TRAFFIC_BYTES = (2 * 125134 + 500009 + 2 * 250085 + 500013 + 2 * 250082 + 1000474) * 1024 / 3
# the same 1 GiB copy (read + write) took 423 us: 5.08 TB/s, the practical ceiling seen
COPY_GBPS = 2 * 1073741824 / 423e-6 / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--layout", type=int, default=0, help="0: mode-major copies of X-hat, 1: strided gathers")
    ap.add_argument("--graph", type=int, default=0,
                    help="main leg: 0 direct launches (fit estimate on its own stream), 1 one HIP graph per iteration")
    ap.add_argument("--legs", default="main,dense,precision,learned,combined,standins,gather")
    ap.add_argument("--train-instances", type=int, default=200)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (reference for HBM byte counters)")
    args = ap.parse_args()
    legs = set(args.legs.split(","))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        n = (1 << 30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}), flush=True)
        return

    import paper_1701_06600_amd as P
    import synth

    dev = torch.device("cuda:0")
    if "main" not in legs and "mixonly" not in legs and "mixplan" not in legs:
        # only the named side legs (profiling runs); no headline line
        out = {"legs": sorted(legs)}
        _extra_legs(P, synth, torch, dev, args, legs, out)
        print(json.dumps(out), flush=True)
        return
    w = synth.WORKLOADS["cprand-400cube-f32"]
    R, S = w.R, w.S
    prob = synth.problem_for(w)
    print("[bench] generating %s on the GPU" % (w.name,), flush=True)
    X = synth.device_tensor(prob, dev, "f32")
    Xv = P.View(X, w.dims)
    init = [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in prob.init]
    torch.cuda.synchronize()
    if "mixonly" in legs:
        # only the mixing of the tensor, twice (for hardware counters of the mixing passes)
        for _ in range(2):
            Xh, signs, nrm = P.cprand_mix(Xv, w.seed)
        torch.cuda.synchronize()
        print(json.dumps({"mixonly": True, "dims": list(w.dims)}), flush=True)
        return

    # the main run goes to the paper's fit target F-hat >= 1 - 1.2 eta (or
    # 200 iterations) with the |dF| <= 1e-4 rule off: that rule stops the
    # sampled iteration on a plateau far from the noise floor on this tensor
    # (reported separately below as "paper_stop_rule")
    def opts(mix, max_iters=w.max_iters, tol=0.0, seed=w.seed):
        kind = P.MIX_FFT if mix is True else (P.MIX_NONE if mix is False else mix)
        return P.make_opts(R, S, P_hat=w.P_hat, max_iters=max_iters, seed=seed, tol=tol,
                           fit_target=w.fit_target, mix=kind, layout=args.layout, use_graph=args.graph)

    if "mixplan" in legs:
        # the plan's setup (mixing passes with the folded norm and mode-major
        # copy) and one iteration, twice (for hardware counters of the passes)
        plan = P.Plan(Xv, opts(True, max_iters=1))
        for _ in range(2):
            r = plan.run(Xv, [M.clone() for M in init])
        torch.cuda.synchronize()
        print(json.dumps({"mixplan": True, "fused": r["fused"], "mix_ms": r["mix_ms"]}), flush=True)
        return

    plan = P.Plan(Xv, opts(True))
    last = {}

    def step():
        A = [M.clone() for M in init]
        r = plan.run(Xv, A)
        last["A"] = A
        return r

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] timing %d steps" % args.steps, flush=True)
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runs.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_s = t1 - t0
    iters = sum(r["iters"] for r in runs)
    value = iters / total_s
    loop_ms = sum(r["loop_ms"] for r in runs)
    setup_ms = sum(r["setup_ms"] for r in runs) / len(runs)

    # dominant kernel: the mixing pass (HIP events around each pass, in the timed steps)
    P_el = math.prod(w.dims)
    mix_ms = [sum(r["mix_ms"][m] for r in runs) / len(runs) for m in range(3)]
    # pass 0 reads FP32 and writes complex64; the last pass also writes its
    # mode-major copy when the plan folded that copy into it
    mix_bytes = [P_el * (4 + 8), P_el * 16, P_el * (24 if runs[-1]["fused"] & 2 else 16)]
    mix_launch_ms = sum(mix_ms) / 3
    mix_achieved = sum(mix_bytes) / 3 / (mix_launch_ms * 1e-3) / 1e9

    normX = P.cprand_norm(Xv)
    truth = prob.factors

    def evaluate(r, A):
        F, sc = _evaluate(P, Xv, normX, r["lambda"], A, R, truth)
        return {"exact_fit": F, "score": sc}

    main_eval = evaluate(runs[-1], last["A"])

    # CPRAND-MIX, plain CPRAND and CPRAND-PREMIX (Alg. 5, orthonormal DCT-II)
    # over five sampling seeds, to the fit target and with the paper's stop
    # rule: the iteration count of one sampled run depends on its trajectory
    seeds = [w.seed + k for k in range(5)]
    methods = {}
    dct_pass_ms = None
    for name, mix in (("mix", P.MIX_FFT), ("plain", P.MIX_NONE), ("premix_dct", P.MIX_DCT)):
        entry = {}
        for rule, tol in (("to_fit_target", 0.0), ("paper_stop_rule", w.tol)):
            recs = []
            for sd in seeds:
                pl = P.Plan(Xv, opts(mix, tol=tol, seed=sd))
                rr, sec, A_c = _timed_median(pl, Xv, init, 3)
                pl.close()
                if name == "premix_dct" and dct_pass_ms is None:
                    dct_pass_ms = rr["mix_ms"][:3]
                recs.append({"seed": sd, "iters": rr["iters"], "ms_per_decomposition": sec * 1e3,
                             "iters_per_s": rr["iters"] / sec, "final_fit_est": rr["fit_est"], **evaluate(rr, A_c)})
            entry[rule] = _medians(recs)
            entry[rule]["runs"] = recs
            m_ = entry[rule]
            print("[bench] %s %s: median %g iters, %.2f ms, fit %.5f, score %.4f"
                  % (name, rule, m_["iters"], m_["ms_per_decomposition"], m_["exact_fit"], m_["score"]), flush=True)
        methods[name] = entry
    # the DCT passes of PREMIX: 4 B read + 4 B written per element each
    pm_gbs = [P_el * 8 / (ms * 1e-3) / 1e9 for ms in dct_pass_ms]
    methods["premix_dct"]["dct_pass_ms"] = dct_pass_ms
    methods["premix_dct"]["dct_pass_GBps"] = pm_gbs
    methods["premix_dct"]["dct_pass_frac_of_hbm"] = [g / HBM_PEAK_GBS for g in pm_gbs]

    # gather / sampled-MTTKRP leg: one launch over many samples of X-hat
    Xh, signs, nrm = P.cprand_mix(Xv, w.seed)
    Ah = [P.cprand_mix_factor(M, signs[sum(w.dims[:m]):sum(w.dims[:m + 1])]) for m, M in enumerate(init)]
    Sg = 300 * 256
    idx, _ = P.cprand_sample(w.dims, 0, Sg, w.seed, 0)
    ws = P.workspace(Xh, R, Sg)
    Wg = torch.empty((w.dims[0], R), dtype=torch.float32, device=dev)
    Vg = torch.empty((R, R), dtype=torch.float64, device=dev)
    for _ in range(2):
        P.cprand_mttkrp_sampled(Xh, 0, Ah, R, Sg, idx, unmix_signs=signs[:w.dims[0]], W=Wg, V=Vg, ws=ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        P.cprand_mttkrp_sampled(Xh, 0, Ah, R, Sg, idx, unmix_signs=signs[:w.dims[0]], W=Wg, V=Vg, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    g_ms = e0.elapsed_time(e1) / reps
    g_bytes = Sg * w.dims[0] * 8
    gather_gbs = g_bytes / (g_ms * 1e-3) / 1e9

    out = {
        "metric": "ALS iters/s + sampled-MTTKRP GB/s at equal fit (+-1e-3), learned/BF16 vs plain",
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "launch": "HIP graph per iteration" if args.graph else "direct launches, fit estimate on a second stream",
        "config": {"workload": "CPRAND-MIX, 400x400x400 FP32, R=10, congruence 0.5, 1% noise, "
                               "S=300, P-hat=2^14, run to F-hat >= 1 - 1.2 eta = 0.988 (200 iterations at most)",
                   "layout": "strided X-hat gathers" if args.layout else "mode-major X-hat copies"},
        "iters_per_step": iters / args.steps,
        "final_fit_est": runs[-1]["fit_est"],
        "exact_fit": main_eval["exact_fit"],
        "score": main_eval["score"],
        "loop_iters_per_s": iters / (loop_ms * 1e-3),
        "setup_ms": setup_ms,
        "mix_pass_ms": mix_ms,
        "methods_400cube": methods,
        "gather_mttkrp": {"samples": Sg, "ms": g_ms, "useful_GBps": gather_gbs,
                          "frac_of_hbm": gather_gbs / HBM_PEAK_GBS},
        "roofline": {"kernel": "mix_pass_pipe", "bound": "hbm", "achieved": mix_achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": mix_achieved / HBM_PEAK_GBS,
                     "traffic": MIX_TRAFFIC_BYTES, "algorithmic_bytes": sum(mix_bytes) / 3,
                     "copy_GBps": COPY_GBPS},
    }

    if "dense" in legs:
        out["dense"] = dense_leg(P, torch, Xv, w, init, normX, out)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(X, w, prob, iters / args.steps)
    del X, Xh, Xv, plan
    torch.cuda.empty_cache()
    _extra_legs(P, synth, torch, dev, args, legs, out)
    print(json.dumps(out), flush=True)


def _extra_legs(P, synth, torch, dev, args, legs, out):
    """The legs beside the main one, each on its own workload."""
    if "precision" in legs:
        out["precision_form"] = precision_leg(P, synth, torch, dev, max(1, args.steps // 2))
        torch.cuda.empty_cache()
    theta = None
    if "learned" in legs:
        out["learned_proposal"], theta = learned_leg(P, synth, torch, dev, args.train_instances)
        torch.cuda.empty_cache()
    if "combined" in legs:
        if theta is None:
            theta, _ = _train_proposal(P, synth, torch, dev, args.train_instances,
                                       synth.WORKLOADS["cprand-1000cube-f32-spiky"])
        out["combined"] = combined_leg(P, synth, torch, dev, theta)
        torch.cuda.empty_cache()
    if "standins" in legs:
        out["standins"] = standin_leg(P, synth, torch, dev)
        torch.cuda.empty_cache()
    if "gather" in legs:
        out["gather_throughput"] = gather_leg(P, synth, torch, dev)


def _events_ms(torch, fn, reps):
    """Mean milliseconds of fn() over reps calls, HIP events on the current stream."""
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def dense_leg(P, torch, Xv, w, init, normX, main_out):
    """The paper's comparison with dense CP-ALS (Section 4.1) on the 400^3
    tensor, as relative numbers on one GPU: the full MTTKRP of every mode
    (HBM-bound, one read of X), the exact fit check against the sampled one
    (P-hat = 2^14), and CP-ALS iterations against CPRAND / CPRAND-MIX
    iterations (rank 10, S = 300, and the paper's R = 5, S = 90)."""
    import statistics
    R, dims = w.R, w.dims
    P_el = math.prod(dims)
    lam = torch.full((R,), 0.5, dtype=torch.float64, device="cuda")
    A = [M.clone() for M in init]
    ws = P.full_workspace(Xv, R)
    res = {"workload": "400x400x400 FP32, R=10"}
    mt = []
    for n in range(3):
        W = torch.empty((dims[n], R), dtype=torch.float64, device="cuda")
        ms = _events_ms(torch, lambda: P.cprand_mttkrp_full(Xv, n, A, R, W=W, ws=ws), 10)
        gbs = P_el * 4 / (ms * 1e-3) / 1e9
        mt.append({"mode": n, "ms": ms, "GBps": gbs, "frac_of_hbm": gbs / HBM_PEAK_GBS})
    res["mttkrp_full"] = mt
    fo = torch.empty(1, dtype=torch.float64, device="cuda")
    ex_ms = _events_ms(torch, lambda: P.cprand_fit_exact(Xv, normX, A, lam, R, fit_out=fo, ws=ws), 10)
    wsf = P.workspace(Xv, R, 1, w.P_hat)
    est_ms = _events_ms(torch, lambda: P.cprand_fit_est(Xv, normX, A, lam, R, w.P_hat, w.seed, fit_out=fo, ws=wsf), 20)
    res["fit_check"] = {"exact_ms": ex_ms, "sampled_ms": est_ms, "speedup": ex_ms / est_ms}
    cp = {}
    for r_, s_ in ((R, w.S), (5, 90)):
        Ac = [M[:, :r_].contiguous() for M in init]
        P.cprand_cpals(Xv, Ac, r_, 2)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            Ac = [M[:, :r_].contiguous() for M in init]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = P.cprand_cpals(Xv, Ac, r_, 10)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) / o["iters"])
        cp_ms = statistics.median(times) * 1e3
        entry = {"R": r_, "S": s_, "cpals_ms_per_iter": cp_ms}
        for name, mix in (("cprand", P.MIX_NONE), ("cprand_mix", P.MIX_FFT)):
            o = P.make_opts(r_, s_, P_hat=w.P_hat, max_iters=20, seed=w.seed, mix=mix, use_graph=0)
            pl = P.Plan(Xv, o)
            Ai = [M[:, :r_].contiguous() for M in init]
            rr, sec, _ = _timed_median(pl, Xv, Ai, 3)
            pl.close()
            per = rr["loop_ms"] / rr["iters"]
            entry[name + "_ms_per_iter"] = per
            entry["speedup_" + name] = cp_ms / per
        cp["R%d_S%d" % (r_, s_)] = entry
        print("[bench] dense R=%d: CP-ALS %.3f ms/iter, CPRAND %.3f, CPRAND-MIX %.3f"
              % (r_, cp_ms, entry["cprand_ms_per_iter"], entry["cprand_mix_ms_per_iter"]), flush=True)
    res["per_iteration"] = cp
    return res


def _score(truth, A):
    """Factor match score (Section 4.2, eq. score): per pair of true and
    computed components the product over modes of their signed cosines
    (lambda ignored), the best one-to-one assignment (Hungarian), averaged
    over the true components."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment
    C = None
    for T, M in zip(truth, A):
        Tn = T / np.maximum(np.linalg.norm(T, axis=0), 1e-300)
        Mn = M / np.maximum(np.linalg.norm(M, axis=0), 1e-300)
        c = Tn.T @ Mn
        C = c if C is None else C * c
    rows, cols = linear_sum_assignment(-C)
    return float(C[rows, cols].sum() / C.shape[0])


def _evaluate(P, Xv, normX, lam, A, R, truth):
    """Exact fit of a result by the library's full-MTTKRP fit check, and its
    factor match score against the true factors (host, evaluation only)."""
    import torch
    F = float(P.cprand_fit_exact(Xv, normX, A, lam, R).item())
    torch.cuda.synchronize()
    return F, _score(truth, [M.double().cpu().numpy() for M in A])


def _timed_median(plan, Xv, init, reps):
    """One warm-up decomposition, then `reps` timed ones (each synchronised);
    returns the last run record, the median wall time and the last factors."""
    import statistics
    import torch
    plan.run(Xv, [M.clone() for M in init])
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        A = [M.clone() for M in init]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.run(Xv, A)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return r, statistics.median(times), A


def _medians(recs):
    import statistics
    keys = ("iters", "ms_per_decomposition", "iters_per_s", "final_fit_est", "exact_fit", "score")
    return {k: statistics.median([r[k] for r in recs]) for k in keys}


def _timed_runs(plan, Xv, init, reps):
    """One warm-up decomposition, then `reps` timed ones; returns the last
    run record and the mean wall time per decomposition."""
    import torch
    plan.run(Xv, [M.clone() for M in init])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        A = [M.clone() for M in init]
        r = plan.run(Xv, A)
    torch.cuda.synchronize()
    r["A"] = A
    return r, (time.perf_counter() - t0) / reps


def precision_leg(P, synth, torch, dev, reps):
    """BF16 tensor copies on MFMA with one FP32 refinement vs the FP32 path,
    same tensor, seeds and stop rule."""
    w = synth.WORKLOADS["cprand-150pow4-bf16"]
    prob = synth.problem_for(w)
    print("[bench] generating %s" % w.name, flush=True)
    X = synth.device_tensor(prob, dev, "f32")
    Xv = P.View(X, w.dims)
    init = [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in prob.init]
    res = {}
    # layout 0: mode-major copies of every mode (FP32, and BF16 for the BF16
    # form); layout 1: strided gathers from X (the BF16 form from one BF16
    # conversion of X)
    for layout, key in ((0, None), (1, "strided")):
        out = res if key is None else res.setdefault(key, {})
        for name, prec in (("fp32", P.PREC_NATIVE), ("bf16_refine", P.PREC_BF16_REFINE)):
            opts = P.make_opts(w.R, w.S, P_hat=w.P_hat, max_iters=w.max_iters, seed=w.seed, tol=w.tol,
                               fit_target=w.fit_target, precision=prec, layout=layout, use_graph=0)
            plan = P.Plan(Xv, opts)
            r, sec = _timed_runs(plan, Xv, init, reps)
            plan.close()
            out[name] = {"iters": r["iters"], "s_per_decomposition": sec, "iters_per_s": r["iters"] / sec,
                         "loop_iters_per_s": r["iters"] / (r["loop_ms"] * 1e-3), "setup_ms": r["setup_ms"],
                         "final_fit_est": r["fit_est"]}
            print("[bench] precision %s layout %d: %d iters, %.3f s, F-hat %.5f"
                  % (name, layout, r["iters"], sec, r["fit_est"]), flush=True)
        d = abs(out["bf16_refine"]["final_fit_est"] - out["fp32"]["final_fit_est"])
        out["equal_fit"] = d <= 1e-3
        out["fit_diff"] = d
        out["speedup_per_decomposition"] = out["fp32"]["s_per_decomposition"] / out["bf16_refine"]["s_per_decomposition"]
    res["workload"] = "150x150x150x150, R=20, congruence 0.5, 1% noise, S=1000, paper stop rule"
    return res


def _method_runs(P, Xv, init, normX, truth, R, make, seeds, label):
    """One warm-up and one timed decomposition per seed for a method (the
    plan built by make(seed)); per-seed records and their medians."""
    recs = []
    for sd in seeds:
        plan = P.Plan(Xv, make(sd))
        r, sec, A = _timed_median(plan, Xv, init, 1)
        plan.close()
        F, sc = _evaluate(P, Xv, normX, r["lambda"], A, R, truth)
        recs.append({"seed": sd, "iters": r["iters"], "ms_per_decomposition": sec * 1e3,
                     "iters_per_s": r["iters"] / sec, "final_fit_est": r["fit_est"], "exact_fit": F, "score": sc,
                     "setup_ms": r["setup_ms"], "fell_back": bool(r["flags"] & P.W_FALLBACK)})
    out = _medians(recs)
    out["runs"] = recs
    print("[bench] %s: median %g iters, %.2f ms, F-hat %.5f, fit %.5f, score %.4f"
          % (label, out["iters"], out["ms_per_decomposition"], out["final_fit_est"], out["exact_fit"], out["score"]),
          flush=True)
    return out


def learned_leg(P, synth, torch, dev, n_inst, nseeds=5):
    """Uniform, CPRAND-MIX, CPRAND-PREMIX, learned, exact-marginal and
    factor-leverage-product sampling on the coherent 1000^3 workload, with
    the network trained on the GPU first; each method runs to F-hat >= 0.988
    (200 iterations at most) over several sampling seeds.  The unmixed
    methods estimate the fit on the importance-weighted fit set (the uniform
    one overstates the fit on this tensor); the mixed ones on the uniform set
    of the mixed tensor."""
    w = synth.WORKLOADS["cprand-1000cube-f32-spiky"]
    R, S = w.R, w.S
    theta, training = _train_proposal(P, synth, torch, dev, n_inst, w)

    prob = synth.problem_for(w)
    print("[bench] generating %s" % w.name, flush=True)
    X = synth.device_tensor(prob, dev, "f32")
    Xv = P.View(X, w.dims)
    init = [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in prob.init]
    normX = P.cprand_norm(Xv)
    seeds = [w.seed + k for k in range(nseeds)]
    res = {"workload": "1000x1000x1000 FP32, R=50, congruence 0.9, 10% rows x20, 1% noise, S=2000; each method "
                       "runs until F-hat >= 1 - 1.2 eta = 0.988 or 200 iterations (no |dF| rule); medians over "
                       + str(nseeds) + " sampling seeds",
           "training": training}
    runs = (("uniform", P.PROPOSAL_UNIFORM, P.MIX_NONE), ("mix", P.PROPOSAL_UNIFORM, P.MIX_FFT),
            ("premix_dct", P.PROPOSAL_UNIFORM, P.MIX_DCT), ("learned", P.PROPOSAL_LEARNED, P.MIX_NONE),
            ("marginal", P.PROPOSAL_MARGINAL, P.MIX_NONE), ("leverage", P.PROPOSAL_LEVERAGE, P.MIX_NONE))
    for name, prop, mix in runs:
        adaptive = prop != P.PROPOSAL_UNIFORM

        def make(sd, prop=prop, mix=mix, adaptive=adaptive):
            return P.make_opts(R, S, P_hat=w.P_hat, max_iters=w.max_iters, seed=sd, tol=0.0,
                               fit_target=w.fit_target, mix=mix, proposal=prop, alpha=0.1, layout=1,
                               use_graph=1 if adaptive else 0, fit_beta=0.5 if mix == P.MIX_NONE else 0.0,
                               mlp_params=theta if prop == P.PROPOSAL_LEARNED else None)
        res[name] = _method_runs(P, Xv, init, normX, prob.factors, R, make, seeds, "learned-leg " + name)
        res[name]["reached_target"] = res[name]["exact_fit"] >= w.fit_target - 1e-3
    del X, Xv
    torch.cuda.empty_cache()
    return res, theta


def _train_proposal(P, synth, torch, dev, n_inst, w):
    """The proposal network trained on the GPU on seeded 100^3 instances of
    the coherent generator (true factors, random starts and CPRAND iterates)."""
    from paper_1701_06600_amd.training import proposal_training_set
    R, S = w.R, w.S
    print("[bench] training the proposal network on %d instances of 100^3" % n_inst, flush=True)
    t0 = time.perf_counter()
    inst = []
    for k, p in enumerate(synth.training_problems(n_inst, (100, 100, 100), R, w.congruence, w.spiky, w.noise)):
        Xk = synth.device_tensor(p, dev, "f32")
        inst.append((P.View(Xk, p.dims), [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in p.factors],
                     [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in p.init]))
    Xt, tt, goff = proposal_training_set(inst, R, S)
    del inst
    t_build = time.perf_counter() - t0
    theta = torch.as_tensor(synth.mlp_init(11), dtype=torch.float32, device=dev)
    t1 = time.perf_counter()
    epochs = 300
    hist = P.cprand_mlp_train(theta, Xt, tt, goff, epochs=epochs, lr=3e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    rows = Xt.shape[0]
    del Xt, tt, goff
    print("[bench] training: %d rows, loss %.4f -> %.4f, %.1f s" % (rows, hist[0], hist[-1], t_train), flush=True)
    return theta, {"instances": n_inst, "rows": rows, "epochs": epochs, "loss_first": hist[0],
                   "loss_last": hist[-1], "build_s": t_build, "train_s": t_train}


def combined_leg(P, synth, torch, dev, theta, nseeds=3):
    """The order-5 workload of the metric's comparison: every method runs
    with the paper's stop rule (|dF| <= 1e-4, F-hat >= 1 - 1.2 eta, 200
    iterations) on its own fit estimate, over several sampling seeds: plain
    FP32 CPRAND-MIX (the reference, estimate on the mixed tensor), the
    learned proposal with BF16 products and FP32 refinement, without
    refinement, and in FP32, and for context CPRAND-PREMIX, the
    factor-leverage proposal and uniform sampling.  The unmixed methods
    estimate the fit on the importance-weighted fit set (on this tensor the
    uniform set of Section 3.4 overstates the fit by up to 0.06).  Equal fit:
    median exact fit within 1e-3 of the reference's."""
    w = synth.WORKLOADS["cprand-60pow5-bf16-spiky"]
    prob = synth.problem_for(w)
    print("[bench] generating %s" % w.name, flush=True)
    X = synth.device_tensor(prob, dev, "f32")
    Xv = P.View(X, w.dims)
    init = [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in prob.init]
    normX = P.cprand_norm(Xv)
    seeds = [w.seed + k for k in range(nseeds)]
    res = {"workload": "60^5 FP32 (BF16 copies for the BF16 forms), R=25, congruence 0.7, 10% rows x20, 5% noise, "
                       "S=1000; every method stops on its own fit estimate by the paper's rule (|dF| <= 1e-4, "
                       "F-hat >= 1 - 1.2 eta = 0.94, 200 iterations); medians over " + str(nseeds) + " sampling seeds"}
    methods = (
        # name, proposal, mix, precision, layout (0 mode-major copies, 1 strided gathers)
        ("mix_fp32", P.PROPOSAL_UNIFORM, P.MIX_FFT, P.PREC_NATIVE, 0),
        ("learned_bf16_refine", P.PROPOSAL_LEARNED, P.MIX_NONE, P.PREC_BF16_REFINE, 1),
        ("learned_bf16", P.PROPOSAL_LEARNED, P.MIX_NONE, P.PREC_BF16, 1),
        ("learned_fp32", P.PROPOSAL_LEARNED, P.MIX_NONE, P.PREC_NATIVE, 1),
        ("leverage_fp32", P.PROPOSAL_LEVERAGE, P.MIX_NONE, P.PREC_NATIVE, 1),
        ("premix_fp32", P.PROPOSAL_UNIFORM, P.MIX_DCT, P.PREC_NATIVE, 1),
        ("uniform_fp32", P.PROPOSAL_UNIFORM, P.MIX_NONE, P.PREC_NATIVE, 1),
    )
    for name, prop, mix, prec, layout in methods:
        adaptive = prop != P.PROPOSAL_UNIFORM

        def make(sd, prop=prop, mix=mix, prec=prec, layout=layout, adaptive=adaptive):
            return P.make_opts(w.R, w.S, P_hat=w.P_hat, max_iters=w.max_iters, seed=sd, tol=w.tol,
                               fit_target=w.fit_target, mix=mix, proposal=prop, precision=prec, alpha=0.1,
                               layout=layout, use_graph=1 if adaptive else 0,
                               fit_beta=0.5 if mix == P.MIX_NONE else 0.0,
                               mlp_params=theta if prop == P.PROPOSAL_LEARNED else None)
        res[name] = _method_runs(P, Xv, init, normX, prob.factors, w.R, make, seeds, "combined " + name)
        torch.cuda.empty_cache()
    ref = res["mix_fp32"]
    for name, *_ in methods[1:]:
        r = res[name]
        r["equal_fit"] = abs(r["exact_fit"] - ref["exact_fit"]) <= 1e-3 or r["exact_fit"] > ref["exact_fit"]
        r["speedup_vs_mix_fp32"] = ref["ms_per_decomposition"] / r["ms_per_decomposition"]
    a = res["learned_bf16_refine"]
    res["equal_fit"] = bool(a["equal_fit"])
    res["speedup_vs_mix_fp32"] = a["speedup_vs_mix_fp32"]
    del X, Xv
    torch.cuda.empty_cache()
    return res


def gather_leg(P, synth, torch, dev, reps=10):
    """Throughput of the sampled MTTKRP at the shape of a mode step but with
    enough uniformly drawn samples (many independent draws' worth, one
    launch) that each call moves about 1 GB of fibers: FP32 fibers of 1000
    (the 1000^3 tensor, mode 0, contiguous), the same tensor's BF16 copy
    (twice the samples), and complex64 fibers of 400 (the mixed 400^3
    tensor, mode 0), rank 10.  Useful bytes = S I_n b_X per call;
    the 1000^3 tensor has 10^6 fibers per mode, so few of the 256,000 draws
    repeat a fiber (the cache cannot serve them)."""
    R = 10
    res = {}
    cases = []
    w4 = synth.WORKLOADS["cprand-1000cube-f32-spiky"]
    prob4 = synth.problem_for(w4)
    print("[bench] generating %s for the gather leg" % w4.name, flush=True)
    X4 = synth.device_tensor(prob4, dev, "f32")
    A4 = [torch.as_tensor(M[:, :R], dtype=torch.float32, device=dev).contiguous() for M in prob4.init]
    cases.append(("f32_1000cube_mode0", P.View(X4, w4.dims), w4.dims, 0, 256000, 4, A4, None))
    # the BF16 form of the same tensor (a mode-0-major BF16 copy): twice the
    # samples for the same 1.024 GB of fibers, on BF16 MFMA
    Yb = P.mode_major_copy(P.View(X4, w4.dims), 0, dtype=torch.bfloat16)
    cases.append(("bf16_1000cube_mode0", P.View(Yb.data, Yb.dims, Yb.strides, dtype=P.BF16), w4.dims, 0, 512000, 2,
                  A4, None))
    w2 = synth.WORKLOADS["cprand-400cube-f32"]
    prob2 = synth.problem_for(w2)
    X2 = synth.device_tensor(prob2, dev, "f32")
    Xh, signs, _ = P.cprand_mix(P.View(X2, w2.dims), w2.seed)
    del X2
    init2 = [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in prob2.init]
    Ah = [P.cprand_mix_factor(M, signs[sum(w2.dims[:m]):sum(w2.dims[:m + 1])]) for m, M in enumerate(init2)]
    cases.append(("c64_400cube_mixed_mode0", Xh, w2.dims, 0, 320000, 8, Ah, signs[:w2.dims[0]]))
    for name, Xv, dims, n, S, bx, A, sg in cases:
        idx, _ = P.cprand_sample(dims, n, S, 1701066100, 0)
        ws = P.workspace(Xv, R, S)
        Wg = torch.empty((dims[n], R), dtype=torch.float32, device=dev)
        Vg = torch.empty((R, R), dtype=torch.float64, device=dev)
        ms = _events_ms(torch, lambda: P.cprand_mttkrp_sampled(Xv, n, A, R, S, idx, unmix_signs=sg, W=Wg, V=Vg,
                                                               ws=ws), reps)
        useful = S * dims[n] * bx
        gbs = useful / (ms * 1e-3) / 1e9
        res[name] = {"samples": S, "fiber_len": dims[n], "bytes_per_call": useful, "ms_per_call": ms,
                     "useful_GBps": gbs, "frac_of_hbm": gbs / HBM_PEAK_GBS}
        print("[bench] gather %s: %.3f ms per call, %.0f GB/s useful (%.2f of HBM)"
              % (name, ms, gbs, gbs / HBM_PEAK_GBS), flush=True)
    del X4, Xh, Yb
    torch.cuda.empty_cache()
    return res


def standin_leg(P, synth, torch, dev):
    """Synthetic tensors at the shapes of the paper's real-data runs (the
    datasets are not available, so fits are not comparable to the paper's):
    COIL-100, 128 x 128 x 3 x 7200, R = 20, CPRAND-MIX with S = 400 and
    1000, stop after 5 iterations without improvement; hazardous gases,
    25,900 x 72 x 899, R = 5, S = 1000, plain CPRAND, stop after 10 without
    improvement.  Whole decompositions (mixing included), with the paper's
    CPU timings for context."""
    out = {}
    paper = {"coil-standin-f32": "CPRAND-MIX S=400: 8.38x the 204 s of CP-ALS (about 24 s), fit 0.674; S=1000: "
                                 "2.84x (about 72 s), fit 0.684 (Intel Xeon E5-2650, MATLAB, FP64, real images)",
             "gas-standin-f32": "CPRAND: 53.6 s median, fit 0.715 (Intel Xeon E5-2650, MATLAB, FP64, real sensor data)"}
    for key, mix, S_list in (("coil-standin-f32", P.MIX_FFT, (400, 1000)), ("gas-standin-f32", P.MIX_NONE, (1000,))):
        w = synth.WORKLOADS[key]
        prob = synth.problem_for(w)
        print("[bench] generating %s" % key, flush=True)
        X = synth.device_tensor(prob, dev, "f32")
        Xv = P.View(X, w.dims)
        init = [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in prob.init]
        normX = P.cprand_norm(Xv)
        entry = {"dims": list(w.dims), "R": w.R, "noise": w.noise, "paper_context": paper[key]}
        for S in S_list:
            o = P.make_opts(w.R, S, P_hat=w.P_hat, max_iters=w.max_iters, seed=w.seed, tol=0.0, patience=w.patience,
                            mix=mix, layout=0, use_graph=0)
            plan = P.Plan(Xv, o)
            r, sec, A = _timed_median(plan, Xv, init, 1)
            plan.close()
            F, sc = _evaluate(P, Xv, normX, r["lambda"], A, w.R, prob.factors)
            entry["S%d" % S] = {"iters": r["iters"], "s_per_decomposition": sec, "iters_per_s": r["iters"] / sec,
                                "setup_ms": r["setup_ms"], "mix_pass_ms": r["mix_ms"][:len(w.dims)],
                                "final_fit_est": r["fit_est"], "exact_fit": F, "score": sc}
            print("[bench] %s S=%d: %d iters, %.3f s, setup %.1f ms, F-hat %.4f, fit %.4f"
                  % (key, S, r["iters"], sec, r["setup_ms"], r["fit_est"], F), flush=True)
            torch.cuda.empty_cache()
        out[key] = entry
        del X, Xv, A
        torch.cuda.empty_cache()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(Xdev, w, prob, gpu_iters):
    """The oracle (numpy FP64) on the same tensor: the mixing pass plus a
    bounded number of ALS iterations; rate = iterations / wall time.  Run
    with the BLAS thread pool as configured and again with one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import cprand as OC
    from oracle.tensor import from_colmajor

    X = from_colmajor(Xdev.double().cpu().numpy(), w.dims)
    k = int(max(1, min(5, round(gpu_iters))))
    pools = threadpool_info()
    threads = max([p.get("num_threads", 1) for p in pools] or [1])
    t0 = time.perf_counter()
    lam, A, hist = OC.cprand_mix(X, w.R, w.S, prob.init, w.seed, k, P_hat=w.P_hat)
    dt = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        lam, A, hist1 = OC.cprand_mix(X, w.R, w.S, prob.init, w.seed, k, P_hat=w.P_hat)
        dt1 = time.perf_counter() - t1
    return {"value": len(hist) / dt, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "sample": "mixing pass + %d ALS iterations of the same decomposition, numpy FP64, %.1f s"
                      % (len(hist), dt),
            "cpu_model": _cpu_model(), "host_logical_cpus": os.cpu_count(),
            "single_thread": {"value": len(hist1) / dt1, "seconds": dt1}}


if __name__ == "__main__":
    main()
