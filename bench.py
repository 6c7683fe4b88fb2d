"""Benchmark: ALS iterations per second of CPRAND-MIX on a 400x400x400 FP32
tensor (rank 10, column congruence 0.5, 1% noise, S = 10 R ceil(ln R) = 300,
P-hat = 2^14, stop after 200 iterations, |dF| <= 1e-4 or F >= 1 - 1.2 eta).

One step = one whole decomposition on the GPU: ||X||, random signs, the
mixing pass along every mode, the factor mixes, then the ALS loop (sample,
sampled Khatri-Rao rows, fiber gather, MTTKRP on MFMA, FP64 solve,
normalisation, factor remix, sampled fit estimate, stop test).  `value` is
outer iterations per second of the whole step (mixing included).

Also reported (not part of `value`):
  - loop-only iterations per second and the one-time setup time,
  - plain CPRAND (no mixing) on the same tensor,
  - the roofline of the dominant kernel (the mixing pass), from HIP events
    recorded around each pass inside the timed steps,
  - a gather/MTTKRP throughput leg: one cprand_mttkrp_sampled launch over
    many samples of the mixed tensor, timed with HIP events,
  - the CPU oracle (numpy FP64) on a bounded sample of the same work.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--layout", type=int, default=1, help="0: mode-major copies of X-hat, 1: strided gathers")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1701_06600_amd as P
    import synth

    w = synth.WORKLOADS["cprand-400cube-f32"]
    R, S = w.R, w.S
    dev = torch.device("cuda:0")
    prob = synth.problem_for(w)
    print("[bench] generating %s on the GPU" % (w.name,), flush=True)
    X = synth.device_tensor(prob, dev, "f32")
    Xv = P.View(X, w.dims)
    init = [torch.as_tensor(M, dtype=torch.float32, device=dev) for M in prob.init]
    torch.cuda.synchronize()

    def opts(mix):
        return P.make_opts(R, S, P_hat=w.P_hat, max_iters=w.max_iters, seed=w.seed, tol=w.tol,
                           fit_target=w.fit_target, mix=P.MIX_FFT if mix else P.MIX_NONE,
                           layout=args.layout, use_graph=1)

    plan = P.Plan(Xv, opts(True))

    def step():
        A = [M.clone() for M in init]
        return plan.run(Xv, A)

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
    mix_bytes = [P_el * (4 + 8)] + [P_el * 16] * 2       # pass 0 reads FP32, writes complex64
    mix_launch_ms = sum(mix_ms) / 3
    mix_achieved = sum(mix_bytes) / 3 / (mix_launch_ms * 1e-3) / 1e9

    # plain CPRAND on the same tensor
    plan0 = P.Plan(Xv, opts(False))
    A0 = [M.clone() for M in init]
    plan0.run(Xv, A0)
    t2 = time.perf_counter()
    r0 = [plan0.run(Xv, [M.clone() for M in init]) for _ in range(max(1, args.steps))]
    torch.cuda.synchronize()
    plain_rate = sum(r["iters"] for r in r0) / (time.perf_counter() - t2)

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
        "config": {"workload": "CPRAND-MIX, 400x400x400 FP32, R=10, congruence 0.5, 1% noise, "
                               "S=300, P-hat=2^14, paper stop rule",
                   "layout": "strided X-hat gathers" if args.layout else "mode-major X-hat copies"},
        "iters_per_step": iters / args.steps,
        "final_fit_est": runs[-1]["fit_est"],
        "loop_iters_per_s": iters / (loop_ms * 1e-3),
        "setup_ms": setup_ms,
        "mix_pass_ms": mix_ms,
        "plain_cprand_iters_per_s": plain_rate,
        "plain_cprand_iters_per_step": r0[-1]["iters"],
        "gather_mttkrp": {"samples": Sg, "ms": g_ms, "useful_GBps": gather_gbs,
                          "frac_of_hbm": gather_gbs / HBM_PEAK_GBS},
        "roofline": {"kernel": "mix_pass_kernel", "bound": "hbm", "achieved": mix_achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": mix_achieved / HBM_PEAK_GBS,
                     "traffic": None},
    }

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(X, w, prob, iters / args.steps)
    print(json.dumps(out), flush=True)


def cpu_baseline(Xdev, w, prob, gpu_iters):
    """The oracle (numpy FP64) on the same tensor: the mixing pass plus a
    bounded number of ALS iterations; rate = iterations / wall time,
    directly comparable to `value` when the iteration count matches."""
    import numpy as np

    from oracle import cprand as OC
    from oracle.tensor import from_colmajor

    X = from_colmajor(Xdev.double().cpu().numpy(), w.dims)
    k = int(max(1, min(5, round(gpu_iters))))
    t0 = time.perf_counter()
    lam, A, hist = OC.cprand_mix(X, w.R, w.S, prob.init, w.seed, k, P_hat=w.P_hat)
    dt = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": len(hist) / dt, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "sample": "mixing pass + %d ALS iterations of the same decomposition, numpy FP64, %.1f s"
                      % (len(hist), dt)}


if __name__ == "__main__":
    main()
