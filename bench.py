"""Benchmark: TEI Gram assembly on one MI355X.

A step is one pass of the hot path over the workload: the canonical Newton
kernel (tc_newton_kernel) and the TEI/Coulomb matrix J = sum_k c_k
G1_k o G2_k o G3_k (tc_tei_gram: Toeplitz products, Grams, Hadamard/sum over
k), with the side matrices already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]
                    [--prec fp64|ozaki8] [--no-cpu-baseline]

Prints ONE JSON line.  GFLOP/s counts the algorithmic flops of the
Toeplitz-Gram method, F = sum_l R_N (2 n^2 R_f + 2 n R_f^2).
The roofline entry is for the dominant kernel (the implicit-Toeplitz
product): its launch (one mode, all R_N terms) is timed with HIP events on
the stream it runs on, and compared with the matrix-core peak of its dtype.
The cpu_baseline entry times the FP64 oracle on a bounded sample of the same
workload (a few columns of J) on this host's cores.
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

# published MI355X peaks (dense), TFLOP/s
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "int8": 5000.0}
PREC_DTYPE = {"fp64": "f64", "fp32": "f32", "ozaki8": "i8"}
PREC_PEAK = {"fp64": "fp64", "fp32": "fp32", "ozaki8": "int8"}
WORKLOAD_DESC = {
    "c1": "128-cell grid on [-10,10]^3, R_N=20 sinc terms, R_f=8 s-Gaussians",
    "c2": "1024-cell grid on [-10,10]^3, R_N=30 sinc terms, R_f=256 s/p Gaussian products",
    "c3": "4096-cell grid on [-12,12]^3, R_N=32 sinc terms, R_f=1024 s/p Gaussian products",
    "c5": "2048-cell grid on [-10,10]^3, R_N=30 sinc terms, R_f=512 s/p Gaussian products",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--prec", default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=0,
                    help="columns of J in the oracle sample (0 = size for ~15 s)")
    return ap.parse_args()


def timed_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms


def cpu_baseline(w, cols_req):
    from oracle import oracle
    c, ps = None, []
    for l in range(3):
        t, a, cc, p = oracle.newton_kernel(w.n[l], w.h[l], w.R_N, w.u0, w.hu)
        ps.append(p)
    c = a * w.h[0] * w.h[1] * w.h[2]
    per_col = sum(w.R_N * (2.0 * nl * nl + 2.0 * nl * w.R_f) for nl in w.n)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(0)
    if cols_req <= 0:
        # calibrate on one column, then size the sample for ~15 s
        t0 = time.perf_counter()
        oracle.tei_gram_columns(c, ps, w.U, [0])
        dt = time.perf_counter() - t0
        cols_req = int(max(1, min(64, 15.0 / max(dt, 1e-3))))
    cols = rng.choice(w.R_f, size=min(cols_req, w.R_f), replace=False)
    t0 = time.perf_counter()
    oracle.tei_gram_columns(c, ps, w.U, cols)
    dt = time.perf_counter() - t0
    flops = per_col * len(cols)
    return {
        "value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
        "sample": (f"{len(cols)} of {w.R_f} columns of J ({flops:.3g} algorithmic flops, "
                   f"{dt:.1f} s), compensated FP64 oracle"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1504_06289_amd as tc
    from paper_1504_06289_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = wl.config(args.workload)
    dev = torch.device("cuda:0")
    U = [torch.from_numpy(u).to(dev) for u in w.U]
    prec = args.prec
    F = w.flops()

    # kernel vectors per mode (equal h in all modes -> one set, aliased)
    state = {}

    def step(prec=prec):
        t, c, p = tc.newton_kernel(w.n[0], w.h[0], w.R_N, w.u0, w.hu, device=dev)
        cd = torch.from_numpy(c).to(dev, non_blocking=False)
        state["J"] = tc.tei_gram(cd, [p, p, p], U, prec=prec)

    ms = timed_steps(step, args.steps, args.warmup, torch)
    value = F / (ms * 1e-3) / 1e9

    # dominant kernel: one implicit-Toeplitz launch (one mode, all R_N terms)
    t, c, p = tc.newton_kernel(w.n[0], w.h[0], w.R_N, w.u0, w.hu, device=dev)
    Wbuf = torch.empty((w.R_N, w.R_f, w.n[0]), dtype=torch.float64, device=dev)
    ms_toep = timed_steps(lambda: tc.convolve(p, U[0], prec=prec, out=Wbuf),
                          max(args.steps, 5), 2, torch)
    toep_flops = 2.0 * w.n[0] * w.n[0] * w.R_f * w.R_N
    achieved = toep_flops / (ms_toep * 1e-3) / 1e12
    peak = PEAK_TFLOPS[PREC_PEAK[prec]]
    out = {
        "metric": "TEI Gram assembly GFLOP/s (mixed vs FP64, normalised error <= 1e-7)",
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_DESC[args.workload]}",
                   "n": w.n[0], "R_N": w.R_N, "R_f": w.R_f, "precision": prec,
                   "flops_per_step": F},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "toeplitz (W = T_k U, one mode, all terms)",
                     "kernel_ms": round(ms_toep, 4)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_cols)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
