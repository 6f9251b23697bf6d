"""Benchmark: TEI Gram assembly on one MI355X.

A step is one pass of the hot path over the workload: the canonical Newton
kernel (tc_newton_kernel) and the TEI/Coulomb matrix J = sum_k c_k
G1_k o G2_k o G3_k (tc_tei_gram: Toeplitz products or FFT convolutions,
Grams, Hadamard/sum over k), with the side matrices already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]
                    [--prec ozaki8|fp64|fp32|bf16x3|bf16x6] [--no-cpu-baseline] [--no-extra]

Prints ONE JSON line.
  value       F / t, F = sum_l R_N (2 n^2 R_f + 2 n R_f^2): the algorithmic
              flops of the Toeplitz-Gram method (the same F for every route,
              so the FFT route shows as a higher rate of the same work).
  routes      ms per step of each (precision, Toeplitz algorithm) pair.
  roofline    the dominant kernel of the headline route, timed per launch with
              HIP events recorded by the library on the launch stream
              (tc_profile_*) over a second timed region of K steps, against
              the peak of its arithmetic or of HBM.  While timing kernels the
              library runs the three modes in turn (each kernel alone on the
              device); the headline region runs them concurrently.
  rows        the adjoint (2048 cells, R_f=512, forward + backward of w^T J w),
              the 64-instance batched workload, the Coulomb entries of the
              4096-cell functions against a 64-term density, and the density
              fitting + pivoted Cholesky of the factorised TEI matrix of the
              4096-cell products, per-call times.
  cpu_baseline  the FP64 oracle on a bounded sample (columns of J).
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

# published MI355X dense peaks
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "int8": 5000.0}  # TFLOP/s (TOP/s)
HBM_GBS = 8000.0
PREC_DTYPE = {"fp64": "f64", "fp32": "f32", "ozaki8": "i8", "bf16x3": "bf16", "bf16x6": "bf16"}
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
    ap.add_argument("--prec", default="ozaki8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the route comparison and the adjoint/batched rows")
    ap.add_argument("--cpu-cols", type=int, default=0,
                    help="columns of J in the oracle sample (0 = size for ~15 s)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the benchmark, run one device-to-device copy of MIB MiB (a "
                         "plain copy kernel of known size, used to scale HBM byte counters)")
    return ap.parse_args()


def timed(fn, steps, warmup, torch):
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
    ps = []
    for l in range(3):
        t, a, cc, p = oracle.newton_kernel(w.n[l], w.h[l], w.R_N, w.u0, w.hu)
        ps.append(p)
    c = a * w.h[0] * w.h[1] * w.h[2]
    per_col = sum(w.R_N * (2.0 * nl * nl + 2.0 * nl * w.R_f) for nl in w.n)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(0)
    if cols_req <= 0:
        t0 = time.perf_counter()
        oracle.tei_gram_columns(c, ps, w.U, [0])
        dt = time.perf_counter() - t0
        cols_req = int(max(1, min(64, 12.0 / max(dt, 1e-3))))
    cols = rng.choice(w.R_f, size=min(cols_req, w.R_f), replace=False)
    t0 = time.perf_counter()
    Jc = oracle.tei_gram_columns(c, ps, w.U, cols)
    dt = time.perf_counter() - t0
    # the same columns with plain (uncompensated) FP64 sums: the fair speed baseline
    t0 = time.perf_counter()
    oracle.tei_gram_columns(c, ps, w.U, cols, compensated=False)
    dt_plain = time.perf_counter() - t0
    flops = per_col * len(cols)
    out = {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "sample": (f"{len(cols)} of {w.R_f} columns of J ({flops:.3g} algorithmic flops, "
                      f"{dt:.1f} s), compensated FP64 oracle"),
           "plain_fp64_value": flops / dt_plain / 1e9,
           "plain_fp64_s": dt_plain,
           "cpu_model": cpu_model()}
    return out, cols, Jc


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def sampled_error(J, Jc, S):
    """Normalised error max |dJ_ij| / sqrt(J_ii J_jj) over the sampled columns
    S of J against the oracle's columns Jc ([len(S)][R_f]); rows outside S use
    the GPU diagonal."""
    block = Jc[:, S]
    d = np.diag(block)
    dg = np.sqrt(np.abs(np.diag(J)))
    return float(np.max(np.abs(J[:, S] - Jc.T) / np.outer(dg, np.sqrt(d))))


def kernel_roofline(name, per_launch_ms, w, prec, cls=None):
    """Algorithmic work of one launch of `name` on workload w (one mode) and
    the matching roofline.  cls: the term classes when the int8 FFT route
    runs (the int8 Gram then processes the terms of class != -2, and the FFT
    convolution transforms those of class -1 and convolves those of class
    B >= 0 directly over 2B + 1 lags); otherwise every kernel takes all terms."""
    n, R_f, R_N = w.n[0], w.R_f, w.R_N
    if cls is not None and name == "gram_i8":
        R_N = int((cls != -2).sum())
    s = per_launch_ms * 1e-3
    peak = PEAK["int8" if name.endswith("_i8") else "fp32" if name.endswith("_f32")
                else "bf16" if name.endswith("_bf16") else "fp64"]
    if name in ("gram_i8", "gram_f64", "gram_f32", "gram_bf16"):
        # U^T W_k for every k; G_k is symmetric, so the algorithm needs its
        # upper triangle only: R_f (R_f + 1) / 2 entries of 2n flops each
        flops = 1.0 * n * R_f * (R_f + 1) * R_N
        out = {"bound": "mfma", "achieved": flops / s / 1e12, "unit": "TFLOP/s", "peak": peak,
               "work": f"n R_f (R_f+1) R_N = {flops:.4g} flops per launch (upper triangles)"}
        if name == "gram_i8":
            # executed matrix-core work: 10 slice products over the padded
            # upper-triangle tiles (the counter SQ_INSTS_VALU_MFMA_MOPS_I8 x 512)
            n_pad = -(-n // 128) * 128
            R_f_pad = -(-R_f // 64) * 64
            T = 128 if (R_f >= 256 and R_f_pad % 128 == 0) else 64
            nt = R_f_pad // T
            ex = 10 * 2.0 * n_pad * T * T * (nt * (nt + 1) // 2) * R_N
            out["executed"] = {"TOP/s": ex / s / 1e12, "frac": ex / s / 1e12 / PEAK["int8"],
                               "ops": ex}
    elif name in ("toeplitz_i8", "toeplitz_f64", "toeplitz_f32", "toeplitz_bf16"):
        flops = 2.0 * n * n * R_f * R_N
        out = {"bound": "mfma", "achieved": flops / s / 1e12, "unit": "TFLOP/s", "peak": peak,
               "work": f"2 n^2 R_f R_N = {flops:.4g} flops per launch"}
        if name == "toeplitz_i8":
            ex = 10 * flops
            out["executed"] = {"TOP/s": ex / s / 1e12, "frac": ex / s / 1e12 / PEAK["int8"]}
    elif name in ("fft_conv", "fft_conv_split"):
        # FP64 vector work of the spectral product and the inverse transform:
        # per (k, j) the complex product and the real-FFT twist over M + 1
        # frequencies (14 flops each) and a complex M-point inverse FFT
        # (5 M log2 M, the conventional count); bound by the FP64 vector ALUs
        M = 1
        while 2 * M < 2 * n - 1:
            M *= 2
        lg = max(1, M.bit_length() - 1)
        n_fft, n_out, direct = R_N, R_N, 0.0
        if cls is not None and name == "fft_conv_split":
            n_fft = int((cls == -1).sum())
            n_out = int((cls != -2).sum())
            direct = float(sum(2 * (2 * int(b) + 1) for b in cls if b >= 0))
        flops = R_f * (n_fft * (5.0 * M * lg + 14.0 * (M + 1)) + direct * n)
        out = {"bound": "alu", "achieved": flops / s / 1e12, "unit": "TFLOP/s",
               "peak": PEAK["fp64"],
               "work": f"R_f (T_fft (5 M log2 M + 14 (M+1)) + sum_narrow 2 (2B+1) n) = {flops:.4g} "
                       f"FP64 flops per launch (T_fft = {n_fft} transformed terms)"}
        out_bytes = (4 if name == "fft_conv_split" else 8) * n_out * R_f * n
        in_bytes = 16 * (M + 1) * (R_f + R_N)
        out["hbm_bytes"] = out_bytes + in_bytes
        out["hbm_GBs"] = (out_bytes + in_bytes) / s / 1e9
    elif name == "hadamard_sum":
        # reads the upper triangles of the 3 R_N Grams, writes all of J
        byts = 8.0 * (3 * R_N * R_f * (R_f + 1) / 2 + R_f * R_f)
        out = {"bound": "hbm", "achieved": byts / s / 1e9, "unit": "GB/s", "peak": HBM_GBS,
               "work": f"8 B (3 R_N R_f (R_f+1)/2 + R_f^2) = {byts:.4g} bytes per launch"}
    else:
        return None
    out["frac"] = out["achieved"] / out["peak"]
    out["kernel"] = name
    out["kernel_ms"] = per_launch_ms
    out["traffic"] = measured_traffic(name, w)
    return out


# Library kernel name -> HIP source it is compiled from.
KERNEL_SOURCE = {"gram_i8": "ozaki.hip", "toeplitz_i8": "ozaki.hip", "split_rows": "ozaki.hip",
                 "fft_conv_split": "fft.hip", "fft_conv": "fft.hip", "rfft_rows": "fft.hip",
                 "gram_f64": "gram.hip", "toeplitz_f64": "toeplitz.hip",
                 "gram_f32": "fp32.hip", "toeplitz_f32": "fp32.hip",
                 "gram_bf16": "bf16.hip", "toeplitz_bf16": "bf16.hip",
                 "hadamard_sum": "reduce.hip"}


def measured_traffic(name, w):
    """HBM bytes per launch of kernel `name` from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by
    what the counter reads for a copy kernel of known size), or None when
    there is no summary for this kernel and workload or the kernel's source
    has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles",
                        f"hbm_traffic_n{w.n[0]}_rf{w.R_f}_rn{w.R_N}.md")
    src = KERNEL_SOURCE.get(name)
    if src is None or not os.path.exists(path):
        return None
    with open(os.path.join(ROOT, "paper_1504_06289_amd", "csrc", src), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        # | kernel | source | sha256 | FETCH KiB | WRITE KiB | fetch x | write x | bytes |
        if len(cells) == 8 and cells[0] == name:
            if cells[1] != src or cells[2] != digest:
                return None
            return float(cells[7])
    return None


def mfma_pct(prof, w, prec, cls=None):
    """% of the dtype's MFMA peak executed by the matrix-core kernels of one
    step (Gram and direct Toeplitz products), from their measured times."""
    out = {}
    for name in ("gram_i8", "toeplitz_i8", "gram_f64", "toeplitz_f64", "gram_f32",
                 "toeplitz_f32", "gram_bf16", "toeplitz_bf16"):
        if name in prof:
            r = kernel_roofline(name, prof[name][0] / prof[name][1], w, prec, cls)
            ex = r.get("executed", {"frac": r["frac"]})["frac"]
            out[name] = round(100.0 * ex, 2)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1504_06289_amd as tc
    from paper_1504_06289_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = wl.config(args.workload)
    U = [torch.from_numpy(u).to(dev) for u in w.U]
    F = w.flops()
    shapes = sorted(set((nl, w.R_f, w.R_N) for nl in w.n))

    def step(prec):
        t, c, p = tc.newton_kernel(w.n[0], w.h[0], w.R_N, w.u0, w.hu, device=dev)
        # the weights through pinned memory: an asynchronous copy, so the host
        # does not wait for the previous step before enqueueing this one
        cd = torch.from_numpy(c).pin_memory().to(dev, non_blocking=True)
        return tc.tei_gram(cd, [p, p, p], U, prec=prec)

    def with_algo(prec, algo, fn):
        for s in shapes:
            tc.tune_set(*s, prec, algo)
        try:
            return fn()
        finally:
            for s in shapes:
                tc.tune_set(*s, prec, "auto")

    # headline: the chosen precision, algorithm picked by the autotuner
    t, c, p = tc.newton_kernel(w.n[0], w.h[0], w.R_N, w.u0, w.hu, device=dev)
    tuned = tc.autotune(torch.from_numpy(c).to(dev), [p, p, p], U, prec=args.prec)
    ms = timed(lambda: step(args.prec), args.steps, args.warmup, torch)
    value = F / (ms * 1e-3) / 1e9
    # host time of one tc_tei_gram call (enqueue only; the GPU runs behind)
    t_, c_, p_ = tc.newton_kernel(w.n[0], w.h[0], w.R_N, w.u0, w.hu, device=dev)
    cd_ = torch.from_numpy(c_).to(dev)
    host = []
    for _ in range(max(3, args.steps)):
        torch.cuda.synchronize()
        h0 = time.perf_counter()
        tc.tei_gram(cd_, [p_, p_, p_], U, prec=args.prec)
        host.append((time.perf_counter() - h0) * 1e3)
    torch.cuda.synchronize()
    host_ms = float(np.median(host))

    # per-kernel times: a second timed region of the same K steps with the
    # library's HIP-event timing on (the three modes then run in turn, so each
    # duration is the kernel's own)
    tc.profile_enable(True)
    tc.profile_read()
    ms_prof = timed(lambda: step(args.prec), args.steps, 0, torch)
    prof = tc.profile_read()
    tc.profile_enable(False)
    K = args.steps
    kernels = {k: {"total_ms": round(v[0] / K, 4), "launches": v[1] // K} for k, v in prof.items()}
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    # terms the int8 Gram processes on the FFT route (smooth terms take the
    # low-rank path); every term otherwise
    cls = tc.term_classes(p)
    route_cls = None
    if args.prec == "ozaki8" and tc.tune_get(w.n[0], w.R_f, w.R_N, args.prec) == "fft":
        route_cls = cls
    roof = kernel_roofline(dom[0], dom[1][0] / dom[1][1], w, args.prec, route_cls)

    out = {
        "metric": "TEI Gram assembly GFLOP/s + % MFMA peak, mixed vs FP64, at rel err \u22641e-7",
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "value_kind": ("dense-equivalent: F / t with F = sum over modes of R_N (2 n^2 R_f + "
                       "2 n R_f^2), the flops of the direct Toeplitz-Gram formulation; the FFT "
                       "route and the rank-32 smooth-term path execute fewer operations"),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_DESC[args.workload]}",
                   "n": w.n[0], "R_N": w.R_N, "R_f": w.R_f, "precision": args.prec,
                   "algorithm": tc.tune_get(w.n[0], w.R_f, w.R_N, args.prec),
                   "flops_per_step": F},
        "roofline": roof,
        "mfma_peak_pct": mfma_pct(prof, w, args.prec, route_cls),
        "other_rooflines": {k: {"achieved": round(r["achieved"], 2), "unit": r["unit"],
                                "frac": round(r["frac"], 4), "kernel_ms": round(r["kernel_ms"], 4)}
                            for k, r in ((k, kernel_roofline(k, v[0] / v[1], w, args.prec, route_cls))
                                         for k, v in prof.items() if k != dom[0]) if r},
        "term_classes": {"narrow": int((cls >= 0).sum()), "smooth": int((cls == -2).sum()),
                         "general": int((cls == -1).sum())},
        "kernels_one_step": kernels,
        "profiled_ms_per_step": round(ms_prof, 4),
        "host_enqueue_ms_tei_gram": round(host_ms, 4),
        "autotune_ms_per_mode": {"direct": round(tuned[0][0], 4), "fft": round(tuned[0][1], 4)},
    }
    for s in shapes:
        tc.tune_set(*s, args.prec, "auto")

    if not args.no_extra:
        routes = {}
        for prec in ("fp64", "fp32", "bf16x3", "bf16x6", "ozaki8"):
            for algo in ("direct", "fft"):
                k = max(2, args.steps // 3)
                routes[f"{prec}/{algo}"] = round(
                    with_algo(prec, algo, lambda: timed(lambda: step(prec), k, 1, torch)), 4)
        out["routes_ms_per_step"] = routes
        best64 = min(routes["fp64/direct"], routes["fp64/fft"])
        out["speedup_mixed_vs_fp64"] = {
            "direct": round(routes["fp64/direct"] / routes["ozaki8/direct"], 3),
            "best_route": round(best64 / min(routes["ozaki8/direct"], routes["ozaki8/fft"]), 3)}
        out["rows"] = extra_rows(tc, wl, torch, dev, args)

    if not args.no_cpu_baseline:
        base, S, Jc = cpu_baseline(w, args.cpu_cols)
        out["cpu_baseline"] = base
        # error of the timed step's J (bitwise reproducible, so one more step
        # gives the same J) and of the binary64 route's J on the oracle's columns
        J_head = step(args.prec).cpu().numpy()
        J_64 = with_algo("fp64", "fft" if w.n[0] <= 4096 else "direct",
                         lambda: step("fp64")).cpu().numpy()
        out["e_J"] = {args.prec: sampled_error(J_head, Jc, S), "fp64": sampled_error(J_64, Jc, S),
                      "columns": int(len(S)),
                      "metric": "max_ij |dJ_ij| / sqrt(J_ii J_jj) over the sampled columns"}
    print(json.dumps(out), flush=True)
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()


def extra_rows(tc, wl, torch, dev, args):
    rows = {}
    # adjoint: forward (Grams saved) + backward of f = w^T J w, 2048 cells, R_f = 512
    w5 = wl.config("c5")
    U5 = [torch.from_numpy(u).to(dev) for u in w5.U]
    t, c, p = tc.newton_kernel(w5.n[0], w5.h[0], w5.R_N, w5.u0, w5.hu, device=dev)
    cd = torch.from_numpy(c).to(dev)
    wv = torch.from_numpy(w5.meta["w"]).to(dev)
    Jbar = torch.outer(wv, wv).contiguous()
    for prec in ("fp64", "ozaki8"):
        def fb():
            J, G = tc.tei_gram(cd, [p, p, p], U5, prec=prec, save_G=True)
            return tc.tei_gram_backward(cd, [p, p, p], U5, Jbar, G=G, prec=prec)
        rows[f"adjoint_c5_{prec}_ms"] = round(timed(fb, 3, 1, torch), 4)
    # batched: 64 independent instances in one call
    insts = wl.batched_instances(64, seed=0)
    kern = {}
    batch = []
    for wi in insts:
        key = wi.n[0]
        if key not in kern:
            t, c, p = tc.newton_kernel(wi.n[0], wi.h[0], wi.R_N, wi.u0, wi.hu, device=dev)
            kern[key] = (torch.from_numpy(c).to(dev), p)
        c, p = kern[key]
        batch.append((c, [p, p, p], [torch.from_numpy(u).to(dev) for u in wi.U]))
    Fb = sum(wi.flops() for wi in insts)
    for prec in ("fp64", "ozaki8"):
        # direct/FFT choice per distinct mode shape and (int8) the batch route
        # from the autotuner; the batch then runs as one captured graph
        tc.autotune_batched(batch, prec=prec)
        route = tc.batch_tune_get(batch, prec)
        msb = timed(lambda: tc.tei_gram_batched(batch, prec=prec), 2, 1, torch)
        g = tc.TeiGramGraph(batch, prec=prec)
        msg = timed(g.replay, 3, 1, torch)
        del g
        rows[f"batched_c4_{prec}_route"] = route
        rows[f"batched_c4_{prec}_ms"] = round(msb, 3)
        rows[f"batched_c4_{prec}_graph_ms"] = round(msg, 3)
        rows[f"batched_c4_{prec}_GFLOPs"] = round(Fb / (msg * 1e-3) / 1e9, 1)
        if prec == "ozaki8":
            # every batch route, eager (A/B of the work queue against fork-join)
            per_route = {}
            for r in ("fork_join", "queue", "queue_t64", "queue_k2", "queue_t64_k2"):
                tc.batch_tune_set(batch, prec, r)
                per_route[r] = round(timed(lambda: tc.tei_gram_batched(batch, prec=prec), 2, 1,
                                           torch), 3)
            tc.batch_tune_set(batch, prec, route)
            rows["batched_c4_ozaki8_ms_per_route"] = per_route
            # the persistent Gram launch of the queue route, timed by the library
            tc.batch_tune_set(batch, prec, "queue_t64")
            tc.profile_enable(True)
            tc.profile_read()
            tc.tei_gram_batched(batch, prec=prec)
            prof = tc.profile_read()
            tc.profile_enable(False)
            tc.batch_tune_set(batch, prec, route)
            gq = prof.get("gram_queue")
            if gq:
                # ten int8 slice products over the upper triangles of the
                # Grams of every listed term (all terms on the direct route,
                # the non-smooth ones on the int8 FFT route)
                ops = 0.0
                for wi, (c, p3, U3) in zip(insts, batch):
                    nl, R_f = wi.n[0], wi.R_f
                    if tc.tune_get(nl, R_f, wi.R_N, prec) == "fft" and nl <= 4096:
                        nk = int((tc.term_classes(p3[0]) != -2).sum())
                    else:
                        nk = wi.R_N
                    ops += 3 * 10.0 * nk * nl * R_f * (R_f + 1)
                rows["batched_c4_gram_queue"] = {
                    "kernel_ms": round(gq[0], 4), "launches": gq[1],
                    "TOP/s": round(ops / (gq[0] * 1e-3) / 1e12, 1),
                    "frac_int8_peak": round(ops / (gq[0] * 1e-3) / 1e12 / PEAK["int8"], 4),
                    "work": "10 slice products x n R_f (R_f + 1) per listed term and mode"}
    rows["batched_c4_flops"] = Fb
    # Coulomb entries of the 4096-cell functions against a 64-term density
    w3 = wl.config("c3")
    R_rho = 64
    V, d = wl.density(w3.n, w3.b, R_rho, seed=1)
    t, c, p = tc.newton_kernel(w3.n[0], w3.h[0], w3.R_N, w3.u0, w3.hu, device=dev)
    cd = torch.from_numpy(c).to(dev)
    U3 = [torch.from_numpy(u).to(dev) for u in w3.U]
    V3 = [torch.from_numpy(v).to(dev) for v in V]
    dd = torch.from_numpy(d).to(dev)
    msc = timed(lambda: tc.coulomb(cd, [p, p, p], U3, V3, dd), 5, 1, torch)
    n3 = w3.n[0]
    Fc = 3.0 * w3.R_N * (2.0 * n3 * n3 * R_rho + 2.0 * n3 * w3.R_f * R_rho)
    tc.profile_enable(True)
    tc.profile_read()
    tc.coulomb(cd, [p, p, p], U3, V3, dd)
    prof = tc.profile_read()
    tc.profile_enable(False)
    cg = prof.get("cross_gram_f64")
    rows["coulomb_c3_rho64_fp64_ms"] = round(msc, 4)
    rows["coulomb_c3_rho64_fp64_GFLOPs"] = round(Fc / (msc * 1e-3) / 1e9, 1)
    if cg:
        ms_cg = cg[0] / cg[1]
        fl = 2.0 * n3 * w3.R_f * R_rho * w3.R_N
        rows["coulomb_cross_gram_f64"] = {"kernel_ms": round(ms_cg, 4),
                                          "TFLOP/s": round(fl / (ms_cg * 1e-3) / 1e12, 2),
                                          "frac": round(fl / (ms_cg * 1e-3) / 1e12 / PEAK["fp64"], 4)}
    rows["coulomb_kernels"] = {k: round(v[0], 4) for k, v in prof.items()}
    # 1D density fitting of the three side matrices of the 4096-cell products
    # (tolerance 1e-6), the Grams of the fitted rows, and the pivoted Cholesky
    # of the factorised TEI matrix (tolerance 1e-8 of its trace)
    import time as _time
    for _rep in range(2):  # the second pass is reported
        torch.cuda.synchronize()
        t0 = _time.perf_counter()
        fits = [tc.density_fit(U3[l], 1e-6) for l in range(3)]
        torch.cuda.synchronize()
        t1 = _time.perf_counter()
        R = max(f[3] for f in fits)
        Ud = [f[0][:R].contiguous() for f in fits]
        Vd = [f[1][:, :R].contiguous() for f in fits]
        J, G = tc.tei_gram(cd, [p, p, p], Ud, prec="fp64", save_G=True)
        torch.cuda.synchronize()
        t2 = _time.perf_counter()
        Lb, piv, res = tc.tei_cholesky(cd, Vd, [G[l].contiguous() for l in range(3)], 1e-8)
        torch.cuda.synchronize()
        t3 = _time.perf_counter()
    rows["tei_cholesky_c3"] = {"fit_ranks": [int(f[3]) for f in fits], "R_B": int(Lb.shape[0]),
                               "fit_ms": round(1e3 * (t1 - t0), 2),
                               "fitted_grams_ms": round(1e3 * (t2 - t1), 2),
                               "cholesky_ms": round(1e3 * (t3 - t2), 2)}
    # nuclear potential matrix of the 4096-cell products: three nuclei (a
    # water-like geometry in bohr) on the grid of the functions
    geom = np.array([[0.0, 0.0, 0.0], [1.43, 1.11, 0.0], [-1.43, 1.11, 0.0]])
    Zn = np.array([8.0, 1.0, 1.0])
    posn = [[int((x + w3.b) / w3.h[l]) for l, x in enumerate(g)] for g in geom]
    msn = timed(lambda: tc.nuclear(cd, [p, p, p], U3, w3.h, Zn, posn), 3, 1, torch)
    tc.profile_enable(True)
    tc.profile_read()
    tc.nuclear(cd, [p, p, p], U3, w3.h, Zn, posn)
    prof = tc.profile_read()
    tc.profile_enable(False)
    dg = prof.get("diag_gram_f64")
    Tn = len(Zn) * w3.R_N
    # upper triangles over every cell: dense-equivalent, since groups of narrow
    # terms contract only over the cells near their nucleus
    fl = 3 * Tn * 2.0 * n3 * w3.R_f * (w3.R_f + 1) / 2
    row = {"ms": round(msn, 3), "nuclei": len(Zn), "terms": Tn}
    if dg:
        ms_dg = dg[0] / dg[1]
        row["diag_gram_f64"] = {"kernel_ms": round(ms_dg, 4),
                                "dense_equiv_TFLOP/s": round(fl / 3 / (ms_dg * 1e-3) / 1e12, 2),
                                "frac": round(fl / 3 / (ms_dg * 1e-3) / 1e12 / PEAK["fp64"], 4)}
    rows["nuclear_c3_h2o"] = row
    # canonical-to-Tucker transform of a density with 2048 terms on the
    # 4096-cell grid, Tucker ranks 24, two sweeps, 20 subspace steps
    Vt_, dt_ = wl.density(w3.n, w3.b, 2048, seed=5)
    At = [torch.from_numpy(v).to(dev) for v in Vt_]
    ctd = torch.from_numpy(dt_).to(dev)
    c2t = lambda: tc.canonical_to_tucker(ctd, At, (24, 24, 24), 2, 20)
    msc2t = timed(c2t, 2, 1, torch)
    tc.profile_enable(True)
    tc.profile_read()
    c2t()
    prof = tc.profile_read()
    tc.profile_enable(False)
    rows["c2t_n4096_R2048_r24"] = {"ms": round(msc2t, 2),
                                   "kernels_ms": {k: round(v[0], 3) for k, v in prof.items()}}
    # lattices of hydrogen atoms (Z = 1, spacing 2 bohr): the interaction
    # energy of the 256^3 lattice on the n = 128 L grid, and the assembled
    # lattice sum of the 128^3 lattice on a 34304-cell grid, each with the
    # generation of its kernel vectors on the device
    import math as _m
    L, n0 = 256, 128
    h = 2.0 / n0
    lo, hu = _m.log(1e-14), 0.25
    R_N = int(_m.ceil((_m.log(200.0) - lo) / hu)) + 1

    def energy():
        t, c, p = tc.newton_kernel(n0 * L, h, R_N, lo, hu, device=dev)
        return tc.lattice_energy(torch.from_numpy(c).to(dev), [p, p, p], [h, h, h], n0,
                                 (L, L, L), 1.0)
    mse = timed(energy, 5, 1, torch)
    rows["lattice_energy_L256"] = {"ms": round(mse, 3), "E": energy(), "R_N": R_N,
                                   "n": n0 * L}
    L, n0 = 128, 268
    h = 2.0 / n0
    R_N = int(_m.ceil((_m.log(2e4 / h) - lo) / hu)) + 1
    t, c, p = tc.newton_kernel(n0 * L, h, R_N, lo, hu, device=dev)
    msk = timed(lambda: tc.newton_kernel(n0 * L, h, R_N, lo, hu, device=dev), 5, 1, torch)
    mss = timed(lambda: tc.lattice_sum([p, p, p], n0, (L, L, L)), 5, 1, torch)
    n = n0 * L
    rows["lattice_sum_L128"] = {"kernel_ms": round(msk, 3), "sum_ms": round(mss, 3),
                                "R_N": R_N, "n": n,
                                "sum_GBps_algorithmic": round(
                                    3 * 8.0 * R_N * (3 * n - 1) / (mss * 1e-3) / 1e9, 1)}
    return rows


if __name__ == "__main__":
    main()
