"""Benchmark: messenger-field Wiener-filter solves per second on one MI355X.

Workload (the nside 512 temperature problem): HEALPix nside 512, lmax 1024,
C_l = 6000/(l(l+1)) exp(-(l/800)^2), noise variance 30^2/hits with hits = 1 + 19 cos^2 theta
(5 % seeded jitter), |z| < 0.15 band plus 100 discs of 3 deg masked.  One step = one Wiener
filter solve of 300 messenger iterations at lambda = 1 in FP64 (each iteration: pixel
update, forward SHT, harmonic update, inverse SHT), one map, inputs resident in HBM.

Prints one JSON line.  Besides solves/s it reports the SHT-pair FLOP/s, per-solve latency
percentiles, the roofline position of the dominant kernel (timed with HIP events on the
plan's stream) and the CPU oracle timed on a bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WF solves/s & SHT-pair FLOP/s at nside=512; p50/p99 latency at 1e-5 rel err"
PEAK_FP64_VALU = 256 * 4 * 16 * 2 * 2.4e9   # CUs x SIMDs x lanes x (FMA = 2 flop) x clock
KERNELS = ["pixel_update", "fft_fwd", "leg_analysis", "harmonic", "leg_synth", "fft_inv"]


def cpu_baseline(nside, lmax, iters_sample, wl, d_host, M):
    """The FP64 oracle as it stands, all host cores, a bounded number of iterations."""
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    oracle.solve(nside, lmax, wl.cl, M, M * d_host, niter=iters_sample)
    dt = time.perf_counter() - t0
    per_iter = dt / iters_sample
    return {"value": 1.0 / (per_iter * 300.0), "unit": "solves/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d of the 300 messenger iterations of the nside 512 / lmax 1024 solve "
                      "(%.1f s, FFT phi step), extrapolated to one solve" % (iters_sample, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=300, help="messenger iterations per solve")
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--lmax", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--no-graph", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the solver on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1210_4931_amd import mfwf
    from paper_1210_4931_amd import workloads as W

    nside, lmax, K = args.nside, args.lmax, args.iters
    wl = W.config2(0, nside, lmax)
    dev = torch.device("cuda:0")
    plan = mfwf.Plan(nside, lmax, max_batch=1)
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x)).to(dev, dt)  # noqa
    plan.set_covariances(wl.cl, t(1.0 / wl.noise_var), t(wl.mask, torch.uint8))
    # d = Y(signal alm) + noise, built on the device with the library's own synthesis
    sig = plan.sht_inv(t(wl.signal_alm[None], torch.complex128))
    d = sig + t(np.sqrt(wl.noise_var) * wl.noise_white)[None]
    torch.cuda.synchronize()

    use_graph = not args.no_graph
    for _ in range(args.warmup):
        plan.solve(d, iters=K, use_graph=use_graph, want_map=False)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        plan.solve(d, iters=K, use_graph=use_graph, want_map=False)  # synchronises its stream
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    # per-kernel mean durations with HIP events on the plan's stream
    kt = plan.time_kernels(nmaps=1, reps=20)
    work, full, npair, fftmax = plan.work()
    leg_flops = 7.0 * work        # per direction: 3 (FP64 recurrence) + 4 (complex x real FMA)
    sht_pair_flops = 2.0 * leg_flops
    ktimes = dict(zip(KERNELS, kt))
    dom = max(("leg_analysis", "leg_synth"), key=lambda k: ktimes[k])
    achieved = leg_flops / (ktimes[dom] * 1e-3)
    iter_ms = ms_per_step / K
    pair_ms = ktimes["fft_fwd"] + ktimes["leg_analysis"] + ktimes["leg_synth"] + ktimes["fft_inv"]

    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "temperature Wiener filter, HEALPix nside %d, lmax %d, %d "
                               "messenger iterations at lambda=1, 1 map, FP64" % (nside, lmax, K),
                   "nside": nside, "lmax": lmax, "iterations": K, "batch": 1,
                   "graph": use_graph},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99))},
        "iteration_ms": iter_ms,
        "sht_pair_tflops": sht_pair_flops / (pair_ms * 1e-3) / 1e12,
        "kernel_ms": ktimes,
        "legendre_triples": {"evaluated": work, "full_triangle": full},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12,
                     "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU, "traffic": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nside, lmax, args.cpu_iters, wl,
                                           d.cpu().numpy()[0], wl.mask / wl.noise_var)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
