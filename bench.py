"""Benchmark: messenger-field Wiener-filter solves per second on one MI355X.

Workload (the nside 512 temperature problem): HEALPix nside 512, lmax 1024,
C_l = 6000/(l(l+1)) exp(-(l/800)^2), noise variance 30^2/hits with hits = 1 + 19 cos^2 theta
(5 % seeded jitter), |z| < 0.15 band plus 100 discs of 3 deg masked.  One solve = 300
messenger iterations at lambda = 1 (each: pixel update, forward SHT, harmonic update, inverse
SHT) from s = 0; inputs are resident in HBM before timing.

Headline form: the batched FP32 form -- `--batch` right-hand sides (one signal, independent
seeded noise draws) solved together, Legendre contractions on the matrix cores, FP64 maps and
FFTs; its accuracy against the FP64 oracle (1e-5 relative) is checked by the GPU tests.  One
step = one batched solve, value = solved maps per second.  Reported beside it: the plain FP64
single-solve path (1 map, every step FP64) with its latency, the SHT-pair FLOP/s of both
forms, the roofline position of each form's dominant kernel (HIP events on the plan's stream),
the T, Q, U form, a serving stream of mixed-shape requests (solves/s and p50/p99 latency at
saturation and under Poisson arrivals at 0.8 of it) and the CPU oracle on a bounded sample
of the same solve.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WF solves/s & SHT-pair FLOP/s at nside=512; p50/p99 latency at 1e-5 rel err"
PEAK_FP64_VALU = 256 * 4 * 16 * 2 * 2.4e9     # 78.6 TFLOP/s: CUs x SIMDs x lanes x FMA x clock
PEAK_FP32_MFMA = 157.3e12                      # dense FP32 matrix-core peak
KERNELS = ["pixel_update", "fft_fwd", "leg_analysis", "harmonic", "leg_synth", "fft_inv"]
# the stages of the batched T, Q, U form, in the order mfwf_time_kernels reports them
POL_B_KERNELS = ["pixel_update", "fft_fwd", "gemm_analysis", "combine_filter", "gemm_synthesis", "fft_inv"]

PEAK_HBM = 8.0e12                              # HBM3E bytes/s

# HBM bytes per iteration of two kernels of the batched FP32 form (nside 512, lmax 1024, 64
# maps) from rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by the factors a 256 MiB copy gives:
# profiles/ring_step_and_gemms_nside512_lmax1024_b64_hbm_traffic.md.  The ring step's bytes
# depend on how many maps share a workgroup of each transform class (the tuned "g0", "g1":
# more maps per workgroup write larger column pieces), so they are kept per (g0, g1).  Valid only
# for the kernel source they were taken on, identified by the SHA-256 of the source file.
TRAFFIC = {
    "ring_step": {"bytes": {(1, 1): 4.362e+09, (2, 1): 3.9462e+09}, "source": "ringfft.hip",
                  "sha256": "c9b4266582b594104aa72a0f282339b23db43c2dc5f7bafaa90cdc95b24237aa"},
    # the analysis GEMM's, per (column tile choice "cta", lambda generated "lamgen")
    "gemm_analysis": {"bytes": {(1, 0): 5.3876e+09}, "source": "batched.hip",
                      "sha256": "cf741d30ae83034de945d059f9844b1e0fee8f93c8168cea03ce9daf44a0597d"},
}
# What the shader counters say limits the ring step (VALU issue and LDS bank conflicts, not
# HBM): profiles/batched_nside512_lmax1024_b64_shader_counters.md, same kernel sources.
RING_COUNTERS = {"valu_busy": [0.43, 0.53], "lds_bank_conflict_share": [0.25, 0.27],
                 "mfma_busy": 0.0, "hbm_traffic_over_algorithmic": {"g0=1,g1=1": 1.15, "g0=2,g1=1": 1.04},
                 "profile": "profiles/batched_nside512_lmax1024_b64_shader_counters.md"}


_T0 = time.perf_counter()


def note(msg):
    """Progress of a long run on stderr (the JSON result line stays alone on stdout)."""
    print("[bench %6.1f s] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


def measured_traffic(kernel, shape=None):
    """Counter-measured bytes per launch of `kernel` (per iteration for the ring step, for the
    plan's tuned (g0, g1)), or None where the source changed since or no figure was taken."""
    import hashlib
    t = TRAFFIC[kernel]
    b = t["bytes"].get(shape) if isinstance(t["bytes"], dict) else t["bytes"]
    if b is None:
        return None
    src = os.path.join(ROOT, "paper_1210_4931_amd", "csrc", t["source"])
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return b if h == t["sha256"] else None


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE_ONE_ITER = """
import json, sys, time
import numpy as np
sys.path.insert(0, %r)
import oracle
from paper_1210_4931_amd import workloads as W
wl = W.config2(0, %d, %d)
d = np.load(%r)
M = wl.mask / wl.noise_var
t0 = time.perf_counter()
oracle.solve(%d, %d, wl.cl, M, M * d, niter=1)
print(json.dumps({"seconds": time.perf_counter() - t0, "threads": oracle.num_threads()}))
"""


def cpu_baseline(nside, lmax, K, wl, d_host, M):
    """The FP64 oracle as it stands, timed on the host: with all cores, one solve with 1 and
    with 3 iterations (the difference gives the cost of an iteration, the rest the set-up);
    with OMP_NUM_THREADS=1 (a child process), one solve of 1 iteration, set-up included.
    Both extrapolated to K iterations; value = the all-core rate."""
    import subprocess
    import tempfile
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    oracle.solve(nside, lmax, wl.cl, M, M * d_host, niter=1)
    t1 = time.perf_counter()
    oracle.solve(nside, lmax, wl.cl, M, M * d_host, niter=3)
    t2 = time.perf_counter()
    per_iter = max((t2 - t1) - (t1 - t0), 1e-9) / 2.0
    setup = max((t1 - t0) - per_iter, 0.0)
    one = None
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "d.npy")
        np.save(path, d_host)
        code = _ORACLE_ONE_ITER % (ROOT, nside, lmax, path, nside, lmax)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           env=dict(os.environ, OMP_NUM_THREADS="1"), timeout=600)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
    out = {"value": 1.0 / (setup + K * per_iter), "unit": "solves/s", "cores": oracle.num_threads(),
           "kind": "oracle", "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "sample": "one solve of the nside %d / lmax %d problem with 1 and with 3 messenger "
                     "iterations on %d threads (%.1f s in all; %.2f s per iteration, %.2f s "
                     "set-up), extrapolated to %d iterations"
                     % (nside, lmax, oracle.num_threads(), t2 - t0, per_iter, setup, K)}
    if one is not None:
        out["single_core"] = {"value": 1.0 / (K * one["seconds"]), "unit": "solves/s",
                              "cores": one["threads"],
                              "sample": "one solve of 1 messenger iteration, set-up included "
                                        "(%.1f s), extrapolated to %d iterations"
                                        % (one["seconds"], K)}
    return out


def batched_extras(K, use_graph):
    """Other batched FP32 forms at 300 iterations: the nside 512 problem with B = 1 and
    B = 16 maps (the matrix-core kernels on 2 and 32 real columns), and the downgraded nside
    256 / lmax 512 problem with 64 right-hand sides, 32 Wiener-filter data sets and 32
    constrained-realisation fluctuation sources (Eq. 9), in one batch."""
    import torch
    from paper_1210_4931_amd import mfwf
    from paper_1210_4931_amd import workloads as W
    dev = torch.device("cuda:0")
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x)).to(dev, dt)  # noqa
    out = {}
    wl = W.config2(0, 512, 1024)
    for B in (1, 16):
        p = mfwf.Plan(512, 1024, max_batch=B, dtype="f32")
        p.set_covariances(wl.cl, t(1.0 / wl.noise_var), t(wl.mask, torch.uint8))
        sig = p.sht_inv(t(wl.signal_alm[None], torch.complex128))[0]
        d = torch.stack([sig + t(np.sqrt(wl.noise_var) * W.batch_noise(b, wl.npix)) for b in range(B)])
        el, lat = timed_solves(p, d, K, 2, 1, use_graph)
        out["nside512_f32_b%d" % B] = {"solves_per_s": 2 * B / el, "ms_per_solve_call": 1e3 * el / 2,
                                       "iteration_ms": 1e3 * el / 2 / K}
        del p
    w = W.config4(0)
    nside, lmax, B = 256, 512, 64
    ninv, mask = t(1.0 / w.noise_var), t(w.mask, torch.uint8)
    p = mfwf.Plan(nside, lmax, max_batch=B, dtype="f32")
    p.set_covariances(w.cl, ninv, mask)
    ls, _ = W.alm_l_m(lmax)
    draws_wf = [W.config4_draws(b) for b in range(32)]
    sig = p.sht_inv(t(np.stack([np.sqrt(w.cl[ls]) * h for h, _ in draws_wf]), torch.complex128))
    M = t(w.mask / w.noise_var)
    d = sig + t(np.sqrt(w.noise_var))[None] * t(np.stack([g for _, g in draws_wf]))
    draws_cr = [W.fluctuation_draws(32 + k, nside, lmax) for k in range(32)]
    rho_cr = p.fluctuation_rhs(t(np.stack([g for g, _ in draws_cr])),
                               t(np.stack([h for _, h in draws_cr]), torch.complex128))
    rho = torch.cat([M[None] * d, rho_cr], 0)
    p.solve(rho, iters=K, source_is_rho=True, use_graph=use_graph, want_map=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        p.solve(rho, iters=K, source_is_rho=True, use_graph=use_graph, want_map=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["config4_nside256_b64_wf32_cr32"] = {"solves_per_s": 2 * B / el, "ms_per_solve_call": 1e3 * el / 2,
                                             "iteration_ms": 1e3 * el / 2 / K}
    del p
    return out


def tqu(nside, lmax, K, steps, use_graph, batch):
    """T, Q, U Wiener filter: Wishart 3x3 noise blocks, the temperature problem's mask,
    EE/TE/BB spectra from TT.  The plain FP64 path (one map) and the batched FP32 form
    (`batch` maps: one signal, seeded noise draws), each with per-stage times and the roofline
    position of its dominant kernel."""
    import torch
    from paper_1210_4931_amd import mfwf
    from paper_1210_4931_amd import workloads as W
    w = W.config3(0, nside, lmax)
    dev = torch.device("cuda:0")
    ninv6, mask = torch.as_tensor(w.ninv6).to(dev), torch.as_tensor(w.mask).to(dev)
    plan = mfwf.Plan(nside, lmax, max_batch=1, spin=2)
    plan.set_covariances(w.cl4, ninv6, mask)
    sig = plan.sht_inv(torch.as_tensor(w.signal_alm[None]).to(dev)).cpu().numpy()[0]
    d1 = w.data_from_signal_maps(sig)
    d = torch.as_tensor(d1[None]).to(dev)
    el, lat = timed_solves(plan, d, K, steps, 1, use_graph)
    kt = dict(zip(KERNELS, plan.time_kernels(1, 5)))
    work = plan.work()[0]
    del plan
    # per evaluated (l, m, pair) and direction: 3 recurrence, 6 forming F+ and F- from it,
    # 4 for T and 16 for E, B (complex-by-real products with the ring-Fourier values)
    flops = 29.0 * work
    dom = max(("leg_analysis", "leg_synth"), key=lambda k: kt[k])
    out = {"workload": "T, Q, U Wiener filter, nside %d, lmax %d, %d iterations, 3x3 Wishart "
                       "noise blocks" % (nside, lmax, K),
           "fp64_single": {
               "solves_per_s": steps / el, "ms_per_solve": 1e3 * el / steps,
               "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                              "p99": 1e3 * float(np.percentile(lat, 99))},
               "kernel_ms": kt,
               "roofline": {"bound": "alu", "kernel": dom + "_pol",
                            "achieved": flops / (kt[dom] * 1e-3) / 1e12,
                            "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                            "frac": flops / (kt[dom] * 1e-3) / PEAK_FP64_VALU}}}
    # batched FP32 form
    B = batch
    p32 = mfwf.Plan(nside, lmax, max_batch=B, spin=2, dtype="f32")
    p32.set_covariances(w.cl4, ninv6, mask)
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    chol = torch.as_tensor(w.noise_chol).to(dev)
    sig_t = torch.as_tensor(sig).to(dev)
    dB = torch.empty((B, 3, w.npix), dtype=torch.float64, device=dev)
    for b in range(B):
        g = torch.randn((w.npix, 3, 1), generator=gen, device=dev, dtype=torch.float64)
        dB[b] = sig_t + torch.matmul(chol, g)[:, :, 0].T
    torch.cuda.synchronize()
    el32, lat32 = timed_solves(p32, dB, K, steps, 1, use_graph)
    names = POL_B_KERNELS
    kt32 = dict(zip(names, p32.time_kernels(B, 3)))
    # three GEMMs per direction: lambda on 2 columns, F+ and F- on 4 columns per map
    gflops = 2.0 * work * 10 * B
    domg = max(("gemm_analysis", "gemm_synthesis"), key=lambda k: kt32[k])
    out["f32_batched"] = {
        "batch": B, "solves_per_s": B * steps / el32, "ms_per_step": 1e3 * el32 / steps,
        "iteration_ms": 1e3 * el32 / steps / K,
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat32, 50)),
                       "p99": 1e3 * float(np.percentile(lat32, 99))},
        "kernel_ms": kt32,
        "roofline": {"bound": "mfma", "kernel": domg + " (3 launches)",
                     "achieved": gflops / (kt32[domg] * 1e-3) / 1e12,
                     "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": gflops / (kt32[domg] * 1e-3) / PEAK_FP32_MFMA}}
    return out


def cooled(plan, d):
    """Converged solve with the cooling schedule of Sect. 3 (mfwf_solve_cooled, default
    options): one untimed run creates the plans of the truncated stages, the second is
    timed (wall clock, inputs resident)."""
    import torch
    plan.solve_cooled(d, want_map=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info, st, conv = plan.solve_cooled(d, want_map=False)
    el = time.perf_counter() - t0
    n = d.shape[0]
    return {"maps": n, "seconds": el, "solves_per_s": n / el, "iterations": info[0].iters_done,
            "converged": conv, "chi2_per_dof": info[0].chi2 / info[0].n_dof,
            "stages": [[int(x[0]), round(float(x[1]), 4), int(x[2]), int(x[3])] for x in st],
            "stage_columns": ["l_iter", "lambda", "lmax_SHT", "iterations"]}


def bounded(plan, d):
    """Solve under the error bound of Sect. 2.2 (mfwf_solve_bounded, default options),
    timed after one untimed run."""
    import torch
    plan.solve_bounded(d, want_map=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info, tr, nup, reached = plan.solve_bounded(d, want_map=False)
    el = time.perf_counter() - t0
    return {"maps": d.shape[0], "seconds": el, "iterations": len(tr), "b_updates": nup,
            "reached_lambda_1": reached, "first_lambda": float(tr[0, 0]),
            "chi2_per_dof": info[0].chi2 / info[0].n_dof,
            "max_chi2_over_b": float((tr[:, 1] / tr[:, 2]).max())}


def timed_solves(plan, d, K, steps, warmup, use_graph):
    import torch
    for _ in range(warmup):
        plan.solve(d, iters=K, use_graph=use_graph, want_map=False)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        plan.solve(d, iters=K, use_graph=use_graph, want_map=False)  # synchronises its stream
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, lat


def kernel_mode(args):
    """--kernels FORM: run each stage of one messenger iteration `--reps` times through
    mfwf_time_kernels (after two solve iterations), on the temperature workload at --nside /
    --lmax with --batch maps (FP32 form) or one map (FP64); with --copy also a 256 MiB device
    copy three times, the reference for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes;
    with --solve-iters N also a timed solve of N iterations; with --spin 2 the T, Q, U
    workload instead (Wishart 3x3 noise, the temperature mask).  For hardware-counter runs."""
    import torch
    from paper_1210_4931_amd import mfwf
    from paper_1210_4931_amd import workloads as W
    maps = args.batch if args.kernels == "f32" else 1
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)  # noqa
    plan = mfwf.Plan(args.nside, args.lmax, max_batch=maps, dtype=args.kernels, spin=args.spin)
    if args.spin == 2:
        w = W.config3(0, args.nside, args.lmax)
        plan.set_covariances(w.cl4, t(w.ninv6), t(w.mask, torch.uint8))
        sig = plan.sht_inv(t(w.signal_alm[None], torch.complex128)).cpu().numpy()[0]
        d = t(w.data_from_signal_maps(sig)[None]).expand(maps, -1, -1).contiguous()
    else:
        wl = W.config2(0, args.nside, args.lmax)
        plan.set_covariances(wl.cl, t(1.0 / wl.noise_var), t(wl.mask, torch.uint8))
        sig = plan.sht_inv(t(wl.signal_alm[None], torch.complex128))
        d = (sig + t(np.sqrt(wl.noise_var) * wl.noise_white)[None]).expand(maps, -1).contiguous()
    plan.solve(d, iters=2, use_graph=False)
    ms = plan.time_kernels(maps, args.reps)
    if args.copy:
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
    torch.cuda.synchronize()
    out = {"mode": "kernels", "form": args.kernels, "spin": args.spin, "nside": args.nside, "lmax": args.lmax,
           "maps": maps, "kernel_ms": dict(zip(POL_B_KERNELS if args.spin == 2 and args.kernels == "f32"
                                               else KERNELS, ms))}
    if args.solve_iters > 0:
        plan.solve(d, iters=args.solve_iters)  # warm: graph capture, caches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve(d, iters=args.solve_iters)
        torch.cuda.synchronize()
        out["solve_ms_per_iter"] = 1e3 * (time.perf_counter() - t0) / args.solve_iters
    print(json.dumps(out), flush=True)


def tqu_cooled_mode(args):
    """--tqu-cooled: converged T, Q, U solves with the cooling schedule (Sect. 3) on the T, Q,
    U workload (Wishart 3x3 noise, EE/BB/TE tied to TT, the nside 512 mask): data from its
    signal with the FP64 path, then mfwf_solve_cooled twice (the second run timed) on one map
    with the FP64 path and on --tqu-batch maps (the first map and noisier copies) with the
    batched FP32 form.  One JSON line per form."""
    import torch
    from paper_1210_4931_amd import mfwf
    from paper_1210_4931_amd import workloads as W

    def dev(x, dt=torch.float64):
        return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)

    w = W.config3(0, args.nside, args.lmax)
    ninv6, mask = dev(w.ninv6), dev(w.mask, torch.uint8)

    def run(plan, x, tag, nmaps):
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info, stages, conv = plan.solve_cooled(x)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        print(json.dumps({"mode": "tqu_cooled", "form": tag, "nside": args.nside,
                          "lmax": args.lmax, "maps": nmaps, "seconds": el,
                          "solves_per_s": nmaps / el, "iterations": info[0].iters_done,
                          "converged": conv, "chi2_per_dof": info[0].chi2 / info[0].n_dof,
                          "stages": stages[:, :4].tolist()}), flush=True)

    p64 = mfwf.Plan(args.nside, args.lmax, max_batch=1, spin=2)
    p64.set_covariances(w.cl4, ninv6, mask)
    sig = p64.sht_inv(dev(w.signal_alm[None], torch.complex128)).cpu().numpy()[0]
    d1 = w.data_from_signal_maps(sig)
    run(p64, dev(d1[None]), "fp64", 1)
    del p64
    rng = np.random.default_rng(5)
    B = args.tqu_batch
    ds = np.stack([d1] + [d1 + rng.standard_normal(d1.shape) for _ in range(B - 1)])
    p32 = mfwf.Plan(args.nside, args.lmax, max_batch=B, spin=2, dtype="f32")
    p32.set_covariances(w.cl4, ninv6, mask)
    run(p32, dev(ds), "f32_batched", B)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=300, help="messenger iterations per solve")
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--lmax", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=64, help="maps per batched FP32 solve")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-tqu", action="store_true", help="skip the T, Q, U measurement")
    ap.add_argument("--tqu-steps", type=int, default=2)
    ap.add_argument("--tqu-batch", type=int, default=32, help="maps per batched T, Q, U solve")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-cooled", action="store_true",
                    help="skip the converged solves with the cooling schedule")
    ap.add_argument("--serve-requests", type=int, default=8,
                    help="requests per serving phase (saturation, Poisson at 0.5, 0.8 and 0.95 "
                         "of it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other batched forms (B = 1, 16; the nside 256 64-RHS batch)")
    ap.add_argument("--kernels", choices=["f64", "f32"], default=None,
                    help="profiling mode: run each kernel of one iteration --reps times")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--spin", type=int, choices=[0, 2], default=0,
                    help="with --kernels: 2 for the T, Q, U workload")
    ap.add_argument("--copy", action="store_true")
    ap.add_argument("--solve-iters", type=int, default=0)
    ap.add_argument("--tqu-cooled", action="store_true",
                    help="mode: converged T, Q, U solves (cooling schedule), FP64 and FP32")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the solver on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.kernels:
        return kernel_mode(args)
    if args.tqu_cooled:
        return tqu_cooled_mode(args)

    import torch
    from paper_1210_4931_amd import mfwf
    from paper_1210_4931_amd import workloads as W

    nside, lmax, K, B = args.nside, args.lmax, args.iters, args.batch
    use_graph = not args.no_graph
    wl = W.config2(0, nside, lmax)
    dev = torch.device("cuda:0")
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x)).to(dev, dt)  # noqa
    ninv, mask = t(1.0 / wl.noise_var), t(wl.mask, torch.uint8)

    # ---- plain FP64 single-solve path --------------------------------------------------
    p64 = mfwf.Plan(nside, lmax, max_batch=1, dtype="f64")
    p64.set_covariances(wl.cl, ninv, mask)
    sig = p64.sht_inv(t(wl.signal_alm[None], torch.complex128))  # signal map Y a
    sigma = t(np.sqrt(wl.noise_var))
    d1 = sig + sigma[None] * t(wl.noise_white)[None]
    el64, lat64 = timed_solves(p64, d1, K, args.fp64_steps, 1, use_graph)
    note("FP64 single-map solves timed")
    kt64 = dict(zip(KERNELS, p64.time_kernels(1, 20)))
    work, full, npair, fftmax = p64.work()
    leg_flops = 7.0 * work          # per map and direction: 3 recurrence + 4 complex-by-real FMA
    dom64 = max(("leg_analysis", "leg_synth"), key=lambda k: kt64[k])
    pair64 = kt64["fft_fwd"] + kt64["leg_analysis"] + kt64["leg_synth"] + kt64["fft_inv"]
    fp64 = {"solves_per_s": args.fp64_steps / el64, "ms_per_solve": 1e3 * el64 / args.fp64_steps,
            "latency_ms": {"p50": 1e3 * float(np.percentile(lat64, 50)),
                           "p99": 1e3 * float(np.percentile(lat64, 99))},
            "iteration_ms": 1e3 * el64 / args.fp64_steps / K,
            "sht_pair_tflops": 2 * leg_flops / (pair64 * 1e-3) / 1e12,
            "kernel_ms": kt64,
            "roofline": {"bound": "alu", "kernel": dom64,
                         "achieved": leg_flops / (kt64[dom64] * 1e-3) / 1e12,
                         "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": leg_flops / (kt64[dom64] * 1e-3) / PEAK_FP64_VALU}}
    if not args.no_cooled:
        fp64["cooled"] = cooled(p64, d1)
        fp64["bounded"] = bounded(p64, d1)
        note("FP64 converged solves done")

    # ---- batched FP32 form (headline) --------------------------------------------------
    p32 = mfwf.Plan(nside, lmax, max_batch=B, dtype="f32")
    p32.set_covariances(wl.cl, ninv, mask)
    # map b: the signal plus its own seeded noise draw (workloads.batch_noise(b))
    dB = torch.empty((B, wl.npix), dtype=torch.float64, device=dev)
    for b in range(B):
        dB[b] = sig[0] + sigma * t(W.batch_noise(b, wl.npix))
    torch.cuda.synchronize()
    el32, lat32 = timed_solves(p32, dB, K, args.steps, args.warmup, use_graph)
    note("batched FP32 solves timed (headline)")
    # accuracy of the timed form: two maps of the batch against the plain FP64 path (itself
    # checked against the CPU oracle by the GPU tests), relative 2-norm over the real
    # harmonic dof (m > 0 twice) and over the map
    a32, m32, _ = p32.solve(dB, iters=K, use_graph=use_graph)
    acc = {}
    for b in (0, B // 2 + 5 if B > 1 else 0):
        a64, m64, _ = p64.solve(dB[b:b + 1].contiguous(), iters=K, use_graph=use_graph)
        w = torch.ones(a64.shape[-1], dtype=torch.float64, device=dev)
        w[lmax + 1:] = 2.0 ** 0.5
        ea = (torch.linalg.norm(w * (a32[b] - a64[0])) / torch.linalg.norm(w * a64[0])).item()
        em = (torch.linalg.norm(m32[b] - m64[0]) / torch.linalg.norm(m64[0])).item()
        acc["map%d" % b] = {"rel_err_alm": ea, "rel_err_map": em}
    del a32, m32
    del p64
    kt32 = dict(zip(KERNELS, p32.time_kernels(B, 20)))
    tun = p32.tuning()
    ring_shape = (tun["g0"], tun["g1"])  # maps per workgroup of the ring step's two classes
    gemm_flops = 2.0 * work * 2 * B   # one FMA per (l, m, ring pair) and column, 2 columns a map
    dom32 = max(("leg_analysis", "leg_synth"), key=lambda k: kt32[k])
    pair32 = kt32["fft_fwd"] + kt32["leg_analysis"] + kt32["leg_synth"] + kt32["fft_inv"]
    achieved = gemm_flops / (kt32[dom32] * 1e-3)
    # the ring step of a chained iteration (kt32["fft_fwd"]: both transform-length classes of
    # the fused inverse transform / pixel update / forward transform kernel) moves at least
    # the synthesis columns in, the analysis columns out (8 B per ring and m a map), rho
    # (8 B a pixel a map) and M (8 B a pixel, shared)
    nring = 4 * nside - 1
    ring_bytes = 8.0 * B * (2 * nring * (lmax + 1) + wl.npix) + 8.0 * wl.npix
    ring_bw = ring_bytes / (kt32["fft_fwd"] * 1e-3)

    out = {
        "metric": METRIC,
        "value": B * args.steps / el32,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "temperature Wiener filter, HEALPix nside %d, lmax %d, %d "
                               "messenger iterations at lambda=1, %d maps per batched solve, "
                               "FP32 matrix-core Legendre steps, FP64 maps/FFTs" % (nside, lmax, K, B),
                   "nside": nside, "lmax": lmax, "iterations": K, "batch": B, "graph": use_graph},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat32, 50)),
                       "p99": 1e3 * float(np.percentile(lat32, 99))},
        "iteration_ms": 1e3 * el32 / args.steps / K,
        "sht_pair_tflops": 2 * gemm_flops / (pair32 * 1e-3) / 1e12,
        "kernel_ms": kt32,
        "fused": {"pixel_update": "inside fft_fwd", "harmonic": "inside leg_analysis",
                  "fft_inv": "inside fft_fwd",
                  "note": "fft_fwd is the ring step of a chained iteration: the previous "
                          "synthesis back to pixels, the pixel update and the forward ring "
                          "transforms in one kernel, with the layout transposes to and from "
                          "the matrix-core column layout"},
        "legendre_triples": {"evaluated": work, "full_triangle": full},
        "accuracy_vs_fp64_path": dict(acc, tolerance=1e-5, iterations=K),
        # the dominant kernel: the ring step (inverse transforms, pixel update, forward
        # transforms), per iteration: HIP events on the plan's stream around the fork of the
        # long class onto the side stream and the join back
        "roofline": {"bound": "hbm", "kernel": "ring_step (k_fft_inv_fwd, both length classes side by side on two streams)",
                     "achieved": ring_bw / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": ring_bw / PEAK_HBM, "algorithmic_bytes": ring_bytes,
                     "ms": kt32["fft_fwd"], "traffic": measured_traffic("ring_step", ring_shape),
                     "ring_step_maps_per_workgroup": list(ring_shape),
                     "counters": RING_COUNTERS if measured_traffic("ring_step", ring_shape) else None},
        "roofline_gemm": {"bound": "mfma", "kernel": "gemm_" + dom32.split("_")[1],
                          "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                          "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                          "ms": kt32[dom32],
                          "traffic": measured_traffic("gemm_analysis", (tun["cta"], tun["lamgen"]))
                          if dom32 == "leg_analysis" else None},
        "fp64_single": fp64,
    }
    note("accuracy and kernel times done")
    if not args.no_cooled:
        out["cooled_f32_batched"] = cooled(p32, dB)
        note("FP32 converged solves done")
    del p32
    if not args.no_tqu:
        out["tqu"] = tqu(nside, lmax, K, args.tqu_steps, use_graph, args.tqu_batch)
        note("T, Q, U done")
    if not args.no_extras:
        out["batched_extras"] = batched_extras(K, use_graph)
        note("batched extras done")
    if not args.no_serve:
        from paper_1210_4931_amd.serving_bench import run_serving
        del dB
        torch.cuda.empty_cache()  # the serving pools take their memory from the same device
        out["serving"] = run_serving(nsides=(128, 256, 512, 1024, 2048),
                                     requests=args.serve_requests, loads=(0.5, 0.8, 0.95), K=K)
        note("serving done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nside, lmax, K, wl, d1.cpu().numpy()[0],
                                           wl.mask / wl.noise_var)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
