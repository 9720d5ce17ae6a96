"""Run each kernel of one messenger iteration a few times (for hardware-counter profiles).

    python -m paper_1210_4931_amd.kernel_probe --nside 512 --lmax 1024 --form f64 --maps 1
    python -m paper_1210_4931_amd.kernel_probe --nside 2048 --lmax 4096 --solve-iters 20

Builds the nside/lmax temperature workload, sets the covariances, runs two solve iterations,
then launches every stage of one iteration `--reps` times through mfwf_time_kernels.  With
--copy it also copies a 256 MiB buffer three times, the reference for scaling the
FETCH_SIZE / WRITE_SIZE counters to bytes.
"""
import argparse
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--lmax", type=int, default=1024)
    ap.add_argument("--form", choices=["f64", "f32"], default="f64")
    ap.add_argument("--maps", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--copy", action="store_true")
    ap.add_argument("--solve-iters", type=int, default=0,
                    help="also time a solve of this many iterations (wall clock, graphs on)")
    args = ap.parse_args()

    import torch
    from paper_1210_4931_amd import mfwf
    from paper_1210_4931_amd import workloads as W

    wl = W.config2(0, args.nside, args.lmax)
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)  # noqa
    plan = mfwf.Plan(args.nside, args.lmax, max_batch=args.maps, dtype=args.form)
    plan.set_covariances(wl.cl, t(1.0 / wl.noise_var), t(wl.mask, torch.uint8))
    sig = plan.sht_inv(t(wl.signal_alm[None], torch.complex128))
    d = (sig + t(np.sqrt(wl.noise_var) * wl.noise_white)[None]).expand(args.maps, -1).contiguous()
    plan.solve(d, iters=2, use_graph=False)
    ms = plan.time_kernels(args.maps, args.reps)
    if args.copy:
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
    torch.cuda.synchronize()
    out = {"kernel_ms": dict(zip(["pixel_update", "fft_fwd", "leg_analysis", "harmonic",
                                  "leg_synth", "fft_inv"], ms))}
    if args.solve_iters > 0:
        import time
        plan.solve(d, iters=args.solve_iters)  # warm: graph capture, caches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve(d, iters=args.solve_iters)
        torch.cuda.synchronize()
        out["solve_ms_per_iter"] = 1e3 * (time.perf_counter() - t0) / args.solve_iters
    print(json.dumps(out))


if __name__ == "__main__":
    main()
