"""Time converged solves with the cooling schedule (Sect. 3) on the T, Q, U workload.

    python -m paper_1210_4931_amd.cooled_probe --nside 512 --lmax 768 --maps 32

Builds the T, Q, U workload (Wishart 3x3 noise, EE/BB/TE spectra tied to TT, the config-2
mask), makes data from its signal with the FP64 path, then runs mfwf_solve_cooled twice
(the second run is timed) on one map with the FP64 path and on `--maps` maps (the first
map and noisier copies) with the batched FP32 form.  Prints one JSON line per form: seconds,
converged solves per second, iterations, whether the final criterion was met, chi^2/n_dof
of the first map and the stages (l_iter, lambda, lmax_SHT, iterations).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--lmax", type=int, default=768)
    ap.add_argument("--maps", type=int, default=32)
    args = ap.parse_args()

    import torch
    from paper_1210_4931_amd import mfwf
    from paper_1210_4931_amd import workloads as W

    mfwf.load()

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
            t = time.perf_counter() - t0
        print(json.dumps({"form": tag, "nside": args.nside, "lmax": args.lmax, "maps": nmaps,
                          "seconds": t, "solves_per_s": nmaps / t,
                          "iterations": info[0].iters_done, "converged": conv,
                          "chi2_per_dof": info[0].chi2 / info[0].n_dof,
                          "stages": stages[:, :4].tolist()}), flush=True)

    p64 = mfwf.Plan(args.nside, args.lmax, max_batch=1, spin=2)
    p64.set_covariances(w.cl4, ninv6, mask)
    sig = p64.sht_inv(dev(w.signal_alm[None], torch.complex128)).cpu().numpy()[0]
    d1 = w.data_from_signal_maps(sig)
    run(p64, dev(d1[None]), "fp64", 1)
    del p64
    rng = np.random.default_rng(5)
    ds = np.stack([d1] + [d1 + rng.standard_normal(d1.shape) for _ in range(args.maps - 1)])
    p32 = mfwf.Plan(args.nside, args.lmax, max_batch=args.maps, spin=2, dtype="f32")
    p32.set_covariances(w.cl4, ninv6, mask)
    run(p32, dev(ds), "f32_batched", args.maps)


if __name__ == "__main__":
    main()
