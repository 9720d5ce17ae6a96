"""Serving measurement: a stream of independent temperature Wiener-filter requests on one GPU.

Each request is drawn from its id (workloads.serve_request): nside uniform over the given
set with lmax = 2 nside, C_l = 6000/(l(l+1)) exp(-(l/1500)^2), noise variance 30^2/hits with
hits log-uniform over a 1000x span, a 10-30 % sky cut (band plus 50 discs), FP32 or FP64
with probability 1/2, K messenger iterations at lambda = 1.  Inputs come from a small bank of
such requests per nside (generated once, data = Y(sqrt(C) h) + sigma g made on the GPU):
the cost of a request does not depend on its values, only on its shape, dtype and K.

Three phases, all through the serving runtime (mfwf.Server):
  - warm-up: one short request per (nside, dtype), which creates the pools;
  - saturation: every request submitted at once, solves/s = requests / makespan;
  - Poisson arrivals at the given fractions of that rate, seeded, one submitting thread and
    one waiting thread; latency = submission to results in the caller's buffers.
Reported: solves/s and p50/p99 latency overall, per nside and per dtype.

Run alone: python -m paper_1210_4931_amd.serving_bench --nsides 128 256 512 --requests 200
"""
import argparse
import json
import sys
import threading
import time

import numpy as np

from . import workloads as W


def _bank(mf, dev, nsides, per_nside):
    """Request templates per nside: (cl, ninv, mask, data) device tensors and lmax."""
    import torch
    bank = {}
    for n in nsides:
        items = []
        for k in range(per_nside):
            r = W.serve_request(10_000 * n + k, nsides=(n,))
            plan = mf.Plan(r.nside, r.lmax, max_batch=1, dtype="f64")
            sig = plan.sht_inv(torch.as_tensor(r.signal_alm[None]).to(dev, torch.complex128))[0]
            d = sig + torch.as_tensor(np.sqrt(r.noise_var) * r.noise_white).to(dev)
            items.append((r.lmax, r.cl, torch.as_tensor(1.0 / r.noise_var).to(dev),
                          torch.as_tensor(r.mask).to(dev, torch.uint8), d))
            del plan
        bank[n] = items
    torch.cuda.synchronize()
    return bank


def _draw(seed, count, nsides, per_nside):
    """(nside, dtype, template) for request ids seed .. seed + count - 1."""
    out = []
    for rid in range(seed, seed + count):
        g = np.random.Generator(np.random.PCG64(rid))
        n = int(nsides[g.integers(len(nsides))])
        dt = "f32" if g.random() < 0.5 else "f64"
        out.append((n, dt, int(g.integers(per_nside))))
    return out


def _stats(lat):
    lat = np.asarray(lat)
    return {"n": int(lat.size), "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "mean_ms": 1e3 * float(lat.mean())}


def _log(msg):
    print("[serving] " + msg, file=sys.stderr, flush=True)


def _run(srv, bank, reqs, K, arrivals=None, tag=""):
    """Submit `reqs` (all at once, or at the given arrival times in seconds) and wait for
    them; returns (latencies by request, makespan from the first submission)."""
    ids = [None] * len(reqs)
    lat = [None] * len(reqs)
    ready = threading.Semaphore(0)
    t_start = time.perf_counter()

    def waiter():
        # completions in the order they happen, each one logged as it is seen
        submitted, open_ids, done = 0, [], 0
        while done < len(reqs):
            while ready.acquire(blocking=not open_ids):
                open_ids.append(submitted)
                submitted += 1
                if submitted == len(reqs):
                    break
            for i in [i for i in open_ids if srv.done(ids[i])]:
                lat[i] = srv.wait(ids[i])
                open_ids.remove(i)
                done += 1
                if tag:
                    _log("%s: request %d (nside %d, %s) done, %d/%d after %.1f s"
                         % (tag, i, reqs[i][0], reqs[i][1], done, len(reqs),
                            time.perf_counter() - t_start))
            time.sleep(0.02)

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for i, (n, dt, k) in enumerate(reqs):
        if arrivals is not None:
            dly = t0 + arrivals[i] - time.perf_counter()
            if dly > 0:
                time.sleep(dly)
        lmax, cl, ninv, mask, d = bank[n][k]
        ids[i] = srv.submit(n, lmax, cl, ninv, d, mask=mask, dtype=dt, iters=K)[0]
        ready.release()
    th.join()
    return lat, time.perf_counter() - t0


def _summary(reqs, lat, span):
    out = {"solves_per_s": len(reqs) / span, **_stats(lat), "per_nside": {}, "per_dtype": {}}
    for n in sorted({r[0] for r in reqs}):
        out["per_nside"][str(n)] = _stats([l for r, l in zip(reqs, lat) if r[0] == n])
    for dt in ("f32", "f64"):
        sel = [l for r, l in zip(reqs, lat) if r[1] == dt]
        if sel:
            out["per_dtype"][dt] = _stats(sel)
    return out


def run_serving(nsides=(128, 256, 512), requests=120, loads=(0.8,), K=300, slots=16,
                per_nside=2, hbm_gb=200.0, seed=0):
    import torch
    from . import mfwf
    mf = mfwf
    mf.load()
    dev = torch.device("cuda:0")
    _log("inputs for nside %s" % (list(nsides),))
    bank = _bank(mf, dev, nsides, per_nside)
    srv = mf.Server(slots=slots, hbm_gb=hbm_gb)
    try:
        # one pool per (nside, dtype), created (plan set-up and kernel-shape tuning) one at a
        # time so that each one's set-up time is logged
        for n in nsides:
            for dt in ("f32", "f64"):
                t0 = time.perf_counter()
                _run(srv, bank, [(n, dt, 0)], 2)
                _log("warm-up: pool nside %d %s ready in %.1f s" % (n, dt, time.perf_counter() - t0))
        reqs = _draw(seed, requests, nsides, per_nside)
        lat, span = _run(srv, bank, reqs, K, tag="saturation")
        sat = _summary(reqs, lat, span)
        rate = sat["solves_per_s"]
        out = {"workload": "serving stream: nside uniform over %s, lmax = 2 nside, FP32/FP64 "
                           "1/2 each, %d messenger iterations, %d slots per pool"
                           % (list(nsides), K, slots),
               "requests_per_phase": requests, "iterations": K, "slots": slots,
               "saturated": sat, "poisson": {}}
        for j, f in enumerate(loads):
            g = np.random.Generator(np.random.PCG64(1000 + j))
            arr = np.cumsum(g.exponential(1.0 / (f * rate), size=requests))
            arr -= arr[0]
            reqs = _draw(seed + (j + 1) * requests, requests, nsides, per_nside)
            lat, span = _run(srv, bank, reqs, K, arr, tag="poisson %.2f" % f)
            out["poisson"][str(f)] = {"offered_per_s": f * rate, **_summary(reqs, lat, span)}
        st = srv.stats()
        out["pools"] = int(st["pools"])
        out["pool_gb"] = st["pool_bytes"] / 1e9
        out["iterations_launched"] = int(st["iterations"])
        return out
    finally:
        srv.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nsides", type=int, nargs="+", default=[128, 256, 512])
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 0.8, 0.95])
    ap.add_argument("--iters", type=int, default=300)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--per-nside", type=int, default=2)
    args = ap.parse_args()
    print(json.dumps(run_serving(tuple(args.nsides), args.requests, tuple(args.loads),
                                 args.iters, args.slots, args.per_nside)), flush=True)


if __name__ == "__main__":
    main()
