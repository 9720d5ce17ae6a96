"""The serving runtime's scheduling core (paper_1210_4931_amd/csrc/serve_core.h, the code the
HIP server runs) on the CPU, driven by a simulated device (tests/serve/sim_backend.cpp): a
fixed cost per iteration and slot count, a fake clock that advances from event to event.
Checks admission by footprint and eviction, slot refill at iteration boundaries, fair sharing
of a lane, that a request for a new pool is not starved by a steady stream for existing ones,
and the latency percentiles the serving benchmark reports.  No GPU involved."""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
F64, F32, ENOMEM = 0, 1, -2  # mfwf.h


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("serve") / "sim_backend")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1210_4931_amd", "csrc"),
                    os.path.join(ROOT, "tests", "serve", "sim_backend.cpp"), "-o", exe], check=True)

    def run(slots, budget, reqs):
        text = "%d %.0f\n" % (slots, budget) + "".join("%r %d %d %d %d\n" % r for r in reqs)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True, timeout=120)
        res = json.loads(out.stdout)
        res["done"] = np.array([r[2] for r in res["requests"]])
        res["status"] = np.array([r[3] for r in res["requests"]])
        return res
    return run


def cost(nside, dtype, nb):
    """The simulated device's milliseconds per iteration (sim_backend.cpp)."""
    return 1e-5 * nside * nside * (2.0 if dtype == F64 else 1.0) * (1.0 + 0.25 * nb)


def pool_bytes(nside, slots):
    return 1e4 * nside * nside * slots


def test_slot_refill_at_iteration_boundaries(sim):
    """Two slots, three requests of 10 iterations at once: the first two run together and
    finish after 10 two-slot iterations; the third takes the first free slot at that
    iteration boundary and finishes 10 one-slot iterations later."""
    r = sim(2, 1e12, [(0.0, 16, 32, F64, 10)] * 3)
    assert (r["status"] == 0).all()
    t2 = 10 * cost(16, F64, 2)
    assert r["done"][0] == pytest.approx(t2) and r["done"][1] == pytest.approx(t2)
    assert r["done"][2] == pytest.approx(t2 + 10 * cost(16, F64, 1))
    assert r["created"] == 1 and r["iterations"] == 20


def test_admission_by_footprint_and_eviction(sim):
    """A budget that holds the pool of one shape at a time (the nside-32 pool gets one slot:
    two would take more than half the budget): requests of two shapes take turns, the idle
    pool is evicted each time, the charged bytes never exceed the budget; a shape whose
    single slot exceeds the budget is refused with MFWF_ENOMEM."""
    budget = 1.2e7
    assert pool_bytes(16, 2) <= budget / 2 < pool_bytes(32, 1) <= budget < pool_bytes(16, 2) + pool_bytes(32, 1)
    reqs = [(0.0, 16, 32, F64, 5), (0.0, 32, 64, F64, 5), (0.0, 16, 32, F64, 5), (0.0, 32, 64, F64, 5),
            (0.0, 128, 256, F64, 5)]
    r = sim(2, budget, reqs)
    assert list(r["status"]) == [0, 0, 0, 0, ENOMEM]
    assert r["evicted"] >= 2 and r["peak_bytes"] <= budget
    # slots halved while a pool would take more than half the budget: a 16-slot server
    # gives nside 32 (16 slots = 1.6e8 bytes) 4 slots within 1.1e8
    r = sim(16, 1.1e8, [(0.0, 32, 64, F64, 5)] * 8)
    assert (r["status"] == 0).all() and r["peak_bytes"] == pool_bytes(32, 4)


def test_fair_share_of_a_lane(sim):
    """Two pools on one lane, one twice as costly per iteration as the other, each with one
    long request: start-time fair queueing on measured durations gives each the same GPU
    time, so the cheap request finishes after about twice its own work (not after both
    requests' work interleaved iteration by iteration), and the costly one right after."""
    K = 200
    big = (0.0, 64, 128, F64, 5)  # first pool: takes lane 0 (largest static weight)
    reqs = [big, (0.0, 16, 32, F64, K), (0.0, 16, 32, F32, K)]  # both go to lane 1
    r = sim(2, 1e12, reqs)
    assert (r["status"] == 0).all()
    c64, c32 = cost(16, F64, 1), cost(16, F32, 1)
    assert r["done"][2] == pytest.approx(2 * K * c32, rel=0.05)
    assert r["done"][1] == pytest.approx(K * (c64 + c32), rel=0.05)


def test_new_pool_is_not_starved_by_a_steady_stream(sim):
    """A budget for two pools, both kept busy by requests arriving faster than they finish;
    a request of a third shape arrives early.  The pools that must make room stop admitting,
    drain and are evicted, so it finishes long before the stream ends."""
    budget = 1.01 * (pool_bytes(16, 2) + pool_bytes(32, 2))
    step = 0.25 * cost(16, F64, 2)  # both pools get requests faster than they finish them
    reqs = []
    for j in range(200):
        reqs.append((j * step, 16 if j % 2 else 32, 32 if j % 2 else 64, F64, 5))
    reqs.insert(10, (9.5 * step, 24, 48, F64, 5))
    r = sim(2, budget, reqs)
    assert (r["status"] == 0).all() and r["evicted"] >= 1
    assert r["done"][10] < reqs[120][0], (r["done"][10], reqs[120][0])
    assert r["done"][-1] > 5 * reqs[-1][0]  # the stream's backlog outlasts its arrivals


def test_latency_percentiles():
    from paper_1210_4931_amd.serving_bench import _stats
    lat = np.arange(1, 101) / 1000.0  # 1 .. 100 ms
    st = _stats(lat)
    assert st["n"] == 100
    assert st["p50_ms"] == pytest.approx(50.5) and st["p99_ms"] == pytest.approx(99.01)
    assert st["mean_ms"] == pytest.approx(50.5)
