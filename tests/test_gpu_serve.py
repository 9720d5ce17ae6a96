"""Serving runtime: continuous batching of independent requests on one GPU.

Every served request must give exactly (bitwise) the result of a standalone solve of the
same inputs: slots are independent maps of a batch, each with its own M row and tau, and
the per-map arithmetic is the same whether a map runs alone or next to others.  A few are
also checked against the oracle.
"""
import random
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1210_4931_amd import workloads as W
from tests.gpu_util import dev, rel, rel_alm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


def _inputs(r):
    d = oracle.alm2map(r.nside, r.lmax, r.signal_alm) + np.sqrt(r.noise_var) * r.noise_white
    return d, 1.0 / r.noise_var


def _standalone(mf, r, d, ninv, iters):
    plan = mf.Plan(r.nside, r.lmax, max_batch=1, dtype=r.dtype)
    plan.set_covariances(r.cl, dev(ninv), dev(r.mask, torch.uint8))
    a, m, _ = plan.solve(dev(d[None]), iters=iters)
    return a[0], m[0]


def test_served_results_equal_standalone_solves(mf):
    srv = mf.Server(slots=4, hbm_gb=50.0)
    rng = random.Random(0)
    reqs, handles = [], []
    for rid in range(14):
        r = W.serve_request(rid, nsides=(16, 32))
        d, ninv = _inputs(r)
        iters = rng.choice([20, 35, 50])
        h = srv.submit(r.nside, r.lmax, r.cl, dev(ninv), dev(d), mask=dev(r.mask, torch.uint8),
                       dtype=r.dtype, iters=iters)
        reqs.append((r, d, ninv, iters))
        handles.append(h)
        time.sleep(rng.uniform(0.0, 0.004))  # arrivals between iteration boundaries
    lat = [srv.wait(h[0]) for h in handles]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and min(lat) > 0.0
    assert st["pools_created"] >= 4  # (16, 32) x (f32, f64)
    for (r, d, ninv, iters), (_, a, m) in zip(reqs, handles):
        a_ref, m_ref = _standalone(mf, r, d, ninv, iters)
        assert torch.equal(a, a_ref) and torch.equal(m, m_ref), (r.rid, r.nside, r.dtype, iters)


def test_neighbouring_slots_keep_their_own_tau(mf):
    """FP32 requests submitted back to back share a batch; their noise levels differ by up
    to 30x, so each slot's tau (and hence its filter C_l / (C_l + lambda tau Omega), applied
    four columns at a time in the batched analysis epilogue) differs from its neighbours'."""
    srv = mf.Server(slots=4, hbm_gb=50.0)
    out = []
    for k, scale in enumerate([1.0, 30.0, 3.0, 10.0]):
        r = W.serve_request(300 + k, nsides=(32,))
        r.dtype = "f32"
        r.noise_var = r.noise_var * scale
        d, ninv = _inputs(r)
        out.append((r, d, ninv, srv.submit(r.nside, r.lmax, r.cl, dev(ninv), dev(d),
                                           mask=dev(r.mask, torch.uint8), dtype="f32", iters=25)))
    for r, d, ninv, (rid, a, m) in out:
        srv.wait(rid)
        a_ref, m_ref = _standalone(mf, r, d, ninv, 25)
        assert torch.equal(a, a_ref) and torch.equal(m, m_ref), rid
    srv.close()


def test_served_results_match_the_oracle(mf):
    srv = mf.Server(slots=2, hbm_gb=50.0)
    out = []
    for rid in (100, 101, 102):
        r = W.serve_request(rid, nsides=(16,))
        d, ninv = _inputs(r)
        h = srv.submit(r.nside, r.lmax, r.cl, dev(ninv), dev(d), mask=dev(r.mask, torch.uint8),
                       dtype=r.dtype, iters=60)
        out.append((r, d, ninv, h))
    for r, d, ninv, (rid, a, m) in out:
        srv.wait(rid)
        M = r.mask / r.noise_var
        ref, ref_map = oracle.solve(r.nside, r.lmax, r.cl, M, M * d, niter=60)
        tol = 1e-10 if r.dtype == "f64" else 1e-5
        assert rel_alm(a.cpu().numpy(), ref, r.lmax) < tol
        assert rel(m.cpu().numpy(), ref_map) < tol
    srv.close()


def test_pools_evicted_to_fit_the_budget(mf):
    """A budget that holds one pool: requests of two shapes alternate, the idle pool is
    evicted each time, every request completes with the standalone result."""
    from paper_1210_4931_amd.mfwf import Server
    small, big = Server.pool_bytes(16, 32, "f64", 2), Server.pool_bytes(32, 64, "f64", 2)
    srv = Server(slots=2, hbm_gb=1.05 * max(small, big) / 1e9)  # one pool, never two
    hs = []
    for k, nside in enumerate([16, 32, 16, 32]):
        r = W.serve_request(200 + k, nsides=(nside,))
        r.dtype = "f64"
        d, ninv = _inputs(r)
        hs.append((r, d, ninv, srv.submit(r.nside, r.lmax, r.cl, dev(ninv), dev(d),
                                          mask=dev(r.mask, torch.uint8), iters=10)))
    for r, d, ninv, (rid, a, m) in hs:
        srv.wait(rid)
        a_ref, m_ref = _standalone(mf, r, d, ninv, 10)
        assert torch.equal(a, a_ref)
    st = srv.stats()
    srv.close()
    assert st["pools_evicted"] >= 1 and st["completed"] == 4


def test_request_for_a_new_pool_is_not_starved(mf):
    """A budget that holds two pools, both kept busy by a steady stream of requests: a
    request of a third shape still completes while the stream goes on (the pools that must
    make room stop admitting, drain and are evicted), and every request gets the standalone
    result."""
    from paper_1210_4931_amd.mfwf import Server
    a, b, c = (Server.pool_bytes(16, 32, "f64", 2), Server.pool_bytes(32, 64, "f64", 2),
               Server.pool_bytes(16, 32, "f32", 2))
    budget = 1.01 * max(a + b, c + max(a, b))
    assert a + b + c > budget
    srv = Server(slots=2, hbm_gb=budget / 1e9)
    shapes = [(16, "f64"), (32, "f64")]
    reqs, k = [], 0

    def submit(nside, dtype):
        nonlocal k
        r = W.serve_request(400 + k, nsides=(nside,))
        k += 1
        r.dtype = dtype
        d, ninv = _inputs(r)
        h = srv.submit(r.nside, r.lmax, r.cl, dev(ninv), dev(d), mask=dev(r.mask, torch.uint8),
                       dtype=dtype, iters=15)
        reqs.append((r, d, ninv, h))
        return h

    for j in range(4):
        submit(*shapes[j % 2])
    hc = submit(16, "f32")
    t0 = time.perf_counter()
    while not srv.done(hc[0]) and time.perf_counter() - t0 < 60.0:
        outstanding = sum(not srv.done(h[0]) for *_, h in reqs)
        if outstanding < 6:
            submit(*shapes[k % 2])
        time.sleep(0.002)
    assert srv.done(hc[0]), "the new-shape request waited behind a steady stream"
    for *_, h in reqs:
        srv.wait(h[0])
    st = srv.stats()
    srv.close()
    assert st["pools_evicted"] >= 1 and st["completed"] == len(reqs)
    for r, d, ninv, (rid, alm, m) in reqs[:6] + [reqs[-1]]:
        a_ref, m_ref = _standalone(mf, r, d, ninv, 15)
        assert torch.equal(alm, a_ref), (r.rid, r.dtype)


def test_served_nside2048_request_equals_standalone(mf):
    """A 2048 / 4096 request (FP64, split ring transforms) next to a small one: bitwise the
    standalone solve.  16 slots per pool would put the 2048 pool at about 200 GB, so the
    server gives that shape fewer slots (2, the first halving that fits half of 100 GB)."""
    from paper_1210_4931_amd.mfwf import Server
    assert Server.pool_bytes(2048, 4096, "f64", 4) > 50e9 >= Server.pool_bytes(2048, 4096, "f64", 2)
    r = W.serve_request(4, nsides=(2048,))
    assert r.dtype == "f64"
    z, _ = W.pixel_centres(r.nside)
    d = np.sqrt(r.noise_var) * r.noise_white + 80.0 * z
    ninv = 1.0 / r.noise_var
    small = W.serve_request(5, nsides=(16,))
    ds, ninvs = _inputs(small)
    srv = mf.Server(slots=16, hbm_gb=100.0)
    h_big = srv.submit(r.nside, r.lmax, r.cl, dev(ninv), dev(d), mask=dev(r.mask, torch.uint8),
                       dtype="f64", iters=3)
    h_small = srv.submit(small.nside, small.lmax, small.cl, dev(ninvs), dev(ds),
                         mask=dev(small.mask, torch.uint8), dtype=small.dtype, iters=20)
    srv.wait(h_big[0])
    srv.wait(h_small[0])
    srv.close()
    a_ref, m_ref = _standalone(mf, r, d, ninv, 3)
    assert torch.equal(h_big[1], a_ref) and torch.equal(h_big[2], m_ref)
    a_ref, m_ref = _standalone(mf, small, ds, ninvs, 20)
    assert torch.equal(h_small[1], a_ref) and torch.equal(h_small[2], m_ref)


def test_served_nside2048_f32_request_equals_standalone(mf):
    """A 2048 / 4096 request in the batched FP32 form (lambda generated in the contractions,
    split ring transforms on the columns, iterations chained as in a standalone solve, the
    map formed when the request retires): bitwise the standalone solve."""
    r = W.serve_request(3, nsides=(2048,))
    assert r.dtype == "f32"
    z, _ = W.pixel_centres(r.nside)
    d = np.sqrt(r.noise_var) * r.noise_white + 80.0 * z
    ninv = 1.0 / r.noise_var
    srv = mf.Server(slots=2, hbm_gb=200.0)
    h = srv.submit(r.nside, r.lmax, r.cl, dev(ninv), dev(d), mask=dev(r.mask, torch.uint8),
                   dtype="f32", iters=3)
    srv.wait(h[0])
    srv.close()
    a_ref, m_ref = _standalone(mf, r, d, ninv, 3)
    assert torch.equal(h[1], a_ref) and torch.equal(h[2], m_ref)


def test_bad_requests_rejected_at_submission(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    srv = mf.Server(slots=2, hbm_gb=10.0)
    r = W.serve_request(7, nsides=(8,))
    d, ninv = _inputs(r)
    with pytest.raises(MFWFError, match="status -4"):
        srv.submit(r.nside, r.lmax, r.cl, dev(np.zeros_like(ninv)), dev(d))
    bad = ninv.copy()
    bad[3] = -1.0
    with pytest.raises(MFWFError, match="status -6"):
        srv.submit(r.nside, r.lmax, r.cl, dev(bad), dev(d))
    with pytest.raises(MFWFError):
        srv.submit(r.nside, r.lmax, r.cl, dev(ninv), dev(d), iters=0)
    with pytest.raises(MFWFError, match="status -1"):  # lmax above 4 nside
        srv.submit(r.nside, 4 * r.nside + 1, np.ones(4 * r.nside + 2), dev(ninv), dev(d),
                   dtype="f32")
    srv.close()
