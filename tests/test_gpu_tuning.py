"""Every kernel shape the autotuner can choose, forced one by one through MFWF_TUNE_FORCE,
against the oracle (FP64 Legendre variants) or bitwise against the default shapes (the
batched form's ring-step grouping and GEMM column tiles, which never change a result); and
the tuner itself: it times, caches under a key of the plan's shape and the library build,
and reuses the cached choice."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1210_4931_amd import workloads as W
from tests.gpu_util import dev, rel, rel_alm, temperature_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


class forced:
    def __init__(self, spec):
        self.spec = spec

    def __enter__(self):
        os.environ["MFWF_TUNE_FORCE"] = self.spec

    def __exit__(self, *a):
        os.environ.pop("MFWF_TUNE_FORCE", None)


# ring pairs 32 (fewer than one 64-lane group) and 128 (a partial group at 4 pairs per
# lane); every m has a different l count, so all block remainders occur
@pytest.mark.parametrize("nside,lmax", [(16, 37), (64, 97)])
def test_every_fp64_legendre_variant_matches_the_oracle(mf, nside, lmax):
    from paper_1210_4931_amd.mfwf import load
    lib = load()
    rng = np.random.default_rng(nside + lmax)
    alm = W.white_alm(rng, lmax)
    ref_map = oracle.alm2map(nside, lmax, alm)
    mp = rng.standard_normal(12 * nside * nside)
    ref_alm = oracle.map2alm(nside, lmax, mp)
    nsyn = 9
    nana = 6
    for v in range(max(nsyn, nana)):
        spec = "synth=%d,ana=%d" % (min(v, nsyn - 1), min(v, nana - 1))
        print("forced", spec, "nside", nside, flush=True)
        with forced(spec):
            plan = mf.Plan(nside, lmax)
        t = plan.tuning()
        assert t["synth"] == min(v, nsyn - 1) and t["ana"] == min(v, nana - 1) and t["source"] == 3
        got_map = plan.sht_inv(dev(alm[None], torch.complex128)).cpu().numpy()[0]
        got_alm = plan.sht_fwd(dev(mp[None])).cpu().numpy()[0]
        assert rel(got_map, ref_map) < 1e-12, (spec, rel(got_map, ref_map))
        assert rel_alm(got_alm, ref_alm, lmax) < 1e-12, (spec, rel_alm(got_alm, ref_alm, lmax))
        del plan
    assert lib is not None


def test_batched_shapes_do_not_change_results(mf):
    """Maps per ring-step workgroup (1, 2, 4 per transform class), GEMM column tiles (64
    columns, or 128 in four or, for the analysis, eight waves) and lambda read from the FP32 table or generated in the GEMMs from the
    FP64 recurrence's segment states, on a 40-map batch (80 active columns): 6 iterations,
    bitwise equal to each other; one run against the oracle."""
    nside, lmax, nmaps, iters = 32, 64, 40, 6
    wl, d, M = temperature_problem(nside, lmax)
    rng = np.random.default_rng(9)
    x = np.stack([d + 3.0 * rng.standard_normal(d.size) * (b % 3) for b in range(nmaps)])
    results = {}
    for spec in ["g0=1,g1=1,cta=2,cts=2,lamgen=0", "g0=2,g1=2,cta=1,cts=1,lamgen=1", "cta=3,lamgen=0",
                 "g0=2,g1=1,cta=3,cts=1,lamgen=1",
                 "g0=4,g1=1,cta=2,cts=1,lamgen=1", "g0=4,g1=4,cta=1,cts=2,lamgen=0",
                 "cta=2,cts=2,lamgen=1"]:
        print("forced", spec, flush=True)
        with forced(spec):
            plan = mf.Plan(nside, lmax, max_batch=nmaps, dtype="f32")
        plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
        assert plan.tuning()["source"] == 3
        assert plan.tuning()["lamgen"] == int(spec.split("lamgen=")[1][0])
        a, m, _ = plan.solve(dev(x), iters=iters)
        results[spec] = (a.cpu(), m.cpu())
        del plan
    first = next(iter(results.values()))
    for spec, (a, m) in results.items():
        assert torch.equal(a, first[0]) and torch.equal(m, first[1]), spec
    ref, _ = oracle.solve(nside, lmax, wl.cl, M, M * x[1], niter=iters)
    assert rel_alm(first[0].numpy()[1], ref, lmax) < 1e-5


def test_malformed_force_is_an_error(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    for spec in ["synth=99", "g0=3", "cta=4", "cts=3", "bogus=1", "synth"]:
        with forced(spec), pytest.raises(MFWFError, match="MFWF_TUNE_FORCE"):
            mf.Plan(8, 16)


def test_autotuner_times_caches_and_reuses(mf, tmp_path):
    """A plan of 256 ring pairs is tuned at creation; the choice is stored under a key of
    the device, library build, nside, lmax, batch, dtype and spin, and the next plan of that
    shape reads it back instead of timing; other shapes get keys of their own.  The tuned
    plans match the oracle."""
    cache = tmp_path / "tune.txt"
    old = os.environ.get("MFWF_TUNE_CACHE")
    os.environ["MFWF_TUNE_CACHE"] = str(cache)
    try:
        nside, lmax = 128, 256
        p1 = mf.Plan(nside, lmax)
        assert p1.tuning()["source"] == 1
        lines = cache.read_text().split("\n")
        key = lines[0].split()[0]
        parts = key.split(":")
        assert parts[0] == "gfx950" and len(parts[1]) == 16
        assert parts[2:] == ["n128", "l256", "b1", "f64", "s0"], parts
        p2 = mf.Plan(nside, lmax)
        assert p2.tuning() == p1.tuning()
        assert len([l for l in cache.read_text().split("\n") if l]) == 1  # read, not timed again
        p3 = mf.Plan(nside, lmax, max_batch=40, dtype="f32")
        t3 = p3.tuning()
        assert t3["source"] == 1
        keys = [l.split()[0] for l in cache.read_text().split("\n") if l]
        assert len(keys) == 2 and keys[1].endswith(":b40:f32:s0")
        rng = np.random.default_rng(3)
        alm = W.white_alm(rng, lmax)
        got = p1.sht_inv(dev(alm[None], torch.complex128)).cpu().numpy()[0]
        for r in (1, 200, 256, 511):
            z, s, start, nphi, phi0 = oracle.rings(nside)
            ring = got[int(start[r - 1]):int(start[r - 1] + nphi[r - 1])]
            assert rel(ring, oracle.alm2map_ring(nside, lmax, alm, r)) < 1e-12
    finally:
        if old is None:
            os.environ.pop("MFWF_TUNE_CACHE", None)
        else:
            os.environ["MFWF_TUNE_CACHE"] = old
