"""The allocation-free template removal (static device scratch) against the allocating entry
point, through the C-ABI: two calls in a row on one device, the second with fewer maps and a
smaller plan, so that stale scratch contents from the first call would show."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import dev, rel, temperature_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


def _maps(nside, lmax, n, seed):
    wl, d, M = temperature_problem(nside, lmax)
    obs = M > 0
    V = oracle.template_matrix(nside, obs)
    rng = np.random.default_rng(seed)
    ds = np.stack([d + rng.standard_normal(4) @ V * (10.0 * (b + 1)) + rng.standard_normal(d.size)
                   for b in range(n)])
    return wl, obs, ds


def test_noalloc_template_removal_matches_allocating_entry_point(mf):
    out = []
    for nside, lmax, n, seed in [(32, 64, 6, 1), (8, 16, 2, 2)]:  # second call: smaller input
        wl, obs, ds = _maps(nside, lmax, n, seed)
        print("noalloc case nside %d maps %d" % (nside, n), flush=True)
        plan = mf.Plan(nside, lmax, max_batch=4)
        plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
        ref = plan.remove_templates(dev(ds)).cpu().numpy()
        got_t = torch.full((n, plan.npix), np.nan, dtype=torch.float64, device="cuda")
        got = plan.remove_templates_noalloc(dev(ds), got_t).cpu().numpy()
        for b in range(n):
            assert rel(got[b], ref[b]) < 1e-13, (nside, b, rel(got[b], ref[b]))
            assert rel(got[b], oracle.remove_templates(nside, obs, ds[b])) < 1e-12
            assert np.array_equal(got[b][~obs], ds[b][~obs])
        out.append(got)
    assert out[1].shape == (2, 12 * 8 * 8)


def test_noalloc_rejects_too_many_maps_and_degenerate_templates(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    nside, lmax = 8, 16
    wl, obs, ds = _maps(nside, lmax, 1, 3)
    plan = mf.Plan(nside, lmax)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    big = torch.zeros((65, plan.npix), dtype=torch.float64, device="cuda")
    with pytest.raises(MFWFError, match="at most 64 maps"):
        plan.remove_templates_noalloc(big, torch.empty_like(big))
    ninv = np.zeros(plan.npix)
    ninv[[5, 300]] = 1.0  # two observed pixels cannot carry four templates
    plan.set_covariances(np.ones(lmax + 1), dev(ninv))
    x = dev(np.ones((1, plan.npix)))
    with pytest.raises(MFWFError, match="degenerate"):
        plan.remove_templates_noalloc(x, torch.empty_like(x))
