"""Failure detection on the data and the per-solve diagnostics: a NaN or Inf in the source of
a solve (the data on an observed pixel, or a caller's rho) is reported as MFWF_ENAN before
the first iteration, in every solve entry point and at serving submission, while non-finite
data on masked pixels is ignored (the mask drops it, Sect. 2.3).  info.dchi2 and
info.rel_change follow the diagnostics history; the error-bound solve reports whether its
last iteration ran at lambda = 1."""
import numpy as np
import pytest
import torch

from tests.gpu_util import dev, temperature_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


def _plan(mf, nside=16, lmax=32, dtype="f64", max_batch=2):
    wl, d, M = temperature_problem(nside, lmax)
    plan = mf.Plan(nside, lmax, max_batch=max_batch, dtype=dtype)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    return plan, wl, d, M


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nonfinite_data_on_observed_pixel_is_enan(mf, dtype):
    from paper_1210_4931_amd.mfwf import MFWFError
    plan, wl, d, M = _plan(mf, dtype=dtype)
    obs = np.nonzero(M > 0)[0]
    masked = np.nonzero(M == 0)[0]
    ref = plan.solve(dev(np.stack([d, d])), iters=20)[0]
    for bad in (np.nan, np.inf):
        x = np.stack([d, d])
        x[1, obs[17]] = bad
        print("solve with %r on observed pixel %d, %s" % (bad, obs[17], dtype), flush=True)
        with pytest.raises(MFWFError, match="non-finite"):
            plan.solve(dev(x), iters=20)
        with pytest.raises(MFWFError, match="non-finite"):
            plan.solve_cooled(dev(x), max_iters=10)
        with pytest.raises(MFWFError, match="non-finite"):
            plan.solve_bounded(dev(x), max_iters=5)
    # masked pixels: whatever the data holds there is dropped (M = 0), bitwise
    x = np.stack([d, d])
    x[:, masked[:5]] = np.nan
    x[:, masked[5:9]] = -np.inf
    got = plan.solve(dev(x), iters=20)[0]
    assert torch.equal(got, ref)
    # a caller's source rho: any non-finite entry
    rho = np.stack([M * d, M * d])
    rho[0, masked[0]] = np.inf
    with pytest.raises(MFWFError, match="non-finite"):
        plan.solve(dev(rho), iters=5, source_is_rho=True)
    # the plan stays usable after a refused solve
    assert torch.equal(plan.solve(dev(np.stack([d, d])), iters=20)[0], ref)


def test_serving_submit_refuses_nonfinite_data(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    nside, lmax = 16, 32
    wl, d, M = temperature_problem(nside, lmax)
    obs = np.nonzero(M > 0)[0]
    srv = mf.Server(slots=4, hbm_gb=8.0)
    try:
        x = d.copy()
        x[obs[3]] = np.nan
        with pytest.raises(MFWFError, match="non-finite"):
            srv.submit(nside, lmax, wl.cl, dev(1.0 / wl.noise_var), dev(x),
                       mask=dev(wl.mask, torch.uint8), iters=10)
        x = d.copy()
        x[np.nonzero(M == 0)[0][:3]] = np.inf  # masked: accepted
        rid, s_alm, _ = srv.submit(nside, lmax, wl.cl, dev(1.0 / wl.noise_var), dev(x),
                                   mask=dev(wl.mask, torch.uint8), iters=10)
        srv.wait(rid)
        assert torch.isfinite(torch.view_as_real(s_alm)).all()
    finally:
        srv.close()


def test_info_dchi2_and_rel_change_follow_history(mf):
    plan, wl, d, M = _plan(mf, max_batch=2)
    x = dev(np.stack([d, 0.5 * d]))
    s_alm, s_map, info, hist = plan.solve(x, lam=[3.0, 1.0], iters=[20, 30], n_check=10)
    # checks at 10, 20 (stage 1), 30, 40, 50 (stage 2)
    assert hist.shape[0] == 5
    for b in range(2):
        k = hist[:, b, 0]
        chi = hist[:, b, 2]
        want = (chi[-1] - chi[-2]) / (k[-1] - k[-2])
        assert abs(info[b].dchi2 - want) <= 1e-12 * abs(chi[-1]), (info[b].dchi2, want)
        assert info[b].dchi2 < 0.0
        assert info[b].rel_change == pytest.approx(info[b].dnorm / info[b].snorm, rel=1e-15)
    # one check in the final stage: no change to report
    _, _, info1, _ = plan.solve(x, lam=[3.0, 1.0], iters=[20, 10], n_check=10)
    assert info1[0].dchi2 == 0.0


def test_bounded_reports_the_last_lambda_run(mf):
    plan, wl, d, M = _plan(mf, nside=32, lmax=64, max_batch=1)
    x = dev(d[None])
    _, _, info, trace, _, reached = plan.solve_bounded(x, max_iters=3)
    assert not reached and len(trace) == 3
    assert info[0].lam == trace[-1, 0] and trace[-1, 0] > 1.0
    _, _, info, trace, _, reached = plan.solve_bounded(x, max_iters=2000)
    assert reached and trace[-1, 0] == 1.0 and info[0].lam == 1.0
