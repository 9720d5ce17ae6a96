"""Early end of a fixed-lambda schedule on the chi^2 change (mfwf_solve_opts.dchi2_tol).

The run stops at a check once chi^2 moved by less than dchi2_tol sigma_chi2 per iteration
since the previous check of the same stage; the result must then be the oracle's iterate
after exactly the reported number of iterations, and the history must show the criterion
met at the last check and not before.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import dev, rel, rel_alm, temperature_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


def _criterion_rows(hist, lam, n_check, thr):
    """Indices of checks where the per-iteration chi^2 change since the previous check of the
    same stage is below thr for every map."""
    out = []
    for r in range(1, hist.shape[0]):
        if hist[r, 0, 1] != hist[r - 1, 0, 1]:
            continue
        dk = hist[r, 0, 0] - hist[r - 1, 0, 0]
        if np.all(np.abs(hist[r, :, 2] - hist[r - 1, :, 2]) / dk < thr):
            out.append(r)
    return out


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_early_stop_matches_oracle_at_reported_count(mf, dtype, tol):
    nside, lmax, n_check, dtol = 32, 64, 10, 1.08e-2
    wl, d, M = temperature_problem(nside, lmax, seed=4)
    rng = np.random.default_rng(8)
    ds = np.stack([d, d + rng.standard_normal(d.size) * np.sqrt(wl.noise_var)])
    plan = mf.Plan(nside, lmax, max_batch=2, dtype=dtype)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    lam, its = [20.0, 1.0], [15, 3000]
    s_alm, s_map, info, hist = plan.solve(dev(ds), lam=lam, iters=its, n_check=n_check,
                                          dchi2_tol=dtol)
    n = info[0].iters_done
    thr = dtol * np.sqrt(2.0 * info[0].n_dof)
    print("stopped after", n, "of", sum(its), "iterations; checks", hist.shape[0])
    assert info[1].iters_done == n and 15 < n < sum(its) and n % n_check == 0
    # the criterion holds at the last check and at no earlier one
    assert _criterion_rows(hist, lam, n_check, thr) == [hist.shape[0] - 1]
    assert hist[-1, 0, 0] == n and hist[-1, 0, 1] == 1.0
    sched = np.repeat(lam, [15, n - 15])
    for b in range(2):
        ref_alm, ref_map = oracle.solve(nside, lmax, wl.cl, M, M * ds[b], lam=sched)
        assert rel_alm(s_alm.cpu().numpy()[b], ref_alm, lmax) < tol
        assert rel(s_map.cpu().numpy()[b], ref_map) < tol
    # dchi2_tol = 0 runs the whole schedule
    _, _, info0, _ = plan.solve(dev(ds), lam=lam, iters=its, n_check=n_check)
    assert info0[0].iters_done == sum(its)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_early_stop_tqu_matches_oracle_at_reported_count(mf, dtype, tol):
    """T, Q, U plans, two maps: the oracle's chi^2 moves by 6.2e-3 and 4.3e-3 sigma_chi2 per
    iteration over the checks ending at 100 and 110 iterations, so a tolerance of 5e-3 stops
    the run at 110."""
    from paper_1210_4931_amd import workloads as W
    nside, lmax, n_check, dtol = 16, 32, 10, 5e-3
    w = W.config3(4, nside, lmax, ndisc=10, band_z=0.15, nu=10)
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    ds = np.stack([d, d + np.random.default_rng(8).standard_normal(d.shape)])
    M6 = w.M6()
    Mb = M6[:, [0, 1, 2, 1, 3, 4, 2, 4, 5]].reshape(-1, 3, 3)
    plan = mf.Plan(nside, lmax, max_batch=2, spin=2, dtype=dtype)
    plan.set_covariances(w.cl4, dev(w.ninv6), dev(w.mask, torch.uint8))
    lam, its = [20.0, 1.0], [15, 585]
    s_alm, s_map, info, hist = plan.solve(dev(ds), lam=lam, iters=its, n_check=n_check,
                                          dchi2_tol=dtol)
    n = info[0].iters_done
    assert n == 110 and info[1].iters_done == n
    thr = dtol * np.sqrt(2.0 * info[0].n_dof)
    assert _criterion_rows(hist, lam, n_check, thr) == [hist.shape[0] - 1]
    _, ms = W.alm_l_m(lmax)
    wgt = np.sqrt(np.where(ms == 0, 1.0, 2.0))
    sched = np.repeat(lam, [15, n - 15])
    for b in range(2):
        rho = np.einsum("pij,jp->ip", Mb, ds[b])
        ref_alm, ref_map = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=sched)
        assert rel(s_alm.cpu().numpy()[b] * wgt, ref_alm * wgt) < tol
        assert rel(s_map.cpu().numpy()[b], ref_map) < tol


def test_early_stop_errors(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    wl, d, M = temperature_problem(8, 16)
    plan = mf.Plan(8, 16)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    with pytest.raises(MFWFError, match="n_check"):
        plan.solve(dev(d[None]), iters=20, dchi2_tol=1e-3)
    with pytest.raises(MFWFError):
        plan.solve(dev(d[None]), iters=20, n_check=5, dchi2_tol=-1.0)
