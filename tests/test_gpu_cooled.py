"""Converged Wiener filter with the cooling schedule of Sect. 3 (mfwf_solve_cooled).

The schedule depends on the data through the chi^2 plateaus, so parity replays it: the GPU
run reports its stages (l_iter, lambda, lmax_SHT, iterations) and the oracle runs the same
stages with transforms truncated at each stage's lmax_SHT (oracle.solve_staged).  The rules
of the schedule are checked on the stages themselves, and the converged result against the
dense fixed point of the iteration.  T, Q, U plans replay against oracle.solve_pol_staged.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import dense
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


def _check_rules(stages, cl, tau, omega, lmax, l0, margin, step, iters_done):
    assert int(stages[0][0]) == min(l0, lmax)
    to_one = False
    for k, (l_it, lam, lk, n, _) in enumerate(stages):
        l_it, lk, n = int(l_it), int(lk), int(n)
        assert n >= 2
        if k:
            lp = int(stages[k - 1][0])
            if lp >= lmax:
                to_one = True
                assert l_it == lmax
            else:
                assert l_it == min(2 * lp, lp + step, lmax)
        if to_one:
            assert lam == 1.0 and lk == lmax
        else:
            assert lam == pytest.approx(max(1.0, cl[l_it] / (tau * omega)), rel=1e-12)
            assert lk == min(lmax, l_it + margin)
    assert sum(int(s[3]) for s in stages) == iters_done


def test_cooled_schedule_rules_and_oracle_replay(mf):
    """FP64, truncated stages: the rules of the schedule and the oracle's replay."""
    nside, lmax, l0, margin = 32, 64, 8, 16
    wl, d, M = temperature_problem(nside, lmax)
    plan = mf.Plan(nside, lmax)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    s_alm, s_map, info, stages, conv = plan.solve_cooled(dev(d[None]), l_iter0=l0,
                                                          l_margin=margin, max_iters=900)
    print("stages (l_iter, lambda, lmax_SHT, iterations, chi2/ndof):\n", stages, conv)
    assert len(stages) >= 3 and any(int(s[2]) < lmax for s in stages)
    _check_rules(stages, wl.cl, info[0].tau, 4 * np.pi / M.size, lmax, l0, margin, 500,
                 info[0].iters_done)
    ref_alm, ref_map = oracle.solve_staged(nside, lmax, wl.cl, M, M * d,
                                           [(int(s[2]), s[1], int(s[3])) for s in stages])
    assert rel_alm(s_alm.cpu().numpy()[0], ref_alm, lmax) < 1e-10
    assert rel(s_map.cpu().numpy()[0], ref_map) < 1e-10


def test_cooled_f32_batch_replay(mf):
    """The batched FP32 form, three maps sharing one schedule, each against the replay."""
    nside, lmax, l0, margin = 32, 64, 8, 16
    wl, d, M = temperature_problem(nside, lmax, seed=1)
    rng = np.random.default_rng(5)
    ds = np.stack([d, d + rng.standard_normal(d.size) * np.sqrt(wl.noise_var),
                   0.5 * d])
    plan = mf.Plan(nside, lmax, max_batch=4, dtype="f32")
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    s_alm, s_map, info, stages, conv = plan.solve_cooled(dev(ds), l_iter0=l0, l_margin=margin,
                                                          max_iters=300)
    _check_rules(stages, wl.cl, info[0].tau, 4 * np.pi / M.size, lmax, l0, margin, 500,
                 info[0].iters_done)
    sched = [(int(s[2]), s[1], int(s[3])) for s in stages]
    for b in range(3):
        ref_alm, ref_map = oracle.solve_staged(nside, lmax, wl.cl, M, M * ds[b], sched)
        assert rel_alm(s_alm.cpu().numpy()[b], ref_alm, lmax) < 1e-5
        assert rel(s_map.cpu().numpy()[b], ref_map) < 1e-5


def test_cooled_solve_converges_closer_than_plain_iterations(mf):
    """At a size where the fixed point is a dense solve: the cooled solve meets its final
    criterion, and ends nearer to the lambda = 1 fixed point than the same number of plain
    lambda = 1 iterations from s = 0."""
    nside, lmax = 16, 32
    wl, d, M = temperature_problem(nside, lmax, seed=2)
    plan = mf.Plan(nside, lmax)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    s_alm, _, info, stages, conv = plan.solve_cooled(dev(d[None]), l_iter0=4, l_margin=8,
                                                      max_iters=6000)
    assert conv
    n = info[0].iters_done
    fp = dense.Problem(nside, lmax, wl.cl, M).messenger_fixed_point(M * d)
    err_cooled = rel(dense.alm_to_real(s_alm.cpu().numpy()[0], lmax), fp)
    s_plain, _, _ = plan.solve(dev(d[None]), iters=n)
    err_plain = rel(dense.alm_to_real(s_plain.cpu().numpy()[0], lmax), fp)
    print("iterations", n, "stages", len(stages), "error vs fixed point: cooled", err_cooled,
          "plain", err_plain)
    assert err_cooled < 0.8 * err_plain


def test_cooled_errors(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    plan = mf.Plan(8, 16)
    with pytest.raises(MFWFError, match="status -4"):
        plan.solve_cooled(torch.zeros((1, 768), dtype=torch.float64, device="cuda"))
    wl, d, M = temperature_problem(8, 16)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    with pytest.raises(MFWFError):
        plan.solve_cooled(dev(d[None]), n_check=1)
    with pytest.raises(MFWFError):
        plan.solve_cooled(dev(d[None]), l_iter0=-1)
    # lmax = 4 nside is beyond what the quadrature supports: the iteration diverges and the
    # solve stops with MFWF_ENAN instead of reporting a plateau
    plan4 = mf.Plan(8, 32)
    wl4, d4, _ = temperature_problem(8, 32)
    plan4.set_covariances(wl4.cl, dev(1.0 / wl4.noise_var), dev(wl4.mask, torch.uint8))
    with pytest.raises(MFWFError, match="status -6"):
        plan4.solve_cooled(dev(d4[None]), max_iters=20000)
    with pytest.raises(MFWFError, match="status -4"):
        mf.Plan(4, 8, spin=2).solve_cooled(torch.zeros((1, 3, 192), dtype=torch.float64,
                                                       device="cuda"))


def _pol_problem(mf, nside, lmax, seed, dtype, max_batch):
    w = W.config3(seed, nside, lmax, ndisc=10, band_z=0.15, nu=10)
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    plan = mf.Plan(nside, lmax, max_batch=max_batch, spin=2, dtype=dtype)
    plan.set_covariances(w.cl4, dev(w.ninv6), dev(w.mask, torch.uint8))
    M6 = w.M6()
    Mb = M6[:, [0, 1, 2, 1, 3, 4, 2, 4, 5]].reshape(-1, 3, 3)
    return plan, w, d, M6, lambda x: np.einsum("pij,jp->ip", Mb, x)


def _rel_teb(a, ref, lmax):
    _, ms = W.alm_l_m(lmax)
    w = np.sqrt(np.where(ms == 0, 1.0, 2.0))
    return rel(a * w, ref * w)


def test_cooled_pol_schedule_rules_and_oracle_replay(mf):
    """T, Q, U (spin 2), FP64: lambda from C^TT at l_iter, truncated (T, E, B) stages; the
    replay by the staged T, Q, U oracle."""
    nside, lmax, l0, margin = 16, 32, 4, 8
    plan, w, d, M6, rho_of = _pol_problem(mf, nside, lmax, 0, "f64", 1)
    s_alm, s_map, info, stages, conv = plan.solve_cooled(dev(d[None]), l_iter0=l0,
                                                          l_margin=margin, max_iters=3000)
    print("stages (l_iter, lambda, lmax_SHT, iterations, chi2/ndof):\n", stages, conv)
    assert len(stages) >= 3 and any(int(s[2]) < lmax for s in stages)
    # converged, with chi^2 near its expectation n_dof (a diverging run would also replay)
    assert conv and 0.8 < info[0].chi2 / info[0].n_dof < 1.2
    assert info[0].n_dof == 3 * int(w.mask.sum())
    _check_rules(stages, w.cl4[0], info[0].tau, 4 * np.pi / w.npix, lmax, l0, margin, 500,
                 info[0].iters_done)
    ref_alm, ref_map = oracle.solve_pol_staged(nside, lmax, w.cl4, M6, rho_of(d),
                                               [(int(s[2]), s[1], int(s[3])) for s in stages])
    assert _rel_teb(s_alm.cpu().numpy()[0], ref_alm, lmax) < 1e-10
    assert rel(s_map.cpu().numpy()[0], ref_map) < 1e-10


def test_cooled_pol_f32_batch_replay(mf):
    """The batched FP32 T, Q, U form, two maps sharing one schedule, each against the replay."""
    nside, lmax, l0, margin = 16, 32, 4, 8
    plan, w, d, M6, rho_of = _pol_problem(mf, nside, lmax, 1, "f32", 2)
    rng = np.random.default_rng(8)
    ds = np.stack([d, d + rng.standard_normal(d.shape)])
    s_alm, s_map, info, stages, conv = plan.solve_cooled(dev(ds), l_iter0=l0, l_margin=margin,
                                                          max_iters=300)
    _check_rules(stages, w.cl4[0], info[0].tau, 4 * np.pi / w.npix, lmax, l0, margin, 500,
                 info[0].iters_done)
    sched = [(int(s[2]), s[1], int(s[3])) for s in stages]
    for b in range(2):
        ref_alm, ref_map = oracle.solve_pol_staged(nside, lmax, w.cl4, M6, rho_of(ds[b]), sched)
        assert _rel_teb(s_alm.cpu().numpy()[b], ref_alm, lmax) < 1e-5
        assert rel(s_map.cpu().numpy()[b], ref_map) < 1e-5


def test_cooled_pol_unstable_band_limit_reported(mf):
    """T, Q, U at nside 32 / lmax 64: the plain lambda = 1 iteration is unstable for this
    problem (the oracle's own chi^2 grows by growing steps after about 225 iterations, the
    temperature part alone as well); the cooled
    solve stops with MFWF_ENAN once chi^2 stands 10 sigma_chi2 above its stage minimum after
    growing rises, long before max_iters, instead of iterating into overflow.  (The FP32 and
    FP64 replays above, on nside 16, settle above a minimum by shrinking rises and finish.)"""
    from paper_1210_4931_amd.mfwf import MFWFError
    nside, lmax = 32, 64
    plan, w, d, M6, rho_of = _pol_problem(mf, nside, lmax, 0, "f64", 1)
    with pytest.raises(MFWFError, match="unstable"):
        plan.solve_cooled(dev(d[None]), l_iter0=8, l_margin=16, max_iters=20000)


def test_f32_solve_kinds_share_a_plan(mf):
    """The batched FP32 plan runs chained iterations in plain and cooled solves; a later solve
    of any kind on the same plan starts from its own state: every result equals the one of a
    fresh plan, bit for bit."""
    nside, lmax = 16, 32
    wl, d, M = temperature_problem(nside, lmax, seed=3)
    rng = np.random.default_rng(11)
    ds = dev(np.stack([d, d + rng.standard_normal(d.size) * np.sqrt(wl.noise_var)]))

    def fresh():
        q = mf.Plan(nside, lmax, max_batch=2, dtype="f32")
        q.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
        return q

    plain_ref = fresh().solve(ds, iters=40)[0]
    cooled_ref = fresh().solve_cooled(ds, l_iter0=4, l_margin=8, max_iters=400)[0]
    bounded_ref = fresh().solve_bounded(ds, max_iters=60)[0]
    q = fresh()
    for _ in range(2):
        assert torch.equal(q.solve_cooled(ds, l_iter0=4, l_margin=8, max_iters=400)[0], cooled_ref)
        assert torch.equal(q.solve_bounded(ds, max_iters=60)[0], bounded_ref)
        assert torch.equal(q.solve(ds, iters=40)[0], plain_ref)
