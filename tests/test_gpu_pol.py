"""T, Q, U (spin 2) HIP path against the FP64 oracle.

FP64 everywhere: the transforms at 1e-12 relative (the spin-2 functions are formed in FP64
on the GPU from the rescaled recurrence, the oracle forms them in long double, so rounding
near the poles differs slightly), the messenger iterate at 1e-10 after 100 iterations.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1210_4931_amd import workloads as W
from tests.gpu_util import dev, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


def _teb(rng, lmax, n=1):
    a = np.stack([np.stack([W.white_alm(rng, lmax) for _ in range(3)]) for _ in range(n)])
    ls, _ = W.alm_l_m(lmax)
    a[:, 1:, ls < 2] = 0.0
    return a


def _rel_teb(a, ref, lmax):
    _, ms = W.alm_l_m(lmax)
    w = np.sqrt(np.where(ms == 0, 1.0, 2.0))
    return rel(a * w, ref * w)


# nside 64 (128 ring pairs): the Legendre kernels carry two pairs per lane
@pytest.mark.parametrize("nside,lmax", [(2, 6), (4, 12), (8, 20), (8, 32), (16, 40), (32, 64),
                                        (64, 128), (64, 201)])
def test_pol_sht_parity(mf, nside, lmax):
    rng = np.random.default_rng(nside * 1000 + lmax)
    a = _teb(rng, lmax, 2)
    plan = mf.Plan(nside, lmax, max_batch=2, spin=2)
    maps = plan.sht_inv(dev(a, torch.complex128)).cpu().numpy()
    mp = rng.standard_normal((2, 3, 12 * nside * nside))
    back = plan.sht_fwd(dev(mp)).cpu().numpy()
    for b in range(2):
        assert rel(maps[b], oracle.alm2map_pol(nside, lmax, a[b])) < 1e-12
        assert _rel_teb(back[b], oracle.map2alm_pol(nside, lmax, mp[b]), lmax) < 1e-12


def test_pol_T_component_equals_temperature_plan(mf):
    nside, lmax = 16, 32
    rng = np.random.default_rng(3)
    a = _teb(rng, lmax)
    p2 = mf.Plan(nside, lmax, spin=2)
    p0 = mf.Plan(nside, lmax, spin=0)
    m2 = p2.sht_inv(dev(a, torch.complex128)).cpu().numpy()
    m0 = p0.sht_inv(dev(a[:, 0], torch.complex128)).cpu().numpy()
    assert rel(m2[0, 0], m0[0]) < 1e-13


def _problem(mf, nside, lmax, seed=0, max_batch=2):
    w = W.config3(seed, nside, lmax, ndisc=10, band_z=0.15, nu=10)
    sig = oracle.alm2map_pol(nside, lmax, w.signal_alm)
    d = w.data_from_signal_maps(sig)
    plan = mf.Plan(nside, lmax, max_batch=max_batch, spin=2)
    plan.set_covariances(w.cl4, dev(w.ninv6), dev(w.mask, torch.uint8))
    M6 = w.M6()
    return plan, w, d, M6


def _rho(M6, d):
    A = np.empty((M6.shape[0], 3, 3))
    A[:, 0, 0], A[:, 0, 1], A[:, 0, 2] = M6[:, 0], M6[:, 1], M6[:, 2]
    A[:, 1, 0], A[:, 1, 1], A[:, 1, 2] = M6[:, 1], M6[:, 3], M6[:, 4]
    A[:, 2, 0], A[:, 2, 1], A[:, 2, 2] = M6[:, 2], M6[:, 4], M6[:, 5]
    return np.einsum("pij,jp->ip", A, d)


def test_pol_solve_parity_with_schedule_and_diagnostics(mf):
    """The T, Q, U Wiener filter (Wishart 3x3 noise blocks, masked band and discs) with a
    lambda schedule, against the oracle iterate; chi^2, |s_k - s_{k-1}| and |s_k| too."""
    nside, lmax = 16, 40
    plan, w, d, M6 = _problem(mf, nside, lmax)
    lam, its = [20.0, 3.0, 1.0], [30, 30, 40]
    s_alm, s_map, info, hist = plan.solve(dev(d[None]), lam=lam, iters=its, n_check=25)
    sched = np.repeat(lam, its)
    ref_alm, ref_map, dg = oracle.solve_pol(nside, lmax, w.cl4, M6, _rho(M6, d), lam=sched,
                                            diag=True)
    assert _rel_teb(s_alm.cpu().numpy()[0], ref_alm, lmax) < 1e-10
    assert rel(s_map.cpu().numpy()[0], ref_map) < 1e-10
    assert info[0].tau == pytest.approx(oracle.tau_pol(M6), rel=1e-12)
    assert info[0].n_dof == 3 * int(w.mask.sum())
    for r, k in enumerate([25, 50, 75, 100]):
        assert hist[r, 0, 2] == pytest.approx(dg[k - 1, 0], rel=1e-9)
        assert hist[r, 0, 3] == pytest.approx(dg[k - 1, 2], rel=1e-6)
        assert hist[r, 0, 4] == pytest.approx(dg[k - 1, 3], rel=1e-9)


def test_pol_batch_graph_and_rho_source(mf):
    nside, lmax = 8, 20
    plan, w, d, M6 = _problem(mf, nside, lmax, seed=1)
    rng = np.random.default_rng(4)
    ds = np.stack([d, d + rng.standard_normal(d.shape)])
    a_g, m_g, _ = plan.solve(dev(ds), iters=30)
    a_e, m_e, _ = plan.solve(dev(ds), iters=30, use_graph=False)
    a_1, m_1, _ = plan.solve(dev(ds[1:2]), iters=30)
    a_r, m_r, _ = plan.solve(dev(np.stack([_rho(M6, x) for x in ds])), iters=30, source_is_rho=True)
    assert torch.equal(a_g, a_e) and torch.equal(m_g, m_e)
    assert torch.equal(a_g[1], a_1[0])
    assert rel(a_r.cpu().numpy(), a_g.cpu().numpy()) < 1e-13
    ref, _ = oracle.solve_pol(nside, lmax, w.cl4, M6, _rho(M6, ds[1]), niter=30)
    assert _rel_teb(a_g.cpu().numpy()[1], ref, lmax) < 1e-10


def test_pol_fluctuation_source_parity_and_solve(mf):
    nside, lmax = 8, 20
    plan, w, d, M6 = _problem(mf, nside, lmax, seed=2)
    rng = np.random.default_rng(5)
    g1 = rng.standard_normal((2, 3, w.npix))
    h = np.stack([np.stack([W.white_alm(rng, lmax) for _ in range(3)]) for _ in range(2)])
    rho = plan.fluctuation_rhs(dev(g1), dev(h, torch.complex128))
    rho_np = rho.cpu().numpy()
    for b in range(2):
        assert rel(rho_np[b], oracle.fluct_rho_pol(nside, lmax, w.cl4, M6, g1[b], h[b])) < 1e-12
    f, _, _ = plan.solve(rho, iters=40, source_is_rho=True)
    ref, _ = oracle.solve_pol(nside, lmax, w.cl4, M6, rho_np[0], niter=40)
    assert _rel_teb(f.cpu().numpy()[0], ref, lmax) < 1e-10


def test_pol_errors(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    nside, lmax = 4, 8
    with pytest.raises(MFWFError):
        mf.Plan(nside, lmax, spin=1)
    plan = mf.Plan(nside, lmax, spin=2)
    w = W.config3(0, nside, lmax, ndisc=1, band_z=0.0)
    bad = w.ninv6.copy()
    bad[5, 1] = 10.0 * np.sqrt(bad[5, 0] * bad[5, 3])  # |TQ| > sqrt(TT QQ): indefinite block
    with pytest.raises(MFWFError, match="status -3"):
        plan.set_covariances(w.cl4, dev(bad), dev(w.mask, torch.uint8))
    cl_bad = w.cl4.copy()
    cl_bad[3, 5] = 2.0 * np.sqrt(cl_bad[0, 5] * cl_bad[1, 5])  # TE^2 > TT EE
    with pytest.raises(MFWFError):
        plan.set_covariances(cl_bad, dev(w.ninv6), dev(w.mask, torch.uint8))
    with pytest.raises(MFWFError, match="status -4"):
        plan.set_covariances(w.cl4, dev(w.ninv6), dev(np.zeros(w.npix, np.uint8), torch.uint8))


def test_pol_full_size_sampled(mf):
    """nside 512, lmax 1024: the polarized synthesis on four rings (pole, polar cap, belt,
    equator) and the analysis for five values of m against the oracle's per-ring and per-m
    evaluations."""
    nside, lmax = 512, 1024
    rng = np.random.default_rng(11)
    a = _teb(rng, lmax)
    plan = mf.Plan(nside, lmax, spin=2)
    maps = plan.sht_inv(dev(a, torch.complex128)).cpu().numpy()[0]
    z, s, start, nphi, phi0 = oracle.rings(nside)
    for r in (1, 2, 300, 700, 1024):
        ref = oracle.alm2map_pol_ring(nside, lmax, a[0], r)
        got = maps[:, start[r - 1]:start[r - 1] + nphi[r - 1]]
        # On the rings next to the poles the FP64 bracket of s^2 F+ cancels to O(s^2) for
        # m = 0 (eps / sin^2 theta = 4e-11 on the first ring at nside 512); the oracle forms
        # it in long double.
        tol = 1e-10 if r <= 2 else 1e-11
        assert rel(got, ref) < tol, (r, rel(got, ref))
    mp = rng.standard_normal((3, 12 * nside * nside))
    back = plan.sht_fwd(dev(mp[None])).cpu().numpy()[0]
    _, ms = W.alm_l_m(lmax)
    for m in (0, 1, 2, 400, 1024):
        ref = oracle.map2alm_pol_m(nside, lmax, mp, m)
        assert rel(back[:, ms == m], ref) < 1e-11, (m, rel(back[:, ms == m], ref))
