"""Batched FP32 form of the T, Q, U filter (spin-2 Legendre contractions on the matrix cores)
against the FP64 oracle.

Tolerance: 1e-5 relative (the FP32 form's accuracy target) over the real (T, E, B) harmonic
dof or the (T, Q, U) maps.  The FP32 pieces are the lambda, F+ and F- tables, the ring-Fourier
coefficients and the harmonic coefficients fed to the matrix cores; everything else (maps,
pixel update with the 3x3 blocks, filter, norms) is FP64.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1210_4931_amd import workloads as W
from tests.gpu_util import dev, rel

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


def _teb(rng, lmax, n):
    a = np.stack([np.stack([W.white_alm(rng, lmax) for _ in range(3)]) for _ in range(n)])
    ls, _ = W.alm_l_m(lmax)
    a[:, 1:, ls < 2] = 0.0
    return a


def _rel_teb(a, ref, lmax):
    _, ms = W.alm_l_m(lmax)
    w = np.sqrt(np.where(ms == 0, 1.0, 2.0))
    return rel(a * w, ref * w)


def _rho(M6, d):
    A = np.empty((M6.shape[0], 3, 3))
    A[:, 0, 0], A[:, 0, 1], A[:, 0, 2] = M6[:, 0], M6[:, 1], M6[:, 2]
    A[:, 1, 0], A[:, 1, 1], A[:, 1, 2] = M6[:, 1], M6[:, 3], M6[:, 4]
    A[:, 2, 0], A[:, 2, 1], A[:, 2, 2] = M6[:, 2], M6[:, 4], M6[:, 5]
    return np.einsum("pij,jp->ip", A, d)


@pytest.mark.parametrize("nside,lmax,nmaps", [(2, 6, 2), (4, 12, 3), (8, 32, 5), (16, 40, 17),
                                             (32, 64, 9)])
def test_pol_f32_sht_pair_parity(mf, nside, lmax, nmaps):
    rng = np.random.default_rng(nside * 7 + lmax)
    a = _teb(rng, lmax, nmaps)
    plan = mf.Plan(nside, lmax, max_batch=16, spin=2, dtype="f32")
    maps = plan.sht_inv(dev(a, torch.complex128)).cpu().numpy()
    mp = rng.standard_normal((nmaps, 3, 12 * nside * nside))
    back = plan.sht_fwd(dev(mp)).cpu().numpy()
    for b in range(0, nmaps, max(1, nmaps // 3)):
        ref = oracle.alm2map_pol(nside, lmax, a[b])
        assert rel(maps[b], ref) < TOL, ("synthesis", b, rel(maps[b], ref))
        refa = oracle.map2alm_pol(nside, lmax, mp[b])
        assert _rel_teb(back[b], refa, lmax) < TOL, ("analysis", b, _rel_teb(back[b], refa, lmax))


def _problem(mf, nside, lmax, max_batch, seed=0):
    w = W.config3(seed, nside, lmax, ndisc=10, band_z=0.15, nu=10)
    sig = oracle.alm2map_pol(nside, lmax, w.signal_alm)
    d = w.data_from_signal_maps(sig)
    plan = mf.Plan(nside, lmax, max_batch=max_batch, spin=2, dtype="f32")
    plan.set_covariances(w.cl4, dev(w.ninv6), dev(w.mask, torch.uint8))
    return plan, w, d, w.M6()


def test_pol_f32_wf_and_cr_batch_parity_300_iterations(mf):
    """Two Wiener-filter data sets and two fluctuation sources in one batch, 300 iterations,
    each against the oracle iterate; the fluctuation sources against the oracle's too."""
    nside, lmax = 16, 32
    plan, w, d, M6 = _problem(mf, nside, lmax, max_batch=4)
    rng = np.random.default_rng(6)
    ds = np.stack([d, d + rng.standard_normal(d.shape)])
    g1 = rng.standard_normal((2, 3, w.npix))
    h = _teb(rng, lmax, 2)
    rho_cr = plan.fluctuation_rhs(dev(g1), dev(h, torch.complex128))
    rho_np = rho_cr.cpu().numpy()
    for b in range(2):
        ref = oracle.fluct_rho_pol(nside, lmax, w.cl4, M6, g1[b], h[b])
        assert rel(rho_np[b], ref) < TOL, ("fluctuation source", b, rel(rho_np[b], ref))
    rho = torch.cat([dev(np.stack([_rho(M6, x) for x in ds])), rho_cr], 0)
    s_alm, s_map, info = plan.solve(rho, iters=300, source_is_rho=True)
    s_alm, s_map, rho_all = s_alm.cpu().numpy(), s_map.cpu().numpy(), rho.cpu().numpy()
    errs = []
    for b in range(4):
        ref_alm, ref_map = oracle.solve_pol(nside, lmax, w.cl4, M6, rho_all[b], niter=300)
        errs.append((_rel_teb(s_alm[b], ref_alm, lmax), rel(s_map[b], ref_map)))
    assert max(max(e) for e in errs) < TOL, errs
    assert info[0].n_dof == 3 * int(w.mask.sum())


def test_pol_f32_batch_invariance_and_graph(mf):
    nside, lmax = 8, 20
    plan, w, d, M6 = _problem(mf, nside, lmax, max_batch=9, seed=1)
    rng = np.random.default_rng(3)
    ds = np.stack([d + rng.standard_normal(d.shape) for _ in range(9)])
    a_all, m_all, _ = plan.solve(dev(ds), iters=12)
    a_one, m_one, _ = plan.solve(dev(ds[6:7]), iters=12)
    assert torch.equal(a_all[6], a_one[0]) and torch.equal(m_all[6], m_one[0])
    a_eg, m_eg, _ = plan.solve(dev(ds), iters=12, use_graph=False)
    assert torch.equal(a_all, a_eg) and torch.equal(m_all, m_eg)


@pytest.mark.parametrize("nside,lmax", [(16, 40), (32, 64)])
def test_pol_f32_chained_iterations_equal_the_map_order(mf, nside, lmax):
    """The T, Q, U batched solve chains its iterations through the synthesis columns (the
    3x3 pixel update inside the ring step): every result, with a change of lambda between
    stages, a chunked batch and checks in the middle of a stage, is bitwise the result of
    the same iterations run from the pixel map, and the chained result equals the oracle's
    iterate."""
    plan, w, d, M6 = _problem(mf, nside, lmax, max_batch=3, seed=4)
    rng = np.random.default_rng(5)
    ds = np.stack([d + rng.standard_normal(d.shape) for _ in range(5)])  # chunks 3, 2
    lam, its = [10.0, 1.0], [6, 14]
    a_ch, m_ch, _ = plan.solve(dev(ds), lam=lam, iters=its)
    a_map, m_map, _ = plan.solve(dev(ds), lam=lam, iters=its, chained=False)
    assert torch.equal(a_ch, a_map) and torch.equal(m_ch, m_map)
    a_chk, m_chk, _, _ = plan.solve(dev(ds), lam=lam, iters=its, n_check=4)
    assert torch.equal(a_ch, a_chk) and torch.equal(m_ch, m_chk)
    ref_alm, ref_map = oracle.solve_pol(nside, lmax, w.cl4, M6, _rho(M6, ds[4]),
                                        lam=np.repeat(lam, its))
    assert _rel_teb(a_ch.cpu().numpy()[4], ref_alm, lmax) < TOL
    assert rel(m_ch.cpu().numpy()[4], ref_map) < TOL


def test_pol_f32_chained_equals_map_order_at_nside_512(mf):
    """At nside 512 the polar rings of more than 1024 pixels take chirp-z transforms of 4096
    points in 512-thread workgroups, the other rings 256-thread ones: a chained T, Q, U solve
    through both ring-step shapes equals the map-order solve bit for bit."""
    nside, lmax = 512, 64
    w = W.config3(6, nside, lmax, ndisc=10, band_z=0.15, nu=10)
    plan = mf.Plan(nside, lmax, max_batch=2, spin=2, dtype="f32")
    plan.set_covariances(w.cl4, dev(w.ninv6), dev(w.mask, torch.uint8))
    rng = np.random.default_rng(7)
    ds = 30.0 * rng.standard_normal((2, 3, w.npix))  # any data: the two orders must agree
    lam, its = [5.0, 1.0], [2, 3]
    a_ch, m_ch, _ = plan.solve(dev(ds), lam=lam, iters=its)
    a_map, m_map, _ = plan.solve(dev(ds), lam=lam, iters=its, chained=False)
    assert torch.equal(a_ch, a_map) and torch.equal(m_ch, m_map)
    assert torch.isfinite(a_ch).all() and float(a_ch.abs().max()) > 0.0


def test_pol_f32_schedule_and_diagnostics(mf):
    nside, lmax = 16, 40
    plan, w, d, M6 = _problem(mf, nside, lmax, max_batch=2, seed=2)
    lam, its = [10.0, 1.0], [20, 30]
    s_alm, s_map, info, hist = plan.solve(dev(d[None]), lam=lam, iters=its, n_check=25)
    ref_alm, ref_map, dg = oracle.solve_pol(nside, lmax, w.cl4, M6, _rho(M6, d),
                                            lam=np.repeat(lam, its), diag=True)
    assert _rel_teb(s_alm.cpu().numpy()[0], ref_alm, lmax) < TOL
    assert rel(s_map.cpu().numpy()[0], ref_map) < TOL
    for r, k in enumerate([25, 50]):
        assert hist[r, 0, 2] == pytest.approx(dg[k - 1, 0], rel=TOL)
        assert hist[r, 0, 4] == pytest.approx(dg[k - 1, 3], rel=TOL)


def test_pol_f32_benchmark_size_300_iterations(mf):
    """nside 512, lmax 1024, 300 iterations (the T, Q, U benchmark solve): the FP32 form
    against the FP64 T, Q, U path, which the FP64 tests pin to the oracle at this size
    (sampled transforms) and over the iteration at small sizes."""
    nside, lmax, B = 512, 1024, 2
    w = W.config3(0, nside, lmax)
    ninv6, mask = dev(w.ninv6), dev(w.mask, torch.uint8)
    p64 = mf.Plan(nside, lmax, max_batch=B, spin=2)
    p64.set_covariances(w.cl4, ninv6, mask)
    sig = p64.sht_inv(dev(w.signal_alm[None], torch.complex128)).cpu().numpy()[0]
    d1 = w.data_from_signal_maps(sig)
    rng = np.random.default_rng(9)
    d = dev(np.stack([d1, d1 + rng.standard_normal(d1.shape)]))
    ref_alm, ref_map, _ = p64.solve(d, iters=300)
    del p64
    p32 = mf.Plan(nside, lmax, max_batch=B, spin=2, dtype="f32")
    p32.set_covariances(w.cl4, ninv6, mask)
    s_alm, s_map, _ = p32.solve(d, iters=300)
    ra, rm = ref_alm.cpu().numpy(), ref_map.cpu().numpy()
    sa, sm = s_alm.cpu().numpy(), s_map.cpu().numpy()
    errs = [(_rel_teb(sa[b], ra[b], lmax), rel(sm[b], rm[b])) for b in range(B)]
    print("T, Q, U FP32 form vs FP64 after 300 iterations at nside 512 (alm, map):", errs)
    assert max(max(e) for e in errs) < TOL, errs
