"""Batched FP32 form (MFMA Legendre contractions) against the FP64 oracle.

Tolerance: 1e-5 relative error per result (the stated accuracy target of the FP32 form), over
the real harmonic dof or the map.  The FP32 pieces are the tabulated lambda_lm, the
ring-Fourier coefficients and the harmonic coefficients fed to the matrix cores; each
rounding is ~6e-8 relative and the sums run over at most a few hundred terms per output with
FP32 accumulation, so one transform lands near 1e-6; the measured error of 300 iterations is
reported by the tests' assertion messages.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1210_4931_amd import workloads as W
from tests.gpu_util import dev, rel, rel_alm, temperature_problem

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


@pytest.mark.parametrize("nside,lmax,nmaps", [(2, 8, 3), (8, 20, 5), (16, 64, 17), (32, 128, 33),
                                             (64, 200, 40)])
def test_f32_sht_pair_parity(mf, nside, lmax, nmaps):
    rng = np.random.default_rng(nside + lmax)
    alm = np.stack([W.white_alm(rng, lmax) for _ in range(nmaps)])
    plan = mf.Plan(nside, lmax, max_batch=32, dtype="f32")
    maps = plan.sht_inv(dev(alm, torch.complex128)).cpu().numpy()
    back = plan.sht_fwd(dev(maps)).cpu().numpy()
    for b in range(0, nmaps, max(1, nmaps // 4)):
        ref = oracle.alm2map(nside, lmax, alm[b])
        assert rel(maps[b], ref) < TOL, ("synthesis", b, rel(maps[b], ref))
        refa = oracle.map2alm(nside, lmax, maps[b])
        assert rel_alm(back[b], refa, lmax) < TOL, ("analysis", b, rel_alm(back[b], refa, lmax))


def _setup(mf, nside, lmax, max_batch, seed=0):
    wl, d, M = temperature_problem(nside, lmax, seed)
    plan = mf.Plan(nside, lmax, max_batch=max_batch, dtype="f32")
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    return plan, wl, d, M


def test_f32_wf_and_cr_batch_parity_300_iterations(mf):
    """The batched workload at a small size: 8 Wiener-filter data sets and 8 fluctuation
    sources in one batch, 300 iterations, each against the oracle iterate."""
    nside, lmax = 32, 64
    plan, wl, d, M = _setup(mf, nside, lmax, max_batch=16)
    rng = np.random.default_rng(4)
    ds = np.stack([d + rng.standard_normal(d.size) * np.sqrt(wl.noise_var) for _ in range(8)])
    draws = [W.fluctuation_draws(100 + k, nside, lmax) for k in range(8)]
    rho_cr = plan.fluctuation_rhs(dev(np.stack([g for g, _ in draws])),
                                  dev(np.stack([h for _, h in draws]), torch.complex128))
    rho = torch.cat([dev(M[None] * ds), rho_cr], 0)
    s_alm, s_map, info = plan.solve(rho, iters=300, source_is_rho=True)
    s_alm, s_map, rho_np = s_alm.cpu().numpy(), s_map.cpu().numpy(), rho.cpu().numpy()
    errs = []
    for b in (0, 5, 8, 15):
        if b >= 8:
            g1, h = draws[b - 8]
            ref_rho = oracle.fluct_rho(nside, lmax, wl.cl, M, g1, h)
            assert rel(rho_np[b], ref_rho) < TOL
        ref_alm, ref_map = oracle.solve(nside, lmax, wl.cl, M, rho_np[b], niter=300)
        errs.append((rel_alm(s_alm[b], ref_alm, lmax), rel(s_map[b], ref_map)))
    assert max(max(e) for e in errs) < TOL, errs


def test_f32_batch_invariance_and_graph(mf):
    nside, lmax = 16, 40
    plan, wl, d, M = _setup(mf, nside, lmax, max_batch=20)
    rng = np.random.default_rng(2)
    ds = np.stack([d + rng.standard_normal(d.size) for _ in range(20)])
    a_all, m_all, _ = plan.solve(dev(ds), iters=15)
    a_one, m_one, _ = plan.solve(dev(ds[7:8]), iters=15)
    assert torch.equal(a_all[7], a_one[0]) and torch.equal(m_all[7], m_one[0])
    a_eg, m_eg, _ = plan.solve(dev(ds), iters=15, use_graph=False)
    assert torch.equal(a_all, a_eg) and torch.equal(m_all, m_eg)


def test_f32_two_stream_ring_step_at_nside_512(mf):
    """At nside 512 the ring step's two transform classes (4096-point chirp-z transforms in
    512-thread workgroups, the other rings in 256-thread ones) run side by side, the first on
    the plan's second stream: graph-replayed, eager, repeated and map-order solves (the last
    without the chained ring step) give the same bits."""
    nside, lmax = 512, 128
    plan, wl, d, M = _setup(mf, nside, lmax, max_batch=3)
    rng = np.random.default_rng(9)
    ds = np.stack([d + rng.standard_normal(d.size) for _ in range(3)])
    a_g, m_g, _ = plan.solve(dev(ds), iters=8)
    a_e, m_e, _ = plan.solve(dev(ds), iters=8, use_graph=False)
    a_r, m_r, _ = plan.solve(dev(ds), iters=8)
    a_m, m_m, _ = plan.solve(dev(ds), iters=8, chained=False)
    for a, m in ((a_e, m_e), (a_r, m_r), (a_m, m_m)):
        assert torch.equal(a_g, a) and torch.equal(m_g, m)
    assert torch.isfinite(a_g).all() and float(a_g.abs().max()) > 0.0


def test_f32_diagnostics(mf):
    nside, lmax = 16, 40
    plan, wl, d, M = _setup(mf, nside, lmax, max_batch=4)
    _, _, info = plan.solve(dev(d[None]), iters=20)
    _, _, dg = oracle.solve(nside, lmax, wl.cl, M, M * d, niter=20, diag=True)
    assert info[0].chi2 == pytest.approx(dg[-1, 0], rel=1e-5)
    assert info[0].snorm == pytest.approx(dg[-1, 3], rel=1e-5)


def test_f32_full_size_sampled(mf):
    """nside 256, lmax 512, 64 right-hand sides (the batched benchmark shape): two sampled
    maps against the oracle after 2 iterations."""
    nside, lmax, B = 256, 512, 64
    wl = W.config2(0, nside, lmax)
    M = wl.mask * (4.0 / wl.noise_var)
    plan = mf.Plan(nside, lmax, max_batch=B, dtype="f32")
    plan.set_covariances(wl.cl, dev(4.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    rng = np.random.default_rng(0)
    sig = plan.sht_inv(dev(wl.signal_alm[None], torch.complex128))
    noise = torch.as_tensor(rng.standard_normal((B, wl.npix)) * np.sqrt(wl.noise_var / 4.0)).cuda()
    d = sig + noise
    s_alm, _, _ = plan.solve(d, iters=2)
    d_np, s_np = d.cpu().numpy(), s_alm.cpu().numpy()
    for b in (0, B - 1):
        ref, _ = oracle.solve(nside, lmax, wl.cl, M, M * d_np[b], niter=2)
        assert rel_alm(s_np[b], ref, lmax) < TOL


def test_f32_benchmark_size_300_iterations(mf):
    """nside 512, lmax 1024, 64 maps, 300 iterations: the benchmark's solve in its launch
    configuration (chained FP32 iterations over a batch of 64).  Two maps of the batch against
    the FP64 path, which the FP64 tests pin to the oracle at this size (two iterations, 5e-12)
    and over 300 iterations at nside 32 (the oracle needs tens of minutes for 300 iterations
    here); and after two iterations one map against the oracle itself."""
    nside, lmax, B = 512, 1024, 64
    wl = W.config2(0, nside, lmax)
    ninv, mask = dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8)
    M = wl.mask / wl.noise_var
    p32 = mf.Plan(nside, lmax, max_batch=B, dtype="f32")
    p32.set_covariances(wl.cl, ninv, mask)
    sig = p32.sht_inv(dev(wl.signal_alm[None], torch.complex128))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    d = sig + dev(np.sqrt(wl.noise_var))[None] * torch.randn((B, wl.npix), generator=gen,
                                                             device="cuda", dtype=torch.float64)
    s2, _, _ = p32.solve(d, iters=2)
    ref2, _ = oracle.solve(nside, lmax, wl.cl, M, M * d[B - 1].cpu().numpy(), niter=2)
    e2 = rel_alm(s2.cpu().numpy()[B - 1], ref2, lmax)
    s_alm, s_map, _ = p32.solve(d, iters=300)
    del p32
    pick = [0, B - 1]
    p64 = mf.Plan(nside, lmax, max_batch=len(pick), dtype="f64")
    p64.set_covariances(wl.cl, ninv, mask)
    ref_alm, ref_map, _ = p64.solve(d[pick].contiguous(), iters=300)
    ra, rm = ref_alm.cpu().numpy(), ref_map.cpu().numpy()
    sa, sm = s_alm.cpu().numpy(), s_map.cpu().numpy()
    errs = [(rel_alm(sa[b], ra[i], lmax), rel(sm[b], rm[i])) for i, b in enumerate(pick)]
    print("64-map FP32 batch at nside 512: 2 iterations vs the oracle", e2,
          "; 300 iterations vs FP64 (alm, map):", errs)
    assert e2 < TOL
    assert max(max(e) for e in errs) < TOL, errs


def test_f32_chained_iterations_chunks_checks_and_stages(mf):
    """The batched solve chains its iterations through the synthesis columns: splitting the
    maps into chunks of max_batch, diagnostics checks in the middle of a stage (which
    materialise the map without touching the chain) and a change of lambda between stages
    leave every result bitwise equal to the plain runs, and the result equals the oracle's
    iterate with the same schedule."""
    nside, lmax = 16, 40
    plan, wl, d, M = _setup(mf, nside, lmax, max_batch=4)
    rng = np.random.default_rng(12)
    ds = np.stack([d + rng.standard_normal(d.size) for _ in range(9)])  # chunks 4, 4, 1
    lam, its = [30.0, 1.0], [7, 23]
    a_all, m_all, _ = plan.solve(dev(ds), lam=lam, iters=its)
    for b in (0, 5, 8):
        a1, m1, _ = plan.solve(dev(ds[b:b + 1]), lam=lam, iters=its)
        assert torch.equal(a_all[b], a1[0]) and torch.equal(m_all[b], m1[0])
    a_chk, m_chk, _, hist = plan.solve(dev(ds), lam=lam, iters=its, n_check=5)
    assert torch.equal(a_all, a_chk) and torch.equal(m_all, m_chk)
    assert hist.shape[0] == 6  # checks at 5, 10, ..., 30
    # the same iterations from the pixel map (forward transforms, layout changes, inverse
    # transforms every iteration): the same values
    a_map, m_map, _ = plan.solve(dev(ds), lam=lam, iters=its, chained=False)
    assert torch.equal(a_all, a_map) and torch.equal(m_all, m_map)
    ref_alm, ref_map = oracle.solve(nside, lmax, wl.cl, M, M * ds[5], lam=np.repeat(lam, its))
    assert rel_alm(a_all.cpu().numpy()[5], ref_alm, lmax) < TOL
    assert rel(m_all.cpu().numpy()[5], ref_map) < TOL


def test_time_kernels_stages_and_state(mf):
    """mfwf_time_kernels: one duration per stage (in the batched temperature form the
    inverse transforms run inside the chained ring step, [1], so [5] reads 0; in the FP64
    path the pixel update runs inside the forward transforms, so [0] reads 0), and a solve
    after it gives the result it gave before (the timing runs leave no state behind)."""
    nside, lmax = 16, 40
    plan, wl, d, M = _setup(mf, nside, lmax, max_batch=4)
    ds = dev(np.stack([d, 2.0 * d]))
    a1, m1, _ = plan.solve(ds, iters=12)
    ms = plan.time_kernels(2, 3)
    assert len(ms) == 6 and all(np.isfinite(ms)) and min(ms) >= 0.0
    assert ms[1] > 0.0 and ms[2] > 0.0 and ms[4] > 0.0 and ms[5] == 0.0
    a2, m2, _ = plan.solve(ds, iters=12)
    assert torch.equal(a1, a2) and torch.equal(m1, m2)
    p64 = mf.Plan(nside, lmax)
    p64.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    b1 = p64.solve(ds[:1], iters=12)[0]
    ms64 = p64.time_kernels(1, 3)  # the FP64 pixel update runs inside the forward transforms
    assert ms64[0] == 0.0 and all(v > 0.0 for v in ms64[1:])
    assert torch.equal(p64.solve(ds[:1], iters=12)[0], b1)


def test_config4_downgraded_wf_and_cr_batch_300_iterations(mf):
    """nside 256, lmax 512, 64 maps in one batch: 32 Wiener-filter data sets (seeds 0-31)
    and 32 fluctuation sources (seeds 32-63), 300 iterations of the FP32 form.  Every map
    against the FP64 path on the same sources (the FP64 path is pinned to the oracle), the
    fluctuation source against the oracle's, and one map of each kind against the oracle
    after two iterations."""
    nside, lmax, B = 256, 512, 64
    w = W.config4(0)
    M = w.mask / w.noise_var
    ninv, mask = dev(1.0 / w.noise_var), dev(w.mask, torch.uint8)
    p64 = mf.Plan(nside, lmax, max_batch=B)
    p64.set_covariances(w.cl, ninv, mask)
    ls, _ = W.alm_l_m(lmax)
    draws_wf = [W.config4_draws(b) for b in range(32)]
    sig = p64.sht_inv(dev(np.stack([np.sqrt(w.cl[ls]) * h for h, _ in draws_wf]),
                          torch.complex128)).cpu().numpy()
    d = sig + np.sqrt(w.noise_var) * np.stack([g for _, g in draws_wf])
    draws_cr = [W.fluctuation_draws(32 + k, nside, lmax) for k in range(32)]
    rho_cr = p64.fluctuation_rhs(dev(np.stack([g for g, _ in draws_cr])),
                                 dev(np.stack([h for _, h in draws_cr]), torch.complex128))
    g1, h = draws_cr[31]
    assert rel(rho_cr[31].cpu().numpy(), oracle.fluct_rho(nside, lmax, w.cl, M, g1, h)) < 1e-12
    rho = torch.cat([dev(M[None] * d), rho_cr], 0)
    ref_alm, ref_map, _ = p64.solve(rho, iters=300, source_is_rho=True)
    del p64
    p32 = mf.Plan(nside, lmax, max_batch=B, dtype="f32")
    p32.set_covariances(w.cl, ninv, mask)
    s_alm, s_map, _ = p32.solve(rho, iters=300, source_is_rho=True)
    sa, sm = s_alm.cpu().numpy(), s_map.cpu().numpy()
    ra, rm = ref_alm.cpu().numpy(), ref_map.cpu().numpy()
    errs = [max(rel_alm(sa[b], ra[b], lmax), rel(sm[b], rm[b])) for b in range(B)]
    print("FP32 form vs FP64 after 300 iterations, worst WF / CR map:", max(errs[:32]),
          max(errs[32:]))
    assert max(errs) < TOL, (int(np.argmax(errs)), max(errs))
    a2, m2, _ = p32.solve(rho[[0, 63]], iters=2, source_is_rho=True)
    rho_np = rho[[0, 63]].cpu().numpy()
    for k in range(2):
        oa, om = oracle.solve(nside, lmax, w.cl, M, rho_np[k], niter=2)
        assert rel_alm(a2[k].cpu().numpy(), oa, lmax) < TOL
        assert rel(m2[k].cpu().numpy(), om) < TOL
