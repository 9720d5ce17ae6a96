"""nside 2048, lmax 4096 (FP64): the polar rings with more than 4096 pixels would need chirp-z
convolutions of 16384 points, beyond one workgroup's LDS in FP64, and take the split
transform instead: four Bluestein transforms of length n / 4 combined by decimation in time.

The split path is checked whole at small sizes, where a lowered split threshold
(MFWF_FFT_SPLIT_LEN, read at plan creation) sends most polar rings through it, including
rings shorter than lmax whose bins alias; and at nside 2048 on sampled outputs the oracle
computes one by one (synthesis on single rings, analysis for single m, the first messenger
iteration for single m, as in the nside 1024 checks).
"""
import os
from contextlib import contextmanager

import numpy as np
import pytest
import torch

import oracle
from paper_1210_4931_amd import workloads as W
from tests.gpu_util import dev, rel

pytestmark = pytest.mark.gpu

NSIDE, LMAX = 2048, 4096
# pole, cap, Bluestein of 8192 points (n = 4092), split (n = 6000, 8188), first belt ring,
# belt, equator, split and pole in the south
RINGS = (1, 3, 1023, 1500, 2047, 2048, 3000, 4096, 6145, 8191)
MS = (0, 1, 1500, 4095, 4096)


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


@contextmanager
def split_len(v):
    old = os.environ.get("MFWF_FFT_SPLIT_LEN")
    os.environ["MFWF_FFT_SPLIT_LEN"] = str(v)
    try:
        yield
    finally:
        if old is None:
            del os.environ["MFWF_FFT_SPLIT_LEN"]
        else:
            os.environ["MFWF_FFT_SPLIT_LEN"] = old


def _teb(rng, lmax):
    a = np.stack([W.white_alm(rng, lmax) for _ in range(3)])
    ls, _ = W.alm_l_m(lmax)
    a[1:, ls < 2] = 0.0
    return a


def _rel_alm(a, ref, lmax):
    _, ms = W.alm_l_m(lmax)
    w = np.sqrt(np.where(ms == 0, 1.0, 2.0))
    return rel(a * w, ref * w)


@pytest.mark.parametrize("nside,lmax,spin", [(16, 32, 0), (16, 64, 0), (32, 80, 0), (64, 128, 0),
                                             (16, 40, 2), (8, 32, 2)])
def test_split_transform_small_vs_oracle(mf, nside, lmax, spin):
    """Split threshold 32: every polar ring with a chirp-z length above 32 (n >= 20) is split;
    lmax up to 4 nside makes rings shorter than lmax fold several aliases per bin."""
    rng = np.random.default_rng(nside + lmax + spin)
    npix = 12 * nside * nside
    if spin == 0:
        a = np.stack([W.white_alm(rng, lmax) for _ in range(2)])
        x = rng.standard_normal((2, npix))
    else:
        a = np.stack([_teb(rng, lmax) for _ in range(2)])
        x = rng.standard_normal((2, 3, npix))
    with split_len(32):
        ps = mf.Plan(nside, lmax, spin=spin, max_batch=2)
    pw = mf.Plan(nside, lmax, spin=spin, max_batch=2)
    maps_s = ps.sht_inv(dev(a, torch.complex128))
    maps_w = pw.sht_inv(dev(a, torch.complex128))
    alm_s = ps.sht_fwd(dev(x))
    alm_w = pw.sht_fwd(dev(x))
    # the split plan takes another path (results differ in rounding) to the same transforms
    assert not torch.equal(maps_s, maps_w) and not torch.equal(alm_s, alm_w)
    maps_s, alm_s = maps_s.cpu().numpy(), alm_s.cpu().numpy()
    for b in range(2):
        if spin == 0:
            ref_m = oracle.alm2map(nside, lmax, a[b])
            ref_a = oracle.map2alm(nside, lmax, x[b])
        else:
            ref_m = oracle.alm2map_pol(nside, lmax, a[b])
            ref_a = oracle.map2alm_pol(nside, lmax, x[b])
        assert rel(maps_s[b], ref_m) < 1e-12, (b, rel(maps_s[b], ref_m))
        assert _rel_alm(alm_s[b], ref_a, lmax) < 1e-12, (b, _rel_alm(alm_s[b], ref_a, lmax))


def test_split_transform_small_solve(mf):
    """30 iterations of the filter on a split plan against the oracle."""
    nside, lmax = 32, 64
    wl = W.config1(seed=3, nside=nside, lmax=lmax)
    sig = oracle.alm2map(nside, lmax, wl.signal_alm)
    d = sig + np.sqrt(wl.noise_var) * wl.noise_white
    M = wl.mask / wl.noise_var
    with split_len(32):
        plan = mf.Plan(nside, lmax)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    s_alm, s_map, _ = plan.solve(dev(d[None]), iters=30)
    ref_alm, ref_map = oracle.solve(nside, lmax, wl.cl, M, M * d, niter=30)
    assert _rel_alm(s_alm.cpu().numpy()[0], ref_alm, lmax) < 1e-11
    assert rel(s_map.cpu().numpy()[0], ref_map) < 1e-11


def test_split_transform_rejects_fp32_spin2_above_1024(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    with pytest.raises(MFWFError, match="FP32"):
        mf.Plan(2048, 4096, dtype="f32", spin=2)


def test_split_transform_small_f32(mf):
    """The batched FP32 form on a split plan (threshold 32): its transforms (FP32 rows through
    the split kernels) and 30 chained iterations (the split rings folded from and stored into
    the matrix-core columns, with the pixel update inside the split sub-transforms) against
    the oracle; a served request on the same shape equals the standalone solve bitwise."""
    nside, lmax, B = 32, 64, 3
    wl = W.config1(seed=3, nside=nside, lmax=lmax)
    sig = oracle.alm2map(nside, lmax, wl.signal_alm)
    M = wl.mask / wl.noise_var
    rng = np.random.default_rng(8)
    d = np.stack([sig + np.sqrt(wl.noise_var) * (wl.noise_white if b == 0 else rng.standard_normal(sig.size))
                  for b in range(B)])
    with split_len(32):
        plan = mf.Plan(nside, lmax, max_batch=B, dtype="f32")
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    a = np.stack([W.white_alm(rng, lmax) for _ in range(B)])
    mp = plan.sht_inv(dev(a, torch.complex128)).cpu().numpy()
    back = plan.sht_fwd(dev(d)).cpu().numpy()
    for b in range(B):
        assert rel(mp[b], oracle.alm2map(nside, lmax, a[b])) < 1e-5
        assert _rel_alm(back[b], oracle.map2alm(nside, lmax, d[b]), lmax) < 1e-5
    s_alm, s_map, _ = plan.solve(dev(d), iters=30)
    for b in range(B):
        ref_alm, ref_map = oracle.solve(nside, lmax, wl.cl, M, M * d[b], niter=30)
        assert _rel_alm(s_alm.cpu().numpy()[b], ref_alm, lmax) < 1e-5
        assert rel(s_map.cpu().numpy()[b], ref_map) < 1e-5
    with split_len(32):  # the server creates the pool's plan when it admits the request
        srv = mf.Server(slots=2, hbm_gb=8.0)
        try:
            rid, sa, sm = srv.submit(nside, lmax, wl.cl, dev(1.0 / wl.noise_var), dev(d[0]),
                                     mask=dev(wl.mask, torch.uint8), dtype="f32", iters=30)
            srv.wait(rid)
        finally:
            srv.close()
    with split_len(32):
        p1 = mf.Plan(nside, lmax, max_batch=1, dtype="f32")
    p1.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    a1, m1, _ = p1.solve(dev(d[:1]), iters=30)
    assert torch.equal(sa, a1[0]) and torch.equal(sm, m1[0])


def test_nside2048_f32_batched_sampled(mf):
    """The batched FP32 form at nside 2048 / lmax 4096, where the contractions generate
    lambda from the FP64 recurrence (no table) and the split rings run on the columns: the
    synthesis on single rings and the analysis of single m against the oracle, and two
    chained iterations on two maps against the FP64 path after the same iterations."""
    rng = np.random.default_rng(47)
    plan = mf.Plan(NSIDE, LMAX, max_batch=2, dtype="f32")
    assert plan.tuning()["lamgen"] == 1
    a = np.stack([W.white_alm(rng, LMAX) for _ in range(2)])
    mp = plan.sht_inv(dev(a, torch.complex128)).cpu().numpy()
    z, s, start, nphi, phi0 = oracle.rings(NSIDE)
    for r in (3, 1500, 2047, 4096, 6145):
        ref = oracle.alm2map_ring(NSIDE, LMAX, a[1], r)
        got = mp[1, start[r - 1]:start[r - 1] + nphi[r - 1]]
        print("FP32 ring", r, "rel", rel(got, ref), flush=True)
        assert rel(got, ref) < 1e-5, (r, rel(got, ref))
    del mp
    x = rng.standard_normal((2, 12 * NSIDE * NSIDE))
    back = plan.sht_fwd(dev(x)).cpu().numpy()
    _, ms = W.alm_l_m(LMAX)
    for m in (0, 1500, 4096):
        ref = oracle.map2alm_m(NSIDE, LMAX, x[0], m)
        print("FP32 m", m, "rel", rel(back[0][ms == m], ref), flush=True)
        assert rel(back[0][ms == m], ref) < 1e-5, (m, rel(back[0][ms == m], ref))
    del back
    wl = W.config2(0, NSIDE, LMAX)
    d = np.sqrt(wl.noise_var) * np.stack([wl.noise_white, W.batch_noise(1, wl.npix)])
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    s32, m32, _ = plan.solve(dev(d), iters=2)
    del plan
    p64 = mf.Plan(NSIDE, LMAX, max_batch=2)
    p64.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    s64, m64, _ = p64.solve(dev(d), iters=2)
    for b in range(2):
        ea = _rel_alm(s32[b].cpu().numpy(), s64[b].cpu().numpy(), LMAX)
        em = rel(m32[b].cpu().numpy(), m64[b].cpu().numpy())
        print("FP32 vs FP64 after 2 iterations, map", b, ea, em, flush=True)
        assert ea < 1e-5 and em < 1e-5


def test_nside2048_sht_sampled(mf):
    rng = np.random.default_rng(41)
    a = W.white_alm(rng, LMAX)
    plan = mf.Plan(NSIDE, LMAX)
    mp = plan.sht_inv(dev(a[None], torch.complex128)).cpu().numpy()[0]
    z, s, start, nphi, phi0 = oracle.rings(NSIDE)
    for r in RINGS:
        ref = oracle.alm2map_ring(NSIDE, LMAX, a, r)
        got = mp[start[r - 1]:start[r - 1] + nphi[r - 1]]
        # next to the poles both sides carry an error growing like l^2 eps (Unsold's sum pins
        # the oracle's: 4.7e-10 at l = 4096 on the first ring)
        tol = 2e-9 if r in (1, 3, 8191) else 3e-11
        print("ring", r, "n", nphi[r - 1], "rel", rel(got, ref))
        assert rel(got, ref) < tol, (r, rel(got, ref))
    del mp
    x = rng.standard_normal(12 * NSIDE * NSIDE)
    back = plan.sht_fwd(dev(x[None])).cpu().numpy()[0]
    _, ms = W.alm_l_m(LMAX)
    for m in MS:
        ref = oracle.map2alm_m(NSIDE, LMAX, x, m)
        print("m", m, "rel", rel(back[ms == m], ref))
        assert rel(back[ms == m], ref) < 3e-11, (m, rel(back[ms == m], ref))


def test_nside2048_first_iteration_sampled(mf):
    wl = W.config2(0, NSIDE, LMAX)
    z, _ = W.pixel_centres(NSIDE)
    d = np.sqrt(wl.noise_var) * wl.noise_white + 80.0 * z + 40.0 * (3.0 * z * z - 1.0)
    M = wl.mask / wl.noise_var
    plan = mf.Plan(NSIDE, LMAX)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    s_alm, _, info = plan.solve(dev(d[None]), iters=1, want_map=False)
    got = s_alm.cpu().numpy()[0]
    tau = oracle.tau(M)
    assert info[0].tau == pytest.approx(tau, rel=1e-15)
    omega = 4.0 * np.pi / M.size
    ls, ms = W.alm_l_m(LMAX)
    t = tau * (M * d)                      # pixel update of Eq. 3 from s = 0, lambda = 1
    for m in MS:
        a = oracle.map2alm_m(NSIDE, LMAX, t, m)
        l = ls[ms == m]
        C = wl.cl[l]
        f = np.where(C > 0, C / np.where(C > 0, C + tau * omega, 1.0), 0.0)
        assert rel(got[ms == m], f * a) < 3e-11, (m, rel(got[ms == m], f * a))


def test_nside2048_pol_sht_sampled(mf):
    """T, Q, U at nside 2048 / lmax 4096 (the split rings carry three rows per map): the
    synthesis on single rings and the analysis of one m (2500: polar and belt rings, 1597
    values of l) against the oracle (whose one-m spin-2 analysis takes about a minute at
    this size), and the adjoint identity <Y a, x> = <a, A x> / Omega over all coefficients."""
    rng = np.random.default_rng(43)
    a = _teb(rng, LMAX)
    plan = mf.Plan(NSIDE, LMAX, spin=2)
    mp = plan.sht_inv(dev(a[None], torch.complex128)).cpu().numpy()[0]
    z, s, start, nphi, phi0 = oracle.rings(NSIDE)
    for r in (3, 1023, 1500, 2047, 4096, 6145):
        ref = oracle.alm2map_pol_ring(NSIDE, LMAX, a, r)
        got = mp[:, start[r - 1]:start[r - 1] + nphi[r - 1]]
        print("ring", r, "n", nphi[r - 1], "rel", rel(got, ref))
        assert rel(got, ref) < (2e-9 if r == 3 else 3e-11), (r, rel(got, ref))
    x = rng.standard_normal((3, 12 * NSIDE * NSIDE))
    back = plan.sht_fwd(dev(x[None])).cpu().numpy()[0]
    _, ms = W.alm_l_m(LMAX)
    wgt = np.where(ms == 0, 1.0, 2.0)
    lhs = float(np.sum(mp * x))
    rhs = float(np.sum(wgt * (np.conj(a) * back).real)) / (4.0 * np.pi / x.shape[1])
    print("adjoint", lhs, rhs)
    assert lhs == pytest.approx(rhs, rel=1e-11)
    m = 2500
    print("oracle spin-2 analysis of m = %d at nside %d (about a minute)" % (m, NSIDE), flush=True)
    ref = oracle.map2alm_pol_m(NSIDE, LMAX, x, m)
    got = back[:, ms == m]
    for c in range(3):
        print("m", m, "component", c, "rel", rel(got[c], ref[c]))
        assert rel(got[c], ref[c]) < 3e-11, (c, rel(got[c], ref[c]))
