"""Pins of the oracle's polarization (spin-2) part against what the mathematics fixes.

The spin-weighted functions are checked against closed forms for l = 2, against the
spin-raising definition itself (finite differences of SciPy's Y_lm), against the spin-2
Unsold sum rule and Gauss-Legendre orthonormality; the polarized transform against its
adjoint and the two symmetries E/B carry (a pure-E field has no B; a rotation of the
polarization angle rotates E into B); the T, Q, U messenger iteration against the paper's
special case of uniform noise and against the dense fixed point of its own linear system.
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle
from paper_1210_4931_amd import workloads as W

FOURPI = 4.0 * math.pi


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def spin_lambdas(lmax, m, z):
    fp, fm = oracle.spin2(lmax, m, z)
    return fp + fm, fp - fm   # 2lambda, (-2)lambda for l = m..lmax


# ----------------------------------------------------------------------------------------
# Spin-weighted functions
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("z", [0.97, 0.4, 0.0, -0.3, -0.999])
def test_spin2_closed_forms_l2(z):
    """The l = 2 spin-2 harmonics in their standard closed forms (e.g. the gravitational-
    wave literature's (-2)Y_22 = sqrt(5/64pi) (1 + cos theta)^2 e^{2 i phi}); the spin +2
    ones follow from (s)Y_lm(pi - theta) = (-1)^(l+m) (-s)Y_lm(theta) (phi shifted by pi)."""
    s = math.sqrt(1 - z * z)
    p2, m2 = spin_lambdas(2, 2, z)
    assert p2[0] == pytest.approx(math.sqrt(5 / (64 * math.pi)) * (1 - z) ** 2, rel=1e-14, abs=1e-16)
    assert m2[0] == pytest.approx(math.sqrt(5 / (64 * math.pi)) * (1 + z) ** 2, rel=1e-14)
    p1, m1 = spin_lambdas(2, 1, z)
    assert m1[1] == pytest.approx(math.sqrt(5 / (16 * math.pi)) * s * (1 + z), rel=1e-13)
    assert p1[1] == pytest.approx(-math.sqrt(5 / (16 * math.pi)) * s * (1 - z), rel=1e-13, abs=1e-16)
    p0, m0 = spin_lambdas(2, 0, z)
    assert p0[2] == pytest.approx(math.sqrt(15 / (32 * math.pi)) * s * s, rel=1e-13)
    assert m0[2] == pytest.approx(p0[2], rel=1e-14)
    # below l = 2 the spin-2 functions vanish
    assert p0[0] == p0[1] == m0[0] == m0[1] == 0.0


def _eth_twice(l, m, theta, lower, h=2e-4):
    """(+-2)lambda_lm(theta) from the definition sqrt((l-2)!/(l+2)!) (eth)^2 Y_lm with
    eth eta = -(sin th)^s [d_theta + i/sin th d_phi] (sin th)^-s eta on spin-s quantities
    (eth-bar: the complex conjugate operator), differentiating SciPy's Y_lm numerically in
    theta; the phi derivative of e^{i m phi} is exact."""
    sg = -1.0 if lower else 1.0   # eth-bar flips the sign of the phi term and of s

    def y(th):
        return sph_harm_y(l, m, th, 0.0).real

    def eth1(th):  # spin 0 -> spin +-1, at phi = 0 (all factors real)
        dy = (y(th + h) - y(th - h)) / (2 * h)
        return -(dy - sg * m / math.sin(th) * y(th))

    def eth2(th):  # spin +1 -> +2 (eth: s = 1) or -1 -> -2 (eth-bar: powers -s = +1)
        # eth: -(sin)^s d(.)((sin)^-s eta); eth-bar: -(sin)^-s d(.)((sin)^s eta): both are
        # -sin * [d_theta -+ ...](eta / sin) on these spins
        f = lambda t: eth1(t) / math.sin(t)
        df = (f(th + h) - f(th - h)) / (2 * h)
        return -math.sin(th) * (df - sg * m / math.sin(th) * f(th))

    return math.sqrt(math.factorial(l - 2) / math.factorial(l + 2)) * eth2(theta)


@pytest.mark.parametrize("l,m", [(2, 0), (3, 1), (4, 3), (5, 2), (6, 6), (7, 4)])
def test_spin2_is_eth_squared_of_scipy_ylm(l, m):
    for theta in (0.35, 1.1, 2.3):
        z = math.cos(theta)
        p2, m2 = spin_lambdas(l, m, z)
        assert p2[l - m] == pytest.approx(_eth_twice(l, m, theta, False), rel=2e-6, abs=2e-7)
        assert m2[l - m] == pytest.approx(_eth_twice(l, m, theta, True), rel=2e-6, abs=2e-7)


@pytest.mark.parametrize("nside,ring,lmax", [(512, 1, 2048), (512, 700, 1024), (8, 3, 300),
                                             (64, 128, 600)])
def test_spin2_unsold(nside, ring, lmax):
    """sum_m |2Y_lm|^2 = (2l+1)/(4 pi) at every point; with 2lambda_{l,-m} =
    (-1)^m (-2)lambda_lm this is sum_m (2 - delta_m0)(F+^2 + F-^2) = (2l+1)/(4 pi)."""
    z, s, *_ = oracle.rings(nside)
    zr, sr = z[ring - 1], s[ring - 1]
    acc = np.zeros(lmax + 1)
    for m in range(lmax + 1):
        fp, fm = oracle.spin2(lmax, m, zr, sr)
        acc[m:] += (1.0 if m == 0 else 2.0) * (fp * fp + fm * fm)
    ell = np.arange(2, lmax + 1)
    assert np.max(np.abs(acc[2:] / ((2 * ell + 1) / FOURPI) - 1.0)) < 1e-12


@pytest.mark.parametrize("m", [0, 1, 2, 3, 9])
def test_spin2_gauss_legendre_orthonormality(m):
    lmax = 40
    x, w = np.polynomial.legendre.leggauss(2 * lmax + 8)
    for spin in (2, -2):
        V = np.array([spin_lambdas(lmax, m, xi)[0 if spin == 2 else 1] for xi in x])
        l0 = max(2, m) - m
        G = 2 * np.pi * (V[:, l0:].T * w) @ V[:, l0:]
        assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-12


# ----------------------------------------------------------------------------------------
# Polarized transform
# ----------------------------------------------------------------------------------------
def _rand_teb(rng, lmax):
    a = np.stack([W.white_alm(rng, lmax) for _ in range(3)])
    ls, _ = W.alm_l_m(lmax)
    a[1:, ls < 2] = 0.0
    return a


def _dot_alm(lmax, a, b):
    _, ms = W.alm_l_m(lmax)
    wgt = np.where(ms == 0, 1.0, 2.0)
    return float(np.sum(wgt * (np.conj(a) * b).real))


@pytest.mark.parametrize("nside,lmax,direct", [(2, 8, True), (4, 12, False), (4, 9, True),
                                               (8, 20, False)])
def test_pol_analysis_is_adjoint_of_synthesis(nside, lmax, direct):
    rng = np.random.default_rng(nside * 100 + lmax)
    npix = 12 * nside * nside
    omega = FOURPI / npix
    a = _rand_teb(rng, lmax)
    mp = rng.standard_normal((3, npix))
    lhs = float(np.sum(oracle.alm2map_pol(nside, lmax, a, direct) * mp))
    rhs = _dot_alm(lmax, a, oracle.map2alm_pol(nside, lmax, mp, direct)) / omega
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_pol_direct_phi_sums_equal_fft_and_T_is_spin0():
    nside, lmax = 4, 14
    rng = np.random.default_rng(1)
    a = _rand_teb(rng, lmax)
    m1 = oracle.alm2map_pol(nside, lmax, a, direct=True)
    m2 = oracle.alm2map_pol(nside, lmax, a, direct=False)
    assert rel(m2, m1) < 1e-13
    assert np.array_equal(m2[0], oracle.alm2map(nside, lmax, a[0]))
    b1 = oracle.map2alm_pol(nside, lmax, m1, direct=True)
    b2 = oracle.map2alm_pol(nside, lmax, m1, direct=False)
    assert rel(b2, b1) < 1e-13


def test_pure_E_field_has_no_B():
    """A pure-E field analyses to B = 0 up to the quadrature error of the round trip,
    while a sign error between F+ and F- would turn O(1) of E into B."""
    nside, lmax = 16, 16
    rng = np.random.default_rng(5)
    a = _rand_teb(rng, lmax)
    a[0] = 0.0
    a[2] = 0.0
    back = oracle.map2alm_pol(nside, lmax, oracle.alm2map_pol(nside, lmax, a))
    e_err = rel(back[1], a[1])
    assert e_err < 5e-3
    assert np.linalg.norm(back[2]) / np.linalg.norm(a[1]) < 5e-3
    # and the same for pure B
    a2 = np.zeros_like(a)
    a2[2] = a[1]
    back2 = oracle.map2alm_pol(nside, lmax, oracle.alm2map_pol(nside, lmax, a2))
    assert np.linalg.norm(back2[1]) / np.linalg.norm(a2[2]) < 5e-3


@pytest.mark.parametrize("psi", [0.3, 1.0])
def test_rotation_of_polarization_angle(psi):
    """Q + iU -> e^{2 i psi}(Q + iU) maps (E, B) -> (E cos 2psi - B sin 2psi,
    E sin 2psi + B cos 2psi); T untouched."""
    nside, lmax = 4, 10
    rng = np.random.default_rng(7)
    mp = rng.standard_normal((3, 12 * nside * nside))
    c, s = math.cos(2 * psi), math.sin(2 * psi)
    rot = mp.copy()
    rot[1], rot[2] = c * mp[1] - s * mp[2], s * mp[1] + c * mp[2]
    a = oracle.map2alm_pol(nside, lmax, mp)
    b = oracle.map2alm_pol(nside, lmax, rot)
    assert rel(b[0], a[0]) < 1e-15
    assert rel(b[1], c * a[1] - s * a[2]) < 1e-13
    assert rel(b[2], s * a[1] + c * a[2]) < 1e-13


# ----------------------------------------------------------------------------------------
# T, Q, U messenger iteration
# ----------------------------------------------------------------------------------------
def _filter3(cl4, l, mu):
    TT, EE, BB, TE = cl4[:, l]
    S = np.array([[TT, TE, 0.0], [TE, EE, 0.0], [0.0, 0.0, BB]])
    return S @ np.linalg.inv(S + mu * np.eye(3))


@pytest.mark.parametrize("lam", [1.0, 4.0])
def test_pol_uniform_noise_solves_in_one_iteration(lam):
    """N_p = sigma^2 I everywhere: tau M = I, t = d after one update, and the harmonic
    update gives s = S (S + lam sigma^2 Omega I)^{-1} A d; further iterations change
    nothing (the paper's N ~ 1 case, Sect. 2.1)."""
    nside, lmax = 4, 10
    npix = 12 * nside * nside
    omega = FOURPI / npix
    rng = np.random.default_rng(3)
    cl4 = W.pol_cls(W.cl_config1(lmax))
    sig2 = 2.5
    M6 = np.tile([1 / sig2, 0, 0, 1 / sig2, 0, 1 / sig2], (npix, 1))
    d = rng.standard_normal((3, npix))
    s1, _ = oracle.solve_pol(nside, lmax, cl4, M6, d / sig2, lam=[lam])
    a = oracle.map2alm_pol(nside, lmax, d)
    ls, _ = W.alm_l_m(lmax)
    ref = np.zeros_like(a)
    for k, l in enumerate(ls):
        ref[:, k] = _filter3(cl4, l, lam * sig2 * omega) @ a[:, k]
    assert rel(s1, ref) < 1e-13
    s3, _ = oracle.solve_pol(nside, lmax, cl4, M6, d / sig2, lam=[lam] * 3)
    assert rel(s3, ref) < 1e-12


def _small_pol_problem(nside=2, lmax=4, seed=0, nu=30):
    w = W.config3(seed, nside, lmax, ndisc=1, band_z=0.0, nu=nu)
    cl4 = W.pol_cls(W.cl_config1(lmax))
    sig = oracle.alm2map_pol(nside, lmax, w.signal_alm)
    d = w.data_from_signal_maps(sig)
    M6 = w.M6()
    rho = np.einsum("pij,jp->ip", _unpack(M6), d)
    return w, cl4, M6, rho


def _unpack(M6):
    A = np.empty((M6.shape[0], 3, 3))
    A[:, 0, 0], A[:, 0, 1], A[:, 0, 2] = M6[:, 0], M6[:, 1], M6[:, 2]
    A[:, 1, 0], A[:, 1, 1], A[:, 1, 2] = M6[:, 1], M6[:, 3], M6[:, 4]
    A[:, 2, 0], A[:, 2, 1], A[:, 2, 2] = M6[:, 2], M6[:, 4], M6[:, 5]
    return A


def test_pol_iteration_converges_to_dense_fixed_point():
    """At lambda = 1 the iterate's fixed point solves s = D A(tau rho + (I - tau M) Y s)
    (Eqs. 3-4 with 3x3 blocks).  Built as a dense real-linear system over the coefficients
    (the map s -> D A (I - tau M) Y s applied to unit vectors) and solved directly, it must
    equal the iterate run to stall."""
    nside, lmax = 2, 4
    w, cl4, M6, rho = _small_pol_problem(nside, lmax)
    npix = 12 * nside * nside
    omega = FOURPI / npix
    tau = oracle.tau_pol(M6)
    Mb = _unpack(M6)
    ls, _ = W.alm_l_m(lmax)
    F = [_filter3(cl4, l, tau * omega) for l in range(lmax + 1)]

    def D(a):
        out = np.zeros_like(a)
        for k, l in enumerate(ls):
            out[:, k] = F[l] @ a[:, k]
        return out

    def op(s):
        y = oracle.alm2map_pol(nside, lmax, s)
        return D(oracle.map2alm_pol(nside, lmax, y - tau * np.einsum("pij,jp->ip", Mb, y)))

    # real coordinates: (component, index, re/im); imaginary parts of m = 0 stay 0
    n = 3 * len(ls)
    basis = []
    for c in range(3):
        for k in range(len(ls)):
            for part in (1.0, 1j):
                if part == 1j and k <= lmax:  # m = 0 entries are real
                    continue
                e = np.zeros((3, len(ls)), dtype=np.complex128)
                e[c, k] = part
                basis.append(e)
    flat = lambda a: np.concatenate([[a[c, k].real for c in range(3) for k in range(len(ls))],
                                      [a[c, k].imag for c in range(3) for k in range(len(ls)) if k > lmax]])
    cols = np.stack([flat(op(e)) for e in basis], axis=1)
    P = np.stack([flat(e) for e in basis], axis=1)   # coordinates of the basis vectors
    b = flat(D(oracle.map2alm_pol(nside, lmax, tau * rho)))
    x = np.linalg.solve(P - cols, b)
    s_dense = sum(xi * e for xi, e in zip(np.linalg.solve(P, P @ x), basis))
    radius = np.max(np.abs(np.linalg.eigvals(np.linalg.solve(P, cols))))
    assert radius < 0.95
    k = int(math.ceil(math.log(1e-15) / math.log(radius))) + 20
    s_it, _ = oracle.solve_pol(nside, lmax, cl4, M6, rho, niter=k)
    assert rel(s_it, s_dense) < 1e-11


def test_pol_chi2_decreases_at_fixed_lambda_and_masked_data_ignored():
    nside, lmax = 4, 8
    w = W.config3(2, nside, lmax, ndisc=5, band_z=0.2, nu=10)
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    M6 = w.M6()
    rho = np.einsum("pij,jp->ip", _unpack(M6), d)
    _, _, dg = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, niter=30, diag=True)
    assert np.all(np.diff(dg[:, 0]) < 1e-12 * dg[0, 0])
    d2 = d.copy()
    d2[:, w.mask == 0] += 100.0
    rho2 = np.einsum("pij,jp->ip", _unpack(M6), d2)
    a1, m1 = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, niter=5)
    a2, m2 = oracle.solve_pol(nside, lmax, w.cl4, M6, rho2, niter=5)
    assert np.array_equal(a1, a2) and np.array_equal(m1, m2)


def test_pol_chi2_is_the_eq6_quadratic_form_at_the_iterate():
    """chi^2(s, lambda) of Eq. (6) with blocks: s^T S^-1 s over real harmonic dof (l >= 2)
    plus sum_p (d - Ys)^T [N_p + (lambda - 1) tau]^-1 (d - Ys) over observed pixels,
    evaluated here from the returned iterate with the noise covariance N_p itself."""
    nside, lmax, lam = 4, 8, 2.0
    w = W.config3(4, nside, lmax, ndisc=5, band_z=0.2, nu=10)
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    M6 = w.M6()
    rho = np.einsum("pij,jp->ip", _unpack(M6), d)
    s, smap, dg = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=[lam] * 6, diag=True)
    tau = oracle.tau_pol(M6)
    ls, ms = W.alm_l_m(lmax)
    harm = 0.0
    for k, l in enumerate(ls):
        if l < 2:
            continue
        TT, EE, BB, TE = w.cl4[:, l]
        Si = np.linalg.inv(np.array([[TT, TE, 0], [TE, EE, 0], [0, 0, BB]]))
        wgt = 1.0 if ms[k] == 0 else 2.0
        harm += wgt * ((s[:, k].real @ Si @ s[:, k].real) + (s[:, k].imag @ Si @ s[:, k].imag))
    Ncov = np.einsum("pik,pjk->pij", w.noise_chol, w.noise_chol)
    pix = 0.0
    for p in np.nonzero(w.mask)[0]:
        r = d[:, p] - smap[:, p]
        pix += r @ np.linalg.solve(Ncov[p] + (lam - 1.0) * tau * np.eye(3), r)
    assert dg[-1, 1] == pytest.approx(harm, rel=1e-11)
    assert dg[-1, 0] == pytest.approx(harm + pix, rel=1e-10)


def test_pol_fluctuation_source_quadratic_forms():
    """rho = L_p g1 + Omega Y(K h): with h = 0, rho_p^T M_p^{-1} rho_p = |g1_p|^2 (any
    factor L L^T = M); with g1 = 0, the analysis of rho gives x ~ K h with
    x^T S_l x = |h|^2 per (l, m) for any factor K K^T = S^-1 (up to the round trip)."""
    nside, lmax = 8, 8
    w = W.config3(1, nside, lmax, ndisc=3, band_z=0.1, nu=10)
    M6 = w.M6()
    rng = np.random.default_rng(2)
    g1 = rng.standard_normal((3, w.npix))
    h = np.stack([W.white_alm(rng, lmax) for _ in range(3)])
    r1 = oracle.fluct_rho_pol(nside, lmax, w.cl4, M6, g1, np.zeros_like(h))
    Mb = _unpack(M6)
    obs = np.nonzero(w.mask)[0]
    q = np.array([r1[:, p] @ np.linalg.solve(Mb[p], r1[:, p]) for p in obs])
    assert np.max(np.abs(q - np.sum(g1[:, obs] ** 2, axis=0))) < 1e-11 * np.max(q)
    assert np.all(r1[:, w.mask == 0] == 0.0)
    r2 = oracle.fluct_rho_pol(nside, lmax, w.cl4, M6, np.zeros_like(g1), h)
    x = oracle.map2alm_pol(nside, lmax, r2) / (FOURPI / w.npix)
    ls, ms = W.alm_l_m(lmax)
    got, want = 0.0, 0.0
    for k, l in enumerate(ls):
        if l < 2:
            continue
        TT, EE, BB, TE = w.cl4[:, l]
        S = np.array([[TT, TE, 0], [TE, EE, 0], [0, 0, BB]])
        wgt = 1.0 if ms[k] == 0 else 2.0
        got += wgt * (x[:, k].real @ S @ x[:, k].real + x[:, k].imag @ S @ x[:, k].imag)
        want += wgt * np.sum(np.abs(h[:, k]) ** 2)
    assert got == pytest.approx(want, rel=2e-2)


def _pol_rho(M6, d):
    return np.einsum("pij,jp->ip", _unpack(M6), d)


def test_pol_staged_solve_without_truncation_equals_the_iteration():
    """Stages at the full band limit are the plain iteration with that lambda sequence."""
    nside, lmax = 8, 16
    w = W.config3(3, nside, lmax, ndisc=5, band_z=0.15, nu=10)
    M6 = w.M6()
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    rho = _pol_rho(M6, d)
    a1, m1 = oracle.solve_pol_staged(nside, lmax, w.cl4, M6, rho, [(lmax, 4.0, 6), (lmax, 1.0, 9)])
    b1, n1 = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=[4.0] * 6 + [1.0] * 9)
    assert rel(a1, b1) < 1e-12 and rel(m1, n1) < 1e-12


def test_pol_staged_truncated_stage_is_the_band_limited_problem():
    """One stage at lmax_k < lmax is the iteration of the problem with band limit lmax_k
    (spectra cut there); the coefficients above lmax_k are zero."""
    nside, lmax, lk = 8, 20, 9
    w = W.config3(5, nside, lmax, ndisc=5, band_z=0.15, nu=10)
    M6 = w.M6()
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    rho = _pol_rho(M6, d)
    a, m = oracle.solve_pol_staged(nside, lmax, w.cl4, M6, rho, [(lk, 3.0, 8)])
    b, n = oracle.solve_pol(nside, lk, w.cl4[:, :lk + 1], M6, rho, lam=[3.0] * 8)
    ls, ms = W.alm_l_m(lmax)
    low = (ls <= lk) & (ms <= lk)
    assert np.all(a[:, ~low] == 0)
    assert rel(a[:, low], b) < 1e-12 and rel(m, n) < 1e-12


def test_pol_staged_reduces_to_temperature_staging():
    """With no polarized signal (EE = BB = TE = 0) and no T-P noise correlation, T decouples:
    its stages are the temperature staged solve (itself pinned to dense harmonics) with the
    same tau, Q and U stay zero."""
    nside, lmax = 8, 24
    w = W.config3(6, nside, lmax, ndisc=5, band_z=0.15, nu=10)
    M6 = w.M6()
    MT = M6[:, 0]
    M6d = np.zeros_like(M6)
    M6d[:, 0] = MT
    M6d[:, 3] = M6d[:, 5] = 0.5 * MT   # Q, U noise weaker than T: tau is set by T alone
    cl4 = w.cl4.copy()
    cl4[1:] = 0.0
    rng = np.random.default_rng(4)
    rho = rng.standard_normal((3, w.npix)) * (MT > 0)
    stages = [(10, 6.0, 5), (18, 2.0, 4), (24, 1.0, 6)]
    a, m = oracle.solve_pol_staged(nside, lmax, cl4, M6d, rho, stages)
    at, mt = oracle.solve_staged(nside, lmax, cl4[0], MT, rho[0], stages)
    assert rel(a[0], at) < 1e-12 and rel(m[0], mt) < 1e-12
    assert np.all(a[1:] == 0) and np.abs(m[1:]).max() == 0.0


def test_pol_plain_iteration_unstable_at_lmax_2nside_nside32():
    """A property of the discretised method, not of an implementation: on the nside 32 grid
    with lmax = 64 the T, Q, U iteration at lambda = 1 first lowers chi^2, then grows without
    bound (an eigenvalue of the iteration above 1, from the pixelisation's quadrature), and so
    does the temperature iteration alone with this problem's T noise and mask; T, Q, U on
    nside 16 / lmax 32 and the temperature workloads stay stable.  The cooled solve reports
    such a run instead of iterating on."""
    nside, lmax, n = 32, 64, 600
    w = W.config3(0, nside, lmax, ndisc=10, band_z=0.15, nu=10)
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    M6 = w.M6()
    rho = np.einsum("pij,jp->ip", _unpack(M6), d)
    _, _, dg = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=[1.0] * n, diag=True)
    chi = dg[:, 0]
    sigma = math.sqrt(2.0 * 3 * int(w.mask.sum()))
    k = int(np.argmin(chi))
    assert 100 < k < 400
    assert chi[-1] > chi[k] + 10.0 * sigma
    assert np.all(np.diff(chi[k + 50:]) > 0.0)
    # by growing steps (an eigenvalue above 1), unlike a run settling above a minimum it
    # passed through, whose rises shrink
    assert chi[-1] - chi[-51] > 2.0 * (chi[k + 150] - chi[k + 100]) > 0.0
    # not a spin-2 effect: the temperature iteration on the T noise and mask alone
    MT = M6[:, 0]
    _, _, dgt = oracle.solve(nside, lmax, w.cl4[0], MT, MT * d[0], lam=[1.0] * n, diag=True)
    ct = dgt[:, 0]
    kt = int(np.argmin(ct))
    assert 100 < kt < 400 and ct[-1] > ct[kt] + 10.0 * math.sqrt(2.0 * int(w.mask.sum()))


# ----------------------------------------------------------------------------------------
# The polarized transform against its definition, and the sampled forms against the full
# ones; the T, Q, U iteration at lambda > 1 with correlated noise blocks.
# ----------------------------------------------------------------------------------------
from oracle import dense  # noqa: E402


@pytest.mark.parametrize("nside,lmax", [(2, 8), (4, 9), (4, 16)])
def test_pol_synthesis_equals_the_definition(nside, lmax):
    """The oracle's (T, Q, U) synthesis (ring pairs, FFT, alias folds up to lmax = 4 nside,
    half-pixel phases) equals the term-by-term sum of Q + iU = sum 2a_lm 2Y_lm over m = -l..l
    with the E/B reality conditions (oracle.dense.pol_synthesis_direct); the analysis equals
    Omega times the transpose of that sum."""
    rng = np.random.default_rng(nside * 31 + lmax)
    a = _rand_teb(rng, lmax)
    ref = dense.pol_synthesis_direct(nside, lmax, a)
    got = oracle.alm2map_pol(nside, lmax, a)
    for c in range(3):
        assert rel(got[c], ref[c]) < 1e-13, c
    Y = dense.pol_synthesis_matrix(nside, lmax)
    npix = 12 * nside * nside
    mp = rng.standard_normal((3, npix))
    ana = (FOURPI / npix) * (Y.T @ mp.ravel())
    n = (lmax + 1) ** 2
    back = oracle.map2alm_pol(nside, lmax, mp)
    for c in range(3):
        assert rel(dense.alm_to_real(back[c], lmax), ana[c * n:(c + 1) * n]) < 1e-13, c


@pytest.mark.parametrize("nside,lmax", [(4, 8), (4, 16), (8, 20), (8, 32)])
def test_pol_sampled_ring_and_m_equal_the_full_transforms(nside, lmax):
    """T, Q, U of one ring and T, E, B of one m (the forms the large-size GPU checks use)
    equal the rows and columns of the full polarized synthesis and analysis on every ring
    and every m, lmax up to 4 nside (all alias folds)."""
    rng = np.random.default_rng(nside + 7 * lmax)
    a = _rand_teb(rng, lmax)
    full = oracle.alm2map_pol(nside, lmax, a)
    z, s, start, nphi, phi0 = oracle.rings(nside)
    scale = np.linalg.norm(full)
    for r in range(1, 4 * nside):
        got = oracle.alm2map_pol_ring(nside, lmax, a, r)
        sl = slice(int(start[r - 1]), int(start[r - 1] + nphi[r - 1]))
        assert np.abs(got - full[:, sl]).max() < 1e-13 * scale, r
    mp = rng.standard_normal((3, 12 * nside * nside))
    ana = oracle.map2alm_pol(nside, lmax, mp)
    _, ms = W.alm_l_m(lmax)
    ascale = np.abs(ana).max()
    for m in range(lmax + 1):
        got = oracle.map2alm_pol_m(nside, lmax, mp, m)
        assert np.abs(got - ana[:, ms == m]).max() < 1e-13 * ascale, m


def _pol_dense_problem(nside, lmax, seed, nu=4):
    """A T, Q, U problem with correlated 3x3 noise blocks (Wishart with nu degrees of
    freedom), the definition-based synthesis matrix Y [3 npix, 3 (lmax+1)^2], the noise
    precision blocks Mb [npix][3][3] and the real-basis signal blocks S."""
    w = W.config3(seed, nside, lmax, ndisc=3, band_z=0.1, nu=nu)
    d = w.data_from_signal_maps(dense.pol_synthesis_direct(nside, lmax, w.signal_alm))
    M6 = w.M6()
    n = (lmax + 1) ** 2
    Y = dense.pol_synthesis_matrix(nside, lmax)
    Mb = _unpack(M6)
    ell = dense.real_ell(lmax)
    S = np.zeros((3 * n, 3 * n))
    TT, EE, BB, TE = (w.cl4[c][ell] for c in range(4))
    k = np.arange(n)
    S[k, k], S[n + k, n + k], S[2 * n + k, 2 * n + k] = TT, EE, BB
    S[k, n + k] = S[n + k, k] = TE
    keep = np.diag(S) > 0.0
    return w, d, M6, Y, Mb, S, keep


def _blocks(Mb, V):
    """Per-pixel 3x3 blocks applied to pixel vectors: V [3 npix, ...] (component-major)."""
    npix = Mb.shape[0]
    Vr = V.reshape((3, npix) + V.shape[1:])
    return np.einsum("pij,jp...->ip...", Mb, Vr).reshape(V.shape)


def _pol_fixed_point(Y, Mb, S, keep, rho, lam, tau, omega):
    """The s that one T, Q, U iteration at constant lambda maps to itself:
    s = D Omega Y^T B^-1 [lam tau rho + (1 - tau M) Y s], B = 1 + (lam - 1) tau M per pixel
    block (inverted by numpy), D = S (S + lam tau Omega)^-1, on the coefficients with power."""
    eye = np.eye(3)
    Bi = np.linalg.inv(eye + (lam - 1.0) * tau * Mb)
    Yk = Y[:, keep]
    Sk = S[np.ix_(keep, keep)]
    D = Sk @ np.linalg.inv(Sk + lam * tau * omega * np.eye(Sk.shape[0]))
    G = D @ (omega * Yk.T @ _blocks(Bi @ (eye - tau * Mb), Yk))
    b = D @ (omega * Yk.T @ _blocks(Bi, lam * tau * rho))
    return np.linalg.solve(np.eye(G.shape[0]) - G, b), G


def _real3(a, lmax):
    return np.concatenate([dense.alm_to_real(a[c], lmax) for c in range(3)])


@pytest.mark.parametrize("lam", [3.0, 10.0])
def test_pol_fixed_point_at_lambda_above_one_with_correlated_blocks(lam):
    """The oracle's T, Q, U iteration at constant lambda > 1 converges to the dense fixed
    point of Eqs. (3)-(4) with full 3x3 blocks: B^-1 = [1 + (lam - 1) tau M_p]^-1 per pixel
    by numpy, the (T, E, B) signal blocks per l, the definition-based synthesis.  A
    transposed block, a wrong B^-1 or a lambda on the wrong term moves the fixed point."""
    nside, lmax = 4, 4
    w, d, M6, Y, Mb, S, keep = _pol_dense_problem(nside, lmax, seed=11)
    npix = 12 * nside * nside
    omega, tau = FOURPI / npix, oracle.tau_pol(M6)
    Mo = M6[w.mask > 0]
    corr = np.abs(Mo[:, [1, 2, 4]]) / np.sqrt(Mo[:, [0, 0, 3]] * Mo[:, [3, 5, 5]])
    assert np.median(corr) > 0.2  # strongly correlated blocks
    rho = _blocks(Mb, d.ravel()).reshape(3, npix)
    x, G = _pol_fixed_point(Y, Mb, S, keep, rho.ravel(), lam, tau, omega)
    radius = np.max(np.abs(np.linalg.eigvals(G)))
    assert radius < 0.999
    k = int(math.ceil(math.log(1e-14) / math.log(radius))) + 20
    s, _ = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=[lam] * k)
    got = _real3(s, lmax)
    assert np.all(got[~keep] == 0.0)
    assert rel(got[keep], x) < 1e-10


@pytest.mark.parametrize("lam", [3.0, 10.0])
def test_pol_chi2_decreases_at_fixed_lambda_above_one(lam):
    """At fixed lambda the iteration lowers chi^2(x, lambda) of Eq. (6) (Sect. 2.2), here with
    lambda > 1 and strongly correlated noise blocks; nside 8 / lmax 8 keeps the quadrature
    gap of the pixelisation far below the decrease."""
    nside, lmax = 8, 8
    w = W.config3(12, nside, lmax, ndisc=5, band_z=0.2, nu=4)
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    M6 = w.M6()
    rho = np.einsum("pij,jp->ip", _unpack(M6), d)
    _, _, dg = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=[lam] * 40, diag=True)
    assert np.all(np.diff(dg[:, 0]) < 0.0), np.diff(dg[:, 0]).max()
    assert dg[-1, 0] < 0.5 * dg[0, 0]


def test_pol_s_lambda_closed_form_within_the_quadrature_bound():
    """Sect. 2.2: at constant lambda the iteration converges to s(lambda) =
    S (S + N + (lambda - 1) T)^-1 d, the minimiser of chi^2(x, lambda): in harmonic form
    (S^-1 + Y^T M_lam Y) x = Y^T M_lam d, M_lam = M [1 + (lam - 1) tau M]^-1 per block.  The
    messenger fixed point solves the same system with E = (1 - Omega Y^T Y)/(lam tau Omega)
    added to the matrix, so their distance is at most |(A + E)^-1| |E| (an exact perturbation
    bound, A the closed form's matrix), which the check takes as its tolerance; E vanishes
    where the pixel sum is an exact quadrature, and the distance shrinks with it (nside 8 ->
    16 at lmax 4)."""
    lmax = 4
    gaps = {}
    for nside in (8, 16):
        w, d, M6, Y, Mb, S, keep = _pol_dense_problem(nside, lmax, seed=13, nu=10)
        npix = 12 * nside * nside
        omega, tau = FOURPI / npix, oracle.tau_pol(M6)
        Yk = Y[:, keep]
        Sk = S[np.ix_(keep, keep)]
        Gk = omega * Yk.T @ Yk
        for lam in (3.0, 10.0):
            Ml = Mb @ np.linalg.inv(np.eye(3) + (lam - 1.0) * tau * Mb)
            A = np.linalg.inv(Sk) + Yk.T @ _blocks(Ml, Yk)
            x_closed = np.linalg.solve(A, Yk.T @ _blocks(Ml, d.ravel()))
            x_fp, _ = _pol_fixed_point(Y, Mb, S, keep, _blocks(Mb, d.ravel()), lam, tau, omega)
            E = (np.eye(Gk.shape[0]) - Gk) / (lam * tau * omega)
            bound = np.linalg.norm(np.linalg.inv(A + E), 2) * np.linalg.norm(E, 2)
            gaps[nside, lam] = rel(x_fp, x_closed)
            print("nside", nside, "lambda", lam, "gap", gaps[nside, lam], "bound", bound)
            assert gaps[nside, lam] <= bound
            if nside == 16:
                assert bound < 0.2
    for lam in (3.0, 10.0):
        assert gaps[16, lam] < 0.25 * gaps[8, lam]
