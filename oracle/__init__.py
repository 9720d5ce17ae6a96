"""Plain FP64 CPU oracle for the messenger-field Wiener filter (temperature and T, Q, U).

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the HIP library: the
C file ``mfwf_oracle.c`` re-derives geometry, Legendre and spin-2 functions, phi transforms,
the spin-0 and polarized SHT, the messenger iteration (temperature and T, Q, U with 3x3
noise blocks), chi^2 and the fluctuation sources from the paper and textbook definitions, and
``dense.py`` builds explicit matrices at tiny sizes from SciPy's spherical harmonics.

Array conventions: maps are HEALPix RING order float64; alm are complex128, m-major
packing (m, l = m..lmax).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mfwf_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-ffp-contract=off",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.or_npix.restype = ctypes.c_long
        L.or_nalm.restype = ctypes.c_long
        L.or_tau.restype = ctypes.c_double
        L.or_ring.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.POINTER(ctypes.c_long),
                              ctypes.POINTER(ctypes.c_int), _dp]
        L.or_legendre.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
        L.or_dft.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.or_fft.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.or_alm2map.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int]
        L.or_map2alm.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int]
        L.or_tau.argtypes = [ctypes.c_long, _dp]
        L.or_solve.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp,
                               ctypes.c_int, _dp, _dp, _dp]
        L.or_fluct_rho.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                   ctypes.c_int]
        L.or_spin2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp,
                               _dp]
        L.or_alm2map_pol.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int]
        L.or_map2alm_pol.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int]
        L.or_solve_pol.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                                   ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, _dp]
        L.or_fluct_rho_pol.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                       ctypes.c_int]
        L.or_alm2map_pol_ring.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp]
        L.or_map2alm_pol_m.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp]
        L.or_alm2map_ring.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp]
        L.or_map2alm_m.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp]
        _lib_handle = L
    return _lib_handle


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def num_threads() -> int:
    return lib().or_num_threads()


def nalm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def ring(nside: int, i: int):
    """(z, sin theta, start pixel, n_phi, phi_0) of ring i = 1..4 nside - 1."""
    z, s, p0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st, n = ctypes.c_long(), ctypes.c_int()
    lib().or_ring(nside, i, ctypes.byref(z), ctypes.byref(s), ctypes.byref(st), ctypes.byref(n),
                  ctypes.byref(p0))
    return z.value, s.value, st.value, n.value, p0.value


def rings(nside: int):
    """Arrays over all rings: z, sin theta, start, n_phi, phi_0."""
    out = [ring(nside, i) for i in range(1, 4 * nside)]
    return tuple(np.array(c) for c in zip(*out))


def pixel_angles(nside: int):
    """(theta, phi) of every RING-ordered pixel centre, from the oracle geometry."""
    z, s, start, nphi, phi0 = rings(nside)
    th, ph = [], []
    for k in range(len(z)):
        j = np.arange(nphi[k])
        th.append(np.full(nphi[k], np.arctan2(s[k], z[k])))
        ph.append(phi0[k] + 2.0 * np.pi * j / nphi[k])
    return np.concatenate(th), np.concatenate(ph)


def legendre(lmax: int, m: int, z: float, sth: float | None = None) -> np.ndarray:
    """lambda_lm(z) for l = m..lmax (orthonormal, Condon-Shortley phase)."""
    if sth is None:
        sth = float(np.sqrt((1.0 - z) * (1.0 + z)))
    out = np.zeros(lmax - m + 1)
    lib().or_legendre(lmax, m, float(z), float(sth), _p(out))
    return out


def dft(x, sign=-1):
    x = _c128(x)
    out = np.zeros_like(x)
    lib().or_dft(len(x), sign, _p(x.view(np.float64)), _p(out.view(np.float64)))
    return out


def fft(x, sign=-1):
    x = _c128(x)
    out = np.zeros_like(x)
    lib().or_fft(len(x), sign, _p(x.view(np.float64)), _p(out.view(np.float64)))
    return out


def alm2map(nside, lmax, alm, direct=False):
    alm = _c128(alm)
    assert alm.shape == (nalm(lmax),)
    out = np.zeros(12 * nside * nside)
    lib().or_alm2map(nside, lmax, _p(alm.view(np.float64)), _p(out), int(direct))
    return out


def map2alm(nside, lmax, m, direct=False):
    m = _f64(m)
    assert m.shape == (12 * nside * nside,)
    out = np.zeros(nalm(lmax), dtype=np.complex128)
    lib().or_map2alm(nside, lmax, _p(m), _p(out.view(np.float64)), int(direct))
    return out


def tau(M):
    M = _f64(M)
    return lib().or_tau(len(M), _p(M))


def solve(nside, lmax, cl, M, rho, niter=None, lam=None, direct=False, diag=False):
    """Run the messenger iteration; returns (s_alm, s_map[, diag[niter, 4]]).

    lam: per-iteration lambda schedule (default lambda = 1 for niter iterations).
    diag columns: chi^2(s_k, lambda_k), its harmonic part, |s_k - s_{k-1}|, |s_k|.
    """
    if lam is None:
        lam = np.ones(niter)
    lam = _f64(lam)
    niter = len(lam)
    cl, M, rho = _f64(cl), _f64(M), _f64(rho)
    npix = 12 * nside * nside
    assert cl.shape == (lmax + 1,) and M.shape == (npix,) and rho.shape == (npix,)
    s_alm = np.zeros(nalm(lmax), dtype=np.complex128)
    s_map = np.zeros(npix)
    dg = np.zeros((niter, 4)) if diag else None
    rc = lib().or_solve(nside, lmax, _p(cl), _p(M), _p(rho), niter, _p(lam), int(direct),
                        _p(s_alm.view(np.float64)), _p(s_map), _p(dg) if diag else None)
    if rc != 0:
        raise ValueError("oracle solve failed with status %d (no observed pixel)" % rc)
    return (s_alm, s_map, dg) if diag else (s_alm, s_map)


def template_matrix(nside, observed):
    """V of Eq. (12): the monopole and the three dipole templates (1, x, y, z of each pixel
    centre's unit vector) on the observed pixels, zero elsewhere; [4][npix]."""
    z, s, start, nphi, phi0 = rings(nside)
    npix = 12 * nside * nside
    V = np.zeros((4, npix))
    for k in range(len(z)):
        phi = phi0[k] + 2.0 * np.pi * np.arange(nphi[k]) / nphi[k]
        sl = slice(int(start[k]), int(start[k]) + int(nphi[k]))
        V[0, sl] = 1.0
        V[1, sl] = s[k] * np.cos(phi)
        V[2, sl] = s[k] * np.sin(phi)
        V[3, sl] = z[k]
    return V * (np.asarray(observed) != 0)[None, :]


def remove_templates(nside, observed, d):
    """Eq. (12): d = lim_{sigma -> inf} (1 + sigma V V^T)^{-1} d_raw, V = template_matrix.
    By the Woodbury identity, (1 + sigma V V^T)^{-1} = 1 - V (1/sigma + V^T V)^{-1} V^T, whose
    limit is the projection d_raw - V (V^T V)^{-1} V^T d_raw."""
    V = template_matrix(nside, observed)
    d = _f64(d)
    return d - V.T @ np.linalg.solve(V @ V.T, V @ d)


def _l_of_index(lmax):
    """l of each coefficient in the m-major packing (m, l = m..lmax)."""
    return np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])


def solve_staged(nside, lmax, cl, M, rho, stages):
    """The messenger iteration run in stages with truncated transforms (the cooling schedule
    of Sect. 3): stage (lmax_k, lambda_k, n_k) runs n_k iterations of Eqs. (3)-(4) at
    lambda_k, with analysis and synthesis up to lmax_k <= lmax; the iterate passes from one
    stage to the next as its pixel map.  tau = 1 / max M.  Returns (s_alm, s_map), s_alm in
    the lmax packing with zeros above the last stage's lmax_k."""
    cl, M, rho = _f64(cl), _f64(M), _f64(rho)
    npix = 12 * nside * nside
    tau = 1.0 / M.max()
    omega = 4.0 * np.pi / npix
    s_map = np.zeros(npix)
    s_alm, lk = np.zeros(0, dtype=np.complex128), 0
    for lk, lam, n in stages:
        lk, n = int(lk), int(n)
        C = cl[_l_of_index(lk)]
        f = np.where(C > 0.0, C / np.where(C > 0.0, C + lam * tau * omega, 1.0), 0.0)
        for _ in range(n):
            t = (lam * tau * rho + (1.0 - tau * M) * s_map) / (1.0 + (lam - 1.0) * tau * M)
            s_alm = f * map2alm(nside, lk, t)
            s_map = alm2map(nside, lk, s_alm)
    out = np.zeros(nalm(lmax), dtype=np.complex128)
    if s_alm.size:
        ls_full = _l_of_index(lmax)
        ms_full = np.concatenate([np.full(lmax + 1 - m, m) for m in range(lmax + 1)])
        keep = (ls_full <= lk) & (ms_full <= lk)
        out[keep] = s_alm
    return out, s_map


def fluct_rho(nside, lmax, cl, M, g1, h, direct=False):
    """Constrained-realisation source rho = M^{1/2} g1 + Omega Y(C^{-1/2} h) (Eq. 9)."""
    cl, M, g1, h = _f64(cl), _f64(M), _f64(g1), _c128(h)
    out = np.zeros(12 * nside * nside)
    lib().or_fluct_rho(nside, lmax, _p(cl), _p(M), _p(g1), _p(h.view(np.float64)), _p(out),
                       int(direct))
    return out


# ---- polarization (T, Q, U maps [3][npix]; T, E, B alm [3][nalm]) -------------------------

def spin2(lmax, m, z, sth=None):
    """(F+, F-) for l = m..lmax at z: F+- = (2lambda_lm +- (-2)lambda_lm) / 2."""
    if sth is None:
        sth = np.sqrt((1.0 - z) * (1.0 + z))
    fp, fm = np.zeros(lmax - m + 1), np.zeros(lmax - m + 1)
    lib().or_spin2(lmax, m, float(z), float(sth), _p(fp), _p(fm))
    return fp, fm


def alm2map_pol(nside, lmax, alm, direct=False):
    """(T, E, B) alm [3][nalm] -> (T, Q, U) maps [3][npix]."""
    alm = _c128(alm)
    assert alm.shape == (3, nalm(lmax))
    out = np.zeros((3, 12 * nside * nside))
    lib().or_alm2map_pol(nside, lmax, _p(alm.view(np.float64)), _p(out), int(direct))
    return out


def map2alm_pol(nside, lmax, maps, direct=False):
    """(T, Q, U) maps -> (T, E, B) alm with the analysis Omega Y^T."""
    maps = _f64(maps)
    assert maps.shape == (3, 12 * nside * nside)
    out = np.zeros((3, nalm(lmax)), dtype=np.complex128)
    lib().or_map2alm_pol(nside, lmax, _p(maps), _p(out.view(np.float64)), int(direct))
    return out


def tau_pol(M6):
    """tau = 1 / max_p lambda_max(M_p) over the packed 3x3 blocks [npix][6] (0 if none)."""
    M6 = _f64(M6)
    A = np.empty((M6.shape[0], 3, 3))
    A[:, 0, 0], A[:, 0, 1], A[:, 0, 2] = M6[:, 0], M6[:, 1], M6[:, 2]
    A[:, 1, 0], A[:, 1, 1], A[:, 1, 2] = M6[:, 1], M6[:, 3], M6[:, 4]
    A[:, 2, 0], A[:, 2, 1], A[:, 2, 2] = M6[:, 2], M6[:, 4], M6[:, 5]
    mx = np.linalg.eigvalsh(A)[:, -1].max()
    return 1.0 / mx if mx > 0 else 0.0


def solve_pol(nside, lmax, cl4, M6, rho, niter=None, lam=None, direct=False, diag=False):
    """Messenger iteration with T, Q, U.  cl4 [4][lmax+1] = TT, EE, BB, TE; M6 [npix][6]
    packed inverse noise blocks; rho [3][npix].  Returns (s_alm [3][nalm], s_map [3][npix]
    [, diag[niter, 4]])."""
    if lam is None:
        lam = np.ones(niter)
    lam = _f64(lam)
    niter = len(lam)
    cl4, M6, rho = _f64(cl4), _f64(M6), _f64(rho)
    npix = 12 * nside * nside
    assert cl4.shape == (4, lmax + 1) and M6.shape == (npix, 6) and rho.shape == (3, npix)
    tau = tau_pol(M6)
    s_alm = np.zeros((3, nalm(lmax)), dtype=np.complex128)
    s_map = np.zeros((3, npix))
    dg = np.zeros((niter, 4)) if diag else None
    rc = lib().or_solve_pol(nside, lmax, _p(cl4), _p(M6), _p(rho), tau, niter, _p(lam),
                            int(direct), _p(s_alm.view(np.float64)), _p(s_map),
                            _p(dg) if diag else None)
    if rc != 0:
        raise ValueError("oracle polarized solve failed with status %d" % rc)
    return (s_alm, s_map, dg) if diag else (s_alm, s_map)


def solve_pol_staged(nside, lmax, cl4, M6, rho, stages):
    """The T, Q, U messenger iteration in stages with truncated transforms (the cooling
    schedule of Sect. 3 with the T+P blocks): stage (lmax_k, lambda_k, n_k) runs n_k
    iterations of Eq. (3) with the 3x3 noise blocks and Eq. (4) with the 3x3 (T, E, B) signal
    blocks S_l = [[TT, TE, 0], [TE, EE, 0], [0, 0, BB]], s = S_l (S_l + lambda tau Omega)^-1 a,
    transforms up to lmax_k; the iterate passes between stages as its pixel maps.
    tau = 1 / max_p lambda_max(M_p).  Returns (s_alm [3][nalm(lmax)] with zeros above the last
    stage's lmax_k, s_map [3][npix])."""
    cl4, M6, rho = _f64(cl4), _f64(M6), _f64(rho)
    npix = 12 * nside * nside
    assert cl4.shape == (4, lmax + 1) and M6.shape == (npix, 6) and rho.shape == (3, npix)
    tau = tau_pol(M6)
    omega = 4.0 * np.pi / npix
    Mb = M6[:, [0, 1, 2, 1, 3, 4, 2, 4, 5]].reshape(npix, 3, 3)  # packed TT TQ TU QQ QU UU
    eye = np.eye(3)
    s_map = np.zeros((3, npix))
    s_alm, lk = np.zeros((3, 0), dtype=np.complex128), 0
    for lk, lam, n in stages:
        lk, n = int(lk), int(n)
        TT, EE, BB, TE = (cl4[c, :lk + 1] for c in range(4))
        S = np.zeros((lk + 1, 3, 3))
        S[:, 0, 0], S[:, 0, 1], S[:, 1, 0], S[:, 1, 1], S[:, 2, 2] = TT, TE, TE, EE, BB
        F = S @ np.linalg.inv(S + lam * tau * omega * eye)  # S (S + mu)^-1 per l
        Fi = F[_l_of_index(lk)]                               # per coefficient
        A = eye + (lam - 1.0) * tau * Mb                      # [npix][3][3]
        for _ in range(n):
            b = lam * tau * rho.T + s_map.T - tau * np.einsum("pij,pj->pi", Mb, s_map.T)
            t = np.linalg.solve(A, b[..., None])[..., 0].T
            a = map2alm_pol(nside, lk, t)
            s_alm = np.einsum("kij,jk->ik", Fi, a)
            s_map = alm2map_pol(nside, lk, s_alm)
    out = np.zeros((3, nalm(lmax)), dtype=np.complex128)
    if s_alm.shape[1]:
        ls_full = _l_of_index(lmax)
        ms_full = np.concatenate([np.full(lmax + 1 - m, m) for m in range(lmax + 1)])
        keep = (ls_full <= lk) & (ms_full <= lk)
        out[:, keep] = s_alm
    return out, s_map


def fluct_rho_pol(nside, lmax, cl4, M6, g1, h, direct=False):
    """rho = L_p g1 + Omega Y_pol(K_l h) with M_p = L_p L_p^T and K_l K_l^T = S_l^{-1}."""
    cl4, M6, g1, h = _f64(cl4), _f64(M6), _f64(g1), _c128(h)
    out = np.zeros((3, 12 * nside * nside))
    lib().or_fluct_rho_pol(nside, lmax, _p(cl4), _p(M6), _p(g1), _p(h.view(np.float64)),
                           _p(out), int(direct))
    return out


def alm2map_pol_ring(nside, lmax, alm, ring):
    """T, Q, U of one ring (1-based ring index) of the polarized synthesis: [3][n_phi]."""
    alm = _c128(alm)
    z, s, start, nphi, phi0 = rings(nside)
    out = np.zeros((3, int(nphi[ring - 1])))
    lib().or_alm2map_pol_ring(nside, lmax, _p(alm.view(np.float64)), ring, _p(out))
    return out


def map2alm_pol_m(nside, lmax, maps, m):
    """aT, aE, aB for one m, l = m..lmax, of the polarized analysis: [3][lmax - m + 1]."""
    maps = _f64(maps)
    out = np.zeros((3, lmax - m + 1), dtype=np.complex128)
    lib().or_map2alm_pol_m(nside, lmax, _p(maps), m, _p(out.view(np.float64)))
    return out


def alm2map_ring(nside, lmax, alm, ring):
    """The temperature map on one ring (1-based ring index) of the synthesis: [n_phi]."""
    alm = _c128(alm)
    z, s, start, nphi, phi0 = rings(nside)
    out = np.zeros(int(nphi[ring - 1]))
    lib().or_alm2map_ring(nside, lmax, _p(alm.view(np.float64)), ring, _p(out))
    return out


def map2alm_m(nside, lmax, m_map, m):
    """a_lm for one m, l = m..lmax, of the temperature analysis (Omega included)."""
    m_map = _f64(m_map)
    out = np.zeros(lmax - m + 1, dtype=np.complex128)
    lib().or_map2alm_m(nside, lmax, _p(m_map), m, _p(out.view(np.float64)))
    return out
