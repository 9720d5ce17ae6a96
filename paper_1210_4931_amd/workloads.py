"""Seeded synthetic workloads for the messenger-field Wiener filter.

This module only draws random numbers and lays out input arrays (power spectra, noise
variance maps, masks, white-noise draws).  It performs none of the solver's arithmetic:
no spherical-harmonic transform, no messenger update, no filter.  The product path, the
tests and the CPU oracle all take their inputs from here, so both sides of every parity
check see byte-identical inputs.

The paper analyses WMAP7 V-band maps (Sect. 3: nside 512, lmax 1024, masks keeping about
70-73 % of the sky, inhomogeneous pixel noise, Eq. 10/11 covariance blocks) and times a
Planck-like temperature map (Sect. 4).  Neither dataset is available, so these seeded
stand-ins reproduce the shapes: HEALPix nside/lmax, a falling CMB-like C_l, a Galactic-cut
band plus point-source discs, and a scan-pattern hit map.

Draw order inside one workload is fixed: signal (unit-white harmonic draw), pixel noise,
mask disc centres, hit-map jitter.  RNG: numpy PCG64 seeded with the workload seed.

Alm layout everywhere: complex, m-major, (m, l = m..lmax), index m*(2*lmax+3-m)//2 + l-m.
Maps are HEALPix RING order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def nalm(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def alm_l_m(lmax: int):
    """Arrays (l, m) for every packed alm index."""
    ls, ms = [], []
    for m in range(lmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


def pixel_centres(nside: int):
    """(z, phi) of every RING-ordered pixel centre.

    Written independently of the solver's geometry tables; used here only to place mask
    discs and the hit pattern on the sphere.
    """
    ns = nside
    zs, phis = [], []
    for i in range(1, 4 * ns):
        if i < ns:
            npr, z, shift = 4 * i, 1.0 - i * i / (3.0 * ns * ns), 0.5
        elif i <= 3 * ns:
            npr, z = 4 * ns, 4.0 / 3.0 - 2.0 * i / (3.0 * ns)
            shift = 0.5 if (i - ns) % 2 == 0 else 0.0
        else:
            k = 4 * ns - i
            npr, z, shift = 4 * k, -(1.0 - k * k / (3.0 * ns * ns)), 0.5
        j = np.arange(npr)
        zs.append(np.full(npr, z))
        phis.append((j + shift) * (2.0 * np.pi / npr))
    return np.concatenate(zs), np.concatenate(phis)


def white_alm(rng: np.random.Generator, lmax: int) -> np.ndarray:
    """Unit-white draw in the real harmonic basis, in the complex m>=0 packing.

    m = 0 entries are real N(0,1); m > 0 entries are (x + i y)/sqrt(2) with x, y ~ N(0,1),
    so every real degree of freedom has unit variance.
    """
    z = rng.standard_normal((nalm(lmax), 2))
    h = (z[:, 0] + 1j * z[:, 1]) / math.sqrt(2.0)
    h[: lmax + 1] = z[: lmax + 1, 0]
    return h


def disc_mask(z, phi, centres, radius_rad, band_z):
    """1 = observed, 0 = masked.  A pixel is masked if |z| < band_z or its centre lies
    within radius_rad of any disc centre."""
    st = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    xyz = np.stack([st * np.cos(phi), st * np.sin(phi), z], axis=1)
    masked = np.abs(z) < band_z
    cosr = math.cos(radius_rad)
    for c in centres:
        masked |= (xyz @ c) > cosr
    return (~masked).astype(np.uint8)


def _unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@dataclasses.dataclass
class TemperatureWorkload:
    """Inputs of one temperature Wiener-filter problem."""
    name: str
    nside: int
    lmax: int
    cl: np.ndarray            # [lmax+1] signal power spectrum, C_0 = C_1 = 0
    signal_alm: np.ndarray    # [nalm] complex: sqrt(C_l) * unit-white draw
    noise_white: np.ndarray   # [npix] unit normals (pixel noise = sqrt(var) * noise_white)
    noise_var: np.ndarray     # [npix] per-pixel noise variance
    mask: np.ndarray          # [npix] uint8, 1 = observed

    @property
    def npix(self):
        return 12 * self.nside * self.nside

    @property
    def ninv(self):
        return 1.0 / self.noise_var

    def data_from_signal_map(self, signal_map: np.ndarray) -> np.ndarray:
        """d = s + n (Eq. 1), given the synthesised signal map."""
        return signal_map + np.sqrt(self.noise_var) * self.noise_white


def cl_config1(lmax):
    ell = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    cl[2:] = 1000.0 / (ell[2:] * (ell[2:] + 1.0))
    return cl


def cl_damped(lmax, lscale):
    ell = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    cl[2:] = 6000.0 / (ell[2:] * (ell[2:] + 1.0)) * np.exp(-(ell[2:] / lscale) ** 2)
    return cl


def config1(seed: int = 0, nside: int = 32, lmax: int = 64) -> TemperatureWorkload:
    """Small temperature problem: nside 32, lmax 64, C_l = 1000/(l(l+1)), log-uniform noise
    variance in [1, 10], |z| < 0.2 band plus 20 discs of 3 deg masked."""
    rng = np.random.Generator(np.random.PCG64(seed))
    npix = 12 * nside * nside
    cl = cl_config1(lmax)
    h = white_alm(rng, lmax)
    g = rng.standard_normal(npix)
    centres = _unit_vectors(rng, 20)
    u = rng.random(npix)
    z, phi = pixel_centres(nside)
    mask = disc_mask(z, phi, centres, math.radians(3.0), 0.2)
    ls, _ = alm_l_m(lmax)
    return TemperatureWorkload("nside32_lmax64_T", nside, lmax, cl, np.sqrt(cl[ls]) * h, g,
                               10.0 ** u, mask)


def scan_hits(z, xi):
    """Smooth scan pattern 1 + 19 cos^2(theta) with 5 % seeded jitter."""
    return (1.0 + 19.0 * z * z) * (1.0 + 0.05 * xi)


def config2(seed: int = 0, nside: int = 512, lmax: int = 1024, lscale: float = 800.0,
            ndisc: int = 100, band_z: float = 0.15) -> TemperatureWorkload:
    """Large temperature problem: nside 512, lmax 1024, C_l = 6000/(l(l+1)) exp(-(l/800)^2),
    noise variance 30^2/hits, |z| < 0.15 band plus 100 discs of 3 deg masked."""
    rng = np.random.Generator(np.random.PCG64(seed))
    npix = 12 * nside * nside
    cl = cl_damped(lmax, lscale)
    h = white_alm(rng, lmax)
    g = rng.standard_normal(npix)
    centres = _unit_vectors(rng, ndisc)
    xi = rng.uniform(-1.0, 1.0, npix)
    z, phi = pixel_centres(nside)
    mask = disc_mask(z, phi, centres, math.radians(3.0), band_z)
    hits = scan_hits(z, xi)
    ls, _ = alm_l_m(lmax)
    return TemperatureWorkload(f"nside{nside}_lmax{lmax}_T", nside, lmax, cl,
                               np.sqrt(cl[ls]) * h, g, 900.0 / hits, mask)


def batch_noise(b: int, npix: int) -> np.ndarray:
    """Unit-white pixel noise of map b of the batched nside 512 benchmark (one signal, B noise
    realisations): PCG64 seeded with 1000 + b.  Map b's data is sig + sqrt(noise_var) *
    batch_noise(b), sig the synthesis of config2(0).signal_alm."""
    return np.random.Generator(np.random.PCG64(1000 + b)).standard_normal(npix)


def config4(seed: int = 0, nside: int = 256, lmax: int = 512, lscale: float = 800.0,
            ndisc: int = 100, band_z: float = 0.15, parent_nside: int = 512,
            parent_lmax: int = 1024) -> TemperatureWorkload:
    """Downgraded large problem (nside 256, lmax 512): the mask of config 2 (the same disc
    centres, drawn exactly as config 2 draws them at the parent resolution, and the same band)
    evaluated at nside-256 pixel centres; M = 4 hits / 30^2, the parent pixel's inverse
    variance as the sum over its 4 children, hits from the scan law at the nside-256 centres
    with a jitter of their own; C_l as config 2.  The signal and noise of this workload are
    those of config4_draws(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white_alm(rng, parent_lmax)                  # the parent's signal and noise draws,
    rng.standard_normal(12 * parent_nside ** 2)  # consumed so that the discs match
    centres = _unit_vectors(rng, ndisc)
    xi = rng.uniform(-1.0, 1.0, 12 * nside * nside)
    z, phi = pixel_centres(nside)
    mask = disc_mask(z, phi, centres, math.radians(3.0), band_z)
    hits = scan_hits(z, xi)
    cl = cl_damped(lmax, lscale)
    h, g = config4_draws(seed, nside, lmax)
    ls, _ = alm_l_m(lmax)
    return TemperatureWorkload(f"nside{nside}_lmax{lmax}_T_downgraded", nside, lmax, cl,
                               np.sqrt(cl[ls]) * h, g, 900.0 / (4.0 * hits), mask)


def config4_draws(seed: int, nside: int = 256, lmax: int = 512):
    """Signal (unit-white harmonic) and noise (unit-white pixel) draws of one Wiener-filter
    data set of the downgraded workload, from seed + 2^20 (apart from the mask's stream)."""
    rng = np.random.Generator(np.random.PCG64(seed + (1 << 20)))
    h = white_alm(rng, lmax)
    g = rng.standard_normal(12 * nside * nside)
    return h, g


def fluctuation_draws(seed: int, nside: int, lmax: int):
    """White-noise draws for one constrained-realisation source (Eq. 9): g1 per pixel and a
    unit-white harmonic draw h (real basis, complex packing)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = white_alm(rng, lmax)
    g1 = rng.standard_normal(12 * nside * nside)
    return g1, h


# ---- temperature + polarization (T, Q, U) -----------------------------------------------

def pol_cls(cl_tt):
    """[4][lmax+1] = TT, EE, BB, TE with EE = 0.05 TT, TE = 0.5 cos(2 pi l / 300)
    sqrt(TT EE), BB = 0.01 EE (l < 2 all zero, as TT)."""
    lmax = len(cl_tt) - 1
    ell = np.arange(lmax + 1, dtype=np.float64)
    ee = 0.05 * cl_tt
    te = 0.5 * np.cos(2.0 * np.pi * ell / 300.0) * np.sqrt(cl_tt * ee)
    return np.stack([cl_tt, ee, 0.01 * ee, te])


def pack_sym3(A):
    """[..., 3, 3] symmetric -> [..., 6] = (TT, TQ, TU, QQ, QU, UU)."""
    return np.stack([A[..., 0, 0], A[..., 0, 1], A[..., 0, 2], A[..., 1, 1], A[..., 1, 2],
                     A[..., 2, 2]], axis=-1)


@dataclasses.dataclass
class PolWorkload:
    """Inputs of one T, Q, U Wiener-filter problem."""
    name: str
    nside: int
    lmax: int
    cl4: np.ndarray           # [4][lmax+1] TT, EE, BB, TE
    signal_alm: np.ndarray    # [3][nalm] complex T, E, B signal draw
    noise_white: np.ndarray   # [3][npix] unit normals
    noise_chol: np.ndarray    # [npix][3][3] lower factor of N_p (pixel noise = chol @ white)
    ninv6: np.ndarray         # [npix][6] packed N_p^{-1} (observed pixels; all pixels)
    mask: np.ndarray          # [npix] uint8, 1 = observed

    @property
    def npix(self):
        return 12 * self.nside * self.nside

    def M6(self):
        """Packed N^{-1} with masked pixels zeroed."""
        return self.ninv6 * self.mask[:, None]

    def data_from_signal_maps(self, signal_maps):
        """d = s + n (Eq. 1) with n_p = chol(N_p) g_p."""
        n = np.einsum("pij,jp->ip", self.noise_chol, self.noise_white)
        return signal_maps + n


def config3(seed: int = 0, nside: int = 512, lmax: int = 1024, lscale: float = 800.0,
            ndisc: int = 100, band_z: float = 0.15, nu: int = 10) -> PolWorkload:
    """T, Q, U problem: C^TT as the nside 512 temperature problem, EE/TE/BB from pol_cls,
    noise N_p = (30^2 / hits_p) W_p / nu with W_p ~ Wishart(nu, diag(1, 2, 2)), the same
    mask for T and P.  Signal (T, E, B) alm = L_l h with L_l L_l^T the 3x3 signal block.
    Draw order: signal, pixel noise, disc centres, hit jitter, Wishart draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    npix = 12 * nside * nside
    cl4 = pol_cls(cl_damped(lmax, lscale))
    h = np.stack([white_alm(rng, lmax) for _ in range(3)])
    g = rng.standard_normal((3, npix))
    centres = _unit_vectors(rng, ndisc)
    xi = rng.uniform(-1.0, 1.0, npix)
    z, phi = pixel_centres(nside)
    mask = disc_mask(z, phi, centres, math.radians(3.0), band_z)
    hits = scan_hits(z, xi)
    x = rng.standard_normal((npix, nu, 3)) * np.sqrt(np.array([1.0, 2.0, 2.0]))
    W = np.einsum("pki,pkj->pij", x, x)
    N = (900.0 / hits)[:, None, None] * W / nu
    ls, _ = alm_l_m(lmax)
    tt, ee, bb, te = cl4[0][ls], cl4[1][ls], cl4[2][ls], cl4[3][ls]
    a = np.sqrt(tt)
    b = np.where(a > 0, te / np.where(a > 0, a, 1.0), 0.0)
    c = np.sqrt(np.maximum(ee - b * b, 0.0))
    sig = np.stack([a * h[0], b * h[0] + c * h[1], np.sqrt(bb) * h[2]])
    return PolWorkload(f"nside{nside}_lmax{lmax}_TQU", nside, lmax, cl4, sig, g,
                       np.linalg.cholesky(N), pack_sym3(np.linalg.inv(N)), mask)



# ---- serving requests ----------------------------------------------------------------------

@dataclasses.dataclass
class ServeRequest:
    """One independent temperature Wiener-filter request."""
    rid: int
    nside: int
    lmax: int
    dtype: str
    cl: np.ndarray
    noise_var: np.ndarray
    mask: np.ndarray
    signal_alm: np.ndarray
    noise_white: np.ndarray


def serve_request(rid: int, nsides=(128, 256, 512, 1024), lscale: float = 1500.0,
                  ndisc: int = 50) -> ServeRequest:
    """A serving request seeded by its id: nside uniform over `nsides`, lmax = 2 nside,
    C_l = 6000/(l(l+1)) exp(-(l/1500)^2), hits = 10^(3u) (a 1000x span), noise variance
    30^2/hits, a sky cut f ~ U[0.10, 0.30] made of the band |z| < 0.75 f and `ndisc` discs
    whose common radius gives the rest, 2 pi (1 - cos r) ndisc = 0.25 f 4 pi (overlaps
    ignored), dtype FP32 or FP64 with probability 1/2.  Draw order: shape, dtype, cut,
    signal, noise, disc centres, hits."""
    rng = np.random.Generator(np.random.PCG64(rid))
    nside = int(nsides[rng.integers(len(nsides))])
    dtype = "f32" if rng.random() < 0.5 else "f64"
    f = rng.uniform(0.10, 0.30)
    lmax = 2 * nside
    npix = 12 * nside * nside
    cl = cl_damped(lmax, lscale)
    h = white_alm(rng, lmax)
    g = rng.standard_normal(npix)
    centres = _unit_vectors(rng, ndisc)
    u = rng.random(npix)
    radius = math.acos(1.0 - 0.5 * f / ndisc)
    z, phi = pixel_centres(nside)
    mask = disc_mask(z, phi, centres, radius, 0.75 * f)
    ls, _ = alm_l_m(lmax)
    return ServeRequest(rid, nside, lmax, dtype, cl, 900.0 / 10.0 ** (3.0 * u), mask,
                        np.sqrt(cl[ls]) * h, g)
