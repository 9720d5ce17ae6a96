"""Dense linear-algebra toolkit for tiny HEALPix problems (TEST INFRASTRUCTURE).

Builds the explicit real-basis synthesis matrix Y from ``scipy.special.sph_harm_y`` at the
pixel centres, then states the solver's equations as plain matrices:

* textbook Wiener filter, Eq. (2):           (C^-1 + Y^T M Y) s = Y^T rho
* messenger fixed point at constant lambda:  the s that Eqs. (3)-(4) map to itself
* exact k-step iterate of Eqs. (3)-(4) from s = 0
* spectral radius of the iteration operator (the contraction of Eq. 5)

Real harmonic basis (orthonormal on the sphere): Y_l0, sqrt(2) Re Y_lm, -sqrt(2) Im Y_lm
(m > 0), with coefficient vector x = (a_l0, sqrt(2) Re a_lm, sqrt(2) Im a_lm), so that
Y x equals the complex-packed synthesis and |x|^2 counts m > 0 twice.
"""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y

from . import nalm, pixel_angles


def lm_arrays(lmax):
    ls, ms = [], []
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            ls.append(l)
            ms.append(m)
    return np.array(ls), np.array(ms)


def alm_to_real(alm, lmax):
    alm = np.asarray(alm)
    ls, ms = lm_arrays(lmax)
    pos = ms > 0
    return np.concatenate([alm[~pos].real, np.sqrt(2.0) * alm[pos].real,
                           np.sqrt(2.0) * alm[pos].imag])


def real_to_alm(x, lmax):
    ls, ms = lm_arrays(lmax)
    pos = ms > 0
    n0, npos = int((~pos).sum()), int(pos.sum())
    alm = np.zeros(nalm(lmax), dtype=np.complex128)
    alm[~pos] = x[:n0]
    alm[pos] = (x[n0:n0 + npos] + 1j * x[n0 + npos:]) / np.sqrt(2.0)
    return alm


def real_ell(lmax):
    """Multipole l of every real-basis coefficient, same order as alm_to_real."""
    ls, ms = lm_arrays(lmax)
    pos = ms > 0
    return np.concatenate([ls[~pos], ls[pos], ls[pos]])


def synthesis_matrix(nside, lmax):
    """Explicit Y [npix, (lmax+1)^2] in the real basis, from SciPy's Y_lm."""
    th, ph = pixel_angles(nside)
    ls, ms = lm_arrays(lmax)
    pos = ms > 0
    cols0 = [sph_harm_y(l, 0, th, ph).real for l in ls[~pos]]
    colsr = [np.sqrt(2.0) * sph_harm_y(l, m, th, ph).real for l, m in zip(ls[pos], ms[pos])]
    colsi = [-np.sqrt(2.0) * sph_harm_y(l, m, th, ph).imag for l, m in zip(ls[pos], ms[pos])]
    return np.stack(cols0 + colsr + colsi, axis=1)


class Problem:
    """One temperature problem in dense form (tiny sizes only)."""

    def __init__(self, nside, lmax, cl, M, Y=None):
        self.nside, self.lmax = nside, lmax
        self.npix = 12 * nside * nside
        self.omega = 4.0 * np.pi / self.npix
        self.Y = synthesis_matrix(nside, lmax) if Y is None else Y
        self.cr = np.asarray(cl, dtype=np.float64)[real_ell(lmax)]
        self.keep = self.cr > 0.0
        self.M = np.asarray(M, dtype=np.float64)
        self.tau = 1.0 / self.M.max()

    # -- operators restricted to modes with C_l > 0 ------------------------------------
    def _Yk(self):
        return self.Y[:, self.keep]

    def iteration_operator(self, lam=1.0):
        """Linear part of one messenger iteration on the harmonic vector s:
        s' = D_lam Omega Y^T W_lam (1 - tau M) Y s,  W_lam = 1/(1 + (lam-1) tau M)."""
        Yk, c = self._Yk(), self.cr[self.keep]
        D = c / (c + lam * self.tau * self.omega)
        W = 1.0 / (1.0 + (lam - 1.0) * self.tau * self.M)
        return (D[:, None] * self.omega) * (Yk.T @ ((W * (1.0 - self.tau * self.M))[:, None] * Yk))

    def iteration_source(self, rho, lam=1.0):
        Yk, c = self._Yk(), self.cr[self.keep]
        D = c / (c + lam * self.tau * self.omega)
        W = 1.0 / (1.0 + (lam - 1.0) * self.tau * self.M)
        return D * self.omega * (Yk.T @ (W * lam * self.tau * rho))

    def _expand(self, sk):
        s = np.zeros(self.Y.shape[1])
        s[self.keep] = sk
        return s

    def textbook_wf(self, rho):
        """(C^-1 + Y^T M Y) s = Y^T rho (Eq. 2 with rho = M d), modes with C > 0."""
        Yk, c = self._Yk(), self.cr[self.keep]
        A = np.diag(1.0 / c) + Yk.T @ (self.M[:, None] * Yk)
        return self._expand(np.linalg.solve(A, Yk.T @ rho))

    def messenger_fixed_point(self, rho, lam=1.0):
        """The s with s = G s + b for the constant-lambda iteration (G, b above)."""
        G = self.iteration_operator(lam)
        b = self.iteration_source(rho, lam)
        return self._expand(np.linalg.solve(np.eye(len(b)) - G, b))

    def fixed_point_matrix(self):
        """F = C^-1 + I/(tau Omega) - Y^T (tau^-1 - M) Y; F s = Y^T rho at lambda = 1."""
        Yk, c = self._Yk(), self.cr[self.keep]
        return (np.diag(1.0 / c + 1.0 / (self.tau * self.omega))
                - Yk.T @ ((1.0 / self.tau - self.M)[:, None] * Yk))

    def k_step(self, rho, k, lam=1.0):
        """Exact k-th iterate from s = 0 at constant lambda."""
        G = self.iteration_operator(lam)
        b = self.iteration_source(rho, lam)
        s = np.zeros(len(b))
        for _ in range(k):
            s = G @ s + b
        return self._expand(s)

    def spectral_radius(self, lam=1.0):
        return float(np.max(np.abs(np.linalg.eigvals(self.iteration_operator(lam)))))

    def gram_eigs(self):
        """Eigenvalues of Omega Y^T Y (all modes); 1 where the pixel sum is an exact
        quadrature."""
        return np.linalg.eigvalsh(self.omega * (self.Y.T @ self.Y))


# ---- polarization: (T, Q, U) from (T, E, B) written from the definition ------------------

def pol_synthesis_direct(nside, lmax, alm3):
    """(T, Q, U) maps [3][npix] of (T, E, B) coefficients [3][nalm] summed term by term from
    the definition: T = sum a^T_lm Y_lm (SciPy), Q + iU = sum_{l, |m| <= l} 2a_lm 2Y_lm with
    2a_lm = -(a^E_lm + i a^B_lm), the reality of the scalar E and B fields
    a_{l,-m} = (-1)^m conj(a_lm), 2Y_lm = 2lambda_lm(theta) e^{i m phi} and
    2lambda_{l,-m} = (-1)^m (-2)lambda_lm.  The spin-weighted functions 2lambda, (-2)lambda
    are the oracle's (oracle.spin2, pinned separately to the spin-raising definition)."""
    from . import spin2
    alm3 = np.asarray(alm3, dtype=np.complex128)
    th, ph = pixel_angles(nside)
    npix = th.size
    ls, ms = lm_arrays(lmax)
    out = np.zeros((3, npix))
    # T: sum over m >= 0 with the m < 0 terms as conjugates (real field)
    for k, (l, m) in enumerate(zip(ls, ms)):
        y = sph_harm_y(l, m, th, ph)
        out[0] += (alm3[0, k] * y).real * (1.0 if m == 0 else 2.0)
    P = np.zeros(npix, dtype=np.complex128)
    zs, inv = np.unique(np.cos(th), return_inverse=True)
    for m in range(lmax + 1):
        lp = np.zeros((zs.size, lmax - m + 1))
        lm_ = np.zeros((zs.size, lmax - m + 1))
        for u, z in enumerate(zs):
            fp, fm = spin2(lmax, m, z)
            lp[u], lm_[u] = fp + fm, fp - fm           # 2lambda, (-2)lambda, l = m..lmax
        e = np.exp(1j * m * ph)
        sel = ms == m
        aE, aB = alm3[1, sel], alm3[2, sel]
        P += (lp[inv] @ (-(aE + 1j * aB))) * e        # the +m term
        if m > 0:
            # the -m term: 2a_{l,-m} 2lambda_{l,-m} e^{-i m phi}
            #   = -(conj aE + i conj aB) (-2)lambda_lm e^{-i m phi}
            P += (lm_[inv] @ (-(np.conj(aE) + 1j * np.conj(aB)))) * np.conj(e)
    out[1], out[2] = P.real, P.imag
    return out


def pol_synthesis_matrix(nside, lmax):
    """The same synthesis as a real matrix [3 npix, 3 (lmax+1)^2]: rows (T, Q, U) pixels,
    columns the real-basis coordinates (alm_to_real) of T, then E, then B."""
    n = (lmax + 1) ** 2
    cols = []
    for c in range(3):
        for j in range(n):
            x = np.zeros(n)
            x[j] = 1.0
            a = np.zeros((3, nalm(lmax)), dtype=np.complex128)
            a[c] = real_to_alm(x, lmax)
            cols.append(pol_synthesis_direct(nside, lmax, a).ravel())
    return np.stack(cols, axis=1)
