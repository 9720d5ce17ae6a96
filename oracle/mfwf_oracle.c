/*
 * Plain FP64 CPU oracle for the messenger-field Wiener filter
 * (Elsner & Wandelt, "Efficient Wiener filtering without preconditioning").
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no code with the HIP path: geometry,
 * Legendre recurrence, phi transforms, SHT, messenger iteration and chi^2 are all written
 * here again, slowly and directly, from the paper and the textbook definitions.
 *
 * Conventions (all readings are listed in the design notes):
 *   maps   HEALPix RING order, double[npix]
 *   alm    complex m-major packing (m, l = m..lmax), stored as interleaved re/im doubles
 *   Y      synthesis: f(p) = sum_{l, |m|<=l} a_lm Y_lm(theta_p, phi_p), a_{l,-m} = (-1)^m conj(a_lm)
 *   A      analysis: a_lm = Omega * sum_p f(p) conj(Y_lm(theta_p, phi_p)),  Omega = 4 pi / npix
 *          (uniform pixel weights: A is exactly Omega * Y^T in the real harmonic basis)
 *
 * Precision: every quantity is double.  Associated-Legendre seeds carry an explicit
 * power-of-two exponent so that sin(theta)^m never underflows before the l-recurrence has
 * grown it back into range.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------------------
 * HEALPix RING geometry (Gorski et al. 2005, the pixelisation used in Sect. 3).
 * Rings are numbered i = 1 .. 4 nside - 1 from north to south.
 *   north cap  i < nside        : z = 1 - i^2/(3 nside^2), 4i pixels, phi_0 = pi/(4i)
 *   belt       nside <= i <= 3ns: z = 4/3 - 2i/(3 nside), 4 nside pixels,
 *                                 phi_0 = pi/(4 nside) if (i - nside) even, else 0
 *   south cap  mirror of the north cap (z -> -z)
 * Pixel j of a ring sits at phi_0 + 2 pi j / n_phi.
 * sin(theta) is returned separately, computed from 1 - |z| without cancellation.
 * ------------------------------------------------------------------------------------ */
long or_npix(int nside) { return 12L * nside * nside; }
int or_nrings(int nside) { return 4 * nside - 1; }

void or_ring(int nside, int i, double *z, double *sth, long *start, int *nphi, double *phi0)
{
    long ns = nside, npix = 12L * ns * ns;
    if (i < nside) {
        double omz = (double)i * i / (3.0 * ns * ns); /* 1 - z */
        *z = 1.0 - omz;
        *sth = sqrt(omz * (2.0 - omz));
        *nphi = 4 * i;
        *start = 2L * i * (i - 1);
        *phi0 = M_PI / (4.0 * i);
    } else if (i <= 3 * nside) {
        *z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns);
        *sth = sqrt((1.0 - *z) * (1.0 + *z));
        *nphi = 4 * nside;
        *start = 2L * ns * (ns - 1) + (long)(i - nside) * 4L * ns;
        *phi0 = ((i - nside) % 2 == 0) ? M_PI / (4.0 * ns) : 0.0;
    } else {
        int k = 4 * nside - i;
        double omz = (double)k * k / (3.0 * ns * ns);
        *z = -(1.0 - omz);
        *sth = sqrt(omz * (2.0 - omz));
        *nphi = 4 * k;
        *start = npix - 2L * k * (k + 1);
        *phi0 = M_PI / (4.0 * k);
    }
}

long or_nalm(int lmax) { return (long)(lmax + 1) * (lmax + 2) / 2; }
static long aidx(int lmax, int l, int m) { return (long)m * (2 * lmax + 3 - m) / 2 + (l - m); }

/* ------------------------------------------------------------------------------------
 * Orthonormal associated Legendre functions with the Condon-Shortley phase,
 *   Y_lm(theta, phi) = lambda_lm(cos theta) e^{i m phi},
 *   lambda_mm     = (-1)^m sqrt(1/(4 pi)) prod_{k=1..m} sqrt((2k+1)/(2k)) sin(theta)
 *   lambda_{m+1,m}= sqrt(2m+3) z lambda_mm
 *   lambda_lm     = (z lambda_{l-1,m} - eps_{l-1,m} lambda_{l-2,m}) / eps_lm,
 *   eps_lm        = sqrt((l^2 - m^2)/(4 l^2 - 1)).
 * The running pair is held as (mantissa, shared power-of-two exponent); values are written
 * out with ldexp, so anything below the double range becomes 0.
 * eps must hold eps_lm for l = 0..lmax (eps[l] for the given m; eps[m] = 0).
 * ------------------------------------------------------------------------------------ */
static void legendre_eps(int lmax, int m, double *eps)
{
    for (int l = 0; l <= lmax; l++)
        eps[l] = (l <= m) ? 0.0 : sqrt(((double)l * l - (double)m * m) / (4.0 * l * l - 1.0));
}

static void legendre_with_eps(int lmax, int m, double z, double sth, const double *eps,
                              double *out)
{
    int ex;
    long e = 0;
    double r = sqrt(1.0 / (4.0 * M_PI));
    for (int k = 1; k <= m; k++) {
        r *= -sqrt((2.0 * k + 1.0) / (2.0 * k)) * sth;
        r = frexp(r, &ex);
        e += ex;
    }
    double p2 = 0.0, p1 = r; /* scaled lambda_{l-2}, lambda_{l-1} */
    out[0] = ldexp(p1, (int)(e < -2000 ? -2000 : e));
    for (int l = m + 1; l <= lmax; l++) {
        double cur = (z * p1 - eps[l - 1] * p2) / eps[l];
        p2 = p1;
        p1 = cur;
        if (fabs(p1) > 0x1p+300) {
            p1 = ldexp(p1, -300);
            p2 = ldexp(p2, -300);
            e += 300;
        }
        out[l - m] = ldexp(p1, (int)(e < -2000 ? -2000 : e));
    }
}

/* lambda_lm(z), l = m..lmax, written to out[0 .. lmax-m]. */
void or_legendre(int lmax, int m, double z, double sth, double *out)
{
    double *eps = (double *)malloc(sizeof(double) * (lmax + 1));
    legendre_eps(lmax, m, eps);
    legendre_with_eps(lmax, m, z, sth, eps, out);
    free(eps);
}

/* ------------------------------------------------------------------------------------
 * Complex DFT, X_k = sum_j x_j exp(sign * 2 pi i j k / n).
 * or_dft: the definition summed directly, O(n^2).
 * or_fft: textbook recursive Cooley-Tukey decimation in time over the smallest prime
 *         factor; a prime length falls back to the direct sum.
 * ------------------------------------------------------------------------------------ */
void or_dft(int n, int sign, const double *xin, double *xout)
{
    const cplx *x = (const cplx *)xin;
    cplx *X = (cplx *)xout;
    for (int k = 0; k < n; k++) {
        cplx acc = 0;
        for (int j = 0; j < n; j++) {
            long jk = ((long)j * k) % n;
            double a = sign * 2.0 * M_PI * (double)jk / n;
            acc += x[j] * (cos(a) + I * sin(a));
        }
        X[k] = acc;
    }
}

static void fft_rec(int n, long stride, const cplx *in, cplx *out, int sign, cplx *scratch)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = n;
    for (int f = 2; (long)f * f <= n; f++)
        if (n % f == 0) {
            p = f;
            break;
        }
    if (p == n) { /* prime length: direct sum */
        for (int k = 0; k < n; k++) {
            cplx acc = 0;
            for (int j = 0; j < n; j++) {
                long jk = ((long)j * k) % n;
                double a = sign * 2.0 * M_PI * (double)jk / n;
                acc += in[j * stride] * (cos(a) + I * sin(a));
            }
            out[k] = acc;
        }
        return;
    }
    int q = n / p;
    /* sub-transforms of the p decimated sequences x[p*j + r], stored out[r*q + k] */
    for (int r = 0; r < p; r++)
        fft_rec(q, stride * p, in + r * stride, out + (long)r * q, sign, scratch + n);
    /* combine: X[k + q s] = sum_r exp(sign 2 pi i r (k + q s)/n) Y_r[k] */
    for (int k = 0; k < q; k++)
        for (int s = 0; s < p; s++) {
            int kk = k + q * s;
            cplx acc = 0;
            for (int r = 0; r < p; r++) {
                long e = ((long)r * kk) % n;
                double a = sign * 2.0 * M_PI * (double)e / n;
                acc += out[(long)r * q + k] * (cos(a) + I * sin(a));
            }
            scratch[kk] = acc;
        }
    memcpy(out, scratch, sizeof(cplx) * n);
}

void or_fft(int n, int sign, const double *xin, double *xout)
{
    /* scratch: the recursion uses one n-sized block per level, sum over levels <= 2n */
    cplx *scratch = (cplx *)malloc(sizeof(cplx) * (2 * (size_t)n + 2));
    fft_rec(n, 1, (const cplx *)xin, (cplx *)xout, sign, scratch);
    free(scratch);
}

/* ------------------------------------------------------------------------------------
 * phi step for one ring.
 * Synthesis: f_j = sum_{m=-lmax}^{lmax} F(m) e^{i m phi_j},  F(-m) = conj F(m).
 * Analysis:  G(m) = sum_j t_j e^{-i m phi_j},  m = 0..lmax.
 * direct = 1: evaluate the sums as written (cos/sin of m phi_j).
 * direct = 0: fold the harmonics into the n_phi DFT bins (m mod n_phi) with the ring
 *             offset phase e^{i m phi_0}, then one length-n_phi DFT.
 * ------------------------------------------------------------------------------------ */
static void ring_synth(int lmax, int nphi, double phi0, const cplx *F, double *f, int direct)
{
    if (direct) {
        for (int j = 0; j < nphi; j++) {
            double phi = phi0 + 2.0 * M_PI * j / nphi;
            double acc = creal(F[0]);
            for (int m = 1; m <= lmax; m++)
                acc += 2.0 * (creal(F[m]) * cos(m * phi) - cimag(F[m]) * sin(m * phi));
            f[j] = acc;
        }
        return;
    }
    cplx *B = (cplx *)calloc(nphi, sizeof(cplx));
    cplx *x = (cplx *)malloc(sizeof(cplx) * nphi);
    for (int m = 0; m <= lmax; m++) {
        cplx ph = cos(m * phi0) + I * sin(m * phi0);
        B[m % nphi] += F[m] * ph;
        if (m > 0)
            B[(nphi - m % nphi) % nphi] += conj(F[m] * ph);
    }
    or_fft(nphi, +1, (const double *)B, (double *)x);
    for (int j = 0; j < nphi; j++)
        f[j] = creal(x[j]);
    free(B);
    free(x);
}

static void ring_analysis(int lmax, int nphi, double phi0, const double *t, cplx *G, int direct)
{
    if (direct) {
        for (int m = 0; m <= lmax; m++) {
            cplx acc = 0;
            for (int j = 0; j < nphi; j++) {
                double a = m * (phi0 + 2.0 * M_PI * j / nphi);
                acc += t[j] * (cos(a) - I * sin(a));
            }
            G[m] = acc;
        }
        return;
    }
    cplx *x = (cplx *)malloc(sizeof(cplx) * nphi);
    cplx *X = (cplx *)malloc(sizeof(cplx) * nphi);
    for (int j = 0; j < nphi; j++)
        x[j] = t[j];
    or_fft(nphi, -1, (const double *)x, (double *)X);
    for (int m = 0; m <= lmax; m++)
        G[m] = X[m % nphi] * (cos(m * phi0) - I * sin(m * phi0));
    free(x);
    free(X);
}

/* ------------------------------------------------------------------------------------
 * Spin-0 SHT.  Every ring is handled on its own (no north/south pairing).
 * ------------------------------------------------------------------------------------ */
void or_alm2map(int nside, int lmax, const double *alm_in, double *map, int direct)
{
    const cplx *alm = (const cplx *)alm_in;
    int nr = or_nrings(nside);
#pragma omp parallel
    {
        double *lam = (double *)malloc(sizeof(double) * (lmax + 1));
        double *eps = (double *)malloc(sizeof(double) * (lmax + 1));
        cplx *F = (cplx *)malloc(sizeof(cplx) * (lmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int i = 1; i <= nr; i++) {
            double z, sth, phi0;
            long start;
            int nphi;
            or_ring(nside, i, &z, &sth, &start, &nphi, &phi0);
            for (int m = 0; m <= lmax; m++) {
                legendre_eps(lmax, m, eps);
                legendre_with_eps(lmax, m, z, sth, eps, lam);
                cplx acc = 0;
                for (int l = m; l <= lmax; l++)
                    acc += lam[l - m] * alm[aidx(lmax, l, m)];
                F[m] = acc;
            }
            ring_synth(lmax, nphi, phi0, F, map + start, direct);
        }
        free(lam);
        free(eps);
        free(F);
    }
}

void or_map2alm(int nside, int lmax, const double *map, double *alm_out, int direct)
{
    cplx *alm = (cplx *)alm_out;
    int nr = or_nrings(nside);
    double omega = 4.0 * M_PI / (double)or_npix(nside);
    cplx *G = (cplx *)malloc(sizeof(cplx) * (size_t)nr * (lmax + 1));
    double *zr = (double *)malloc(sizeof(double) * nr);
    double *sr = (double *)malloc(sizeof(double) * nr);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 1; i <= nr; i++) {
        double phi0;
        long start;
        int nphi;
        or_ring(nside, i, &zr[i - 1], &sr[i - 1], &start, &nphi, &phi0);
        ring_analysis(lmax, nphi, phi0, map + start, G + (size_t)(i - 1) * (lmax + 1), direct);
    }
#pragma omp parallel
    {
        double *lam = (double *)malloc(sizeof(double) * (lmax + 1));
        double *eps = (double *)malloc(sizeof(double) * (lmax + 1));
        cplx *acc = (cplx *)malloc(sizeof(cplx) * (lmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m <= lmax; m++) {
            legendre_eps(lmax, m, eps);
            for (int l = m; l <= lmax; l++)
                acc[l - m] = 0;
            for (int r = 0; r < nr; r++) {
                legendre_with_eps(lmax, m, zr[r], sr[r], eps, lam);
                cplx g = G[(size_t)r * (lmax + 1) + m];
                for (int l = m; l <= lmax; l++)
                    acc[l - m] += lam[l - m] * g;
            }
            for (int l = m; l <= lmax; l++)
                alm[aidx(lmax, l, m)] = omega * acc[l - m];
        }
        free(lam);
        free(eps);
        free(acc);
    }
    free(G);
    free(zr);
    free(sr);
}

/* ------------------------------------------------------------------------------------
 * Messenger-field iteration (Sect. 2.1, Eqs. 3 and 4), temperature.
 *
 * M = N^{-1} per pixel (0 in masked pixels), tau = min diag N over observed pixels
 * = 1 / max M.  With rho = M d (Wiener filter) or the fluctuation source (Eq. 9),
 * Eq. (3) solved for t and multiplied through by N gives, per pixel,
 *     t = [lambda tau rho + (1 - tau M) s] / [1 + (lambda - 1) tau M],
 * which needs no inverse of Nbar = N - tau and is continuous into the mask.
 * The harmonic-space messenger covariance is tau * Omega (the analysis A = Omega Y^T maps
 * pixel-white variance tau to tau Omega per real harmonic dof), so Eq. (4) gives
 *     s_lm = C_l / (C_l + lambda tau Omega) * (A t)_lm,   s_lm = 0 where C_l = 0.
 * Start s = t = 0, t-update first.  lam[k] is lambda for iteration k.
 *
 * diag (optional, [niter][4]) per iteration: chi^2(s, lambda_k) (Eq. 6), its harmonic
 * part, |s_k - s_{k-1}|, |s_k|, all over the real harmonic dof (m > 0 counted twice).
 * chi^2 pixel part: sum over M > 0 of (d - s)^2 M / (1 + (lambda-1) tau M) with d = rho/M.
 * Returns 0, or -4 if max M <= 0 (tau undefined).
 * ------------------------------------------------------------------------------------ */
static double alm_dot_w(int lmax, const cplx *a, const cplx *b, const double *w)
{
    double acc = 0.0;
    for (int m = 0; m <= lmax; m++)
        for (int l = m; l <= lmax; l++) {
            long k = aidx(lmax, l, m);
            double wt = (w ? w[l] : 1.0) * (m == 0 ? 1.0 : 2.0);
            acc += wt * creal(conj(a[k]) * b[k]);
        }
    return acc;
}

double or_tau(long npix, const double *M)
{
    double mx = 0.0;
    for (long p = 0; p < npix; p++)
        if (M[p] > mx)
            mx = M[p];
    return mx > 0.0 ? 1.0 / mx : 0.0;
}

int or_solve(int nside, int lmax, const double *cl, const double *M, const double *rho,
             int niter, const double *lam, int direct, double *s_alm_out, double *s_map_out,
             double *diag)
{
    long npix = or_npix(nside), nalm = or_nalm(lmax);
    double tau = or_tau(npix, M);
    if (tau <= 0.0)
        return -4;
    double omega = 4.0 * M_PI / (double)npix;
    double *s_map = (double *)calloc(npix, sizeof(double));
    double *t = (double *)malloc(sizeof(double) * npix);
    cplx *a = (cplx *)malloc(sizeof(cplx) * nalm);
    cplx *s = (cplx *)calloc(nalm, sizeof(cplx));
    cplx *s_old = (cplx *)calloc(nalm, sizeof(cplx));
    double *icl = (double *)malloc(sizeof(double) * (lmax + 1));
    for (int l = 0; l <= lmax; l++)
        icl[l] = cl[l] > 0.0 ? 1.0 / cl[l] : 0.0;

    for (int k = 0; k < niter; k++) {
        double L = lam[k];
        for (long p = 0; p < npix; p++)
            t[p] = (L * tau * rho[p] + (1.0 - tau * M[p]) * s_map[p]) / (1.0 + (L - 1.0) * tau * M[p]);
        or_map2alm(nside, lmax, t, (double *)a, direct);
        memcpy(s_old, s, sizeof(cplx) * nalm);
        for (int m = 0; m <= lmax; m++)
            for (int l = m; l <= lmax; l++) {
                long i = aidx(lmax, l, m);
                s[i] = cl[l] > 0.0 ? cl[l] / (cl[l] + L * tau * omega) * a[i] : 0.0;
            }
        or_alm2map(nside, lmax, (const double *)s, s_map, direct);
        if (diag) {
            double harm = alm_dot_w(lmax, s, s, icl);
            double pix = 0.0;
            for (long p = 0; p < npix; p++)
                if (M[p] > 0.0) {
                    double r = rho[p] / M[p] - s_map[p];
                    pix += r * r * M[p] / (1.0 + (L - 1.0) * tau * M[p]);
                }
            for (long i = 0; i < nalm; i++)
                s_old[i] = s[i] - s_old[i];
            diag[4 * k + 0] = harm + pix;
            diag[4 * k + 1] = harm;
            diag[4 * k + 2] = sqrt(alm_dot_w(lmax, s_old, s_old, NULL));
            diag[4 * k + 3] = sqrt(alm_dot_w(lmax, s, s, NULL));
        }
    }
    if (s_alm_out)
        memcpy(s_alm_out, s, sizeof(cplx) * nalm);
    if (s_map_out)
        memcpy(s_map_out, s_map, sizeof(double) * npix);
    free(s_map);
    free(t);
    free(a);
    free(s);
    free(s_old);
    free(icl);
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Fluctuation source (Sect. 2.3, Eq. 9).  The replacement Nbar^{-1} d ->
 * Nbar^{-1} N (N^{-1/2} g1 + S^{-1/2} g2) is, in the per-pixel form above, the source
 *     rho = M^{1/2} g1 + Omega * Y(C^{-1/2} h),
 * with h unit-white in the real harmonic basis and C^{-1/2} := 0 where C_l = 0.  The
 * factor Omega makes Y^T rho_2 = (Omega Y^T Y) C^{-1/2} h ~ C^{-1/2} h.  In masked pixels
 * (M = 0) the update becomes t = s + lambda tau rho, the identity replacement of
 * Nbar^{-1} N the paper prescribes there.
 * ------------------------------------------------------------------------------------ */
void or_fluct_rho(int nside, int lmax, const double *cl, const double *M, const double *g1,
                  const double *h_in, double *rho, int direct)
{
    long npix = or_npix(nside), nalm = or_nalm(lmax);
    const cplx *h = (const cplx *)h_in;
    cplx *x = (cplx *)malloc(sizeof(cplx) * nalm);
    for (int m = 0; m <= lmax; m++)
        for (int l = m; l <= lmax; l++) {
            long i = aidx(lmax, l, m);
            x[i] = cl[l] > 0.0 ? h[i] / sqrt(cl[l]) : 0.0;
        }
    or_alm2map(nside, lmax, (const double *)x, rho, direct);
    double omega = 4.0 * M_PI / (double)npix;
    for (long p = 0; p < npix; p++)
        rho[p] = sqrt(M[p]) * g1[p] + omega * rho[p];
    free(x);
}

/* ------------------------------------------------------------------------------------
 * Spin-2 functions (polarization, HEALPix / Zaldarriaga-Seljak convention).
 *   Q + iU = sum 2a_lm 2Y_lm,  Q - iU = sum (-2)a_lm (-2)Y_lm,
 *   a_E = -(2a + (-2)a) / 2,   a_B = i (2a - (-2)a) / 2,
 *   (+-2)Y_lm = sqrt((l-2)!/(l+2)!) (eth or eth-bar)^2 Y_lm,  (s)Y_lm = (s)lambda_lm e^{i m phi}.
 * With F+ = (2lambda + (-2)lambda)/2 and F- = (2lambda - (-2)lambda)/2, working out the
 * two eth operators on lambda_lm e^{i m phi} (and the Legendre equation) gives
 *   F+_lm = N_l/s^2 [(2m^2 - l(l+1) + l(l-1) z^2) lambda_lm + 2 c_lm z lambda_{l-1,m}]
 *   F-_lm = 2 m N_l/s^2 [c_lm lambda_{l-1,m} - (l-1) z lambda_lm]
 *   N_l = 1/sqrt((l-1) l (l+1) (l+2)),  c_lm = sqrt((2l+1)(l^2 - m^2)/(2l-1)),
 * s = sin(theta); both vanish for l < 2.  Near the poles the bracket of F+ cancels by up to
 * s^4 for m = 0, so the values are formed in long double (64-bit mantissa) from a long
 * double recurrence at the point (z, s = sqrt((1-z)(1+z))), then rounded.
 * Out: fp[l-m], fm[l-m] for l = m..lmax.
 * ------------------------------------------------------------------------------------ */
void or_spin2(int lmax, int m, double z_in, double sth_in, double *fp, double *fm)
{
    /* evaluate at the point z_in exactly: s^2 = (1 - z)(1 + z) in long double (the bracket
       of F+ cancels to O(s^4) near the poles, so z and s must lie on the unit circle to
       the working precision; a separately rounded sin(theta) would break that) */
    (void)sth_in;
    long double z = z_in, s2 = (1.0L - z) * (1.0L + z), s = sqrtl(s2);
    int ex;
    long e = 0;
    long double r = sqrtl(1.0L / (4.0L * (long double)M_PI));
    for (int k = 1; k <= m; k++) {
        r *= -sqrtl((2.0L * k + 1.0L) / (2.0L * k)) * s;
        r = frexpl(r, &ex);
        e += ex;
    }
    long double prev = 0.0L, cur = r; /* scaled lambda_{l-1,m}, lambda_{l,m} at l = m */
    for (int l = m; l <= lmax; l++) {
        if (l > m) {
            long double eps_l = sqrtl(((long double)l * l - (long double)m * m) / (4.0L * l * l - 1.0L));
            long double eps_l1 = (l - 1 > m)
                ? sqrtl(((long double)(l - 1) * (l - 1) - (long double)m * m) / (4.0L * (l - 1) * (l - 1) - 1.0L))
                : 0.0L;
            long double nxt = (z * cur - eps_l1 * prev) / eps_l;
            prev = cur;
            cur = nxt;
            if (fabsl(cur) > 0x1p+300L) {
                cur = ldexpl(cur, -300);
                prev = ldexpl(prev, -300);
                e += 300;
            }
        }
        if (l < 2) {
            fp[l - m] = fm[l - m] = 0.0;
            continue;
        }
        long double L = l, mm = m;
        long double N = 1.0L / sqrtl((L - 1.0L) * L * (L + 1.0L) * (L + 2.0L));
        long double c = (l > m) ? sqrtl((2.0L * L + 1.0L) * (L * L - mm * mm) / (2.0L * L - 1.0L)) : 0.0L;
        long double bp = (2.0L * mm * mm - L * (L + 1.0L) + L * (L - 1.0L) * z * z) * cur + 2.0L * c * z * prev;
        long double bm = c * prev - (L - 1.0L) * z * cur;
        long double vp = N / s2 * bp, vm = 2.0L * mm * N / s2 * bm;
        int ee = (int)(e < -20000 ? -20000 : e);
        fp[l - m] = (double)ldexpl(vp, ee);
        fm[l - m] = (double)ldexpl(vm, ee);
    }
}

/* ------------------------------------------------------------------------------------
 * Polarized SHT, maps [3][npix] (T, Q, U), alm [3][nalm] (T, E, B).  T is the spin-0
 * transform.  Per ring and m, from the definitions above (sums over m >= 0 folded with
 * F(-m) = conj F(m) as for spin 0):
 *   synthesis  FQ(m) = -sum_l (aE F+ + i aB F-),   FU(m) = -sum_l (aB F+ - i aE F-)
 *   analysis   aE = -Omega sum_rings (F+ GQ + i F- GU),  aB = -Omega sum_rings (F+ GU - i F- GQ)
 * (the analysis is the adjoint of the synthesis, times Omega).  Every ring on its own.
 * ------------------------------------------------------------------------------------ */
void or_alm2map_pol(int nside, int lmax, const double *alm_in, double *map, int direct)
{
    long npix = or_npix(nside), nalm = or_nalm(lmax);
    or_alm2map(nside, lmax, alm_in, map, direct);
    const cplx *aE = (const cplx *)alm_in + nalm, *aB = (const cplx *)alm_in + 2 * nalm;
    int nr = or_nrings(nside);
#pragma omp parallel
    {
        double *fp = (double *)malloc(sizeof(double) * (lmax + 1));
        double *fm = (double *)malloc(sizeof(double) * (lmax + 1));
        cplx *FQ = (cplx *)malloc(sizeof(cplx) * (lmax + 1));
        cplx *FU = (cplx *)malloc(sizeof(cplx) * (lmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int i = 1; i <= nr; i++) {
            double z, sth, phi0;
            long start;
            int nphi;
            or_ring(nside, i, &z, &sth, &start, &nphi, &phi0);
            for (int m = 0; m <= lmax; m++) {
                or_spin2(lmax, m, z, sth, fp, fm);
                cplx q = 0, u = 0;
                for (int l = m; l <= lmax; l++) {
                    long k = aidx(lmax, l, m);
                    q += -(aE[k] * fp[l - m] + I * aB[k] * fm[l - m]);
                    u += -(aB[k] * fp[l - m] - I * aE[k] * fm[l - m]);
                }
                FQ[m] = q;
                FU[m] = u;
            }
            ring_synth(lmax, nphi, phi0, FQ, map + npix + start, direct);
            ring_synth(lmax, nphi, phi0, FU, map + 2 * npix + start, direct);
        }
        free(fp);
        free(fm);
        free(FQ);
        free(FU);
    }
}

void or_map2alm_pol(int nside, int lmax, const double *map, double *alm_out, int direct)
{
    long npix = or_npix(nside), nalm = or_nalm(lmax);
    or_map2alm(nside, lmax, map, alm_out, direct);
    cplx *aE = (cplx *)alm_out + nalm, *aB = (cplx *)alm_out + 2 * nalm;
    int nr = or_nrings(nside);
    double omega = 4.0 * M_PI / (double)npix;
    cplx *GQ = (cplx *)malloc(sizeof(cplx) * (size_t)nr * (lmax + 1));
    cplx *GU = (cplx *)malloc(sizeof(cplx) * (size_t)nr * (lmax + 1));
    double *zr = (double *)malloc(sizeof(double) * nr);
    double *sr = (double *)malloc(sizeof(double) * nr);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 1; i <= nr; i++) {
        double phi0;
        long start;
        int nphi;
        or_ring(nside, i, &zr[i - 1], &sr[i - 1], &start, &nphi, &phi0);
        ring_analysis(lmax, nphi, phi0, map + npix + start, GQ + (size_t)(i - 1) * (lmax + 1), direct);
        ring_analysis(lmax, nphi, phi0, map + 2 * npix + start, GU + (size_t)(i - 1) * (lmax + 1), direct);
    }
#pragma omp parallel
    {
        double *fp = (double *)malloc(sizeof(double) * (lmax + 1));
        double *fm = (double *)malloc(sizeof(double) * (lmax + 1));
        cplx *accE = (cplx *)malloc(sizeof(cplx) * (lmax + 1));
        cplx *accB = (cplx *)malloc(sizeof(cplx) * (lmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m <= lmax; m++) {
            for (int l = m; l <= lmax; l++)
                accE[l - m] = accB[l - m] = 0;
            for (int r = 0; r < nr; r++) {
                or_spin2(lmax, m, zr[r], sr[r], fp, fm);
                cplx gq = GQ[(size_t)r * (lmax + 1) + m], gu = GU[(size_t)r * (lmax + 1) + m];
                for (int l = m; l <= lmax; l++) {
                    accE[l - m] += -(fp[l - m] * gq + I * fm[l - m] * gu);
                    accB[l - m] += -(fp[l - m] * gu - I * fm[l - m] * gq);
                }
            }
            for (int l = m; l <= lmax; l++) {
                aE[aidx(lmax, l, m)] = omega * accE[l - m];
                aB[aidx(lmax, l, m)] = omega * accB[l - m];
            }
        }
        free(fp);
        free(fm);
        free(accE);
        free(accB);
    }
    free(GQ);
    free(GU);
    free(zr);
    free(sr);
}

/* Sampled outputs of the same transforms, for checks at sizes where the whole transform
 * would take minutes: T, Q, U of one ring (1-based ring index i; out[3][n_phi]) and
 * aT, aE, aB of one m (out[3][lmax - m + 1]). */
void or_alm2map_pol_ring(int nside, int lmax, const double *alm_in, int i, double *out)
{
    long nalm = or_nalm(lmax);
    const cplx *aT = (const cplx *)alm_in, *aE = aT + nalm, *aB = aT + 2 * nalm;
    double z, sth, phi0;
    long start;
    int nphi;
    or_ring(nside, i, &z, &sth, &start, &nphi, &phi0);
    double *lam = (double *)malloc(sizeof(double) * (lmax + 1));
    double *eps = (double *)malloc(sizeof(double) * (lmax + 1));
    double *fp = (double *)malloc(sizeof(double) * (lmax + 1));
    double *fm = (double *)malloc(sizeof(double) * (lmax + 1));
    cplx *F = (cplx *)malloc(sizeof(cplx) * 3 * (lmax + 1));
    for (int m = 0; m <= lmax; m++) {
        legendre_eps(lmax, m, eps);
        legendre_with_eps(lmax, m, z, sth, eps, lam);
        or_spin2(lmax, m, z, sth, fp, fm);
        cplx t = 0, q = 0, u = 0;
        for (int l = m; l <= lmax; l++) {
            long k = aidx(lmax, l, m);
            t += lam[l - m] * aT[k];
            q += -(aE[k] * fp[l - m] + I * aB[k] * fm[l - m]);
            u += -(aB[k] * fp[l - m] - I * aE[k] * fm[l - m]);
        }
        F[m] = t;
        F[lmax + 1 + m] = q;
        F[2 * (lmax + 1) + m] = u;
    }
    for (int c = 0; c < 3; c++)
        ring_synth(lmax, nphi, phi0, F + c * (lmax + 1), out + (long)c * nphi, 0);
    free(lam);
    free(eps);
    free(fp);
    free(fm);
    free(F);
}

/* Sampled outputs of the temperature transforms (Sect. 2.1 basis change): the map on one
 * ring (1-based ring index i; out[n_phi]) and the coefficients of one m (out[lmax - m + 1],
 * Omega included).  The per-m analysis takes G_r(m) straight from its definition,
 * sum_j t_j e^{-i m phi_j}, with the phase argument reduced as (m j mod n_phi). */
void or_alm2map_ring(int nside, int lmax, const double *alm_in, int i, double *out)
{
    const cplx *alm = (const cplx *)alm_in;
    double z, sth, phi0;
    long start;
    int nphi;
    or_ring(nside, i, &z, &sth, &start, &nphi, &phi0);
    double *lam = (double *)malloc(sizeof(double) * (lmax + 1));
    double *eps = (double *)malloc(sizeof(double) * (lmax + 1));
    cplx *F = (cplx *)malloc(sizeof(cplx) * (lmax + 1));
    for (int m = 0; m <= lmax; m++) {
        legendre_eps(lmax, m, eps);
        legendre_with_eps(lmax, m, z, sth, eps, lam);
        cplx t = 0;
        for (int l = m; l <= lmax; l++)
            t += lam[l - m] * alm[aidx(lmax, l, m)];
        F[m] = t;
    }
    ring_synth(lmax, nphi, phi0, F, out, 0);
    free(lam);
    free(eps);
    free(F);
}

void or_map2alm_m(int nside, int lmax, const double *map, int m, double *out_in)
{
    long npix = or_npix(nside);
    cplx *out = (cplx *)out_in;
    int nr = or_nrings(nside), nl = lmax - m + 1;
    double omega = 4.0 * M_PI / (double)npix;
    for (int k = 0; k < nl; k++)
        out[k] = 0;
#pragma omp parallel
    {
        double *lam = (double *)malloc(sizeof(double) * (lmax + 1));
        double *eps = (double *)malloc(sizeof(double) * (lmax + 1));
        cplx *acc = (cplx *)calloc(nl, sizeof(cplx));
        legendre_eps(lmax, m, eps);
#pragma omp for schedule(dynamic, 16)
        for (int i = 1; i <= nr; i++) {
            double z, sth, phi0;
            long start;
            int nphi;
            or_ring(nside, i, &z, &sth, &start, &nphi, &phi0);
            cplx g = 0;
            for (int j = 0; j < nphi; j++) {
                long mj = ((long)m * j) % nphi;
                double ang = -(double)m * phi0 - 2.0 * M_PI * (double)mj / (double)nphi;
                g += map[start + j] * (cos(ang) + I * sin(ang));
            }
            legendre_with_eps(lmax, m, z, sth, eps, lam);
            for (int l = m; l <= lmax; l++)
                acc[l - m] += lam[l - m] * g;
        }
#pragma omp critical
        for (int k = 0; k < nl; k++)
            out[k] += acc[k];
        free(lam);
        free(eps);
        free(acc);
    }
    for (int k = 0; k < nl; k++)
        out[k] *= omega;
}

void or_map2alm_pol_m(int nside, int lmax, const double *map, int m, double *out_in)
{
    long npix = or_npix(nside);
    cplx *out = (cplx *)out_in;
    int nr = or_nrings(nside), nl = lmax - m + 1;
    double omega = 4.0 * M_PI / (double)npix;
    for (int k = 0; k < 3 * nl; k++)
        out[k] = 0;
#pragma omp parallel
    {
        double *lam = (double *)malloc(sizeof(double) * (lmax + 1));
        double *eps = (double *)malloc(sizeof(double) * (lmax + 1));
        double *fp = (double *)malloc(sizeof(double) * (lmax + 1));
        double *fm = (double *)malloc(sizeof(double) * (lmax + 1));
        cplx *G = (cplx *)malloc(sizeof(cplx) * 3 * (lmax + 1));
        cplx *acc = (cplx *)calloc(3 * nl, sizeof(cplx));
        legendre_eps(lmax, m, eps);
#pragma omp for schedule(dynamic, 4)
        for (int i = 1; i <= nr; i++) {
            double z, sth, phi0;
            long start;
            int nphi;
            or_ring(nside, i, &z, &sth, &start, &nphi, &phi0);
            for (int c = 0; c < 3; c++)
                ring_analysis(lmax, nphi, phi0, map + c * npix + start, G + c * (lmax + 1), 0);
            legendre_with_eps(lmax, m, z, sth, eps, lam);
            or_spin2(lmax, m, z, sth, fp, fm);
            cplx gt = G[m], gq = G[lmax + 1 + m], gu = G[2 * (lmax + 1) + m];
            for (int l = m; l <= lmax; l++) {
                acc[l - m] += lam[l - m] * gt;
                acc[nl + l - m] += -(fp[l - m] * gq + I * fm[l - m] * gu);
                acc[2 * nl + l - m] += -(fp[l - m] * gu - I * fm[l - m] * gq);
            }
        }
#pragma omp critical
        for (int k = 0; k < 3 * nl; k++)
            out[k] += acc[k];
        free(lam);
        free(eps);
        free(fp);
        free(fm);
        free(G);
        free(acc);
    }
    for (int k = 0; k < 3 * nl; k++)
        out[k] *= omega;
}

/* ------------------------------------------------------------------------------------
 * Small dense linear algebra for the 3x3 blocks: Gaussian elimination with partial
 * pivoting (textbook), real and complex right-hand sides.  Returns 0, or -1 if singular.
 * ------------------------------------------------------------------------------------ */
static int solve3(const double Ain[9], const double bin[3], double x[3])
{
    double A[9], b[3];
    memcpy(A, Ain, sizeof A);
    memcpy(b, bin, sizeof b);
    for (int c = 0; c < 3; c++) {
        int piv = c;
        for (int r = c + 1; r < 3; r++)
            if (fabs(A[3 * r + c]) > fabs(A[3 * piv + c]))
                piv = r;
        if (A[3 * piv + c] == 0.0)
            return -1;
        if (piv != c) {
            for (int k = 0; k < 3; k++) {
                double t = A[3 * c + k];
                A[3 * c + k] = A[3 * piv + k];
                A[3 * piv + k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < 3; r++) {
            double f = A[3 * r + c] / A[3 * c + c];
            for (int k = c; k < 3; k++)
                A[3 * r + k] -= f * A[3 * c + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 2; r >= 0; r--) {
        double acc = b[r];
        for (int k = r + 1; k < 3; k++)
            acc -= A[3 * r + k] * x[k];
        x[r] = acc / A[3 * r + r];
    }
    return 0;
}

/* M_p packed (TT, TQ, TU, QQ, QU, UU) -> full 3x3 */
static void unpack6(const double *m6, double A[9])
{
    A[0] = m6[0]; A[1] = m6[1]; A[2] = m6[2];
    A[3] = m6[1]; A[4] = m6[3]; A[5] = m6[4];
    A[6] = m6[2]; A[7] = m6[4]; A[8] = m6[5];
}

/* S_l for (T, E, B): TT, EE, BB, TE from cl[4][lmax+1]; no TB, EB */
static void signal3(int lmax, const double *cl, int l, double S[9])
{
    double TT = cl[l], EE = cl[lmax + 1 + l], BB = cl[2 * (lmax + 1) + l], TE = cl[3 * (lmax + 1) + l];
    S[0] = TT; S[1] = TE; S[2] = 0.0;
    S[3] = TE; S[4] = EE; S[5] = 0.0;
    S[6] = 0.0; S[7] = 0.0; S[8] = BB;
}

/* x^T S^+ x over the components with positive power: the (T, E) block inverted where both
 * have power (else the one that has), B where BB > 0. */
static double quad_sinv(const double S[9], const double x[3])
{
    double acc = 0.0;
    double TT = S[0], EE = S[4], TE = S[1], BB = S[8];
    if (TT > 0.0 && EE > 0.0) {
        double det = TT * EE - TE * TE;
        acc += (EE * x[0] * x[0] - 2.0 * TE * x[0] * x[1] + TT * x[1] * x[1]) / det;
    } else if (TT > 0.0) {
        acc += x[0] * x[0] / TT;
    } else if (EE > 0.0) {
        acc += x[1] * x[1] / EE;
    }
    if (BB > 0.0)
        acc += x[2] * x[2] / BB;
    return acc;
}

/* ------------------------------------------------------------------------------------
 * Messenger iteration with T, Q, U (Sect. 2.1, Eqs. 3-4 with 3x3 blocks).
 *   M    [npix][6] packed N_p^{-1} (zero in masked pixels)
 *   cl   [4][lmax+1]: TT, EE, BB, TE
 *   rho  [3][npix], tau given (= 1 / max_p lambda_max(M_p))
 * Per pixel: t = [I + (lam-1) tau M]^{-1} [lam tau rho + (I - tau M) s]   (3x3 solve)
 * Per (l, m): s = S_l (S_l + lam tau Omega I)^{-1} a, i.e. s = S_l x with
 *             (S_l + lam tau Omega I) x = a   (real and imaginary parts separately).
 * diag per iteration: chi^2 = sum_lm w_m (s^T S^+ s) + sum_{p observed} q^T [M + (lam-1) tau M^2]^{-1} q
 * with q = rho - M s (observed: det M_p > 0), its harmonic part, |s_k - s_{k-1}|, |s_k|
 * (real harmonic dof of all three components).
 * ------------------------------------------------------------------------------------ */
int or_solve_pol(int nside, int lmax, const double *cl, const double *M, const double *rho,
                 double tau, int niter, const double *lam, int direct, double *s_alm_out,
                 double *s_map_out, double *diag)
{
    long npix = or_npix(nside), nalm = or_nalm(lmax);
    if (!(tau > 0.0))
        return -4;
    double omega = 4.0 * M_PI / (double)npix;
    double *s_map = (double *)calloc(3 * npix, sizeof(double));
    double *t = (double *)malloc(sizeof(double) * 3 * npix);
    cplx *a = (cplx *)malloc(sizeof(cplx) * 3 * nalm);
    cplx *s = (cplx *)calloc(3 * nalm, sizeof(cplx));
    cplx *s_old = (cplx *)calloc(3 * nalm, sizeof(cplx));
    int rc = 0;
    for (int k = 0; k < niter && rc == 0; k++) {
        double Lk = lam[k];
        for (long p = 0; p < npix; p++) {
            double Mp[9], A[9], b[3], x[3];
            unpack6(M + 6 * p, Mp);
            for (int i = 0; i < 3; i++) {
                double acc = Lk * tau * rho[i * npix + p] + s_map[i * npix + p];
                for (int j = 0; j < 3; j++) {
                    acc -= tau * Mp[3 * i + j] * s_map[j * npix + p];
                    A[3 * i + j] = (i == j ? 1.0 : 0.0) + (Lk - 1.0) * tau * Mp[3 * i + j];
                }
                b[i] = acc;
            }
            if (solve3(A, b, x) != 0)
                rc = -3;
            for (int i = 0; i < 3; i++)
                t[i * npix + p] = x[i];
        }
        or_map2alm_pol(nside, lmax, t, (double *)a, direct);
        memcpy(s_old, s, sizeof(cplx) * 3 * nalm);
        for (int l = 0; l <= lmax; l++) {
            double S[9], A[9];
            signal3(lmax, cl, l, S);
            for (int i = 0; i < 9; i++)
                A[i] = S[i] + ((i % 4 == 0) ? Lk * tau * omega : 0.0);
            for (int m = 0; m <= l; m++) {
                long i0 = aidx(lmax, l, m);
                double re[3], im[3], xr[3], xi[3];
                for (int c = 0; c < 3; c++) {
                    re[c] = creal(a[c * nalm + i0]);
                    im[c] = cimag(a[c * nalm + i0]);
                }
                solve3(A, re, xr);
                solve3(A, im, xi);
                for (int c = 0; c < 3; c++) {
                    double sr = 0.0, si = 0.0;
                    for (int j = 0; j < 3; j++) {
                        sr += S[3 * c + j] * xr[j];
                        si += S[3 * c + j] * xi[j];
                    }
                    s[c * nalm + i0] = sr + I * si;
                }
            }
        }
        or_alm2map_pol(nside, lmax, (const double *)s, s_map, direct);
        if (diag) {
            double harm = 0.0, pix = 0.0, dn = 0.0, sn = 0.0;
            for (int l = 0; l <= lmax; l++) {
                double S[9];
                signal3(lmax, cl, l, S);
                for (int m = 0; m <= l; m++) {
                    long i0 = aidx(lmax, l, m);
                    double w = (m == 0) ? 1.0 : 2.0, xr[3], xi[3];
                    for (int c = 0; c < 3; c++) {
                        cplx v = s[c * nalm + i0], d = v - s_old[c * nalm + i0];
                        xr[c] = creal(v);
                        xi[c] = cimag(v);
                        dn += w * creal(conj(d) * d);
                        sn += w * creal(conj(v) * v);
                    }
                    harm += w * (quad_sinv(S, xr) + quad_sinv(S, xi));
                }
            }
            for (long p = 0; p < npix; p++) {
                double Mp[9], B[9], q[3], y[3];
                unpack6(M + 6 * p, Mp);
                double det = Mp[0] * (Mp[4] * Mp[8] - Mp[5] * Mp[7]) - Mp[1] * (Mp[3] * Mp[8] - Mp[5] * Mp[6]) +
                             Mp[2] * (Mp[3] * Mp[7] - Mp[4] * Mp[6]);
                if (!(det > 0.0))
                    continue;
                for (int i = 0; i < 3; i++) {
                    double acc = rho[i * npix + p];
                    for (int j = 0; j < 3; j++) {
                        acc -= Mp[3 * i + j] * s_map[j * npix + p];
                        double m2 = 0.0;
                        for (int k2 = 0; k2 < 3; k2++)
                            m2 += Mp[3 * i + k2] * Mp[3 * k2 + j];
                        B[3 * i + j] = Mp[3 * i + j] + (Lk - 1.0) * tau * m2;
                    }
                    q[i] = acc;
                }
                solve3(B, q, y);
                pix += q[0] * y[0] + q[1] * y[1] + q[2] * y[2];
            }
            diag[4 * k + 0] = harm + pix;
            diag[4 * k + 1] = harm;
            diag[4 * k + 2] = sqrt(dn);
            diag[4 * k + 3] = sqrt(sn);
        }
    }
    if (s_alm_out)
        memcpy(s_alm_out, s, sizeof(cplx) * 3 * nalm);
    if (s_map_out)
        memcpy(s_map_out, s_map, sizeof(double) * 3 * npix);
    free(s_map);
    free(t);
    free(a);
    free(s);
    free(s_old);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * Fluctuation source with T, Q, U (Eq. 9 with blocks):
 *   rho = L_p g1 + Omega * Y_pol(K_l h),   M_p = L_p L_p^T (Cholesky; 0 in masked pixels),
 *   K_l = L_S^{-T} with S_l = L_S L_S^T over the components with positive power (so that
 *   K K^T = S_l^{-1} there), 0 elsewhere.
 * g1 [3][npix], h [3][nalm] complex unit-white.
 * ------------------------------------------------------------------------------------ */
static void chol3(const double A[9], double L[9])
{
    memset(L, 0, 9 * sizeof(double));
    for (int j = 0; j < 3; j++) {
        double d = A[3 * j + j];
        for (int k = 0; k < j; k++)
            d -= L[3 * j + k] * L[3 * j + k];
        if (!(d > 0.0))
            return; /* zero (masked) or non-definite block: remaining column stays 0 */
        L[3 * j + j] = sqrt(d);
        for (int i = j + 1; i < 3; i++) {
            double v = A[3 * i + j];
            for (int k = 0; k < j; k++)
                v -= L[3 * i + k] * L[3 * j + k];
            L[3 * i + j] = v / L[3 * j + j];
        }
    }
}

void or_fluct_rho_pol(int nside, int lmax, const double *cl, const double *M, const double *g1,
                      const double *h_in, double *rho, int direct)
{
    long npix = or_npix(nside), nalm = or_nalm(lmax);
    const cplx *h = (const cplx *)h_in;
    cplx *x = (cplx *)calloc(3 * nalm, sizeof(cplx));
    for (int l = 0; l <= lmax; l++) {
        double S[9];
        signal3(lmax, cl, l, S);
        /* K on the (T, E) block: positive-power components only */
        double TT = S[0], EE = S[4], TE = S[1], BB = S[8];
        double K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (TT > 0.0 && EE > 0.0) {
            /* S = L L^T, L = [[a, 0], [b, c]]; K = L^{-T} = [[1/a, -b/(a c)], [0, 1/c]] */
            double aa = sqrt(TT), bb = TE / aa, cc = sqrt(EE - bb * bb);
            K[0] = 1.0 / aa;
            K[1] = -bb / (aa * cc);
            K[4] = 1.0 / cc;
        } else if (TT > 0.0) {
            K[0] = 1.0 / sqrt(TT);
        } else if (EE > 0.0) {
            K[4] = 1.0 / sqrt(EE);
        }
        if (BB > 0.0)
            K[8] = 1.0 / sqrt(BB);
        for (int m = 0; m <= l; m++) {
            long i0 = aidx(lmax, l, m);
            for (int c = 0; c < 3; c++) {
                cplx acc = 0;
                for (int j = 0; j < 3; j++)
                    acc += K[3 * c + j] * h[j * nalm + i0];
                x[c * nalm + i0] = acc;
            }
        }
    }
    or_alm2map_pol(nside, lmax, (const double *)x, rho, direct);
    double omega = 4.0 * M_PI / (double)npix;
    for (long p = 0; p < npix; p++) {
        double Mp[9], L[9];
        unpack6(M + 6 * p, Mp);
        chol3(Mp, L);
        double v[3];
        for (int i = 0; i < 3; i++) {
            double acc = 0.0;
            for (int j = 0; j < 3; j++)
                acc += L[3 * i + j] * g1[j * npix + p];
            v[i] = acc;
        }
        for (int i = 0; i < 3; i++)
            rho[i * npix + p] = v[i] + omega * rho[i * npix + p];
    }
    free(x);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
