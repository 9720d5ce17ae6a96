// Ring phi steps of the SHT (Sect. 2.1 basis change; HEALPix rings, Gorski et al. 2005).
//
// One workgroup per (ring pair, map).  The north and south rings of a pair have the same
// length n and offset phi_0, so they travel together as one complex sequence
// x = t_N + i t_S and one length-n complex DFT serves both.
//
// Power-of-two n: in-LDS radix-2 transform.  The forward transform is decimation in
// frequency (natural order in, bit-reversed out), so no permutation pass is needed.
// Other n (polar rings n = 4i): Bluestein's chirp-z algorithm turns the length-n DFT into a
// circular convolution of power-of-two length M >= 2n - 1, done as DIF -> pointwise product
// with the precomputed transformed chirp (stored bit-reversed) -> DIT (bit-reversed in,
// natural out).  Twiddles come from one table of the largest length.
//
// Forward (analysis, a_lm side):  G_r(m) = sum_j t_{r,j} e^{-i m phi_{r,j}}, m = 0..lmax,
// read from DFT bin m mod n (phase e^{-i m phi_0}).  Inverse (synthesis): the harmonics
// F_r(m), m = -lmax..lmax with F(-m) = conj F(m), are folded into the n DFT bins and
// transformed back.  Layout of the ring-Fourier array: [map][m][ring] complex.
#include "mfwf_internal.h"

namespace mfwf {

static constexpr int kFFTThreads = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}

// Forward DFT, decimation in frequency, natural order in -> bit-reversed order out.
__device__ void fft_dif(double2 *buf, int len, const double2 *__restrict__ tw, int fftmax) {
    for (int span = len; span >= 2; span >>= 1) {
        const int half = span >> 1;
        const int tstride = fftmax / span;
        for (int b = threadIdx.x; b < (len >> 1); b += kFFTThreads) {
            const int grp = b / half, k = b - grp * half;
            const int i = grp * span + k, j = i + half;
            double2 u = buf[i], v = buf[j];
            buf[i] = cadd(u, v);
            buf[j] = cmul(csub(u, v), tw[k * tstride]);
        }
        __syncthreads();
    }
}

// Forward DFT, decimation in time, bit-reversed order in -> natural order out.
__device__ void fft_dit(double2 *buf, int len, const double2 *__restrict__ tw, int fftmax) {
    for (int span = 2; span <= len; span <<= 1) {
        const int half = span >> 1;
        const int tstride = fftmax / span;
        for (int b = threadIdx.x; b < (len >> 1); b += kFFTThreads) {
            const int grp = b / half, k = b - grp * half;
            const int i = grp * span + k, j = i + half;
            double2 u = buf[i], v = cmul(buf[j], tw[k * tstride]);
            buf[i] = cadd(u, v);
            buf[j] = csub(u, v);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bitrev(int k, int logn) {
    return logn == 0 ? 0 : (int)(__brev((unsigned)k) >> (32 - logn));
}

// Length-n forward DFT of buf[0..n) in place.  On return the transform value of bin k is
// read with dft_bin(): buf[bitrev(k)] for power-of-two n, c_k conj(buf[k]) for Bluestein.
__device__ void ring_dft(double2 *buf, const PairFFT &pf, const double2 *__restrict__ tw,
                         int fftmax, const double2 *__restrict__ chirp,
                         const double2 *__restrict__ bhat) {
    const int n = pf.nphi, M = pf.fftlen;
    if (!pf.bluestein) {
        fft_dif(buf, n, tw, fftmax);
        return;
    }
    const double2 *c = chirp + pf.chirp_off;
    for (int j = threadIdx.x; j < M; j += kFFTThreads)
        buf[j] = (j < n) ? cmul(buf[j], c[j]) : make_double2(0.0, 0.0);
    __syncthreads();
    fft_dif(buf, M, tw, fftmax);
    const double2 *bh = bhat + pf.bhat_off;  // bit-reversed, already divided by M
    for (int j = threadIdx.x; j < M; j += kFFTThreads) buf[j] = cconj(cmul(buf[j], bh[j]));
    __syncthreads();
    fft_dit(buf, M, tw, fftmax);
}

__device__ __forceinline__ double2 dft_bin(const double2 *buf, const PairFFT &pf, int logn,
                                           const double2 *__restrict__ chirp, int k) {
    if (!pf.bluestein) return buf[bitrev(k, logn)];
    return cmul(chirp[pf.chirp_off + k], cconj(buf[k]));
}

// e^{i m phi_0}: phi_0 = pi / n (half_shift) or 0
__device__ __forceinline__ double2 ring_phase(int m, int n, int half_shift) {
    if (!half_shift) return make_double2(1.0, 0.0);
    double s, c;
    sincospi((double)(m % (2 * n)) / (double)n, &s, &c);
    return make_double2(c, s);
}

__global__ void __launch_bounds__(kFFTThreads)
k_fft_fwd(const double *__restrict__ maps, double2 *__restrict__ phase,
          const PairFFT *__restrict__ pfft, const double2 *__restrict__ tw, int fftmax,
          const double2 *__restrict__ chirp, const double2 *__restrict__ bhat, long npix,
          int nring, int nm, int lmax) {
    extern __shared__ double2 buf[];
    const int p = blockIdx.x, b = blockIdx.y;
    const PairFFT pf = pfft[p];
    const int n = pf.nphi;
    const bool equator = (pf.startS == pf.startN);
    const double *tN = maps + (long)b * npix + pf.startN;
    const double *tS = maps + (long)b * npix + pf.startS;
    for (int j = threadIdx.x; j < n; j += kFFTThreads)
        buf[j] = make_double2(tN[j], equator ? 0.0 : tS[j]);
    __syncthreads();
    ring_dft(buf, pf, tw, fftmax, chirp, bhat);
    const int logn = 31 - __clz(n);
    const int rN = p, rS = nring - 1 - p;
    double2 *out = phase + (long)b * nm * nring;
    for (int m = threadIdx.x; m <= lmax; m += kFFTThreads) {
        const int k = m % n;
        const int kr = (n - k) % n;
        const double2 X = dft_bin(buf, pf, logn, chirp, k);
        const double2 Y = cconj(dft_bin(buf, pf, logn, chirp, kr));
        const double2 ph = cconj(ring_phase(m, n, pf.half_shift));
        // X_N = (X_k + conj X_{-k}) / 2,  X_S = (X_k - conj X_{-k}) / (2i)
        const double2 gN = make_double2(0.5 * (X.x + Y.x), 0.5 * (X.y + Y.y));
        out[(long)m * nring + rN] = cmul(gN, ph);
        if (!equator) {
            const double2 gS = make_double2(0.5 * (X.y - Y.y), -0.5 * (X.x - Y.x));
            out[(long)m * nring + rS] = cmul(gS, ph);
        }
    }
}

__global__ void __launch_bounds__(kFFTThreads)
k_fft_inv(const double2 *__restrict__ phase, double *__restrict__ maps,
          const PairFFT *__restrict__ pfft, const double2 *__restrict__ tw, int fftmax,
          const double2 *__restrict__ chirp, const double2 *__restrict__ bhat, long npix,
          int nring, int nm, int lmax) {
    extern __shared__ double2 buf[];
    __shared__ double2 partN[kFFTThreads], partS[kFFTThreads];
    const int p = blockIdx.x, b = blockIdx.y;
    const PairFFT pf = pfft[p];
    const int n = pf.nphi;
    const bool equator = (pf.startS == pf.startN);
    const int rN = p, rS = nring - 1 - p;
    const double2 *F = phase + (long)b * nm * nring;

    // Fold harmonics into bins: B(k) = sum_{m = k mod n} F(m) e^{i m phi0}
    //                                 + sum_{m >= 1, m = -k mod n} conj(F(m) e^{i m phi0}).
    // T threads per bin split the alias sum; partials are combined in a fixed order.
    int T = kFFTThreads / n;
    if (T < 1) T = 1;
    const int nbins_pass = kFFTThreads / T;  // bins handled per pass
    for (int k0 = 0; k0 < n; k0 += nbins_pass) {
        const int k = k0 + threadIdx.x / T, t = threadIdx.x % T;
        double2 sN = make_double2(0.0, 0.0), sS = make_double2(0.0, 0.0);
        if (k < n && (int)threadIdx.x < nbins_pass * T) {
            for (int m = k + t * n; m <= lmax; m += T * n) {
                const double2 ph = ring_phase(m, n, pf.half_shift);
                sN = cadd(sN, cmul(F[(long)m * nring + rN], ph));
                if (!equator) sS = cadd(sS, cmul(F[(long)m * nring + rS], ph));
            }
            const int mneg0 = (k == 0) ? n : n - k;
            for (int m = mneg0 + t * n; m <= lmax; m += T * n) {
                const double2 ph = ring_phase(m, n, pf.half_shift);
                sN = cadd(sN, cconj(cmul(F[(long)m * nring + rN], ph)));
                if (!equator) sS = cadd(sS, cconj(cmul(F[(long)m * nring + rS], ph)));
            }
        }
        if (T > 1) {
            partN[threadIdx.x] = sN;
            partS[threadIdx.x] = sS;
            __syncthreads();
            if (t == 0 && k < n) {
                for (int u = 1; u < T; u++) {
                    sN = cadd(sN, partN[threadIdx.x + u]);
                    sS = cadd(sS, partS[threadIdx.x + u]);
                }
            }
            __syncthreads();
        }
        // x_j = sum_k X_k e^{+2 pi i j k/n} = conj(DFT(conj X))_j with X = B_N + i B_S
        if (t == 0 && k < n) buf[k] = cconj(make_double2(sN.x - sS.y, sN.y + sS.x));
    }
    __syncthreads();
    ring_dft(buf, pf, tw, fftmax, chirp, bhat);
    const int logn = 31 - __clz(n);
    double *sNmap = maps + (long)b * npix + pf.startN;
    double *sSmap = maps + (long)b * npix + pf.startS;
    for (int j = threadIdx.x; j < n; j += kFFTThreads) {
        const double2 x = cconj(dft_bin(buf, pf, logn, chirp, j));
        sNmap[j] = x.x;
        if (!equator) sSmap[j] = x.y;
    }
}

int launch_fft_fwd(const Plan &p, const double *maps, double2 *phase, int nb) {
    size_t lds = sizeof(double2) * (size_t)p.fftmax;
    hipLaunchKernelGGL(k_fft_fwd, dim3(p.npair, nb), dim3(kFFTThreads), lds, p.stream, maps,
                       phase, p.d_pfft, p.d_tw, p.fftmax, p.d_chirp, p.d_bhat, p.npix, p.nring,
                       p.nm, p.lmax);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_fft_inv(const Plan &p, const double2 *phase, double *maps, int nb) {
    size_t lds = sizeof(double2) * (size_t)p.fftmax;
    hipLaunchKernelGGL(k_fft_inv, dim3(p.npair, nb), dim3(kFFTThreads), lds, p.stream, phase,
                       maps, p.d_pfft, p.d_tw, p.fftmax, p.d_chirp, p.d_bhat, p.npix, p.nring,
                       p.nm, p.lmax);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// Maximum dynamic LDS the FFT kernels may request (set once per process).
int fft_set_lds_limit(size_t bytes) {
    MFWF_HIP(hipFuncSetAttribute((const void *)k_fft_fwd,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    MFWF_HIP(hipFuncSetAttribute((const void *)k_fft_inv,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return MFWF_OK;
}

}  // namespace mfwf
