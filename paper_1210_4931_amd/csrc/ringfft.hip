// Ring phi steps of the SHT (Sect. 2.1 basis change; HEALPix rings, Gorski et al. 2005).
//
// One workgroup per (map, ring pair).  The north and south rings of a pair have the same
// length n and offset phi_0, so they travel together as one complex sequence
// x = t_N + i t_S and one length-n complex DFT serves both.
//
// Power-of-two n: in-LDS self-sorting (Stockham) transform with radix-8 passes (a final
// radix-4 or radix-2 pass when needed): each thread keeps its butterflies' inputs in
// registers across a barrier, so the passes run in place in one LDS buffer, and the output
// is in natural order.  Other n (polar rings n = 4i): Bluestein's chirp-z algorithm turns
// the length-n DFT into a circular convolution of power-of-two length M >= 2n - 1 (forward
// transform, pointwise product with the precomputed transformed chirp, and a second forward
// transform of the conjugate).  Twiddles come from a two-level table held in LDS.
//
// Forward (analysis side):  G_r(m) = sum_j t_{r,j} e^{-i m phi_{r,j}}, m = 0..lmax, read
// from DFT bin k = m mod n.  Inverse (synthesis): F_r(m), m = -lmax..lmax with
// F(-m) = conj F(m), folded into the n bins and transformed back.  With phi_0 = pi/n
// ("half shift"), e^{i m phi_0} = e^{i pi k / n} (-1)^q for m = k + q n, so each bin needs one
// phase factor and its aliases only a sign.
//
// Ring-Fourier layout: [map][ring][m] complex, so both kernels stream contiguous rows; the
// values are FP64 (per-map path) or FP32 (batched form, which rounds once on the way to the
// FP32 contractions; the transforms themselves always run in FP64).  The forward transform
// can apply the messenger pixel update (Eq. 3) to its input as it reads it.
// Grid (map, pair): the workgroups of one ring pair run back to back, so the pair's chirp
// tables and noise precision are fetched into L2 once for all maps.
// Pairs are launched in classes by transform length: most pairs need at most half the
// largest length (less LDS and fewer registers per thread, more workgroups per CU); the long
// Bluestein transforms of the largest polar rings form the second class; polar rings whose
// chirp-z transform would outgrow LDS (nside 2048) form a third, split into four shorter
// transforms (below).
#include <mutex>
#include <type_traits>

#include "fft_core.h"
#include "sym3.h"

namespace mfwf {

__device__ __forceinline__ void put_c(double2 *q, double2 v) { *q = v; }
__device__ __forceinline__ void put_c(float2 *q, double2 v) { *q = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double2 get_c(const double2 *q) { return *q; }
__device__ __forceinline__ double2 get_c(const float2 *q) {
    const float2 v = *q;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ double2 get_v(const double2 &v) { return v; }
__device__ __forceinline__ double2 get_v(const float2 &v) { return make_double2(v.x, v.y); }

// Eq. (3) at one pixel: t = [lam tau rho + (1 - tau M) s] / [1 + (lam - 1) tau M] with
// lt = lam tau, l1t = (lam - 1) tau.  Every product-sum is an explicit fma, so that each
// kernel that forms t (the forward transforms with the update fused, the chained ring step,
// the split transforms) rounds it alike whatever the compiler contracts around it.
__device__ __forceinline__ double messenger_pixel(double s, double m, double r, double lam,
                                                  double lt, double l1t, double tau) {
    const double num = fma(fma(-tau, m, 1.0), s, lt * r);
    return (lam == 1.0) ? num : num / fma(l1t, m, 1.0);
}

// The coefficients m = 0, 1, ... of one ring: a row (consecutive) or a column of the
// matrix-core layout [m][ring][C2] (stride cs elements).
template <typename T, bool STRIDED>
struct RingSeq {
    T *p;
    long cs;
    __device__ __forceinline__ T &operator[](int m) const { return p[STRIDED ? (long)m * cs : m]; }
};

// Ring-Fourier rows of a transformed pair: G_r(m) = sum_j t_{r,j} e^{-i m phi_{r,j}}, m = 0..lmax,
// for the north ring (outN) and, off the equator, the south ring (outS), from the DFT of
// x = t_N + i t_S in buf.
template <int TPB, typename OutT, bool STRIDED = false>
__device__ __forceinline__ void store_rows(const double2 *buf, const PairFFT &pf,
                                           const Twiddles &tw, int fftmax,
                                           const double2 *__restrict__ chirp, int lmax,
                                           RingSeq<OutT, STRIDED> outN, RingSeq<OutT, STRIDED> outS) {
    const int n = pf.nphi, tid = threadIdx.x & (TPB - 1);
    const bool equator = (pf.startS == pf.startN);
    // e^{-i m phi0} = e^{-i pi m / n} with a half shift: from the twiddle table when it holds
    // the 2n-th roots, else from the thread's first m by steps of e^{-i pi TPB / n} (a few
    // steps, a few ulp)
    const bool tab = fftmax % (2 * n) == 0;
    double2 phm = make_double2(1.0, 0.0), phstep = make_double2(1.0, 0.0);
    if (pf.half_shift && !tab) {
        double sn, cs;
        sincospi((double)tid / (double)n, &sn, &cs);
        phm = make_double2(cs, -sn);
        sincospi((double)TPB / (double)n, &sn, &cs);
        phstep = make_double2(cs, -sn);
    }
    for (int m = tid; m <= lmax; m += TPB) {
        const int q = (n > lmax) ? 0 : m / n, k = m - q * n;  // no alias when n > lmax
        const int kr = (k == 0) ? 0 : n - k;
        const double2 X = dft_bin(buf, pf, chirp, k);
        const double2 Y = cconj(dft_bin(buf, pf, chirp, kr));
        // e^{-i m phi0} = (-1)^q e^{-i pi k / n} with a half shift, 1 otherwise
        double2 ph = make_double2(1.0, 0.0);
        if (pf.half_shift) {
            if (tab) {
                ph = cscale(cconj(half_bin_phase(k, n, tw, fftmax)), (q & 1) ? -1.0 : 1.0);
            } else {
                ph = phm;
                phm = cmul(phm, phstep);
            }
        }
        // X_N = (X_k + conj X_{-k}) / 2,  X_S = (X_k - conj X_{-k}) / (2i)
        const double2 gN = make_double2(0.5 * (X.x + Y.x), 0.5 * (X.y + Y.y));
        put_c(&outN[m], cmul(gN, ph));
        if (!equator) {
            const double2 gS = make_double2(0.5 * (X.y - Y.y), -0.5 * (X.x - Y.x));
            put_c(&outS[m], cmul(gS, ph));
        }
    }
}

// Forward transform of maps[b] (PIX = false) or of the messenger field of Eq. (3),
// t = [lam tau rho + (1 - tau M) s] / [1 + (lam - 1) tau M], with s = maps[b], rho = rho[b].
template <int TPB, int EPT, typename OutT, bool PIX>
__global__ void __launch_bounds__(TPB)
k_fft_fwd(const double *__restrict__ maps, const double *__restrict__ rho,
          const double *__restrict__ M, double lam, double tau, long mstride,
          const double *__restrict__ tau_b, OutT *__restrict__ phase,
          const PairFFT *__restrict__ pfft, const int *__restrict__ plist,
          const double2 *__restrict__ twlo, const double2 *__restrict__ twhi, int ntwhi,
          int fftmax, const double2 *__restrict__ chirp, const double2 *__restrict__ bhat,
          long npix, int nring, int nm, int lmax, int fftlen_class) {
    extern __shared__ double2 buf[];
    const int p = plist[blockIdx.y], b = blockIdx.x;
    const PairFFT pf = pfft[p];
    const int n = pf.nphi;
    const bool equator = (pf.startS == pf.startN);
    const Twiddles tw = load_twiddles(buf, fft_area(fftlen_class, TPB), twlo, twhi, ntwhi);
    if (PIX && tau_b) tau = tau_b[b];  // per-map tau and M rows (serving slots)
    const double lt = lam * tau, l1t = (lam - 1.0) * tau;
    // Every class has n <= EPT * TPB, so each thread reads at most EPT pixels of each ring.
    // All of them are loaded (clamped to the ring, so every address is valid) before any is
    // used: one memory latency per workgroup instead of one per pixel row.
    const double *sp = maps + (long)b * npix;
    const double *rp = rho + (long)b * npix;
    const double *mp = M + (long)b * mstride;
    double xN[EPT], xS[EPT], mN[EPT], mS[EPT], rN[EPT], rS[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        const int j = min((int)threadIdx.x + u * TPB, n - 1);
        xN[u] = sp[pf.startN + j];
        xS[u] = sp[pf.startS + j];
        if constexpr (PIX) {
            mN[u] = mp[pf.startN + j];
            mS[u] = mp[pf.startS + j];
            rN[u] = rp[pf.startN + j];
            rS[u] = rp[pf.startS + j];
        }
    }
    auto pix = [&](double x, double m, double r) {
        if constexpr (!PIX) {
            return x;
        } else {
            return messenger_pixel(x, m, r, lam, lt, l1t, tau);
        }
    };
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        const int j = threadIdx.x + u * TPB;
        if (j < n)
            buf[lds_ix(j)] = make_double2(pix(xN[u], mN[u], rN[u]), equator ? 0.0 : pix(xS[u], mS[u], rS[u]));
    }
    __syncthreads();
    ring_dft_c<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
    store_rows<TPB>(buf, pf, tw, fftmax, chirp, lmax,
                    RingSeq<OutT, false>{phase + ((long)b * nring + p) * nm, 1},
                    RingSeq<OutT, false>{phase + ((long)b * nring + (nring - 1 - p)) * nm, 1});
}

// Fold the ring-Fourier rows FN, FS of a pair into the bins of its inverse transform, in
// LDS (x_j = sum_k X_k e^{+2 pi i j k / n} is then conj(DFT(conj X))_j with X = B_N + i B_S).
template <int TPB, int EPT, typename Seq>
__device__ __forceinline__ void fold_bins(double2 *buf, Seq FN, Seq FS, const PairFFT &pf,
                                          const Twiddles &tw, int fftmax, int lmax) {
    using InT = std::remove_cv_t<std::remove_reference_t<decltype(FN[0])>>;
    const int n = pf.nphi, tid = threadIdx.x & (TPB - 1);
    const bool equator = (pf.startS == pf.startN);
    // alias-sum partials, used only with T > 1, i.e. n <= TPB / 2: after element TPB / 2
    double2 *partN = buf + lds_ix(TPB / 2);
    double2 *partS = partN + TPB;
    // Fold harmonics into bins: S(k) = sum_q sgn_q F(k + q n) over |k + q n| <= lmax with
    // F(-m) = conj F(m) and sgn_q = (-1)^q under a half shift; then B(k) = e^{i pi k/n} S(k).
    // T threads per bin split the alias sum; partials are combined in a fixed order.
    int T = TPB / n;
    if (T < 1) T = 1;
    const int nbins_pass = TPB / T;
    const double sgn_step = pf.half_shift ? -1.0 : 1.0;
    const double sg_stride = (T & 1) ? sgn_step : 1.0;
    if (n > lmax) {
        // n > lmax: a bin k has at most two aliases, m = k (k <= lmax) and m = -(n - k)
        // (n - k <= lmax), so the sum is made from the coefficients themselves, each read
        // once (in the matrix-core columns a coefficient costs a cache line of its own):
        // thread i reads m = i + u TPB, stores the positive term of bin m (zero for bins
        // above lmax), then after a barrier adds the negative term to bin n - m.  The bin's
        // phase and the packing x = conj(ph (B_N + i B_S)) are linear, so each term is packed
        // on its own.
        constexpr int MU = EPT;  // coefficients per thread per ring (lmax < n <= EPT TPB)
        InT fN[MU], fS[MU];
#pragma unroll
        for (int u = 0; u < MU; u++) {
            if (u * TPB > lmax) break;  // uniform
            const int m = min(tid + u * TPB, lmax);
            fN[u] = FN[m];
            fS[u] = FS[m];
        }
        auto term = [&](double2 gN, double2 gS, double2 ph) {
            if (equator) gS = make_double2(0.0, 0.0);
            if (pf.half_shift) {
                gN = cmul(gN, ph);
                gS = cmul(gS, ph);
            }
            return cconj(make_double2(gN.x - gS.y, gN.y + gS.x));
        };
        // bin phases e^{i pi m / n} of the thread's m (table, or steps of e^{i pi TPB / n}
        // from its first m); bin n - m has e^{i pi (n - m) / n} = -conj(e^{i pi m / n})
        const bool tab = fftmax % (2 * n) == 0;
        double2 ph[MU], phm = make_double2(1.0, 0.0), phstep = make_double2(1.0, 0.0);
        if (pf.half_shift && !tab) {
            double sn, cs;
            sincospi((double)tid / (double)n, &sn, &cs);
            phm = make_double2(cs, sn);
            sincospi((double)TPB / (double)n, &sn, &cs);
            phstep = make_double2(cs, sn);
        }
#pragma unroll
        for (int u = 0; u < MU; u++) {
            ph[u] = make_double2(1.0, 0.0);
            if (pf.half_shift) {
                if (tab) {
                    ph[u] = half_bin_phase(min(tid + u * TPB, n - 1), n, tw, fftmax);
                } else {
                    ph[u] = phm;
                    phm = cmul(phm, phstep);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < EPT; u++) {
            const int k = tid + u * TPB;
            if (k < n)
                buf[lds_ix(k)] = (k <= lmax) ? term(get_c(&fN[u]), get_c(&fS[u]), ph[u]) : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < MU; u++) {
            const int m = tid + u * TPB;
            if (m >= 1 && m <= lmax) {  // negative alias of bin n - m: sgn conj F(m)
                const int k = n - m;
                const double2 x = term(cscale(cconj(get_c(&fN[u])), sgn_step),
                                       cscale(cconj(get_c(&fS[u])), sgn_step),
                                       make_double2(-ph[u].x, ph[u].y));
                buf[lds_ix(k)] = cadd(buf[lds_ix(k)], x);
            }
        }
        return;
    }
    if (T == 1) {
        // n > TPB / 2: thread i folds bins k = i + u TPB (n <= EPT * TPB).  The first
        // positive alias (m = k) and the first negative one (m = k - n, read as conj F(n - k))
        // of every bin, the only ones when n > lmax, are loaded together (clamped addresses,
        // values selected); further aliases (rings with n <= lmax) are added after them in
        // alias order.
        // bins in flight per thread: FP64 input holds 4 (16 registers each), FP32 input 8
        constexpr int CH = sizeof(InT) == sizeof(double2) ? 4 : 8;
        const double2 zero = make_double2(0.0, 0.0);
#pragma unroll
        for (int u0 = 0; u0 < EPT; u0 += CH) {
            if (u0 * TPB >= n) break;  // uniform: no bins from here on
            InT aN[CH], aS[CH], cN[CH], cS[CH];
#pragma unroll
            for (int v = 0; v < CH; v++) {
                if ((u0 + v) * TPB >= n) break;  // uniform
                const int kc = min(tid + (u0 + v) * TPB, n - 1);
                const int mpos = min(kc, lmax), mneg = min(n - kc, lmax);
                aN[v] = FN[mpos];
                aS[v] = FS[mpos];
                cN[v] = FN[mneg];
                cS[v] = FS[mneg];
            }
#pragma unroll
            for (int v = 0; v < CH; v++) {
                const int k = tid + (u0 + v) * TPB;
                if (k >= n) continue;
                const bool vp = k <= lmax, vn = n - k <= lmax;
                double2 sN = cadd(vp ? get_c(&aN[v]) : zero, vn ? cscale(cconj(get_c(&cN[v])), sgn_step) : zero);
                double2 sS = cadd(vp ? get_c(&aS[v]) : zero, vn ? cscale(cconj(get_c(&cS[v])), sgn_step) : zero);
                if (n <= lmax) {
                    double sg = sgn_step;
                    for (int m = k + n; m <= lmax; m += n, sg *= sgn_step) {
                        sN = cadd(sN, cscale(get_v(FN[m]), sg));
                        sS = cadd(sS, cscale(get_v(FS[m]), sg));
                    }
                    sg = 1.0;  // sgn_step^2
                    for (int mm = 2 * n - k; mm <= lmax; mm += n) {
                        sN = cadd(sN, cscale(cconj(get_v(FN[mm])), sg));
                        sS = cadd(sS, cscale(cconj(get_v(FS[mm])), sg));
                        sg *= sgn_step;
                    }
                }
                if (equator) sS = zero;
                if (pf.half_shift) {
                    const double2 ph = half_bin_phase(k, n, tw, fftmax);
                    sN = cmul(sN, ph);
                    sS = cmul(sS, ph);
                }
                buf[lds_ix(k)] = cconj(make_double2(sN.x - sS.y, sN.y + sS.x));
            }
        }
    }
    for (int k0 = 0; T > 1 && k0 < n; k0 += nbins_pass) {
        const int k = k0 + tid / T, t = tid % T;
        double2 sN = make_double2(0.0, 0.0), sS = make_double2(0.0, 0.0);
        if (k < n && tid < nbins_pass * T) {
            // m = k + q n >= 0, q = t, t + T, ...
            double sg = (t & 1) ? sgn_step : 1.0;
            for (int m = k + t * n; m <= lmax; m += T * n, sg *= sg_stride) {
                sN = cadd(sN, cscale(get_v(FN[m]), sg));
                if (!equator) sS = cadd(sS, cscale(get_v(FS[m]), sg));
            }
            // m = k + q n < 0, q = -1 - t, -1 - t - T, ...: F(m) = conj F(-m)
            sg = ((t + 1) & 1) ? sgn_step : 1.0;
            for (int mm = (t + 1) * n - k; mm <= lmax; mm += T * n, sg *= sg_stride) {
                sN = cadd(sN, cscale(cconj(get_v(FN[mm])), sg));
                if (!equator) sS = cadd(sS, cscale(cconj(get_v(FS[mm])), sg));
            }
        }
        if (T > 1) {
            partN[tid] = sN;
            partS[tid] = sS;
            __syncthreads();
            if (t == 0 && k < n) {
                for (int u = 1; u < T; u++) {
                    sN = cadd(sN, partN[tid + u]);
                    sS = cadd(sS, partS[tid + u]);
                }
            }
            __syncthreads();
        }
        if (t == 0 && k < n) {
            if (pf.half_shift) {
                const double2 ph = half_bin_phase(k, n, tw, fftmax);
                sN = cmul(sN, ph);
                sS = cmul(sS, ph);
            }
            // x_j = sum_k X_k e^{+2 pi i j k/n} = conj(DFT(conj X))_j with X = B_N + i B_S
            buf[lds_ix(k)] = cconj(make_double2(sN.x - sS.y, sN.y + sS.x));
        }
    }
}

template <int TPB, int EPT, typename InT>
__global__ void __launch_bounds__(TPB)
k_fft_inv(const InT *__restrict__ phase, double *__restrict__ maps,
          const PairFFT *__restrict__ pfft, const int *__restrict__ plist,
          const double2 *__restrict__ twlo, const double2 *__restrict__ twhi, int ntwhi,
          int fftmax, const double2 *__restrict__ chirp, const double2 *__restrict__ bhat,
          long npix, int nring, int nm, int lmax, int fftlen_class) {
    extern __shared__ double2 buf[];
    const int p = plist[blockIdx.y], b = blockIdx.x;
    const PairFFT pf = pfft[p];
    const int n = pf.nphi;
    const bool equator = (pf.startS == pf.startN);
    const Twiddles tw = load_twiddles(buf, fft_area(fftlen_class, TPB), twlo, twhi, ntwhi);
    const RingSeq<const InT, false> FN{phase + ((long)b * nring + p) * nm, 1};
    const RingSeq<const InT, false> FS{phase + ((long)b * nring + (nring - 1 - p)) * nm, 1};
    fold_bins<TPB, EPT>(buf, FN, FS, pf, tw, fftmax, lmax);
    __syncthreads();
    ring_dft_c<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
    double *sNmap = maps + (long)b * npix + pf.startN;
    double *sSmap = maps + (long)b * npix + pf.startS;
    for (int j = threadIdx.x; j < n; j += TPB) {
        const double2 x = cconj(dft_bin(buf, pf, chirp, j));
        sNmap[j] = x.x;
        if (!equator) sSmap[j] = x.y;
    }
}

// Split rings: a polar ring n = 4 i whose chirp-z transform would not fit LDS.  Decimation
// in time splits its DFT into four of length i,
//   X_k = sum_{r < 4} e^{-2 pi i r k / n} Z_r(k mod i),   Z_r = DFT_i(x_{4 j + r}),
// each Z_r a Bluestein transform of length i, one workgroup each (k_fft_split_sub).  The
// sub-spectra wait in global scratch, one area of 2 n elements per (row, pair): [0, n) holds
// the folded bins of an inverse transform, [n, 2 n) the four sub-spectra Z[r i + k].
// Forward: k_fft_split_sub from the pixels, then k_fft_fwd_split_combine (combined spectrum
// in LDS, rows stored as in k_fft_fwd).  Inverse: k_fft_inv_split_fold (bins folded as in
// k_fft_inv), k_fft_split_sub from those bins, k_fft_inv_split_combine to the pixels.

// Z_r of one (row, pair, r): grid (row, pair of the class, r); FROM_MAP: x = t_N + i t_S from
// maps (PIX: t the messenger field of Eq. (3) formed from s = maps, rho and M, as k_fft_fwd
// forms it), else x = the folded bins in the scratch area
template <int TPB, int EPT, bool FROM_MAP, bool PIX = false>
__global__ void __launch_bounds__(TPB)
k_fft_split_sub(const double *__restrict__ maps, double2 *__restrict__ scratch, long sstride,
                int sub_area, const PairFFT *__restrict__ pfft, const int *__restrict__ plist,
                const double2 *__restrict__ twlo, const double2 *__restrict__ twhi, int ntwhi,
                int fftmax, const double2 *__restrict__ chirp, const double2 *__restrict__ bhat,
                long npix, const double *__restrict__ rho = nullptr,
                const double *__restrict__ M = nullptr, double lam = 1.0, double tau = 0.0,
                long mstride = 0, const double *__restrict__ tau_b = nullptr) {
    extern __shared__ double2 buf[];
    const int p = plist[blockIdx.y], b = blockIdx.x, r = blockIdx.z;
    const PairFFT pf = pfft[p];
    PairFFT sub = pf;
    sub.nphi = pf.nphi / 4;
    sub.bluestein = 1;
    const int n = pf.nphi, i = sub.nphi;
    const bool equator = (pf.startS == pf.startN);
    const Twiddles tw = load_twiddles(buf, sub_area, twlo, twhi, ntwhi);
    double2 *G = scratch + ((long)b * gridDim.y + blockIdx.y) * sstride;
    double2 *Z = G + sstride / 2 + (long)r * i;
    const double *sp = maps + (long)b * npix;
    if (PIX && tau_b) tau = tau_b[b];
    const double lt = lam * tau, l1t = (lam - 1.0) * tau;
    const double *rp = rho + (long)b * npix;
    const double *mp = M + (long)b * mstride;
    auto pix = [&](long q) {
        if constexpr (!PIX) {
            return sp[q];
        } else {
            return messenger_pixel(sp[q], mp[q], rp[q], lam, lt, l1t, tau);
        }
    };
    for (int j = threadIdx.x; j < i; j += TPB) {
        const int jj = 4 * j + r;
        if constexpr (FROM_MAP)
            buf[lds_ix(j)] = make_double2(pix(pf.startN + jj), equator ? 0.0 : pix(pf.startS + jj));
        else
            buf[lds_ix(j)] = G[jj];
    }
    __syncthreads();
    ring_dft<TPB, EPT>(buf, sub, tw, fftmax, chirp, bhat);
    for (int k = threadIdx.x; k < i; k += TPB) Z[k] = dft_bin(buf, sub, chirp, k);
    (void)n;
}

// X_k from the sub-spectra Z for k = threadIdx.x, +TPB, ... < n; f(k, X_k)
template <int TPB, typename F>
__device__ __forceinline__ void split_combine(const double2 *Z, int n, F f) {
    const int i = n / 4;
    for (int k = threadIdx.x; k < n; k += TPB) {
        const int kk = k - (k / i) * i;
        double sn, cs;  // w = e^{-2 pi i k / n}; w^2, w^3 as products (a few ulp)
        sincospi(2.0 * (double)k / (double)n, &sn, &cs);
        const double2 w1 = make_double2(cs, -sn), w2 = cmul(w1, w1), w3 = cmul(w2, w1);
        double2 X = cadd(Z[kk], cmul(w1, Z[i + kk]));
        X = cadd(X, cmul(w2, Z[2 * i + kk]));
        X = cadd(X, cmul(w3, Z[3 * i + kk]));
        f(k, X);
    }
}

// forward, second step: the combined spectrum in LDS, stored as ring-Fourier rows
// ([row][ring][nm]) or, COLS, into the matrix-core columns ([m][ring][C2], map b at 2b)
template <int TPB, int EPT, typename OutT, bool COLS = false>
__global__ void __launch_bounds__(TPB)
k_fft_fwd_split_combine(OutT *__restrict__ phase, const double2 *__restrict__ scratch,
                        long sstride, const PairFFT *__restrict__ pfft,
                        const int *__restrict__ plist, const double2 *__restrict__ twlo,
                        const double2 *__restrict__ twhi, int ntwhi, int fftmax,
                        const double2 *__restrict__ chirp, const double2 *__restrict__ bhat,
                        long npix, int nring, int nm, int lmax, int fftlen_class, int C2 = 0) {
    extern __shared__ double2 buf[];
    const int p = plist[blockIdx.y], b = blockIdx.x;
    PairFFT pf = pfft[p];
    const Twiddles tw = load_twiddles(buf, fft_area(fftlen_class, TPB), twlo, twhi, ntwhi);
    const double2 *Z = scratch + ((long)b * gridDim.y + blockIdx.y) * sstride + sstride / 2;
    split_combine<TPB>(Z, pf.nphi, [&](int k, double2 X) { buf[lds_ix(k)] = X; });
    __syncthreads();
    pf.bluestein = 0;  // the spectrum sits in LDS in natural order
    if constexpr (COLS) {
        const long cs = (long)nring * (C2 / 2);
        store_rows<TPB>(buf, pf, tw, fftmax, chirp, lmax,
                        RingSeq<OutT, true>{phase + (long)p * (C2 / 2) + b, cs},
                        RingSeq<OutT, true>{phase + (long)(nring - 1 - p) * (C2 / 2) + b, cs});
    } else {
        store_rows<TPB>(buf, pf, tw, fftmax, chirp, lmax,
                        RingSeq<OutT, false>{phase + ((long)b * nring + p) * nm, 1},
                        RingSeq<OutT, false>{phase + ((long)b * nring + (nring - 1 - p)) * nm, 1});
    }
    (void)bhat;
    (void)npix;
}

// inverse, first step: the folded bins (as k_fft_inv leaves them before its transform) to
// the scratch area
template <int TPB, int EPT, typename InT, bool COLS = false>
__global__ void __launch_bounds__(TPB)
k_fft_inv_split_fold(const InT *__restrict__ phase, double2 *__restrict__ scratch, long sstride,
                     const PairFFT *__restrict__ pfft, const int *__restrict__ plist,
                     const double2 *__restrict__ twlo, const double2 *__restrict__ twhi,
                     int ntwhi, int fftmax, const double2 *__restrict__ chirp,
                     const double2 *__restrict__ bhat, long npix, int nring, int nm, int lmax,
                     int fftlen_class, int C2 = 0) {
    extern __shared__ double2 buf[];
    const int p = plist[blockIdx.y], b = blockIdx.x;
    const PairFFT pf = pfft[p];
    const Twiddles tw = load_twiddles(buf, fft_area(fftlen_class, TPB), twlo, twhi, ntwhi);
    if constexpr (COLS) {  // the matrix-core columns [m][ring][C2], map b at 2b
        const long cs = (long)nring * (C2 / 2);
        fold_bins<TPB, EPT>(buf, RingSeq<const InT, true>{phase + (long)p * (C2 / 2) + b, cs},
                            RingSeq<const InT, true>{phase + (long)(nring - 1 - p) * (C2 / 2) + b, cs},
                            pf, tw, fftmax, lmax);
    } else {
        const RingSeq<const InT, false> FN{phase + ((long)b * nring + p) * nm, 1};
        const RingSeq<const InT, false> FS{phase + ((long)b * nring + (nring - 1 - p)) * nm, 1};
        fold_bins<TPB, EPT>(buf, FN, FS, pf, tw, fftmax, lmax);
    }
    __syncthreads();
    double2 *G = scratch + ((long)b * gridDim.y + blockIdx.y) * sstride;
    for (int j = threadIdx.x; j < pf.nphi; j += TPB) G[j] = buf[lds_ix(j)];
    (void)chirp;
    (void)bhat;
    (void)npix;
}

// inverse, last step: pixel k of the pair = conj(X_k)
template <int TPB>
__global__ void __launch_bounds__(TPB)
k_fft_inv_split_combine(double *__restrict__ maps, const double2 *__restrict__ scratch,
                        long sstride, const PairFFT *__restrict__ pfft,
                        const int *__restrict__ plist, long npix) {
    const int p = plist[blockIdx.y], b = blockIdx.x;
    const PairFFT pf = pfft[p];
    const bool equator = (pf.startS == pf.startN);
    const double2 *Z = scratch + ((long)b * gridDim.y + blockIdx.y) * sstride + sstride / 2;
    double *sNmap = maps + (long)b * npix + pf.startN;
    double *sSmap = maps + (long)b * npix + pf.startS;
    split_combine<TPB>(Z, pf.nphi, [&](int k, double2 X) {
        sNmap[k] = X.x;
        if (!equator) sSmap[k] = -X.y;
    });
}

// One iteration's ring steps in one pass over a pair (batched FP32 form), on the
// matrix-core columns [m][ring][C2] (map b at column 2b) in place: the synthesis F is folded
// and transformed back to the pair's pixels s (optionally stored to smap), the messenger
// field t of Eq. (3) is formed from s, rho and M on the spot, and its transform overwrites
// the columns with G = the analysis input.  The map s never travels through memory; the
// arithmetic is that of k_fft_inv followed by k_fft_fwd<PIX>, value for value.
//
// A workgroup takes G maps b0 .. b0 + G - 1 of one pair (G groups of TPB threads, one
// transform each in its own LDS area): the column entries of those maps for one (m, ring)
// are adjacent (8 G bytes), so the fold of the rings longer than lmax and the stores of the
// analysis input move them with one vector access per (m, ring) instead of G separate
// 8-byte pieces of one cache line from G workgroups.  The 1-D grid (workgroup L runs on XCD
// L mod 8) hands every XCD whole pairs, all map groups of a pair in a row, so that the
// groups sharing a 128-byte column segment meet in one L2.

// e^{s i pi (tid + u' TPB) / n}, u' = sub + u G, as the per-map code forms it: a sincospi of
// tid / n times u' steps of e^{s i pi TPB / n}, multiplied in order
template <int TPB, int G>
struct PhaseChain {
    double2 cur, step;
    __device__ __forceinline__ PhaseChain(int tid, int sub, int n, double sign) {
        double sn, cs;
        sincospi((double)tid / (double)n, &sn, &cs);
        cur = make_double2(cs, sign * sn);
        sincospi((double)TPB / (double)n, &sn, &cs);
        step = make_double2(cs, sign * sn);
        for (int k = 0; k < sub; k++) cur = cmul(cur, step);  // wave-uniform count
    }
    __device__ __forceinline__ double2 next() {  // value for u, then advance to u + 1
        const double2 v = cur;
#pragma unroll
        for (int k = 0; k < G; k++) cur = cmul(cur, step);
        return v;
    }
};

template <int G>
__device__ __forceinline__ void load_g(const float2 *p, float2 (&v)[G]) {
    if constexpr (G == 1) {
        v[0] = *p;
    } else {
#pragma unroll
        for (int h = 0; h < G / 2; h++) {
            const float4 q = reinterpret_cast<const float4 *>(p)[h];
            v[2 * h] = make_float2(q.x, q.y);
            v[2 * h + 1] = make_float2(q.z, q.w);
        }
    }
}

template <int G>
__device__ __forceinline__ void store_g(float2 *p, const float2 (&v)[G]) {
    if constexpr (G == 1) {
        *p = v[0];
    } else {
#pragma unroll
        for (int h = 0; h < G / 2; h++)
            reinterpret_cast<float4 *>(p)[h] = make_float4(v[2 * h].x, v[2 * h].y, v[2 * h + 1].x, v[2 * h + 1].y);
    }
}

// fold_bins for rings longer than lmax, for the G transforms of the workgroup at once
// (buf + s area for map s): a thread reads the G maps' coefficients of its m together
template <int TPB, int EPT, int G>
__device__ __forceinline__ void fold_cols_group(double2 *buf, int area, const float2 *FN,
                                                const float2 *FS, long cs, const PairFFT &pf,
                                                const Twiddles &tw, int fftmax, int lmax) {
    constexpr int MU = (EPT + G - 1) / G;  // bins per thread (n <= EPT TPB)
    const int n = pf.nphi, tid = threadIdx.x & (TPB - 1), sub = threadIdx.x / TPB;
    const bool equator = (pf.startS == pf.startN);
    const double sgn_step = pf.half_shift ? -1.0 : 1.0;
    float2 fN[MU][G], fS[MU][G];
#pragma unroll
    for (int u = 0; u < MU; u++) {
        if (u * G * TPB > lmax) break;  // uniform: no thread has a coefficient from here on
        const int m = min((int)threadIdx.x + u * G * TPB, lmax);
        load_g<G>(FN + (long)m * cs, fN[u]);
        load_g<G>(FS + (long)m * cs, fS[u]);
    }
    auto term = [&](double2 gN, double2 gS, double2 ph) {
        if (equator) gS = make_double2(0.0, 0.0);
        if (pf.half_shift) {
            gN = cmul(gN, ph);
            gS = cmul(gS, ph);
        }
        return cconj(make_double2(gN.x - gS.y, gN.y + gS.x));
    };
    const bool tab = fftmax % (2 * n) == 0;
    double2 ph[MU];
    if (pf.half_shift && !tab) {
        PhaseChain<TPB, G> chain(tid, sub, n, 1.0);
#pragma unroll
        for (int u = 0; u < MU; u++) ph[u] = chain.next();
    } else {
#pragma unroll
        for (int u = 0; u < MU; u++)
            ph[u] = pf.half_shift ? half_bin_phase(min((int)threadIdx.x + u * G * TPB, n - 1), n, tw, fftmax)
                                  : make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < MU; u++) {
        const int k = threadIdx.x + u * G * TPB;
        if (k < n) {
#pragma unroll
            for (int s = 0; s < G; s++)
                buf[s * area + lds_ix(k)] =
                    (k <= lmax) ? term(get_c(&fN[u][s]), get_c(&fS[u][s]), ph[u]) : make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MU; u++) {
        const int m = threadIdx.x + u * G * TPB;
        if (m >= 1 && m <= lmax) {  // negative alias of bin n - m: sgn conj F(m)
            const int k = n - m;
#pragma unroll
            for (int s = 0; s < G; s++) {
                const double2 x = term(cscale(cconj(get_c(&fN[u][s])), sgn_step),
                                       cscale(cconj(get_c(&fS[u][s])), sgn_step),
                                       make_double2(-ph[u].x, ph[u].y));
                buf[s * area + lds_ix(k)] = cadd(buf[s * area + lds_ix(k)], x);
            }
        }
    }
}

// store_rows for the G transforms of the workgroup, into the columns (G maps adjacent)
template <int TPB, int G>
__device__ __forceinline__ void store_cols_group(const double2 *buf, int area, const PairFFT &pf,
                                                 const Twiddles &tw, int fftmax,
                                                 const double2 *__restrict__ chirp, int lmax,
                                                 float2 *outN, float2 *outS, long cs) {
    const int n = pf.nphi, tid = threadIdx.x & (TPB - 1), sub = threadIdx.x / TPB;
    const bool equator = (pf.startS == pf.startN);
    const bool tab = fftmax % (2 * n) == 0;
    PhaseChain<TPB, G> chain(tid, sub, n, -1.0);  // used only with a half shift and !tab
    for (int m = threadIdx.x; m <= lmax; m += G * TPB) {
        const int q = (n > lmax) ? 0 : m / n, k = m - q * n;  // no alias when n > lmax
        const int kr = (k == 0) ? 0 : n - k;
        double2 ph = make_double2(1.0, 0.0);
        if (pf.half_shift) {
            if (tab) {
                ph = cscale(cconj(half_bin_phase(k, n, tw, fftmax)), (q & 1) ? -1.0 : 1.0);
            } else {
                ph = chain.next();
            }
        }
        double2 ck = make_double2(1.0, 0.0), ckr = ck;
        if (pf.bluestein) {
            ck = chirp[pf.chirp_off + k];
            ckr = chirp[pf.chirp_off + kr];
        }
        float2 vN[G], vS[G];
#pragma unroll
        for (int s = 0; s < G; s++) {
            const double2 bk = buf[s * area + lds_ix(k)], bkr = buf[s * area + lds_ix(kr)];
            const double2 X = pf.bluestein ? cmul(ck, cconj(bk)) : bk;
            const double2 Y = cconj(pf.bluestein ? cmul(ckr, cconj(bkr)) : bkr);
            // X_N = (X_k + conj X_{-k}) / 2,  X_S = (X_k - conj X_{-k}) / (2i)
            const double2 gN = make_double2(0.5 * (X.x + Y.x), 0.5 * (X.y + Y.y));
            const double2 gS = make_double2(0.5 * (X.y - Y.y), -0.5 * (X.x - Y.x));
            put_c(&vN[s], cmul(gN, ph));
            put_c(&vS[s], cmul(gS, ph));
        }
        store_g<G>(outN + (long)m * cs, vN);
        if (!equator) store_g<G>(outS + (long)m * cs, vS);
    }
}

template <int TPB, int EPT, int G>
__global__ void __launch_bounds__(TPB * G)
k_fft_inv_fwd(float2 *__restrict__ data, int C2, int nmap, int ngrp, int npl, double *__restrict__ smap,
              const double *__restrict__ rho, const double *__restrict__ M, double lam,
              double tau, long mstride, const double *__restrict__ tau_b,
              const PairFFT *__restrict__ pfft, const int *__restrict__ plist,
              const double2 *__restrict__ twlo, const double2 *__restrict__ twhi, int ntwhi,
              int fftmax, const double2 *__restrict__ chirp, const double2 *__restrict__ bhat,
              long npix, int nring, int nm, int lmax, int fftlen_class) {
    extern __shared__ double2 lds[];
    const int L = blockIdx.x, x = L & 7, sl = L >> 3, j = sl / ngrp;
    const int g = sl - j * ngrp, pi = 8 * j + x;
    if (pi >= npl) return;  // whole workgroup, before any barrier
    const int p = plist[pi];
    const PairFFT pf = pfft[p];
    const int n = pf.nphi;
    const bool equator = (pf.startS == pf.startN);
    const int area = fft_area(fftlen_class, TPB);
    const Twiddles tw = load_twiddles(lds, G * area, twlo, twhi, ntwhi);
    const int sub = threadIdx.x / TPB, tid = threadIdx.x & (TPB - 1);
    double2 *buf = lds + sub * area;
    const int b0 = g * G, b = b0 + sub;
    const bool live = b < nmap;  // maps past the batch: zero columns, no pixel arrays
    const int pS = nring - 1 - p;
    const long cs = (long)nring * (C2 / 2);  // float2 elements from m to m + 1
    float2 *FN = data + (long)p * (C2 / 2) + b0;
    float2 *FS = data + (long)pS * (C2 / 2) + b0;
    if (n > lmax) {
        fold_cols_group<TPB, EPT, G>(lds, area, FN, FS, cs, pf, tw, fftmax, lmax);
    } else {
        fold_bins<TPB, EPT>(buf, RingSeq<const float2, true>{FN + sub, cs},
                            RingSeq<const float2, true>{FS + sub, cs}, pf, tw, fftmax, lmax);
    }
    __syncthreads();
    ring_dft_c<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
    if (tau_b && live) tau = tau_b[b];
    const double lt = lam * tau, l1t = (lam - 1.0) * tau;
    const double *rp = rho + (long)b * npix;
    const double *mp = M + (long)b * mstride;
    double mN[EPT], mS[EPT], rN[EPT], rS[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        if (u * TPB >= n) break;  // uniform: the ring's pixels end here
        const int jj = min(tid + u * TPB, n - 1);
        mN[u] = live ? mp[pf.startN + jj] : 0.0;
        mS[u] = live ? mp[pf.startS + jj] : 0.0;
        rN[u] = live ? rp[pf.startN + jj] : 0.0;
        rS[u] = live ? rp[pf.startS + jj] : 0.0;
    }
    auto pix = [&](double xx, double m, double r) {
        return messenger_pixel(xx, m, r, lam, lt, l1t, tau);
    };
    double2 v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        if (u * TPB >= n) break;
        const int jj = tid + u * TPB;
        const double2 xs = cconj(dft_bin(buf, pf, chirp, min(jj, n - 1)));  // (s_N, s_S) at jj
        if (smap && live && jj < n) {
            smap[(long)b * npix + pf.startN + jj] = xs.x;
            if (!equator) smap[(long)b * npix + pf.startS + jj] = xs.y;
        }
        v[u] = make_double2(pix(xs.x, mN[u], rN[u]), equator ? 0.0 : pix(xs.y, mS[u], rS[u]));
    }
    __syncthreads();  // every read of the inverse transform is done
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        const int jj = tid + u * TPB;
        if (jj < n) buf[lds_ix(jj)] = v[u];
    }
    __syncthreads();
    ring_dft_c<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
    store_cols_group<TPB, G>(lds, area, pf, tw, fftmax, chirp, lmax, FN, FS, cs);
}

// One T, Q, U iteration's ring steps in one pass over a pair and map b (batched FP32 form),
// on the matrix-core columns: T [m][ring][C2] (map b at float2 b) and (Q, U) [m][ring][2 C2]
// (map b at float2 2b, 2b + 1).  The synthesis (T, Q, U) is folded and transformed back to
// the pair's pixels one component at a time, the three s values of each pixel kept in
// registers; the 3x3 messenger update of Eq. (3) forms t; each component of t is transformed
// forward and overwrites its columns with the analysis input.  The arithmetic is that of the
// regrouping into rows, k_fft_inv, k_pixel_update_pol and k_fft_fwd, value for value.  One
// transform area of LDS; TPB <= 512 (registers).
template <int TPB, int EPT>
__global__ void __launch_bounds__(TPB)
k_fft_inv_fwd_pol(float *__restrict__ colT, float *__restrict__ colP, int C2, int nmap, int npl, const double *__restrict__ rho,
                  const double *__restrict__ M6, double lam, double tau,
                  const PairFFT *__restrict__ pfft, const int *__restrict__ plist,
                  const double2 *__restrict__ twlo, const double2 *__restrict__ twhi, int ntwhi,
                  int fftmax, const double2 *__restrict__ chirp, const double2 *__restrict__ bhat,
                  long npix, int nring, int nm, int lmax, int fftlen_class) {
    extern __shared__ double2 lds[];
    const int L = blockIdx.x, x = L & 7, sl = L >> 3, j = sl / nmap;
    const int b = sl - j * nmap, pi = 8 * j + x;
    if (pi >= npl) return;  // whole workgroup, before any barrier
    const int p = plist[pi];
    const PairFFT pf = pfft[p];
    const int n = pf.nphi, tid = threadIdx.x;
    const bool equator = (pf.startS == pf.startN);
    const Twiddles tw = load_twiddles(lds, fft_area(fftlen_class, TPB), twlo, twhi, ntwhi);
    double2 *buf = lds;
    const int pS = nring - 1 - p;
    const long csT = (long)nring * (C2 / 2), csP = (long)nring * C2;  // float2 per step of m
    float2 *TN = reinterpret_cast<float2 *>(colT) + (long)p * (C2 / 2) + b;
    float2 *TS = reinterpret_cast<float2 *>(colT) + (long)pS * (C2 / 2) + b;
    float2 *QN = reinterpret_cast<float2 *>(colP) + (long)p * C2 + 2 * b;
    float2 *QS = reinterpret_cast<float2 *>(colP) + (long)pS * C2 + 2 * b;
    // (s_N, s_S) of the thread's pixels per component, then (t_N, t_S)
    double2 sT[EPT], sQ[EPT], sU[EPT];
    auto inverse = [&](RingSeq<const float2, true> FN, RingSeq<const float2, true> FS,
                       double2 (&sv)[EPT]) __attribute__((always_inline)) {
        fold_bins<TPB, EPT>(buf, FN, FS, pf, tw, fftmax, lmax);
        __syncthreads();
        ring_dft_c<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
#pragma unroll
        for (int u = 0; u < EPT; u++) sv[u] = cconj(dft_bin(buf, pf, chirp, min(tid + u * TPB, n - 1)));
        __syncthreads();  // every read of this component's transform is done
    };
    inverse(RingSeq<const float2, true>{TN, csT}, RingSeq<const float2, true>{TS, csT}, sT);
    inverse(RingSeq<const float2, true>{QN, csP}, RingSeq<const float2, true>{QS, csP}, sQ);
    inverse(RingSeq<const float2, true>{QN + 1, csP}, RingSeq<const float2, true>{QS + 1, csP}, sU);
    const double lt = lam * tau, l1t = (lam - 1.0) * tau;
    const double *rp = rho + 3L * b * npix;
#pragma unroll
    for (int u = 0; u < EPT; u++) {
        const int jj = tid + u * TPB;
        if (jj >= n) continue;
        {
            const long q = pf.startN + jj;
            const double s3[3] = {sT[u].x, sQ[u].x, sU[u].x};
            const double r3[3] = {rp[q], rp[q + npix], rp[q + 2 * npix]};
            double t3[3];
            pol_messenger_pixel(load_sym3(M6, q), s3, r3, lam, lt, l1t, tau, t3);
            sT[u].x = t3[0];
            sQ[u].x = t3[1];
            sU[u].x = t3[2];
        }
        if (!equator) {
            const long q = pf.startS + jj;
            const double s3[3] = {sT[u].y, sQ[u].y, sU[u].y};
            const double r3[3] = {rp[q], rp[q + npix], rp[q + 2 * npix]};
            double t3[3];
            pol_messenger_pixel(load_sym3(M6, q), s3, r3, lam, lt, l1t, tau, t3);
            sT[u].y = t3[0];
            sQ[u].y = t3[1];
            sU[u].y = t3[2];
        }
    }
    auto forward = [&](const double2 (&tv)[EPT], RingSeq<float2, true> GN, RingSeq<float2, true> GS)
                       __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < EPT; u++) {
            const int jj = tid + u * TPB;
            if (jj < n) buf[lds_ix(jj)] = make_double2(tv[u].x, equator ? 0.0 : tv[u].y);
        }
        __syncthreads();
        ring_dft_c<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
        store_rows<TPB>(buf, pf, tw, fftmax, chirp, lmax, GN, GS);
        __syncthreads();  // every read of this transform is done before the next is written
    };
    forward(sT, RingSeq<float2, true>{TN, csT}, RingSeq<float2, true>{TS, csT});
    forward(sQ, RingSeq<float2, true>{QN, csP}, RingSeq<float2, true>{QS, csP});
    forward(sU, RingSeq<float2, true>{QN + 1, csP}, RingSeq<float2, true>{QS + 1, csP});
    (void)nm;
}

// Largest number of maps per workgroup of the columns ring step for class c: as many
// transforms as fit one CU's LDS and 1024 threads, at most 4, no more than the batch needs.
int fft_cols_group_max(const Plan &p, int c, int nb) {
    int ept;
    const int tpb = fft_class_shape(p, c, ept);
    const size_t area = sizeof(double2) * fft_area(p.fft_class_len[c], tpb);
    const size_t tw = sizeof(double2) * (64 + p.fft_ntwhi);
    int g = 1;
    while (2 * g <= 4 && 2 * g * tpb <= 1024 && 2 * g * area + tw <= 160 * 1024 && g < nb) g *= 2;
    return g;
}

// Maps per workgroup used: the plan's (tuned) choice, within what this batch allows.
int fft_cols_group(const Plan &p, int c, int nb) {
    const int gmax = fft_cols_group_max(p, c, nb);
    int g = 1;
    while (2 * g <= gmax && 2 * g <= p.ring_group[c]) g *= 2;
    return g;
}

size_t fft_cols_lds(const Plan &p, int c, int g) {
    int ept;
    const int tpb = fft_class_shape(p, c, ept);
    return sizeof(double2) * ((size_t)g * fft_area(p.fft_class_len[c], tpb) + 64 + p.fft_ntwhi);
}

// (threads per workgroup, elements per thread) of a class: 8 elements (one radix-8
// butterfly per pass) per thread and as many threads as the length needs, so that a
// workgroup of a long class still brings 8 to 16 waves.
int fft_class_shape(const Plan &p, int c, int &ept) {
    const int len = p.fft_class_len[c];
    ept = 8;
    if (c == 2) return 1024;  // split rings: up to 8192 points in LDS at any plan size
    return len <= 2048 ? 256 : len / 8;
}

size_t fft_class_lds(const Plan &p, int c) {
    int ept;
    const int tpb = fft_class_shape(p, c, ept);
    return sizeof(double2) * ((size_t)fft_area(p.fft_class_len[c], tpb) + 64 + p.fft_ntwhi);
}

// rs: row stride of the ring-Fourier rows (nm for the FP64 rows, nm32 for the FP32 rows)
#define MFWF_FFT_ARGS(c, rs)                                                                    \
    p.d_pfft, p.d_plist + p.fft_class_off[c], p.d_twlo, p.d_twhi, p.fft_ntwhi, p.fftmax,        \
        p.d_chirp, p.d_bhat, p.npix, p.nring, rs, p.lmax, p.fft_class_len[c]

// split rings (class 2): FP64 rows, FP32 rows, or the matrix-core columns of the FP32 form
static constexpr int kSplitSubTPB = 512, kSplitTPB = 1024;

static int split_check(const Plan &p, int nb) {
    if (nb > p.fftsplit_rows)
        return fail(MFWF_EINVAL, "split ring transforms of " + std::to_string(nb) +
                                     " rows: the plan holds scratch for " +
                                     std::to_string(p.fftsplit_rows));
    int ept;
    if (fft_class_shape(p, 2, ept) != kSplitTPB || p.fftsplit_sublen > kSplitSubTPB * 8)
        return fail(MFWF_EINVAL, "split ring class shape");
    return MFWF_OK;
}

static size_t split_sub_lds(const Plan &p) {
    return sizeof(double2) * ((size_t)fft_area(p.fftsplit_sublen, kSplitSubTPB) + 64 + p.fft_ntwhi);
}

template <bool FROM_MAP, bool PIX = false>
static int split_sub(const Plan &p, const double *maps, int nb, const double *rho = nullptr,
                     double lam = 1.0) {
    const int cnt = p.fft_class_count[2];
    hipLaunchKernelGGL((k_fft_split_sub<kSplitSubTPB, 8, FROM_MAP, PIX>), dim3(nb, cnt, 4),
                       dim3(kSplitSubTPB), split_sub_lds(p), p.stream, maps, p.d_fftsplit,
                       p.fftsplit_stride, fft_area(p.fftsplit_sublen, kSplitSubTPB), p.d_pfft,
                       p.d_plist + p.fft_class_off[2], p.d_twlo, p.d_twhi, p.fft_ntwhi, p.fftmax,
                       p.d_chirp, p.d_bhat, p.npix, rho, p.d_M, lam, p.tau, p.mstride, p.d_tau);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// forward split transforms of nb maps (PIX: of the messenger field formed from maps, rho and
// M) into rows of OutT (row stride rs) or, COLS, into the matrix-core columns
template <typename OutT, bool PIX, bool COLS>
static int fwd_split(const Plan &p, const double *maps, const double *rho, double lam, OutT *out,
                     int rs, int nb) {
    MFWF_TRY(split_check(p, nb));
    MFWF_TRY((split_sub<true, PIX>(p, maps, nb, rho, lam)));
    hipLaunchKernelGGL((k_fft_fwd_split_combine<kSplitTPB, 8, OutT, COLS>),
                       dim3(nb, p.fft_class_count[2]), dim3(kSplitTPB), fft_class_lds(p, 2),
                       p.stream, out, p.d_fftsplit, p.fftsplit_stride, MFWF_FFT_ARGS(2, rs), p.C2);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

template <typename InT, bool COLS>
static int inv_split(const Plan &p, const InT *in, int rs, double *maps, int nb) {
    MFWF_TRY(split_check(p, nb));
    hipLaunchKernelGGL((k_fft_inv_split_fold<kSplitTPB, 8, InT, COLS>),
                       dim3(nb, p.fft_class_count[2]), dim3(kSplitTPB), fft_class_lds(p, 2),
                       p.stream, in, p.d_fftsplit, p.fftsplit_stride, MFWF_FFT_ARGS(2, rs), p.C2);
    MFWF_HIP(hipGetLastError());
    MFWF_TRY(split_sub<false>(p, nullptr, nb));
    hipLaunchKernelGGL((k_fft_inv_split_combine<256>), dim3(nb, p.fft_class_count[2]), dim3(256),
                       0, p.stream, maps, p.d_fftsplit, p.fftsplit_stride, p.d_pfft,
                       p.d_plist + p.fft_class_off[2], p.npix);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

template <typename OutT, bool PIX>
static int fwd_classes(const Plan &p, const double *maps, const double *rho, double lam,
                       OutT *out, int nb) {
    if (p.fft_class_count[2] > 0)
        MFWF_TRY((fwd_split<OutT, PIX, false>(p, maps, rho, lam, out,
                                              sizeof(OutT) == sizeof(float2) ? p.nm32 : p.nm, nb)));
    for (int c = 1; c >= 0; c--) {  // long transforms first
        const int cnt = p.fft_class_count[c];
        if (cnt == 0) continue;
        int ept;
        const int tpb = fft_class_shape(p, c, ept);
        const dim3 grid(nb, cnt);  // maps of one pair adjacent: its tables and M stay in L2
        const size_t lds = fft_class_lds(p, c);
        const int rs = sizeof(OutT) == sizeof(float2) ? p.nm32 : p.nm;
        if (tpb == 256)
            hipLaunchKernelGGL((k_fft_fwd<256, 8, OutT, PIX>), grid, dim3(256), lds, p.stream, maps, rho, p.d_M, lam, p.tau, p.mstride, p.d_tau, out, MFWF_FFT_ARGS(c, rs));
        else if (tpb == 512)
            hipLaunchKernelGGL((k_fft_fwd<512, 8, OutT, PIX>), grid, dim3(512), lds, p.stream, maps, rho, p.d_M, lam, p.tau, p.mstride, p.d_tau, out, MFWF_FFT_ARGS(c, rs));
        else
            hipLaunchKernelGGL((k_fft_fwd<1024, 8, OutT, PIX>), grid, dim3(1024), lds, p.stream, maps, rho, p.d_M, lam, p.tau, p.mstride, p.d_tau, out, MFWF_FFT_ARGS(c, rs));
        MFWF_HIP(hipGetLastError());
    }
    return MFWF_OK;
}

template <typename InT>
static int inv_classes(const Plan &p, const InT *in, double *maps, int nb) {
    if (p.fft_class_count[2] > 0)
        MFWF_TRY((inv_split<InT, false>(p, in, sizeof(InT) == sizeof(float2) ? p.nm32 : p.nm, maps, nb)));
    for (int c = 1; c >= 0; c--) {
        const int cnt = p.fft_class_count[c];
        if (cnt == 0) continue;
        int ept;
        const int tpb = fft_class_shape(p, c, ept);
        const dim3 grid(nb, cnt);  // maps of one pair adjacent: its tables and M stay in L2
        const size_t lds = fft_class_lds(p, c);
        const int rs = sizeof(InT) == sizeof(float2) ? p.nm32 : p.nm;
        if (tpb == 256)
            hipLaunchKernelGGL((k_fft_inv<256, 8, InT>), grid, dim3(256), lds, p.stream, in, maps, MFWF_FFT_ARGS(c, rs));
        else if (tpb == 512)
            hipLaunchKernelGGL((k_fft_inv<512, 8, InT>), grid, dim3(512), lds, p.stream, in, maps, MFWF_FFT_ARGS(c, rs));
        else
            hipLaunchKernelGGL((k_fft_inv<1024, 8, InT>), grid, dim3(1024), lds, p.stream, in, maps, MFWF_FFT_ARGS(c, rs));
        MFWF_HIP(hipGetLastError());
    }
    return MFWF_OK;
}

int launch_fft_fwd(const Plan &p, const double *maps, double2 *phase, int nb) {
    return fwd_classes<double2, false>(p, maps, nullptr, 1.0, phase, nb);
}

int launch_fft_fwd_pix(const Plan &p, const double *maps, const double *rho, double lam,
                       double2 *phase, int nb) {
    return fwd_classes<double2, true>(p, maps, rho, lam, phase, nb);
}

int launch_fft_fwd_f32(const Plan &p, const double *maps, const double *rho, double lam,
                       float2 *phase, int nb) {
    if (rho) return fwd_classes<float2, true>(p, maps, rho, lam, phase, nb);
    return fwd_classes<float2, false>(p, maps, nullptr, 1.0, phase, nb);
}

int launch_fft_inv(const Plan &p, const double2 *phase, double *maps, int nb) {
    return inv_classes<double2>(p, phase, maps, nb);
}

int launch_fft_inv_f32(const Plan &p, const float2 *phase, double *maps, int nb) {
    return inv_classes<float2>(p, phase, maps, nb);
}

int ring_fork(const Plan &p) {
    if (!p.side) return MFWF_OK;
    MFWF_HIP(hipEventRecord(p.side_fork, p.stream));
    MFWF_HIP(hipStreamWaitEvent(p.side, p.side_fork, 0));
    return MFWF_OK;
}

int ring_join(const Plan &p) {
    if (!p.side) return MFWF_OK;
    MFWF_HIP(hipEventRecord(p.side_join, p.side));
    MFWF_HIP(hipStreamWaitEvent(p.stream, p.side_join, 0));
    return MFWF_OK;
}

int launch_fft_inv_fwd_cols(const Plan &p, const double *rho, double lam, double *smap, int nb) {
    if (p.fft_class_count[2] > 0) {
        // split rings (nside 2048): the synthesis columns folded and transformed back to the
        // pixels of those rings (into smap, or the plan's map workspace t), then the
        // messenger field's split transforms into the columns
        float2 *data = reinterpret_cast<float2 *>(p.d_ph32);
        double *maps = smap ? smap : p.d_t;
        MFWF_TRY((inv_split<float2, true>(p, data, p.nm32, maps, nb)));
        MFWF_TRY((fwd_split<float2, true, true>(p, maps, rho, lam, data, p.nm32, nb)));
    }
    MFWF_TRY(ring_fork(p));  // class 1 on the side stream, class 0 on the plan's stream
    for (int c = 1; c >= 0; c--) {
        const int cnt = p.fft_class_count[c];
        if (cnt == 0) continue;
        const hipStream_t st = (c == 1 && p.side) ? p.side : p.stream;
        int ept;
        const int tpb = fft_class_shape(p, c, ept);
        const int g = fft_cols_group(p, c, nb);
        const int ngrp = (nb + g - 1) / g;
        const dim3 grid(8 * ngrp * ((cnt + 7) / 8));  // whole pairs per XCD
        const size_t lds = fft_cols_lds(p, c, g);
        const int rs = p.nm32;  // unused by the kernel (no rows)
        float2 *data = reinterpret_cast<float2 *>(p.d_ph32);
#define MFWF_INVFWD(T, G)                                                                           \
    hipLaunchKernelGGL((k_fft_inv_fwd<T, 8, G>), grid, dim3(T * G), lds, st, data, p.C2, nb,        \
                       ngrp, cnt, smap, rho, p.d_M, lam, p.tau, p.mstride, p.d_tau, MFWF_FFT_ARGS(c, rs))
        if (tpb == 256 && g == 4) MFWF_INVFWD(256, 4);
        else if (tpb == 256 && g == 2) MFWF_INVFWD(256, 2);
        else if (tpb == 256) MFWF_INVFWD(256, 1);
        else if (tpb == 512 && g == 2) MFWF_INVFWD(512, 2);
        else if (tpb == 512) MFWF_INVFWD(512, 1);
        else MFWF_INVFWD(1024, 1);
#undef MFWF_INVFWD
        MFWF_HIP(hipGetLastError());
    }
    return ring_join(p);
}



// The chained T, Q, U ring step runs where every ring class fits its register budget
// (workgroups of at most 512 threads) and no ring needs the split transforms.
bool fft_pol_chain_ok(const Plan &p) {
    if (p.fft_class_count[2] > 0) return false;
    for (int c = 0; c < 2; c++) {
        int ept;
        if (p.fft_class_count[c] > 0 && fft_class_shape(p, c, ept) > 512) return false;
    }
    return true;
}

int launch_fft_inv_fwd_pol_cols(const Plan &p, const double *rho, double lam, int nb) {
    if (!fft_pol_chain_ok(p)) return fail(MFWF_EINVAL, "chained T, Q, U ring step: ring class too long");
    MFWF_TRY(ring_fork(p));  // class 1 on the side stream, class 0 on the plan's stream
    for (int c = 1; c >= 0; c--) {
        const int cnt = p.fft_class_count[c];
        if (cnt == 0) continue;
        const hipStream_t st = (c == 1 && p.side) ? p.side : p.stream;
        int ept;
        const int tpb = fft_class_shape(p, c, ept);
        const dim3 grid(8 * nb * ((cnt + 7) / 8));  // whole pairs per XCD
        const size_t lds = fft_cols_lds(p, c, 1);
#define MFWF_INVFWD_POL(T)                                                                          \
    hipLaunchKernelGGL((k_fft_inv_fwd_pol<T, 8>), grid, dim3(T), lds, st, p.d_ph32, p.d_ph32p,       \
                       p.C2, nb, cnt, rho, p.d_M, lam, p.tau, MFWF_FFT_ARGS(c, p.nm32))
        if (tpb == 256) MFWF_INVFWD_POL(256);
        else MFWF_INVFWD_POL(512);
#undef MFWF_INVFWD_POL
        MFWF_HIP(hipGetLastError());
    }
    return ring_join(p);
}

int fft_max_length() { return 8 * 1024; }

// Maximum dynamic LDS the FFT kernels may request (set once per process).
template <typename OutT, bool PIX>
static int fwd_lds(int bytes) {
    const void *fns[] = {(const void *)k_fft_fwd<256, 8, OutT, PIX>,
                         (const void *)k_fft_fwd<512, 8, OutT, PIX>,
                         (const void *)k_fft_fwd<1024, 8, OutT, PIX>};
    for (const void *f : fns)
        MFWF_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    return MFWF_OK;
}
static int inv_fwd_lds(int bytes) {
    const void *fns[] = {(const void *)k_fft_inv_fwd<256, 8, 1>, (const void *)k_fft_inv_fwd<256, 8, 2>,
                         (const void *)k_fft_inv_fwd<256, 8, 4>, (const void *)k_fft_inv_fwd<512, 8, 1>,
                         (const void *)k_fft_inv_fwd<512, 8, 2>, (const void *)k_fft_inv_fwd<1024, 8, 1>};
    for (const void *f : fns)
        MFWF_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    return MFWF_OK;
}
template <typename InT>
static int inv_lds(int bytes) {
    const void *fns[] = {(const void *)k_fft_inv<256, 8, InT>, (const void *)k_fft_inv<512, 8, InT>,
                         (const void *)k_fft_inv<1024, 8, InT>};
    for (const void *f : fns)
        MFWF_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    return MFWF_OK;
}

// The attribute belongs to the kernel functions, so it is shared by every plan in the
// process: it only ever rises, so that a plan created later with shorter transforms cannot
// lower it below what an existing plan's launches ask for.
int fft_set_lds_limit(size_t bytes) {
    static std::mutex mu;
    static size_t current = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (bytes <= current) return MFWF_OK;
    current = bytes;
    MFWF_TRY((fwd_lds<double2, false>((int)bytes)));
    MFWF_TRY((fwd_lds<double2, true>((int)bytes)));
    MFWF_TRY((fwd_lds<float2, false>((int)bytes)));
    MFWF_TRY((fwd_lds<float2, true>((int)bytes)));
    MFWF_TRY(inv_lds<double2>((int)bytes));
    MFWF_TRY(inv_lds<float2>((int)bytes));
    MFWF_TRY(inv_fwd_lds((int)bytes));
    MFWF_HIP(hipFuncSetAttribute((const void *)k_fft_inv_fwd_pol<256, 8>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    MFWF_HIP(hipFuncSetAttribute((const void *)k_fft_inv_fwd_pol<512, 8>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    const void *split_fns[] = {(const void *)k_fft_split_sub<kSplitSubTPB, 8, true, false>,
                               (const void *)k_fft_split_sub<kSplitSubTPB, 8, true, true>,
                               (const void *)k_fft_split_sub<kSplitSubTPB, 8, false, false>,
                               (const void *)k_fft_fwd_split_combine<kSplitTPB, 8, double2, false>,
                               (const void *)k_fft_fwd_split_combine<kSplitTPB, 8, float2, false>,
                               (const void *)k_fft_fwd_split_combine<kSplitTPB, 8, float2, true>,
                               (const void *)k_fft_inv_split_fold<kSplitTPB, 8, double2, false>,
                               (const void *)k_fft_inv_split_fold<kSplitTPB, 8, float2, false>,
                               (const void *)k_fft_inv_split_fold<kSplitTPB, 8, float2, true>};
    for (const void *f : split_fns)
        MFWF_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return MFWF_OK;
}

}  // namespace mfwf
