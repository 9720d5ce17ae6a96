// Device routines of the ring phi transforms, shared by the FP64 per-map kernels
// (ringfft.hip) and the batched kernels (batched.hip): complex helpers, small in-register
// DFTs, in-place Stockham passes in LDS, twiddles from a two-level table in LDS, and the
// Bluestein wrapper for non-power-of-two ring lengths.
#pragma once

#include "mfwf_internal.h"

namespace mfwf {

// complex product with its two fused multiply-adds written out: the ring transforms are
// compiled without floating-point contraction, so that every kernel that runs them (per-map,
// chained on the columns, split) rounds each operation alike
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) {
    return make_double2(a.x * s, a.y * s);
}
__device__ __forceinline__ double2 mul_minus_i(double2 a) { return make_double2(a.y, -a.x); }

// Transform element i lives at LDS slot i + i/8: one pad slot per 8 elements spreads the
// strided butterfly writes of the first passes (element strides of 8 and 64) over all LDS
// banks.
__host__ __device__ __forceinline__ constexpr int lds_ix(int i) { return i + (i >> 3); }

// Transform slots of a workgroup with TPB threads and transforms up to fftlen: the padded
// transform, and at least room for the inverse transform's alias-sum partials (2 TPB
// slots after the padded first TPB/2 elements, used only for rings of n <= TPB/2).
__host__ __device__ __forceinline__ constexpr int fft_area(int fftlen, int tpb) {
    return lds_ix(fftlen) > lds_ix(tpb / 2) + 2 * tpb ? lds_ix(fftlen) : lds_ix(tpb / 2) + 2 * tpb;
}

// W_N^t = exp(-2 pi i t / N) for the plan's largest transform length N, as
// hi[t / 64] * lo[t % 64] from two short tables held in LDS.
struct Twiddles {
    const double2 *lo, *hi;
    __device__ __forceinline__ double2 operator()(int t) const { return cmul(hi[t >> 6], lo[t & 63]); }
};

// Dynamic LDS of one ring-transform workgroup: [area transform slots][64 lo][N/64 hi].
__device__ __forceinline__ Twiddles load_twiddles(double2 *lds, int area,
                                                  const double2 *__restrict__ glo,
                                                  const double2 *__restrict__ ghi, int nhi) {
    double2 *lo = lds + area, *hi = lo + 64;
    for (int j = threadIdx.x; j < 64 + nhi; j += blockDim.x) {
        if (j < 64) lo[j] = glo[j];
        else hi[j - 64] = ghi[j - 64];
    }
    __syncthreads();
    return Twiddles{lo, hi};
}

// Forward R-point DFT in registers, natural order in and out (R = 2, 4, 8).
template <int R>
__device__ __forceinline__ void small_dft(double2 (&v)[R]) {
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const double2 s13 = cadd(v[1], v[3]), d13 = mul_minus_i(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else {
        double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        small_dft<4>(e);
        small_dft<4>(o);
        const double h = 0.70710678118654752440;  // W8 = (1 - i)/sqrt 2
        o[1] = make_double2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
        o[2] = mul_minus_i(o[2]);
        o[3] = make_double2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
#pragma unroll
        for (int k = 0; k < 4; k++) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
}

// Elementwise step applied to the inputs of a first pass (Bluestein's algorithm): none;
// times the chirp c_i for i < nv and zero beyond (the zero-padded chirped sequence); or
// times the transformed kernel k_i, conjugated.
enum { kPreNone = 0, kPreChirp = 1, kPreKernelConj = 2 };

// One Stockham pass of radix R over buf[0..n): inputs j + r n/R, output (j/Ns) Ns R + j%Ns
// + r Ns, twiddle exp(-2 pi i (j%Ns) r / (Ns R)).  All reads precede all writes.  The
// transform belongs to the TPB threads of the thread's group (threadIdx.x mod TPB; a
// workgroup may hold several groups, one transform each, which pass the barriers together).
// EPT: most transform elements one thread handles (n <= EPT * TPB).  PRE != kPreNone only
// on a first pass (Ns = 1, no twiddles), with its table pre.
template <int TPB, int EPT, int R, int PRE = kPreNone>
__device__ __forceinline__ void stockham_pass(double2 *buf, int n, int Ns, const Twiddles &tw,
                                              int fftmax, const double2 *__restrict__ pre = nullptr,
                                              int nv = 0) {
    constexpr int MAXB = EPT / R;
    const int nbf = n / R;
    double2 v[MAXB][R];
#pragma unroll
    for (int b = 0; b < MAXB; b++) {
        const int j = (threadIdx.x & (TPB - 1)) + b * TPB;
        if (j < nbf) {
#pragma unroll
            for (int r = 0; r < R; r++) v[b][r] = buf[lds_ix(j + r * nbf)];
            if constexpr (PRE == kPreChirp) {
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const int i = j + r * nbf;
                    v[b][r] = (i < nv) ? cmul(v[b][r], pre[min(i, nv - 1)]) : make_double2(0.0, 0.0);
                }
            } else if constexpr (PRE == kPreKernelConj) {
#pragma unroll
                for (int r = 0; r < R; r++) v[b][r] = cconj(cmul(v[b][r], pre[j + r * nbf]));
            }
        }
    }
    __syncthreads();
    const int ts = fftmax / (Ns * R);
#pragma unroll
    for (int b = 0; b < MAXB; b++) {
        const int j = (threadIdx.x & (TPB - 1)) + b * TPB;
        if (j < nbf) {
            const int kk = j & (Ns - 1);
            if (PRE == kPreNone && Ns > 1) {
                // one table twiddle w per butterfly; w^r as products (a few ulp in FP64)
                double2 wr[R];
                wr[1] = tw(kk * ts);
#pragma unroll
                for (int r = 2; r < R; r++) wr[r] = cmul(wr[r / 2], wr[r - r / 2]);
#pragma unroll
                for (int r = 1; r < R; r++) v[b][r] = cmul(v[b][r], wr[r]);
            }
            small_dft<R>(v[b]);
            const int base = (j - kk) * R + kk;
#pragma unroll
            for (int r = 0; r < R; r++) buf[lds_ix(base + r * Ns)] = v[b][r];
        }
    }
    __syncthreads();
}

// Forward DFT of buf[0..n), n a power of two <= EPT * TPB, natural order in and out; PRE
// (with pre, nv) on the inputs of the first pass.
template <int TPB, int EPT, int PRE = kPreNone>
__device__ __forceinline__ void fft_stockham(double2 *buf, int n, const Twiddles &tw, int fftmax,
                                             const double2 *__restrict__ pre = nullptr, int nv = 0) {
    int Ns = 1;
    if constexpr (PRE != kPreNone) {
        if (n >= 8) {
            stockham_pass<TPB, EPT, 8, PRE>(buf, n, 1, tw, fftmax, pre, nv);
            Ns = 8;
        } else if (n == 4) {
            stockham_pass<TPB, EPT, 4, PRE>(buf, n, 1, tw, fftmax, pre, nv);
            Ns = 4;
        } else {
            stockham_pass<TPB, EPT, 2, PRE>(buf, n, 1, tw, fftmax, pre, nv);
            Ns = 2;
        }
    }
    while (Ns < n) {
        const int left = n / Ns;
        if (left >= 8) {
            stockham_pass<TPB, EPT, 8>(buf, n, Ns, tw, fftmax);
            Ns *= 8;
        } else if (left == 4) {
            stockham_pass<TPB, EPT, 4>(buf, n, Ns, tw, fftmax);
            Ns *= 4;
        } else {
            stockham_pass<TPB, EPT, 2>(buf, n, Ns, tw, fftmax);
            Ns *= 2;
        }
    }
}

// ---- compile-time transform lengths ---------------------------------------------------
// The same Stockham passes with the length N, the radix and the stride Ns of every pass known
// at compile time: a thread's LDS slots are one base plus constant offsets (the pad slot
// every 8 elements folds into the constant), the butterfly-count guard disappears when the
// threads divide the butterflies, and the twiddle index is a shift.  Arithmetic and its
// order are those of stockham_pass / fft_stockham, so results are bitwise the same.

__device__ __forceinline__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// nout: outputs that are read afterwards; the last pass (Ns R = N) stores only those
template <int TPB, int N, int R, int Ns, int PRE>
__device__ __forceinline__ void stockham_pass_c(double2 *buf, const Twiddles &tw, int lgmax,
                                                const double2 *__restrict__ pre, int nv, int nout) {
    constexpr int NBF = N / R;
    constexpr int MAXB = (NBF + TPB - 1) / TPB;
    constexpr bool ALL = (NBF % TPB == 0);
    double2 v[MAXB][R];
#pragma unroll
    for (int b = 0; b < MAXB; b++) {
        const int j = (threadIdx.x & (TPB - 1)) + b * TPB;
        if (ALL || j < NBF) {
            if constexpr (PRE == kPreChirp) {
                // the chirped sequence, zero from nv on: only its first nv elements are read
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const int i = j + r * NBF;
                    v[b][r] = make_double2(0.0, 0.0);
                    if (i < nv) v[b][r] = cmul(buf[lds_ix(i)], pre[i]);
                }
            } else if constexpr (NBF % 8 == 0) {
                const int jb = lds_ix(j);
#pragma unroll
                for (int r = 0; r < R; r++) v[b][r] = buf[jb + r * (NBF / 8) * 9];
            } else {
#pragma unroll
                for (int r = 0; r < R; r++) v[b][r] = buf[lds_ix(j + r * NBF)];
            }
            if constexpr (PRE == kPreKernelConj) {
#pragma unroll
                for (int r = 0; r < R; r++) v[b][r] = cconj(cmul(v[b][r], pre[j + r * NBF]));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; b++) {
        const int j = (threadIdx.x & (TPB - 1)) + b * TPB;
        if (ALL || j < NBF) {
            const int kk = j & (Ns - 1);
            if constexpr (PRE == kPreNone && Ns > 1) {
                double2 wr[R];
                wr[1] = tw(kk << (lgmax - ilog2c(Ns * R)));
#pragma unroll
                for (int r = 2; r < R; r++) wr[r] = cmul(wr[r / 2], wr[r - r / 2]);
#pragma unroll
                for (int r = 1; r < R; r++) v[b][r] = cmul(v[b][r], wr[r]);
            }
            small_dft<R>(v[b]);
            const int base = (j - kk) * R + kk;
            if constexpr (Ns % 8 == 0) {
                const int bb = lds_ix(base);
#pragma unroll
                for (int r = 0; r < R; r++)
                    if (Ns * R < N || base + r * Ns < nout) buf[bb + r * (Ns / 8) * 9] = v[b][r];
            } else if constexpr (Ns == 1 && R == 8) {
#pragma unroll
                for (int r = 0; r < R; r++) buf[9 * j + r] = v[b][r];  // lds_ix(8 j + r)
            } else {
#pragma unroll
                for (int r = 0; r < R; r++) buf[lds_ix(base + r * Ns)] = v[b][r];
            }
        }
    }
    __syncthreads();
}

// The passes of fft_stockham for length N: radix 8 while at least 8 remain, then 4 or 2;
// outputs from nout on are not stored (where nothing reads them).
template <int TPB, int N, int Ns, int PRE>
__device__ __forceinline__ void fft_passes_c(double2 *buf, const Twiddles &tw, int lgmax,
                                             const double2 *__restrict__ pre, int nv, int nout = N) {
    if constexpr (Ns < N) {
        constexpr int left = N / Ns;
        constexpr int R = left >= 8 ? 8 : left;
        stockham_pass_c<TPB, N, R, Ns, (Ns == 1 ? PRE : kPreNone)>(buf, tw, lgmax, pre, nv, nout);
        fft_passes_c<TPB, N, Ns * R, PRE>(buf, tw, lgmax, pre, nv, nout);
    }
}

// ring_dft with the power-of-two length of the pair's transform (n itself, or Bluestein's M)
// dispatched to compile-time lengths from TPB EPT down to MINC; shorter lengths take the
// run-time passes.
template <int TPB, int EPT, int N, int MINC>
__device__ __forceinline__ bool ring_dft_fixed(double2 *buf, const PairFFT &pf, const Twiddles &tw,
                                               int lgmax, const double2 *__restrict__ chirp,
                                               const double2 *__restrict__ bhat) {
    if constexpr (N < MINC) {
        return false;
    } else {
        if (pf.fftlen == N) {
            if (!pf.bluestein) {
                fft_passes_c<TPB, N, 1, kPreNone>(buf, tw, lgmax, nullptr, 0);
            } else {
                // only the first n bins of the convolution are read (dft_bin, k < n)
                fft_passes_c<TPB, N, 1, kPreChirp>(buf, tw, lgmax, chirp + pf.chirp_off, pf.nphi);
                fft_passes_c<TPB, N, 1, kPreKernelConj>(buf, tw, lgmax, bhat + pf.bhat_off, N, pf.nphi);
            }
            return true;
        }
        return ring_dft_fixed<TPB, EPT, N / 2, MINC>(buf, pf, tw, lgmax, chirp, bhat);
    }
}

// Length-n forward DFT of elements 0..n-1 in place.  On return the transform value of bin k
// is read with dft_bin(): element k for power-of-two n, c_k conj(element k) for Bluestein.
template <int TPB, int EPT>
__device__ __forceinline__ void ring_dft(double2 *buf, const PairFFT &pf, const Twiddles &tw,
                                         int fftmax, const double2 *__restrict__ chirp,
                                         const double2 *__restrict__ bhat) {
    const int n = pf.nphi, M = pf.fftlen;
    if (!pf.bluestein) {
        fft_stockham<TPB, EPT>(buf, n, tw, fftmax);
        return;
    }
    // the chirped input, zero-padded to M, transformed; times the transformed conj chirp
    // (already divided by M) and conjugated, transformed again: the conjugated convolution.
    // Both elementwise steps ride on the reads of the transforms' first passes.
    fft_stockham<TPB, EPT, kPreChirp>(buf, M, tw, fftmax, chirp + pf.chirp_off, n);
    fft_stockham<TPB, EPT, kPreKernelConj>(buf, M, tw, fftmax, bhat + pf.bhat_off, M);
}

// ring_dft on compile-time lengths where the pair's transform length allows (the results
// equal ring_dft's bit for bit)
template <int TPB, int EPT>
__device__ __forceinline__ void ring_dft_c(double2 *buf, const PairFFT &pf, const Twiddles &tw,
                                           int fftmax, const double2 *__restrict__ chirp,
                                           const double2 *__restrict__ bhat) {
    const int lgmax = __builtin_ctz(fftmax);
    if (!ring_dft_fixed<TPB, EPT, TPB * EPT, 64>(buf, pf, tw, lgmax, chirp, bhat))
        ring_dft<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
}

__device__ __forceinline__ double2 dft_bin(const double2 *buf, const PairFFT &pf,
                                           const double2 *__restrict__ chirp, int k) {
    if (!pf.bluestein) return buf[lds_ix(k)];
    return cmul(chirp[pf.chirp_off + k], cconj(buf[lds_ix(k)]));
}

// e^{i pi k / n}: from the twiddle table when 2n divides the largest length, else sincospi
__device__ __forceinline__ double2 half_bin_phase(int k, int n, const Twiddles &tw, int fftmax) {
    if (fftmax % (2 * n) == 0) return cconj(tw(k * (fftmax / (2 * n))));
    double s, c;
    sincospi((double)k / (double)n, &s, &c);
    return make_double2(c, s);
}

}  // namespace mfwf
