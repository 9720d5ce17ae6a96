// Batched FP32 path: many right-hand sides share one plan and the Legendre steps become
// dense contractions on the matrix cores (MFMA), the GPU form of the transforms that
// Sect. 3 names as the cost driver.
//
// For one m, with columns c = (map, re/im) of all maps in the batch:
//   synthesis  E[p][c] = sum_{l+m even} lambda_lm(z_p) s'[l][c],  O likewise over odd l+m,
//              F_N = E + O, F_S = E - O                      ([pairs x L] x [L x cols])
//   analysis   a[l][c] = sum_p lambda_lm(z_p) X_{(l+m) mod 2}[p][c],
//              X_0 = G_N + G_S, X_1 = G_N - G_S              ([L x pairs] x [pairs x cols])
// lambda_lm is tabulated once per plan in FP32 (computed from the FP64 recurrence and start
// seeds, zero below each pair's start index), as rows [m][pair][l - m] padded to 64 values of
// l and 64 pairs.  The products run on v_mfma_f32_32x32x2f32 with FP32 accumulation; the
// ring-Fourier array ([ring][m][cols]) and the coefficients ([alm][cols]) are FP32 with the
// maps innermost, so tiles of columns are contiguous.  Maps, the pixel update and every
// diagnostic stay FP64.  The ring FFTs are the FP64 transforms of the per-map path; one
// workgroup runs several maps of a ring pair in turn.
#include "fft_core.h"

namespace mfwf {

typedef float floatx16 __attribute__((ext_vector_type(16)));

static constexpr int kMapsPerFFTBlock = 16;

// ---------------------------------------------------------------------------------------
// lambda table: one lane per ring pair, one workgroup per (pair tile of 64, m).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(64)
k_lam_table(const double *__restrict__ Atab, const double *__restrict__ ctab,
            const long *__restrict__ mofs, const int *__restrict__ lstart,
            const double2 *__restrict__ seed, const double *__restrict__ zp,
            const long *__restrict__ loff, const int *__restrict__ Lp, float *__restrict__ lam,
            int lmax, int npair) {
    const int p = blockIdx.x * 64 + threadIdx.x, m = blockIdx.y;
    const int L = Lp[m];
    float *row = lam + loff[m] + (long)p * L;
    const long off = mofs[m] - m;
    if (p >= npair) {
        for (int r = 0; r < L; r++) row[r] = 0.f;
        return;
    }
    const int ls = lstart[(long)m * npair + p];
    const double2 sd = seed[(long)m * npair + p];
    const double z = zp[p];
    double u1 = 0.0, u2 = 0.0;
    for (int r = 0; r < L; r++) {
        const int l = m + r;
        float v = 0.f;
        if (l <= lmax && l >= ls) {
            double mu;
            if (l == ls) {
                mu = sd.y;
                u1 = sd.x;
            } else {
                mu = fma(Atab[off + l] * z, u1, -u2);
            }
            u2 = u1;
            u1 = mu;
            v = (float)(ctab[off + l] * mu);  // lambda = c mu
        }
        row[r] = v;
    }
}

// ---------------------------------------------------------------------------------------
// Batched ring FFTs: workgroup = (ring pair, group of maps); FP32 ring-Fourier
// [ring][m][C2], column 2b (re) and 2b + 1 (im) of map b.
// ---------------------------------------------------------------------------------------
template <int TPB, int EPT>
__global__ void __launch_bounds__(TPB)
k_fft_fwd_b(const double *__restrict__ maps, float *__restrict__ ph32,
            const PairFFT *__restrict__ pfft, const int *__restrict__ plist,
            const double2 *__restrict__ twlo, const double2 *__restrict__ twhi, int ntwhi,
            int fftmax, const double2 *__restrict__ chirp, const double2 *__restrict__ bhat,
            long npix, int nring, int nm, int lmax, int fftlen_class, int nb, int C2) {
    extern __shared__ double2 buf[];
    const int p = plist[blockIdx.x];
    const PairFFT pf = pfft[p];
    const int n = pf.nphi;
    const bool equator = (pf.startS == pf.startN);
    const Twiddles tw = load_twiddles(buf, fftlen_class, TPB, twlo, twhi, ntwhi);
    float *outN = ph32 + (long)p * nm * C2;
    float *outS = ph32 + (long)(nring - 1 - p) * nm * C2;
    const int b0 = blockIdx.y * kMapsPerFFTBlock;
    for (int g = 0; g < kMapsPerFFTBlock; g++) {
        const int b = b0 + g;
        if (b >= nb) break;
        const double *tN = maps + (long)b * npix + pf.startN;
        const double *tS = maps + (long)b * npix + pf.startS;
        for (int j = threadIdx.x; j < n; j += TPB)
            buf[j] = make_double2(tN[j], equator ? 0.0 : tS[j]);
        __syncthreads();
        ring_dft<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
        for (int m = threadIdx.x; m <= lmax; m += TPB) {
            const int q = m / n, k = m - q * n;
            const int kr = (k == 0) ? 0 : n - k;
            const double2 X = dft_bin(buf, pf, chirp, k);
            const double2 Y = cconj(dft_bin(buf, pf, chirp, kr));
            double2 ph = make_double2(1.0, 0.0);
            if (pf.half_shift) ph = cscale(cconj(half_bin_phase(k, n, tw, fftmax)), (q & 1) ? -1.0 : 1.0);
            const double2 gN = cmul(make_double2(0.5 * (X.x + Y.x), 0.5 * (X.y + Y.y)), ph);
            *reinterpret_cast<float2 *>(outN + (long)m * C2 + 2 * b) = make_float2((float)gN.x, (float)gN.y);
            if (!equator) {
                const double2 gS = cmul(make_double2(0.5 * (X.y - Y.y), -0.5 * (X.x - Y.x)), ph);
                *reinterpret_cast<float2 *>(outS + (long)m * C2 + 2 * b) = make_float2((float)gS.x, (float)gS.y);
            }
        }
        __syncthreads();
    }
}

template <int TPB, int EPT>
__global__ void __launch_bounds__(TPB)
k_fft_inv_b(const float *__restrict__ ph32, double *__restrict__ maps,
            const PairFFT *__restrict__ pfft, const int *__restrict__ plist,
            const double2 *__restrict__ twlo, const double2 *__restrict__ twhi, int ntwhi,
            int fftmax, const double2 *__restrict__ chirp, const double2 *__restrict__ bhat,
            long npix, int nring, int nm, int lmax, int fftlen_class, int nb, int C2) {
    extern __shared__ double2 buf[];
    const int p = plist[blockIdx.x];
    const PairFFT pf = pfft[p];
    const int n = pf.nphi;
    double2 *partN = buf + fftlen_class;
    double2 *partS = partN + TPB;
    const bool equator = (pf.startS == pf.startN);
    const Twiddles tw = load_twiddles(buf, fftlen_class, TPB, twlo, twhi, ntwhi);
    const float *FN = ph32 + (long)p * nm * C2;
    const float *FS = ph32 + (long)(nring - 1 - p) * nm * C2;
    int T = TPB / n;
    if (T < 1) T = 1;
    const int nbins_pass = TPB / T;
    const double sgn_step = pf.half_shift ? -1.0 : 1.0;
    const double sg_stride = (T & 1) ? sgn_step : 1.0;
    const int b0 = blockIdx.y * kMapsPerFFTBlock;
    for (int g = 0; g < kMapsPerFFTBlock; g++) {
        const int b = b0 + g;
        if (b >= nb) break;
        auto ld = [&](const float *F, int m) {
            const float2 v = *reinterpret_cast<const float2 *>(F + (long)m * C2 + 2 * b);
            return make_double2(v.x, v.y);
        };
        for (int k0 = 0; k0 < n; k0 += nbins_pass) {
            const int k = k0 + threadIdx.x / T, t = threadIdx.x % T;
            double2 sN = make_double2(0.0, 0.0), sS = make_double2(0.0, 0.0);
            if (k < n && (int)threadIdx.x < nbins_pass * T) {
                double sg = (t & 1) ? sgn_step : 1.0;
                for (int m = k + t * n; m <= lmax; m += T * n, sg *= sg_stride) {
                    sN = cadd(sN, cscale(ld(FN, m), sg));
                    if (!equator) sS = cadd(sS, cscale(ld(FS, m), sg));
                }
                sg = ((t + 1) & 1) ? sgn_step : 1.0;
                for (int mm = (t + 1) * n - k; mm <= lmax; mm += T * n, sg *= sg_stride) {
                    sN = cadd(sN, cscale(cconj(ld(FN, mm)), sg));
                    if (!equator) sS = cadd(sS, cscale(cconj(ld(FS, mm)), sg));
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
            if (t == 0 && k < n) {
                if (pf.half_shift) {
                    const double2 ph = half_bin_phase(k, n, tw, fftmax);
                    sN = cmul(sN, ph);
                    sS = cmul(sS, ph);
                }
                buf[k] = cconj(make_double2(sN.x - sS.y, sN.y + sS.x));
            }
        }
        __syncthreads();
        ring_dft<TPB, EPT>(buf, pf, tw, fftmax, chirp, bhat);
        double *sNmap = maps + (long)b * npix + pf.startN;
        double *sSmap = maps + (long)b * npix + pf.startS;
        for (int j = threadIdx.x; j < n; j += TPB) {
            const double2 x = cconj(dft_bin(buf, pf, chirp, j));
            sNmap[j] = x.x;
            if (!equator) sSmap[j] = x.y;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// MFMA GEMMs.  Workgroup of 4 waves; wave w owns columns [128 cg + 32 w, +32).
// v_mfma_f32_32x32x2f32 operands: A[i][k] in lane i + 32k, B[k][j] in lane j + 32k,
// accumulator register r of lane L holds D[8 (r/4) + 4 (L/32) + r%4][L%32].
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// analysis: workgroup = (m, tile of 64 values of l); K loop over pair chunks of 32.
__global__ void __launch_bounds__(256)
k_gemm_analysis(const float *__restrict__ lam, const long *__restrict__ loff,
                const int *__restrict__ Lp, const int *__restrict__ minls32,
                const int2 *__restrict__ items, const float *__restrict__ ph32,
                const long *__restrict__ mofs, float *__restrict__ a32, int lmax, int npair,
                int Rp, int nring, int nm, int C2, int ncols) {
    __shared__ float sl[32][64 + 1];        // lambda tile [pair][l]
    __shared__ float sx[2][32][128 + 4];    // X_0, X_1 tiles [pair][col]
    const int2 it = items[blockIdx.x];
    const int m = it.x, t = it.y, cg = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int L = Lp[m];
    const int lhi = m + 64 * t + 63;  // last l of the tile
    const int nchunk = Rp / 32;
    floatx16 ce, co;
#pragma unroll
    for (int r = 0; r < 16; r++) ce[r] = co[r] = 0.f;
    const float *lrow = lam + loff[m];
    const bool active = (128 * cg + 32 * w) < ncols;
    for (int pc = 0; pc < nchunk; pc++) {
        if (minls32[m * nchunk + pc] > lhi) continue;  // no pair of the chunk starts yet
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * 64; e += 256) {
            const int pp = e >> 6, rr = e & 63;
            sl[pp][rr] = lrow[(long)(32 * pc + pp) * L + 64 * t + rr];
        }
        for (int e = threadIdx.x; e < 32 * 128; e += 256) {
            const int pp = e >> 7, c = e & 127, col = 128 * cg + c;
            const int p = 32 * pc + pp;
            float gn = 0.f, gs = 0.f;
            if (p < npair && col < ncols) {
                gn = ph32[((long)p * nm + m) * C2 + col];
                if (nring - 1 - p != p) gs = ph32[((long)(nring - 1 - p) * nm + m) * C2 + col];
            }
            sx[0][pp][c] = gn + gs;
            sx[1][pp][c] = gn - gs;
        }
        __syncthreads();
        if (active) {
            const int i = lane & 31, kq = lane >> 5;
#pragma unroll 4
            for (int kk = 0; kk < 16; kk++) {
                const int pp = 2 * kk + kq;
                const float ae = sl[pp][2 * i], ao = sl[pp][2 * i + 1];
                const float be = sx[0][pp][32 * w + i], bo = sx[1][pp][32 * w + i];
                ce = __builtin_amdgcn_mfma_f32_32x32x2f32(ae, be, ce, 0, 0, 0);
                co = __builtin_amdgcn_mfma_f32_32x32x2f32(ao, bo, co, 0, 0, 0);
            }
        }
    }
    if (!active) return;
    const long base = mofs[m] - m;
    const int col = 128 * cg + 32 * w + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int i = acc_row(r, lane);
        const int le = m + 64 * t + 2 * i, lo = le + 1;
        if (le <= lmax) a32[(base + le) * C2 + col] = ce[r];
        if (lo <= lmax) a32[(base + lo) * C2 + col] = co[r];
    }
}

// synthesis: workgroup = (m, tile of 64 ring pairs); K loop over chunks of 64 values of l.
__global__ void __launch_bounds__(256)
k_gemm_synthesis(const float *__restrict__ lam, const long *__restrict__ loff,
                 const int *__restrict__ Lp, const int *__restrict__ minls64,
                 const float *__restrict__ s32, const long *__restrict__ mofs,
                 float *__restrict__ ph32, int lmax, int npair, int Rp, int nring, int nm,
                 int C2, int ncols) {
    __shared__ float sl[64][64 + 1];    // lambda tile [pair][l]
    __shared__ float ss[64][128 + 4];   // coefficient tile [l][col]
    const int m = blockIdx.x / (Rp / 64), pt = blockIdx.x % (Rp / 64), cg = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int L = Lp[m], Lm = lmax - m + 1;
    const bool active = (128 * cg + 32 * w) < ncols;
    floatx16 acc[2][2];  // [parity][pair tile of 32]
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[a][b][r] = 0.f;
    const float *lrow = lam + loff[m] + (long)(64 * pt) * L;
    const long base = mofs[m];
    const int first = max(0, minls64[m * (Rp / 64) + pt] - m) / 64;  // first chunk with lambda != 0
    for (int rc = first; rc * 64 < Lm; rc++) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int pp = e >> 6, rr = e & 63;
            sl[pp][rr] = lrow[(long)pp * L + 64 * rc + rr];
        }
        for (int e = threadIdx.x; e < 64 * 128; e += 256) {
            const int rr = e >> 7, c = e & 127, col = 128 * cg + c;
            const int r = 64 * rc + rr;
            ss[rr][c] = (r < Lm && col < ncols) ? s32[(base + r) * C2 + col] : 0.f;
        }
        __syncthreads();
        if (active) {
            const int i = lane & 31, kq = lane >> 5;
#pragma unroll
            for (int par = 0; par < 2; par++) {
#pragma unroll 4
                for (int kk = 0; kk < 16; kk++) {
                    const int rr = 4 * kk + 2 * kq + par;  // two same-parity l per step
                    const float bv = ss[rr][32 * w + i];
                    const float a0 = sl[i][rr], a1 = sl[32 + i][rr];
                    acc[par][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bv, acc[par][0], 0, 0, 0);
                    acc[par][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bv, acc[par][1], 0, 0, 0);
                }
            }
        }
    }
    if (!active) return;
    // rows are relative l = m + r: parity of r equals parity of l + m
    const int col = 128 * cg + 32 * w + (lane & 31);
#pragma unroll
    for (int tt = 0; tt < 2; tt++)
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int p = 64 * pt + 32 * tt + acc_row(r, lane);
            if (p >= npair) continue;
            const float E = acc[0][tt][r], O = acc[1][tt][r];
            ph32[((long)p * nm + m) * C2 + col] = E + O;
            const int rS = nring - 1 - p;
            if (rS != p) ph32[((long)rS * nm + m) * C2 + col] = E - O;
        }
}

// ---------------------------------------------------------------------------------------
// Harmonic update on [alm][C2] FP32 rows (Eq. 4), and conversions to / from the FP64
// per-map alm layout [map][nalm] complex through LDS-transposed tiles.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_harmonic_b(const float *__restrict__ a32, float *__restrict__ s32, const long *__restrict__ mofs,
             const double *__restrict__ cl, int lmax, double scale, double lto, int C2,
             int ncols) {
    const int m = blockIdx.x;
    const long base = mofs[m] - m;
    const long n = (long)(lmax - m + 1) * ncols;
    for (long e = threadIdx.x; e < n; e += 256) {
        const int l = m + (int)(e / ncols);
        const double C = cl[l];
        const double f = C > 0.0 ? C / (C + lto) * scale : 0.0;
        const long i = (base + l) * C2 + e % ncols;
        s32[i] = (float)(f * (double)a32[i]);
    }
}

// alm FP64 [nb][nalm] (complex) -> x32 [nalm][C2] FP32, times f(l) (mode: 3 copy, 2 C^-1/2)
__global__ void __launch_bounds__(256)
k_alm_to_cols(const double2 *__restrict__ alm, float *__restrict__ x32,
              const double *__restrict__ cl, const int *__restrict__ lofi, long nalm, int nb,
              int C2, int mode) {
    __shared__ float tile[64][65];  // [alm within tile][col within tile]
    const long i0 = (long)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;  // columns c0 .. c0+63 = maps c0/2 .. c0/2+31
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
        const int ii = e & 63, bb = e >> 6;
        const long i = i0 + ii;
        const int b = c0 / 2 + bb;
        double2 v = make_double2(0.0, 0.0);
        if (i < nalm && b < nb) {
            v = alm[(long)b * nalm + i];
            if (mode == 2) {
                const double C = cl[lofi[i]];
                const double f = C > 0.0 ? 1.0 / sqrt(C) : 0.0;
                v = make_double2(f * v.x, f * v.y);
            }
        }
        tile[ii][2 * bb] = (float)v.x;
        tile[ii][2 * bb + 1] = (float)v.y;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int ii = e >> 6, cc = e & 63;
        const long i = i0 + ii;
        if (i < nalm && c0 + cc < C2) x32[i * C2 + c0 + cc] = tile[ii][cc];
    }
}

// x32 [nalm][C2] FP32 -> alm FP64 [nb][nalm], times f (mode 1: Omega; mode 3: 1)
__global__ void __launch_bounds__(256)
k_cols_to_alm(const float *__restrict__ x32, double2 *__restrict__ alm, long nalm, int nb, int C2,
              double scale) {
    __shared__ float tile[64][65];
    const long i0 = (long)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int ii = e >> 6, cc = e & 63;
        const long i = i0 + ii;
        tile[ii][cc] = (i < nalm && c0 + cc < C2) ? x32[i * C2 + c0 + cc] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
        const int ii = e & 63, bb = e >> 6;
        const long i = i0 + ii;
        const int b = c0 / 2 + bb;
        if (i < nalm && b < nb)
            alm[(long)b * nalm + i] = make_double2(scale * tile[ii][2 * bb], scale * tile[ii][2 * bb + 1]);
    }
}

// ---------------------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------------------
int launch_lam_table(const Plan &p) {
    hipLaunchKernelGGL(k_lam_table, dim3(p.Rp / 64, p.nm), dim3(64), 0, p.stream, p.d_A, p.d_c,
                       p.d_mofs, p.d_lstart, p.d_seed, p.d_z, p.d_loff, p.d_Lp, p.d_lam, p.lmax,
                       p.npair);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

#define MFWF_FFTB_ARGS(c)                                                                       \
    p.d_pfft, p.d_plist + p.fft_class_off[c], p.d_twlo, p.d_twhi, p.fft_ntwhi, p.fftmax,        \
        p.d_chirp, p.d_bhat, p.npix, p.nring, p.nm, p.lmax, p.fft_class_len[c], nb, p.C2

int launch_fft_fwd_b(const Plan &p, const double *maps, int nb) {
    const int ng = (nb + kMapsPerFFTBlock - 1) / kMapsPerFFTBlock;
    for (int c = 1; c >= 0; c--) {
        const int cnt = p.fft_class_count[c];
        if (cnt == 0) continue;
        int ept;
        const int tpb = fft_class_shape(p, c, ept);
        const dim3 grid(cnt, ng);
        const size_t lds = fft_class_lds(p, c);
        if (ept == 8)
            hipLaunchKernelGGL((k_fft_fwd_b<256, 8>), grid, dim3(256), lds, p.stream, maps, p.d_ph32, MFWF_FFTB_ARGS(c));
        else if (tpb == 256)
            hipLaunchKernelGGL((k_fft_fwd_b<256, 16>), grid, dim3(256), lds, p.stream, maps, p.d_ph32, MFWF_FFTB_ARGS(c));
        else
            hipLaunchKernelGGL((k_fft_fwd_b<512, 16>), grid, dim3(512), lds, p.stream, maps, p.d_ph32, MFWF_FFTB_ARGS(c));
        MFWF_HIP(hipGetLastError());
    }
    return MFWF_OK;
}

int launch_fft_inv_b(const Plan &p, double *maps, int nb) {
    const int ng = (nb + kMapsPerFFTBlock - 1) / kMapsPerFFTBlock;
    for (int c = 1; c >= 0; c--) {
        const int cnt = p.fft_class_count[c];
        if (cnt == 0) continue;
        int ept;
        const int tpb = fft_class_shape(p, c, ept);
        const dim3 grid(cnt, ng);
        const size_t lds = fft_class_lds(p, c);
        if (ept == 8)
            hipLaunchKernelGGL((k_fft_inv_b<256, 8>), grid, dim3(256), lds, p.stream, p.d_ph32, maps, MFWF_FFTB_ARGS(c));
        else if (tpb == 256)
            hipLaunchKernelGGL((k_fft_inv_b<256, 16>), grid, dim3(256), lds, p.stream, p.d_ph32, maps, MFWF_FFTB_ARGS(c));
        else
            hipLaunchKernelGGL((k_fft_inv_b<512, 16>), grid, dim3(512), lds, p.stream, p.d_ph32, maps, MFWF_FFTB_ARGS(c));
        MFWF_HIP(hipGetLastError());
    }
    return MFWF_OK;
}

static int active_cols(int nb) { return 32 * ((2 * nb + 31) / 32); }

int launch_gemm_analysis(const Plan &p, int nb) {
    const int nc = active_cols(nb);
    hipLaunchKernelGGL(k_gemm_analysis, dim3(p.n_ana_items, (nc + 127) / 128), dim3(256), 0,
                       p.stream, p.d_lam, p.d_loff, p.d_Lp, p.d_minls32, p.d_ana_items, p.d_ph32,
                       p.d_mofs, p.d_a32, p.lmax, p.npair, p.Rp, p.nring, p.nm, p.C2, nc);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_gemm_synthesis(const Plan &p, int nb) {
    const int nc = active_cols(nb);
    hipLaunchKernelGGL(k_gemm_synthesis, dim3(p.nm * (p.Rp / 64), (nc + 127) / 128), dim3(256), 0,
                       p.stream, p.d_lam, p.d_loff, p.d_Lp, p.d_minls64, p.d_s32, p.d_mofs,
                       p.d_ph32, p.lmax, p.npair, p.Rp, p.nring, p.nm, p.C2, nc);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_harmonic_b(const Plan &p, double scale, double lto, int nb) {
    hipLaunchKernelGGL(k_harmonic_b, dim3(p.nm), dim3(256), 0, p.stream, p.d_a32, p.d_s32,
                       p.d_mofs, p.d_cl, p.lmax, scale, lto, p.C2, active_cols(nb));
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_alm_to_cols(const Plan &p, const double2 *alm, float *x32, int nb, int mode) {
    hipLaunchKernelGGL(k_alm_to_cols, dim3((p.nalm + 63) / 64, (p.C2 + 63) / 64), dim3(256), 0,
                       p.stream, alm, x32, p.d_cl, p.d_lofi, p.nalm, nb, p.C2, mode);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_cols_to_alm(const Plan &p, const float *x32, double2 *alm, int nb, double scale) {
    hipLaunchKernelGGL(k_cols_to_alm, dim3((p.nalm + 63) / 64, (p.C2 + 63) / 64), dim3(256), 0,
                       p.stream, x32, alm, p.nalm, nb, p.C2, scale);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int batched_set_lds_limit(size_t bytes) {
    const void *fns[] = {(const void *)k_fft_fwd_b<256, 8>, (const void *)k_fft_fwd_b<256, 16>,
                         (const void *)k_fft_fwd_b<512, 16>, (const void *)k_fft_inv_b<256, 8>,
                         (const void *)k_fft_inv_b<256, 16>, (const void *)k_fft_inv_b<512, 16>};
    for (const void *f : fns)
        MFWF_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return MFWF_OK;
}

}  // namespace mfwf
