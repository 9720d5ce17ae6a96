// Batched FP32 form of the T, Q, U messenger iteration: the spin-2 Legendre steps as
// matrix-core contractions over the batch, like the temperature batched form.
//
// With F+-_lm = ((2)lambda_lm +- (-2)lambda_lm)/2 (HEALPix / Zaldarriaga-Seljak convention)
// the polarized transforms split into real-table contractions over complex columns:
//   analysis   a_E = -Omega (P_Q + i R_U),  a_B = -Omega (P_U - i R_Q),
//              P = sum_r F+ (G_Q, G_U),  R = sum_r F- (G_Q, G_U)
//   synthesis  Q = -(P'_E + i R'_B),  U = -(P'_B - i R'_E),
//              P' = sum_l F+ (s_E, s_B),  R' = sum_l F- (s_E, s_B)
// so each direction is three GEMMs on the batched kernels: lambda on the T columns, F+ and F-
// on the four columns (re, im of Q and U, or of E and B) of every map.  F+ has lambda's mirror
// symmetry, F+(-z) = (-1)^{l+m} F+(z); F- the opposite one, F-(-z) = -(-1)^{l+m} F-(z), which
// the GEMM kernels take as a flipped south ring.
//
// Tables: FP32 [m][pair][l - m] like lambda, F+- = (s^2 F+-) / s^2 with
//   s^2 F+ = (pc0 + pc1 z^2) mu_l + pc2 z mu_{l-1},  s^2 F- = pc3 mu_{l-1} + pc4 z mu_l
// from the FP64 rescaled recurrence (lambda = c mu) and the plan's five spin-2 coefficients
// per (l, m); s^2 = (1 - z)(1 + z).
//
// Column layouts: T [..][2 Bp] (re, im of map b at 2b), Q/U or E/B [..][4 Bp] (map b at 4b:
// re, im of the first component, re, im of the second).  Ring-Fourier rows of the transforms:
// [3 B][ring][m] FP32, map b's T, Q, U at rows 3b, 3b + 1, 3b + 2.
#include "mfwf_internal.h"

namespace mfwf {

// ---------------------------------------------------------------------------------------
// lambda, F+ and F- tables: one lane per ring pair, one workgroup per (pair tile of 64, m)
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(64)
k_pol_tables(const double *__restrict__ Atab, const double *__restrict__ ctab,
             const double *__restrict__ pc, const long *__restrict__ mofs,
             const int *__restrict__ lstart, const double2 *__restrict__ seed,
             const double *__restrict__ zp, const long *__restrict__ loff,
             const int *__restrict__ Lp, float *__restrict__ lam, float *__restrict__ fp,
             float *__restrict__ fm, int lmax, int npair) {
    const int p = blockIdx.x * 64 + threadIdx.x, m = blockIdx.y;
    const int L = Lp[m];
    const long ro = loff[m] + (long)p * L;
    const long off = mofs[m] - m;
    if (p >= npair) {
        for (int r = 0; r < L; r++) {
            lam[ro + r] = 0.f;
            fp[ro + r] = 0.f;
            fm[ro + r] = 0.f;
        }
        return;
    }
    const int ls = lstart[(long)m * npair + p];
    const double2 sd = seed[(long)m * npair + p];
    const double z = zp[p], s2 = (1.0 - z) * (1.0 + z);
    double u1 = 0.0, u2 = 0.0;  // mu_{l-1}, mu_{l-2}
    for (int r = 0; r < L; r++) {
        const int l = m + r;
        float v = 0.f, vp = 0.f, vm = 0.f;
        if (l <= lmax && l >= ls) {
            double mu, mup;
            if (l == ls) {
                mu = sd.y;
                mup = sd.x;
            } else {
                mu = fma(Atab[off + l] * z, u1, -u2);
                mup = u1;
            }
            u2 = mup;
            u1 = mu;
            const double *q = pc + 5 * (off + l);
            v = (float)(ctab[off + l] * mu);
            vp = (float)(fma(fma(q[1], z * z, q[0]), mu, q[2] * z * mup) / s2);
            vm = (float)(fma(q[3], mup, q[4] * z * mu) / s2);
        }
        lam[ro + r] = v;
        fp[ro + r] = vp;
        fm[ro + r] = vm;
    }
}

// ---------------------------------------------------------------------------------------
// Layout changes between the rows [3B][ring][m] and the column layouts, through LDS tiles
// of 64 values of m x 32 maps of one ring (T, Q, U together).  Each thread issues all of its
// loads before it stores any of them (clamped in-range addresses, values selected).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_rows_to_cols_pol(const float2 *__restrict__ phf, float *__restrict__ colT,
                   float *__restrict__ colP, int nring, int nm, int rs, int nb, int Bp) {
    __shared__ float2 tile[3][32][64 + 1];  // [component][map][m]
    const int ring = blockIdx.x, m0 = 64 * blockIdx.y, b0 = 32 * blockIdx.z;
    float2 v[24];
#pragma unroll
    for (int u = 0; u < 24; u++) {
        const int e = threadIdx.x + 256 * u;
        const int c = e >> 11, bb = (e >> 6) & 31, mm = e & 63, b = b0 + bb, m = m0 + mm;
        const float2 x = phf[((3L * min(b, nb - 1) + c) * nring + ring) * rs + min(m, nm - 1)];
        v[u] = (b < nb && m < nm) ? x : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 24; u++) {
        const int e = threadIdx.x + 256 * u;
        tile[e >> 11][(e >> 6) & 31][e & 63] = v[u];
    }
    __syncthreads();
    const long C2 = 2L * Bp;
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const int e = threadIdx.x + 256 * u, mm = e >> 5, bb = e & 31, b = b0 + bb, m = m0 + mm;
        if (b >= Bp || m >= nm) continue;
        const long row = (long)m * nring + ring;
        const float2 t = tile[0][bb][mm], q = tile[1][bb][mm], u2 = tile[2][bb][mm];
        *reinterpret_cast<float2 *>(colT + row * C2 + 2 * b) = t;
        *reinterpret_cast<float4 *>(colP + row * 2 * C2 + 4 * b) = make_float4(q.x, q.y, u2.x, u2.y);
    }
}

// T rows from colT; Q and U rows from colQU = (Q, U) per map (formed by the F- synthesis's
// epilogue from P' and R').
__global__ void __launch_bounds__(256)
k_cols_to_rows_pol(const float *__restrict__ colT, const float *__restrict__ colQU,
                   float2 *__restrict__ phf, int nring, int nm, int rs, int nb, int Bp) {
    __shared__ float2 tile[3][64][32 + 1];  // [component][m][map]
    const int ring = blockIdx.x, m0 = 64 * blockIdx.y, b0 = 32 * blockIdx.z;
    const long C2 = 2L * Bp;
    float2 vt[8];
    float4 vq[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const int e = threadIdx.x + 256 * u, mm = e >> 5, bb = e & 31;
        const int b = min(b0 + bb, nb - 1), m = min(m0 + mm, nm - 1);
        const long row = (long)m * nring + ring;
        vt[u] = *reinterpret_cast<const float2 *>(colT + row * C2 + 2 * b);
        vq[u] = *reinterpret_cast<const float4 *>(colQU + row * 2 * C2 + 4 * b);
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const int e = threadIdx.x + 256 * u, mm = e >> 5, bb = e & 31;
        const bool on = b0 + bb < nb && m0 + mm < nm;
        const float2 z = make_float2(0.f, 0.f);
        tile[0][mm][bb] = on ? vt[u] : z;
        tile[1][mm][bb] = on ? make_float2(vq[u].x, vq[u].y) : z;  // Q
        tile[2][mm][bb] = on ? make_float2(vq[u].z, vq[u].w) : z;  // U
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 24; u++) {
        const int e = threadIdx.x + 256 * u;
        const int c = e >> 11, bb = (e >> 6) & 31, mm = e & 63, b = b0 + bb, m = m0 + mm;
        if (b < nb && m < nm) phf[((3L * b + c) * nring + ring) * rs + m] = tile[c][mm][bb];
    }
}

// ---------------------------------------------------------------------------------------
// Analysis combination, one thread per (coefficient, map), maps innermost:
//   a_T = Omega A_T,  a_E = -Omega (P_Q + i R_U),  a_B = -Omega (P_U - i R_Q)
// then (mode kPolFilter) the Eq. (4) update with the 3x3 (T, E, B) signal block,
//   s = S (S + lto)^{-1} a,  on (T, E): [[D + mu TT, mu TE], [mu TE, D + mu EE]] / det,
//   on B: BB / (BB + mu)  (D = TT EE - TE^2, det = (TT + mu)(EE + mu) - TE^2),
// or (mode kPolRaw) s = a.  Written as FP32 columns: T to outT [alm][2 Bp], (E, B) to
// outEB [alm][4 Bp].  The arithmetic is FP64.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_pol_combine(const float *__restrict__ aT, const float *__restrict__ aP,
              const float *__restrict__ aR, const int *__restrict__ lofi,
              const double *__restrict__ cl4, int lmax, long nalm, int Bp, double omega,
              double lto, int mode, float *__restrict__ outT, float *__restrict__ outEB) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nalm * Bp) return;
    const long i = e / Bp;
    const int b = (int)(e - i * Bp);
    const long C2 = 2L * Bp;
    const float2 t = *reinterpret_cast<const float2 *>(aT + i * C2 + 2 * b);
    const float4 P = *reinterpret_cast<const float4 *>(aP + i * 2 * C2 + 4 * b);  // P_Q, P_U
    const float4 R = *reinterpret_cast<const float4 *>(aR + i * 2 * C2 + 4 * b);  // R_Q, R_U
    double2 a0 = make_double2(omega * t.x, omega * t.y);
    double2 a1 = make_double2(-omega * ((double)P.x - R.w), -omega * ((double)P.y + R.z));
    double2 a2 = make_double2(-omega * ((double)P.z + R.y), -omega * ((double)P.w - R.x));
    if (mode == kPolFilter) {
        const int l = lofi[i], L1 = lmax + 1;
        const double TT = cl4[l], EE = cl4[L1 + l], BB = cl4[2 * L1 + l], TE = cl4[3 * L1 + l];
        const double mu = lto, D = TT * EE - TE * TE;
        const double det = (TT + mu) * (EE + mu) - TE * TE;
        const double ftt = (D + mu * TT) / det, fte = mu * TE / det, fee = (D + mu * EE) / det;
        const double fbb = BB > 0.0 ? BB / (BB + mu) : 0.0;
        const double2 s0 = make_double2(ftt * a0.x + fte * a1.x, ftt * a0.y + fte * a1.y);
        const double2 s1 = make_double2(fte * a0.x + fee * a1.x, fte * a0.y + fee * a1.y);
        a2 = make_double2(fbb * a2.x, fbb * a2.y);
        a0 = s0;
        a1 = s1;
    }
    *reinterpret_cast<float2 *>(outT + i * C2 + 2 * b) = make_float2((float)a0.x, (float)a0.y);
    *reinterpret_cast<float4 *>(outEB + i * 2 * C2 + 4 * b) =
        make_float4((float)a1.x, (float)a1.y, (float)a2.x, (float)a2.y);
}

// ---------------------------------------------------------------------------------------
// FP64 coefficients [B][3][nalm] (T, E, B) <-> FP32 columns T [alm][2 Bp], (E, B)
// [alm][4 Bp], through LDS tiles of 64 coefficients x 32 maps.  Columns of maps nb..Bp-1
// are written as zeros.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_alm_to_cols_pol(const double2 *__restrict__ alm, float *__restrict__ colT,
                  float *__restrict__ colEB, long nalm, int nb, int Bp) {
    __shared__ float2 tile[3][64][32 + 1];  // [component][coefficient][map]
    const long i0 = (long)blockIdx.x * 64;
    const int b0 = 32 * blockIdx.y;
    for (int e = threadIdx.x; e < 3 * 32 * 64; e += 256) {
        const int c = e >> 11, bb = (e >> 6) & 31, ii = e & 63;
        const long i = i0 + ii;
        const int b = b0 + bb;
        double2 v = make_double2(0.0, 0.0);
        if (i < nalm && b < nb) v = alm[(3L * b + c) * nalm + i];
        tile[c][ii][bb] = make_float2((float)v.x, (float)v.y);
    }
    __syncthreads();
    const long C2 = 2L * Bp;
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
        const int ii = e >> 5, bb = e & 31;
        const long i = i0 + ii;
        const int b = b0 + bb;
        if (i >= nalm || b >= Bp) continue;
        const float2 t = tile[0][ii][bb], x = tile[1][ii][bb], y = tile[2][ii][bb];
        *reinterpret_cast<float2 *>(colT + i * C2 + 2 * b) = t;
        *reinterpret_cast<float4 *>(colEB + i * 2 * C2 + 4 * b) = make_float4(x.x, x.y, y.x, y.y);
    }
}

__global__ void __launch_bounds__(256)
k_cols_to_alm_pol(const float *__restrict__ colT, const float *__restrict__ colEB,
                  double2 *__restrict__ alm, long nalm, int nb, int Bp) {
    __shared__ float2 tile[3][64][32 + 1];
    const long i0 = (long)blockIdx.x * 64;
    const int b0 = 32 * blockIdx.y;
    const long C2 = 2L * Bp;
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
        const int ii = e >> 5, bb = e & 31;
        const long i = i0 + ii;
        const int b = b0 + bb;
        float2 t = make_float2(0.f, 0.f), x = t, y = t;
        if (i < nalm && b < Bp) {
            t = *reinterpret_cast<const float2 *>(colT + i * C2 + 2 * b);
            const float4 v = *reinterpret_cast<const float4 *>(colEB + i * 2 * C2 + 4 * b);
            x = make_float2(v.x, v.y);
            y = make_float2(v.z, v.w);
        }
        tile[0][ii][bb] = t;
        tile[1][ii][bb] = x;
        tile[2][ii][bb] = y;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * 32 * 64; e += 256) {
        const int c = e >> 11, bb = (e >> 6) & 31, ii = e & 63;
        const long i = i0 + ii;
        const int b = b0 + bb;
        if (i < nalm && b < nb) {
            const float2 v = tile[c][ii][bb];
            alm[(3L * b + c) * nalm + i] = make_double2(v.x, v.y);
        }
    }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
int launch_pol_tables(const Plan &p) {
    hipLaunchKernelGGL(k_pol_tables, dim3(p.Rp / 64, p.nm), dim3(64), 0, p.stream, p.d_A, p.d_c,
                       p.d_pc, p.d_mofs, p.d_lstart, p.d_seed, p.d_z, p.d_loff, p.d_Lp, p.d_lam,
                       p.d_fp, p.d_fm, p.lmax, p.npair);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_rows_to_cols_pol(const Plan &p, int nb) {
    hipLaunchKernelGGL(k_rows_to_cols_pol, dim3(p.nring, (p.nm + 63) / 64, (p.Bp + 31) / 32),
                       dim3(256), 0, p.stream, p.d_phf, p.d_ph32, p.d_ph32p, p.nring, p.nm, p.nm32,
                       nb, p.Bp);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_cols_to_rows_pol(const Plan &p, int nb) {
    hipLaunchKernelGGL(k_cols_to_rows_pol, dim3(p.nring, (p.nm + 63) / 64, (nb + 31) / 32),
                       dim3(256), 0, p.stream, p.d_ph32, p.d_ph32p, p.d_phf, p.nring,
                       p.nm, p.nm32, nb, p.Bp);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_pol_combine(const Plan &p, double lto, int mode) {
    const long n = p.nalm * p.Bp;
    hipLaunchKernelGGL(k_pol_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p.stream,
                       p.d_a32, p.d_ap32, p.d_ar32, p.d_lofi, p.d_cl, p.lmax, p.nalm, p.Bp,
                       p.omega, lto, mode, p.d_s32, p.d_seb32);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_alm_to_cols_pol(const Plan &p, const double2 *alm, int nb) {
    hipLaunchKernelGGL(k_alm_to_cols_pol, dim3((unsigned)((p.nalm + 63) / 64), (p.Bp + 31) / 32),
                       dim3(256), 0, p.stream, alm, p.d_s32, p.d_seb32, p.nalm, nb, p.Bp);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_cols_to_alm_pol(const Plan &p, double2 *alm, int nb) {
    hipLaunchKernelGGL(k_cols_to_alm_pol, dim3((unsigned)((p.nalm + 63) / 64), (nb + 31) / 32),
                       dim3(256), 0, p.stream, p.d_s32, p.d_seb32, alm, p.nalm, nb, p.Bp);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// The three analysis GEMMs (raw sums into d_a32, d_ap32, d_ar32) from the columns d_ph32,
// d_ph32p; then the combination (filter with lto, or raw) into d_s32, d_seb32.
int pol_analysis_b(const Plan &p, int nb, double lto, int mode) {
    MFWF_TRY(launch_gemm_analysis_raw(p, nb, 2, p.d_lam, p.d_ph32, p.d_a32, 0));
    MFWF_TRY(launch_gemm_analysis_raw(p, nb, 4, p.d_fp, p.d_ph32p, p.d_ap32, 0));
    MFWF_TRY(launch_gemm_analysis_raw(p, nb, 4, p.d_fm, p.d_ph32p, p.d_ar32, 1));
    return launch_pol_combine(p, lto, mode);
}

// The three synthesis GEMMs from d_s32, d_seb32: T into d_ph32, P' into d_ph32p, then R' with
// (Q, U) formed from P' and R' in its epilogue over d_ph32p; rows: then the regrouping into
// T, Q, U rows d_phf.
int pol_synthesis_b(const Plan &p, int nb, bool rows) {
    MFWF_TRY(launch_gemm_synthesis_on(p, nb, 2, p.d_lam, p.d_s32, p.d_ph32, 0));
    MFWF_TRY(launch_gemm_synthesis_on(p, nb, 4, p.d_fp, p.d_seb32, p.d_ph32p, 0));
    MFWF_TRY(launch_gemm_synthesis_on(p, nb, 4, p.d_fm, p.d_seb32, p.d_ph32p, 1, 1));
    return rows ? launch_cols_to_rows_pol(p, nb) : MFWF_OK;
}

}  // namespace mfwf
