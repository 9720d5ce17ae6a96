// Harmonic-space kernels: the signal update of Eq. (4) and the harmonic diagnostics.
//
// With T = tau * 1 in pixel space and analysis A = Omega Y^T, the messenger covariance per
// real harmonic degree of freedom is tau * Omega, so Eq. (4),
//   (S^-1 + (lambda T)^-1) s = (lambda T)^-1 t,  reads  s_lm = C_l / (C_l + lambda tau Omega) a_lm
// with a = A t.  S^-1 is never formed; C_l = 0 gives s_lm = 0.
// The Legendre kernels work with lambda_lm = c_lm mu_lm: partial analysis sums are
// multiplied by c_lm here, and the synthesis input is written pre-multiplied by c_lm.
// Grid (m, map): one block per m row of the packed alm, threads over l.
#include "mfwf_internal.h"

namespace mfwf {

static constexpr int kHT = 256;

// mode 0: s = C/(C + lto) * scale * c * sum_g in_g        (Wiener-filter update, Eq. 4)
// mode 1: s = scale * c * sum_g in_g                       (analysis, scale = Omega)
// mode 2: s = C^{-1/2} * in  (C = 0 -> 0)                  (fluctuation source, h -> C^-1/2 h)
// mode 3: s = in                                           (synthesis input)
// out_s (nullable) <- s;  out_sp (nullable) <- c * s;  prev (nullable) <- old out_s.
__global__ void __launch_bounds__(kHT)
k_harmonic(const double2 *__restrict__ in, int ngroup, long nalm, int nb,
           const long *__restrict__ mofs, const double *__restrict__ cl,
           const double *__restrict__ ctab, int lmax, double scale, double lto, int mode,
           double2 *__restrict__ out_s, double2 *__restrict__ out_sp,
           double2 *__restrict__ prev, const double *__restrict__ tau_b, double lto_per_tau) {
    const int m = blockIdx.x, b = blockIdx.y;
    if (tau_b) lto = lto_per_tau * tau_b[b];  // per-map tau (serving slots)
    const long toff = mofs[m] - m;
    const long base = (long)b * nalm + toff;
    for (int l = m + threadIdx.x; l <= lmax; l += kHT) {
        const long i = base + l;
        const double c = ctab[toff + l];
        double2 a = in[i];
        for (int g = 1; g < ngroup; g++) {
            const double2 q = in[(long)g * nb * nalm + i];
            a.x += q.x;
            a.y += q.y;
        }
        const double C = cl[l];
        double f;
        if (mode == 0) f = C > 0.0 ? C / (C + lto) * scale * c : 0.0;
        else if (mode == 1) f = scale * c;
        else if (mode == 2) f = C > 0.0 ? 1.0 / sqrt(C) : 0.0;
        else f = 1.0;
        const double2 s = make_double2(f * a.x, f * a.y);
        if (prev) prev[i] = out_s[i];
        if (out_s) out_s[i] = s;
        if (out_sp) out_sp[i] = make_double2(c * s.x, c * s.y);
    }
}

int launch_harmonic(const Plan &p, const double2 *in, int ngroup, double scale, double lto,
                    int mode, double2 *out_s, double2 *out_sp, double2 *prev, int nb,
                    double lto_per_tau) {
    hipLaunchKernelGGL(k_harmonic, dim3(p.nm, nb), dim3(kHT), 0, p.stream, in, ngroup, p.nalm,
                       nb, p.d_mofs, p.d_cl, p.d_c, p.lmax, scale, lto, mode, out_s, out_sp,
                       prev, mode == 0 ? p.d_tau : nullptr, lto_per_tau);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// Per (m, map) partial sums over the real harmonic dof (m > 0 counted twice):
//   [0] s^T S^-1 s = sum |s_lm|^2 / C_l  (C_l > 0),  [1] |s - prev|^2,  [2] |s|^2
__global__ void __launch_bounds__(kHT)
k_harm_diag(const double2 *__restrict__ s, const double2 *__restrict__ prev, long nalm,
            const long *__restrict__ mofs, const double *__restrict__ cl, int lmax, int nm,
            double *__restrict__ partial) {
    __shared__ double sh[3][kHT];
    const int m = blockIdx.x, b = blockIdx.y;
    const long base = (long)b * nalm + mofs[m] - m;
    const double w = (m == 0) ? 1.0 : 2.0;
    double h = 0.0, d = 0.0, n = 0.0;
    for (int l = m + threadIdx.x; l <= lmax; l += kHT) {
        const double2 v = s[base + l], u = prev[base + l];
        const double q = v.x * v.x + v.y * v.y;
        if (cl[l] > 0.0) h += q / cl[l];
        d += (v.x - u.x) * (v.x - u.x) + (v.y - u.y) * (v.y - u.y);
        n += q;
    }
    sh[0][threadIdx.x] = h;
    sh[1][threadIdx.x] = d;
    sh[2][threadIdx.x] = n;
    __syncthreads();
    for (int o = kHT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 3) partial[((long)b * nm + m) * 3 + threadIdx.x] = w * sh[threadIdx.x][0];
}

// diag[b][1..3] = sums over m in fixed order
__global__ void k_harm_diag_final(const double *__restrict__ partial, int nm, int nb,
                                  double *__restrict__ diag) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double h = 0.0, d = 0.0, n = 0.0;
    for (int m = 0; m < nm; m++) {
        h += partial[((long)b * nm + m) * 3 + 0];
        d += partial[((long)b * nm + m) * 3 + 1];
        n += partial[((long)b * nm + m) * 3 + 2];
    }
    diag[8 * b + 1] = h;
    diag[8 * b + 2] = d;
    diag[8 * b + 3] = n;
}

int launch_harm_diag(const Plan &p, const double2 *salm, const double2 *salm_prev, int nb,
                     double *partial, double *diag) {
    hipLaunchKernelGGL(k_harm_diag, dim3(p.nm, nb), dim3(kHT), 0, p.stream, salm, salm_prev,
                       p.nalm, p.d_mofs, p.d_cl, p.lmax, p.nm, partial);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_harm_diag_final, dim3((nb + 63) / 64), dim3(64), 0, p.stream, partial,
                       p.nm, nb, diag);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// Coefficients of rows (maps x components) from the packing of one band limit to another:
// dst[r][m, l] = src[r][m, l] for l <= lsrc, 0 above (m-major, l = m..lmax in both).
__global__ void k_repack_alm(const double2 *__restrict__ src, const long *__restrict__ mofs_src,
                             long nsrc, int lsrc, double2 *__restrict__ dst,
                             const long *__restrict__ mofs_dst, long ndst, int ldst) {
    const int m = blockIdx.x;
    const long r = blockIdx.y;
    const long od = r * ndst + mofs_dst[m] - m;
    const long os = (m <= lsrc) ? r * nsrc + mofs_src[m] - m : 0;
    for (int l = m + threadIdx.x; l <= ldst; l += kHT)
        dst[od + l] = (l <= lsrc) ? src[os + l] : make_double2(0.0, 0.0);
}

int launch_repack_alm(const Plan &src, const double2 *a_src, const Plan &dst, double2 *a_dst,
                      int rows) {
    hipLaunchKernelGGL(k_repack_alm, dim3(dst.nm, rows), dim3(kHT), 0, dst.stream, a_src,
                       src.d_mofs, src.nalm, src.lmax, a_dst, dst.d_mofs, dst.nalm, dst.lmax);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

}  // namespace mfwf
