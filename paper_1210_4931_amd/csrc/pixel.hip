// Pixel-space kernels: the messenger update of Eq. (3), the chi^2 pixel term of Eq. (6),
// covariance set-up and the pixel part of the fluctuation source of Eq. (9).
// All of them stream RING-ordered [nb][npix] double arrays: HBM-bound, grid-stride loops
// with coalesced 8-byte accesses, FP64 reductions in a fixed order (deterministic).
#include "mfwf_internal.h"

namespace mfwf {

static constexpr int kThreads = 256;

static int grid_for(long n) {
    long g = (n + kThreads - 1) / kThreads;
    if (g > 8192) g = 8192;  // enough blocks to fill 256 CUs many times over
    if (g < 1) g = 1;
    return (int)g;
}

__global__ void k_fill(double *__restrict__ x, long n, double v) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        x[i] = v;
}

int launch_fill(double *x, long n, double v, hipStream_t s) {
    if (n <= 0) return MFWF_OK;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, x, n, v);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

__global__ void k_mask_product(const double *__restrict__ ninv, const uint8_t *__restrict__ mask,
                               double *__restrict__ M, long npix) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < npix;
         i += (long)gridDim.x * blockDim.x)
        M[i] = (mask == nullptr || mask[i] != 0) ? ninv[i] : 0.0;
}

int launch_mask_product(const double *ninv, const uint8_t *mask, double *M, long npix,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_mask_product, dim3(grid_for(npix)), dim3(kThreads), 0, s, ninv, mask,
                       M, npix);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// Block reduction of a few doubles through LDS, fixed tree order.
template <int K>
__device__ void block_sum(double (&v)[K], double (*sh)[kThreads]) {
    for (int k = 0; k < K; k++) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < K; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    for (int k = 0; k < K; k++) v[k] = sh[k][0];
}

// partial[block] = (max M, #(M > 0), #(M non-finite or negative))
__global__ void k_max_count(const double *__restrict__ M, long npix, double *__restrict__ partial) {
    __shared__ double sh[3][kThreads];
    double mx = 0.0, cnt = 0.0, bad = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < npix;
         i += (long)gridDim.x * blockDim.x) {
        double m = M[i];
        if (!(m >= 0.0) || isinf(m)) bad += 1.0;
        else {
            mx = fmax(mx, m);
            cnt += (m > 0.0) ? 1.0 : 0.0;
        }
    }
    sh[0][threadIdx.x] = mx;
    sh[1][threadIdx.x] = cnt;
    sh[2][threadIdx.x] = bad;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x + 0] = sh[0][0];
        partial[3 * blockIdx.x + 1] = sh[1][0];
        partial[3 * blockIdx.x + 2] = sh[2][0];
    }
}

__global__ void k_max_count_final(const double *__restrict__ partial, int nblocks,
                                  double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double mx = 0.0, cnt = 0.0, bad = 0.0;
    for (int b = 0; b < nblocks; b++) {
        mx = fmax(mx, partial[3 * b]);
        cnt += partial[3 * b + 1];
        bad += partial[3 * b + 2];
    }
    out[0] = mx;
    out[1] = cnt;
    out[2] = bad;
}

int launch_reduce_max_count(const double *M, long npix, double *partial, int nblocks,
                            double *out3, hipStream_t s) {
    hipLaunchKernelGGL(k_max_count, dim3(nblocks), dim3(kThreads), 0, s, M, npix, partial);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_max_count_final, dim3(1), dim3(64), 0, s, partial, nblocks, out3);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// Non-finite entries of x[0..n) per block (a solve's source rho: data on masked pixels has
// already been dropped there, so only observed pixels count), then their total.
__global__ void k_count_nonfinite(const double *__restrict__ x, long n, double *__restrict__ partial) {
    __shared__ double sh[kThreads];
    double bad = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        bad += isfinite(x[i]) ? 0.0 : 1.0;
    sh[threadIdx.x] = bad;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(const double *__restrict__ partial, int nblocks, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; b++) s += partial[b];
    out[0] = s;
}

int launch_count_nonfinite(const double *x, long n, double *partial, int nblocks, double *out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_count_nonfinite, dim3(nblocks), dim3(kThreads), 0, s, x, n, partial);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, s, partial, nblocks, out);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

__global__ void k_rho_from_data(const double *__restrict__ d, const double *__restrict__ M,
                                double *__restrict__ rho, long npix, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        double m = M[i % npix];
        // masked pixels: rho = 0 whatever d holds there (M d with M = 0, even for d = inf)
        rho[i] = m > 0.0 ? m * d[i] : 0.0;
    }
}

int launch_rho_from_data(const double *d, const double *M, double *rho, long npix, int nb,
                         hipStream_t s) {
    long n = npix * nb;
    hipLaunchKernelGGL(k_rho_from_data, dim3(grid_for(n)), dim3(kThreads), 0, s, d, M, rho,
                       npix, n);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// chi^2 pixel term of Eq. (6): sum over observed pixels of (d - s)^2 / (N + (lam - 1) tau)
// with d = rho / M, i.e. (rho - M s)^2 / (M (1 + (lam - 1) tau M)).
// grid (nblocks, nb): partial[b][block]
__global__ void k_chi2_pix(const double *__restrict__ rho, const double *__restrict__ M,
                           const double *__restrict__ smap, long npix, double lam, double tau,
                           double *__restrict__ partial) {
    __shared__ double sh[1][kThreads];
    const long off = (long)blockIdx.y * npix;
    double acc[1] = {0.0};
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < npix;
         i += (long)gridDim.x * blockDim.x) {
        double m = M[i];
        if (m > 0.0) {
            double r = rho[off + i] - m * smap[off + i];
            acc[0] += r * r / (m * (1.0 + (lam - 1.0) * tau * m));
        }
    }
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
}

// diag[b][0] = sum_block partial[b][block]  (one thread per map, fixed order)
__global__ void k_sum_partials(const double *__restrict__ partial, int nblocks, int nb,
                               double *__restrict__ diag, int slot) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double acc = 0.0;
    for (int k = 0; k < nblocks; k++) acc += partial[(long)b * nblocks + k];
    diag[8 * b + slot] = acc;
}

int launch_chi2_pix(const double *rho, const double *M, const double *smap, long npix, int nb,
                    double lam, double tau, double *partial, int nblocks, double *diag,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_chi2_pix, dim3(nblocks, nb), dim3(kThreads), 0, s, rho, M, smap, npix,
                       lam, tau, partial);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials, dim3((nb + 63) / 64), dim3(64), 0, s, partial, nblocks,
                       nb, diag, 0);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// Pixel term of chi^2(lambda, s) (Eq. 6) and its derivative in lambda, for the error-bound
// schedule of Sect. 2.2: with r = rho - M s and u = tau M on observed pixels,
//   P = sum r^2 / (M (1 + (lam - 1) u)),  dP/dlam = -sum r^2 tau / (1 + (lam - 1) u)^2.
// partial[b][block][2]; k_sum_pairs adds the blocks in fixed order into out[b][2].
__global__ void k_chi2_pix_dlam(const double *__restrict__ rho, const double *__restrict__ M,
                                const double *__restrict__ smap, long npix, double lam,
                                double tau, double *__restrict__ partial) {
    __shared__ double sh[2][kThreads];
    const long off = (long)blockIdx.y * npix;
    double acc[2] = {0.0, 0.0};
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < npix;
         i += (long)gridDim.x * blockDim.x) {
        const double m = M[i];
        if (m > 0.0) {
            const double r = rho[off + i] - m * smap[off + i];
            const double q = 1.0 / (1.0 + (lam - 1.0) * tau * m);
            acc[0] += r * r / m * q;
            acc[1] -= r * r * tau * q * q;
        }
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        const long o = ((long)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        partial[o] = acc[0];
        partial[o + 1] = acc[1];
    }
}

__global__ void k_sum_pairs(const double *__restrict__ partial, int nblocks, int nb,
                            double *__restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double a = 0.0, c = 0.0;
    for (int k = 0; k < nblocks; k++) {
        a += partial[((long)b * nblocks + k) * 2];
        c += partial[((long)b * nblocks + k) * 2 + 1];
    }
    out[2 * b] = a;
    out[2 * b + 1] = c;
}

int launch_sum_pairs(const double *partial, int nblocks, int nb, double *out2, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_pairs, dim3((nb + 63) / 64), dim3(64), 0, s, partial, nblocks, nb, out2);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_chi2_pix_dlam(const double *rho, const double *M, const double *smap, long npix,
                         int nb, double lam, double tau, double *partial, int nblocks,
                         double *out2, hipStream_t s) {
    hipLaunchKernelGGL(k_chi2_pix_dlam, dim3(nblocks, nb), dim3(kThreads), 0, s, rho, M, smap,
                       npix, lam, tau, partial);
    MFWF_HIP(hipGetLastError());
    return launch_sum_pairs(partial, nblocks, nb, out2, s);
}

// rho = M^{1/2} g1 + Omega * (Y C^{-1/2} h)  (Eq. 9 in per-pixel form)
__global__ void k_fluct_combine(const double *__restrict__ g1, const double *__restrict__ M,
                                const double *__restrict__ ysh, double *__restrict__ rho,
                                long npix, long n, double omega) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        rho[i] = sqrt(M[i % npix]) * g1[i] + omega * ysh[i];
}

int launch_fluct_combine(const double *g1, const double *M, const double *ysh, double *rho,
                         long npix, int nb, double omega, hipStream_t s) {
    long n = npix * nb;
    hipLaunchKernelGGL(k_fluct_combine, dim3(grid_for(n)), dim3(kThreads), 0, s, g1, M, ysh,
                       rho, npix, n, omega);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

}  // namespace mfwf
