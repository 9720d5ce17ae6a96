// Monopole and dipole template removal of Eq. (12):
//   d = lim_{sigma -> inf} (1 + sigma V V^T)^{-1} d_raw,  V = (1, x, y, z) on observed pixels,
// (x, y, z) the unit vector of the pixel centre.  By the Woodbury identity the limit is the
// projection d_raw - V (V^T V)^{-1} V^T d_raw: the sums V^T V (10 distinct entries) and
// V^T d (4 per map) come from one pass over the map, the 4 x 4 solve is done on the host,
// the subtraction is a second pass.  Pixel positions come from the ring-pair tables (the
// north and south rings of a pair share n_phi and phi_0 and have opposite z).
// For T, Q, U maps the templates apply to T; Q and U pass through.
#include <mutex>

#include "mfwf_internal.h"

namespace mfwf {

static constexpr int kTG = 64;   // pair groups of the first pass (one workgroup each per map)
static constexpr int kTT = 256;  // threads per workgroup

__device__ __forceinline__ bool observed_pixel(const double *__restrict__ M, int spin, long i) {
    if (spin == 2) return M[6 * i] > 0.0 || M[6 * i + 3] > 0.0 || M[6 * i + 5] > 0.0;
    return M[i] > 0.0;
}

// template values at pixel j of a ring with n pixels, phi_0 = pi / n if hs, cos theta = z
__device__ __forceinline__ void template_values(int j, int n, int hs, double z, double s,
                                                double v[4]) {
    double sn, cs;
    sincospi((double)(2 * j + hs) / (double)n, &sn, &cs);  // phi = phi_0 + 2 pi j / n
    v[0] = 1.0;
    v[1] = s * cs;
    v[2] = s * sn;
    v[3] = z;
}

// partial[b][g][0..9] = upper triangle of V^T V, [10..13] = V^T d, over pairs g, g + kTG, ...
__global__ void __launch_bounds__(kTT)
k_template_sums(const PairFFT *__restrict__ pfft, const double *__restrict__ zp,
                const double *__restrict__ M, int spin, const double *__restrict__ d,
                long mapstride, int npair, double *__restrict__ partial) {
    __shared__ double sh[14][kTT];
    const int g = blockIdx.x, b = blockIdx.y;
    double acc[14];
#pragma unroll
    for (int k = 0; k < 14; k++) acc[k] = 0.0;
    const double *db = d + (long)b * mapstride;
    for (int p = g; p < npair; p += kTG) {
        const PairFFT pf = pfft[p];
        const double z = zp[p], s = sqrt((1.0 - z) * (1.0 + z));
        const int nh = (pf.startS == pf.startN) ? 1 : 2;
        for (int h = 0; h < nh; h++) {
            const long st = h ? pf.startS : pf.startN;
            for (int j = threadIdx.x; j < pf.nphi; j += kTT) {
                const long i = st + j;
                if (!observed_pixel(M, spin, i)) continue;
                double v[4];
                template_values(j, pf.nphi, pf.half_shift, h ? -z : z, s, v);
                const double x = db[i];
                int k = 0;
#pragma unroll
                for (int a = 0; a < 4; a++)
#pragma unroll
                    for (int c = a; c < 4; c++) acc[k++] += v[a] * v[c];
#pragma unroll
                for (int a = 0; a < 4; a++) acc[10 + a] += v[a] * x;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 14; k++) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = kTT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 14; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 14) partial[((long)b * kTG + g) * 14 + threadIdx.x] = sh[threadIdx.x][0];
}

// out[b][k] = sum over the groups in fixed order
__global__ void k_template_final(const double *__restrict__ partial, int nb,
                                 double *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 14 * nb) return;
    const int b = e / 14, k = e - 14 * b;
    double s = 0.0;
    for (int g = 0; g < kTG; g++) s += partial[((long)b * kTG + g) * 14 + k];
    out[e] = s;
}

// d_out = d - V coef[b] on observed pixels (T), d elsewhere; Q, U copied for spin 2
__global__ void __launch_bounds__(kTT)
k_template_subtract(const PairFFT *__restrict__ pfft, const double *__restrict__ zp,
                    const double *__restrict__ M, int spin, const double *__restrict__ d,
                    double *__restrict__ dout, long npix, long mapstride,
                    const double *__restrict__ coef) {
    const int p = blockIdx.x, b = blockIdx.y;
    const PairFFT pf = pfft[p];
    const double z = zp[p], s = sqrt((1.0 - z) * (1.0 + z));
    const double k0 = coef[4 * b], k1 = coef[4 * b + 1], k2 = coef[4 * b + 2], k3 = coef[4 * b + 3];
    const double *db = d + (long)b * mapstride;
    double *ob = dout + (long)b * mapstride;
    const int nh = (pf.startS == pf.startN) ? 1 : 2;
    for (int h = 0; h < nh; h++) {
        const long st = h ? pf.startS : pf.startN;
        for (int j = threadIdx.x; j < pf.nphi; j += kTT) {
            const long i = st + j;
            double x = db[i];
            if (observed_pixel(M, spin, i)) {
                double v[4];
                template_values(j, pf.nphi, pf.half_shift, h ? -z : z, s, v);
                x -= k0 * v[0] + k1 * v[1] + k2 * v[2] + k3 * v[3];
            }
            ob[i] = x;
            if (spin == 2) {
                ob[npix + i] = db[npix + i];
                ob[2 * npix + i] = db[2 * npix + i];
            }
        }
    }
}

int launch_template_sums(const Plan &p, const double *d, int nb, double *partial, double *out14) {
    const long mapstride = (long)p.ncomp * p.npix;
    hipLaunchKernelGGL(k_template_sums, dim3(kTG, nb), dim3(kTT), 0, p.stream, p.d_pfft, p.d_z,
                       p.d_M, p.spin, d, mapstride, p.npair, partial);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_template_final, dim3((14 * nb + 255) / 256), dim3(256), 0, p.stream,
                       partial, nb, out14);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int template_partial_doubles(int nb) { return kTG * 14 * nb; }

int launch_template_subtract(const Plan &p, const double *d, double *dout, int nb,
                             const double *coef) {
    hipLaunchKernelGGL(k_template_subtract, dim3(p.npair, nb), dim3(kTT), 0, p.stream, p.d_pfft,
                       p.d_z, p.d_M, p.spin, d, dout, p.npix, (long)p.ncomp * p.npix, coef);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// ---- allocation-free variant -------------------------------------------------------------
// For callers that cannot allocate device memory: the same removal with every intermediate
// (per map kTG x 14 partial sums, the 14 totals, the 4 template coefficients and a status
// flag) in one file-scope device array of fixed size, and the 4 x 4 solve on the device.
// Every value is written before it is read, so nothing needs clearing between calls.  Each
// device holds its own copy of the array for the life of the process; calls that overlap on
// one device (two streams, two host threads) race on it.
static constexpr int kNaPartial = kTG * 14;                    // doubles per map
static constexpr long kNaOffTot = (long)kNoAllocMaxMaps * kNaPartial;
static constexpr long kNaOffCoef = kNaOffTot + 14L * kNoAllocMaxMaps;
static constexpr long kNaOffFlag = kNaOffCoef + 4L * kNoAllocMaxMaps;
static constexpr long kNaDoubles = kNaOffFlag + kNoAllocMaxMaps;  // 467,968 bytes
static __device__ __align__(256) double scratch[kNaDoubles];

// Per map b < nb: G = V^T V from its upper triangle u[0..9], c = V^T d = u[10..13];
// G = L L^T, G k = c; flag[b] = 1 (and k = 0) when a pivot falls to 1e-12 of the trace,
// i.e. the templates are degenerate on the observed pixels.
__global__ void k_template_solve(const double *__restrict__ tot, int nb,
                                 double *__restrict__ coef, double *__restrict__ flag) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double *u = tot + 14L * b;
    double G[4][4], L[4][4], y[4], k[4];
    int q = 0;
    for (int a = 0; a < 4; a++)
        for (int e = a; e < 4; e++) G[a][e] = G[e][a] = u[q++];
    const double trace = G[0][0] + G[1][1] + G[2][2] + G[3][3];
    bool ok = true;
    for (int i = 0; i < 4; i++) {
        for (int j = 0; j < 4; j++) L[i][j] = 0.0;
        for (int j = 0; j <= i; j++) {
            double v = G[i][j];
            for (int t = 0; t < j; t++) v -= L[i][t] * L[j][t];
            if (i == j) {
                ok = ok && (v > 1e-12 * trace);
                L[i][i] = ok ? sqrt(v) : 1.0;
            } else {
                L[i][j] = v / L[j][j];
            }
        }
    }
    for (int i = 0; i < 4; i++) {  // L y = c
        double v = u[10 + i];
        for (int t = 0; t < i; t++) v -= L[i][t] * y[t];
        y[i] = v / L[i][i];
    }
    for (int i = 3; i >= 0; i--) {  // L^T k = y
        double v = y[i];
        for (int t = i + 1; t < 4; t++) v -= L[t][i] * k[t];
        k[i] = v / L[i][i];
    }
    for (int i = 0; i < 4; i++) coef[4L * b + i] = ok ? k[i] : 0.0;
    flag[b] = ok ? 0.0 : 1.0;
}

// Device address of this device's copy of the array, looked up once per device with that
// device current (the array's name is only a host-side handle).
static int noalloc_scratch(int device, double **out) {
    static std::mutex mu;
    static double *addr[64] = {};
    if (device < 0 || device >= 64) return fail(MFWF_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void *ptr = nullptr;
        MFWF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        addr[device] = static_cast<double *>(ptr);
    }
    *out = addr[device];
    return MFWF_OK;
}

static int remove_templates_noalloc_on(const Plan &p, const double *d_raw, double *d_out,
                                       int nmaps) {
    double *ws = nullptr;
    MFWF_TRY(noalloc_scratch(p.device, &ws));
    double *partial = ws, *tot = ws + kNaOffTot, *coef = ws + kNaOffCoef, *flag = ws + kNaOffFlag;
    MFWF_TRY(launch_template_sums(p, d_raw, nmaps, partial, tot));
    hipLaunchKernelGGL(k_template_solve, dim3(1), dim3(kNoAllocMaxMaps), 0, p.stream, tot, nmaps,
                       coef, flag);
    MFWF_HIP(hipGetLastError());
    MFWF_TRY(launch_template_subtract(p, d_raw, d_out, nmaps, coef));
    double hflag[kNoAllocMaxMaps];
    MFWF_HIP(hipMemcpyAsync(hflag, flag, sizeof(double) * nmaps, hipMemcpyDeviceToHost, p.stream));
    MFWF_HIP(hipStreamSynchronize(p.stream));
    for (int b = 0; b < nmaps; b++)
        if (hflag[b] != 0.0)
            return fail(MFWF_EINVAL, "the monopole and dipole templates are degenerate on the "
                                     "observed pixels (map " + std::to_string(b) + ")");
    return MFWF_OK;
}

int remove_templates_noalloc(const Plan &p, const double *d_raw, double *d_out, int nmaps) {
    static_assert(kNoAllocMaxMaps <= 1024, "one workgroup solves every map");
    if (nmaps > kNoAllocMaxMaps)
        return fail(MFWF_EINVAL, "at most " + std::to_string(kNoAllocMaxMaps) +
                                     " maps per call (fixed device scratch), got " +
                                     std::to_string(nmaps));
    int cur = 0;
    MFWF_HIP(hipGetDevice(&cur));
    if (cur == p.device) return remove_templates_noalloc_on(p, d_raw, d_out, nmaps);
    MFWF_HIP(hipSetDevice(p.device));  // the plan's stream and the array copy live there
    const int st = remove_templates_noalloc_on(p, d_raw, d_out, nmaps);
    MFWF_HIP(hipSetDevice(cur));
    return st;
}

}  // namespace mfwf
