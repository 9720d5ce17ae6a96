// Per-lane state of the rescaled Legendre recurrence shared by the temperature and the
// polarization kernels: mu_l = A_lm z mu_{l-1} - mu_{l-2}, lambda_lm = c_lm mu_lm, started
// at each (m, ring pair)'s first non-negligible l from two stored values.
#pragma once

#include "mfwf_internal.h"

namespace mfwf {

static constexpr int kW = 64;  // wavefront

__device__ __forceinline__ int wave_min_uniform(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_max_uniform(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return __builtin_amdgcn_readfirstlane(v);
}

template <int P>
struct PairState {
    double z[P], u1[P], u2[P];  // mu_{l-1}, mu_{l-2}
    double2 sd[P];              // (mu_{l_s - 1}, mu_{l_s})
    int ls[P];
    int lo, hi;  // wave-uniform: smallest start, largest start <= lmax (m if none)

    __device__ __forceinline__ void load(int m, int g, int npair, int lmax,
                                         const double *__restrict__ zp,
                                         const int *__restrict__ lstart,
                                         const double2 *__restrict__ seed) {
        int mylo = lmax + 1, myhi = m;
#pragma unroll
        for (int k = 0; k < P; k++) {
            const int p = g * kW * P + k * kW + (int)threadIdx.x;
            const bool valid = p < npair;
            z[k] = valid ? zp[p] : 0.0;
            ls[k] = valid ? lstart[(long)m * npair + p] : lmax + 1;
            sd[k] = valid ? seed[(long)m * npair + p] : make_double2(0.0, 0.0);
            u1[k] = 0.0;
            u2[k] = 0.0;
            mylo = min(mylo, ls[k]);
            if (ls[k] <= lmax) myhi = max(myhi, ls[k]);
        }
        lo = wave_min_uniform(mylo);
        hi = wave_max_uniform(myhi);
    }

    // mu_l for every pair, injecting the seeds at each pair's own start.  The two forms
    // associate A z mu differently on purpose: the blocks with and without injection then
    // share no subexpression, so the compiler cannot hoist a whole block's A z products
    // above the branch (that costs 2 U P registers and halves occupancy).
    template <bool INJ>
    __device__ __forceinline__ void step(int l, double A, double (&cur)[P]) {
#pragma unroll
        for (int k = 0; k < P; k++) {
            double v;
            if (INJ) {
                v = fma(A * z[k], u1[k], -u2[k]);
                const bool start = (l == ls[k]);
                v = start ? sd[k].y : v;
                u1[k] = start ? sd[k].x : u1[k];
            } else {
                v = fma(A, z[k] * u1[k], -u2[k]);
            }
            u2[k] = u1[k];
            u1[k] = v;
            cur[k] = v;
        }
    }
};

// (x, y) of every lane after exchanging lanes 32..63 of x with lanes 0..31 of y (SWAP32),
// or the odd 16-lane rows of x with the even rows of y (v_permlane{32,16}_swap, one 32-bit
// half at a time): x + y then holds x summed over lanes L and L + 32 (L + 16) in the lower
// lanes (even rows) and y summed over L - 32 (L - 16) and L in the upper lanes (odd rows).
template <bool SWAP32>
__device__ __forceinline__ double swap_add(double x, double y) {
    const unsigned long long a = __double_as_longlong(x), b = __double_as_longlong(y);
    const unsigned alo = (unsigned)a, ahi = (unsigned)(a >> 32), blo = (unsigned)b, bhi = (unsigned)(b >> 32);
    unsigned xl, yl, xh, yh;
    if constexpr (SWAP32) {
        const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
        xl = l[0], yl = l[1], xh = h[0], yh = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
        xl = l[0], yl = l[1], xh = h[0], yh = h[1];
    }
    return __longlong_as_double(((unsigned long long)xh << 32) | xl) +
           __longlong_as_double(((unsigned long long)yh << 32) | yl);
}

}  // namespace mfwf
