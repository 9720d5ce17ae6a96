// Legendre steps of the SHT, FP64 on the vector ALUs (Sect. 3 names the transforms as the
// cost driver, O(nside lmax^2)).
//
//   synthesis  F_{N/S,r}(m) = E_r(m) +/- O_r(m),
//              E = sum_{l+m even} lambda_lm(z_r) s_lm,   O = sum_{l+m odd} lambda_lm(z_r) s_lm
//   analysis   a_lm = sum_pairs lambda_lm(z_r) (G_N + (-1)^{l+m} G_S)_r(m)   (Omega and the
//              sum over pair groups are applied by the harmonic kernel)
//
// lambda_lm(-z) = (-1)^{l+m} lambda_lm(z), so one recurrence serves the north and south
// ring of a pair.  The recurrence lambda_l = alpha_lm z lambda_{l-1} - beta_lm lambda_{l-2}
// runs in FP64, started per (m, pair) at the first l where |lambda_lm| >= 2^-100 from two
// host-computed values (earlier terms are below 2^-100 and are dropped); before its start a
// pair carries lambda = 0 and contributes nothing.
//
// Work split: one 64-lane wave per (pair group g, m-pair); lane L handles ring pairs
// g*64*P + k*64 + L, k < P (adjacent lanes = adjacent latitudes, so start indices are
// close).  Each wave processes m and lmax - m, so every wave walks lmax + 2 values of l.
// The recurrence coefficients and the alm of the current l are wave-uniform loads.
// The analysis reduces over the wave's lanes every C values of l through LDS (transpose
// and sum, fixed order, deterministic).
#include <type_traits>

#include "mfwf_internal.h"

namespace mfwf {

static constexpr int kW = 64;  // wavefront

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

template <int P>
struct PairState {
    double z[P], l1[P], l2[P];
    double2 sd[P];
    int ls[P];
    int lo, hi;  // wave-uniform: first start, last start (capped to lmax + 1)

    __device__ void load(int m, int g, int npair, int lmax, const double *__restrict__ zp,
                         const int *__restrict__ lstart, const double2 *__restrict__ seed) {
        int mylo = lmax + 1, myhi = m;
#pragma unroll
        for (int k = 0; k < P; k++) {
            const int p = g * kW * P + k * kW + (int)threadIdx.x;
            const bool valid = p < npair;
            z[k] = valid ? zp[p] : 0.0;
            ls[k] = valid ? lstart[(long)m * npair + p] : lmax + 1;
            sd[k] = valid ? seed[(long)m * npair + p] : make_double2(0.0, 0.0);
            l1[k] = 0.0;
            l2[k] = 0.0;
            mylo = min(mylo, ls[k]);
            if (ls[k] <= lmax) myhi = max(myhi, ls[k]);
        }
        lo = wave_min(mylo);
        hi = wave_max(myhi);
    }

    // lambda_l for every pair, injecting the seeds at each pair's own start.
    template <bool INJ>
    __device__ __forceinline__ void step(int l, double2 c, double (&cur)[P]) {
#pragma unroll
        for (int k = 0; k < P; k++) {
            double v = c.x * (z[k] * l1[k]) - c.y * l2[k];
            if (INJ) {
                if (l == ls[k]) {
                    v = sd[k].y;
                    l1[k] = sd[k].x;
                }
            }
            l2[k] = l1[k];
            l1[k] = v;
            cur[k] = v;
        }
    }
};

// ---------------------------------------------------------------------------------------
// Synthesis
// ---------------------------------------------------------------------------------------
template <int NB, int P>
__device__ void synth_one_m(int m, int g, const double2 *__restrict__ alm, long nalm,
                            const double2 *__restrict__ ab, const long *__restrict__ mofs,
                            const int *__restrict__ lstart, const double2 *__restrict__ seed,
                            const double *__restrict__ zp, double2 *__restrict__ phase, int lmax,
                            int npair, int nring, int nm, int b0) {
    PairState<P> st;
    st.load(m, g, npair, lmax, zp, lstart, seed);
    const long off = mofs[m] - m;  // packed index of (l, m) = off + l
    const double2 *abm = ab + off;
    double Er[P][NB], Ei[P][NB], Or[P][NB], Oi[P][NB];
#pragma unroll
    for (int k = 0; k < P; k++)
#pragma unroll
        for (int j = 0; j < NB; j++) Er[k][j] = Ei[k][j] = Or[k][j] = Oi[k][j] = 0.0;

    auto run = [&](int la, int lb, auto inj) {
        constexpr bool INJ = decltype(inj)::value;
        for (int l = la; l <= lb; l++) {
            const double2 c = abm[l];
            double cur[P];
            st.template step<INJ>(l, c, cur);
            const bool odd = ((l + m) & 1) != 0;
#pragma unroll
            for (int j = 0; j < NB; j++) {
                const double2 a = alm[(long)(b0 + j) * nalm + off + l];
#pragma unroll
                for (int k = 0; k < P; k++) {
                    if (odd) {
                        Or[k][j] = fma(cur[k], a.x, Or[k][j]);
                        Oi[k][j] = fma(cur[k], a.y, Oi[k][j]);
                    } else {
                        Er[k][j] = fma(cur[k], a.x, Er[k][j]);
                        Ei[k][j] = fma(cur[k], a.y, Ei[k][j]);
                    }
                }
            }
        }
    };
    const int hiA = min(st.hi, lmax);
    run(st.lo, hiA, std::integral_constant<bool, true>{});
    run(max(st.lo, hiA + 1), lmax, std::integral_constant<bool, false>{});

#pragma unroll
    for (int k = 0; k < P; k++) {
        const int p = g * kW * P + k * kW + (int)threadIdx.x;
        if (p >= npair) continue;
        const int rN = p, rS = nring - 1 - p;
#pragma unroll
        for (int j = 0; j < NB; j++) {
            double2 *out = phase + (long)(b0 + j) * nm * nring + (long)m * nring;
            out[rN] = make_double2(Er[k][j] + Or[k][j], Ei[k][j] + Oi[k][j]);
            if (rS != rN) out[rS] = make_double2(Er[k][j] - Or[k][j], Ei[k][j] - Oi[k][j]);
        }
    }
}

template <int NB, int P>
__global__ void __launch_bounds__(kW)
k_leg_synth(const double2 *__restrict__ alm, long nalm, const double2 *__restrict__ ab,
            const long *__restrict__ mofs, const int *__restrict__ lstart,
            const double2 *__restrict__ seed, const double *__restrict__ zp,
            double2 *__restrict__ phase, int lmax, int npair, int nring, int nm) {
    const int g = blockIdx.x, mi = blockIdx.y, b0 = blockIdx.z * NB;
    synth_one_m<NB, P>(mi, g, alm, nalm, ab, mofs, lstart, seed, zp, phase, lmax, npair, nring,
                       nm, b0);
    const int m2 = lmax - mi;
    if (m2 > mi)
        synth_one_m<NB, P>(m2, g, alm, nalm, ab, mofs, lstart, seed, zp, phase, lmax, npair,
                           nring, nm, b0);
}

// ---------------------------------------------------------------------------------------
// Analysis
// ---------------------------------------------------------------------------------------
template <int NB>
struct AnaChunk {
    static constexpr int C = 16 / NB;      // values of l per reduction
    static constexpr int V = 2 * NB * C;   // doubles reduced per lane per chunk (= 32)
    static constexpr int LD = V + 2;       // LDS row stride (keeps 16-byte alignment)
};

template <int NB, int P>
__device__ void analysis_one_m(int m, int g, const double2 *__restrict__ phase, int nring,
                               int nm, const double2 *__restrict__ ab,
                               const long *__restrict__ mofs, const int *__restrict__ lstart,
                               const double2 *__restrict__ seed, const double *__restrict__ zp,
                               double2 *__restrict__ apart, long nalm, int nb_total, int lmax,
                               int npair, int b0, double *red) {
    constexpr int C = AnaChunk<NB>::C, V = AnaChunk<NB>::V, LD = AnaChunk<NB>::LD;
    static_assert(V == 32, "reduction assumes 32 values per lane");
    PairState<P> st;
    st.load(m, g, npair, lmax, zp, lstart, seed);
    const long off = mofs[m] - m;
    const double2 *abm = ab + off;
    // X_even = G_N + G_S (l + m even), X_odd = G_N - G_S; the equator ring counts once.
    double2 Xe[P][NB], Xo[P][NB];
#pragma unroll
    for (int k = 0; k < P; k++) {
        const int p = g * kW * P + k * kW + (int)threadIdx.x;
        const bool valid = p < npair;
        const int rN = p, rS = nring - 1 - p;
#pragma unroll
        for (int j = 0; j < NB; j++) {
            const double2 *G = phase + (long)(b0 + j) * nm * nring + (long)m * nring;
            double2 gN = valid ? G[rN] : make_double2(0.0, 0.0);
            double2 gS = (valid && rS != rN) ? G[rS] : make_double2(0.0, 0.0);
            Xe[k][j] = make_double2(gN.x + gS.x, gN.y + gS.y);
            Xo[k][j] = make_double2(gN.x - gS.x, gN.y - gS.y);
        }
    }
    double2 *outg = apart + (long)g * nb_total * nalm;
    // l in [m, lo') receive no contribution from any pair of this group
    const int lo = st.lo - ((st.lo + m) & 1);  // chunks start at even l + m
    for (int l = m + (int)threadIdx.x; l < min(lo, lmax + 1); l += kW)
#pragma unroll
        for (int j = 0; j < NB; j++) outg[(long)(b0 + j) * nalm + off + l] = make_double2(0.0, 0.0);

    for (int c0 = lo; c0 <= lmax; c0 += C) {
        double acc[V];
#pragma unroll
        for (int v = 0; v < V; v++) acc[v] = 0.0;
        auto chunk = [&](auto inj) {
            constexpr bool INJ = decltype(inj)::value;
#pragma unroll
            for (int c = 0; c < C; c++) {
                const int l = c0 + c;
                if (l > lmax) break;
                const double2 cc = abm[l];
                double cur[P];
                st.template step<INJ>(l, cc, cur);
#pragma unroll
                for (int j = 0; j < NB; j++)
#pragma unroll
                    for (int k = 0; k < P; k++) {
                        const double2 X = (c & 1) ? Xo[k][j] : Xe[k][j];
                        acc[2 * (c * NB + j)] = fma(cur[k], X.x, acc[2 * (c * NB + j)]);
                        acc[2 * (c * NB + j) + 1] = fma(cur[k], X.y, acc[2 * (c * NB + j) + 1]);
                    }
            }
        };
        if (c0 <= st.hi)
            chunk(std::integral_constant<bool, true>{});
        else
            chunk(std::integral_constant<bool, false>{});
        // transpose-reduce across the 64 lanes: lane L sums value v = L/2 over half L%2
#pragma unroll
        for (int v = 0; v < V; v += 2)
            *reinterpret_cast<double2 *>(&red[threadIdx.x * LD + v]) = make_double2(acc[v], acc[v + 1]);
        __syncthreads();
        const int v = threadIdx.x >> 1, h = threadIdx.x & 1;
        double s = 0.0;
#pragma unroll 8
        for (int q = 0; q < 32; q++) s += red[(h * 32 + q) * LD + v];
        s += __shfl_xor(s, 1);
        __syncthreads();
        // v = 2 (c NB + j) + comp
        const int comp = v & 1, cj = v >> 1, c = cj / NB, j = cj - c * NB;
        const int l = c0 + c;
        if (h == 0 && l <= lmax)
            reinterpret_cast<double *>(outg + (long)(b0 + j) * nalm + off + l)[comp] = s;
    }
}

template <int NB, int P>
__global__ void __launch_bounds__(kW)
k_leg_analysis(const double2 *__restrict__ phase, int nring, int nm,
               const double2 *__restrict__ ab, const long *__restrict__ mofs,
               const int *__restrict__ lstart, const double2 *__restrict__ seed,
               const double *__restrict__ zp, double2 *__restrict__ apart, long nalm,
               int nb_total, int lmax, int npair) {
    __shared__ double red[kW * AnaChunk<NB>::LD];
    const int g = blockIdx.x, mi = blockIdx.y, b0 = blockIdx.z * NB;
    analysis_one_m<NB, P>(mi, g, phase, nring, nm, ab, mofs, lstart, seed, zp, apart, nalm,
                          nb_total, lmax, npair, b0, red);
    const int m2 = lmax - mi;
    if (m2 > mi)
        analysis_one_m<NB, P>(m2, g, phase, nring, nm, ab, mofs, lstart, seed, zp, apart, nalm,
                              nb_total, lmax, npair, b0, red);
}

// ---------------------------------------------------------------------------------------
template <int P>
static void synth_launch(const Plan &p, const double2 *alm, double2 *phase, int nb) {
    dim3 grid(p.ngroup, (p.lmax + 2) / 2, nb);
    hipLaunchKernelGGL((k_leg_synth<1, P>), grid, dim3(kW), 0, p.stream, alm, p.nalm, p.d_ab,
                       p.d_mofs, p.d_lstart, p.d_seed, p.d_z, phase, p.lmax, p.npair, p.nring,
                       p.nm);
}

template <int P>
static void analysis_launch(const Plan &p, const double2 *phase, double2 *apart, int nb) {
    dim3 grid(p.ngroup, (p.lmax + 2) / 2, nb);
    hipLaunchKernelGGL((k_leg_analysis<1, P>), grid, dim3(kW), 0, p.stream, phase, p.nring, p.nm,
                       p.d_ab, p.d_mofs, p.d_lstart, p.d_seed, p.d_z, apart, p.nalm, nb,
                       p.lmax, p.npair);
}

int launch_leg_synth(const Plan &p, const double2 *alm, double2 *phase, int nb) {
    switch (p.P) {
        case 1: synth_launch<1>(p, alm, phase, nb); break;
        case 2: synth_launch<2>(p, alm, phase, nb); break;
        case 4: synth_launch<4>(p, alm, phase, nb); break;
        default: set_error("unsupported pairs-per-lane"); return MFWF_EINVAL;
    }
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_leg_analysis(const Plan &p, const double2 *phase, double2 *apart, int nb) {
    switch (p.P) {
        case 1: analysis_launch<1>(p, phase, apart, nb); break;
        case 2: analysis_launch<2>(p, phase, apart, nb); break;
        case 4: analysis_launch<4>(p, phase, apart, nb); break;
        default: set_error("unsupported pairs-per-lane"); return MFWF_EINVAL;
    }
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

}  // namespace mfwf
