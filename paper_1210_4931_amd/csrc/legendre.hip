// Legendre steps of the SHT, FP64 on the vector ALUs (Sect. 3 names the transforms as the
// cost driver, O(nside lmax^2)).
//
//   synthesis  F_{N/S,r}(m) = E_r(m) +/- O_r(m),
//              E = sum_{l+m even} lambda_lm(z_r) s_lm,   O = sum_{l+m odd} lambda_lm(z_r) s_lm
//   analysis   a_lm = sum_pairs lambda_lm(z_r) (G_N + (-1)^{l+m} G_S)_r(m)
//
// lambda_lm(-z) = (-1)^{l+m} lambda_lm(z), so one recurrence serves the north and south
// ring of a pair.  The orthonormal recurrence
//     lambda_l = alpha_lm z lambda_{l-1} - beta_lm lambda_{l-2}
// is run in the rescaled form lambda_l = c_lm mu_l with c_l = beta_l c_{l-2}
// (c_m = c_{m+1} = 1), which turns it into
//     mu_l = A_lm z mu_{l-1} - mu_{l-2},   A_lm = alpha_lm c_{l-1} / c_l,
// two FP64 operations per (l, ring pair) instead of three.  The synthesis reads the
// c-scaled coefficients c_lm s_lm and the analysis returns sum mu_l X, which the harmonic
// kernel multiplies by c_lm.  Each (m, pair) starts at the first l where |lambda_lm| >= 2^-100,
// from two host-computed values (mu_{l_s - 1}, mu_{l_s}); earlier terms are below 2^-100 and
// are dropped, and a pair carries mu = 0 (no contribution) before its start.
//
// Work split: one 64-lane wave per (pair group g, m-pair); lane L handles ring pairs
// g*64*P + k*64 + L, k < P (adjacent lanes = adjacent latitudes, so start indices are
// close).  Each wave processes m and lmax - m, so every wave walks lmax + 2 values of l.
// The l loop is wave-uniform: its bounds come through readfirstlane, so it runs on the
// scalar unit and A_lm and the coefficients of each l are scalar loads, fetched U values of
// l at a time (optionally one block ahead).  Blocks start at even l + m, so the even/odd
// split is fixed at compile time inside a block.  Lanes inject their seeds only in blocks
// that can contain a start index.
// The analysis reduces over the wave's lanes every C values of l through LDS (transpose
// and sum, fixed order, deterministic).
#include <type_traits>

#include "leg_core.h"

namespace mfwf {

// ---------------------------------------------------------------------------------------
// Synthesis
// ---------------------------------------------------------------------------------------
template <int NB, int P>
struct SynthAcc {
    double Er[P][NB], Ei[P][NB], Or[P][NB], Oi[P][NB];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < P; k++)
#pragma unroll
            for (int j = 0; j < NB; j++) Er[k][j] = Ei[k][j] = Or[k][j] = Oi[k][j] = 0.0;
    }
    template <bool ODD>
    __device__ __forceinline__ void add(const double (&cur)[P], const double2 (&a)[NB]) {
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
            for (int k = 0; k < P; k++) {
                if (ODD) {
                    Or[k][j] = fma(cur[k], a[j].x, Or[k][j]);
                    Oi[k][j] = fma(cur[k], a[j].y, Oi[k][j]);
                } else {
                    Er[k][j] = fma(cur[k], a[j].x, Er[k][j]);
                    Ei[k][j] = fma(cur[k], a[j].y, Ei[k][j]);
                }
            }
    }
};

template <int NB, int U>
struct SynthBlockData {
    double A[U];
    double2 a[U][NB];
    __device__ __forceinline__ void fetch(int l, const double *__restrict__ Am,
                                          const double2 *const (&am)[NB]) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            A[u] = Am[l + u];
#pragma unroll
            for (int j = 0; j < NB; j++) a[u][j] = am[j][l + u];
        }
    }
};

template <int NB, int P, int U, bool INJ>
__device__ __forceinline__ void synth_block(int l, PairState<P> &st, SynthAcc<NB, P> &acc,
                                            const SynthBlockData<NB, U> &bd) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        double cur[P];
        st.template step<INJ>(l + u, bd.A[u], cur);
        if (u & 1)
            acc.template add<true>(cur, bd.a[u]);
        else
            acc.template add<false>(cur, bd.a[u]);
    }
}

template <int NB, int P, int U, bool PF>
__device__ __forceinline__ void synth_one_m(int m, int g, const double2 *__restrict__ alm,
                                            long nalm, const double *__restrict__ Atab,
                                            const long *__restrict__ mofs,
                                            const int *__restrict__ lstart,
                                            const double2 *__restrict__ seed,
                                            const double *__restrict__ zp,
                                            double2 *__restrict__ phase, int lmax, int npair,
                                            int nring, int nm, int b0) {
    PairState<P> st;
    st.load(m, g, npair, lmax, zp, lstart, seed);
    const long off = mofs[m] - m;  // packed index of (l, m) = off + l
    const double *Am = Atab + off;
    const double2 *am[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) am[j] = alm + (long)(b0 + j) * nalm + off;
    SynthAcc<NB, P> acc;
    acc.zero();

    int l = st.lo - ((st.lo + m) & 1);  // even l + m; mu = 0 there for every lane
    if (PF) {
        SynthBlockData<NB, U> cur, nxt;
        if (l + U - 1 <= lmax) cur.fetch(l, Am, am);
        for (; l + U - 1 <= lmax; l += U) {
            const bool more = l + 2 * U - 1 <= lmax;
            if (more) nxt.fetch(l + U, Am, am);
            if (l <= st.hi)
                synth_block<NB, P, U, true>(l, st, acc, cur);
            else
                synth_block<NB, P, U, false>(l, st, acc, cur);
            if (more) cur = nxt;
        }
    } else {
        for (; l + U - 1 <= lmax; l += U) {
            SynthBlockData<NB, U> cur;
            cur.fetch(l, Am, am);
            if (l <= st.hi)
                synth_block<NB, P, U, true>(l, st, acc, cur);
            else
                synth_block<NB, P, U, false>(l, st, acc, cur);
        }
    }
    for (; l <= lmax; l++) {  // tail: fewer than U values of l
        double2 a[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) a[j] = am[j][l];
        double cur[P];
        st.template step<true>(l, Am[l], cur);
        if ((l + m) & 1)
            acc.template add<true>(cur, a);
        else
            acc.template add<false>(cur, a);
    }

#pragma unroll
    for (int k = 0; k < P; k++) {
        const int p = g * kW * P + k * kW + (int)threadIdx.x;
        if (p >= npair) continue;
        const int rN = p, rS = nring - 1 - p;
#pragma unroll
        for (int j = 0; j < NB; j++) {
            // ring-Fourier layout [map][ring][m]
            double2 *out = phase + (long)(b0 + j) * nm * nring + m;
            out[(long)rN * nm] = make_double2(acc.Er[k][j] + acc.Or[k][j], acc.Ei[k][j] + acc.Oi[k][j]);
            if (rS != rN)
                out[(long)rS * nm] = make_double2(acc.Er[k][j] - acc.Or[k][j], acc.Ei[k][j] - acc.Oi[k][j]);
        }
    }
}

template <int NB, int P, int U, bool PF>
__global__ void __launch_bounds__(kW)
k_leg_synth(const double2 *__restrict__ alm, long nalm, const double *__restrict__ Atab,
            const long *__restrict__ mofs, const int *__restrict__ lstart,
            const double2 *__restrict__ seed, const double *__restrict__ zp,
            double2 *__restrict__ phase, int lmax, int npair, int nring, int nm) {
    const int g = blockIdx.x, mi = blockIdx.y, b0 = blockIdx.z * NB;
    const int npass = (lmax - mi > mi) ? 2 : 1;
    for (int pass = 0; pass < npass; pass++)
        synth_one_m<NB, P, U, PF>(pass == 0 ? mi : lmax - mi, g, alm, nalm, Atab, mofs, lstart,
                                  seed, zp, phase, lmax, npair, nring, nm, b0);
}

// ---------------------------------------------------------------------------------------
// Analysis
// ---------------------------------------------------------------------------------------
template <int NB>
struct AnaChunk {
    static constexpr int C = 16 / NB;      // values of l per reduction
    static constexpr int V = 2 * NB * C;   // doubles reduced per lane per chunk (= 32)
    static constexpr int LD = V + 2;       // LDS row stride of the plain transpose-reduce
    static constexpr int Q = V / 4;        // doubles per lane after the two lane swaps
};

// acc[2 (c NB + j) + comp] += sum_k mu_{c0+c}(pair k) X_{parity(c)}[k][j]
template <int NB, int P, bool INJ, bool FULL>
__device__ __forceinline__ void analysis_chunk(int c0, int lmax, PairState<P> &st,
                                               const double (&A)[AnaChunk<NB>::C],
                                               const double2 (&Xe)[P][NB],
                                               const double2 (&Xo)[P][NB],
                                               double (&acc)[AnaChunk<NB>::V]) {
    constexpr int C = AnaChunk<NB>::C;
#pragma unroll
    for (int c = 0; c < C; c++) {
        if (!FULL && c0 + c > lmax) break;
        double cur[P];
        st.template step<INJ>(c0 + c, A[c], cur);
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
            for (int k = 0; k < P; k++) {
                const double2 X = (c & 1) ? Xo[k][j] : Xe[k][j];
                acc[2 * (c * NB + j)] = fma(cur[k], X.x, acc[2 * (c * NB + j)]);
                acc[2 * (c * NB + j) + 1] = fma(cur[k], X.y, acc[2 * (c * NB + j) + 1]);
            }
    }
}

template <int NB, int P, bool PF>
__device__ __forceinline__ void analysis_one_m(int m, int g, const double2 *__restrict__ phase,
                                               int nring, int nm, const double *__restrict__ Atab,
                                               const long *__restrict__ mofs,
                                               const int *__restrict__ lstart,
                                               const double2 *__restrict__ seed,
                                               const double *__restrict__ zp,
                                               double2 *__restrict__ apart, long nalm,
                                               int nb_total, int lmax, int npair, int b0,
                                               double *red) {
    constexpr int C = AnaChunk<NB>::C, V = AnaChunk<NB>::V, LD = AnaChunk<NB>::LD, Q = AnaChunk<NB>::Q;
    static_assert(V == 32, "reduction assumes 32 values per lane");
    PairState<P> st;
    st.load(m, g, npair, lmax, zp, lstart, seed);
    const long off = mofs[m] - m;
    const double *Am = Atab + off;
    // X_even = G_N + G_S (l + m even), X_odd = G_N - G_S; the equator ring counts once.
    double2 Xe[P][NB], Xo[P][NB];
#pragma unroll
    for (int k = 0; k < P; k++) {
        const int p = g * kW * P + k * kW + (int)threadIdx.x;
        const bool valid = p < npair;
        const int rN = p, rS = nring - 1 - p;
#pragma unroll
        for (int j = 0; j < NB; j++) {
            const double2 *G = phase + (long)(b0 + j) * nm * nring + m;  // [map][ring][m]
            double2 gN = valid ? G[(long)rN * nm] : make_double2(0.0, 0.0);
            double2 gS = (valid && rS != rN) ? G[(long)rS * nm] : make_double2(0.0, 0.0);
            Xe[k][j] = make_double2(gN.x + gS.x, gN.y + gS.y);
            Xo[k][j] = make_double2(gN.x - gS.x, gN.y - gS.y);
        }
    }
    double2 *outg = apart + (long)g * nb_total * nalm;
    // l in [m, lo) receive no contribution from any pair of this group
    const int lo = st.lo - ((st.lo + m) & 1);  // chunks start at even l + m
    for (int l = m + (int)threadIdx.x; l < min(lo, lmax + 1); l += kW)
#pragma unroll
        for (int j = 0; j < NB; j++) outg[(long)(b0 + j) * nalm + off + l] = make_double2(0.0, 0.0);

    double Acur[C], Anxt[C];
    if (PF && lo + C - 1 <= lmax) {
#pragma unroll
        for (int c = 0; c < C; c++) Acur[c] = Am[lo + c];
    }
    for (int c0 = lo; c0 <= lmax; c0 += C) {
        double acc[V];
#pragma unroll
        for (int v = 0; v < V; v++) acc[v] = 0.0;
        const bool inj = c0 <= st.hi;
        if (c0 + C - 1 <= lmax) {
            if (PF) {
                if (c0 + 2 * C - 1 <= lmax) {
#pragma unroll
                    for (int c = 0; c < C; c++) Anxt[c] = Am[c0 + C + c];
                }
            } else {
#pragma unroll
                for (int c = 0; c < C; c++) Acur[c] = Am[c0 + c];
            }
            if (inj)
                analysis_chunk<NB, P, true, true>(c0, lmax, st, Acur, Xe, Xo, acc);
            else
                analysis_chunk<NB, P, false, true>(c0, lmax, st, Acur, Xe, Xo, acc);
            if (PF) {
#pragma unroll
                for (int c = 0; c < C; c++) Acur[c] = Anxt[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; c++) Acur[c] = (c0 + c <= lmax) ? Am[c0 + c] : 0.0;
            analysis_chunk<NB, P, true, false>(c0, lmax, st, Acur, Xe, Xo, acc);
        }
        // sum over the 64 lanes.  P < 4: two lane swaps halve the values a lane holds twice
        // (the 16-lane row r = L / 16 then holds values Q r .. Q r + Q - 1, each summed over
        // four lanes), then through LDS lane L sums value v = L / 2 over half L % 2 of its
        // row.  P = 4 (whose registers the swaps would exceed): all values through LDS, lane
        // L summing value L / 2 over half L % 2 of the wave.
        const int v = threadIdx.x >> 1, h = threadIdx.x & 1;
        double s = 0.0;
        if constexpr (P < 4) {
            double h1[V / 2], h2[Q];
#pragma unroll
            for (int i = 0; i < V / 2; i++) h1[i] = swap_add<true>(acc[i], acc[i + V / 2]);
#pragma unroll
            for (int i = 0; i < Q; i++) h2[i] = swap_add<false>(h1[i], h1[i + Q]);
#pragma unroll
            for (int i = 0; i < Q; i += 2)
                *reinterpret_cast<double2 *>(&red[threadIdx.x * Q + i]) = make_double2(h2[i], h2[i + 1]);
            __syncthreads();
            const int r = v / Q, jq = v - Q * r;
#pragma unroll
            for (int q = 0; q < 8; q++) s += red[(16 * r + 8 * h + q) * Q + jq];
        } else {
#pragma unroll
            for (int i = 0; i < V; i += 2)
                *reinterpret_cast<double2 *>(&red[threadIdx.x * LD + i]) = make_double2(acc[i], acc[i + 1]);
            __syncthreads();
#pragma unroll 8
            for (int q = 0; q < 32; q++) s += red[(h * 32 + q) * LD + v];
        }
        s += __shfl_xor(s, 1);
        __syncthreads();
        // v = 2 (c NB + j) + comp
        const int comp = v & 1, cj = v >> 1, c = cj / NB, j = cj - c * NB;
        const int l = c0 + c;
        if (h == 0 && l <= lmax)
            reinterpret_cast<double *>(outg + (long)(b0 + j) * nalm + off + l)[comp] = s;
    }
}

template <int NB, int P, bool PF>
__global__ void __launch_bounds__(kW)
k_leg_analysis(const double2 *__restrict__ phase, int nring, int nm,
               const double *__restrict__ Atab, const long *__restrict__ mofs,
               const int *__restrict__ lstart, const double2 *__restrict__ seed,
               const double *__restrict__ zp, double2 *__restrict__ apart, long nalm,
               int nb_total, int lmax, int npair) {
    __shared__ __align__(16) double red[kW * (P < 4 ? AnaChunk<NB>::Q : AnaChunk<NB>::LD)];
    const int g = blockIdx.x, mi = blockIdx.y, b0 = blockIdx.z * NB;
    const int npass = (lmax - mi > mi) ? 2 : 1;
    for (int pass = 0; pass < npass; pass++)
        analysis_one_m<NB, P, PF>(pass == 0 ? mi : lmax - mi, g, phase, nring, nm, Atab, mofs,
                                  lstart, seed, zp, apart, nalm, nb_total, lmax, npair, b0, red);
}

// ---------------------------------------------------------------------------------------
// Variant tables: index = tuning choice stored in the plan.
// ---------------------------------------------------------------------------------------
using SynthFn = void (*)(const double2 *, long, const double *, const long *, const int *,
                         const double2 *, const double *, double2 *, int, int, int, int);
using AnaFn = void (*)(const double2 *, int, int, const double *, const long *, const int *,
                       const double2 *, const double *, double2 *, long, int, int, int);

static const SynthFn kSynth[] = {
    k_leg_synth<1, 1, 8, false>, k_leg_synth<1, 2, 8, false>, k_leg_synth<1, 4, 8, false>,
    k_leg_synth<1, 1, 8, true>,  k_leg_synth<1, 2, 8, true>,  k_leg_synth<1, 4, 8, true>,
    k_leg_synth<1, 1, 4, true>,  k_leg_synth<1, 2, 4, true>,  k_leg_synth<1, 4, 4, true>,
};
static const int kSynthP[] = {1, 2, 4, 1, 2, 4, 1, 2, 4};
static const AnaFn kAna[] = {
    k_leg_analysis<1, 1, false>, k_leg_analysis<1, 2, false>, k_leg_analysis<1, 4, false>,
    k_leg_analysis<1, 1, true>,  k_leg_analysis<1, 2, true>,  k_leg_analysis<1, 4, true>,
};
static const int kAnaP[] = {1, 2, 4, 1, 2, 4};

int leg_synth_variants() { return (int)(sizeof(kSynth) / sizeof(kSynth[0])); }
int leg_analysis_variants() { return (int)(sizeof(kAna) / sizeof(kAna[0])); }
int leg_synth_pairs_per_lane(int v) { return kSynthP[v]; }
int leg_analysis_pairs_per_lane(int v) { return kAnaP[v]; }

static int groups(int npair, int P) { return (npair + 64 * P - 1) / (64 * P); }

int launch_leg_synth(const Plan &p, const double2 *alm_scaled, double2 *phase, int nb) {
    const int v = p.synth_variant;
    dim3 grid(groups(p.npair, kSynthP[v]), (p.lmax + 2) / 2, nb);
    hipLaunchKernelGGL(kSynth[v], grid, dim3(kW), 0, p.stream, alm_scaled, p.nalm, p.d_A,
                       p.d_mofs, p.d_lstart, p.d_seed, p.d_z, phase, p.lmax, p.npair, p.nring,
                       p.nm);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_leg_analysis(const Plan &p, const double2 *phase, double2 *apart, int nb) {
    const int v = p.ana_variant;
    dim3 grid(groups(p.npair, kAnaP[v]), (p.lmax + 2) / 2, nb);
    hipLaunchKernelGGL(kAna[v], grid, dim3(kW), 0, p.stream, phase, p.nring, p.nm, p.d_A,
                       p.d_mofs, p.d_lstart, p.d_seed, p.d_z, apart, p.nalm, nb, p.lmax,
                       p.npair);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

}  // namespace mfwf
