// Temperature and polarization (T, Q, U maps; T, E, B harmonics): the spin-2 Legendre
// steps and the 3x3-block kernels of the messenger iteration (Sect. 2.1 with the
// T+P noise and signal blocks of Sect. 3).
//
// Spin-2 functions (HEALPix / Zaldarriaga-Seljak convention):
//   F+_lm = ((2)lambda_lm + (-2)lambda_lm)/2,  F-_lm = ((2)lambda_lm - (-2)lambda_lm)/2,
//   synthesis  Q_r(m) = -sum_l (aE F+ + i aB F-),   U_r(m) = -sum_l (aB F+ - i aE F-)
//   analysis   aE = -Omega sum_r (F+ G_Q + i F- G_U),  aB = -Omega sum_r (F+ G_U - i F- G_Q)
// (the analysis is the adjoint of the synthesis, times Omega).  Applying the spin-raising
// operator twice to lambda_lm e^{i m phi} gives, with s = sin theta,
//   s^2 F+ = N_l [(2m^2 - l(l+1) + l(l-1) z^2) lambda_lm + 2 c_lm z lambda_{l-1,m}]
//   s^2 F- = 2 m N_l [c_lm lambda_{l-1,m} - (l-1) z lambda_lm]
//   N_l = ((l-1) l (l+1) (l+2))^{-1/2},  c_lm = ((2l+1)(l^2 - m^2)/(2l-1))^{1/2}.
// With lambda = c mu (the rescaled recurrence) the plan tabulates five numbers per (l, m),
//   pc = (N (2m^2 - l(l+1)) c_l, N l(l-1) c_l, 2 N c_lm c_{l-1}, 2 m N c_lm c_{l-1},
//         -2 m N (l-1) c_l),
// so s^2 F+ = (pc0 + pc1 z^2) mu_l + pc2 z mu_{l-1} and s^2 F- = pc3 mu_{l-1} + pc4 z mu_l:
// the recurrence that gives lambda for T also gives both spin-2 functions.  The 1/s^2 is
// applied once per ring (after the l sum in synthesis, to G_Q, G_U before it in analysis).
// Mirror rings: F+(-z) = (-1)^{l+m} F+(z), F-(-z) = -(-1)^{l+m} F-(z).
//
// Layouts: maps [B][3][npix] (T, Q, U); alm [B][3][nalm] (T, E, B); ring-Fourier rows
// [3B][nring][m] (the per-map transforms run on 3B maps); M [npix][6] packed symmetric
// (TT, TQ, TU, QQ, QU, UU); spectra [4][lmax+1] (TT, EE, BB, TE).
#include "leg_core.h"
#include "sym3.h"

namespace mfwf {

// ---------------------------------------------------------------------------------------
// Legendre synthesis, T + E/B -> ring-Fourier rows of T, Q, U
// ---------------------------------------------------------------------------------------
struct PolSynthAcc {
    double2 T[2], P[2], R[2], X[2], Y[2];  // [parity]: sum mu aT, F+ aE, F- aB, F+ aB, F- aE
};

__device__ __forceinline__ void cfma(double2 &acc, double f, double2 a) {
    acc.x = fma(f, a.x, acc.x);
    acc.y = fma(f, a.y, acc.y);
}

template <bool INJ, int PAR, int P>
__device__ __forceinline__ void pol_synth_step(int l, PairState<P> &st, const double (&zz)[P],
                                               double A, const double *__restrict__ pc,
                                               double2 aT, double2 aE, double2 aB,
                                               PolSynthAcc (&acc)[P]) {
    double cur[P];
    st.template step<INJ>(l, A, cur);
#pragma unroll
    for (int k = 0; k < P; k++) {
        const double mu = cur[k], mup = st.u2[k], z = st.z[k];
        const double fp = fma(fma(pc[1], zz[k], pc[0]), mu, pc[2] * z * mup);
        const double fm = fma(pc[3], mup, pc[4] * z * mu);
        cfma(acc[k].T[PAR], mu, aT);
        cfma(acc[k].P[PAR], fp, aE);
        cfma(acc[k].R[PAR], fm, aB);
        cfma(acc[k].X[PAR], fp, aB);
        cfma(acc[k].Y[PAR], fm, aE);
    }
}

// P ring pairs per lane: pairs g kW P + k kW + lane, k < P (the pairs of PairState)
template <int U, int P>
__device__ __forceinline__ void pol_synth_one_m(int m, int g, int b, const double2 *__restrict__ alm,
                                                long nalm, const double *__restrict__ Atab,
                                                const double *__restrict__ pctab,
                                                const long *__restrict__ mofs,
                                                const int *__restrict__ lstart,
                                                const double2 *__restrict__ seed,
                                                const double *__restrict__ zp,
                                                double2 *__restrict__ phase, int lmax,
                                                int npair, int nring, int nm) {
    PairState<P> st;
    st.load(m, g, npair, lmax, zp, lstart, seed);
    double zz[P];
#pragma unroll
    for (int k = 0; k < P; k++) zz[k] = st.z[k] * st.z[k];
    const long off = mofs[m] - m;
    const double *Am = Atab + off;
    const double *pcm = pctab + 5 * off;
    const double2 *aT = alm + (3L * b + 0) * nalm + off;
    const double2 *aE = alm + (3L * b + 1) * nalm + off;
    const double2 *aB = alm + (3L * b + 2) * nalm + off;
    PolSynthAcc acc[P];
#pragma unroll
    for (int k = 0; k < P; k++)
#pragma unroll
        for (int q = 0; q < 2; q++)
            acc[k].T[q] = acc[k].P[q] = acc[k].R[q] = acc[k].X[q] = acc[k].Y[q] = make_double2(0.0, 0.0);

    int l = st.lo - ((st.lo + m) & 1);  // blocks start at even l + m
    for (; l + U - 1 <= lmax; l += U) {
        const bool inj = l <= st.hi;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int lu = l + u;
            if (inj) {
                if (u & 1) pol_synth_step<true, 1>(lu, st, zz, Am[lu], pcm + 5 * lu, aT[lu], aE[lu], aB[lu], acc);
                else pol_synth_step<true, 0>(lu, st, zz, Am[lu], pcm + 5 * lu, aT[lu], aE[lu], aB[lu], acc);
            } else {
                if (u & 1) pol_synth_step<false, 1>(lu, st, zz, Am[lu], pcm + 5 * lu, aT[lu], aE[lu], aB[lu], acc);
                else pol_synth_step<false, 0>(lu, st, zz, Am[lu], pcm + 5 * lu, aT[lu], aE[lu], aB[lu], acc);
            }
        }
    }
    for (; l <= lmax; l++) {
        if ((l + m) & 1) pol_synth_step<true, 1>(l, st, zz, Am[l], pcm + 5 * l, aT[l], aE[l], aB[l], acc);
        else pol_synth_step<true, 0>(l, st, zz, Am[l], pcm + 5 * l, aT[l], aE[l], aB[l], acc);
    }

#pragma unroll
    for (int k = 0; k < P; k++) {
        const int p = g * kW * P + k * kW + (int)threadIdx.x;
        if (p >= npair) continue;
        const int rN = p, rS = nring - 1 - p;
        const double z = st.z[k];
        const double is2 = 1.0 / ((1.0 - z) * (1.0 + z));
        auto row = [&](int c, int r) { return phase + ((3L * b + c) * nring + r) * nm + m; };
        const PolSynthAcc &a = acc[k];
        const double2 Ts = make_double2(a.T[0].x + a.T[1].x, a.T[0].y + a.T[1].y);
        const double2 Td = make_double2(a.T[0].x - a.T[1].x, a.T[0].y - a.T[1].y);
        const double2 Ps = make_double2(a.P[0].x + a.P[1].x, a.P[0].y + a.P[1].y);
        const double2 Pd = make_double2(a.P[0].x - a.P[1].x, a.P[0].y - a.P[1].y);
        const double2 Rs = make_double2(a.R[0].x + a.R[1].x, a.R[0].y + a.R[1].y);
        const double2 Rd = make_double2(a.R[0].x - a.R[1].x, a.R[0].y - a.R[1].y);
        const double2 Xs = make_double2(a.X[0].x + a.X[1].x, a.X[0].y + a.X[1].y);
        const double2 Xd = make_double2(a.X[0].x - a.X[1].x, a.X[0].y - a.X[1].y);
        const double2 Ys = make_double2(a.Y[0].x + a.Y[1].x, a.Y[0].y + a.Y[1].y);
        const double2 Yd = make_double2(a.Y[0].x - a.Y[1].x, a.Y[0].y - a.Y[1].y);
        // Q_N = -(P + iR), Q_S = -(P' - iR'), U_N = -(X - iY), U_S = -(X' + iY')
        *row(0, rN) = Ts;
        *row(1, rN) = make_double2(is2 * (-Ps.x + Rs.y), is2 * (-Ps.y - Rs.x));
        *row(2, rN) = make_double2(is2 * (-Xs.x - Ys.y), is2 * (-Xs.y + Ys.x));
        if (rS != rN) {
            *row(0, rS) = Td;
            *row(1, rS) = make_double2(is2 * (-Pd.x - Rd.y), is2 * (-Pd.y + Rd.x));
            *row(2, rS) = make_double2(is2 * (-Xd.x + Yd.y), is2 * (-Xd.y - Yd.x));
        }
    }
}

template <int U, int P>
__global__ void __launch_bounds__(kW)
k_leg_synth_pol(const double2 *__restrict__ alm, long nalm, const double *__restrict__ Atab,
                const double *__restrict__ pctab, const long *__restrict__ mofs,
                const int *__restrict__ lstart, const double2 *__restrict__ seed,
                const double *__restrict__ zp, double2 *__restrict__ phase, int lmax, int npair,
                int nring, int nm) {
    const int g = blockIdx.x, mi = blockIdx.y, b = blockIdx.z;
    const int npass = (lmax - mi > mi) ? 2 : 1;
    for (int pass = 0; pass < npass; pass++)
        pol_synth_one_m<U, P>(pass == 0 ? mi : lmax - mi, g, b, alm, nalm, Atab, pctab, mofs, lstart,
                              seed, zp, phase, lmax, npair, nring, nm);
}

// ---------------------------------------------------------------------------------------
// Legendre analysis, ring-Fourier rows of T, Q, U -> partial sums of T (mu-scaled), E, B
// ---------------------------------------------------------------------------------------
static constexpr int kPC = 2;              // values of l per reduction chunk
static constexpr int kPV = 6 * kPC;        // doubles per lane per chunk
static constexpr int kPQ = kPV / 4;        // doubles per lane after the two lane swaps
static_assert(kW == 64 && kPV % 4 == 0, "the chunk reduction assumes one wave of 64 lanes");


struct PolAnaIn {
    double2 Xe, Xo;          // T: G_N + G_S, G_N - G_S
    double2 QP, QM, UP, UM;  // (G_N +- G_S) / s^2 for Q and U
};

template <bool INJ, int PAR, int P>
__device__ __forceinline__ void pol_ana_step(int l, int c, PairState<P> &st, const double (&zz)[P],
                                             double A, const double *__restrict__ pc,
                                             const PolAnaIn (&in)[P], double (&acc)[kPV]) {
    double cur[P];
    st.template step<INJ>(l, A, cur);
    double *a = acc + 6 * c;
#pragma unroll
    for (int k = 0; k < P; k++) {  // the lane's pairs, summed in order
        const double mu = cur[k], mup = st.u2[k], z = st.z[k];
        const double fp = fma(fma(pc[1], zz[k], pc[0]), mu, pc[2] * z * mup);
        const double fm = fma(pc[3], mup, pc[4] * z * mu);
        const double2 X = PAR ? in[k].Xo : in[k].Xe;
        // even l + m: E -= F+ QP + i F- UM, B -= F+ UP - i F- QM; odd: QP <-> QM, UP <-> UM
        const double2 Qa = PAR ? in[k].QM : in[k].QP, Ub = PAR ? in[k].UP : in[k].UM;
        const double2 Ua = PAR ? in[k].UM : in[k].UP, Qb = PAR ? in[k].QP : in[k].QM;
        a[0] = fma(mu, X.x, a[0]);
        a[1] = fma(mu, X.y, a[1]);
        a[2] -= fma(fp, Qa.x, -fm * Ub.y);
        a[3] -= fma(fp, Qa.y, fm * Ub.x);
        a[4] -= fma(fp, Ua.x, fm * Qb.y);
        a[5] -= fma(fp, Ua.y, -fm * Qb.x);
    }
}

// P ring pairs per lane: pairs g kW P + k kW + lane, k < P (the pairs of PairState)
template <int P>
__device__ __forceinline__ void pol_analysis_one_m(int m, int g, int b,
                                                   const double2 *__restrict__ phase, int nring,
                                                   int nm, const double *__restrict__ Atab,
                                                   const double *__restrict__ pctab,
                                                   const long *__restrict__ mofs,
                                                   const int *__restrict__ lstart,
                                                   const double2 *__restrict__ seed,
                                                   const double *__restrict__ zp,
                                                   double2 *__restrict__ apart, long nalm,
                                                   int nb_total, int lmax, int npair,
                                                   double *red) {
    PairState<P> st;
    st.load(m, g, npair, lmax, zp, lstart, seed);
    double zz[P];
#pragma unroll
    for (int k = 0; k < P; k++) zz[k] = st.z[k] * st.z[k];
    const long off = mofs[m] - m;
    const double *Am = Atab + off;
    const double *pcm = pctab + 5 * off;
    PolAnaIn in[P];
#pragma unroll
    for (int k = 0; k < P; k++) {
        const int p = g * kW * P + k * kW + (int)threadIdx.x;
        const bool valid = p < npair;
        const double z = st.z[k];
        const int rN = p, rS = nring - 1 - p;
        const bool south = valid && rS != rN;
        auto G = [&](int c, int r, bool ok) {
            return ok ? phase[((3L * b + c) * nring + r) * nm + m] : make_double2(0.0, 0.0);
        };
        const double2 tN = G(0, rN, valid), tS = G(0, rS, south);
        const double2 qN = G(1, rN, valid), qS = G(1, rS, south);
        const double2 uN = G(2, rN, valid), uS = G(2, rS, south);
        const double is2 = valid ? 1.0 / ((1.0 - z) * (1.0 + z)) : 0.0;
        in[k].Xe = make_double2(tN.x + tS.x, tN.y + tS.y);
        in[k].Xo = make_double2(tN.x - tS.x, tN.y - tS.y);
        in[k].QP = make_double2(is2 * (qN.x + qS.x), is2 * (qN.y + qS.y));
        in[k].QM = make_double2(is2 * (qN.x - qS.x), is2 * (qN.y - qS.y));
        in[k].UP = make_double2(is2 * (uN.x + uS.x), is2 * (uN.y + uS.y));
        in[k].UM = make_double2(is2 * (uN.x - uS.x), is2 * (uN.y - uS.y));
    }
    double2 *outg = apart + (long)g * nb_total * 3 * nalm;
    const int lo = st.lo - ((st.lo + m) & 1);
    for (int l = m + (int)threadIdx.x; l < min(lo, lmax + 1); l += kW)
        for (int c = 0; c < 3; c++) outg[(3L * b + c) * nalm + off + l] = make_double2(0.0, 0.0);

    // the recurrence and F+- coefficients of a chunk's values of l (wave-uniform), loaded one
    // chunk ahead so that their latency passes behind the current chunk's arithmetic
    struct Coef {
        double A, pc[5];
    };
    auto load_coef = [&](int l0, Coef (&cf)[kPC]) __attribute__((always_inline)) {
#pragma unroll
        for (int c = 0; c < kPC; c++) {
            const int l = min(l0 + c, lmax);
            cf[c].A = Am[l];
#pragma unroll
            for (int j = 0; j < 5; j++) cf[c].pc[j] = pcm[5 * l + j];
        }
    };
    Coef cf[kPC], nf[kPC];
    load_coef(lo, cf);
    for (int c0 = lo; c0 <= lmax; c0 += kPC) {
        if (c0 + kPC <= lmax) load_coef(c0 + kPC, nf);
        double acc[kPV];
#pragma unroll
        for (int v = 0; v < kPV; v++) acc[v] = 0.0;
        const bool inj = c0 <= st.hi;
        if (c0 + kPC - 1 <= lmax && !inj) {
#pragma unroll
            for (int c = 0; c < kPC; c++) {
                if (c & 1) pol_ana_step<false, 1>(c0 + c, c, st, zz, cf[c].A, cf[c].pc, in, acc);
                else pol_ana_step<false, 0>(c0 + c, c, st, zz, cf[c].A, cf[c].pc, in, acc);
            }
        } else {
#pragma unroll
            for (int c = 0; c < kPC; c++) {
                if (c0 + c > lmax) break;
                if (c & 1) pol_ana_step<true, 1>(c0 + c, c, st, zz, cf[c].A, cf[c].pc, in, acc);
                else pol_ana_step<true, 0>(c0 + c, c, st, zz, cf[c].A, cf[c].pc, in, acc);
            }
        }
        // sum over the 64 lanes: two lane swaps halve the values a lane holds twice (the
        // 16-lane row r = L / 16 then holds values kPQ r .. kPQ r + kPQ - 1, each summed over
        // four lanes), then through LDS lane t < 2 kPV sums value t / 2 over half t % 2 of its
        // row
        double h1[kPV / 2], h2[kPQ];
#pragma unroll
        for (int i = 0; i < kPV / 2; i++) h1[i] = swap_add<true>(acc[i], acc[i + kPV / 2]);
#pragma unroll
        for (int i = 0; i < kPQ; i++) h2[i] = swap_add<false>(h1[i], h1[i + kPQ]);
        if constexpr (kPQ % 2 == 0) {
#pragma unroll
            for (int i = 0; i < kPQ; i += 2)
                *reinterpret_cast<double2 *>(&red[threadIdx.x * kPQ + i]) = make_double2(h2[i], h2[i + 1]);
        } else {
#pragma unroll
            for (int i = 0; i < kPQ; i++) red[threadIdx.x * kPQ + i] = h2[i];
        }
        __syncthreads();
        const int v = threadIdx.x >> 1, h = threadIdx.x & 1;
        double s = 0.0;
        if (v < kPV) {
            const int r = v / kPQ, j = v - kPQ * r;
#pragma unroll
            for (int q = 0; q < 8; q++) s += red[(16 * r + 8 * h + q) * kPQ + j];
        }
        s += __shfl_xor(s, 1);
        __syncthreads();
        // v = 6 c + 2 comp + (re/im)
        const int c = v / 6, k = v - 6 * c, comp = k >> 1, ri = k & 1;
        const int l = c0 + c;
        if (h == 0 && v < kPV && l <= lmax)
            reinterpret_cast<double *>(outg + (3L * b + comp) * nalm + off + l)[ri] = s;
#pragma unroll
        for (int c = 0; c < kPC; c++) cf[c] = nf[c];
    }
}

template <int P>
__global__ void __launch_bounds__(kW)
k_leg_analysis_pol(const double2 *__restrict__ phase, int nring, int nm,
                   const double *__restrict__ Atab, const double *__restrict__ pctab,
                   const long *__restrict__ mofs, const int *__restrict__ lstart,
                   const double2 *__restrict__ seed, const double *__restrict__ zp,
                   double2 *__restrict__ apart, long nalm, int nb_total, int lmax, int npair) {
    __shared__ __align__(16) double red[kW * kPQ];
    const int g = blockIdx.x, mi = blockIdx.y, b = blockIdx.z;
    const int npass = (lmax - mi > mi) ? 2 : 1;
    for (int pass = 0; pass < npass; pass++)
        pol_analysis_one_m<P>(pass == 0 ? mi : lmax - mi, g, b, phase, nring, nm, Atab, pctab, mofs,
                              lstart, seed, zp, apart, nalm, nb_total, lmax, npair, red);
}

// ring pairs per lane of the analysis: two where there are pairs for more than one wave
// (each lane sums its pairs before the sum over lanes, whose cost is per value of l)
static int pol_ana_pairs(const Plan &p) { return p.npair > kW ? 2 : 1; }
static int pol_ana_groups(const Plan &p) {
    const int P = pol_ana_pairs(p);
    return (p.npair + kW * P - 1) / (kW * P);
}
int pol_ngroup(const Plan &p) { return pol_ana_groups(p); }

int launch_leg_synth_pol(const Plan &p, const double2 *alm_scaled, double2 *phase, int nb) {
    // two ring pairs per lane where there are pairs for more than one wave: each value of l's
    // coefficients and harmonics (wave-uniform loads) then serve twice the arithmetic
    const int P = p.npair > kW ? 2 : 1;
    dim3 grid((p.npair + kW * P - 1) / (kW * P), (p.lmax + 2) / 2, nb);
#define MFWF_SYNPOL(PP)                                                                          \
    hipLaunchKernelGGL((k_leg_synth_pol<4, PP>), grid, dim3(kW), 0, p.stream, alm_scaled, p.nalm,   \
                       p.d_A, p.d_pc, p.d_mofs, p.d_lstart, p.d_seed, p.d_z, phase, p.lmax,         \
                       p.npair, p.nring, p.nm)
    if (P == 2) MFWF_SYNPOL(2);
    else MFWF_SYNPOL(1);
#undef MFWF_SYNPOL
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_leg_analysis_pol(const Plan &p, const double2 *phase, double2 *apart, int nb) {
    dim3 grid(pol_ana_groups(p), (p.lmax + 2) / 2, nb);
    if (pol_ana_pairs(p) == 2)
        hipLaunchKernelGGL(k_leg_analysis_pol<2>, grid, dim3(kW), 0, p.stream, phase, p.nring, p.nm,
                           p.d_A, p.d_pc, p.d_mofs, p.d_lstart, p.d_seed, p.d_z, apart, p.nalm, nb,
                           p.lmax, p.npair);
    else
        hipLaunchKernelGGL(k_leg_analysis_pol<1>, grid, dim3(kW), 0, p.stream, phase, p.nring, p.nm,
                           p.d_A, p.d_pc, p.d_mofs, p.d_lstart, p.d_seed, p.d_z, apart, p.nalm, nb,
                           p.lmax, p.npair);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// ---------------------------------------------------------------------------------------
// Harmonic update with the 3x3 (T, E, B) signal blocks (Eq. 4):
//   S_l = [[TT, TE, 0], [TE, EE, 0], [0, 0, BB]],  s = S (S + mu I)^{-1} a,  mu = lam tau Omega.
// On the (T, E) block, with D = TT EE - TE^2 and det = (TT + mu)(EE + mu) - TE^2,
//   S (S + mu)^{-1} = [[D + mu TT, mu TE], [mu TE, D + mu EE]] / det   (no cancellation);
// on B, BB / (BB + mu).  S^{-1} is never formed; S = 0 gives s = 0.
// mode 0: s = S (S + lto)^{-1} a,  a = scale * (c sum_g T, sum_g E, sum_g B)
// mode 1: s = a
// mode 2: s = K h, K = L^{-T} with S = L L^T on the components with power (fluctuation)
// mode 3: s = in
// out_s <- s; out_sp <- (c s_T, s_E, s_B) (synthesis input); prev <- old out_s.
// ---------------------------------------------------------------------------------------
static constexpr int kHP = 256;

__global__ void __launch_bounds__(kHP)
k_harmonic_pol(const double2 *__restrict__ in, int ngroup, long nalm, int nb,
               const long *__restrict__ mofs, const double *__restrict__ cl4,
               const double *__restrict__ ctab, int lmax, double scale, double lto, int mode,
               double2 *__restrict__ out_s, double2 *__restrict__ out_sp,
               double2 *__restrict__ prev) {
    const int m = blockIdx.x, b = blockIdx.y;
    const long toff = mofs[m] - m;
    const int L1 = lmax + 1;
    for (int l = m + threadIdx.x; l <= lmax; l += kHP) {
        const long i = toff + l;
        const double c = ctab[i];
        double2 a[3];
        for (int q = 0; q < 3; q++) {
            double2 v = in[(3L * b + q) * nalm + i];
            if (mode <= 1) {
                for (int g = 1; g < ngroup; g++) {
                    const double2 w = in[((long)g * nb * 3 + 3L * b + q) * nalm + i];
                    v.x += w.x;
                    v.y += w.y;
                }
                const double f = (q == 0) ? scale * c : scale;
                v = make_double2(f * v.x, f * v.y);
            }
            a[q] = v;
        }
        const double TT = cl4[l], EE = cl4[L1 + l], BB = cl4[2 * L1 + l], TE = cl4[3 * L1 + l];
        double2 s[3];
        if (mode == 0) {
            const double mu = lto, D = TT * EE - TE * TE;
            const double det = (TT + mu) * (EE + mu) - TE * TE;
            const double ftt = (D + mu * TT) / det, fte = mu * TE / det, fee = (D + mu * EE) / det;
            const double fbb = BB > 0.0 ? BB / (BB + mu) : 0.0;
            s[0] = make_double2(ftt * a[0].x + fte * a[1].x, ftt * a[0].y + fte * a[1].y);
            s[1] = make_double2(fte * a[0].x + fee * a[1].x, fte * a[0].y + fee * a[1].y);
            s[2] = make_double2(fbb * a[2].x, fbb * a[2].y);
        } else if (mode == 2) {
            double k00 = 0.0, k01 = 0.0, k11 = 0.0;
            if (TT > 0.0 && EE > 0.0) {
                const double ra = sqrt(TT), rb = TE / ra, rc = sqrt(EE - rb * rb);
                k00 = 1.0 / ra;
                k01 = -rb / (ra * rc);
                k11 = 1.0 / rc;
            } else if (TT > 0.0) {
                k00 = 1.0 / sqrt(TT);
            } else if (EE > 0.0) {
                k11 = 1.0 / sqrt(EE);
            }
            const double kbb = BB > 0.0 ? 1.0 / sqrt(BB) : 0.0;
            s[0] = make_double2(k00 * a[0].x + k01 * a[1].x, k00 * a[0].y + k01 * a[1].y);
            s[1] = make_double2(k11 * a[1].x, k11 * a[1].y);
            s[2] = make_double2(kbb * a[2].x, kbb * a[2].y);
        } else {
            s[0] = a[0];
            s[1] = a[1];
            s[2] = a[2];
        }
        for (int q = 0; q < 3; q++) {
            const long o = (3L * b + q) * nalm + i;
            if (prev) prev[o] = out_s[o];
            if (out_s) out_s[o] = s[q];
            if (out_sp) out_sp[o] = (q == 0) ? make_double2(c * s[q].x, c * s[q].y) : s[q];
        }
    }
}

int launch_harmonic_pol(const Plan &p, const double2 *in, int ngroup, double scale, double lto,
                        int mode, double2 *out_s, double2 *out_sp, double2 *prev, int nb) {
    hipLaunchKernelGGL(k_harmonic_pol, dim3(p.nm, nb), dim3(kHP), 0, p.stream, in, ngroup,
                       p.nalm, nb, p.d_mofs, p.d_cl, p.d_c, p.lmax, scale, lto, mode, out_s,
                       out_sp, prev);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// ---------------------------------------------------------------------------------------
// 3x3 pixel blocks
// ---------------------------------------------------------------------------------------
static constexpr int kPT = 256;

static int pgrid(long n) {
    long g = (n + kPT - 1) / kPT;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

__device__ __forceinline__ double sym3_det(const Sym3 &M) {
    return M.a * (M.d * M.f - M.e * M.e) - M.b * (M.b * M.f - M.e * M.c) + M.c * (M.b * M.e - M.d * M.c);
}

// x = M^{-1} y by the adjugate (M symmetric positive definite here)
__device__ __forceinline__ void sym3_solve(const Sym3 &M, const double y[3], double x[3]) {
    const double A = M.d * M.f - M.e * M.e, B = M.c * M.e - M.b * M.f, C = M.b * M.e - M.c * M.d;
    const double D = M.a * M.f - M.c * M.c, E = M.b * M.c - M.a * M.e, F = M.a * M.d - M.b * M.b;
    const double det = M.a * A + M.b * B + M.c * C;
    x[0] = (A * y[0] + B * y[1] + C * y[2]) / det;
    x[1] = (B * y[0] + D * y[1] + E * y[2]) / det;
    x[2] = (C * y[0] + E * y[1] + F * y[2]) / det;
}

__device__ __forceinline__ Sym3 sym3_square(const Sym3 &M) {
    return Sym3{M.a * M.a + M.b * M.b + M.c * M.c, M.a * M.b + M.b * M.d + M.c * M.e,
                M.a * M.c + M.b * M.e + M.c * M.f, M.b * M.b + M.d * M.d + M.e * M.e,
                M.b * M.c + M.d * M.e + M.e * M.f, M.c * M.c + M.e * M.e + M.f * M.f};
}

// eigenvalues of a symmetric 3x3 (closed form through the trigonometric solution of the
// characteristic cubic), largest first
__device__ __forceinline__ void sym3_eig(const Sym3 &M, double &emax, double &emin) {
    const double p1 = M.b * M.b + M.c * M.c + M.e * M.e;
    const double q = (M.a + M.d + M.f) / 3.0;
    if (p1 == 0.0) {
        emax = fmax(M.a, fmax(M.d, M.f));
        emin = fmin(M.a, fmin(M.d, M.f));
        return;
    }
    const double p2 = (M.a - q) * (M.a - q) + (M.d - q) * (M.d - q) + (M.f - q) * (M.f - q) + 2.0 * p1;
    const double pp = sqrt(p2 / 6.0);
    const Sym3 Bm{(M.a - q) / pp, M.b / pp, M.c / pp, (M.d - q) / pp, M.e / pp, (M.f - q) / pp};
    double r = sym3_det(Bm) / 2.0;
    r = fmin(1.0, fmax(-1.0, r));
    const double phi = acos(r) / 3.0;
    emax = q + 2.0 * pp * cos(phi);
    emin = q + 2.0 * pp * cos(phi + 2.0 * M_PI / 3.0);
}

__global__ void k_mask_product_pol(const double *__restrict__ ninv6, const uint8_t *__restrict__ mask,
                                   double *__restrict__ M6, long npix) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < 6 * npix;
         i += (long)gridDim.x * blockDim.x)
        M6[i] = (mask == nullptr || mask[i / 6] != 0) ? ninv6[i] : 0.0;
}

// partial[block] = (max lambda_max, #(det M > 0), #(non-finite, or lambda_min < -1e-12 lambda_max))
__global__ void __launch_bounds__(kPT)
k_pol_stats(const double *__restrict__ M6, long npix, double *__restrict__ partial) {
    __shared__ double sh[3][kPT];
    double mx = 0.0, cnt = 0.0, bad = 0.0;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix;
         p += (long)gridDim.x * blockDim.x) {
        const Sym3 M = load_sym3(M6, p);
        const double sum = M.a + M.b + M.c + M.d + M.e + M.f;
        if (!isfinite(sum)) {
            bad += 1.0;
            continue;
        }
        double emax, emin;
        sym3_eig(M, emax, emin);
        if (emin < -1e-12 * fabs(emax)) bad += 1.0;
        mx = fmax(mx, emax);
        cnt += (sym3_det(M) > 0.0) ? 1.0 : 0.0;
    }
    sh[0][threadIdx.x] = mx;
    sh[1][threadIdx.x] = cnt;
    sh[2][threadIdx.x] = bad;
    __syncthreads();
    for (int w = kPT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; k++) partial[3 * blockIdx.x + k] = sh[k][0];
}

__global__ void k_pol_stats_final(const double *__restrict__ partial, int nblocks,
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

int launch_pol_covariance(const double *ninv6, const uint8_t *mask, double *M6, long npix,
                          double *partial, int nblocks, double *out3, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_product_pol, dim3(pgrid(6 * npix)), dim3(kPT), 0, s, ninv6, mask, M6,
                       npix);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pol_stats, dim3(nblocks), dim3(kPT), 0, s, M6, npix, partial);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pol_stats_final, dim3(1), dim3(64), 0, s, partial, nblocks, out3);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// rho = M d per pixel (masked pixels: 0)
__global__ void k_rho_from_data_pol(const double *__restrict__ d, const double *__restrict__ M6,
                                    double *__restrict__ rho, long npix, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const long b = i / npix, p = i - b * npix;
        const Sym3 M = load_sym3(M6, p);
        const double *db = d + 3 * b * npix;
        double x[3] = {db[p], db[npix + p], db[2 * npix + p]}, y[3];
        const bool obs = (M.a != 0.0 || M.d != 0.0 || M.f != 0.0);
        sym3_mv(M, x, y);
        double *rb = rho + 3 * b * npix;
        for (int k = 0; k < 3; k++) rb[k * npix + p] = obs ? y[k] : 0.0;
    }
}

// Eq. (3) with blocks, multiplied through by N:
//   t = [I + (lam - 1) tau M]^{-1} [lam tau rho + (I - tau M) s]
__global__ void k_pixel_update_pol(const double *__restrict__ rho, const double *__restrict__ M6,
                                   const double *__restrict__ smap, double *__restrict__ t,
                                   long npix, long n, double lam, double tau) {
    const double lt = lam * tau, l1t = (lam - 1.0) * tau;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const long b = i / npix, p = i - b * npix;
        const Sym3 M = load_sym3(M6, p);
        const long o = 3 * b * npix + p;
        const double s[3] = {smap[o], smap[o + npix], smap[o + 2 * npix]};
        const double r[3] = {rho[o], rho[o + npix], rho[o + 2 * npix]};
        double x[3];
        pol_messenger_pixel(M, s, r, lam, lt, l1t, tau, x);
        for (int k = 0; k < 3; k++) t[o + k * npix] = x[k];
    }
}

int launch_rho_from_data_pol(const double *d, const double *M6, double *rho, long npix, int nb,
                             hipStream_t s) {
    const long n = npix * nb;
    hipLaunchKernelGGL(k_rho_from_data_pol, dim3(pgrid(n)), dim3(kPT), 0, s, d, M6, rho, npix, n);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_pixel_update_pol(const double *rho, const double *M6, const double *smap, double *t,
                            long npix, int nb, double lam, double tau, hipStream_t s) {
    const long n = npix * nb;
    hipLaunchKernelGGL(k_pixel_update_pol, dim3(pgrid(n)), dim3(kPT), 0, s, rho, M6, smap, t, npix,
                       n, lam, tau);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// chi^2 pixel term with blocks: sum over pixels with det M > 0 of
//   q^T [M + (lam - 1) tau M^2]^{-1} q,  q = rho - M s  (= (d - s)^T M [I + (lam-1) tau M]^{-1} (d - s))
// grid (nblocks, nb): partial[b][block]
__global__ void __launch_bounds__(kPT)
k_chi2_pix_pol(const double *__restrict__ rho, const double *__restrict__ M6,
               const double *__restrict__ smap, long npix, double lam, double tau,
               double *__restrict__ partial) {
    __shared__ double sh[kPT];
    const long off = 3L * blockIdx.y * npix;
    const double l1t = (lam - 1.0) * tau;
    double acc = 0.0;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix;
         p += (long)gridDim.x * blockDim.x) {
        const Sym3 M = load_sym3(M6, p);
        if (!(sym3_det(M) > 0.0)) continue;
        double s[3] = {smap[off + p], smap[off + npix + p], smap[off + 2 * npix + p]}, Ms[3], q[3], x[3];
        sym3_mv(M, s, Ms);
        for (int k = 0; k < 3; k++) q[k] = rho[off + k * npix + p] - Ms[k];
        const Sym3 M2 = sym3_square(M);
        const Sym3 B{M.a + l1t * M2.a, M.b + l1t * M2.b, M.c + l1t * M2.c, M.d + l1t * M2.d,
                     M.e + l1t * M2.e, M.f + l1t * M2.f};
        sym3_solve(B, q, x);
        acc += q[0] * x[0] + q[1] * x[1] + q[2] * x[2];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kPT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void k_sum_partials_pol(const double *__restrict__ partial, int nblocks, int nb,
                                   double *__restrict__ diag) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double acc = 0.0;
    for (int k = 0; k < nblocks; k++) acc += partial[(long)b * nblocks + k];
    diag[8 * b + 0] = acc;
}

int launch_chi2_pix_pol(const double *rho, const double *M6, const double *smap, long npix,
                        int nb, double lam, double tau, double *partial, int nblocks,
                        double *diag, hipStream_t s) {
    hipLaunchKernelGGL(k_chi2_pix_pol, dim3(nblocks, nb), dim3(kPT), 0, s, rho, M6, smap, npix,
                       lam, tau, partial);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials_pol, dim3((nb + 63) / 64), dim3(64), 0, s, partial, nblocks,
                       nb, diag);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// Pixel term of chi^2(lambda, s) for T, Q, U and its derivative in lambda (the error-bound
// schedule of Sect. 2.2): with q = rho - M s and B = M + (lam - 1) tau M^2 per observed block,
//   P = q^T B^-1 q,  dP/dlam = -tau |M B^-1 q|^2
// (dB/dlam = tau M^2, and M commutes with B).  partial[b][block][2], summed by
// launch_sum_pairs into out[b][2].
__global__ void __launch_bounds__(kPT)
k_chi2_pix_dlam_pol(const double *__restrict__ rho, const double *__restrict__ M6,
                    const double *__restrict__ smap, long npix, double lam, double tau,
                    double *__restrict__ partial) {
    __shared__ double sh[2][kPT];
    const long off = 3L * blockIdx.y * npix;
    const double l1t = (lam - 1.0) * tau;
    double acc = 0.0, dacc = 0.0;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix;
         p += (long)gridDim.x * blockDim.x) {
        const Sym3 M = load_sym3(M6, p);
        if (!(sym3_det(M) > 0.0)) continue;
        double s[3] = {smap[off + p], smap[off + npix + p], smap[off + 2 * npix + p]}, Ms[3], q[3],
               x[3], Mx[3];
        sym3_mv(M, s, Ms);
        for (int k = 0; k < 3; k++) q[k] = rho[off + k * npix + p] - Ms[k];
        const Sym3 M2 = sym3_square(M);
        const Sym3 B{M.a + l1t * M2.a, M.b + l1t * M2.b, M.c + l1t * M2.c, M.d + l1t * M2.d,
                     M.e + l1t * M2.e, M.f + l1t * M2.f};
        sym3_solve(B, q, x);
        sym3_mv(M, x, Mx);
        acc += q[0] * x[0] + q[1] * x[1] + q[2] * x[2];
        dacc -= tau * (Mx[0] * Mx[0] + Mx[1] * Mx[1] + Mx[2] * Mx[2]);
    }
    sh[0][threadIdx.x] = acc;
    sh[1][threadIdx.x] = dacc;
    __syncthreads();
    for (int w = kPT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long o = ((long)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        partial[o] = sh[0][0];
        partial[o + 1] = sh[1][0];
    }
}

int launch_chi2_pix_dlam_pol(const double *rho, const double *M6, const double *smap, long npix,
                             int nb, double lam, double tau, double *partial, int nblocks,
                             double *out2, hipStream_t s) {
    hipLaunchKernelGGL(k_chi2_pix_dlam_pol, dim3(nblocks, nb), dim3(kPT), 0, s, rho, M6, smap,
                       npix, lam, tau, partial);
    MFWF_HIP(hipGetLastError());
    return launch_sum_pairs(partial, nblocks, nb, out2, s);
}

// Harmonic diagnostics over T, E, B (real dof, m > 0 twice):
//   [0] s^T S^+ s (the (T, E) block inverted where both have power, else the one that has;
//   B where BB > 0), [1] |s - prev|^2, [2] |s|^2
__device__ __forceinline__ double quad_sinv(double TT, double EE, double BB, double TE,
                                            double x0, double x1, double x2) {
    double acc = 0.0;
    if (TT > 0.0 && EE > 0.0) {
        const double det = TT * EE - TE * TE;
        acc += (EE * x0 * x0 - 2.0 * TE * x0 * x1 + TT * x1 * x1) / det;
    } else if (TT > 0.0) {
        acc += x0 * x0 / TT;
    } else if (EE > 0.0) {
        acc += x1 * x1 / EE;
    }
    if (BB > 0.0) acc += x2 * x2 / BB;
    return acc;
}

__global__ void __launch_bounds__(kHP)
k_harm_diag_pol(const double2 *__restrict__ s, const double2 *__restrict__ prev, long nalm,
                const long *__restrict__ mofs, const double *__restrict__ cl4, int lmax, int nm,
                double *__restrict__ partial) {
    __shared__ double sh[3][kHP];
    const int m = blockIdx.x, b = blockIdx.y;
    const long toff = mofs[m] - m;
    const int L1 = lmax + 1;
    const double w = (m == 0) ? 1.0 : 2.0;
    double h = 0.0, d = 0.0, n = 0.0;
    for (int l = m + threadIdx.x; l <= lmax; l += kHP) {
        double2 v[3];
        for (int q = 0; q < 3; q++) {
            const long o = (3L * b + q) * nalm + toff + l;
            v[q] = s[o];
            const double2 u = prev[o];
            d += (v[q].x - u.x) * (v[q].x - u.x) + (v[q].y - u.y) * (v[q].y - u.y);
            n += v[q].x * v[q].x + v[q].y * v[q].y;
        }
        const double TT = cl4[l], EE = cl4[L1 + l], BB = cl4[2 * L1 + l], TE = cl4[3 * L1 + l];
        h += quad_sinv(TT, EE, BB, TE, v[0].x, v[1].x, v[2].x) +
             quad_sinv(TT, EE, BB, TE, v[0].y, v[1].y, v[2].y);
    }
    sh[0][threadIdx.x] = h;
    sh[1][threadIdx.x] = d;
    sh[2][threadIdx.x] = n;
    __syncthreads();
    for (int o = kHP / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 3) partial[((long)b * nm + m) * 3 + threadIdx.x] = w * sh[threadIdx.x][0];
}

__global__ void k_harm_diag_pol_final(const double *__restrict__ partial, int nm, int nb,
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

int launch_harm_diag_pol(const Plan &p, const double2 *salm, const double2 *salm_prev, int nb,
                         double *partial, double *diag) {
    hipLaunchKernelGGL(k_harm_diag_pol, dim3(p.nm, nb), dim3(kHP), 0, p.stream, salm, salm_prev,
                       p.nalm, p.d_mofs, p.d_cl, p.lmax, p.nm, partial);
    MFWF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_harm_diag_pol_final, dim3((nb + 63) / 64), dim3(64), 0, p.stream, partial,
                       p.nm, nb, diag);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// Fluctuation source with blocks: rho = L_p g1 + Omega Y(K h), M_p = L_p L_p^T (Cholesky;
// a column stops at the first non-positive pivot, so masked pixels give 0)
__global__ void k_fluct_combine_pol(const double *__restrict__ g1, const double *__restrict__ M6,
                                    const double *__restrict__ ysh, double *__restrict__ rho,
                                    long npix, long n, double omega) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const long b = i / npix, p = i - b * npix;
        const Sym3 M = load_sym3(M6, p);
        double L00 = 0.0, L10 = 0.0, L20 = 0.0, L11 = 0.0, L21 = 0.0, L22 = 0.0;
        if (M.a > 0.0) {
            L00 = sqrt(M.a);
            L10 = M.b / L00;
            L20 = M.c / L00;
            const double d1 = M.d - L10 * L10;
            if (d1 > 0.0) {
                L11 = sqrt(d1);
                L21 = (M.e - L20 * L10) / L11;
                const double d2 = M.f - L20 * L20 - L21 * L21;
                if (d2 > 0.0) L22 = sqrt(d2);
            }
        }
        const long o = 3 * b * npix + p;
        const double x0 = g1[o], x1 = g1[o + npix], x2 = g1[o + 2 * npix];
        rho[o] = L00 * x0 + omega * ysh[o];
        rho[o + npix] = L10 * x0 + L11 * x1 + omega * ysh[o + npix];
        rho[o + 2 * npix] = L20 * x0 + L21 * x1 + L22 * x2 + omega * ysh[o + 2 * npix];
    }
}

int launch_fluct_combine_pol(const double *g1, const double *M6, const double *ysh, double *rho,
                             long npix, int nb, double omega, hipStream_t s) {
    const long n = npix * nb;
    hipLaunchKernelGGL(k_fluct_combine_pol, dim3(pgrid(n)), dim3(kPT), 0, s, g1, M6, ysh, rho, npix,
                       n, omega);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

}  // namespace mfwf
