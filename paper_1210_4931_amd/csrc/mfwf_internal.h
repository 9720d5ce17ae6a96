// Internal declarations of the mfwf HIP library: the plan object, device table layout
// and the launch wrappers of every kernel.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "mfwf.h"

namespace mfwf {

// Status propagation with a thread-local message.
void set_error(const std::string &msg);
#define MFWF_HIP(call)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::mfwf::set_error(std::string(#call) + ": " + hipGetErrorString(e_));          \
            return MFWF_EDEVICE;                                                           \
        }                                                                                  \
    } while (0)
#define MFWF_TRY(call)                                                                     \
    do {                                                                                   \
        int s_ = (call);                                                                   \
        if (s_ != MFWF_OK) return s_;                                                      \
    } while (0)

// Ring pair p (0-based, p = 0 .. 2 nside - 1) couples north ring p and south ring
// nring - 1 - p (0-based ring indices, north to south).  The last pair is the equator,
// whose north and south ring coincide.
struct PairFFT {
    int nphi;        // pixels per ring of this pair
    int fftlen;      // length of the power-of-two transform used (nphi or Bluestein M)
    int bluestein;   // 0: nphi is a power of two; 1: Bluestein of length nphi; 2: split,
                     // nphi = 4 i with four Bluestein transforms of length i (fftlen, chirp
                     // and kernel tables of length i)
    int half_shift;  // 1 if phi_0 = pi / nphi, 0 if phi_0 = 0
    long startN;     // first pixel of the north ring
    long startS;     // first pixel of the south ring (== startN on the equator)
    long chirp_off;  // offset of the chirp table of this length (Bluestein only)
    long bhat_off;   // offset of the transformed chirp kernel (Bluestein only)
};

// Legendre work split: the wave of lanes handling ring pairs [g * 64 * P, (g+1) * 64 * P)
// for one m.  Seeds: for every (m, pair) the first l with |lambda_lm| >= 2^-100 and the
// two values (lambda_{l_s - 1, m}, lambda_{l_s, m}); l_s = lmax + 1 if never reached.
struct Plan {
    int nside, lmax, spin, dtype, max_batch;
    int device = 0;  // HIP device current when the plan was created
    int ncomp = 1;  // components per map: 1 (T) or 3 (T, Q, U / T, E, B)
    hipStream_t stream;
    long npix;
    int nring, npair, nm;
    long nalm;
    double omega;
    int synth_variant = 0;  // index into the Legendre synthesis kernel variants
    int ana_variant = 0;    // index into the Legendre analysis kernel variants
    int ngroup;             // pair groups (waves per m) of the chosen analysis variant
    int ring_group[2] = {1, 1};  // maps per workgroup of the columns ring step, per class
    int gemm_ct[2] = {2, 2};     // column tiles of the analysis GEMM (1: 64 columns, 2: 128 in
                                 // 4 waves, 3: 128 in 8 waves) and the synthesis GEMM (1, 2)
    int tune_source = 0;         // 0 defaults, 1 autotuned (timed or cached), 3 forced
    int ngroup_max;         // largest pair-group count of any analysis variant

    // plan tables (device)
    double *d_z = nullptr;       // [npair] cos(theta) of the north ring of each pair
    double *d_A = nullptr;       // [nalm] A_lm of mu_l = A z mu_{l-1} - mu_{l-2}
    double *d_c = nullptr;       // [nalm] c_lm, lambda_lm = c_lm mu_lm
    int *d_lstart = nullptr;     // [nm][npair]
    double2 *d_seed = nullptr;   // [nm][npair] (mu_{l_s - 1}, mu_{l_s})
    PairFFT *d_pfft = nullptr;   // [npair]
    double2 *d_tw = nullptr;     // [fftmax] exp(-2 pi i k / fftmax)
    double2 *d_twlo = nullptr;   // [64] exp(-2 pi i t / fftmax)
    double2 *d_twhi = nullptr;   // [fft_ntwhi] exp(-2 pi i 64 h / fftmax)
    int fft_ntwhi = 1;
    double2 *d_chirp = nullptr;  // Bluestein chirps exp(-i pi k^2 / n), per distinct n
    double2 *d_bhat = nullptr;   // Bluestein kernels FFT_M(conj chirp) / M, natural order
    int fftmax;                  // largest power-of-two transform length
    int *d_plist = nullptr;      // [npair] pair indices grouped by FFT class
    // classes: 0 short transforms, 1 the longest in-LDS ones, 2 split rings (FP64 rows only)
    int fft_class_off[3] = {0, 0, 0}, fft_class_count[3] = {0, 0, 0}, fft_class_len[3] = {1, 1, 1};
    // FP32 ring step: the longest ring class runs on a side stream forked from `stream` (and
    // joined back) while the short class runs on `stream`; the classes touch disjoint rings
    hipStream_t side = nullptr;
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    double2 *d_fftsplit = nullptr;  // split rings: [rows][class-2 pairs][fftsplit_stride]
    long fftsplit_stride = 0;       // 2 x the longest split ring
    int fftsplit_rows = 0;          // rows (maps x components) one launch may carry
    int fftsplit_sublen = 1;        // longest Bluestein length of the split sub-transforms
    long *d_mofs = nullptr;      // [nm] packed offset of (l = m, m)
    double *d_pc = nullptr;      // [nalm][5] spin-2 coefficients of mu_l, mu_{l-1} (spin 2)

    // covariances
    double *d_cl = nullptr;  // [lmax+1], or [4][lmax+1] TT, EE, BB, TE (spin 2)
    double *d_M = nullptr;   // [npix] inverse noise variance times mask, or [npix][6] blocks
    double tau = 0.0;
    long ndof = 0;
    bool have_cov = false;
    // serving slots: one M row and one tau per map (mstride = npix, d_tau [B]); otherwise
    // one M for all maps (mstride = 0, d_tau null)
    long mstride = 0;
    double *d_tau = nullptr;

    // workspaces, sized for max_batch maps
    double *d_rho = nullptr;     // [B][npix]
    double *d_t = nullptr;       // [B][npix]
    double *d_smap = nullptr;    // [B][npix]
    double2 *d_phase = nullptr;  // [B][nring][nm] ring Fourier coefficients
    double2 *d_apart = nullptr;  // [ngroup][B][nalm] partial analysis sums
    double2 *d_salm = nullptr;   // [B][nalm]
    double2 *d_salm_prev = nullptr;
    double2 *d_sp = nullptr;     // [B][nalm] c_lm-scaled synthesis input
    double *d_red = nullptr;     // reduction partials
    double *d_diag = nullptr;    // [B][8] diagnostics
    int nred_blocks;
    double work_tuples = 0.0;  // (l, m, pair) triples with l >= start index

    // batched FP32 form (dtype MFWF_F32): lambda table and column-major work arrays
    int Rp = 0;                  // ring pairs padded to 64
    int Bp = 0;                  // maps padded to 16
    int C2 = 0;                  // columns = 2 Bp (re, im of each map)
    float *d_lam = nullptr;      // lambda_lm(z_p) FP32, rows [m][pair][l - m] padded to 128
                                 // (null when the temperature GEMMs generate their rows)
    bool lam_gen = false;        // temperature GEMMs generate lambda from d_lck instead of d_lam
    double2 *d_lck = nullptr;    // recurrence state entering every 16-row segment of the rows,
                                 // [(segoff[m] + seg) Rp + pair] (temperature FP32 plans)
    long *d_segoff = nullptr;    // [nm] first segment of m
    long *d_loff = nullptr;      // [nm] offset of m's rows
    int *d_Lp = nullptr;         // [nm] padded row length
    int *d_minls32 = nullptr;    // [nm][Rp/32] smallest start index in each 32-pair chunk
    int2 *d_ana_items = nullptr; // (m, 128-row l tile) work items of the analysis GEMM
    int2 *d_syn_items = nullptr; // (m, 64-pair tile) work items of the synthesis GEMM
    int *d_ana_tab = nullptr;    // [8][ana_per_xcd] item list of each XCD (-1 = none)
    int *d_syn_tab = nullptr;    // [8][syn_per_xcd]
    int ana_per_xcd = 0, syn_per_xcd = 0;
    int *d_lofi = nullptr;       // [nalm] l of each packed index
    float2 *d_phf = nullptr;     // [B][nring][nm32] ring-Fourier rows of the transforms
    int nm32 = 0;                // row stride of d_phf: nm rounded up to whole 128-byte lines
    // batched FP32 iterations chained through the synthesis columns d_ph32: each iteration
    // starts with the previous one's inverse ring transforms, fused with its own pixel update
    // and forward transforms; d_smap is written only by iterations that keep diagnostics
    bool chain = false;
    bool chain_ready = false;    // d_ph32 holds the synthesis of the iterate in d_smap
    float *d_ph32 = nullptr;     // [nm][nring][C2] ring-Fourier, maps innermost
    float *d_a32 = nullptr;      // [nalm][C2] analysis output
    float *d_s32 = nullptr;      // [nalm][C2] synthesis input
    // batched FP32 form with spin 2 (T, Q, U); T uses the arrays above
    float *d_fp = nullptr;       // F+_lm(z_p) FP32, rows like d_lam
    float *d_fm = nullptr;       // F-_lm(z_p) FP32
    float *d_ph32p = nullptr;    // [nm][nring][2 C2] Q, U ring-Fourier (analysis input; synthesis out)
    float *d_ap32 = nullptr;     // [nalm][2 C2] F+ analysis sums
    float *d_ar32 = nullptr;     // [nalm][2 C2] F- analysis sums
    float *d_seb32 = nullptr;    // [nalm][2 C2] E, B synthesis input
};

// ---- plan internals (api.hip) used by the serving runtime -------------------------------
int plan_create(int nside, int lmax, int spin, int dtype, int max_batch, void *stream,
                bool per_slot, Plan &p);
void plan_destroy(Plan &p);
int plan_iteration(Plan &p, const double *rho, int nb, double lam);
int plan_finish_alm(Plan &p, int nb);
int plan_set_cl(Plan &p, const double *cl);
int fail(int status, const std::string &msg);

// ---- kernels (launch wrappers) --------------------------------------------------------
// pixel.hip
int launch_fill(double *x, long n, double v, hipStream_t s);
int launch_mask_product(const double *ninv, const uint8_t *mask, double *M, long npix,
                        hipStream_t s);
int launch_reduce_max_count(const double *M, long npix, double *partial, int nblocks,
                            double *out2, hipStream_t s);
int launch_rho_from_data(const double *d, const double *M, double *rho, long npix, int nb,
                         hipStream_t s);
// out[0] = number of non-finite entries of x[0..n) (partial: nblocks doubles)
int launch_count_nonfinite(const double *x, long n, double *partial, int nblocks, double *out,
                           hipStream_t s);
int launch_chi2_pix(const double *rho, const double *M, const double *smap, long npix, int nb,
                    double lam, double tau, double *partial, int nblocks, double *diag,
                    hipStream_t s);
int launch_fluct_combine(const double *g1, const double *M, const double *ysh, double *rho,
                         long npix, int nb, double omega, hipStream_t s);

// ringfft.hip
int launch_fft_fwd(const Plan &p, const double *maps, double2 *phase, int nb);
// the forward transforms of the messenger field t of Eq. (3), formed from rho, M and s = maps
// on the fly (FP64 rows)
int launch_fft_fwd_pix(const Plan &p, const double *maps, const double *rho, double lam,
                       double2 *phase, int nb);
int launch_fft_inv(const Plan &p, const double2 *phase, double *maps, int nb);
// FP32 rows [map][ring][m]; with rho the input is the messenger field of Eq. (3) built from
// rho, M and s = maps on the fly
int launch_fft_fwd_f32(const Plan &p, const double *maps, const double *rho, double lam,
                       float2 *phase, int nb);
int launch_fft_inv_f32(const Plan &p, const float2 *phase, double *maps, int nb);
// synthesis columns d_ph32 -> maps s (to smap if not null) -> t of Eq. (3) -> the columns of
// its forward transform, in place (one iteration's ring steps without the map in memory)
// Fork the plan's side stream from its stream before the two in-LDS ring classes of the
// chained FP32 ring step, and join it back after them (no-ops without a side stream).
int ring_fork(const Plan &p);
int ring_join(const Plan &p);
int launch_fft_inv_fwd_cols(const Plan &p, const double *rho, double lam, double *smap, int nb);
// T, Q, U batched form: one iteration's ring steps on the columns d_ph32 / d_ph32p from the
// synthesis columns d_ph32 / d_ph32p (chained iterations), where fft_pol_chain_ok
bool fft_pol_chain_ok(const Plan &p);
int launch_fft_inv_fwd_pol_cols(const Plan &p, const double *rho, double lam, int nb);
int fft_class_shape(const Plan &p, int c, int &ept);  // threads per workgroup of class c
size_t fft_class_lds(const Plan &p, int c);           // dynamic LDS bytes of class c
// maps per workgroup of the columns ring step of class c for nb maps, and its dynamic LDS
int fft_cols_group(const Plan &p, int c, int nb);
int fft_cols_group_max(const Plan &p, int c, int nb);
size_t fft_cols_lds(const Plan &p, int c, int g);

// legendre.hip (alm_scaled: c_lm-scaled coefficients; apart: sums of mu_lm X)
int launch_leg_synth(const Plan &p, const double2 *alm_scaled, double2 *phase, int nb);
int launch_leg_analysis(const Plan &p, const double2 *phase, double2 *apart, int nb);
int leg_synth_variants();
int leg_analysis_variants();
int leg_synth_pairs_per_lane(int v);
int leg_analysis_pairs_per_lane(int v);

// batched.hip (FP32 form)
int launch_lam_table(const Plan &p);
int launch_lam_ckpt(const Plan &p);  // d_lck from the recurrence
int launch_rows_to_cols(const Plan &p, int nb);  // d_phf -> d_ph32
int launch_cols_to_rows(const Plan &p, int nb);  // d_ph32 -> d_phf
int launch_zero_map_cols(const Plan &p, int b);  // map b's columns of d_ph32 = 0
int launch_gemm_analysis(const Plan &p, int nb, float *a_out, float *s_out, double scale_s,
                         double lto, double lto_per_tau = 0.0);
int launch_gemm_synthesis(const Plan &p, int nb);
int launch_alm_to_cols(const Plan &p, const double2 *alm, float *x32, int nb, int mode);
int launch_cols_to_alm(const Plan &p, const float *x32, double2 *alm, int nb, double scale);
// w real columns per map (width w Bp); flip: the table has the opposite mirror symmetry
int launch_gemm_analysis_raw(const Plan &p, int nb, int w, const float *table, const float *cols,
                             float *a_out, int flip);
int launch_gemm_synthesis_on(const Plan &p, int nb, int w, const float *table, const float *s_in,
                             float *out, int flip, int comb = 0);

// polbatched.hip (batched FP32 form, spin 2)
enum PolCombineMode { kPolFilter = 0, kPolRaw = 1 };
int launch_pol_tables(const Plan &p);
int launch_rows_to_cols_pol(const Plan &p, int nb);            // d_phf -> d_ph32, d_ph32p
int launch_cols_to_rows_pol(const Plan &p, int nb);            // d_ph32, d_ph32p -> d_phf
int launch_pol_combine(const Plan &p, double lto, int mode);   // -> d_s32, d_seb32
int launch_alm_to_cols_pol(const Plan &p, const double2 *alm, int nb);  // -> d_s32, d_seb32
int launch_cols_to_alm_pol(const Plan &p, double2 *alm, int nb);        // d_s32, d_seb32 ->
int pol_analysis_b(const Plan &p, int nb, double lto, int mode);
int pol_synthesis_b(const Plan &p, int nb, bool rows = true);

// polar.hip (spin 2: maps [B][3][npix], alm [B][3][nalm], rows [3B][nring][nm])
int pol_ngroup(const Plan &p);
int launch_leg_synth_pol(const Plan &p, const double2 *alm_scaled, double2 *phase, int nb);
int launch_leg_analysis_pol(const Plan &p, const double2 *phase, double2 *apart, int nb);
int launch_harmonic_pol(const Plan &p, const double2 *in, int ngroup, double scale, double lto,
                        int mode, double2 *out_s, double2 *out_sp, double2 *prev, int nb);
int launch_pol_covariance(const double *ninv6, const uint8_t *mask, double *M6, long npix,
                          double *partial, int nblocks, double *out3, hipStream_t s);
int launch_rho_from_data_pol(const double *d, const double *M6, double *rho, long npix, int nb,
                             hipStream_t s);
int launch_pixel_update_pol(const double *rho, const double *M6, const double *smap, double *t,
                            long npix, int nb, double lam, double tau, hipStream_t s);
int launch_chi2_pix_pol(const double *rho, const double *M6, const double *smap, long npix,
                        int nb, double lam, double tau, double *partial, int nblocks,
                        double *diag, hipStream_t s);
int launch_harm_diag_pol(const Plan &p, const double2 *salm, const double2 *salm_prev, int nb,
                         double *partial, double *diag);
int launch_fluct_combine_pol(const double *g1, const double *M6, const double *ysh, double *rho,
                             long npix, int nb, double omega, hipStream_t s);

// error-bound schedule (Sect. 2.2): pixel term of chi^2 and its lambda-derivative per map
// (out2[b][2]; partial holds nb x nblocks x 2 doubles)
int launch_chi2_pix_dlam(const double *rho, const double *M, const double *smap, long npix,
                         int nb, double lam, double tau, double *partial, int nblocks,
                         double *out2, hipStream_t s);
int launch_chi2_pix_dlam_pol(const double *rho, const double *M6, const double *smap, long npix,
                             int nb, double lam, double tau, double *partial, int nblocks,
                             double *out2, hipStream_t s);
// out2[b][0..1] = sum over nblocks of partial[b][block][0..1], in block order
int launch_sum_pairs(const double *partial, int nblocks, int nb, double *out2, hipStream_t s);

// templates.hip (Eq. 12: monopole and dipole template removal)
int launch_template_sums(const Plan &p, const double *d, int nb, double *partial, double *out14);
int template_partial_doubles(int nb);
int launch_template_subtract(const Plan &p, const double *d, double *dout, int nb,
                             const double *coef);
// the same removal with every intermediate in the library's static device array (no
// allocation, no plan workspace); at most kNoAllocMaxMaps maps per call
constexpr int kNoAllocMaxMaps = 64;
int remove_templates_noalloc(const Plan &p, const double *d_raw, double *d_out, int nmaps);

// harmonic.hip
enum HarmMode { kHarmWiener = 0, kHarmAnalysis = 1, kHarmInvSqrtC = 2, kHarmCopy = 3 };
// mode 0 filter: C_l / (C_l + lto), or with p.d_tau set, lto = lto_per_tau * tau_b[map]
int launch_harmonic(const Plan &p, const double2 *in, int ngroup, double scale, double lto,
                    int mode, double2 *out_s, double2 *out_sp, double2 *prev, int nb,
                    double lto_per_tau = 0.0);
int launch_harm_diag(const Plan &p, const double2 *salm, const double2 *salm_prev, int nb,
                     double *partial, double *diag);
// coefficients of `rows` maps/components from src's band-limit packing to dst's (zeros above
// src's lmax), on dst's stream
int launch_repack_alm(const Plan &src, const double2 *a_src, const Plan &dst, double2 *a_dst,
                      int rows);

}  // namespace mfwf
