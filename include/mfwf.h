/*
 * mfwf.h -- messenger-field Wiener filter on the HEALPix sphere, HIP library for gfx950.
 *
 * Solves (S^-1 + N^-1) s_WF = N^-1 d (Eq. 2 of Elsner & Wandelt, "Efficient Wiener
 * filtering without preconditioning") with the messenger iteration of Sect. 2.1:
 * a pixel-space update of the messenger field t (Eq. 3, T = tau*1, Nbar = N - T), a
 * forward spherical-harmonic transform, a harmonic-space update of s (Eq. 4) and an
 * inverse transform, repeated.  Fluctuation sources for constrained realisations follow
 * Sect. 2.3 (Eq. 9).
 *
 * Conventions shared by every entry point
 *   - Maps are HEALPix RING order, npix = 12 nside^2 doubles per map.
 *   - Harmonic coefficients ("alm") are complex, m-major, (m, l = m..lmax), stored as
 *     interleaved (re, im) doubles: nalm = (lmax+1)(lmax+2)/2 complex values per map,
 *     index of (l, m) = m (2 lmax + 3 - m)/2 + (l - m).  a_{l,-m} = (-1)^m conj(a_lm).
 *   - Synthesis Y: map(p) = sum_{l,|m|<=l} a_lm Y_lm(p).  Analysis A = Omega Y^T:
 *     a_lm = Omega sum_p map(p) conj(Y_lm(p)), Omega = 4 pi / npix (uniform pixel weights).
 *   - Batched arrays are map-major: [nmaps][npix] and [nmaps][2*nalm].
 *   - Polarization (plans with spin = 2): every map is (T, Q, U) and every coefficient set
 *     (T, E, B), component-major within a map: [nmaps][3][npix] and [nmaps][3][2*nalm].
 *     Q, U follow the HEALPix / Zaldarriaga-Seljak convention: Q + iU = sum 2a_lm 2Y_lm,
 *     a_E = -(2a + (-2)a)/2, a_B = i (2a - (-2)a)/2, spin-weighted harmonics from the
 *     spin-raising operator, (+-2)Y_lm = sqrt((l-2)!/(l+2)!) (eth or eth-bar)^2 Y_lm.
 *     The analysis is again Omega times the adjoint of the synthesis.
 *   - Every pointer named "device" is a device pointer owned by the caller; the library
 *     keeps no reference to it after the call returns.  Host pointers are read during the
 *     call only.
 *   - All device work is enqueued on the plan's stream (the stream given at plan creation,
 *     or the null stream).  An MFWF_F32 plan also owns one non-blocking stream and two
 *     events: its iterations fork part of the ring step onto that stream from the plan's
 *     stream and join it back before the next launch, so the work stays ordered on the
 *     plan's stream as seen by the caller (graph capture of that stream records both).
 *     mfwf_solve and mfwf_set_covariances synchronise the plan's stream before returning;
 *     the transforms and mfwf_fluctuation_rhs return without waiting.
 *   - Status: 0 on success, a negative mfwf_status on failure; mfwf_last_error() then
 *     describes the failure (per calling thread).  On failure, outputs are undefined.
 *   - A plan serves one host thread / stream at a time; distinct plans are independent.
 */
#ifndef MFWF_H
#define MFWF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfwf_plan_s *mfwf_plan;

typedef enum {
    MFWF_OK = 0,
    MFWF_EINVAL = -1,  /* bad argument (size, pointer, unsupported option)        */
    MFWF_ENOMEM = -2,  /* device or host allocation failed                         */
    MFWF_ENOTSPD = -3, /* a noise block is not positive semi-definite              */
    MFWF_ENOCOV = -4,  /* covariances not set, or no observed pixel (tau undefined) */
    MFWF_EDEVICE = -5, /* HIP runtime error                                        */
    MFWF_ENAN = -6     /* non-finite value met in the input or the iterate          */
} mfwf_status;

typedef enum {
    MFWF_F64 = 0, /* every step in double precision                               */
    MFWF_F32 = 1  /* batched form: the Legendre contractions (Sect. 3's transform
                     cost) run as FP32 matrix-core products over all maps of a call,
                     from an FP32 table of lambda_lm; maps, the pixel update, the ring
                     transforms, the harmonic filter's arithmetic and all norms stay
                     FP64.  ~1e-7 relative error per transform, 8e-6 after 300
                     iterations at nside 512 / lmax 1024                          */
} mfwf_dtype;

/*
 * Create a plan for HEALPix resolution nside (power of two, 1..2048; 1..1024 for MFWF_F32
 * with spin 2)
 * and band limit lmax (1..4*nside).  spin: 0 = temperature only, 2 = temperature and
 * polarization (T, Q, U maps, T, E, B coefficients, 3x3 noise and signal blocks).
 * max_batch (>= 1): largest number of maps one call processes at once (larger calls are
 * split).  hip_stream: a hipStream_t
 * or NULL for the null stream.  The plan precomputes the ring geometry (HEALPix,
 * Gorski et al. 2005), the Legendre recurrence coefficients and, for every (m, ring
 * pair), the first l at which the normalised associated Legendre function exceeds 2^-100
 * together with its two starting values, and ring-FFT tables.  It allocates its device
 * workspaces up front (MFWF_F32 adds the FP32 lambda table, 4 bytes x ring pairs x
 * (lmax+1)(lmax+2)/2 roughly: 2.2 GB at nside 512 / lmax 1024, for nside <= 1024, and for
 * temperature plans the FP64 state of the Legendre recurrence at every 16th l of each
 * (m, ring pair), a quarter of the table's size, from which the contractions can generate
 * lambda themselves (the only form above nside 1024: 36 GB at nside 2048 / lmax 4096);
 * column-major work arrays for max_batch maps; with spin 2 also FP32 tables of the spin-2
 * functions F+-_lm = ((2)lambda_lm +- (-2)lambda_lm)/2, two more tables of that size).  *out receives
 * the handle.  Ring transforms whose chirp-z convolution would exceed 8192 points (polar
 * rings of more than 4096 pixels, nside 2048) are split into four chirp-z transforms of a
 * quarter length each, with a device scratch of 32 bytes x ring pixels of those rings per
 * map and component; the environment variable MFWF_FFT_SPLIT_LEN (a power of two >= 16,
 * read here) lowers that 8192 so that tests can send small plans through the split path.
 * Errors: MFWF_EINVAL for out-of-range sizes or spin not 0 or 2; MFWF_ENOMEM, MFWF_EDEVICE.
 */
int mfwf_plan_create(int nside, int lmax, int spin, int dtype, int max_batch, void *hip_stream,
                     mfwf_plan *out);

/* Release every device and host resource of the plan.  NULL is accepted. */
int mfwf_plan_destroy(mfwf_plan plan);

/*
 * Set the signal and noise covariances (Sect. 2.1, Eq. 2).
 *   cl    host, [ncl][lmax+1] signal power spectrum C_l (ncl = 1 for temperature);
 *         C_l = 0 removes the multipole from the solution.  Negative C_l -> MFWF_EINVAL.
 *         spin 2: ncl = 4, rows TT, EE, BB, TE; S_l = [[TT, TE, 0], [TE, EE, 0], [0, 0, BB]]
 *         must be positive semi-definite (TE^2 <= TT EE), else MFWF_EINVAL.
 *   ninv  device, [npix] inverse noise variance N^-1 per pixel (>= 0); spin 2: [npix][6],
 *         the symmetric 3x3 block N_p^-1 of (T, Q, U) packed (TT, TQ, TU, QQ, QU, UU).
 *   mask  device, [npix] uint8, 1 = observed, 0 = masked (M = 0); NULL = all observed.
 * The plan stores M = ninv * mask and tau = min diag N over observed pixels = 1 / max M
 * (spin 2: tau = 1 / max_p lambda_max(M_p), the largest T = tau 1 with N - T >= 0 in every
 * pixel; the chi^2 degrees of freedom count 3 per pixel with det M_p > 0).
 * Errors: MFWF_ENOCOV if max M <= 0, MFWF_ENAN if M has a non-finite or negative entry;
 * spin 2: MFWF_ENOTSPD if a block is non-finite or not positive semi-definite.
 */
int mfwf_set_covariances(mfwf_plan plan, const double *cl, int ncl, const double *ninv,
                         const uint8_t *mask);

/* As mfwf_set_covariances with an instrumental transfer function (Sect. 3): the signal
 * covariance in the data is S_l = b_l^2 C_l (every spectrum of a spin-2 plan scaled alike),
 * so the filter returns the beam-convolved sky.  bl: host [lmax+1] finite, or NULL (b = 1).
 * Errors: as mfwf_set_covariances, MFWF_EINVAL for a non-finite b_l. */
int mfwf_set_covariances_beam(mfwf_plan plan, const double *cl, int ncl, const double *bl,
                              const double *ninv, const uint8_t *mask);

/* Monopole and dipole removal of Eq. (12): d = lim_{sigma -> inf} (1 + sigma V V^T)^-1 d_raw
 * with V the templates 1, x, y, z (unit vector of the pixel centre) on the observed pixels
 * of the plan's covariances, i.e. d = d_raw - V (V^T V)^-1 V^T d_raw; masked pixels keep
 * d_raw.  d_raw, d_out: device [nmaps][npix] (spin 2: [nmaps][3][npix], templates on T,
 * Q and U copied); d_out may equal d_raw.  Errors: MFWF_ENOCOV before
 * mfwf_set_covariances, MFWF_EINVAL if the templates are degenerate on the observed pixels. */
int mfwf_remove_templates(mfwf_plan plan, const double *d_raw, double *d_out, int nmaps);

/* For callers that cannot allocate device memory (code under stream capture, serving loops
 * that forbid hipMalloc): mfwf_remove_templates with no allocation and no use of the plan's
 * workspaces.  The partial sums, the 4 x 4 solves (done on the device) and a status flag per
 * map live in one static device array of 467,968 bytes that each device holds for the life
 * of the process.  At most 64 maps per call (more -> MFWF_EINVAL, nothing launched).  Calls
 * that overlap on one device (from two streams or threads) race on that array and must be
 * serialised by the caller.  Same arguments, results and errors as mfwf_remove_templates;
 * waits for the plan's stream before returning. */
int mfwf_remove_templates_noalloc(mfwf_plan plan, const double *d_raw, double *d_out, int nmaps);

/*
 * Synthesis map = Y alm for nmaps maps (the inverse transform that closes each
 * iteration, Sect. 2.1).  alm: device [nmaps][2*nalm]; map: device [nmaps][npix]
 * (spin 2: [nmaps][3][2*nalm] T, E, B -> [nmaps][3][npix] T, Q, U).
 */
int mfwf_sht_inv(mfwf_plan plan, const double *alm, double *map, int nmaps);

/*
 * Analysis alm = Omega Y^T map for nmaps maps (the forward transform of Sect. 2.1).
 * map: device [nmaps][npix]; alm: device [nmaps][2*nalm] (spin 2: [nmaps][3][...]).
 */
int mfwf_sht_fwd(mfwf_plan plan, const double *map, double *alm, int nmaps);

/*
 * Constrained-realisation source (Sect. 2.3, Eq. 9): the replacement
 * Nbar^-1 d -> Nbar^-1 N (N^-1/2 g1 + S^-1/2 g2) becomes, in the per-pixel form used by
 * mfwf_solve, the source
 *     rho = M^{1/2} g1 + Omega * Y(C^{-1/2} h)
 * (C^{-1/2} := 0 where C_l = 0).  Masked pixels (M = 0) automatically receive the
 * identity replacement of Nbar^-1 N that the paper prescribes.
 *   g1   device [nrhs][npix] unit normal draws per pixel.
 *   h    device [nrhs][2*nalm] unit-white harmonic draws in the real basis, complex
 *        packing: m = 0 entries real N(0,1), m > 0 entries (x + i y)/sqrt(2).
 *   rho  device [nrhs][npix] output; pass it to mfwf_solve with source_is_rho = 1.
 * spin 2: g1, rho [nrhs][3][npix], h [nrhs][3][2*nalm]; M^{1/2} is the Cholesky factor
 * L_p (L_p L_p^T = M_p) and C^{-1/2} the factor K_l = L_S^{-T} of S_l = L_S L_S^T on the
 * components with power (K K^T = S_l^{-1} there).
 * Requires mfwf_set_covariances.  The draws are inputs: the library draws nothing.
 */
int mfwf_fluctuation_rhs(mfwf_plan plan, const double *g1, const double *h, int nrhs,
                         double *rho);

/* Iteration schedule and options for mfwf_solve. */
typedef struct {
    int n_stages;          /* number of (lambda, iters) stages; 0 = one stage {1.0, 300} */
    const double *lambda;  /* host [n_stages], each >= 1 (Sect. 2.2)                     */
    const int *iters;      /* host [n_stages], iterations per stage (>= 0)              */
    int n_check;           /* diagnostics every n_check iterations (0 = only at the end) */
    double dchi2_tol;      /* 0: run the whole schedule; > 0 (needs n_check > 0): end
                              early once the change of chi^2 between two checks of one
                              stage, per iteration, is below dchi2_tol sigma_chi2 for
                              every map of a chunk (maps are solved in chunks of at most
                              max_batch; sigma_chi2 = sqrt(2 n_dof), Sect. 2.2);
                              iters_done reports where each map stopped; the host then
                              waits for the stream at every check                        */
    int source_is_rho;     /* 0: input is the data d (rho = M d); 1: input is rho        */
    int use_graph;         /* 1: replay each iteration as a captured hipGraph            */
    double *history;       /* host [history_rows][nmaps][5] or NULL: at every check,
                              (iteration k, lambda, chi^2 of Eq. 6, |s_k - s_{k-1}|,
                              |s_k|) per map; checks at k = n_check, 2 n_check, ... and
                              at the last iteration; rows beyond history_rows are not
                              written                                                    */
    int history_rows;      /* capacity of history in rows                                */
    int order;             /* FP32 form: 0 = chained iterations (each starts from the
                              previous synthesis in the matrix-core columns; T, and T, Q,
                              U up to nside 512), 1 = every iteration from the pixel map
                              (forward transforms, layout change, contractions, layout
                              change, inverse transforms).  Same values either way; 1
                              exists to check that.  Ignored by FP64 plans.              */
} mfwf_solve_opts;

/* Per-map diagnostics after the last iteration (Eq. 6 and Sect. 2.2). */
typedef struct {
    int iters_done;    /* iterations run                                               */
    double lambda;     /* lambda of the last iteration                                 */
    double chi2;       /* chi^2(s, lambda) of Eq. (6) at the final iterate             */
    double chi2_harm;  /* its harmonic part s^T S^-1 s                                 */
    double dnorm;      /* |s_k - s_{k-1}| over the real harmonic dof (m > 0 twice)     */
    double snorm;      /* |s_k|                                                        */
    double tau;        /* tau = 1 / max M                                              */
    long n_dof;        /* number of observed pixels (chi^2 degrees of freedom)          */
    int n_checks;      /* diagnostic checks made (rows of opts->history filled, up to
                          its capacity)                                                 */
    double dchi2;      /* change of chi^2 per iteration between the last two checks of
                          the final stage (negative while chi^2 falls); 0 with fewer
                          than two checks there, and for mfwf_solve_bounded, whose
                          lambda changes every iteration                                */
    double rel_change; /* dnorm / snorm: relative change of the last iteration (0 if
                          snorm = 0)                                                    */
} mfwf_solve_info;

/*
 * Run the messenger iteration for nmaps right-hand sides.
 *   input      device [nmaps][npix]: d (source_is_rho = 0) or rho (source_is_rho = 1).
 *   s_alm_out  device [nmaps][2*nalm] or NULL: final harmonic iterate s_lm.
 *   s_map_out  device [nmaps][npix] or NULL: its synthesis Y s.
 *   opts       NULL = lambda = 1 for 300 iterations.
 *   info       host [nmaps] or NULL.
 * Starts from s = t = 0; each iteration at lambda runs, per pixel,
 *     t = [lambda tau rho + (1 - tau M) s] / [1 + (lambda - 1) tau M]
 * (Eq. 3 multiplied through by N, no inverse of Nbar), then
 *     s_lm = C_l / (C_l + lambda tau Omega) * (A t)_lm     (Eq. 4, T = tau Omega per
 * harmonic dof under A = Omega Y^T), then s = Y s_lm.  Non-convergence is not an error.
 * Errors: MFWF_ENAN if the source holds a NaN or Inf (data on an observed pixel, or any
 * entry of a given rho), checked before the first iteration; MFWF_ENOCOV without
 * covariances; MFWF_EINVAL for bad options.
 * spin 2: input and s_map_out [nmaps][3][npix], s_alm_out [nmaps][3][2*nalm]; the pixel
 * update solves the 3x3 system [I + (lambda - 1) tau M_p] t = lambda tau rho +
 * (I - tau M_p) s per pixel and the harmonic update is s = S_l (S_l + lambda tau Omega I)^-1 a
 * per (l, m) on (T, E, B).
 */
int mfwf_solve(mfwf_plan plan, const double *input, int nmaps, double *s_alm_out,
               double *s_map_out, const mfwf_solve_opts *opts, mfwf_solve_info *info);

/*
 * ---- Converged Wiener filter with the cooling schedule of Sect. 3 ------------------------
 * lambda starts from the signal power at l_iter: lambda = max(1, C^TT_{l_iter} / (tau Omega))
 * (the messenger covariance lambda T then equals the signal power at l_iter, so modes above
 * l_iter are held back), with l_iter = l_iter0 at first.  Each stage iterates Eqs. (3)-(4)
 * at its lambda until chi^2(lambda, s) of Eq. (6) reaches a plateau; the next stage takes
 * l_iter' = min(2 l_iter, l_iter + l_step_max) and its lambda, never below 1.  The solve
 * ends when the change of chi^2 at lambda = 1 over the full band limit falls below
 * final_tol sigma_chi2 per iteration (sigma_chi2 = sqrt(2 n_dof), Sect. 2.2).  While lambda
 * holds back the modes above l_iter, the transforms run only up to
 * lmax_SHT = min(lmax, l_iter + l_margin) (Sect. 3): those stages run on plans of the same
 * nside with that band limit, which the plan creates on first use and keeps (covariances
 * copied from it), and the iterate passes between stages as its pixel map.
 * A plateau: |chi^2_k - chi^2_{k - n_check}| / n_check < tol sigma_chi2 for every map of
 * the batch, checked every n_check iterations.  The input is data d (rho = M d).
 * Spin 0 or spin 2, MFWF_F64 or MFWF_F32.  For spin 2 (the T+P analysis of Sect. 3) lambda
 * follows the temperature spectrum, C^TT_{l_iter}, the stages truncate the (T, E, B)
 * spectra at lmax_SHT and chi^2 is the T, Q, U form of Eq. (6) with 3 n_observed dof.
 */
typedef struct {
    int l_iter0;         /* first l_iter (0: 20)                                          */
    int l_step_max;      /* largest increase of l_iter per stage (0: 500)                 */
    int l_margin;        /* lmax_SHT = min(lmax, l_iter + l_margin) (0: 100; < 0: lmax)   */
    int n_check;         /* iterations between chi^2 evaluations (0: 5)                   */
    double plateau_tol;  /* stage end, in sigma_chi2 per iteration (0: 1e-2)              */
    double final_tol;    /* end of the solve at lambda = 1, full lmax (0: 1e-4)           */
    int max_iters;       /* cap on the iterations of all stages (0: 20000)                */
    double *stages;      /* host [stage_rows][5] or NULL, per stage: l_iter, lambda,
                            lmax_SHT, iterations, chi^2 / n_dof at its end (map 0)        */
    int stage_rows;      /* capacity of stages in rows                                    */
    int n_stages;        /* out: stages run (rows beyond stage_rows are not written)      */
    int converged;       /* out: 1 if the final criterion was met, 0 if max_iters ended it */
} mfwf_cool_opts;

/* input, outputs and info as in mfwf_solve (nmaps maps of data; the maps of one batch of
 * max_batch share one schedule, and stages reports the last batch's).  opts may be NULL
 * (all defaults).  Errors: as mfwf_solve, MFWF_EINVAL for negative options or
 * n_check = 1; MFWF_ENAN when chi^2 becomes non-finite or, at a check, stands more than
 * 10 sigma_chi2 above its lowest value in the current stage after three rises between
 * checks, each larger than the one before (at fixed lambda the iteration lowers chi^2 up to
 * the pixelisation's quadrature gap, and may settle above a minimum it passed through by
 * shrinking rises; growing rises mean an unstable iteration: lmax too high for the nside
 * and noise pattern, as at lmax = 2 nside for some problems, whose plain iteration grows
 * after a few hundred to a few thousand iterations). */
int mfwf_solve_cooled(mfwf_plan plan, const double *data, int nmaps, double *s_alm_out,
                      double *s_map_out, mfwf_cool_opts *opts, mfwf_solve_info *info);

/*
 * ---- Wiener filter under an error bound (Sect. 2.2) ----------------------------------------
 * At fixed lambda the iteration minimises chi^2(x, lambda) of Eq. (6), whose minimum
 * chi^2_min(lambda) lies below chi^2_min(1) for lambda > 1.  With a target b <= chi^2_min(1)
 * (initially b = n_dof - m_sigma sigma_chi2, sigma_chi2 = sqrt(2 n_dof)): from x = 0, lambda is
 * set so that chi^2(lambda, 0) = b; each iteration at lambda lowers chi^2(lambda, x) below b,
 * and lambda is then lowered until chi^2(lambda, x) = b again, so chi^2(lambda, x) <= b holds
 * throughout.  When lambda stops falling (it has converged at lambda > 1 because b lies
 * below chi^2_min(1)), b is raised to b' = chi^2_min(lambda) + (lambda - 1) tau x^T S^-2 x
 * (evaluated as chi^2(lambda, x) minus (lambda - 1) times the lambda-derivative of its pixel
 * term, equal at the minimiser), which stays below chi^2_min(1) to second order.  On the
 * pixelised sphere the iteration's fixed point misses the exact minimiser of chi^2 by the
 * quadrature gap, so an iteration at fixed lambda can raise chi^2(lambda, x) by that
 * margin; lambda is then raised until the bound holds again.  The solve ends with one
 * iteration at lambda = 1 once lambda <= 1 + lam_tol.  A batch takes one lambda per
 * iteration, the largest its maps need, so every map keeps its bound.  chi^2(lambda, x) is
 * decreasing and convex in lambda; the new lambda comes from a safeguarded Newton search on
 * the pixel term (one pass over the maps per step) and meets the bound exactly.
 * Spin 0 or spin 2, MFWF_F64 or MFWF_F32; input data d (rho = M d).  For spin 2 the pixel
 * term is the T, Q, U form q^T B^-1 q, q = rho - M s, B = M + (lambda - 1) tau M^2 per block,
 * with derivative -tau |M B^-1 q|^2, and n_dof counts 3 per observed pixel.
 */
typedef struct {
    double m_sigma;      /* initial b = n_dof - m_sigma sigma_chi2 (0: 5)                   */
    double lam_tol;      /* end once lambda <= 1 + lam_tol (0: 1e-3)                        */
    double stall_frac;   /* lambda stalls when it falls by less than this fraction (0: 1e-3) */
    int stall_iters;     /* stalled iterations in a row before b is raised (0: 5)           */
    int max_iters;       /* cap on the iterations (0: 5000)                                 */
    double *trace;       /* host [trace_rows][3] or NULL, per iteration: lambda used,
                            chi^2(lambda, x) after it and b (map 0)                         */
    int trace_rows;      /* capacity of trace in rows                                       */
    int n_iters;         /* out: iterations run                                             */
    int n_b_updates;     /* out: times b was raised                                         */
    int reached_one;     /* out: 1 if the last iteration ran at lambda = 1 (0: max_iters
                            ended the solve before it)                                      */
} mfwf_bound_opts;

/* input, outputs and info as in mfwf_solve; opts may be NULL (all defaults).  Errors: as
 * mfwf_solve; MFWF_EINVAL for negative options; MFWF_ENAN if chi^2 is not
 * finite. */
int mfwf_solve_bounded(mfwf_plan plan, const double *data, int nmaps, double *s_alm_out,
                       double *s_map_out, mfwf_bound_opts *opts, mfwf_solve_info *info);

/*
 * Time the plan's kernels on its stream with HIP events (diagnostic).  Runs `reps`
 * back-to-back launches of each stage of one iteration on the current workspaces for
 * nmaps maps and writes the mean duration in milliseconds of each kernel to ms_out:
 * [0] pixel update, [1] forward ring FFT, [2] Legendre analysis, [3] harmonic update,
 * [4] Legendre synthesis, [5] inverse ring FFT.  A stage that runs inside another kernel
 * reads 0: in the FP64 temperature path the pixel update runs in [1]; in the batched FP32
 * temperature form the pixel update runs in [1] and the
 * harmonic update in [2], and [1] is the whole ring step of a chained iteration (layout
 * transposes, the previous synthesis back to pixels, pixel update, forward transforms), so
 * [5] is 0 as well.  Requires mfwf_set_covariances.
 */
int mfwf_time_kernels(mfwf_plan plan, int nmaps, int reps, double *ms_out);

/*
 * Work statistics of the plan (host, 4 doubles):
 * [0] (l, m, ring pair) triples the Legendre steps evaluate, i.e. l >= the pair's start
 *     index (terms below 2^-100 skipped); [1] the full triangle: ring pairs * nalm;
 * [2] ring pairs; [3] the largest ring-FFT length used.
 */
int mfwf_plan_work(mfwf_plan plan, double *out4);

/*
 * Kernel shapes the plan uses (host, 8 ints): [0] FP64 Legendre synthesis variant (0..8),
 * [1] analysis variant (0..5), [2] maps per workgroup of the batched form's ring step for
 * the shorter transforms and [3] for the longest (1, 2, 4), [4] column tile of the analysis
 * GEMM (1: 64 columns in 4 waves, 2: 128 columns in 4 waves, 3: 128 columns in 8 waves) and
 * [5] largest column tile of the synthesis GEMM, in units of 64 columns (1, 2), [6] 1 if the
 * temperature GEMMs generate lambda_lm from the FP64 recurrence (its state every 16 values
 * of l, tabulated per plan) instead of reading the FP32 table (0; no table above nside 1024),
 * [7] how they were set: 0 defaults, 1 by the autotuner at plan creation (timed, or read
 * from its cache), 3 from the environment variable MFWF_TUNE_FORCE.  None of them changes a
 * result of the batched form; the FP64 Legendre variants add the ring pairs' partial sums
 * in different groupings.  The autotuner (MFWF_AUTOTUNE unset or not "0", plans of 256 ring pairs or
 * more) times every applicable value of each at plan creation and caches the choice per
 * (device, library build, nside, lmax, max_batch, dtype, spin) in $MFWF_TUNE_CACHE (default
 * $XDG_CACHE_HOME/mfwf/tune.txt or ~/.cache/mfwf/tune.txt).  MFWF_TUNE_FORCE =
 * "synth=3,ana=1,g0=2,g1=1,cta=1,cts=2,lamgen=1" (any subset) sets them at plan creation for any
 * plan size; a malformed value makes mfwf_plan_create fail with MFWF_EINVAL.
 */
int mfwf_plan_tuning(mfwf_plan plan, int *out8);

/*
 * ---- Serving: many independent requests on one GPU (continuous batching) --------------
 * Each request is one temperature Wiener-filter solve with its own data, noise variance
 * map and mask.  Requests with the same (nside, lmax, dtype, lambda, C_l) share a pool: a
 * plan with `slots` map slots, each holding its own M = N^-1 mask and tau = 1 / max M.  A
 * worker thread admits queued requests into free slots between iterations, runs one
 * messenger iteration (Eqs. 3-4) over the occupied slots of every busy pool (pools on
 * separate streams overlap on the GPU), and retires a request after its `iters`
 * iterations by copying s_lm and Y s into the caller's buffers.  Pools are created on
 * demand while their estimated device footprint fits the HBM budget; idle pools are
 * evicted (least recently used first) to make room.  Results equal those of mfwf_solve on
 * the same inputs (starting from s = 0).
 */
typedef struct mfwf_server_s *mfwf_server;

typedef struct {
    int nside, lmax;        /* as in mfwf_plan_create (temperature)                       */
    int dtype;              /* MFWF_F64 or MFWF_F32                                        */
    int iters;              /* messenger iterations (>= 1)                                 */
    double lambda;          /* constant lambda of Sect. 2.2 (>= 1)                         */
    const double *cl;       /* host [lmax+1], copied by mfwf_server_submit                 */
    const double *ninv;     /* device [npix] inverse noise variance (>= 0)                 */
    const uint8_t *mask;    /* device [npix], 1 = observed; NULL = all observed            */
    const double *data;     /* device [npix] data d                                        */
    double *s_alm_out;      /* device [2*nalm] or NULL: final s_lm                         */
    double *s_map_out;      /* device [npix] or NULL: Y s                                  */
} mfwf_request;

/* Device bytes a pool of this shape is charged against the HBM budget (an estimate of
 * its plan's allocations, with a fixed allowance for tables and workspaces), so callers
 * can size the budget.  Host only, no device call.  Errors: MFWF_EINVAL. */
int mfwf_server_pool_bytes(int nside, int lmax, int dtype, int slots, double *bytes);

/* Start a server on the current device with `slots` map slots per pool and a device
 * memory budget (GB) for its pools.  A shape whose pool would take more than half the
 * budget gets fewer slots: the first of slots, slots / 2, slots / 4, ..., 1 whose
 * mfwf_server_pool_bytes fits half the budget (at least one slot, refused with
 * MFWF_ENOMEM at submission if one slot exceeds the whole budget).
 * Errors: MFWF_EINVAL, MFWF_ENOMEM, MFWF_EDEVICE. */
int mfwf_server_create(int slots, double hbm_budget_gb, mfwf_server *out);

/* Queue one request; *id receives its handle.  The device arrays must hold their final
 * contents when this is called and stay valid until mfwf_server_wait returns for the
 * request (they are read when it is admitted and written when it retires).  ninv * mask
 * is checked here: MFWF_ENAN (negative or non-finite) or MFWF_ENOCOV (no observed pixel);
 * so is the data: MFWF_ENAN if it holds a NaN or Inf on an observed pixel;
 * MFWF_EINVAL for bad sizes or options (nside a power of two up to 2048). */
int mfwf_server_submit(mfwf_server s, const mfwf_request *req, uint64_t *id);

/* *done = 1 once the request's results are in the caller's buffers. */
int mfwf_server_poll(mfwf_server s, uint64_t id, int *done);

/* Block until the request is done; *latency_s (nullable) receives the time from
 * submission to the completion of the result copies.  Returns the request's status (e.g.
 * MFWF_ENOMEM when no pool of its shape fits the budget); the id is released. */
int mfwf_server_wait(mfwf_server s, uint64_t id, double *latency_s);

/* Counters (host, 8 doubles): [0] requests completed, [1] submitted but not yet seen by
 * the worker, [2] occupied slots, [3] pools, [4] budgeted bytes of the pools,
 * [5] iterations launched (summed over pools), [6] pools created, [7] pools evicted. */
int mfwf_server_stats(mfwf_server s, double *out8);

/* Finish every queued request, stop the worker and release the pools. */
int mfwf_server_destroy(mfwf_server s);

/* Message describing the last failure on this thread ("" if none). */
const char *mfwf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MFWF_H */
