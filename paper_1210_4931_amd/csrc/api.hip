// C-ABI of the mfwf library: plan construction (HEALPix ring geometry, Legendre recurrence
// tables and start seeds, ring-FFT tables, kernel-variant autotuning), covariance set-up,
// the transforms, the fluctuation source and the messenger-iteration driver (Sect. 2.1).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <thread>
#include <vector>

#include "mfwf_internal.h"

struct mfwf_plan_s {
    mfwf::Plan p;
    // Cooling schedule (Sect. 3): its early stages run on plans of the same nside with a
    // smaller band limit, created on first use and kept, by lmax.  cl holds the spectra
    // given to mfwf_set_covariances ([ncl][lmax+1]); cov_gen counts those calls, so a
    // sub-plan copies the covariances again after they change.
    struct Sub {
        mfwf::Plan p;
        long gen = -1;
    };
    std::map<int, std::unique_ptr<Sub>> sub;
    std::vector<double> cl;
    long cov_gen = 0;
};

namespace mfwf {

int fft_set_lds_limit(size_t bytes);  // ringfft.hip
int fft_max_length();                 // ringfft.hip

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

int fail(int status, const std::string &msg) {
    set_error(msg);
    return status;
}

template <typename T>
static int dalloc(T **ptr, size_t count, const char *what) {
    *ptr = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)ptr, sizeof(T) * count);
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(MFWF_ENOMEM, std::string("hipMalloc of ") + what + " (" +
                                     std::to_string(sizeof(T) * count) + " bytes) failed: " +
                                     hipGetErrorString(e));
    }
    return MFWF_OK;
}

template <typename T>
static int upload(T *dst, const std::vector<T> &src, hipStream_t s) {
    MFWF_HIP(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
    return MFWF_OK;
}

// ---- host-side plan tables ----------------------------------------------------------------

struct RingGeom {
    double z, sth;
    int nphi, half_shift;  // phi_0 = pi / nphi if half_shift, else 0
    long start;
};

// HEALPix RING ring i (1-based, north to south).
static RingGeom ring_geom(int nside, int i) {
    RingGeom r{};
    const double ns = nside;
    const long npix = 12L * nside * nside;
    if (i < nside) {
        const double omz = (double)i * i / (3.0 * ns * ns);
        r.z = 1.0 - omz;
        r.sth = std::sqrt(omz * (2.0 - omz));
        r.nphi = 4 * i;
        r.start = 2L * i * (i - 1);
        r.half_shift = 1;
    } else if (i <= 3 * nside) {
        r.z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns);
        r.sth = std::sqrt((1.0 - r.z) * (1.0 + r.z));
        r.nphi = 4 * nside;
        r.start = 2L * nside * (nside - 1) + (long)(i - nside) * 4L * nside;
        r.half_shift = ((i - nside) % 2 == 0) ? 1 : 0;
    } else {
        const int k = 4 * nside - i;
        const double omz = (double)k * k / (3.0 * ns * ns);
        r.z = -(1.0 - omz);
        r.sth = std::sqrt(omz * (2.0 - omz));
        r.nphi = 4 * k;
        r.start = npix - 2L * k * (k + 1);
        r.half_shift = 1;
    }
    return r;
}

static bool is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }
static int next_pow2(long n) {
    int v = 1;
    while (v < n) v <<= 1;
    return v;
}

// In-place radix-2 forward DFT (natural order in and out) for plan-time tables.
static void host_fft(std::vector<double2> &x) {
    const int n = (int)x.size();
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        for (int k = 0; k < len / 2; k++) {
            const double a = -2.0 * M_PI * k / len;
            const double wr = std::cos(a), wi = std::sin(a);
            for (int i = k; i < n; i += len) {
                double2 u = x[i], v = x[i + len / 2];
                double2 t = make_double2(v.x * wr - v.y * wi, v.x * wi + v.y * wr);
                x[i] = make_double2(u.x + t.x, u.y + t.y);
                x[i + len / 2] = make_double2(u.x - t.x, u.y - t.y);
            }
        }
    }
}

// Orthonormal recurrence lambda_l = alpha_l z lambda_{l-1} - beta_l lambda_{l-2} with
// eps_lm = sqrt((l^2 - m^2)/(4 l^2 - 1)), alpha = 1/eps_lm, beta = eps_{l-1,m}/eps_lm, and its
// rescaled form lambda_l = c_l mu_l, c_m = c_{m+1} = 1, c_l = beta_l c_{l-2}:
//   mu_l = A_l z mu_{l-1} - mu_{l-2},  A_l = alpha_l c_{l-1} / c_l  (A_m = 0: seed value).
static void build_recurrence(int lmax, std::vector<double2> &ab, std::vector<double> &A,
                             std::vector<double> &c, std::vector<long> &mofs) {
    const long nalm = (long)(lmax + 1) * (lmax + 2) / 2;
    ab.assign(nalm, make_double2(0.0, 0.0));
    A.assign(nalm, 0.0);
    c.assign(nalm, 1.0);
    mofs.resize(lmax + 1);
    for (int m = 0; m <= lmax; m++) {
        const long off = (long)m * (2 * lmax + 3 - m) / 2;
        mofs[m] = off;
        double eps_prev = 0.0;  // eps_{m,m} = 0
        for (int l = m + 1; l <= lmax; l++) {
            const double eps = std::sqrt(((double)l * l - (double)m * m) / (4.0 * l * l - 1.0));
            const double alpha = 1.0 / eps, beta = eps_prev / eps;
            ab[off + l - m] = make_double2(alpha, beta);
            if (l >= m + 2) c[off + l - m] = beta * c[off + l - m - 2];
            A[off + l - m] = alpha * c[off + l - m - 1] / c[off + l - m];
            eps_prev = eps;
        }
    }
}

// For every (m, pair): first l with |lambda_lm(z)| >= 2^-100 and (mu_{l-1}, mu_l) there.
// lambda_mm = (-1)^m sqrt(1/4pi) prod_{k<=m} sqrt((2k+1)/(2k)) sin(theta) is carried as a
// mantissa and a power-of-two exponent (it underflows double long before m = lmax near
// the poles); the l-recurrence runs in the same scaled form until the threshold.
static void build_seeds(int lmax, int npair, const std::vector<RingGeom> &geo,
                        const std::vector<double2> &ab, const std::vector<double> &c,
                        const std::vector<long> &mofs, std::vector<int> &lstart,
                        std::vector<double2> &seed) {
    const int nm = lmax + 1;
    lstart.assign((size_t)nm * npair, lmax + 1);
    seed.assign((size_t)nm * npair, make_double2(0.0, 0.0));
    auto work = [&](int p0, int p1) {
        for (int p = p0; p < p1; p++) {
            const double z = geo[p].z, sth = geo[p].sth;
            int ex;
            double rmm = std::frexp(std::sqrt(1.0 / (4.0 * M_PI)), &ex);
            long emm = ex;
            for (int m = 0; m <= lmax; m++) {
                if (m > 0) {
                    rmm *= -std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * sth;
                    rmm = std::frexp(rmm, &ex);
                    emm += ex;
                }
                double p1v = rmm, p2v = 0.0;
                long e = emm;
                auto thr_of = [](long e_) {
                    const long t = -100 - e_;
                    return t > 1000 ? INFINITY : std::ldexp(1.0, (int)t);
                };
                double thr = thr_of(e);
                const double2 *abm = ab.data() + mofs[m] - m;
                const double *cm = c.data() + mofs[m] - m;
                const size_t slot = (size_t)m * npair + p;
                for (int l = m;; l++) {
                    if (l > m) {
                        const double2 cc = abm[l];
                        const double cur = cc.x * (z * p1v) - cc.y * p2v;
                        p2v = p1v;
                        p1v = cur;
                        if (std::fabs(p1v) > 0x1p+300) {
                            p1v = std::ldexp(p1v, -300);
                            p2v = std::ldexp(p2v, -300);
                            e += 300;
                            thr = thr_of(e);
                        }
                    }
                    if (std::fabs(p1v) >= thr) {
                        lstart[slot] = l;
                        const double lam_prev = std::ldexp(p2v, (int)e);
                        const double lam = std::ldexp(p1v, (int)e);
                        seed[slot] = make_double2(l > m ? lam_prev / cm[l - 1] : 0.0, lam / cm[l]);
                        break;
                    }
                    if (l == lmax) break;
                }
            }
        }
    };
    unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    if ((int)nt > npair) nt = npair;
    std::vector<std::thread> th;
    const int chunk = (npair + nt - 1) / nt;
    for (unsigned t = 0; t < nt; t++) {
        const int a = t * chunk, b = std::min(npair, (int)(t + 1) * chunk);
        if (a < b) th.emplace_back(work, a, b);
    }
    for (auto &t : th) t.join();
}

static void free_plan(Plan &p) {
    void *ptrs[] = {p.d_z,    p.d_A,    p.d_c,     p.d_lstart, p.d_seed,  p.d_pfft, p.d_plist,
                    p.d_tw,   p.d_twlo, p.d_twhi, p.d_chirp, p.d_bhat, p.d_mofs,   p.d_cl,    p.d_M, p.d_pc, p.d_tau,
                    p.d_rho,  p.d_t,    p.d_smap,  p.d_phase,  p.d_apart, p.d_salm,
                    p.d_salm_prev, p.d_sp, p.d_red, p.d_diag, p.d_lam, p.d_lck, p.d_segoff, p.d_loff, p.d_Lp,
                    p.d_minls32, p.d_ana_items, p.d_syn_items, p.d_ana_tab, p.d_syn_tab, p.d_lofi, p.d_phf, p.d_ph32, p.d_a32,
                    p.d_s32, p.d_fp, p.d_fm, p.d_ph32p, p.d_ap32, p.d_ar32, p.d_seb32,
                    p.d_fftsplit};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (p.side_fork) (void)hipEventDestroy(p.side_fork);
    if (p.side_join) (void)hipEventDestroy(p.side_join);
    if (p.side) (void)hipStreamDestroy(p.side);
    p.side = nullptr;
    p.side_fork = p.side_join = nullptr;
}

static int device_name(std::string &name) {
    int dev = 0;
    MFWF_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    MFWF_HIP(hipGetDeviceProperties(&prop, dev));
    name = prop.gcnArchName;
    if (name.compare(0, 6, "gfx950") != 0)
        return fail(MFWF_EDEVICE, "library is built for gfx950, device is " + name);
    return MFWF_OK;
}

// ---- autotuning ---------------------------------------------------------------------------
// Kernel shapes the plan chooses by timing (none changes what a result is, only how the work
// is laid out; the Legendre variants of the FP64 path also change the order in which the
// ring pairs' partial sums are added):
//   synth, ana  FP64 Legendre kernels: ring pairs per lane 1/2/4, coefficient block 4/8,
//               prefetch of the next block (9 synthesis, 6 analysis variants)
//   g0, g1      maps per workgroup of the batched form's ring step, short-transform class
//               and longest-transform class (1, 2 or 4; as LDS and 1024 threads allow)
//   cta, cts    largest column tile of the analysis / synthesis GEMMs, x 64 columns (1 or 2)
//   lamgen      temperature GEMMs: lambda read from the FP32 table (0) or generated from the
//               FP64 recurrence's segment states (1; the only choice above nside 1024)
// With MFWF_AUTOTUNE != 0 (default) a plan of at least 256 ring pairs times every value of
// each knob that applies to it on its own stream (3 launches after a warm-up, on filled
// work arrays) and keeps the fastest.  Choices are cached per (device, library source hash,
// nside, lmax, max_batch, dtype, spin) in $MFWF_TUNE_CACHE, default
// $XDG_CACHE_HOME/mfwf/tune.txt or ~/.cache/mfwf/tune.txt, so later plans of the same shape
// reuse them.  MFWF_TUNE_FORCE="synth=3,ana=1,cta=1,lamgen=1" (any subset) sets knobs
// directly, for every plan size, and skips timing.
#ifndef MFWF_SRC_HASH
#define MFWF_SRC_HASH "unversioned"
#endif

enum { kKnobSynth = 0, kKnobAna, kKnobG0, kKnobG1, kKnobCtA, kKnobCtS, kKnobLamGen, kNumKnobs };
static const char *const kKnobName[kNumKnobs] = {"synth", "ana", "g0", "g1", "cta", "cts", "lamgen"};

static void get_knobs(const Plan &p, int k[kNumKnobs]) {
    k[kKnobSynth] = p.synth_variant;
    k[kKnobAna] = p.ana_variant;
    k[kKnobG0] = p.ring_group[0];
    k[kKnobG1] = p.ring_group[1];
    k[kKnobCtA] = p.gemm_ct[0];
    k[kKnobCtS] = p.gemm_ct[1];
    k[kKnobLamGen] = p.lam_gen ? 1 : 0;
}

static bool knob_valid(int knob, int v) {
    switch (knob) {
        case kKnobSynth: return v >= 0 && v < leg_synth_variants();
        case kKnobAna: return v >= 0 && v < leg_analysis_variants();
        case kKnobG0: case kKnobG1: return v == 1 || v == 2 || v == 4;
        case kKnobLamGen: return v == 0 || v == 1;
        case kKnobCtA: return v >= 1 && v <= 3;
        default: return v == 1 || v == 2;
    }
}

static void set_knobs(Plan &p, const int k[kNumKnobs]) {
    p.synth_variant = k[kKnobSynth];
    p.ana_variant = k[kKnobAna];
    p.ring_group[0] = k[kKnobG0];
    p.ring_group[1] = k[kKnobG1];
    p.gemm_ct[0] = k[kKnobCtA];
    p.gemm_ct[1] = k[kKnobCtS];
    // generation needs the segment states, the table the table; otherwise the one there is
    p.lam_gen = p.d_lck != nullptr && (k[kKnobLamGen] || p.d_lam == nullptr);
}

static std::string tune_cache_path() {
    if (const char *e = std::getenv("MFWF_TUNE_CACHE")) return e;
    if (const char *x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/mfwf/tune.txt";
    const char *home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/mfwf/tune.txt";
}

static std::string tune_key(const Plan &p, const std::string &devname) {
    return devname.substr(0, 6) + ":" + MFWF_SRC_HASH + ":n" + std::to_string(p.nside) + ":l" +
           std::to_string(p.lmax) + ":b" + std::to_string(p.max_batch) + ":" +
           (p.dtype == MFWF_F32 ? "f32" : "f64") + ":s" + std::to_string(p.spin);
}

static bool tune_lookup(const std::string &key, int k[kNumKnobs]) {
    std::ifstream f(tune_cache_path());
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string kk;
        int v[kNumKnobs];
        if (!(is >> kk) || kk != key) continue;
        bool ok = true;
        for (int q = 0; q < kNumKnobs && ok; q++) ok = (is >> v[q]) && knob_valid(q, v[q]);
        if (ok) {
            for (int q = 0; q < kNumKnobs; q++) k[q] = v[q];
            found = true;
        }
    }
    return found;
}

static void tune_store(const std::string &key, const int k[kNumKnobs]) {
    const std::string path = tune_cache_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); i++)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    f << key;
    for (int q = 0; q < kNumKnobs; q++) f << " " << k[q];
    f << "\n";
}

// MFWF_TUNE_FORCE: "name=value" pairs separated by commas; returns false (with the error set)
// on a malformed string, an unknown name or a value out of range
static bool tune_force(const char *env, Plan &p) {
    int k[kNumKnobs];
    get_knobs(p, k);
    std::istringstream is(env);
    std::string tok;
    while (std::getline(is, tok, ',')) {
        const size_t eq = tok.find('=');
        if (eq == std::string::npos) return fail(MFWF_EINVAL, "MFWF_TUNE_FORCE: expected name=value"), false;
        const std::string name = tok.substr(0, eq);
        int q = 0;
        while (q < kNumKnobs && name != kKnobName[q]) q++;
        char *end = nullptr;
        const long v = std::strtol(tok.c_str() + eq + 1, &end, 10);
        if (q == kNumKnobs || !end || *end != '\0' || !knob_valid(q, (int)v))
            return fail(MFWF_EINVAL, "MFWF_TUNE_FORCE: bad entry '" + tok + "'"), false;
        k[q] = (int)v;
    }
    set_knobs(p, k);
    return true;
}

static int time_launches(Plan &p, int reps, const std::function<int()> &launch, float &ms) {
    hipEvent_t e0, e1;
    MFWF_HIP(hipEventCreate(&e0));
    MFWF_HIP(hipEventCreate(&e1));
    int st = launch();  // warm-up
    if (st == MFWF_OK) st = (hipEventRecord(e0, p.stream) == hipSuccess) ? MFWF_OK : MFWF_EDEVICE;
    for (int r = 0; r < reps && st == MFWF_OK; r++) st = launch();
    if (st == MFWF_OK) st = (hipEventRecord(e1, p.stream) == hipSuccess) ? MFWF_OK : MFWF_EDEVICE;
    if (st == MFWF_OK) st = (hipEventSynchronize(e1) == hipSuccess) ? MFWF_OK : MFWF_EDEVICE;
    if (st == MFWF_OK) st = (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ? MFWF_OK : MFWF_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == MFWF_EDEVICE && g_err.empty()) set_error("event timing failed");
    return st;
}

// the fastest value of one knob for the launch it shapes (the others held)
static int tune_knob(Plan &p, int knob, const std::vector<int> &values,
                     const std::function<int()> &launch) {
    int k[kNumKnobs];
    get_knobs(p, k);
    float best = INFINITY;
    int bestv = k[knob];
    for (int v : values) {
        k[knob] = v;
        set_knobs(p, k);
        float ms = 0.f;
        MFWF_TRY(time_launches(p, 3, launch, ms));
        if (ms < best) {
            best = ms;
            bestv = v;
        }
    }
    k[knob] = bestv;
    set_knobs(p, k);
    return MFWF_OK;
}

static int autotune(Plan &p, const std::string &devname) {
    const std::string key = tune_key(p, devname);
    int k[kNumKnobs];
    get_knobs(p, k);
    if (tune_lookup(key, k)) {
        set_knobs(p, k);
        return MFWF_OK;
    }
    const int B = p.max_batch;
    if (p.dtype == MFWF_F64 && p.spin == 0) {
        // timing inputs: a fixed non-zero pattern (all variants do the same arithmetic on it)
        MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_sp), 2 * p.nalm, 0.25, p.stream));
        MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_phase), 2L * p.nm * p.nring, 0.5, p.stream));
        std::vector<int> sv(leg_synth_variants()), av(leg_analysis_variants());
        for (int v = 0; v < (int)sv.size(); v++) sv[v] = v;
        for (int v = 0; v < (int)av.size(); v++) av[v] = v;
        MFWF_TRY(tune_knob(p, kKnobSynth, sv, [&] { return launch_leg_synth(p, p.d_sp, p.d_phase, 1); }));
        MFWF_TRY(tune_knob(p, kKnobAna, av, [&] { return launch_leg_analysis(p, p.d_phase, p.d_apart, 1); }));
        MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_sp), 2 * p.nalm, 0.0, p.stream));
        MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_phase), 2L * p.nm * p.nring, 0.0, p.stream));
    }
    if (p.dtype == MFWF_F32) {
        // on zeroed work arrays: the batched kernels' work does not depend on the values
        if (p.spin == 0) {
            for (int c = 1; c >= 0; c--) {
                std::vector<int> gv;
                for (int g = 1; g <= fft_cols_group_max(p, c, B); g *= 2) gv.push_back(g);
                if (gv.size() > 1)
                    MFWF_TRY(tune_knob(p, c == 0 ? kKnobG0 : kKnobG1, gv, [&] {
                        return launch_fft_inv_fwd_cols(p, p.d_rho, 1.0, nullptr, B);
                    }));
            }
        }
        if (p.spin == 0 && p.d_lam && p.d_lck) {  // lambda read from the table or generated
            const std::vector<int> gv = {0, 1};
            MFWF_TRY(tune_knob(p, kKnobLamGen, gv, [&] {
                MFWF_TRY(launch_gemm_analysis(p, B, p.d_a32, nullptr, 1.0, 1.0));
                return launch_gemm_synthesis(p, B);
            }));
        }
        // the widest GEMM launches: 2 columns a map (temperature), 4 (the spin-2 F+- tables)
        const int w = p.spin == 2 ? 4 : 2;
        if (w * B > 64) {  // more than 64 active columns: every column tile applies
            const std::vector<int> cv = {1, 2}, cva = {1, 2, 3};
            MFWF_TRY(tune_knob(p, kKnobCtA, cva, [&] {
                return p.spin == 2 ? launch_gemm_analysis_raw(p, B, 4, p.d_fp, p.d_ph32p, p.d_ap32, 0)
                                   : launch_gemm_analysis(p, B, p.d_a32, nullptr, 1.0, 1.0);
            }));
            MFWF_TRY(tune_knob(p, kKnobCtS, cv, [&] {
                return p.spin == 2 ? launch_gemm_synthesis_on(p, B, 4, p.d_fp, p.d_seb32, p.d_ph32p, 0, 0)
                                   : launch_gemm_synthesis(p, B);
            }));
        }
    }
    get_knobs(p, k);
    tune_store(key, k);
    return MFWF_OK;
}

static void default_variants(Plan &p) {
    // pairs per lane 4 / 2 / 1 by problem size, prefetched 8-wide blocks
    const int P = p.npair >= 1024 ? 4 : (p.npair >= 512 ? 2 : 1);
    for (int v = 0; v < leg_synth_variants(); v++)
        if (leg_synth_pairs_per_lane(v) == P && v >= 3 && v < 6) p.synth_variant = v;
    for (int v = 0; v < leg_analysis_variants(); v++)
        if (leg_analysis_pairs_per_lane(v) == P && v >= 3) p.ana_variant = v;
}

// Batched FP32 form: lambda table (filled on the device from the FP64 recurrence), skip
// tables, work items, column-major work arrays.
// Distributes tiles over the 8 XCD lists: all tiles of one m go to one list (they share
// an operand block in that XCD's L2), m-groups largest first onto the least-loaded list.
// Returns the list length; tab = [8][length] item indices, -1 where a list is shorter.
static int balance_xcd(const std::vector<int2> &items, const std::vector<double> &work, int nm,
                       std::vector<int> &tab) {
    std::vector<double> wm(nm, 0.0);
    std::vector<std::vector<int>> of_m(nm);
    for (size_t i = 0; i < items.size(); i++) {
        wm[items[i].x] += work[i];
        of_m[items[i].x].push_back((int)i);
    }
    std::vector<int> order(nm);
    for (int m = 0; m < nm; m++) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return wm[a] > wm[b]; });
    std::vector<std::vector<int>> lists(8);
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int m : order) {
        if (of_m[m].empty()) continue;
        int x = 0;
        for (int k = 1; k < 8; k++)
            if (load[k] < load[x]) x = k;
        lists[x].insert(lists[x].end(), of_m[m].begin(), of_m[m].end());
        load[x] += wm[m];
    }
    size_t per = 0;
    for (auto &l : lists) per = std::max(per, l.size());
    tab.assign(8 * per, -1);
    for (int x = 0; x < 8; x++)
        for (size_t k = 0; k < lists[x].size(); k++) tab[x * per + k] = lists[x][k];
    return (int)per;
}

static int setup_batched(Plan &p, const std::vector<int> &lstart, const std::vector<long> &mofs) {
    p.Rp = ((p.npair + 63) / 64) * 64;
    p.Bp = ((p.max_batch + 15) / 16) * 16;
    p.C2 = 2 * p.Bp;
    std::vector<long> loff(p.nm);
    std::vector<int> Lp(p.nm);
    long tot = 0;
    for (int m = 0; m < p.nm; m++) {
        Lp[m] = ((p.lmax - m + 1 + 127) / 128) * 128;
        loff[m] = tot;
        tot += (long)p.Rp * Lp[m];
    }
    const int n32 = p.Rp / 32;
    std::vector<int> mn32((size_t)p.nm * n32, p.lmax + 1);
    for (int m = 0; m < p.nm; m++)
        for (int q = 0; q < p.npair; q++) {
            int &a = mn32[(size_t)m * n32 + q / 32];
            a = std::min(a, lstart[(size_t)m * p.npair + q]);
        }
    // analysis tiles (m, 128 values of l) and synthesis tiles (m, 64 ring pairs), with their
    // work in active K chunks (chunks whose pairs all start above the tile are skipped)
    std::vector<int2> ana, syn;
    std::vector<double> wana, wsyn;
    for (int m = 0; m < p.nm; m++) {
        const int Lm = p.lmax - m + 1;
        for (int t = 0; 128 * t < Lm; t++) {
            int act = 0;
            for (int pc = 0; pc < n32; pc++) act += mn32[(size_t)m * n32 + pc] <= m + 128 * t + 127;
            ana.push_back(make_int2(m, t));
            wana.push_back(1.0 + act);
        }
        for (int pt = 0; pt < p.Rp / 64; pt++) {
            const int ls = std::min(mn32[(size_t)m * n32 + 2 * pt], mn32[(size_t)m * n32 + 2 * pt + 1]);
            const int first = std::max(0, ls - m) / 64, nrc = (Lm + 63) / 64;
            syn.push_back(make_int2(m, pt));
            wsyn.push_back(1.0 + std::max(0, nrc - first));
        }
    }
    std::vector<int> ana_tab, syn_tab;
    p.ana_per_xcd = balance_xcd(ana, wana, p.nm, ana_tab);
    p.syn_per_xcd = balance_xcd(syn, wsyn, p.nm, syn_tab);
    std::vector<int> lofi(p.nalm);
    for (int m = 0; m < p.nm; m++)
        for (int l = m; l <= p.lmax; l++) lofi[mofs[m] + l - m] = l;
    // temperature: segment states for generating lambda inside the GEMMs (a quarter of the
    // table's bytes); the table itself only where it fits comfortably (nside <= 1024), so
    // that the autotuner can choose between reading it and generating
    std::vector<long> segoff(p.nm);
    long nseg = 0;
    for (int m = 0; m < p.nm; m++) {
        segoff[m] = nseg;
        nseg += Lp[m] / 16;
    }
    const bool table = p.spin == 2 || p.nside <= 1024;
    p.lam_gen = !table;
    if (p.spin == 0) {
        MFWF_TRY(dalloc(&p.d_lck, (size_t)nseg * p.Rp, "lambda segment states"));
        MFWF_TRY(dalloc(&p.d_segoff, segoff.size(), "lambda segment offsets"));
        MFWF_TRY(upload(p.d_segoff, segoff, p.stream));
    }
    if (table) MFWF_TRY(dalloc(&p.d_lam, tot, "lambda table"));
    MFWF_TRY(dalloc(&p.d_loff, loff.size(), "lambda offsets"));
    MFWF_TRY(dalloc(&p.d_Lp, Lp.size(), "lambda row lengths"));
    MFWF_TRY(dalloc(&p.d_minls32, mn32.size(), "start table 32"));
    MFWF_TRY(dalloc(&p.d_ana_items, ana.size(), "analysis items"));
    MFWF_TRY(dalloc(&p.d_syn_items, syn.size(), "synthesis items"));
    MFWF_TRY(dalloc(&p.d_ana_tab, ana_tab.size(), "analysis XCD lists"));
    MFWF_TRY(dalloc(&p.d_syn_tab, syn_tab.size(), "synthesis XCD lists"));
    MFWF_TRY(dalloc(&p.d_lofi, lofi.size(), "l of index"));
    p.nm32 = (p.nm + 15) / 16 * 16;
    MFWF_TRY(dalloc(&p.d_phf, (size_t)p.ncomp * p.max_batch * p.nring * p.nm32, "ring Fourier rows FP32"));
    MFWF_TRY(dalloc(&p.d_ph32, (size_t)p.nring * p.nm * p.C2, "ring Fourier FP32"));
    MFWF_TRY(dalloc(&p.d_a32, (size_t)p.nalm * p.C2, "analysis FP32"));
    MFWF_TRY(dalloc(&p.d_s32, (size_t)p.nalm * p.C2, "synthesis input FP32"));
    MFWF_TRY(upload(p.d_loff, loff, p.stream));
    MFWF_TRY(upload(p.d_Lp, Lp, p.stream));
    MFWF_TRY(upload(p.d_minls32, mn32, p.stream));
    MFWF_TRY(upload(p.d_ana_items, ana, p.stream));
    MFWF_TRY(upload(p.d_syn_items, syn, p.stream));
    MFWF_TRY(upload(p.d_ana_tab, ana_tab, p.stream));
    MFWF_TRY(upload(p.d_syn_tab, syn_tab, p.stream));
    MFWF_TRY(upload(p.d_lofi, lofi, p.stream));
    MFWF_HIP(hipMemsetAsync(p.d_ph32, 0, sizeof(float) * (size_t)p.nring * p.nm * p.C2, p.stream));
    MFWF_HIP(hipMemsetAsync(p.d_a32, 0, sizeof(float) * (size_t)p.nalm * p.C2, p.stream));
    MFWF_HIP(hipMemsetAsync(p.d_s32, 0, sizeof(float) * (size_t)p.nalm * p.C2, p.stream));
    if (p.spin == 2) {
        // F+ and F- tables and the four-column arrays of Q, U (E, B)
        const size_t ph = (size_t)p.nring * p.nm * 2 * p.C2, al = (size_t)p.nalm * 2 * p.C2;
        MFWF_TRY(dalloc(&p.d_fp, tot, "F+ table"));
        MFWF_TRY(dalloc(&p.d_fm, tot, "F- table"));
        MFWF_TRY(dalloc(&p.d_ph32p, ph, "Q, U ring Fourier FP32"));
        MFWF_TRY(dalloc(&p.d_ap32, al, "F+ analysis FP32"));
        MFWF_TRY(dalloc(&p.d_ar32, al, "F- analysis FP32"));
        MFWF_TRY(dalloc(&p.d_seb32, al, "E, B synthesis input FP32"));
        MFWF_HIP(hipMemsetAsync(p.d_ph32p, 0, sizeof(float) * ph, p.stream));
        float *za[] = {p.d_ap32, p.d_ar32, p.d_seb32};
        for (float *q : za) MFWF_HIP(hipMemsetAsync(q, 0, sizeof(float) * al, p.stream));
        MFWF_TRY(launch_pol_tables(p));
    } else {
        if (p.d_lam) MFWF_TRY(launch_lam_table(p));
        MFWF_TRY(launch_lam_ckpt(p));
    }
    return MFWF_OK;
}

static int set_groups(Plan &p) {
    const int P = leg_analysis_pairs_per_lane(p.ana_variant);
    p.ngroup = (p.npair + 64 * P - 1) / (64 * P);
    return MFWF_OK;
}

// Spin-2 coefficients per (l, m) of the rescaled recurrence (lambda = c mu), such that
//   s^2 F+ = (pc0 + pc1 z^2) mu_l + pc2 z mu_{l-1},  s^2 F- = pc3 mu_{l-1} + pc4 z mu_l,
// from s^2 F+ = N [(2m^2 - l(l+1) + l(l-1) z^2) lambda_l + 2 c_lm z lambda_{l-1}] and
// s^2 F- = 2 m N [c_lm lambda_{l-1} - (l-1) z lambda_l], N = ((l-1) l (l+1) (l+2))^-1/2,
// c_lm = ((2l+1)(l^2 - m^2)/(2l-1))^1/2 (both zero below l = 2).
static void build_spin2_table(int lmax, const std::vector<double> &ctab,
                              const std::vector<long> &mofs, std::vector<double> &pc) {
    const long nalm = (long)(lmax + 1) * (lmax + 2) / 2;
    pc.assign(5 * nalm, 0.0);
    for (int m = 0; m <= lmax; m++)
        for (int l = std::max(m, 2); l <= lmax; l++) {
            const long i = mofs[m] + l - m;
            const double L = l, M = m;
            const double N = 1.0 / std::sqrt((L - 1.0) * L * (L + 1.0) * (L + 2.0));
            const double clm = (l > m) ? std::sqrt((2.0 * L + 1.0) * (L * L - M * M) / (2.0 * L - 1.0)) : 0.0;
            const double c0 = ctab[i], c1 = (l > m) ? ctab[i - 1] : 0.0;
            pc[5 * i + 0] = N * (2.0 * M * M - L * (L + 1.0)) * c0;
            pc[5 * i + 1] = N * L * (L - 1.0) * c0;
            pc[5 * i + 2] = 2.0 * N * clm * c1;
            pc[5 * i + 3] = 2.0 * M * N * clm * c1;
            pc[5 * i + 4] = -2.0 * M * N * (L - 1.0) * c0;
        }
}

static int create(int nside, int lmax, int spin, int dtype, int max_batch, void *stream,
                  Plan &p) {
    if (nside < 1 || nside > 2048 || !is_pow2(nside))
        return fail(MFWF_EINVAL, "nside must be a power of two in [1, 2048]");
    if (dtype == MFWF_F32 && spin == 2 && nside > 1024)
        return fail(MFWF_EINVAL, "the batched FP32 form with spin 2 supports nside <= 1024 (its "
                                 "three function tables outgrow the device above)");
    if (lmax < 1 || lmax > 4 * nside) return fail(MFWF_EINVAL, "lmax must be in [1, 4 nside]");
    if (spin != 0 && spin != 2) return fail(MFWF_EINVAL, "spin must be 0 (T) or 2 (T, Q, U)");
    if (dtype != MFWF_F64 && dtype != MFWF_F32) return fail(MFWF_EINVAL, "dtype must be MFWF_F64 or MFWF_F32");
    if (max_batch < 1 || max_batch > 4096) return fail(MFWF_EINVAL, "max_batch out of range");
    if (dtype == MFWF_F32 && max_batch > 512) return fail(MFWF_EINVAL, "MFWF_F32 plans take max_batch <= 512");
    std::string devname;
    MFWF_TRY(device_name(devname));
    MFWF_HIP(hipGetDevice(&p.device));

    p.nside = nside;
    p.lmax = lmax;
    p.spin = spin;
    p.ncomp = (spin == 2) ? 3 : 1;
    p.dtype = dtype;
    p.max_batch = max_batch;
    p.stream = (hipStream_t)stream;
    p.npix = 12L * nside * nside;
    p.nring = 4 * nside - 1;
    p.npair = 2 * nside;
    p.nm = lmax + 1;
    p.nalm = (long)(lmax + 1) * (lmax + 2) / 2;
    p.omega = 4.0 * M_PI / (double)p.npix;
    p.ngroup_max = (p.npair + 63) / 64;  // pairs-per-lane 1 has the most groups

    // geometry of the north ring of every pair
    std::vector<RingGeom> geo(p.npair);
    std::vector<double> zp(p.npair);
    for (int q = 0; q < p.npair; q++) {
        geo[q] = ring_geom(nside, q + 1);
        zp[q] = geo[q].z;
    }
    std::vector<double2> ab;
    std::vector<double> Atab, ctab;
    std::vector<long> mofs;
    build_recurrence(lmax, ab, Atab, ctab, mofs);
    std::vector<int> lstart;
    std::vector<double2> seed;
    build_seeds(lmax, p.npair, geo, ab, ctab, mofs, lstart, seed);
    p.work_tuples = 0.0;
    for (int ls : lstart) p.work_tuples += (ls <= lmax) ? (double)(lmax - ls + 1) : 0.0;

    // ring FFT tables.  Chirp-z lengths above split_len take the split transform: the in-LDS
    // limit, or a smaller power of two from MFWF_FFT_SPLIT_LEN (tests of the split path at
    // sizes the oracle transforms whole)
    int split_len = fft_max_length();
    if (const char *e = std::getenv("MFWF_FFT_SPLIT_LEN")) {
        const long v = std::strtol(e, nullptr, 10);
        if (v >= 16 && v < split_len && is_pow2((int)v)) split_len = (int)v;
    }
    std::vector<PairFFT> pf(p.npair);
    std::vector<double2> chirp, bhat;
    int fftmax = 1;
    for (int q = 0; q < p.npair; q++) {
        const RingGeom &g = geo[q];
        PairFFT &f = pf[q];
        f.nphi = g.nphi;
        f.half_shift = g.half_shift;
        f.startN = g.start;
        const int iS = 4 * nside - (q + 1);
        f.startS = (iS == q + 1) ? g.start : ring_geom(nside, iS).start;
        f.bluestein = is_pow2(g.nphi) ? 0 : 1;
        f.fftlen = f.bluestein ? next_pow2(2L * g.nphi - 1) : g.nphi;
        // a chirp-z transform longer than the in-LDS limit: split n = 4 i into four
        // transforms of length i (polar rings always have n = 4 i)
        if (f.bluestein && f.fftlen > split_len && g.nphi % 4 == 0) {
            f.bluestein = 2;
            f.fftlen = next_pow2(2L * (g.nphi / 4) - 1);
        }
        fftmax = std::max(fftmax, f.fftlen);
        f.chirp_off = f.bhat_off = 0;
        if (f.bluestein) {
            const int n = f.bluestein == 2 ? g.nphi / 4 : g.nphi, M = f.fftlen;
            f.chirp_off = (long)chirp.size();
            for (long k = 0; k < n; k++) {  // c_k = exp(-i pi k^2 / n)
                const long r = (k * k) % (2L * n);
                const double a = M_PI * (double)r / n;
                chirp.push_back(make_double2(std::cos(a), -std::sin(a)));
            }
            std::vector<double2> b(M, make_double2(0.0, 0.0));  // conj(c), wrapped
            for (long k = 0; k < n; k++) {
                const double2 cc = chirp[f.chirp_off + k];
                b[k] = make_double2(cc.x, -cc.y);
                if (k > 0) b[M - k] = make_double2(cc.x, -cc.y);
            }
            host_fft(b);
            f.bhat_off = (long)bhat.size();
            for (int k = 0; k < M; k++) bhat.push_back(make_double2(b[k].x / M, b[k].y / M));
        }
    }
    p.fftmax = fftmax;
    std::vector<double2> tw(fftmax);
    for (int k = 0; k < fftmax; k++) {
        const double a = -2.0 * M_PI * (double)k / fftmax;
        tw[k] = make_double2(std::cos(a), std::sin(a));
    }
    // two-level twiddle table: W^t = hi[t / 64] lo[t % 64]
    p.fft_ntwhi = std::max(1, fftmax / 64);
    std::vector<double2> twlo(64), twhi(p.fft_ntwhi);
    for (int t = 0; t < 64; t++) {
        const double a = -2.0 * M_PI * (double)t / fftmax;
        twlo[t] = make_double2(std::cos(a), std::sin(a));
    }
    for (int h = 0; h < p.fft_ntwhi; h++) {
        const double a = -2.0 * M_PI * (double)(64L * h) / fftmax;
        twhi[h] = make_double2(std::cos(a), std::sin(a));
    }
    // FFT classes: pairs whose transform fits half of the largest length, the rest, and the
    // split rings (whose combined spectrum of n <= fftmax points passes through LDS)
    std::vector<int> plist;
    p.fft_class_len[0] = 1;
    int nsplit_max = 0;
    for (int c = 0; c < 3; c++) {
        p.fft_class_off[c] = (int)plist.size();
        for (int q = 0; q < p.npair; q++) {
            const int cls = pf[q].bluestein == 2 ? 2 : (2 * pf[q].fftlen <= fftmax ? 0 : 1);
            if (cls != c) continue;
            plist.push_back(q);
            if (c == 0) p.fft_class_len[0] = std::max(p.fft_class_len[0], pf[q].fftlen);
            if (c == 2) {
                nsplit_max = std::max(nsplit_max, pf[q].nphi);
                p.fftsplit_sublen = std::max(p.fftsplit_sublen, pf[q].fftlen);
            }
        }
        p.fft_class_count[c] = (int)plist.size() - p.fft_class_off[c];
    }
    p.fft_class_len[1] = fftmax;
    p.fft_class_len[2] = fftmax;
    if (nsplit_max > fftmax)
        return fail(MFWF_EINVAL, "split ring of " + std::to_string(nsplit_max) +
                                     " pixels above the largest transform length");
    if (fftmax > fft_max_length())
        return fail(MFWF_EINVAL, "ring FFT length " + std::to_string(fftmax) + " above the supported " +
                                     std::to_string(fft_max_length()));
    size_t lds = std::max({fft_class_lds(p, 0), fft_class_lds(p, 1), fft_class_lds(p, 2)});
    if (dtype == MFWF_F32)  // the columns ring step of the batched form, G maps per workgroup
        for (int c = 0; c < 2; c++)
            lds = std::max(lds, fft_cols_lds(p, c, fft_cols_group_max(p, c, max_batch)));
    {
        int dev = 0, maxlds = 0;
        MFWF_HIP(hipGetDevice(&dev));
        MFWF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        if (lds > (size_t)maxlds)
            return fail(MFWF_EINVAL, "ring FFT of length " + std::to_string(fftmax) +
                                         " does not fit the device LDS");
        if (lds > 65536) {
            MFWF_TRY(fft_set_lds_limit(lds));
        }
    }

    const long B = max_batch;
    const bool f32 = (dtype == MFWF_F32);
    const long B64 = f32 ? 1 : B;  // the FP32 form has its own column-major work arrays
    const long nc = p.ncomp;
    const long ncl = (spin == 2) ? 4 : 1, nmw = (spin == 2) ? 6 : 1;
    const long apart = (spin == 2) ? (long)pol_ngroup(p) * B64 * 3 * p.nalm : (long)p.ngroup_max * B64 * p.nalm;
    MFWF_TRY(dalloc(&p.d_z, p.npair, "z"));
    MFWF_TRY(dalloc(&p.d_A, Atab.size(), "recurrence A"));
    MFWF_TRY(dalloc(&p.d_c, ctab.size(), "recurrence scale"));
    MFWF_TRY(dalloc(&p.d_mofs, mofs.size(), "m offsets"));
    MFWF_TRY(dalloc(&p.d_lstart, lstart.size(), "l start"));
    MFWF_TRY(dalloc(&p.d_seed, seed.size(), "seeds"));
    MFWF_TRY(dalloc(&p.d_pfft, pf.size(), "fft plan"));
    MFWF_TRY(dalloc(&p.d_plist, plist.size(), "fft pair list"));
    MFWF_TRY(dalloc(&p.d_tw, tw.size(), "twiddles"));
    MFWF_TRY(dalloc(&p.d_twlo, twlo.size(), "twiddles lo"));
    MFWF_TRY(dalloc(&p.d_twhi, twhi.size(), "twiddles hi"));
    MFWF_TRY(dalloc(&p.d_chirp, std::max<size_t>(1, chirp.size()), "chirp"));
    MFWF_TRY(dalloc(&p.d_bhat, std::max<size_t>(1, bhat.size()), "chirp kernel"));
    if (f32 && p.fft_class_count[0] > 0 && p.fft_class_count[1] > 0) {
        // the two in-LDS ring classes of the chained ring step run side by side (default
        // priority, non-blocking: it orders only against the fork and join events)
        MFWF_HIP(hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking));
        MFWF_HIP(hipEventCreateWithFlags(&p.side_fork, hipEventDisableTiming));
        MFWF_HIP(hipEventCreateWithFlags(&p.side_join, hipEventDisableTiming));
    }
    if (p.fft_class_count[2] > 0) {  // split rings: sub-spectra parked between the passes
        p.fftsplit_rows = (int)(nc * B);
        p.fftsplit_stride = 2L * nsplit_max;
        MFWF_TRY(dalloc(&p.d_fftsplit, (long)p.fftsplit_rows * p.fft_class_count[2] * p.fftsplit_stride,
                        "split ring spectra"));
    }
    MFWF_TRY(dalloc(&p.d_cl, ncl * (lmax + 1), "cl"));
    MFWF_TRY(dalloc(&p.d_M, nmw * p.npix, "M"));
    MFWF_TRY(dalloc(&p.d_rho, B * nc * p.npix, "rho"));
    MFWF_TRY(dalloc(&p.d_t, B * nc * p.npix, "t"));
    MFWF_TRY(dalloc(&p.d_smap, B * nc * p.npix, "s map"));
    MFWF_TRY(dalloc(&p.d_phase, B64 * nc * p.nm * p.nring, "ring Fourier"));
    MFWF_TRY(dalloc(&p.d_apart, apart, "analysis partials"));
    MFWF_TRY(dalloc(&p.d_salm, B * nc * p.nalm, "s alm"));
    MFWF_TRY(dalloc(&p.d_salm_prev, B * nc * p.nalm, "previous s alm"));
    MFWF_TRY(dalloc(&p.d_sp, B * nc * p.nalm, "scaled synthesis input"));
    p.nred_blocks = 1024;
    MFWF_TRY(dalloc(&p.d_red, std::max<long>(3L * p.nred_blocks, std::max<long>(B * p.nred_blocks, 3L * B * p.nm)), "reductions"));
    MFWF_TRY(dalloc(&p.d_diag, 8 * B, "diagnostics"));
    if (spin == 2) {
        std::vector<double> pc;
        build_spin2_table(lmax, ctab, mofs, pc);
        MFWF_TRY(dalloc(&p.d_pc, pc.size(), "spin-2 coefficients"));
        MFWF_TRY(upload(p.d_pc, pc, p.stream));
    }

    MFWF_TRY(upload(p.d_z, zp, p.stream));
    MFWF_TRY(upload(p.d_A, Atab, p.stream));
    MFWF_TRY(upload(p.d_c, ctab, p.stream));
    MFWF_TRY(upload(p.d_mofs, mofs, p.stream));
    MFWF_TRY(upload(p.d_lstart, lstart, p.stream));
    MFWF_TRY(upload(p.d_seed, seed, p.stream));
    MFWF_TRY(upload(p.d_pfft, pf, p.stream));
    MFWF_TRY(upload(p.d_plist, plist, p.stream));
    MFWF_TRY(upload(p.d_tw, tw, p.stream));
    MFWF_TRY(upload(p.d_twlo, twlo, p.stream));
    MFWF_TRY(upload(p.d_twhi, twhi, p.stream));
    if (!chirp.empty()) MFWF_TRY(upload(p.d_chirp, chirp, p.stream));
    if (!bhat.empty()) MFWF_TRY(upload(p.d_bhat, bhat, p.stream));
    // defined contents everywhere (workspaces are read by autotuning and mfwf_time_kernels)
    MFWF_TRY(launch_fill(p.d_cl, ncl * (lmax + 1), 0.0, p.stream));
    MFWF_TRY(launch_fill(p.d_M, nmw * p.npix, 0.0, p.stream));
    MFWF_TRY(launch_fill(p.d_rho, B * nc * p.npix, 0.0, p.stream));
    MFWF_TRY(launch_fill(p.d_t, B * nc * p.npix, 0.0, p.stream));
    MFWF_TRY(launch_fill(p.d_smap, B * nc * p.npix, 0.0, p.stream));
    MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_phase), 2 * B64 * nc * p.nm * p.nring, 0.0, p.stream));
    MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_apart), 2L * apart, 0.0, p.stream));
    MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_salm), 2 * B * nc * p.nalm, 0.0, p.stream));
    MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_salm_prev), 2 * B * nc * p.nalm, 0.0, p.stream));
    MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_sp), 2 * B * nc * p.nalm, 0.0, p.stream));

    default_variants(p);
    if (f32) MFWF_TRY(setup_batched(p, lstart, mofs));
    p.tune_source = 0;
    if (const char *env = std::getenv("MFWF_TUNE_FORCE")) {
        if (!tune_force(env, p)) return MFWF_EINVAL;
        p.tune_source = 3;
    } else {
        const char *at = std::getenv("MFWF_AUTOTUNE");
        if (!(at && std::strcmp(at, "0") == 0) && p.npair >= 256) {
            MFWF_TRY(autotune(p, devname));
            p.tune_source = 1;
        }
    }
    MFWF_TRY(set_groups(p));
    MFWF_HIP(hipStreamSynchronize(p.stream));
    return MFWF_OK;
}

// ---- driver ------------------------------------------------------------------------------

// FP32 form: Legendre steps as MFMA GEMMs over the batch (Eqs. 3-4 unchanged)
static int iteration_b(Plan &p, const double *rho, int nb, double lam, bool keep_prev) {
    if (p.chain && p.chain_ready) {
        // the previous synthesis (zero at the start) back to pixels, the pixel update (Eq. 3)
        // and the forward ring transforms, in one kernel on the matrix-core columns
        MFWF_TRY(launch_fft_inv_fwd_cols(p, rho, lam, nullptr, nb));
    } else {
        // pixel update (Eq. 3) applied inside the forward ring transforms
        MFWF_TRY(launch_fft_fwd_f32(p, p.d_smap, rho, lam, p.d_phf, nb));
        MFWF_TRY(launch_rows_to_cols(p, nb));
    }
    if (keep_prev) MFWF_TRY(launch_cols_to_alm(p, p.d_s32, p.d_salm_prev, nb, 1.0));
    // analysis with the harmonic update (Eq. 4) applied in its epilogue
    MFWF_TRY(launch_gemm_analysis(p, nb, nullptr, p.d_s32, p.omega, lam * p.omega * p.tau,
                                  lam * p.omega));
    if (keep_prev) MFWF_TRY(launch_cols_to_alm(p, p.d_s32, p.d_salm, nb, 1.0));
    MFWF_TRY(launch_gemm_synthesis(p, nb));
    p.chain_ready = true;
    if (!p.chain || keep_prev) {  // the map s of this iteration
        MFWF_TRY(launch_cols_to_rows(p, nb));
        MFWF_TRY(launch_fft_inv_f32(p, p.d_phf, p.d_smap, nb));
    }
    return MFWF_OK;
}

// T, Q, U: 3x3 pixel update, transforms of 3 nb maps, spin-2 Legendre steps, 3x3 filter
static int iteration_pol(Plan &p, const double *rho, int nb, double lam, bool keep_prev) {
    MFWF_TRY(launch_pixel_update_pol(rho, p.d_M, p.d_smap, p.d_t, p.npix, nb, lam, p.tau, p.stream));
    MFWF_TRY(launch_fft_fwd(p, p.d_t, p.d_phase, 3 * nb));
    MFWF_TRY(launch_leg_analysis_pol(p, p.d_phase, p.d_apart, nb));
    MFWF_TRY(launch_harmonic_pol(p, p.d_apart, pol_ngroup(p), p.omega, lam * p.tau * p.omega,
                                 kHarmWiener, p.d_salm, p.d_sp, keep_prev ? p.d_salm_prev : nullptr, nb));
    MFWF_TRY(launch_leg_synth_pol(p, p.d_sp, p.d_phase, nb));
    MFWF_TRY(launch_fft_inv(p, p.d_phase, p.d_smap, 3 * nb));
    return MFWF_OK;
}

// T, Q, U in the batched FP32 form: FP64 3x3 pixel update, transforms of 3 nb maps with FP32
// rows, three analysis GEMMs and the 3x3 filter, three synthesis GEMMs
static int iteration_pol_b(Plan &p, const double *rho, int nb, double lam, bool keep_prev) {
    if (p.chain && p.chain_ready) {
        // the previous synthesis (zero at the start) back to pixels, the 3x3 pixel update
        // (Eq. 3) and the forward transforms, in one kernel on the matrix-core columns
        MFWF_TRY(launch_fft_inv_fwd_pol_cols(p, rho, lam, nb));
    } else {
        MFWF_TRY(launch_pixel_update_pol(rho, p.d_M, p.d_smap, p.d_t, p.npix, nb, lam, p.tau, p.stream));
        MFWF_TRY(launch_fft_fwd_f32(p, p.d_t, nullptr, 1.0, p.d_phf, 3 * nb));
        MFWF_TRY(launch_rows_to_cols_pol(p, nb));
    }
    if (keep_prev) MFWF_TRY(launch_cols_to_alm_pol(p, p.d_salm_prev, nb));
    MFWF_TRY(pol_analysis_b(p, nb, lam * p.tau * p.omega, kPolFilter));
    if (keep_prev) MFWF_TRY(launch_cols_to_alm_pol(p, p.d_salm, nb));
    const bool map = !p.chain || keep_prev;  // the map s of this iteration
    MFWF_TRY(pol_synthesis_b(p, nb, map));
    p.chain_ready = true;
    if (map) MFWF_TRY(launch_fft_inv_f32(p, p.d_phf, p.d_smap, 3 * nb));
    return MFWF_OK;
}

static int iteration(Plan &p, const double *rho, int nb, double lam, bool keep_prev) {
    if (p.dtype == MFWF_F32 && p.spin == 2) return iteration_pol_b(p, rho, nb, lam, keep_prev);
    if (p.dtype == MFWF_F32) return iteration_b(p, rho, nb, lam, keep_prev);
    if (p.spin == 2) return iteration_pol(p, rho, nb, lam, keep_prev);
    // the pixel update (Eq. 3) inside the forward ring transforms: t never goes to memory
    MFWF_TRY(launch_fft_fwd_pix(p, p.d_smap, rho, lam, p.d_phase, nb));
    MFWF_TRY(launch_leg_analysis(p, p.d_phase, p.d_apart, nb));
    MFWF_TRY(launch_harmonic(p, p.d_apart, p.ngroup, p.omega, lam * p.omega * p.tau, kHarmWiener,
                             p.d_salm, p.d_sp, keep_prev ? p.d_salm_prev : nullptr, nb,
                             lam * p.omega));
    MFWF_TRY(launch_leg_synth(p, p.d_sp, p.d_phase, nb));
    MFWF_TRY(launch_fft_inv(p, p.d_phase, p.d_smap, nb));
    return MFWF_OK;
}

// ---- plan internals used by the serving runtime ----------------------------------------
int plan_create(int nside, int lmax, int spin, int dtype, int max_batch, void *stream,
                bool per_slot, Plan &p) {
    int st = create(nside, lmax, spin, dtype, max_batch, stream, p);
    if (st != MFWF_OK || !per_slot) return st;
    if (spin != 0) return fail(MFWF_EINVAL, "serving slots are temperature only");
    // one M row and one tau per slot, set when a request is admitted
    (void)hipFree(p.d_M);
    p.d_M = nullptr;
    MFWF_TRY(dalloc(&p.d_M, (long)max_batch * p.npix, "per-slot M"));
    // tau covers the padded batch Bp: the batched analysis epilogue reads it for every
    // active column pair, including the zero columns past the last slot
    MFWF_TRY(dalloc(&p.d_tau, p.Bp, "per-slot tau"));
    MFWF_TRY(launch_fill(p.d_M, (long)max_batch * p.npix, 0.0, p.stream));
    MFWF_TRY(launch_fill(p.d_tau, p.Bp, 0.0, p.stream));
    p.mstride = p.npix;
    p.tau = 0.0;
    p.have_cov = true;
    MFWF_HIP(hipStreamSynchronize(p.stream));
    return MFWF_OK;
}

void plan_destroy(Plan &p) { free_plan(p); }

int plan_iteration(Plan &p, const double *rho, int nb, double lam) {
    return iteration(p, rho, nb, lam, false);
}

// After the last iteration: the FP32 form keeps s in its column layout; bring maps 0..nb-1
// back to the FP64 per-map alm array (the FP64 path writes it every iteration) and, when the
// iterations are chained (the map s is never formed on the way), transform the last
// synthesis back to the pixels of d_smap, as the last iteration of a standalone solve does.
int plan_finish_alm(Plan &p, int nb) {
    if (p.dtype != MFWF_F32) return MFWF_OK;
    MFWF_TRY(launch_cols_to_alm(p, p.d_s32, p.d_salm, nb, 1.0));
    if (p.chain && p.spin == 0) {
        MFWF_TRY(launch_cols_to_rows(p, nb));
        MFWF_TRY(launch_fft_inv_f32(p, p.d_phf, p.d_smap, nb));
    }
    return MFWF_OK;
}

int plan_set_cl(Plan &p, const double *cl) {
    std::vector<double> c(cl, cl + p.lmax + 1);
    for (double v : c)
        if (!(v >= 0.0) || std::isinf(v)) return fail(MFWF_EINVAL, "C_l must be finite and >= 0");
    return upload(p.d_cl, c, p.stream);
}

// One captured iteration of a stage, replayed as often as needed.
struct StageGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~StageGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
    int capture(Plan &p, const double *rho, int nb, double lam) {
        MFWF_HIP(hipStreamBeginCapture(p.stream, hipStreamCaptureModeThreadLocal));
        int st = iteration(p, rho, nb, lam, false);
        hipError_t e = hipStreamEndCapture(p.stream, &graph);
        if (st != MFWF_OK) return st;
        if (e != hipSuccess) return fail(MFWF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return fail(MFWF_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        return MFWF_OK;
    }
    int launch(Plan &p, int count) {
        for (int k = 0; k < count; k++) {
            hipError_t e = hipGraphLaunch(exec, p.stream);
            if (e != hipSuccess) return fail(MFWF_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        }
        return MFWF_OK;
    }
};

// MFWF_ENAN if the source rho of nb maps holds a non-finite value: a NaN or Inf in the
// data on an observed pixel (masked pixels have rho = 0 whatever the data), or in a
// caller's rho.  One pass over rho and a wait for the stream.
static int check_source_finite(const Plan &p, const double *rho, int nb) {
    const long n = (long)p.ncomp * p.npix * nb;
    MFWF_TRY(launch_count_nonfinite(rho, n, p.d_red, p.nred_blocks, p.d_diag, p.stream));
    double bad = 0.0;
    MFWF_HIP(hipMemcpyAsync(&bad, p.d_diag, sizeof(double), hipMemcpyDeviceToHost, p.stream));
    MFWF_HIP(hipStreamSynchronize(p.stream));
    if (bad > 0.0)
        return fail(MFWF_ENAN, "the source has " + std::to_string((long)bad) +
                                   " non-finite values on observed pixels");
    return MFWF_OK;
}

static int solve_chunk(Plan &p, const double *input, int nb, double *s_alm_out,
                       double *s_map_out, const mfwf_solve_opts &o,
                       const std::vector<double> &lam, const std::vector<int> &its,
                       mfwf_solve_info *info, int hist_maps, int hist_b0) {
    const double *rho = input;
    const long nc = p.ncomp;
    if (!o.source_is_rho) {
        if (p.spin == 2)
            MFWF_TRY(launch_rho_from_data_pol(input, p.d_M, p.d_rho, p.npix, nb, p.stream));
        else
            MFWF_TRY(launch_rho_from_data(input, p.d_M, p.d_rho, p.npix, nb, p.stream));
        rho = p.d_rho;
    }
    MFWF_TRY(check_source_finite(p, rho, nb));
    MFWF_TRY(launch_fill(p.d_smap, nc * p.npix * nb, 0.0, p.stream));
    MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_salm), 2 * nc * p.nalm * nb, 0.0, p.stream));
    // batched FP32 form (T; T, Q, U where the chained ring step fits): iterations chained
    // through the synthesis columns, which start at zero (s = 0); the last iteration is a
    // check, so d_smap holds the final map
    struct ChainOff {
        Plan &p;
        ~ChainOff() { p.chain = p.chain_ready = false; }
    } chain_off{p};
    if (o.order == 1) {
        // every iteration from the pixel map
    } else if (p.dtype == MFWF_F32 && p.spin == 0) {
        MFWF_HIP(hipMemsetAsync(p.d_ph32, 0, sizeof(float) * (size_t)p.nring * p.nm * p.C2, p.stream));
        p.chain = p.chain_ready = true;
    } else if (p.dtype == MFWF_F32 && fft_pol_chain_ok(p)) {  // T, Q, U: the synthesis of s = 0
        const size_t cols = (size_t)p.nring * p.nm * p.C2;
        MFWF_HIP(hipMemsetAsync(p.d_ph32, 0, sizeof(float) * cols, p.stream));
        MFWF_HIP(hipMemsetAsync(p.d_ph32p, 0, sizeof(float) * 2 * cols, p.stream));
        p.chain = p.chain_ready = true;
    }
    if (p.dtype == MFWF_F32) {  // previous harmonic iterate = 0 (outside any graph capture)
        MFWF_HIP(hipMemsetAsync(p.d_s32, 0, sizeof(float) * (size_t)p.nalm * p.C2, p.stream));
        if (p.spin == 2)
            MFWF_HIP(hipMemsetAsync(p.d_seb32, 0, sizeof(float) * (size_t)p.nalm * 2 * p.C2, p.stream));
    }
    long total = 0;
    for (int it : its) total += it;
    const long nchk = o.n_check > 0 ? o.n_check : 0;
    long done = 0;
    int rows = 0;
    double last_lam = 1.0;
    const bool graph = o.use_graph && p.stream != nullptr;
    std::vector<double> dg(8L * nb);
    auto diagnostics = [&](double lam_k) -> int {
        if (p.spin == 2) {
            MFWF_TRY(launch_chi2_pix_pol(rho, p.d_M, p.d_smap, p.npix, nb, lam_k, p.tau, p.d_red,
                                         p.nred_blocks, p.d_diag, p.stream));
            return launch_harm_diag_pol(p, p.d_salm, p.d_salm_prev, nb, p.d_red, p.d_diag);
        }
        MFWF_TRY(launch_chi2_pix(rho, p.d_M, p.d_smap, p.npix, nb, lam_k, p.tau, p.d_red,
                                 p.nred_blocks, p.d_diag, p.stream));
        return launch_harm_diag(p, p.d_salm, p.d_salm_prev, nb, p.d_red, p.d_diag);
    };
    // early end: the per-iteration change of chi^2 between two checks of one stage (one
    // lambda) below dchi2_tol sigma_chi2 for every map (sigma_chi2 = sqrt(2 n_dof), Sect. 2.2)
    const double stop_tol = o.dchi2_tol * std::sqrt(2.0 * (double)p.ndof);
    std::vector<double> chi_prev(nb, 0.0);
    long prev_at = -1;       // iteration count at the previous check of the current stage
    // checks of the current stage for info.dchi2: the previous check's chi^2 parts are kept
    // in diag[b][6..7] on the device (no host wait)
    long chk_last = -1, chk_prev = -1;
    bool stopped = false;
    for (size_t s = 0; s < lam.size() && !stopped; s++) {
        long remaining = its[s];
        if (remaining <= 0) continue;
        last_lam = lam[s];
        prev_at = -1;
        chk_last = chk_prev = -1;
        std::unique_ptr<StageGraph> sg;
        while (remaining > 0) {
            // run up to the next check point: a multiple of n_check, or the last iteration
            const long next = nchk ? std::min(total, (done / nchk + 1) * nchk) : total;
            const long run = std::min(remaining, next - done);
            const bool check = (done + run == next);
            const long plain = check ? run - 1 : run;
            if (graph && plain >= 2) {
                if (!sg) {
                    sg.reset(new StageGraph());
                    MFWF_TRY(sg->capture(p, rho, nb, lam[s]));
                }
                MFWF_TRY(sg->launch(p, (int)plain));
            } else {
                for (long k = 0; k < plain; k++) MFWF_TRY(iteration(p, rho, nb, lam[s], false));
            }
            if (check) {
                if (chk_last >= 0)  // diag[b][0..1] of the previous check -> diag[b][6..7]
                    MFWF_HIP(hipMemcpy2DAsync(p.d_diag + 6, 8 * sizeof(double), p.d_diag,
                                              8 * sizeof(double), 2 * sizeof(double), nb,
                                              hipMemcpyDeviceToDevice, p.stream));
                chk_prev = chk_last;
                chk_last = done + run;
                MFWF_TRY(iteration(p, rho, nb, lam[s], true));
                MFWF_TRY(diagnostics(lam[s]));
                if (stop_tol > 0.0) {
                    MFWF_HIP(hipMemcpyAsync(dg.data(), p.d_diag, sizeof(double) * dg.size(),
                                            hipMemcpyDeviceToHost, p.stream));
                    MFWF_HIP(hipStreamSynchronize(p.stream));
                    const long at = done + run;
                    double worst = 0.0;
                    for (int b = 0; b < nb; b++) {
                        const double chi = dg[8 * b + 0] + dg[8 * b + 1];
                        if (!std::isfinite(chi)) return fail(MFWF_ENAN, "chi^2 is not finite");
                        if (prev_at >= 0)
                            worst = std::max(worst, std::fabs(chi - chi_prev[b]) / (double)(at - prev_at));
                        chi_prev[b] = chi;
                    }
                    stopped = prev_at >= 0 && worst < stop_tol;
                    prev_at = at;
                }
                if (o.history && rows < o.history_rows) {
                    MFWF_HIP(hipMemcpyAsync(dg.data(), p.d_diag, sizeof(double) * dg.size(),
                                            hipMemcpyDeviceToHost, p.stream));
                    MFWF_HIP(hipStreamSynchronize(p.stream));
                    for (int b = 0; b < nb; b++) {
                        double *row = o.history + ((long)rows * hist_maps + hist_b0 + b) * 5;
                        row[0] = (double)(done + run);
                        row[1] = lam[s];
                        row[2] = dg[8 * b + 0] + dg[8 * b + 1];
                        row[3] = std::sqrt(dg[8 * b + 2]);
                        row[4] = std::sqrt(dg[8 * b + 3]);
                    }
                }
                rows++;
            }
            done += run;
            remaining -= run;
            if (stopped) break;
        }
    }
    if (total == 0) MFWF_TRY(launch_fill(p.d_diag, 8L * nb, 0.0, p.stream));
    if (s_alm_out)
        MFWF_HIP(hipMemcpyAsync(s_alm_out, p.d_salm, sizeof(double2) * nc * p.nalm * nb,
                                hipMemcpyDeviceToDevice, p.stream));
    if (s_map_out)
        MFWF_HIP(hipMemcpyAsync(s_map_out, p.d_smap, sizeof(double) * nc * p.npix * nb,
                                hipMemcpyDeviceToDevice, p.stream));
    if (info) {
        MFWF_HIP(hipMemcpyAsync(dg.data(), p.d_diag, sizeof(double) * dg.size(),
                                hipMemcpyDeviceToHost, p.stream));
        MFWF_HIP(hipStreamSynchronize(p.stream));
        for (int b = 0; b < nb; b++) {
            mfwf_solve_info &in = info[b];
            in.iters_done = (int)done;
            in.lambda = last_lam;
            in.chi2 = dg[8 * b + 0] + dg[8 * b + 1];
            in.chi2_harm = dg[8 * b + 1];
            in.dnorm = std::sqrt(dg[8 * b + 2]);
            in.snorm = std::sqrt(dg[8 * b + 3]);
            in.tau = p.tau;
            in.n_dof = p.ndof;
            in.n_checks = std::min(rows, o.history ? o.history_rows : rows);
            in.dchi2 = chk_prev >= 0 ? (dg[8 * b + 0] + dg[8 * b + 1] - dg[8 * b + 6] - dg[8 * b + 7]) /
                                           (double)(chk_last - chk_prev)
                                     : 0.0;
            in.rel_change = in.snorm > 0.0 ? in.dnorm / in.snorm : 0.0;
        }
    }
    return MFWF_OK;
}

}  // namespace mfwf

using namespace mfwf;

extern "C" {

const char *mfwf_last_error(void) { return g_err.c_str(); }

int mfwf_plan_create(int nside, int lmax, int spin, int dtype, int max_batch, void *hip_stream,
                     mfwf_plan *out) {
    if (!out) return fail(MFWF_EINVAL, "out is NULL");
    *out = nullptr;
    auto *h = new (std::nothrow) mfwf_plan_s();
    if (!h) return fail(MFWF_ENOMEM, "host allocation failed");
    int st = create(nside, lmax, spin, dtype, max_batch, hip_stream, h->p);
    if (st != MFWF_OK) {
        free_plan(h->p);
        delete h;
        return st;
    }
    *out = h;
    return MFWF_OK;
}

int mfwf_plan_destroy(mfwf_plan plan) {
    if (!plan) return MFWF_OK;
    (void)hipStreamSynchronize(plan->p.stream);
    for (auto &q : plan->sub) free_plan(q.second->p);
    free_plan(plan->p);
    delete plan;
    return MFWF_OK;
}

int mfwf_set_covariances(mfwf_plan plan, const double *cl, int ncl, const double *ninv,
                         const uint8_t *mask) {
    if (!plan || !cl || !ninv) return fail(MFWF_EINVAL, "NULL argument");
    Plan &p = plan->p;
    p.have_cov = false;
    if (p.spin == 2) {
        if (ncl != 4) return fail(MFWF_EINVAL, "ncl must be 4 (TT, EE, BB, TE) for spin 2");
        const int L1 = p.lmax + 1;
        std::vector<double> c(cl, cl + 4L * L1);
        for (int l = 0; l < L1; l++) {
            const double TT = c[l], EE = c[L1 + l], BB = c[2 * L1 + l], TE = c[3 * L1 + l];
            if (!(TT >= 0.0) || !(EE >= 0.0) || !(BB >= 0.0) || std::isinf(TT) || std::isinf(EE) ||
                std::isinf(BB) || !std::isfinite(TE) || TE * TE > TT * EE)
                return fail(MFWF_EINVAL, "each S_l must be finite and positive semi-definite");
        }
        MFWF_TRY(upload(p.d_cl, c, p.stream));
        plan->cl = c;
        plan->cov_gen++;
        MFWF_TRY(launch_pol_covariance(ninv, mask, p.d_M, p.npix, p.d_red, p.nred_blocks, p.d_diag,
                                       p.stream));
        double r[3];
        MFWF_HIP(hipMemcpyAsync(r, p.d_diag, sizeof(r), hipMemcpyDeviceToHost, p.stream));
        MFWF_HIP(hipStreamSynchronize(p.stream));
        if (r[2] > 0.0)
            return fail(MFWF_ENOTSPD, "a 3x3 noise block is not finite and positive semi-definite");
        if (!(r[0] > 0.0)) return fail(MFWF_ENOCOV, "no observed pixel: all blocks are 0, tau undefined");
        p.tau = 1.0 / r[0];  // 1 / max_p lambda_max(M_p)
        p.ndof = 3 * (long)r[1];
        p.have_cov = true;
        return MFWF_OK;
    }
    if (ncl != 1) return fail(MFWF_EINVAL, "ncl must be 1 for temperature");
    std::vector<double> c(cl, cl + p.lmax + 1);
    for (double v : c)
        if (!(v >= 0.0) || std::isinf(v)) return fail(MFWF_EINVAL, "C_l must be finite and >= 0");
    MFWF_TRY(upload(p.d_cl, c, p.stream));
    plan->cl = c;
    plan->cov_gen++;
    MFWF_TRY(launch_mask_product(ninv, mask, p.d_M, p.npix, p.stream));
    MFWF_TRY(launch_reduce_max_count(p.d_M, p.npix, p.d_red, p.nred_blocks, p.d_diag, p.stream));
    double r[3];
    MFWF_HIP(hipMemcpyAsync(r, p.d_diag, sizeof(r), hipMemcpyDeviceToHost, p.stream));
    MFWF_HIP(hipStreamSynchronize(p.stream));
    if (r[2] > 0.0) return fail(MFWF_ENAN, "inverse noise has negative or non-finite entries");
    if (!(r[0] > 0.0)) return fail(MFWF_ENOCOV, "no observed pixel: max N^-1 * mask is 0, tau undefined");
    p.tau = 1.0 / r[0];
    p.ndof = (long)r[1];
    p.have_cov = true;
    return MFWF_OK;
}

int mfwf_set_covariances_beam(mfwf_plan plan, const double *cl, int ncl, const double *bl,
                              const double *ninv, const uint8_t *mask) {
    if (!plan || !cl) return fail(MFWF_EINVAL, "NULL argument");
    if (!bl) return mfwf_set_covariances(plan, cl, ncl, ninv, mask);
    const Plan &p = plan->p;
    if (ncl != (p.spin == 2 ? 4 : 1)) return fail(MFWF_EINVAL, "ncl must be 1 (spin 0) or 4 (spin 2)");
    const long L1 = p.lmax + 1;
    std::vector<double> c(cl, cl + ncl * L1);
    for (long l = 0; l < L1; l++) {
        if (!std::isfinite(bl[l])) return fail(MFWF_EINVAL, "beam must be finite");
        for (int r = 0; r < ncl; r++) c[r * L1 + l] *= bl[l] * bl[l];  // S_l = b_l^2 C_l
    }
    return mfwf_set_covariances(plan, c.data(), ncl, ninv, mask);
}

int mfwf_remove_templates(mfwf_plan plan, const double *d_raw, double *d_out, int nmaps) {
    if (!plan || nmaps < 0) return fail(MFWF_EINVAL, "bad argument");
    Plan &p = plan->p;
    if (!p.have_cov) return fail(MFWF_ENOCOV, "covariances not set (the mask comes from them)");
    if (nmaps == 0) return MFWF_OK;
    if (!d_raw || !d_out) return fail(MFWF_EINVAL, "NULL array");
    const long ms = (long)p.ncomp * p.npix;
    for (int b0 = 0; b0 < nmaps; b0 += p.max_batch) {
        const int nb = std::min(p.max_batch, nmaps - b0);
        double *partial = p.d_red, *out14 = p.d_red + template_partial_doubles(nb);
        MFWF_TRY(launch_template_sums(p, d_raw + b0 * ms, nb, partial, out14));
        std::vector<double> h(14L * nb), coef(4L * nb);
        MFWF_HIP(hipMemcpyAsync(h.data(), out14, sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                                p.stream));
        MFWF_HIP(hipStreamSynchronize(p.stream));
        for (int b = 0; b < nb; b++) {
            // G = V^T V from its upper triangle, c = V^T d; G = L L^T (Cholesky), G k = c
            const double *u = &h[14L * b];
            double G[4][4], L[4][4] = {}, y[4], k[4];
            int q = 0;
            for (int a = 0; a < 4; a++)
                for (int e = a; e < 4; e++) G[a][e] = G[e][a] = u[q++];
            const double tr = G[0][0] + G[1][1] + G[2][2] + G[3][3];
            for (int i = 0; i < 4; i++) {
                for (int j = 0; j <= i; j++) {
                    double v = G[i][j];
                    for (int t = 0; t < j; t++) v -= L[i][t] * L[j][t];
                    if (i == j) {
                        if (!(v > 1e-12 * tr))
                            return fail(MFWF_EINVAL, "the monopole and dipole templates are "
                                                     "degenerate on the observed pixels");
                        L[i][i] = std::sqrt(v);
                    } else {
                        L[i][j] = v / L[j][j];
                    }
                }
            }
            for (int i = 0; i < 4; i++) {
                double v = u[10 + i];
                for (int t = 0; t < i; t++) v -= L[i][t] * y[t];
                y[i] = v / L[i][i];
            }
            for (int i = 3; i >= 0; i--) {
                double v = y[i];
                for (int t = i + 1; t < 4; t++) v -= L[t][i] * k[t];
                k[i] = v / L[i][i];
            }
            for (int i = 0; i < 4; i++) coef[4L * b + i] = k[i];
        }
        MFWF_HIP(hipMemcpyAsync(p.d_diag, coef.data(), sizeof(double) * coef.size(),
                                hipMemcpyHostToDevice, p.stream));
        MFWF_TRY(launch_template_subtract(p, d_raw + b0 * ms, d_out + b0 * ms, nb, p.d_diag));
        MFWF_HIP(hipStreamSynchronize(p.stream));
    }
    return MFWF_OK;
}

int mfwf_remove_templates_noalloc(mfwf_plan plan, const double *d_raw, double *d_out, int nmaps) {
    if (!plan || nmaps < 0) return fail(MFWF_EINVAL, "bad argument");
    const Plan &p = plan->p;
    if (!p.have_cov) return fail(MFWF_ENOCOV, "covariances not set (the mask comes from them)");
    if (nmaps == 0) return MFWF_OK;
    if (!d_raw || !d_out) return fail(MFWF_EINVAL, "NULL array");
    return remove_templates_noalloc(p, d_raw, d_out, nmaps);
}

int mfwf_sht_inv(mfwf_plan plan, const double *alm, double *map, int nmaps) {
    if (!plan || nmaps < 0) return fail(MFWF_EINVAL, "bad argument");
    if (nmaps == 0) return MFWF_OK;
    if (!alm || !map) return fail(MFWF_EINVAL, "NULL array");
    Plan &p = plan->p;
    for (int b0 = 0; b0 < nmaps; b0 += p.max_batch) {
        const int nb = std::min(p.max_batch, nmaps - b0);
        if (p.spin == 2 && p.dtype == MFWF_F32) {
            MFWF_TRY(launch_alm_to_cols_pol(p, reinterpret_cast<const double2 *>(alm) + 3L * b0 * p.nalm, nb));
            MFWF_TRY(pol_synthesis_b(p, nb));
            MFWF_TRY(launch_fft_inv_f32(p, p.d_phf, map + 3L * b0 * p.npix, 3 * nb));
            continue;
        }
        if (p.spin == 2) {
            MFWF_TRY(launch_harmonic_pol(p, reinterpret_cast<const double2 *>(alm) + 3L * b0 * p.nalm,
                                         1, 1.0, 0.0, kHarmCopy, nullptr, p.d_sp, nullptr, nb));
            MFWF_TRY(launch_leg_synth_pol(p, p.d_sp, p.d_phase, nb));
            MFWF_TRY(launch_fft_inv(p, p.d_phase, map + 3L * b0 * p.npix, 3 * nb));
            continue;
        }
        if (p.dtype == MFWF_F32) {
            MFWF_TRY(launch_alm_to_cols(p, reinterpret_cast<const double2 *>(alm) + (long)b0 * p.nalm,
                                        p.d_s32, nb, kHarmCopy));
            MFWF_TRY(launch_gemm_synthesis(p, nb));
            MFWF_TRY(launch_cols_to_rows(p, nb));
            MFWF_TRY(launch_fft_inv_f32(p, p.d_phf, map + (long)b0 * p.npix, nb));
            continue;
        }
        MFWF_TRY(launch_harmonic(p, reinterpret_cast<const double2 *>(alm) + (long)b0 * p.nalm, 1,
                                 1.0, 0.0, kHarmCopy, nullptr, p.d_sp, nullptr, nb));
        MFWF_TRY(launch_leg_synth(p, p.d_sp, p.d_phase, nb));
        MFWF_TRY(launch_fft_inv(p, p.d_phase, map + (long)b0 * p.npix, nb));
    }
    return MFWF_OK;
}

int mfwf_sht_fwd(mfwf_plan plan, const double *map, double *alm, int nmaps) {
    if (!plan || nmaps < 0) return fail(MFWF_EINVAL, "bad argument");
    if (nmaps == 0) return MFWF_OK;
    if (!alm || !map) return fail(MFWF_EINVAL, "NULL array");
    Plan &p = plan->p;
    for (int b0 = 0; b0 < nmaps; b0 += p.max_batch) {
        const int nb = std::min(p.max_batch, nmaps - b0);
        if (p.spin == 2 && p.dtype == MFWF_F32) {
            MFWF_TRY(launch_fft_fwd_f32(p, map + 3L * b0 * p.npix, nullptr, 1.0, p.d_phf, 3 * nb));
            MFWF_TRY(launch_rows_to_cols_pol(p, nb));
            MFWF_TRY(pol_analysis_b(p, nb, 0.0, kPolRaw));
            MFWF_TRY(launch_cols_to_alm_pol(p, reinterpret_cast<double2 *>(alm) + 3L * b0 * p.nalm, nb));
            continue;
        }
        if (p.spin == 2) {
            MFWF_TRY(launch_fft_fwd(p, map + 3L * b0 * p.npix, p.d_phase, 3 * nb));
            MFWF_TRY(launch_leg_analysis_pol(p, p.d_phase, p.d_apart, nb));
            MFWF_TRY(launch_harmonic_pol(p, p.d_apart, pol_ngroup(p), p.omega, 0.0, kHarmAnalysis,
                                         reinterpret_cast<double2 *>(alm) + 3L * b0 * p.nalm,
                                         nullptr, nullptr, nb));
            continue;
        }
        if (p.dtype == MFWF_F32) {
            MFWF_TRY(launch_fft_fwd_f32(p, map + (long)b0 * p.npix, nullptr, 1.0, p.d_phf, nb));
            MFWF_TRY(launch_rows_to_cols(p, nb));
            MFWF_TRY(launch_gemm_analysis(p, nb, p.d_a32, nullptr, 0.0, 0.0));
            MFWF_TRY(launch_cols_to_alm(p, p.d_a32, reinterpret_cast<double2 *>(alm) + (long)b0 * p.nalm,
                                        nb, p.omega));
            continue;
        }
        MFWF_TRY(launch_fft_fwd(p, map + (long)b0 * p.npix, p.d_phase, nb));
        MFWF_TRY(launch_leg_analysis(p, p.d_phase, p.d_apart, nb));
        MFWF_TRY(launch_harmonic(p, p.d_apart, p.ngroup, p.omega, 0.0, kHarmAnalysis,
                                 reinterpret_cast<double2 *>(alm) + (long)b0 * p.nalm, nullptr,
                                 nullptr, nb));
    }
    return MFWF_OK;
}

int mfwf_fluctuation_rhs(mfwf_plan plan, const double *g1, const double *h, int nrhs,
                         double *rho) {
    if (!plan || nrhs < 0) return fail(MFWF_EINVAL, "bad argument");
    Plan &p = plan->p;
    if (!p.have_cov) return fail(MFWF_ENOCOV, "covariances not set");
    if (nrhs == 0) return MFWF_OK;
    if (!g1 || !h || !rho) return fail(MFWF_EINVAL, "NULL array");
    for (int b0 = 0; b0 < nrhs; b0 += p.max_batch) {
        const int nb = std::min(p.max_batch, nrhs - b0);
        // x = C^{-1/2} h, then Y x, then rho = M^{1/2} g1 + Omega Y x
        if (p.spin == 2) {
            if (p.dtype == MFWF_F32) {
                // K h in FP64 (the FP32 tables carry c, so the T component is not c-scaled)
                MFWF_TRY(launch_harmonic_pol(p, reinterpret_cast<const double2 *>(h) + 3L * b0 * p.nalm,
                                             1, 1.0, 0.0, kHarmInvSqrtC, p.d_sp, nullptr, nullptr, nb));
                MFWF_TRY(launch_alm_to_cols_pol(p, p.d_sp, nb));
                MFWF_TRY(pol_synthesis_b(p, nb));
                MFWF_TRY(launch_fft_inv_f32(p, p.d_phf, p.d_t, 3 * nb));
            } else {
                MFWF_TRY(launch_harmonic_pol(p, reinterpret_cast<const double2 *>(h) + 3L * b0 * p.nalm,
                                             1, 1.0, 0.0, kHarmInvSqrtC, nullptr, p.d_sp, nullptr, nb));
                MFWF_TRY(launch_leg_synth_pol(p, p.d_sp, p.d_phase, nb));
                MFWF_TRY(launch_fft_inv(p, p.d_phase, p.d_t, 3 * nb));
            }
            MFWF_TRY(launch_fluct_combine_pol(g1 + 3L * b0 * p.npix, p.d_M, p.d_t,
                                              rho + 3L * b0 * p.npix, p.npix, nb, p.omega, p.stream));
            continue;
        }
        if (p.dtype == MFWF_F32) {
            MFWF_TRY(launch_alm_to_cols(p, reinterpret_cast<const double2 *>(h) + (long)b0 * p.nalm,
                                        p.d_s32, nb, kHarmInvSqrtC));
            MFWF_TRY(launch_gemm_synthesis(p, nb));
            MFWF_TRY(launch_cols_to_rows(p, nb));
            MFWF_TRY(launch_fft_inv_f32(p, p.d_phf, p.d_t, nb));
        } else {
            MFWF_TRY(launch_harmonic(p, reinterpret_cast<const double2 *>(h) + (long)b0 * p.nalm, 1,
                                     1.0, 0.0, kHarmInvSqrtC, nullptr, p.d_sp, nullptr, nb));
            MFWF_TRY(launch_leg_synth(p, p.d_sp, p.d_phase, nb));
            MFWF_TRY(launch_fft_inv(p, p.d_phase, p.d_t, nb));
        }
        MFWF_TRY(launch_fluct_combine(g1 + (long)b0 * p.npix, p.d_M, p.d_t,
                                      rho + (long)b0 * p.npix, p.npix, nb, p.omega, p.stream));
    }
    return MFWF_OK;
}

int mfwf_solve(mfwf_plan plan, const double *input, int nmaps, double *s_alm_out,
               double *s_map_out, const mfwf_solve_opts *opts, mfwf_solve_info *info) {
    if (!plan || nmaps < 0) return fail(MFWF_EINVAL, "bad argument");
    Plan &p = plan->p;
    if (!p.have_cov) return fail(MFWF_ENOCOV, "covariances not set");
    if (nmaps > 0 && !input) return fail(MFWF_EINVAL, "input is NULL");
    mfwf_solve_opts o{};
    std::vector<double> lam{1.0};
    std::vector<int> its{300};
    if (opts) {
        o = *opts;
        if (!(o.dchi2_tol >= 0.0)) return fail(MFWF_EINVAL, "dchi2_tol must be >= 0");
        if (o.dchi2_tol > 0.0 && o.n_check <= 0)
            return fail(MFWF_EINVAL, "dchi2_tol needs n_check > 0 (chi^2 is evaluated at the checks)");
        if (o.n_stages < 0) return fail(MFWF_EINVAL, "n_stages < 0");
        if (o.n_check < 0) return fail(MFWF_EINVAL, "n_check < 0");
        if (o.history && o.history_rows < 0) return fail(MFWF_EINVAL, "history_rows < 0");
        if (o.order != 0 && o.order != 1) return fail(MFWF_EINVAL, "order must be 0 or 1");
        if (o.n_stages > 0) {
            if (!o.lambda || !o.iters) return fail(MFWF_EINVAL, "schedule arrays are NULL");
            lam.assign(o.lambda, o.lambda + o.n_stages);
            its.assign(o.iters, o.iters + o.n_stages);
            for (int s = 0; s < o.n_stages; s++)
                if (!(lam[s] >= 1.0) || std::isinf(lam[s]) || its[s] < 0)
                    return fail(MFWF_EINVAL, "each lambda must be finite and >= 1, iters >= 0");
        }
    }
    for (int b0 = 0; b0 < nmaps; b0 += p.max_batch) {
        const int nb = std::min(p.max_batch, nmaps - b0);
        const long nc = p.ncomp;
        MFWF_TRY(solve_chunk(p, input + nc * b0 * p.npix, nb,
                             s_alm_out ? s_alm_out + 2L * nc * b0 * p.nalm : nullptr,
                             s_map_out ? s_map_out + nc * b0 * p.npix : nullptr, o, lam, its,
                             info ? info + b0 : nullptr, nmaps, b0));
    }
    MFWF_HIP(hipStreamSynchronize(p.stream));
    return MFWF_OK;
}

}  // extern "C"

namespace mfwf {

// The plan of band limit lk for a cooled solve: the plan itself at lk = lmax, else a
// cached plan of the same nside, spin, dtype and batch with the spectra truncated to lk and
// the same M and tau.
static int cooled_plan(mfwf_plan plan, int lk, Plan *&out) {
    Plan &p = plan->p;
    if (lk >= p.lmax) {
        out = &p;
        return MFWF_OK;
    }
    auto it = plan->sub.find(lk);
    if (it == plan->sub.end()) {
        std::unique_ptr<mfwf_plan_s::Sub> q(new mfwf_plan_s::Sub());
        const int st = create(p.nside, lk, p.spin, p.dtype, p.max_batch, p.stream, q->p);
        if (st != MFWF_OK) {
            free_plan(q->p);
            return st;
        }
        it = plan->sub.emplace(lk, std::move(q)).first;
    }
    mfwf_plan_s::Sub &q = *it->second;
    if (q.gen != plan->cov_gen) {
        const int ncl = p.spin == 2 ? 4 : 1;
        const long L = p.lmax + 1, Lk = lk + 1, nmw = p.spin == 2 ? 6 : 1;
        std::vector<double> c((size_t)ncl * Lk);
        for (int r = 0; r < ncl; r++)
            for (long l = 0; l < Lk; l++) c[r * Lk + l] = plan->cl[r * L + l];
        MFWF_TRY(upload(q.p.d_cl, c, q.p.stream));
        MFWF_HIP(hipMemcpyAsync(q.p.d_M, p.d_M, sizeof(double) * nmw * p.npix,
                                hipMemcpyDeviceToDevice, q.p.stream));
        MFWF_HIP(hipStreamSynchronize(q.p.stream));
        q.p.tau = p.tau;
        q.p.ndof = p.ndof;
        q.p.have_cov = true;
        q.gen = plan->cov_gen;
    }
    out = &q.p;
    return MFWF_OK;
}

// chi^2 and norms of nb maps after an iteration run with keep_prev (host dg[8 nb])
static int cooled_diag(Plan &q, const double *rho, int nb, double lam, std::vector<double> &dg) {
    if (q.spin == 2) {
        MFWF_TRY(launch_chi2_pix_pol(rho, q.d_M, q.d_smap, q.npix, nb, lam, q.tau, q.d_red,
                                     q.nred_blocks, q.d_diag, q.stream));
        MFWF_TRY(launch_harm_diag_pol(q, q.d_salm, q.d_salm_prev, nb, q.d_red, q.d_diag));
    } else {
        MFWF_TRY(launch_chi2_pix(rho, q.d_M, q.d_smap, q.npix, nb, lam, q.tau, q.d_red,
                                 q.nred_blocks, q.d_diag, q.stream));
        MFWF_TRY(launch_harm_diag(q, q.d_salm, q.d_salm_prev, nb, q.d_red, q.d_diag));
    }
    MFWF_HIP(hipMemcpyAsync(dg.data(), q.d_diag, sizeof(double) * 8 * nb, hipMemcpyDeviceToHost,
                            q.stream));
    MFWF_HIP(hipStreamSynchronize(q.stream));
    return MFWF_OK;
}

// a rise of chi^2 at fixed lambda that no quadrature gap explains, in sigma_chi2
static constexpr double kUnstableSigmas = 10.0;

struct CoolOpts {
    int l0, step, margin, nchk, max_iters;
    double plateau, final_tol;
};

static int cooled_chunk(mfwf_plan plan, const double *data, int nb, double *s_alm_out,
                        double *s_map_out, const CoolOpts &o, std::vector<double> &stages,
                        bool &converged, mfwf_solve_info *info) {
    Plan &p = plan->p;
    const long nc = p.ncomp;
    if (p.spin == 2)
        MFWF_TRY(launch_rho_from_data_pol(data, p.d_M, p.d_rho, p.npix, nb, p.stream));
    else
        MFWF_TRY(launch_rho_from_data(data, p.d_M, p.d_rho, p.npix, nb, p.stream));
    const double *rho = p.d_rho;
    MFWF_TRY(check_source_finite(p, rho, nb));
    const double sigma = std::sqrt(2.0 * (double)p.ndof), tomega = p.tau * p.omega;
    std::vector<double> dg(8L * nb), prev(nb), last_dchi2(nb, 0.0);
    Plan *cur = nullptr;
    // chained iterations stay within this solve: every plan it used leaves without them
    struct ChainOff {
        mfwf_plan plan;
        ~ChainOff() {
            plan->p.chain = plan->p.chain_ready = false;
            for (auto &kv : plan->sub) kv.second->p.chain = kv.second->p.chain_ready = false;
        }
    } chain_off{plan};
    int l_iter = std::min(o.l0, p.lmax);
    long total = 0;
    double lam = 1.0;
    bool to_one = false;  // l_iter has reached lmax: the next stage is lambda = 1
    converged = false;
    stages.clear();
    for (;;) {
        // this stage: lambda from the signal power at l_iter (b_l = 1), never below 1
        lam = to_one ? 1.0 : std::max(1.0, plan->cl[l_iter] / tomega);
        const int lk = (o.margin < 0 || to_one) ? p.lmax : std::min(p.lmax, l_iter + o.margin);
        const bool final_stage = (lam == 1.0 && lk == p.lmax);
        const double tol = final_stage ? o.final_tol : o.plateau;
        Plan *q = nullptr;
        MFWF_TRY(cooled_plan(plan, lk, q));
        if (q != cur) {
            // the iterate passes as its pixel map (zero at the start)
            if (cur)
                MFWF_HIP(hipMemcpyAsync(q->d_smap, cur->d_smap, sizeof(double) * nc * p.npix * nb,
                                        hipMemcpyDeviceToDevice, q->stream));
            else
                MFWF_TRY(launch_fill(q->d_smap, nc * p.npix * nb, 0.0, q->stream));
            MFWF_TRY(launch_fill(reinterpret_cast<double *>(q->d_salm), 2 * nc * q->nalm * nb, 0.0, q->stream));
            if (q->dtype == MFWF_F32) {  // harmonic iterate of the FP32 form (outside any capture)
                MFWF_HIP(hipMemsetAsync(q->d_s32, 0, sizeof(float) * (size_t)q->nalm * q->C2, q->stream));
                if (q->spin == 2)
                    MFWF_HIP(hipMemsetAsync(q->d_seb32, 0, sizeof(float) * (size_t)q->nalm * 2 * q->C2, q->stream));
            }
            // batched FP32 form: chained iterations once the first one on this plan has run
            // from the map
            q->chain = (q->dtype == MFWF_F32 && (q->spin == 0 || fft_pol_chain_ok(*q)));
            q->chain_ready = false;
            cur = q;
        }
        StageGraph sg;
        bool captured = false, have_prev = false, plateau = false;
        long its = 0;
        // lowest chi^2 of this stage per map, and the last two changes between checks.  At
        // fixed lambda the iteration lowers chi^2 up to the quadrature gap of the
        // pixelisation; on coarse grids it can settle well above a minimum it passed through,
        // rising by shrinking steps.  Rising by growing steps far above that minimum means an
        // eigenvalue above 1: an unstable iteration (lmax too high for the nside's quadrature).
        std::vector<double> smin(nb, INFINITY), d1(nb, 0.0), d2(nb, 0.0);
        std::fill(last_dchi2.begin(), last_dchi2.end(), 0.0);
        while (total < o.max_iters) {
            const long run = std::min<long>(o.nchk, o.max_iters - total);
            long plain = run - 1;
            if (q->chain && !q->chain_ready && plain > 0) {  // before any capture
                MFWF_TRY(iteration(*q, rho, nb, lam, false));
                plain--;
            }
            if (plain >= 2 && q->stream != nullptr) {
                if (!captured) {
                    MFWF_TRY(sg.capture(*q, rho, nb, lam));
                    captured = true;
                }
                MFWF_TRY(sg.launch(*q, (int)plain));
            } else {
                for (long k = 0; k < plain; k++) MFWF_TRY(iteration(*q, rho, nb, lam, false));
            }
            MFWF_TRY(iteration(*q, rho, nb, lam, true));
            MFWF_TRY(cooled_diag(*q, rho, nb, lam, dg));
            its += run;
            total += run;
            double worst = 0.0;
            for (int b = 0; b < nb; b++) {
                const double chi = dg[8 * b] + dg[8 * b + 1];
                if (!std::isfinite(chi))
                    return fail(MFWF_ENAN, "chi^2 is not finite: the iteration diverged (lmax above "
                                           "what the nside's quadrature supports?)");
                const double dc = have_prev ? chi - prev[b] : 0.0;
                if (have_prev && chi > smin[b] + kUnstableSigmas * sigma && dc > d1[b] &&
                    d1[b] > d2[b] && d2[b] > 0.0)
                    return fail(MFWF_ENAN, "chi^2 at fixed lambda grows by increasing steps, more "
                                           "than 10 sigma_chi2 above its minimum in this stage: the "
                                           "iteration is unstable at this band limit (lmax too high "
                                           "for the nside's quadrature)");
                smin[b] = std::min(smin[b], chi);
                d2[b] = d1[b];
                d1[b] = dc;
                if (have_prev) worst = std::max(worst, std::fabs(chi - prev[b]) / (double)run);
                last_dchi2[b] = have_prev ? (chi - prev[b]) / (double)run : 0.0;
                prev[b] = chi;
            }
            if (have_prev && worst < tol * sigma) {
                plateau = true;
                break;
            }
            have_prev = true;
        }
        stages.insert(stages.end(), {(double)l_iter, lam, (double)lk, (double)its,
                                     (dg[0] + dg[1]) / (double)p.ndof});
        if (plateau && final_stage) converged = true;
        if (converged || total >= o.max_iters) break;
        // next stage: l_iter doubles (at most + step); once a stage at l_iter = lmax has
        // settled, lambda goes to 1 over the full band limit
        if (l_iter >= p.lmax)
            to_one = true;
        else
            l_iter = std::min({2 * l_iter, l_iter + o.step, p.lmax});
    }
    // outputs in this plan's packing
    if (cur != &p) {
        MFWF_TRY(launch_repack_alm(*cur, cur->d_salm, p, p.d_salm, (int)(nc * nb)));
        MFWF_HIP(hipMemcpyAsync(p.d_smap, cur->d_smap, sizeof(double) * nc * p.npix * nb,
                                hipMemcpyDeviceToDevice, p.stream));
        MFWF_HIP(hipStreamSynchronize(cur->stream));
    }
    if (s_alm_out)
        MFWF_HIP(hipMemcpyAsync(s_alm_out, p.d_salm, sizeof(double2) * nc * p.nalm * nb,
                                hipMemcpyDeviceToDevice, p.stream));
    if (s_map_out)
        MFWF_HIP(hipMemcpyAsync(s_map_out, p.d_smap, sizeof(double) * nc * p.npix * nb,
                                hipMemcpyDeviceToDevice, p.stream));
    if (info) {
        for (int b = 0; b < nb; b++) {
            mfwf_solve_info &in = info[b];
            in.iters_done = (int)total;
            in.lambda = lam;
            in.chi2 = dg[8 * b + 0] + dg[8 * b + 1];
            in.chi2_harm = dg[8 * b + 1];
            in.dnorm = std::sqrt(dg[8 * b + 2]);
            in.snorm = std::sqrt(dg[8 * b + 3]);
            in.tau = p.tau;
            in.n_dof = p.ndof;
            in.n_checks = 0;
            in.dchi2 = last_dchi2[b];
            in.rel_change = in.snorm > 0.0 ? in.dnorm / in.snorm : 0.0;
        }
    }
    return MFWF_OK;
}

// ---- the error-bound schedule of Sect. 2.2 ----------------------------------------------
struct BoundOpts {
    double m_sigma, lam_tol, stall_frac;
    int stall_iters, max_iters;
};

// G(lambda) = max over maps of chi^2(lambda, s) - b (Eq. 6 at the current iterate) and its
// derivative for the map attaining the max; chi^2 = H + P(lambda) with the harmonic part H
// fixed and the pixel part P from one pass over the maps.
struct BoundEval {
    Plan &p;
    const double *rho;
    int nb;
    std::vector<double> H, b, P, out;
    int evals = 0;
    BoundEval(Plan &q, const double *r, int n) : p(q), rho(r), nb(n), H(n, 0.0), b(n), P(n), out(2 * n) {}
    int operator()(double lam, double &G, double &dG) {
        double *partial = p.d_red, *o2 = p.d_red + 2L * 256 * nb;
        if (p.spin == 2)
            MFWF_TRY(launch_chi2_pix_dlam_pol(rho, p.d_M, p.d_smap, p.npix, nb, lam, p.tau,
                                              partial, 256, o2, p.stream));
        else
            MFWF_TRY(launch_chi2_pix_dlam(rho, p.d_M, p.d_smap, p.npix, nb, lam, p.tau, partial,
                                          256, o2, p.stream));
        MFWF_HIP(hipMemcpyAsync(out.data(), o2, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost,
                                p.stream));
        MFWF_HIP(hipStreamSynchronize(p.stream));
        evals++;
        G = -INFINITY;
        dG = 0.0;
        for (int k = 0; k < nb; k++) {
            P[k] = out[2 * k];
            const double g = H[k] + P[k] - b[k];
            if (!std::isfinite(g))
                return fail(MFWF_ENAN, "chi^2 is not finite: the iteration diverged");
            if (g > G) {
                G = g;
                dG = out[2 * k + 1];
            }
        }
        return MFWF_OK;
    }
};

// The smallest lambda in [1, hi] with chi^2(lambda, s) <= b for every map (G is decreasing and
// convex in lambda): safeguarded Newton on a bracket [lo, hi] with G(lo) > 0 >= G(hi); the
// returned value is the bracket's upper end, where the bound holds.  hi grows if G(hi) > 0.
static int bound_lambda(BoundEval &ev, double hi, double &lam) {
    double G, dG;
    MFWF_TRY(ev(1.0, G, dG));
    if (G <= 0.0) {
        lam = 1.0;
        return MFWF_OK;
    }
    double lo = 1.0, Gh, dGh;
    MFWF_TRY(ev(hi, Gh, dGh));
    for (int k = 0; Gh > 0.0; k++) {
        if (k == 60) return fail(MFWF_ENAN, "no lambda meets the chi^2 bound");
        lo = hi;
        hi *= 4.0;
        MFWF_TRY(ev(hi, Gh, dGh));
    }
    double x = hi, Gx = Gh, dGx = dGh;
    for (int it = 0; it < 60 && hi / lo - 1.0 > 1e-12; it++) {
        double xn = (dGx < 0.0) ? x - Gx / dGx : 0.0;
        if (!(xn > lo && xn < hi)) xn = std::sqrt(lo * hi);
        MFWF_TRY(ev(xn, Gx, dGx));
        x = xn;
        if (Gx > 0.0)
            lo = x;
        else
            hi = x;
        if (std::fabs(Gx) <= 1e-13 * std::fabs(ev.b[0]) + 1e-300 && Gx <= 0.0) break;
    }
    lam = hi;
    return MFWF_OK;
}

static int bounded_chunk(Plan &p, const double *data, int nb, double *s_alm_out,
                         double *s_map_out, const BoundOpts &o, std::vector<double> &trace,
                         int &n_updates, bool &reached_one, mfwf_solve_info *info) {
    const long nc = p.ncomp;
    if (p.spin == 2)
        MFWF_TRY(launch_rho_from_data_pol(data, p.d_M, p.d_rho, p.npix, nb, p.stream));
    else
        MFWF_TRY(launch_rho_from_data(data, p.d_M, p.d_rho, p.npix, nb, p.stream));
    const double *rho = p.d_rho;
    MFWF_TRY(check_source_finite(p, rho, nb));
    MFWF_TRY(launch_fill(p.d_smap, nc * p.npix * nb, 0.0, p.stream));
    MFWF_TRY(launch_fill(reinterpret_cast<double *>(p.d_salm), 2 * nc * p.nalm * nb, 0.0, p.stream));
    if (p.dtype == MFWF_F32) {
        MFWF_HIP(hipMemsetAsync(p.d_s32, 0, sizeof(float) * (size_t)p.nalm * p.C2, p.stream));
        if (p.spin == 2)
            MFWF_HIP(hipMemsetAsync(p.d_seb32, 0, sizeof(float) * (size_t)p.nalm * 2 * p.C2, p.stream));
    }
    const double sigma = std::sqrt(2.0 * (double)p.ndof);
    BoundEval ev(p, rho, nb);
    for (int k = 0; k < nb; k++) ev.b[k] = (double)p.ndof - o.m_sigma * sigma;
    std::vector<double> dg(8L * nb);
    double lam;
    MFWF_TRY(bound_lambda(ev, 1e3, lam));  // x = 0: chi^2(lambda, 0) = b
    n_updates = 0;
    reached_one = false;
    trace.clear();
    int stall = 0;
    double last_lam = lam;  // lambda of the last iteration run
    for (int it = 0; it < o.max_iters; it++) {
        MFWF_TRY(iteration(p, rho, nb, lam, true));
        last_lam = lam;
        // harmonic part of chi^2 at the new iterate
        if (p.spin == 2)
            MFWF_TRY(launch_harm_diag_pol(p, p.d_salm, p.d_salm_prev, nb, p.d_red, p.d_diag));
        else
            MFWF_TRY(launch_harm_diag(p, p.d_salm, p.d_salm_prev, nb, p.d_red, p.d_diag));
        MFWF_HIP(hipMemcpyAsync(dg.data(), p.d_diag, sizeof(double) * 8 * nb, hipMemcpyDeviceToHost,
                                p.stream));
        MFWF_HIP(hipStreamSynchronize(p.stream));
        for (int k = 0; k < nb; k++) ev.H[k] = dg[8 * k + 1];
        double G, dG;
        MFWF_TRY(ev(lam, G, dG));
        trace.insert(trace.end(), {lam, ev.H[0] + ev.P[0], ev.b[0]});
        if (lam == 1.0) {  // the last iteration ran at lambda = 1
            reached_one = true;
            break;
        }
        // the next lambda: the smallest one with chi^2(lambda, x) <= b; it can exceed the
        // current one when this iteration raised chi^2(lambda, x) above b, which the
        // pixelised sphere allows by a margin of its quadrature gap (the iteration's fixed
        // point is not exactly the minimiser of chi^2)
        double nl;
        MFWF_TRY(bound_lambda(ev, lam, nl));
        if (nl > lam * (1.0 - o.stall_frac)) {
            if (++stall >= o.stall_iters) {
                // converged at lambda > 1 with b < chi^2_min(1): b' = chi^2_min(lambda) +
                // (lambda - 1) tau x^T S^-2 x, the first-order expansion of the convex
                // chi^2_min at lambda = 1.  At the minimiser S^-1 x = N'^-1 (d - x), so the
                // increment is (lambda - 1) times minus the lambda-derivative of the pixel
                // term at fixed x, which the pass below returns.
                MFWF_TRY(ev(lam, G, dG));
                for (int k = 0; k < nb; k++)
                    ev.b[k] = ev.H[k] + ev.P[k] - (lam - 1.0) * ev.out[2 * k + 1];
                n_updates++;
                stall = 0;
                MFWF_TRY(bound_lambda(ev, lam, nl));
            }
        } else {
            stall = 0;
        }
        if (nl <= 1.0 + o.lam_tol) nl = 1.0;
        lam = nl;
    }
    MFWF_TRY(cooled_diag(p, rho, nb, last_lam, dg));
    if (s_alm_out)
        MFWF_HIP(hipMemcpyAsync(s_alm_out, p.d_salm, sizeof(double2) * nc * p.nalm * nb,
                                hipMemcpyDeviceToDevice, p.stream));
    if (s_map_out)
        MFWF_HIP(hipMemcpyAsync(s_map_out, p.d_smap, sizeof(double) * nc * p.npix * nb,
                                hipMemcpyDeviceToDevice, p.stream));
    if (info) {
        for (int k = 0; k < nb; k++) {
            mfwf_solve_info &in = info[k];
            in.iters_done = (int)(trace.size() / 3);
            in.lambda = last_lam;
            in.chi2 = dg[8 * k + 0] + dg[8 * k + 1];
            in.chi2_harm = dg[8 * k + 1];
            in.dnorm = std::sqrt(dg[8 * k + 2]);
            in.snorm = std::sqrt(dg[8 * k + 3]);
            in.tau = p.tau;
            in.n_dof = p.ndof;
            in.n_checks = 0;
            in.dchi2 = 0.0;
            in.rel_change = in.snorm > 0.0 ? in.dnorm / in.snorm : 0.0;
        }
    }
    return MFWF_OK;
}

}  // namespace mfwf

extern "C" {

int mfwf_solve_cooled(mfwf_plan plan, const double *data, int nmaps, double *s_alm_out,
                      double *s_map_out, mfwf_cool_opts *opts, mfwf_solve_info *info) {
    if (!plan || nmaps < 0) return fail(MFWF_EINVAL, "bad argument");
    Plan &p = plan->p;
    if (!p.have_cov) return fail(MFWF_ENOCOV, "covariances not set");
    if (nmaps > 0 && !data) return fail(MFWF_EINVAL, "data is NULL");
    mfwf_cool_opts u{};
    if (opts) u = *opts;
    if (u.l_iter0 < 0 || u.l_step_max < 0 || u.n_check < 0 || u.max_iters < 0 ||
        u.plateau_tol < 0.0 || u.final_tol < 0.0 || (u.stages && u.stage_rows < 0))
        return fail(MFWF_EINVAL, "negative option");
    CoolOpts o;
    o.l0 = u.l_iter0 ? u.l_iter0 : 20;
    o.step = u.l_step_max ? u.l_step_max : 500;
    o.margin = u.l_margin ? u.l_margin : 100;
    o.nchk = u.n_check ? u.n_check : 5;
    o.max_iters = u.max_iters ? u.max_iters : 20000;
    o.plateau = u.plateau_tol > 0.0 ? u.plateau_tol : 1e-2;
    o.final_tol = u.final_tol > 0.0 ? u.final_tol : 1e-4;
    if (o.nchk < 2) return fail(MFWF_EINVAL, "n_check must be >= 2");
    std::vector<double> stages;
    bool converged = true;
    for (int b0 = 0; b0 < nmaps; b0 += p.max_batch) {
        const int nb = std::min(p.max_batch, nmaps - b0);
        const long nc = p.ncomp;
        bool conv = false;
        MFWF_TRY(cooled_chunk(plan, data + nc * b0 * p.npix, nb,
                              s_alm_out ? s_alm_out + 2L * nc * b0 * p.nalm : nullptr,
                              s_map_out ? s_map_out + nc * b0 * p.npix : nullptr, o, stages, conv,
                              info ? info + b0 : nullptr));
        converged = converged && conv;
    }
    MFWF_HIP(hipStreamSynchronize(p.stream));
    if (opts) {
        const int ns = (int)(stages.size() / 5);
        opts->n_stages = ns;
        opts->converged = converged ? 1 : 0;
        if (opts->stages)
            for (int r = 0; r < std::min(ns, opts->stage_rows); r++)
                for (int k = 0; k < 5; k++) opts->stages[5 * r + k] = stages[5 * r + k];
    }
    return MFWF_OK;
}

int mfwf_solve_bounded(mfwf_plan plan, const double *data, int nmaps, double *s_alm_out,
                       double *s_map_out, mfwf_bound_opts *opts, mfwf_solve_info *info) {
    if (!plan || nmaps < 0) return fail(MFWF_EINVAL, "bad argument");
    Plan &p = plan->p;
    if (!p.have_cov) return fail(MFWF_ENOCOV, "covariances not set");
    if (nmaps > 0 && !data) return fail(MFWF_EINVAL, "data is NULL");
    mfwf_bound_opts u{};
    if (opts) u = *opts;
    if (u.m_sigma < 0.0 || u.lam_tol < 0.0 || u.stall_frac < 0.0 || u.stall_iters < 0 ||
        u.max_iters < 0 || (u.trace && u.trace_rows < 0))
        return fail(MFWF_EINVAL, "negative option");
    BoundOpts o;
    o.m_sigma = u.m_sigma > 0.0 ? u.m_sigma : 5.0;
    o.lam_tol = u.lam_tol > 0.0 ? u.lam_tol : 1e-3;
    o.stall_frac = u.stall_frac > 0.0 ? u.stall_frac : 1e-3;
    o.stall_iters = u.stall_iters > 0 ? u.stall_iters : 5;
    o.max_iters = u.max_iters > 0 ? u.max_iters : 5000;
    std::vector<double> trace;
    int n_updates = 0;
    bool reached = true;
    for (int b0 = 0; b0 < nmaps; b0 += p.max_batch) {
        const int nb = std::min(p.max_batch, nmaps - b0);
        bool r = false;
        const long nc = p.ncomp;
        MFWF_TRY(bounded_chunk(p, data + nc * b0 * p.npix, nb,
                               s_alm_out ? s_alm_out + 2L * nc * b0 * p.nalm : nullptr,
                               s_map_out ? s_map_out + nc * b0 * p.npix : nullptr, o, trace,
                               n_updates, r, info ? info + b0 : nullptr));
        reached = reached && r;
    }
    MFWF_HIP(hipStreamSynchronize(p.stream));
    if (opts) {
        const int n = (int)(trace.size() / 3);
        opts->n_iters = n;
        opts->n_b_updates = n_updates;
        opts->reached_one = reached ? 1 : 0;
        if (opts->trace)
            for (int r = 0; r < std::min(n, opts->trace_rows); r++)
                for (int k = 0; k < 3; k++) opts->trace[3 * r + k] = trace[3 * r + k];
    }
    return MFWF_OK;
}

int mfwf_plan_work(mfwf_plan plan, double *out4) {
    if (!plan || !out4) return fail(MFWF_EINVAL, "NULL argument");
    const Plan &p = plan->p;
    out4[0] = p.work_tuples;
    out4[1] = (double)p.npair * (double)p.nalm;
    out4[2] = p.npair;
    out4[3] = p.fftmax;
    return MFWF_OK;
}

int mfwf_plan_tuning(mfwf_plan plan, int *out8) {
    if (!plan || !out8) return fail(MFWF_EINVAL, "NULL argument");
    const Plan &p = plan->p;
    int k[kNumKnobs];
    get_knobs(p, k);
    for (int q = 0; q < kNumKnobs; q++) out8[q] = k[q];
    out8[7] = p.tune_source;
    return MFWF_OK;
}

int mfwf_time_kernels(mfwf_plan plan, int nmaps, int reps, double *ms_out) {
    if (!plan || !ms_out || reps < 1 || nmaps < 1) return fail(MFWF_EINVAL, "bad argument");
    Plan &p = plan->p;
    if (!p.have_cov) return fail(MFWF_ENOCOV, "covariances not set");
    if (nmaps > p.max_batch) return fail(MFWF_EINVAL, "nmaps > max_batch");
    const int nb = nmaps;
    const bool f32 = (p.dtype == MFWF_F32);
    for (int k = 0; k < 6; k++) {
        std::function<int()> f;
        if (f32 && p.spin == 2) {
            // 0 pixel update, 1 forward transforms + layout, 2 the three analysis GEMMs,
            // 3 combination and filter, 4 the three synthesis GEMMs, 5 layout + inverse
            switch (k) {
                case 0: f = [&] { return launch_pixel_update_pol(p.d_rho, p.d_M, p.d_smap, p.d_t, p.npix, nb, 1.0, p.tau, p.stream); }; break;
                case 1: f = [&] { MFWF_TRY(launch_fft_fwd_f32(p, p.d_t, nullptr, 1.0, p.d_phf, 3 * nb)); return launch_rows_to_cols_pol(p, nb); }; break;
                case 2: f = [&] {
                    MFWF_TRY(launch_gemm_analysis_raw(p, nb, 2, p.d_lam, p.d_ph32, p.d_a32, 0));
                    MFWF_TRY(launch_gemm_analysis_raw(p, nb, 4, p.d_fp, p.d_ph32p, p.d_ap32, 0));
                    return launch_gemm_analysis_raw(p, nb, 4, p.d_fm, p.d_ph32p, p.d_ar32, 1); }; break;
                case 3: f = [&] { return launch_pol_combine(p, p.tau * p.omega, kPolFilter); }; break;
                case 4: f = [&] {
                    MFWF_TRY(launch_gemm_synthesis_on(p, nb, 2, p.d_lam, p.d_s32, p.d_ph32, 0));
                    MFWF_TRY(launch_gemm_synthesis_on(p, nb, 4, p.d_fp, p.d_seb32, p.d_ph32p, 0));
                    return launch_gemm_synthesis_on(p, nb, 4, p.d_fm, p.d_seb32, p.d_ph32p, 1, 1); }; break;
                default: f = [&] { MFWF_TRY(launch_cols_to_rows_pol(p, nb)); return launch_fft_inv_f32(p, p.d_phf, p.d_smap, 3 * nb); }; break;
            }
            float ms = 0.f;
            MFWF_TRY(time_launches(p, reps, f, ms));
            ms_out[k] = ms / reps;
            continue;
        }
        if (f32) {
            switch (k) {
                case 0: ms_out[k] = 0.0; continue;  // pixel update runs inside the forward transforms
                // 1: the ring step of a chained iteration: the previous synthesis back to
                // pixels, pixel update and forward transforms in one kernel on the columns
                // (the inverse transforms run there, so 5 is empty)
                case 1: f = [&] { return launch_fft_inv_fwd_cols(p, p.d_rho, 1.0, nullptr, nb); }; break;
                case 2: f = [&] { return launch_gemm_analysis(p, nb, nullptr, p.d_s32, p.omega, p.omega * p.tau, p.omega); }; break;
                case 3: ms_out[k] = 0.0; continue;  // harmonic update runs inside the analysis
                case 4: f = [&] { return launch_gemm_synthesis(p, nb); }; break;
                default: ms_out[k] = 0.0; continue;
            }
            float ms = 0.f;
            MFWF_TRY(time_launches(p, reps, f, ms));
            ms_out[k] = ms / reps;
            continue;
        }
        if (p.spin == 2) {
            switch (k) {
                case 0: f = [&] { return launch_pixel_update_pol(p.d_rho, p.d_M, p.d_smap, p.d_t, p.npix, nb, 1.0, p.tau, p.stream); }; break;
                case 1: f = [&] { return launch_fft_fwd(p, p.d_t, p.d_phase, 3 * nb); }; break;
                case 2: f = [&] { return launch_leg_analysis_pol(p, p.d_phase, p.d_apart, nb); }; break;
                case 3: f = [&] { return launch_harmonic_pol(p, p.d_apart, pol_ngroup(p), p.omega, p.tau * p.omega, kHarmWiener, p.d_salm, p.d_sp, nullptr, nb); }; break;
                case 4: f = [&] { return launch_leg_synth_pol(p, p.d_sp, p.d_phase, nb); }; break;
                default: f = [&] { return launch_fft_inv(p, p.d_phase, p.d_smap, 3 * nb); }; break;
            }
            float ms = 0.f;
            MFWF_TRY(time_launches(p, reps, f, ms));
            ms_out[k] = ms / reps;
            continue;
        }
        switch (k) {
            case 0: ms_out[k] = 0.0; continue;  // pixel update runs inside the forward transforms
            case 1: f = [&] { return launch_fft_fwd_pix(p, p.d_smap, p.d_rho, 1.0, p.d_phase, nb); }; break;
            case 2: f = [&] { return launch_leg_analysis(p, p.d_phase, p.d_apart, nb); }; break;
            case 3: f = [&] { return launch_harmonic(p, p.d_apart, p.ngroup, p.omega, p.omega * p.tau, kHarmWiener, p.d_salm, p.d_sp, nullptr, nb, p.omega); }; break;
            case 4: f = [&] { return launch_leg_synth(p, p.d_sp, p.d_phase, nb); }; break;
            default: f = [&] { return launch_fft_inv(p, p.d_phase, p.d_smap, nb); }; break;
        }
        float ms = 0.f;
        MFWF_TRY(time_launches(p, reps, f, ms));
        ms_out[k] = ms / reps;
    }
    return MFWF_OK;
}

}  // extern "C"
