// Serving runtime: independent Wiener-filter requests (each with its own data, noise
// variance map and mask) solved on one GPU by continuous batching.
//
// Requests of the same shape (nside, lmax, dtype, lambda, C_l) share a pool: one plan with
// `slots` map slots, each slot holding its own M row and tau.  A worker thread
//   - admits queued requests into free slots at iteration boundaries (M = N^-1 mask,
//     tau = 1 / max M, rho = M d and s = 0 written into the slot on the pool's stream),
//   - launches messenger iterations (Eqs. 3-4) over the occupied slot range of busy pools (the
//     iteration is captured once per slot count and replayed as a hipGraph; FP32 pools chain
//     their iterations through the synthesis columns as a standalone solve does, a new
//     slot's columns zeroed at admission).  Pools run on a
//     few server-owned lanes (streams), so that pools on different lanes overlap on the GPU.
//     Within a lane the worker picks the busy pool that has used the least GPU time (start-
//     time fair queueing on each iteration's measured duration), so a small pool runs many
//     iterations while a large one runs one instead of advancing in lockstep with it,
//   - retires a slot after its K-th iteration, copying s_lm and Y s into the caller's
//     buffers, and frees the slot for the next request,
//   - creates a pool when a request needs a new shape and its estimated footprint fits the
//     HBM budget, evicting idle pools (least recently used first) to make room; when none
//     is idle, the pools that would make room stop admitting until they drain.
// Latency runs from submission to the completion of the copies into the caller's buffers.
// The scheduling decisions are device-free (serve_core.h, which the CPU simulation of the
// tests also runs); this file is their HIP backend, request validation and the C ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "mfwf_internal.h"
#include "serve_core.h"

namespace mfwf {

using Clock = std::chrono::steady_clock;

struct SrvRequest {
    uint64_t id = 0;
    mfwf_request r{};
    std::vector<double> cl;
    double tau = 0.0;
    Clock::time_point t_arrival, t_done;
    int status = MFWF_OK;
    std::string err;
    bool done = false;
};

// Device bytes of a pool: per-slot maps (rho, t, s, M), ring-Fourier and harmonic
// workspaces, recurrence tables; the FP32 form adds its lambda table and column arrays.
static size_t estimate_pool_bytes(int nside, int lmax, int dtype, int B) {
    const double npix = 12.0 * nside * nside, nring = 4.0 * nside - 1, npair = 2.0 * nside;
    const double nm = lmax + 1, nalm = nm * (lmax + 2) / 2;
    const double groups = npair / 64.0 + 1;
    double b = 8.0 * npix * B * 4 + 16.0 * 3 * B * nalm + 8.0 * 2 * nalm + nm * npair * 20.0;
    if (dtype == MFWF_F32) {
        const double Bp = 16.0 * ((B + 15) / 16);
        b += 16.0 * nm * nring + 16.0 * groups * nalm;           // unused FP64 rows, 1 map
        const double table = 4.0 * npair * (nalm + 64.0 * nm) * 1.05;  // lambda table (padded)
        b += table / 4.0;                                        // recurrence segment states
        if (nside <= 1024) b += table;
        else b += 64.0 * B * nside * nside;                      // split ring scratch
        b += 8.0 * B * nring * (nm + 15) + 4.0 * nring * nm * 2 * Bp;  // rows, column layout
        b += 2 * 4.0 * nalm * 2 * Bp;                            // coefficients in columns
    } else {
        b += 16.0 * B * nm * nring + 16.0 * groups * B * nalm;
        if (nside > 1024) b += 64.0 * B * nside * nside;  // split ring scratch
    }
    return (size_t)(1.1 * b) + (64u << 20);
}

// the plan shapes a pool can take: FP64 and the FP32 form up to nside 2048
static int check_shape(int nside, int lmax, int dtype) {
    if (nside < 1 || nside > 2048 || (nside & (nside - 1)) != 0)
        return fail(MFWF_EINVAL, "nside must be a power of two in [1, 2048]");
    if (lmax < 1 || lmax > 4 * nside) return fail(MFWF_EINVAL, "lmax must be in [1, 4 nside]");
    if (dtype != MFWF_F64 && dtype != MFWF_F32) return fail(MFWF_EINVAL, "bad dtype");
    return MFWF_OK;
}

}  // namespace mfwf

using namespace mfwf;

struct mfwf_server_s;

namespace mfwf {

struct SlotGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// The device side of the scheduling core (serve_core.h): a pool is one plan with `slots`
// map slots, each with its own M row and tau; an iteration over the occupied slot range is
// captured once per slot count and replayed as a hipGraph between two timing events.
struct HipBackend {
    using Request = SrvRequest;
    struct PoolState {
        Plan plan;
        bool plan_ok = false;
        std::map<int, SlotGraph> graphs;  // by slot count
        double lam = 1.0;
    };
    using LaneState = hipStream_t;
    struct Timer {
        hipEvent_t t0 = nullptr, t1 = nullptr;
    };
    using Done = hipEvent_t;

    mfwf_server_s *s = nullptr;
    std::vector<hipEvent_t> spare;  // timing events for reuse

    serve::Key key_of(const Request &q) const {
        return serve::Key{q.r.nside, q.r.lmax, q.r.dtype, q.r.lambda, q.cl};
    }
    int iters_of(const Request &q) const { return q.r.iters; }
    size_t pool_bytes(const serve::Key &k, int slots) const {
        return estimate_pool_bytes(k.nside, k.lmax, k.dtype, slots);
    }
    std::string last_error() const { return mfwf_last_error(); }

    int create(PoolState &P, const serve::Key &key, int slots, LaneState &lane, std::string &err) {
        Plan &p = P.plan;
        p.stream = lane;
        P.plan_ok = true;  // free whatever a failed creation allocated
        P.lam = key.lam;
        int status = plan_create(key.nside, key.lmax, 0, key.dtype, slots, lane, true, p);
        if (status == MFWF_OK) status = plan_set_cl(p, key.cl.data());
        if (status == MFWF_OK && key.dtype == MFWF_F32) {
            // FP32 pools chain their iterations as a standalone solve does: each iteration's
            // ring step starts from the previous synthesis in the columns (zero for a new
            // slot), and the maps are formed only when a request retires
            status = launch_fill(reinterpret_cast<double *>(p.d_ph32), (long)p.nring * p.nm * p.C2 / 2,
                                 0.0, p.stream);
            p.chain = p.chain_ready = true;
        }
        if (status != MFWF_OK) err = std::string("pool plan: ") + mfwf_last_error();
        return status;
    }

    void destroy(PoolState &P) {
        // iterations and result copies may still be in flight on the lane's stream
        if (P.plan.stream) (void)hipStreamSynchronize(P.plan.stream);
        for (auto &g : P.graphs) {
            if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
            if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
        }
        P.graphs.clear();
        if (P.plan_ok) plan_destroy(P.plan);
        P.plan_ok = false;
    }

    // request q into slot b (all on the pool's stream, after any earlier step)
    int admit(PoolState &P, int b, Request &q) {
        Plan &p = P.plan;
        const long off = (long)b * p.npix;
        MFWF_TRY(launch_mask_product(q.r.ninv, q.r.mask, p.d_M + off, p.npix, p.stream));
        MFWF_TRY(launch_fill(p.d_tau + b, 1, q.tau, p.stream));
        MFWF_TRY(launch_rho_from_data(q.r.data, p.d_M + off, p.d_rho + off, p.npix, 1, p.stream));
        MFWF_TRY(launch_fill(p.d_smap + off, p.npix, 0.0, p.stream));
        if (p.chain) MFWF_TRY(launch_zero_map_cols(p, b));  // the slot's synthesis columns: s = 0
        return MFWF_OK;
    }

    int graph(PoolState &P, int nb, hipGraphExec_t &exec) {
        auto it = P.graphs.find(nb);
        if (it != P.graphs.end()) {
            exec = it->second.exec;
            return MFWF_OK;
        }
        SlotGraph g;
        MFWF_HIP(hipStreamBeginCapture(P.plan.stream, hipStreamCaptureModeThreadLocal));
        int st = plan_iteration(P.plan, P.plan.d_rho, nb, P.lam);
        hipError_t e = hipStreamEndCapture(P.plan.stream, &g.graph);
        if (st != MFWF_OK) {
            if (g.graph) (void)hipGraphDestroy(g.graph);
            return st;
        }
        if (e != hipSuccess) return fail(MFWF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g.graph);
            return fail(MFWF_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        P.graphs[nb] = g;
        exec = g.exec;
        return MFWF_OK;
    }

    hipEvent_t take_event() {
        hipEvent_t e = nullptr;
        if (!spare.empty()) {
            e = spare.back();
            spare.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }

    int launch(PoolState &P, int nb, LaneState &lane, Timer &t, std::string &err) {
        hipGraphExec_t exec = nullptr;
        int st = graph(P, nb, exec);
        t.t0 = take_event();
        t.t1 = take_event();
        if (st == MFWF_OK && (!t.t0 || !t.t1)) st = fail(MFWF_EDEVICE, "event creation failed");
        if (st == MFWF_OK && (hipEventRecord(t.t0, lane) != hipSuccess ||
                              hipGraphLaunch(exec, lane) != hipSuccess ||
                              hipEventRecord(t.t1, lane) != hipSuccess))
            st = fail(MFWF_EDEVICE, "graph launch failed");
        if (st != MFWF_OK) {
            recycle(t);
            err = mfwf_last_error();
        }
        return st;
    }

    int poll(Timer &t, bool &done, double &ms, std::string &err) {
        const hipError_t e = hipEventQuery(t.t1);
        done = e != hipErrorNotReady;
        if (!done) return MFWF_OK;
        float f = 0.f;
        if (e == hipSuccess && hipEventElapsedTime(&f, t.t0, t.t1) == hipSuccess) ms = f;
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return MFWF_EDEVICE;
        }
        return MFWF_OK;
    }

    void recycle(Timer &t) {
        if (t.t0) spare.push_back(t.t0);
        if (t.t1) spare.push_back(t.t1);
        t.t0 = t.t1 = nullptr;
    }

    int finish(PoolState &P, int nb) { return plan_finish_alm(P.plan, nb); }

    // copies of slot b's results into the caller's buffers, and an event after them
    int retire(PoolState &P, int b, Request &q, Done &ev) {
        Plan &p = P.plan;
        if (q.r.s_alm_out)
            MFWF_HIP(hipMemcpyAsync(q.r.s_alm_out, p.d_salm + (long)b * p.nalm, sizeof(double2) * p.nalm,
                                    hipMemcpyDeviceToDevice, p.stream));
        if (q.r.s_map_out)
            MFWF_HIP(hipMemcpyAsync(q.r.s_map_out, p.d_smap + (long)b * p.npix, sizeof(double) * p.npix,
                                    hipMemcpyDeviceToDevice, p.stream));
        MFWF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        MFWF_HIP(hipEventRecord(ev, p.stream));
        return MFWF_OK;
    }

    int poll_done(Done &ev, bool &done, std::string &err) {
        const hipError_t e = hipEventQuery(ev);
        done = e != hipErrorNotReady;
        if (!done) return MFWF_OK;
        (void)hipEventDestroy(ev);
        ev = nullptr;
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return MFWF_EDEVICE;
        }
        return MFWF_OK;
    }

    void sync(LaneState &lane) { (void)hipStreamSynchronize(lane); }
    void complete(const std::shared_ptr<Request> &q, int status, const std::string &err);
    void publish(const serve::Stats &st);
};

}  // namespace mfwf

struct mfwf_server_s {
    int device = 0, slots = 0;
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<SrvRequest>> queue;           // submitted, not yet seen by the worker
    std::unordered_map<uint64_t, std::shared_ptr<SrvRequest>> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    // worker-only state: the scheduling core and its device backend
    HipBackend be;
    std::unique_ptr<serve::Core<HipBackend>> core;
    // request validation (caller threads)
    std::mutex vmu;
    hipStream_t vstream = nullptr;
    double *vscratch = nullptr, *vpart = nullptr, *vout = nullptr;
    long vcap = 0;
    // statistics (under mu): completed, queued, occupied slots, pools, pool bytes,
    // iterations launched, pools created, pools evicted
    double stat[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace mfwf {

void HipBackend::complete(const std::shared_ptr<SrvRequest> &q, int status, const std::string &err) {
    std::lock_guard<std::mutex> lk(s->mu);
    q->status = status;
    q->err = err;
    q->done = true;
    q->t_done = Clock::now();
    if (status == MFWF_OK) s->stat[0] += 1;
    s->cv_done.notify_all();
}

void HipBackend::publish(const serve::Stats &st) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stat[2] = st.occupied;
    s->stat[3] = st.pools;
    s->stat[4] = st.bytes;
    s->stat[5] = st.iterations;
    s->stat[6] = st.created;
    s->stat[7] = st.evicted;
}

static void worker_main(mfwf_server s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (!s->core->busy() && s->queue.empty()) {
                if (s->stop) break;
                s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
                continue;
            }
            while (!s->queue.empty()) {
                s->core->add(s->queue.front());
                s->queue.pop_front();
            }
        }
        // nothing launched: every lane with busy pools holds its run-ahead depth, or only
        // result copies are outstanding
        if (!s->core->step()) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    s->core->shutdown();
}

}  // namespace mfwf

// device resources of a server whose worker has stopped (or never started)
static void release(mfwf_server s) {
    if (s->vscratch) (void)hipFree(s->vscratch);
    if (s->vpart) (void)hipFree(s->vpart);
    if (s->vout) (void)hipFree(s->vout);
    if (s->vstream) (void)hipStreamDestroy(s->vstream);
    if (s->core)
        for (auto &L : s->core->lanes)
            if (L.st) (void)hipStreamDestroy(L.st);
    for (hipEvent_t e : s->be.spare) (void)hipEventDestroy(e);
    delete s;
}

extern "C" {

int mfwf_server_pool_bytes(int nside, int lmax, int dtype, int slots, double *bytes) {
    if (!bytes) return fail(MFWF_EINVAL, "bytes is NULL");
    MFWF_TRY(check_shape(nside, lmax, dtype));
    if (slots < 1 || slots > 512) return fail(MFWF_EINVAL, "slots must be in [1, 512]");
    *bytes = (double)estimate_pool_bytes(nside, lmax, dtype, slots);
    return MFWF_OK;
}

int mfwf_server_create(int slots, double hbm_budget_gb, mfwf_server *out) {
    if (!out) return fail(MFWF_EINVAL, "out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > 512) return fail(MFWF_EINVAL, "slots must be in [1, 512]");
    if (!(hbm_budget_gb > 0.0)) return fail(MFWF_EINVAL, "HBM budget must be positive");
    auto *s = new (std::nothrow) mfwf_server_s();
    if (!s) return fail(MFWF_ENOMEM, "host allocation failed");
    s->slots = slots;
    s->budget = (size_t)(hbm_budget_gb * 1e9);
    s->be.s = s;
    s->core.reset(new (std::nothrow) serve::Core<HipBackend>(s->be, slots, s->budget));
    bool ok = s->core && hipGetDevice(&s->device) == hipSuccess &&
              hipStreamCreateWithFlags(&s->vstream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc((void **)&s->vpart, sizeof(double) * 3 * 1024) == hipSuccess &&
              hipMalloc((void **)&s->vout, sizeof(double) * 8) == hipSuccess;
    if (s->core)
        for (auto &L : s->core->lanes)
            ok = ok && hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        release(s);
        return fail(MFWF_EDEVICE, "server set-up failed");
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return MFWF_OK;
}

int mfwf_server_submit(mfwf_server s, const mfwf_request *r, uint64_t *id) {
    if (!s || !r || !id) return fail(MFWF_EINVAL, "NULL argument");
    MFWF_TRY(check_shape(r->nside, r->lmax, r->dtype));
    if (r->iters < 1) return fail(MFWF_EINVAL, "iters must be >= 1");
    if (!(r->lambda >= 1.0) || std::isinf(r->lambda)) return fail(MFWF_EINVAL, "lambda must be finite and >= 1");
    if (!r->cl || !r->ninv || !r->data) return fail(MFWF_EINVAL, "NULL array");
    auto q = std::make_shared<SrvRequest>();
    q->r = *r;
    q->cl.assign(r->cl, r->cl + r->lmax + 1);
    for (double v : q->cl)
        if (!(v >= 0.0) || std::isinf(v)) return fail(MFWF_EINVAL, "C_l must be finite and >= 0");
    // tau = 1 / max(N^-1 mask), checked now so that a bad request fails at submission
    {
        std::lock_guard<std::mutex> lk(s->vmu);
        const long npix = 12L * r->nside * r->nside;
        if (npix > s->vcap) {
            if (s->vscratch) (void)hipFree(s->vscratch);
            s->vscratch = nullptr;
            s->vcap = 0;
            if (hipMalloc((void **)&s->vscratch, 2 * sizeof(double) * npix) != hipSuccess)
                return fail(MFWF_ENOMEM, "validation scratch");
            s->vcap = npix;
        }
        MFWF_TRY(launch_mask_product(r->ninv, r->mask, s->vscratch, npix, s->vstream));
        MFWF_TRY(launch_reduce_max_count(s->vscratch, npix, s->vpart, 1024, s->vout, s->vstream));
        // the source M d behind M (masked pixels give 0 whatever d holds there), and its
        // non-finite entries: NaN or Inf data on an observed pixel
        double *rho = s->vscratch + npix;
        MFWF_TRY(launch_rho_from_data(r->data, s->vscratch, rho, npix, 1, s->vstream));
        MFWF_TRY(launch_count_nonfinite(rho, npix, s->vpart, 1024, s->vout + 3, s->vstream));
        double st[4];
        MFWF_HIP(hipMemcpyAsync(st, s->vout, sizeof(st), hipMemcpyDeviceToHost, s->vstream));
        MFWF_HIP(hipStreamSynchronize(s->vstream));
        if (st[2] > 0.0) return fail(MFWF_ENAN, "inverse noise has negative or non-finite entries");
        if (st[3] > 0.0) return fail(MFWF_ENAN, "data has non-finite values on observed pixels");
        if (!(st[0] > 0.0)) return fail(MFWF_ENOCOV, "no observed pixel: tau undefined");
        q->tau = 1.0 / st[0];
    }
    std::lock_guard<std::mutex> lk(s->mu);
    q->id = s->next_id++;
    q->t_arrival = Clock::now();
    s->reqs[q->id] = q;
    s->queue.push_back(q);
    *id = q->id;
    s->cv_work.notify_one();
    return MFWF_OK;
}

int mfwf_server_poll(mfwf_server s, uint64_t id, int *done) {
    if (!s || !done) return fail(MFWF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MFWF_EINVAL, "unknown request id");
    *done = it->second->done ? 1 : 0;
    return MFWF_OK;
}

int mfwf_server_wait(mfwf_server s, uint64_t id, double *latency_s) {
    if (!s) return fail(MFWF_EINVAL, "NULL argument");
    std::shared_ptr<SrvRequest> q;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return fail(MFWF_EINVAL, "unknown request id");
        q = it->second;
        s->cv_done.wait(lk, [&] { return q->done; });
        s->reqs.erase(id);
    }
    if (latency_s) *latency_s = std::chrono::duration<double>(q->t_done - q->t_arrival).count();
    if (q->status != MFWF_OK) return fail(q->status, q->err);
    return MFWF_OK;
}

int mfwf_server_stats(mfwf_server s, double *out8) {
    if (!s || !out8) return fail(MFWF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    for (int k = 0; k < 8; k++) out8[k] = s->stat[k];
    out8[1] = (double)(s->queue.size());
    return MFWF_OK;
}

int mfwf_server_destroy(mfwf_server s) {
    if (!s) return MFWF_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    release(s);
    return MFWF_OK;
}

}  // extern "C"
