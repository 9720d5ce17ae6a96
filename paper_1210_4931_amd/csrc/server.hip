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
//     HBM budget, evicting idle pools (least recently used first) to make room.
// Latency runs from submission to the completion of the copies into the caller's buffers.
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

namespace mfwf {

using Clock = std::chrono::steady_clock;

// Lanes: streams the worker schedules pools onto.  The process has few hardware queues (4
// by default) and streams beyond them share queues in FIFO order, so the server keeps its
// own small number of streams and orders the work on each itself.
static constexpr int kLanes = 2;
// iterations in flight per lane (host run-ahead bound)
static constexpr int kLaneDepth = 4;

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

struct PoolKey {
    int nside, lmax, dtype;
    double lam;
    std::vector<double> cl;
    bool operator<(const PoolKey &o) const {
        return std::tie(nside, lmax, dtype, lam, cl) < std::tie(o.nside, o.lmax, o.dtype, o.lam, o.cl);
    }
    bool operator==(const PoolKey &o) const { return !(*this < o) && !(o < *this); }
};

struct SlotGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct Pool {
    PoolKey key;
    Plan plan;
    bool plan_ok = false;
    std::vector<std::shared_ptr<SrvRequest>> slot;
    std::vector<int> done_iters;
    std::map<int, SlotGraph> graphs;  // by slot count
    size_t bytes = 0;
    int active = 0;
    Clock::time_point last_used;
    int lane = 0;                    // index of the server lane whose stream the plan uses
    double weight = 0.0;             // static cost guess used to balance pools over lanes
    double vtime = 0.0;              // GPU milliseconds charged to this pool (fair queueing)
    std::map<int, double> cost_ms;   // measured iteration time by slot count (moving average)
    int nslots = 0;                  // map slots of this pool (the server's, or fewer: below)
    bool draining = false;           // admits no new request: a blocked new pool needs its memory

    ~Pool() {
        // iterations and result copies may still be in flight on the lane's stream, which the
        // server owns
        if (plan.stream) (void)hipStreamSynchronize(plan.stream);
        for (auto &g : graphs) {
            if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
            if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
        }
        if (plan_ok) plan_destroy(plan);
    }

    // expected milliseconds of one iteration over nb slots
    double est_cost(int nb) const {
        if (cost_ms.empty()) return 1.0;
        auto it = cost_ms.lower_bound(nb);
        if (it != cost_ms.end() && it->first == nb) return it->second;
        if (it == cost_ms.end()) --it;  // nearest measured slot count, scaled linearly
        return it->second * (double)nb / (double)it->first;
    }
};

// one launched iteration: timing events around its graph
struct Launch {
    Pool *pool;
    int nb;
    hipEvent_t t0, t1;
};

struct Lane {
    hipStream_t stream = nullptr;
    std::deque<Launch> inflight;
};

struct Finishing {
    std::shared_ptr<SrvRequest> req;
    hipEvent_t ev;
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

struct mfwf_server_s {
    int device = 0, slots = 0;
    size_t budget = 0, used = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<SrvRequest>> queue;           // submitted, not yet seen by the worker
    std::unordered_map<uint64_t, std::shared_ptr<SrvRequest>> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    // worker-only state
    std::deque<std::shared_ptr<SrvRequest>> pending;          // seen, waiting for a slot
    std::vector<std::unique_ptr<Pool>> pools;
    std::vector<Finishing> finishing;
    Lane lanes[kLanes];
    std::vector<hipEvent_t> spare_events;  // timing events for reuse
    // request validation (caller threads)
    std::mutex vmu;
    hipStream_t vstream = nullptr;
    double *vscratch = nullptr, *vpart = nullptr, *vout = nullptr;
    long vcap = 0;
    // statistics (under mu)
    double stat[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace mfwf {

static void finish_request(mfwf_server s, const std::shared_ptr<SrvRequest> &q, int status,
                           const std::string &err) {
    std::lock_guard<std::mutex> lk(s->mu);
    q->status = status;
    q->err = err;
    q->done = true;
    q->t_done = Clock::now();
    if (status == MFWF_OK) s->stat[0] += 1;
    s->cv_done.notify_all();
}

static int pool_graph(Pool &P, int nb, hipGraphExec_t &exec) {
    auto it = P.graphs.find(nb);
    if (it != P.graphs.end()) {
        exec = it->second.exec;
        return MFWF_OK;
    }
    SlotGraph g;
    MFWF_HIP(hipStreamBeginCapture(P.plan.stream, hipStreamCaptureModeThreadLocal));
    int st = plan_iteration(P.plan, P.plan.d_rho, nb, P.key.lam);
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

// Put request q into free slot b of pool P (all on the pool's stream, after any earlier step).
static int admit(mfwf_server s, Pool &P, int b, const std::shared_ptr<SrvRequest> &q) {
    Plan &p = P.plan;
    if (P.active == 0) {
        // a pool that wakes up joins at the least GPU time of the busy pools on its lane, so
        // that time it spent idle is not credited to it
        double vmin = -1.0;
        for (auto &Q : s->pools)
            if (Q.get() != &P && Q->lane == P.lane && Q->active > 0 && (vmin < 0.0 || Q->vtime < vmin))
                vmin = Q->vtime;
        if (vmin > P.vtime) P.vtime = vmin;
    }
    const long off = (long)b * p.npix;
    MFWF_TRY(launch_mask_product(q->r.ninv, q->r.mask, p.d_M + off, p.npix, p.stream));
    MFWF_TRY(launch_fill(p.d_tau + b, 1, q->tau, p.stream));
    MFWF_TRY(launch_rho_from_data(q->r.data, p.d_M + off, p.d_rho + off, p.npix, 1, p.stream));
    MFWF_TRY(launch_fill(p.d_smap + off, p.npix, 0.0, p.stream));
    if (p.chain) MFWF_TRY(launch_zero_map_cols(p, b));  // the slot's synthesis columns: s = 0
    P.slot[b] = q;
    P.done_iters[b] = 0;
    P.active++;
    return MFWF_OK;
}

static int retire(mfwf_server s, Pool &P, int b) {
    Plan &p = P.plan;
    std::shared_ptr<SrvRequest> q = P.slot[b];
    if (q->r.s_alm_out)
        MFWF_HIP(hipMemcpyAsync(q->r.s_alm_out, p.d_salm + (long)b * p.nalm, sizeof(double2) * p.nalm,
                                hipMemcpyDeviceToDevice, p.stream));
    if (q->r.s_map_out)
        MFWF_HIP(hipMemcpyAsync(q->r.s_map_out, p.d_smap + (long)b * p.npix, sizeof(double) * p.npix,
                                hipMemcpyDeviceToDevice, p.stream));
    hipEvent_t ev;
    MFWF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    MFWF_HIP(hipEventRecord(ev, p.stream));
    s->finishing.push_back(Finishing{q, ev});
    P.slot[b].reset();
    P.active--;
    return MFWF_OK;
}

static hipEvent_t take_event(mfwf_server s) {
    hipEvent_t e = nullptr;
    if (!s->spare_events.empty()) {
        e = s->spare_events.back();
        s->spare_events.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

static void fail_pool(mfwf_server s, Pool &P, const std::string &err);

// Retire the finished iterations at the head of a lane: each one's measured duration updates
// its pool's cost for that slot count.
static void reap_lane(mfwf_server s, Lane &L) {
    while (!L.inflight.empty()) {
        Launch &x = L.inflight.front();
        const hipError_t e = hipEventQuery(x.t1);
        if (e == hipErrorNotReady) break;
        float ms = 0.f;
        if (e == hipSuccess && hipEventElapsedTime(&ms, x.t0, x.t1) == hipSuccess && ms > 0.f) {
            auto it = x.pool->cost_ms.find(x.nb);
            if (it == x.pool->cost_ms.end())
                x.pool->cost_ms[x.nb] = ms;
            else
                it->second = 0.7 * it->second + 0.3 * ms;
        }
        if (e != hipSuccess) fail_pool(s, *x.pool, hipGetErrorString(e));
        s->spare_events.push_back(x.t0);
        s->spare_events.push_back(x.t1);
        L.inflight.pop_front();
    }
}

static Pool *find_or_create_pool(mfwf_server s, const PoolKey &key, std::string &err, int &status) {
    for (auto &P : s->pools)
        if (P->key == key) return P.get();
    // slots: the server's count, halved while the pool would take more than half the budget
    // (large shapes, e.g. FP64 at nside 2048, whose Legendre partial sums grow with the slots)
    int nslots = s->slots;
    while (nslots > 1 && estimate_pool_bytes(key.nside, key.lmax, key.dtype, nslots) > s->budget / 2)
        nslots /= 2;
    const size_t need = estimate_pool_bytes(key.nside, key.lmax, key.dtype, nslots);
    if (need > s->budget) {
        status = MFWF_ENOMEM;
        err = "a pool of this shape exceeds the server's HBM budget";
        return nullptr;
    }
    while (s->used + need > s->budget) {  // evict the least recently used idle pool
        int victim = -1;
        for (size_t i = 0; i < s->pools.size(); i++) {
            Pool &Q = *s->pools[i];
            if (Q.active == 0 && (victim < 0 || Q.last_used < s->pools[victim]->last_used)) victim = (int)i;
        }
        if (victim < 0) {
            // no idle pool to evict: the least recently used pools that would make room stop
            // admitting requests, so that they drain and the blocked request is served next
            // (otherwise steady arrivals for existing pools could hold it back without bound)
            std::vector<Pool *> order;
            for (auto &Q : s->pools) order.push_back(Q.get());
            std::sort(order.begin(), order.end(),
                      [](const Pool *a, const Pool *b) { return a->last_used < b->last_used; });
            size_t freed = 0;
            for (Pool *Q : order) {
                if (s->used - freed + need <= s->budget) break;
                Q->draining = true;
                freed += Q->bytes;
            }
            return nullptr;  // wait for slots to drain
        }
        // drain the victim's lane so that no launch record refers to it any more
        Lane &L = s->lanes[s->pools[victim]->lane];
        (void)hipStreamSynchronize(L.stream);
        reap_lane(s, L);
        s->used -= s->pools[victim]->bytes;
        s->pools.erase(s->pools.begin() + victim);
        std::lock_guard<std::mutex> lk(s->mu);
        s->stat[7] += 1;
        s->stat[3] = (double)s->pools.size();
        s->stat[4] = (double)s->used;
    }
    for (auto &Q : s->pools) Q->draining = false;  // room made: admission as usual again
    std::unique_ptr<Pool> P(new Pool());
    P->key = key;
    // the lane with the least static load (maps x pixels x l per slot, FP64 counted twice)
    P->weight = (double)key.nside * key.nside * key.lmax * (key.dtype == MFWF_F64 ? 2.0 : 1.0);
    double load[kLanes] = {};
    for (auto &Q : s->pools) load[Q->lane] += Q->weight;
    for (int l = 1; l < kLanes; l++)
        if (load[l] < load[P->lane]) P->lane = l;
    hipStream_t st = s->lanes[P->lane].stream;
    P->plan.stream = st;
    P->plan_ok = true;  // free whatever a failed creation allocated
    P->nslots = nslots;
    status = plan_create(key.nside, key.lmax, 0, key.dtype, nslots, st, true, P->plan);
    if (status == MFWF_OK) status = plan_set_cl(P->plan, key.cl.data());
    if (status == MFWF_OK && key.dtype == MFWF_F32) {
        // FP32 pools chain their iterations as a standalone solve does: each iteration's ring
        // step starts from the previous synthesis in the columns (zero for a new slot), and
        // the maps are formed only when a request retires
        Plan &p = P->plan;
        status = launch_fill(reinterpret_cast<double *>(p.d_ph32), (long)p.nring * p.nm * p.C2 / 2,
                             0.0, p.stream);
        p.chain = p.chain_ready = true;
    }
    if (status != MFWF_OK) {
        err = std::string("pool plan: ") + mfwf_last_error();
        return nullptr;
    }
    P->slot.assign(nslots, nullptr);
    P->done_iters.assign(nslots, 0);
    P->bytes = need;
    P->last_used = Clock::now();
    s->used += need;
    s->pools.push_back(std::move(P));
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stat[6] += 1;
        s->stat[3] = (double)s->pools.size();
        s->stat[4] = (double)s->used;
    }
    return s->pools.back().get();
}

static void fail_pool(mfwf_server s, Pool &P, const std::string &err) {
    for (auto &q : P.slot)
        if (q) finish_request(s, q, MFWF_EDEVICE, err);
    for (auto &q : P.slot) q.reset();
    P.active = 0;
}

static void worker_main(mfwf_server s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            bool busy = !s->pending.empty() || !s->finishing.empty();
            for (auto &P : s->pools) busy = busy || P->active > 0;
            if (!busy && s->queue.empty()) {
                if (s->stop) break;
                s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
                continue;
            }
            while (!s->queue.empty()) {
                s->pending.push_back(s->queue.front());
                s->queue.pop_front();
            }
        }
        // admission at the iteration boundary, first come first served per pool
        for (auto it = s->pending.begin(); it != s->pending.end();) {
            std::shared_ptr<SrvRequest> q = *it;
            PoolKey key{q->r.nside, q->r.lmax, q->r.dtype, q->r.lambda, q->cl};
            std::string err;
            int st = MFWF_OK;
            Pool *P = find_or_create_pool(s, key, err, st);
            if (!P) {
                if (st != MFWF_OK) {
                    finish_request(s, q, st, err);
                    it = s->pending.erase(it);
                } else {
                    ++it;
                }
                continue;
            }
            int b = -1;
            for (int k = 0; k < P->nslots && b < 0 && !P->draining; k++)
                if (!P->slot[k]) b = k;
            if (b < 0) {
                ++it;
                continue;
            }
            st = admit(s, *P, b, q);
            if (st != MFWF_OK) {
                finish_request(s, q, st, mfwf_last_error());
            }
            it = s->pending.erase(it);
        }
        // Fill every lane up to kLaneDepth iterations, each time with the busy pool of that
        // lane that has been charged the least GPU time.
        bool launched = false;
        for (int l = 0; l < kLanes; l++) {
            Lane &L = s->lanes[l];
            reap_lane(s, L);
            while ((int)L.inflight.size() < kLaneDepth) {
                Pool *best = nullptr;
                for (auto &Q : s->pools)
                    if (Q->lane == l && Q->active > 0 && (!best || Q->vtime < best->vtime)) best = Q.get();
                if (!best) break;
                Pool &P = *best;
                int nb = 0;
                for (int k = 0; k < P.nslots; k++)
                    if (P.slot[k]) nb = k + 1;
                hipGraphExec_t exec = nullptr;
                int st = pool_graph(P, nb, exec);
                Launch x{&P, nb, take_event(s), take_event(s)};
                if (st == MFWF_OK && (!x.t0 || !x.t1))
                    st = fail(MFWF_EDEVICE, "event creation failed");
                if (st == MFWF_OK && (hipEventRecord(x.t0, L.stream) != hipSuccess ||
                                      hipGraphLaunch(exec, L.stream) != hipSuccess ||
                                      hipEventRecord(x.t1, L.stream) != hipSuccess))
                    st = fail(MFWF_EDEVICE, "graph launch failed");
                if (st != MFWF_OK) {
                    if (x.t0) s->spare_events.push_back(x.t0);
                    if (x.t1) s->spare_events.push_back(x.t1);
                    fail_pool(s, P, mfwf_last_error());
                    continue;
                }
                L.inflight.push_back(x);
                launched = true;
                P.vtime += P.est_cost(nb);
                P.last_used = Clock::now();
                bool any_retire = false;
                for (int k = 0; k < nb; k++)
                    if (P.slot[k] && ++P.done_iters[k] >= P.slot[k]->r.iters) any_retire = true;
                if (any_retire) {
                    st = plan_finish_alm(P.plan, nb);
                    for (int k = 0; k < nb && st == MFWF_OK; k++)
                        if (P.slot[k] && P.done_iters[k] >= P.slot[k]->r.iters) st = retire(s, P, k);
                    if (st != MFWF_OK) fail_pool(s, P, mfwf_last_error());
                }
                int act = 0;
                for (auto &Q : s->pools) act += Q->active;
                std::lock_guard<std::mutex> lk(s->mu);
                s->stat[5] += 1;
                s->stat[2] = act;
            }
        }
        // completed copies
        for (size_t i = 0; i < s->finishing.size();) {
            hipError_t e = hipEventQuery(s->finishing[i].ev);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            (void)hipEventDestroy(s->finishing[i].ev);
            finish_request(s, s->finishing[i].req, e == hipSuccess ? MFWF_OK : MFWF_EDEVICE,
                           e == hipSuccess ? "" : hipGetErrorString(e));
            s->finishing.erase(s->finishing.begin() + i);
        }
        // nothing launched: every lane with busy pools holds kLaneDepth iterations, or only
        // result copies are outstanding
        if (!launched) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (auto &L : s->lanes) {
        (void)hipStreamSynchronize(L.stream);
        reap_lane(s, L);
    }
    s->pools.clear();
}

}  // namespace mfwf

// device resources of a server whose worker has stopped (or never started)
static void release(mfwf_server s) {
    if (s->vscratch) (void)hipFree(s->vscratch);
    if (s->vpart) (void)hipFree(s->vpart);
    if (s->vout) (void)hipFree(s->vout);
    if (s->vstream) (void)hipStreamDestroy(s->vstream);
    for (auto &L : s->lanes)
        if (L.stream) (void)hipStreamDestroy(L.stream);
    for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
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
    bool ok = hipGetDevice(&s->device) == hipSuccess &&
              hipStreamCreateWithFlags(&s->vstream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc((void **)&s->vpart, sizeof(double) * 3 * 1024) == hipSuccess &&
              hipMalloc((void **)&s->vout, sizeof(double) * 8) == hipSuccess;
    for (auto &L : s->lanes)
        ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
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
