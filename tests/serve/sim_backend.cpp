// CPU simulation of the serving runtime: the scheduling core of the server (serve_core.h,
// the same code the HIP server runs) driven with a simulated device.  Each lane executes
// its launched iterations one after another; an iteration over nb slots of a pool costs
// cost(nside, dtype, nb) milliseconds of simulated time; pool creation, admission and result
// copies take none.  A fake clock advances from event to event.  Reads a scenario on stdin
// and prints one JSON line with every request's arrival, completion and status, and the
// core's statistics.
//
// Scenario: first line "slots budget_bytes", then one request per line
//   "arrival_ms nside lmax dtype iters"   (dtype 0 = FP64, 1 = FP32, as in mfwf.h)
// Pool footprint: bytes_per_slot(nside) x slots, bytes_per_slot = nside^2 x 1e4.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <iostream>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "serve_core.h"

using namespace mfwf;

struct Sim;

struct SimRequest {
    int id = 0, nside = 0, lmax = 0, dtype = 0, iters = 0;
    double arrival = 0.0, done_at = -1.0;
    int status = -100;
};

struct SimBackend {
    using Request = SimRequest;
    struct PoolState {
        int nside = 0, dtype = 0;
        int lane = -1;
    };
    using LaneState = int;          // lane index
    struct Timer {
        double end = 0.0, ms = 0.0;
    };
    struct Done {
        double at = 0.0;
    };

    double now = 0.0;
    double lane_free[serve::kLanes] = {0.0, 0.0};  // simulated time each lane's queue drains
    std::vector<double> events;                    // ends of launched iterations and copies
    std::vector<SimRequest *> completed;
    serve::Stats stats;
    int creates = 0, destroys = 0;
    double peak_bytes = 0.0;

    static double cost(int nside, int dtype, int nb) {
        // a fixed part plus a part per slot, FP64 twice FP32
        return 1e-5 * nside * nside * (dtype == MFWF_F64 ? 2.0 : 1.0) * (1.0 + 0.25 * nb);
    }

    serve::Key key_of(const Request &q) const { return serve::Key{q.nside, q.lmax, q.dtype, 1.0, {}}; }
    int iters_of(const Request &q) const { return q.iters; }
    size_t pool_bytes(const serve::Key &k, int slots) const {
        return (size_t)(1e4 * k.nside * k.nside) * (size_t)slots;
    }
    std::string last_error() const { return "simulated"; }
    int create(PoolState &P, const serve::Key &k, int, LaneState &lane, std::string &) {
        P.nside = k.nside;
        P.dtype = k.dtype;
        P.lane = lane;
        creates++;
        return MFWF_OK;
    }
    void destroy(PoolState &) { destroys++; }
    int admit(PoolState &, int, Request &) { return MFWF_OK; }
    int launch(PoolState &P, int nb, LaneState &lane, Timer &t, std::string &) {
        t.ms = cost(P.nside, P.dtype, nb);
        lane_free[lane] = std::max(lane_free[lane], now) + t.ms;
        t.end = lane_free[lane];
        events.push_back(t.end);
        return MFWF_OK;
    }
    int poll(Timer &t, bool &done, double &ms, std::string &) {
        done = now >= t.end;
        ms = t.ms;
        return MFWF_OK;
    }
    void recycle(Timer &) {}
    int finish(PoolState &, int) { return MFWF_OK; }
    int retire(PoolState &P, int, Request &, Done &d) {
        d.at = lane_free[P.lane];  // after the pool's queued work
        events.push_back(d.at);
        return MFWF_OK;
    }
    int poll_done(Done &d, bool &done, std::string &) {
        done = now >= d.at;
        return MFWF_OK;
    }
    void sync(LaneState &lane) { now = std::max(now, lane_free[lane]); }
    void complete(const std::shared_ptr<Request> &q, int status, const std::string &) {
        q->status = status;
        q->done_at = now;
        completed.push_back(q.get());
    }
    void publish(const serve::Stats &st) {
        stats = st;
        peak_bytes = std::max(peak_bytes, st.bytes);
    }
};

int main() {
    int slots = 0;
    double budget = 0.0;
    std::cin >> slots >> budget;
    std::vector<std::shared_ptr<SimRequest>> reqs;
    double a;
    int n, l, d, k;
    while (std::cin >> a >> n >> l >> d >> k) {
        auto q = std::make_shared<SimRequest>();
        q->id = (int)reqs.size();
        q->arrival = a;
        q->nside = n;
        q->lmax = l;
        q->dtype = d;
        q->iters = k;
        reqs.push_back(q);
    }
    SimBackend be;
    serve::Core<SimBackend> core(be, slots, (size_t)budget);
    for (int i = 0; i < serve::kLanes; i++) core.lanes[i].st = i;
    size_t next = 0;
    long steps = 0;
    while (be.completed.size() < reqs.size() && steps < 50000000) {
        steps++;
        while (next < reqs.size() && reqs[next]->arrival <= be.now) core.add(reqs[next++]);
        const bool launched = core.step();
        if (launched) continue;
        // nothing to launch now: advance the clock to the next event (an iteration or a copy
        // finishing, or an arrival)
        double t = std::numeric_limits<double>::infinity();
        for (double f : be.events)
            if (f > be.now) t = std::min(t, f);
        be.events.erase(std::remove_if(be.events.begin(), be.events.end(),
                                       [&](double f) { return f <= be.now; }),
                        be.events.end());
        if (next < reqs.size()) t = std::min(t, reqs[next]->arrival);
        if (!std::isfinite(t)) {
            if (!core.busy() && next >= reqs.size()) break;
            t = be.now + 1e-3;
        }
        be.now = std::max(t, be.now + 1e-9);
    }
    core.shutdown();
    std::printf("{\"requests\": [");
    for (size_t i = 0; i < reqs.size(); i++)
        std::printf("%s[%d, %.6f, %.6f, %d, %d, %d]", i ? ", " : "", reqs[i]->nside, reqs[i]->arrival,
                    reqs[i]->done_at, reqs[i]->status, reqs[i]->dtype, reqs[i]->iters);
    std::printf("], \"created\": %d, \"destroyed\": %d, \"evicted\": %.0f, \"peak_bytes\": %.0f, "
                "\"iterations\": %.0f, \"end_ms\": %.6f}\n",
                be.creates, be.destroys, be.stats.evicted, be.peak_bytes, be.stats.iterations, be.now);
    return 0;
}
