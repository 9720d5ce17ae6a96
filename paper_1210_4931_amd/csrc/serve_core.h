// Scheduling core of the serving runtime, free of any device call: requests of one shape
// (nside, lmax, dtype, lambda, C_l) share a pool with a fixed number of map slots; requests
// are admitted into free slots first come, first served per pool at iteration boundaries;
// pools run on a few lanes, where the busy pool with the least GPU time so far (start-time
// fair queueing on each iteration's measured duration) launches next; a pool is created when
// its footprint fits the memory budget, idle pools are evicted least recently used first, and
// when none is idle the pools that would make room stop admitting until they drain.
//
// The device work goes through a backend B (the HIP backend of the server; a simulated one in
// the CPU tests), which provides
//   types   Request, PoolState, LaneState, Timer (one launched iteration), Done (one retired
//           request's result copies)
//   Key  key_of(const Request &);            int iters_of(const Request &);
//   size_t pool_bytes(const Key &, int slots);
//   int  create(PoolState &, const Key &, int slots, LaneState &, std::string &err);
//   void destroy(PoolState &);
//   int  admit(PoolState &, int slot, Request &);
//   int  launch(PoolState &, int nb, LaneState &, Timer &, std::string &err);
//   int  poll(Timer &, bool &done, double &ms, std::string &err);   void recycle(Timer &);
//   int  finish(PoolState &, int nb);
//   int  retire(PoolState &, int slot, Request &, Done &);
//   int  poll_done(Done &, bool &done, std::string &err);
//   void sync(LaneState &);
//   void complete(const std::shared_ptr<Request> &, int status, const std::string &err);
//   void publish(const Stats &);              std::string last_error();
// and the status codes of mfwf.h.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "mfwf.h"

namespace mfwf {
namespace serve {

// Lanes: streams the worker schedules pools onto.  The process has few hardware queues (4
// by default) and streams beyond them share queues in FIFO order, so the server keeps its
// own small number of streams and orders the work on each itself.
static constexpr int kLanes = 2;
// iterations in flight per lane (host run-ahead bound)
static constexpr int kLaneDepth = 4;

struct Key {
    int nside, lmax, dtype;
    double lam;
    std::vector<double> cl;
    bool operator<(const Key &o) const {
        return std::tie(nside, lmax, dtype, lam, cl) < std::tie(o.nside, o.lmax, o.dtype, o.lam, o.cl);
    }
    bool operator==(const Key &o) const { return !(*this < o) && !(o < *this); }
};

// completed requests, occupied slots, pools, bytes charged, iterations launched, pools
// created, pools evicted
struct Stats {
    double completed = 0, occupied = 0, pools = 0, bytes = 0, iterations = 0, created = 0, evicted = 0;
};

template <class B>
class Core {
  public:
    using Req = typename B::Request;

    struct Pool {
        Key key;
        typename B::PoolState st{};
        std::vector<std::shared_ptr<Req>> slot;
        std::vector<int> done_iters;
        size_t bytes = 0;
        int active = 0;
        uint64_t last_used = 0;          // tick of the last launch or creation
        int lane = 0;                    // lane whose stream the pool's work goes to
        double weight = 0.0;             // static cost guess used to balance pools over lanes
        double vtime = 0.0;              // GPU milliseconds charged to this pool
        std::map<int, double> cost_ms;   // measured iteration time by slot count (moving average)
        int nslots = 0;                  // map slots (the server's, or fewer for large shapes)
        bool draining = false;           // admits no new request: a blocked new pool needs room

        // expected milliseconds of one iteration over nb slots
        double est_cost(int nb) const {
            if (cost_ms.empty()) return 1.0;
            auto it = cost_ms.lower_bound(nb);
            if (it != cost_ms.end() && it->first == nb) return it->second;
            if (it == cost_ms.end()) --it;  // nearest measured slot count, scaled linearly
            return it->second * (double)nb / (double)it->first;
        }
    };
    struct Launch {
        Pool *pool;
        int nb;
        typename B::Timer t;
    };
    struct Lane {
        typename B::LaneState st{};
        std::deque<Launch> inflight;
    };
    struct Finishing {
        std::shared_ptr<Req> req;
        typename B::Done tok;
    };

    Core(B &be, int slots, size_t budget) : be_(be), slots_(slots), budget_(budget) {}
    Core(const Core &) = delete;
    Core &operator=(const Core &) = delete;

    Lane lanes[kLanes];

    void add(std::shared_ptr<Req> q) { pending_.push_back(std::move(q)); }

    bool busy() const {
        if (!pending_.empty() || !finishing_.empty()) return true;
        for (auto &P : pools_)
            if (P->active > 0) return true;
        return false;
    }

    // One pass of the worker: admission at the iteration boundary, launches up to the lane
    // depth, completed result copies.  Returns whether anything was launched.
    bool step() {
        admit_pending();
        bool launched = false;
        for (int l = 0; l < kLanes; l++) launched |= fill_lane(l);
        for (size_t i = 0; i < finishing_.size();) {
            bool done = false;
            std::string err;
            const int st = be_.poll_done(finishing_[i].tok, done, err);
            if (!done && st == MFWF_OK) {
                ++i;
                continue;
            }
            be_.complete(finishing_[i].req, st, err);
            finishing_.erase(finishing_.begin() + i);
        }
        return launched;
    }

    // Wait for every lane, then release every pool.
    void shutdown() {
        for (auto &L : lanes) {
            be_.sync(L.st);
            reap(L);
        }
        for (auto &P : pools_) be_.destroy(P->st);
        pools_.clear();
    }

    size_t used() const { return used_; }

  private:
    B &be_;
    int slots_;
    size_t budget_, used_ = 0;
    uint64_t tick_ = 0;
    Stats stats_;
    std::deque<std::shared_ptr<Req>> pending_;
    std::vector<std::unique_ptr<Pool>> pools_;
    std::vector<Finishing> finishing_;

    void publish() {
        stats_.pools = (double)pools_.size();
        stats_.bytes = (double)used_;
        int act = 0;
        for (auto &P : pools_) act += P->active;
        stats_.occupied = act;
        be_.publish(stats_);
    }

    void admit_pending() {
        for (auto it = pending_.begin(); it != pending_.end();) {
            std::shared_ptr<Req> q = *it;
            std::string err;
            int st = MFWF_OK;
            Pool *P = find_or_create(be_.key_of(*q), err, st);
            if (!P) {
                if (st != MFWF_OK) {
                    be_.complete(q, st, err);
                    it = pending_.erase(it);
                } else {
                    ++it;  // waits for room
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
            if (P->active == 0) {
                // a pool that wakes up joins at the least GPU time of the busy pools on its
                // lane, so that time it spent idle is not credited to it
                double vmin = -1.0;
                for (auto &Q : pools_)
                    if (Q.get() != P && Q->lane == P->lane && Q->active > 0 && (vmin < 0.0 || Q->vtime < vmin))
                        vmin = Q->vtime;
                if (vmin > P->vtime) P->vtime = vmin;
            }
            st = be_.admit(P->st, b, *q);
            if (st != MFWF_OK) {
                be_.complete(q, st, be_.last_error());
            } else {
                P->slot[b] = q;
                P->done_iters[b] = 0;
                P->active++;
            }
            it = pending_.erase(it);
        }
    }

    Pool *find_or_create(const Key &key, std::string &err, int &status) {
        for (auto &P : pools_)
            if (P->key == key) return P.get();
        // slots: the server's count, halved while the pool would take more than half the
        // budget (large shapes, whose per-slot arrays are large)
        int nslots = slots_;
        while (nslots > 1 && be_.pool_bytes(key, nslots) > budget_ / 2) nslots /= 2;
        const size_t need = be_.pool_bytes(key, nslots);
        if (need > budget_) {
            status = MFWF_ENOMEM;
            err = "a pool of this shape exceeds the server's HBM budget";
            return nullptr;
        }
        while (used_ + need > budget_) {  // evict the least recently used idle pool
            int victim = -1;
            for (size_t i = 0; i < pools_.size(); i++) {
                Pool &Q = *pools_[i];
                if (Q.active == 0 && (victim < 0 || Q.last_used < pools_[victim]->last_used)) victim = (int)i;
            }
            if (victim < 0) {
                // no idle pool to evict: the least recently used pools that would make room
                // stop admitting requests, so that they drain and the blocked request is
                // served next (steady arrivals for existing pools cannot hold it back)
                std::vector<Pool *> order;
                for (auto &Q : pools_) order.push_back(Q.get());
                std::sort(order.begin(), order.end(),
                          [](const Pool *a, const Pool *b) { return a->last_used < b->last_used; });
                size_t freed = 0;
                for (Pool *Q : order) {
                    if (used_ - freed + need <= budget_) break;
                    Q->draining = true;
                    freed += Q->bytes;
                }
                return nullptr;
            }
            // drain the victim's lane so that no launch record refers to it any more
            Lane &L = lanes[pools_[victim]->lane];
            be_.sync(L.st);
            reap(L);
            used_ -= pools_[victim]->bytes;
            be_.destroy(pools_[victim]->st);
            pools_.erase(pools_.begin() + victim);
            stats_.evicted += 1;
            publish();
        }
        for (auto &Q : pools_) Q->draining = false;  // room made: admission as usual again
        std::unique_ptr<Pool> P(new Pool());
        P->key = key;
        // the lane with the least static load (maps x pixels x l per slot, FP64 counted twice)
        P->weight = (double)key.nside * key.nside * key.lmax * (key.dtype == MFWF_F64 ? 2.0 : 1.0);
        double load[kLanes] = {};
        for (auto &Q : pools_) load[Q->lane] += Q->weight;
        for (int l = 1; l < kLanes; l++)
            if (load[l] < load[P->lane]) P->lane = l;
        P->nslots = nslots;
        status = be_.create(P->st, key, nslots, lanes[P->lane].st, err);
        if (status != MFWF_OK) {
            be_.destroy(P->st);  // whatever the failed creation allocated
            return nullptr;
        }
        P->slot.assign(nslots, nullptr);
        P->done_iters.assign(nslots, 0);
        P->bytes = need;
        P->last_used = ++tick_;
        used_ += need;
        pools_.push_back(std::move(P));
        stats_.created += 1;
        publish();
        return pools_.back().get();
    }

    void fail_pool(Pool &P, const std::string &err) {
        for (auto &q : P.slot)
            if (q) be_.complete(q, MFWF_EDEVICE, err);
        for (auto &q : P.slot) q.reset();
        P.active = 0;
    }

    // Retire the finished iterations at the head of a lane: each one's measured duration
    // updates its pool's cost for that slot count.
    void reap(Lane &L) {
        while (!L.inflight.empty()) {
            Launch &x = L.inflight.front();
            bool done = false;
            double ms = 0.0;
            std::string err;
            const int st = be_.poll(x.t, done, ms, err);
            if (st == MFWF_OK && !done) break;
            if (st == MFWF_OK && ms > 0.0) {
                auto it = x.pool->cost_ms.find(x.nb);
                if (it == x.pool->cost_ms.end())
                    x.pool->cost_ms[x.nb] = ms;
                else
                    it->second = 0.7 * it->second + 0.3 * ms;
            }
            if (st != MFWF_OK) fail_pool(*x.pool, err);
            be_.recycle(x.t);
            L.inflight.pop_front();
        }
    }

    // Fill lane l up to kLaneDepth iterations, each time with its busy pool that has been
    // charged the least GPU time.
    bool fill_lane(int l) {
        Lane &L = lanes[l];
        reap(L);
        bool launched = false;
        while ((int)L.inflight.size() < kLaneDepth) {
            Pool *best = nullptr;
            for (auto &Q : pools_)
                if (Q->lane == l && Q->active > 0 && (!best || Q->vtime < best->vtime)) best = Q.get();
            if (!best) break;
            Pool &P = *best;
            int nb = 0;
            for (int k = 0; k < P.nslots; k++)
                if (P.slot[k]) nb = k + 1;
            Launch x{&P, nb, {}};
            std::string err;
            if (be_.launch(P.st, nb, L.st, x.t, err) != MFWF_OK) {
                fail_pool(P, err);
                continue;
            }
            L.inflight.push_back(x);
            launched = true;
            P.vtime += P.est_cost(nb);
            P.last_used = ++tick_;
            bool any_retire = false;
            for (int k = 0; k < nb; k++)
                if (P.slot[k] && ++P.done_iters[k] >= be_.iters_of(*P.slot[k])) any_retire = true;
            if (any_retire) {
                int st = be_.finish(P.st, nb);
                for (int k = 0; k < nb && st == MFWF_OK; k++)
                    if (P.slot[k] && P.done_iters[k] >= be_.iters_of(*P.slot[k])) {
                        Finishing f{P.slot[k], {}};
                        st = be_.retire(P.st, k, *P.slot[k], f.tok);
                        if (st == MFWF_OK) {
                            finishing_.push_back(f);
                            P.slot[k].reset();
                            P.active--;
                        }
                    }
                if (st != MFWF_OK) fail_pool(P, be_.last_error());
            }
            stats_.iterations += 1;
            publish();
        }
        return launched;
    }
};

}  // namespace serve
}  // namespace mfwf
