// Serving: continuous batching of reconstructions of uneven grid and point
// counts (wg_server_* / wg_submit / wg_poll in include/wgeo.h).
//
// Requests queue in arrival order.  max_inflight worker threads each take the
// next request as soon as they are free, so requests that arrive while others
// run are admitted the moment a slot and device memory allow.  A request runs
// on a reconstruction handle taken from a pool of idle handles keyed by grid
// geometry and point capacity: grids and solver state stay resident between
// requests of the same size class.  Creating a handle is admitted only if the
// bytes of all resident handles stay within the HBM budget; idle handles of
// other classes are evicted (least recently used first) to make room, and a
// worker waits when everything resident is busy.  Every handle owns its own
// HIP stream, so the kernels of concurrent requests overlap on the device; a
// request that starts alone, or fills the device (below), runs its distance
// walk persistent, one that starts beside others runs it as independent
// workgroups (see run()).
//
// A request whose grid alone keeps every compute unit busy (kFillCells cells
// or more) gains nothing from overlapping another such request's same phase:
// both would just take twice as long.  Such requests take turns (all sizes
// from kFillCells up share one turn: a 128^3 request beside a 256^3 one slowed
// both); while one holds the turn, a free worker takes the first queued
// request that is smaller, so the large ones keep their arrival order and the
// small ones fill the gaps.  When another large request is queued as one
// starts, the turn ends once its distance walk is enqueued: the walk
// (ALU-bound) runs on the handle's second stream with workgroup slots left
// free on every compute unit, and the next request bins, splats and solves
// (bandwidth-bound) beside it, as consecutive steps of a moving-boundary loop
// do.  Without a successor, for a request with a reverse pass (whose adjoint
// solve would meet the next one's solve), and on a server with one worker
// (where nothing could use the free slots), the walk keeps the whole device
// and the turn lasts to the end.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>

#include "recon.h"

namespace wg {

namespace {

struct Key {
    int n[3];
    double lo[3], h;
    int cap;
    bool operator<(const Key &o) const {
        return std::tie(n[0], n[1], n[2], lo[0], lo[1], lo[2], h, cap) <
               std::tie(o.n[0], o.n[1], o.n[2], o.lo[0], o.lo[1], o.lo[2], o.h, o.cap);
    }
};

// 2^21 cells (128^3) or more: a distance walk of 32768 tiles or more (64-node
// tiles below 2^23 cells, 256-node ones from there), several times the
// wavefronts the device holds at once.  Two such walks only queue behind each
// other and the solves beside them wait for slots: a stream of 128^3 requests
// alone, served four at a time, ran at 0.77x the rate of one at a time while
// only 2^23 cells and more took turns, and at 1.20x once 128^3 ones did too.
constexpr size_t kFillCells = size_t(1) << 21;

bool fills_device(const wg_grid &g) { return (size_t)g.n[0] * g.n[1] * g.n[2] >= kFillCells; }

int capacity_class(int npts) {
    int c = 1 << 14;
    while (c < npts) c <<= 1;
    return c;
}

struct Handle {
    Recon *r = nullptr;
    hipStream_t s = nullptr;
    size_t bytes = 0;
    Key key{};
    uint64_t last_use = 0;
};

struct Buf {
    float *p = nullptr;
    size_t cap = 0;   // floats
};

struct Job {
    uint64_t ticket = 0;
    wg_request req{};
    Buf in[5];   // server-owned copies: points, normals, queries, dL/dphi, dL/dn(q)
    float *xyz = nullptr, *nrm = nullptr, *q = nullptr, *gphi = nullptr, *gnrm = nullptr;   // in[k].p
    int state = 0;   // 0 queued, 1 running, 2 done
    wg_result res{};
};

}  // namespace

class Server {
  public:
    Server(size_t budget, int max_inflight, int device)
        : budget_(budget), device_(device), inflight_(max_inflight) {
        WG_HIP(hipSetDevice(device_));
        WG_HIP(hipStreamCreateWithFlags(&ingest_, hipStreamNonBlocking));
        t0_ = std::chrono::steady_clock::now();
        for (int k = 0; k < max_inflight; ++k) workers_.emplace_back([this] { worker(); });
    }

    ~Server() {
        {
            std::unique_lock<std::mutex> lk(mu_);
            drain_cv_.wait(lk, [this] { return queue_.empty() && running_ == 0; });
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
        (void)hipSetDevice(device_);
        for (auto &h : idle_) destroy(h);
        for (auto &kv : jobs_) free_inputs(*kv.second);
        for (auto &kv : pool_) (void)hipFree(kv.second);
        (void)hipStreamDestroy(ingest_);
    }

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
    }

    int submit(const wg_request &rq, uint64_t *ticket) {
        require(ticket != nullptr, WG_EINVAL, "null ticket");
        require(rq.n_points >= 0 && rq.n_q >= 0, WG_EINVAL, "negative sizes");
        require(rq.n_points == 0 || (rq.d_xyz && rq.d_nrm), WG_EINVAL, "null point inputs");
        require(rq.n_q == 0 || (rq.d_q && rq.d_phi), WG_EINVAL, "null query arguments");
        require(!rq.d_gphi || rq.n_points == 0 || (rq.d_gxyz && rq.d_gnrm_pts), WG_EINVAL, "null gradient outputs");
        require(rq.d_gphi || (!rq.d_gnrm && !rq.d_gq), WG_EINVAL, "query-side gradients need d_gphi");
        const size_t fp = Recon::footprint(rq.grid, capacity_class(rq.n_points));
        require(fp <= budget_, WG_ENOMEM, "request footprint exceeds the server budget");
        WG_HIP(hipSetDevice(device_));
        auto job = std::make_unique<Job>();
        job->req = rq;
        job->res.t_submit = now();
        auto copy = [&](int k, const float *src, size_t n) -> float * {
            if (!src || n == 0) return nullptr;
            job->in[k] = take_buf(n);
            WG_HIP(hipMemcpyAsync(job->in[k].p, src, n * sizeof(float), hipMemcpyDeviceToDevice, ingest_));
            return job->in[k].p;
        };
        try {
            job->xyz = copy(0, rq.d_xyz, 3 * (size_t)rq.n_points);
            job->nrm = copy(1, rq.d_nrm, 3 * (size_t)rq.n_points);
            job->q = copy(2, rq.d_q, 3 * (size_t)rq.n_q);
            job->gphi = copy(3, rq.d_gphi, (size_t)rq.n_q);
            job->gnrm = copy(4, rq.d_gnrm, 3 * (size_t)rq.n_q);
            WG_HIP(hipStreamSynchronize(ingest_));
        } catch (...) {
            (void)hipStreamSynchronize(ingest_);
            free_inputs(*job);
            throw;
        }
        std::unique_lock<std::mutex> lk(mu_);
        job->ticket = ++next_ticket_;
        *ticket = job->ticket;
        Job *j = job.get();
        jobs_[j->ticket] = std::move(job);
        queue_.push_back(j);
        lk.unlock();
        cv_.notify_one();
        return WG_OK;
    }

    int poll(uint64_t ticket, wg_result *out) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = jobs_.find(ticket);
        require(it != jobs_.end(), WG_ESTATE, "unknown ticket");
        Job &j = *it->second;
        if (j.state != 2) return WG_PENDING;
        if (out) *out = j.res;
        int st = j.res.status;
        std::unique_ptr<Job> owned = std::move(it->second);
        jobs_.erase(it);
        lk.unlock();
        free_inputs(*owned);
        return st;
    }

  private:
    // Input copies live in buffers that are reused, never freed while the
    // server runs: hipFree waits for the whole device, so freeing at poll
    // would hold the caller until every running request's kernels finish.
    // Capacities are powers of two; the pool's size is bounded by the most
    // requests ever outstanding at once.
    Buf take_buf(size_t n) {
        {
            std::lock_guard<std::mutex> lk(pool_mu_);
            auto it = pool_.lower_bound(n);
            if (it != pool_.end()) {
                Buf b{it->second, it->first};
                pool_.erase(it);
                return b;
            }
        }
        Buf b;
        b.cap = 1024;
        while (b.cap < n) b.cap <<= 1;
        WG_HIP(hipMalloc(&b.p, b.cap * sizeof(float)));
        return b;
    }

    void free_inputs(Job &j) {
        std::lock_guard<std::mutex> lk(pool_mu_);
        for (Buf &b : j.in)
            if (b.p) pool_.emplace(b.cap, b.p);
        for (Buf &b : j.in) b = Buf{};
        j.xyz = j.nrm = j.q = j.gphi = j.gnrm = nullptr;
    }

    void destroy(Handle &h) {
        if (h.s) (void)hipStreamSynchronize(h.s);
        delete h.r;
        if (h.s) (void)hipStreamDestroy(h.s);
        h.r = nullptr;
        h.s = nullptr;
    }

    // Evict least-recently-used idle handles until `need` more bytes fit in
    // the budget (or nothing idle is left).  Called with lk held.
    void evict_for(size_t need, std::unique_lock<std::mutex> &lk) {
        while (resident_ + need > budget_ && !idle_.empty()) {
            auto victim = idle_.begin();
            for (auto it = idle_.begin(); it != idle_.end(); ++it)
                if (it->last_use < victim->last_use) victim = it;
            Handle h = *victim;
            idle_.erase(victim);
            resident_ -= h.bytes;
            lk.unlock();
            destroy(h);
            lk.lock();
        }
    }

    // A running handle's surface buffers are about to grow by `extra` bytes
    // (a mesh larger than its footprint allowed for): charge them to the
    // budget first, evicting idle handles if needed, or refuse.
    void reserve_growth(Handle &h, size_t extra) {
        std::unique_lock<std::mutex> lk(mu_);
        evict_for(extra, lk);
        require(resident_ + extra <= budget_, WG_ENOMEM, "surface growth exceeds the server budget");
        resident_ += extra;
        h.bytes += extra;
    }

    // Take an idle handle of this class or create one within the budget.
    Handle acquire(const Key &k, const wg_grid &g, std::unique_lock<std::mutex> &lk) {
        const size_t fp = Recon::footprint(g, k.cap);
        for (;;) {
            for (auto it = idle_.begin(); it != idle_.end(); ++it)
                if (!(it->key < k) && !(k < it->key)) {
                    Handle h = *it;
                    idle_.erase(it);
                    return h;
                }
            evict_for(fp, lk);
            if (resident_ + fp <= budget_) {
                resident_ += fp;   // reserve before allocating outside the lock
                lk.unlock();
                Handle h;
                h.key = k;
                try {
                    WG_HIP(hipStreamCreateWithFlags(&h.s, hipStreamNonBlocking));
                    h.r = new Recon(g, k.cap, h.s);
                } catch (...) {
                    if (h.s) (void)hipStreamDestroy(h.s);
                    lk.lock();
                    resident_ -= fp;
                    throw;
                }
                h.bytes = fp;
                lk.lock();
                return h;
            }
            // everything resident is busy: wait for a release
            release_cv_.wait(lk);
        }
    }

    // persistent: the distance walk runs persistent (fastest alone), for a
    // request that started alone and for a device-filling one; otherwise walks
    // go one workgroup per tile group, so that concurrent requests interleave
    // instead of queueing behind a walk that holds every slot.  pipe (a
    // device-filling request with another one queued): the walk runs on the
    // handle's second stream with slots left for the next one's solve
    // (pipelined forward), and the turn ends (end_turn) once it is enqueued;
    // the sampling follows the walk there, and finish() joins both and
    // reports a failed walk.
    void run(Job &j, Handle &h, bool persistent, bool pipe, const std::function<void()> &end_turn) {
        const wg_request &rq = j.req;
        h.r->set_persistent(persistent);
        h.r->set_grow_hook([this, &h](size_t extra) { reserve_growth(h, extra); });
        wg_solve_opts o = rq.opts;
        o.warm_start = 0;   // a request's result must not depend on what ran before it
        int st = WG_OK;
        try {
            st = h.r->forward(j.xyz, j.nrm, rq.n_points, o, &j.res.stats, pipe);
            if (pipe) end_turn();
            if (rq.n_q > 0) h.r->sample(j.q, rq.n_q, rq.d_phi, rq.d_nrm_out, pipe);
            if (j.gphi) {
                wg_stats bs{};
                int st2 = h.r->backward(j.q, rq.n_q, j.gphi, j.gnrm, rq.d_gxyz, rq.d_gnrm_pts, rq.d_gq, o, &bs);
                j.res.stats.ms[6] = bs.ms[6];
                j.res.stats.ms[7] = bs.ms[7];
                j.res.stats.iters += bs.iters;
                if (st == WG_OK) st = st2;
            }
            if (pipe) h.r->finish();
        } catch (...) {
            // nothing of a failed request may still run (its buffers go back
            // to the pool): order the handle stream after the second one
            h.r->join();
            (void)hipStreamSynchronize(h.s);
            throw;
        }
        WG_HIP(hipStreamSynchronize(h.s));
        j.res.status = st;
    }

    void worker() {
        (void)hipSetDevice(device_);
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            std::deque<Job *>::iterator pick;
            cv_.wait(lk, [&] { return (stop_ && queue_.empty()) || (pick = next_job()) != queue_.end(); });
            if (stop_ && queue_.empty()) return;
            Job *j = *pick;
            queue_.erase(pick);
            const bool fills = fills_device(j->req.grid);
            bool turn = fills;   // this request holds the device-filling turn
            bool pipe = false;   // ... and ends it early: another one is queued
            // (not with a reverse pass: its adjoint solve would
            // meet the next one's solve, each then several times slower; not
            // with one worker, where nothing could use the slots its walk
            // leaves free)
            if (fills && !j->gphi && inflight_ > 1)
                for (const Job *q : queue_) pipe = pipe || fills_device(q->req.grid);
            fill_running_ += fills;
            ++running_;
            auto end_turn = [this, &turn] {
                std::lock_guard<std::mutex> g(mu_);   // run() is called with lk released
                if (!turn) return;
                turn = false;
                --fill_running_;
                cv_.notify_all();   // a held device-filling request may start
            };
            j->state = 1;
            Key k{};
            for (int a = 0; a < 3; ++a) {
                k.n[a] = j->req.grid.n[a];
                k.lo[a] = j->req.grid.lo[a];
            }
            k.h = j->req.grid.h;
            k.cap = capacity_class(j->req.n_points);
            Handle h;
            bool have = false;
            try {
                h = acquire(k, j->req.grid, lk);
                have = true;
                j->res.t_start = now();
                const bool persistent = running_ == 1 || fills;
                lk.unlock();
                try {
                    run(*j, h, persistent, pipe, end_turn);
                } catch (const Error &e) {
                    set_error(e.what());
                    j->res.status = e.code;
                }
                lk.lock();
            } catch (const Error &e) {
                set_error(e.what());
                j->res.status = e.code;
            }
            j->res.t_done = now();
            if (have) {
                h.last_use = ++clock_;
                idle_.push_back(h);
            }
            j->state = 2;
            --running_;
            if (turn) {   // a request that failed before its walk
                turn = false;
                --fill_running_;
            }
            release_cv_.notify_all();
            drain_cv_.notify_all();
            if (fills) cv_.notify_all();   // a held device-filling request may start
        }
    }

    // First queued request that may start now: any request while no
    // device-filling one holds the turn, else the first smaller one.
    std::deque<Job *>::iterator next_job() {
        auto it = queue_.begin();
        if (fill_running_ > 0)
            while (it != queue_.end() && fills_device((*it)->req.grid)) ++it;
        return it;
    }

    size_t budget_;
    int device_;
    hipStream_t ingest_ = nullptr;
    std::chrono::steady_clock::time_point t0_;
    std::mutex mu_;
    std::condition_variable cv_, release_cv_, drain_cv_;
    std::deque<Job *> queue_;
    std::map<uint64_t, std::unique_ptr<Job>> jobs_;
    std::list<Handle> idle_;
    std::mutex pool_mu_;
    std::multimap<size_t, float *> pool_;   // idle input buffers by capacity (floats)
    std::vector<std::thread> workers_;
    size_t resident_ = 0;
    uint64_t next_ticket_ = 0, clock_ = 0;
    int inflight_;
    int running_ = 0, fill_running_ = 0;
    bool stop_ = false;
};

}  // namespace wg

struct wg_server {
    wg::Server *impl;
};

template <class F>
static int guarded_s(F &&f) {
    try {
        return f();
    } catch (const wg::Error &e) {
        wg::set_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        wg::set_error(e.what());
        return WG_EDEVICE;
    }
}

extern "C" {

int wg_server_create(wg_server **out, size_t hbm_budget_bytes, int max_inflight, int device) {
    return guarded_s([&] {
        wg::require(out != nullptr, WG_EINVAL, "null argument");
        wg::require(max_inflight >= 1 && max_inflight <= 64, WG_EINVAL, "max_inflight outside [1, 64]");
        *out = new wg_server{new wg::Server(hbm_budget_bytes, max_inflight, device)};
        return WG_OK;
    });
}

int wg_submit(wg_server *s, const wg_request *req, uint64_t *ticket) {
    return guarded_s([&] {
        wg::require(s && req, WG_EINVAL, "null argument");
        return s->impl->submit(*req, ticket);
    });
}

int wg_poll(wg_server *s, uint64_t ticket, wg_result *out) {
    return guarded_s([&] {
        wg::require(s != nullptr, WG_EINVAL, "null server");
        return s->impl->poll(ticket, out);
    });
}

double wg_server_now(wg_server *s) { return s ? s->impl->now() : 0.0; }

void wg_server_destroy(wg_server *s) {
    if (!s) return;
    delete s->impl;
    delete s;
}

}  // extern "C"
