// Serving engine: a request loop with continuous admission over the C ABI of the library.
//
// Each registered pattern is analysed once; its resident replicas (kkt_clone of the
// analysed handle, each bound to its own device workspace) keep the symbolic structure and
// the factors on the device between requests.  Requests (refactor + solve + refinement of
// one system of a registered pattern, 1..max_nrhs right-hand sides) wait in arrival order;
// worker threads, one stream each, take the first request that can run now: a free
// replica of its pattern, or a new replica if the workspaces on the device stay within the
// byte budget (HBM footprint), evicting idle replicas of other patterns (least recently
// used first) when that makes room.  Requests of other patterns pass a request that has to
// wait for memory or a replica, so work of several requests overlaps on the device
// whenever slots and memory allow.  Results do not depend on the mix: every replica of a
// pattern runs the same kernels on the same data.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/kkt.h"

namespace {

using clock_type = std::chrono::steady_clock;

struct Replica {
    kkt_handle *h = nullptr;
    void *ws = nullptr;
    size_t bytes = 0;
    int pattern = -1;
    bool busy = false;
    uint64_t last_use = 0;
};

struct Pattern {
    kkt_handle *tmpl = nullptr;   // the analysed handle (never bound)
    size_t ws_bytes = 0;
    int32_t n = 0;
    int64_t nnz = 0;
};

struct Request {
    int64_t ticket = 0;
    int pattern = 0;
    const double *v = nullptr, *b = nullptr;
    double *x = nullptr;
    int32_t nrhs = 1;
    int64_t ld = 0;
    clock_type::time_point t_submit, t_start, t_end;
    std::vector<kkt_info> info;
    int status = KKT_OK;
    bool done = false;
    bool new_replica = false;
};

}  // namespace

struct kkt_server {
    kkt_server_opts o{};
    int device = -1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<int64_t, Request *> reqs;
    std::vector<Pattern> patterns;
    std::vector<Replica *> replicas;
    size_t used = 0, peak = 0;
    int64_t next_ticket = 1;
    uint64_t use_clock = 0;
    int64_t evictions = 0, created = 0, completed = 0;
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace {

// Picks the first queued request that can run now and reserves its replica (creating one
// in the budget, after evicting idle replicas if needed).  Returns null if none can.  The
// caller holds s->mu.  On return *fresh is a replica that still has to be allocated and
// bound (its bytes are already counted), evicted replicas are in *drop.
Request *admit(kkt_server *s, Replica **rep, bool *fresh, std::vector<Replica *> *drop) {
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
        Request *r = *it;
        const Pattern &p = s->patterns[r->pattern];
        Replica *free_rep = nullptr;
        for (Replica *x : s->replicas)
            if (x->pattern == r->pattern && !x->busy) {
                free_rep = x;
                break;
            }
        if (free_rep) {
            free_rep->busy = true;
            free_rep->last_use = ++s->use_clock;
            *rep = free_rep;
            *fresh = false;
            s->queue.erase(it);
            return r;
        }
        // a new replica: within the budget, after evicting idle replicas of other patterns
        size_t room = s->o.hbm_budget > s->used ? s->o.hbm_budget - s->used : 0;
        if (room < p.ws_bytes) {
            std::vector<Replica *> idle;
            for (Replica *x : s->replicas)
                if (!x->busy && x->pattern != r->pattern) idle.push_back(x);
            std::sort(idle.begin(), idle.end(), [](const Replica *a, const Replica *b) { return a->last_use < b->last_use; });
            size_t gain = 0;
            size_t k = 0;
            while (k < idle.size() && room + gain < p.ws_bytes) gain += idle[k++]->bytes;
            if (room + gain < p.ws_bytes) continue;   // cannot run yet: later requests may
            for (size_t q = 0; q < k; ++q) {
                Replica *x = idle[q];
                s->replicas.erase(std::find(s->replicas.begin(), s->replicas.end(), x));
                s->used -= x->bytes;
                ++s->evictions;
                drop->push_back(x);
            }
        }
        Replica *nr = new (std::nothrow) Replica;
        if (!nr) return nullptr;
        nr->pattern = r->pattern;
        nr->bytes = p.ws_bytes;
        nr->busy = true;
        nr->last_use = ++s->use_clock;
        s->replicas.push_back(nr);
        s->used += nr->bytes;
        s->peak = std::max(s->peak, s->used);
        ++s->created;
        *rep = nr;
        *fresh = true;
        s->queue.erase(it);
        return r;
    }
    return nullptr;
}

void free_replica(Replica *x) {
    if (x->h) kkt_destroy(x->h);      // waits for its last work
    if (x->ws) (void)hipFree(x->ws);
    delete x;
}

void worker(kkt_server *s) {
    (void)hipSetDevice(s->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        Replica *rep = nullptr;
        bool fresh = false;
        std::vector<Replica *> drop;
        Request *r = nullptr;
        s->cv_work.wait(lk, [&] { return s->stop || (r = admit(s, &rep, &fresh, &drop)) != nullptr; });
        if (!r) break;   // stopping with nothing admissible
        lk.unlock();
        for (Replica *x : drop) free_replica(x);
        int rc = st ? KKT_OK : KKT_ERR_DEVICE;
        r->t_start = clock_type::now();
        const Pattern &p = s->patterns[r->pattern];
        if (!rc && fresh) {
            rc = kkt_clone(p.tmpl, &rep->h);
            if (!rc && hipMalloc(&rep->ws, rep->bytes) != hipSuccess) rc = KKT_ERR_NOMEM;
            if (!rc) rc = kkt_bind(rep->h, rep->ws, rep->bytes, s->o.max_nrhs, st);
            r->new_replica = true;
        }
        if (!rc) {
            r->info.resize(r->nrhs);
            if (r->nrhs == 1) {   // the forward substitution rides in the refactorization
                rc = kkt_refactor_refine(rep->h, r->v, r->b, r->x, r->info.data(), st);
            } else {
                rc = kkt_refactor(rep->h, r->v, st);
                if (!rc) rc = kkt_refine(rep->h, r->b, r->x, r->nrhs, r->ld, r->info.data(), st);
            }
        }
        if (rc < 0) (void)hipStreamSynchronize(st);
        r->t_end = clock_type::now();
        lk.lock();
        r->status = rc;
        r->done = true;
        ++s->completed;
        if (rc < 0 && fresh) {   // a replica that failed to come up is dropped
            s->replicas.erase(std::find(s->replicas.begin(), s->replicas.end(), rep));
            s->used -= rep->bytes;
            lk.unlock();
            free_replica(rep);
            lk.lock();
        } else {
            rep->busy = false;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();   // a replica is free again
    }
    lk.unlock();
    if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

void kkt_server_default_opts(kkt_server_opts *o) {
    if (!o) return;
    o->hbm_budget = (size_t)16 << 30;
    o->max_inflight = 4;
    o->max_nrhs = 4;
}

int kkt_server_create(const kkt_server_opts *opts, kkt_server **out) {
    if (!out) return KKT_ERR_ARG;
    *out = nullptr;
    kkt_server_opts o;
    kkt_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.max_inflight < 1 || o.max_inflight > 64 || o.max_nrhs < 1 || o.hbm_budget == 0) return KKT_ERR_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return KKT_ERR_DEVICE;
    kkt_server *s = new (std::nothrow) kkt_server;
    if (!s) return KKT_ERR_NOMEM;
    s->o = o;
    s->device = dev;
    try {
        for (int32_t i = 0; i < o.max_inflight; ++i) s->workers.emplace_back(worker, s);
    } catch (...) {
        kkt_server_destroy(s);
        return KKT_ERR_NOMEM;
    }
    *out = s;
    return KKT_OK;
}

int kkt_server_add_pattern(kkt_server *s, int32_t n, const int64_t *rowptr, const int32_t *colind,
                           const double *values_k1, const kkt_opts *opts, int32_t *pattern) {
    if (!s || !pattern) return KKT_ERR_ARG;
    // several requests run at once: persistent solves take their items by ticket
    kkt_opts o;
    kkt_default_opts(&o);
    if (opts) o = *opts;
    if (o.persistent_solve == 1) o.persistent_solve = 2;
    kkt_handle *h = nullptr;
    int rc = kkt_analyze(n, rowptr, colind, values_k1, &o, &h);
    if (rc) return rc;
    size_t bytes = 0;
    rc = kkt_workspace_bytes(h, s->o.max_nrhs, &bytes);
    if (rc) {
        kkt_destroy(h);
        return rc;
    }
    kkt_stats st{};
    (void)kkt_get_stats(h, &st);
    std::lock_guard<std::mutex> lk(s->mu);
    if (bytes > s->o.hbm_budget) {
        kkt_destroy(h);
        return KKT_ERR_NOMEM;   // one replica alone exceeds the budget
    }
    Pattern p;
    p.tmpl = h;
    p.ws_bytes = bytes;
    p.n = st.n;
    p.nnz = st.nnz_a;
    s->patterns.push_back(p);
    *pattern = (int32_t)s->patterns.size() - 1;
    return KKT_OK;
}

int kkt_server_submit(kkt_server *s, int32_t pattern, const double *d_values, const double *d_b, double *d_x,
                      int32_t nrhs, int64_t ld, int64_t *ticket) {
    if (!s || !d_values || !d_b || !d_x || !ticket || nrhs < 1) return KKT_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (pattern < 0 || pattern >= (int32_t)s->patterns.size() || nrhs > s->o.max_nrhs ||
        ld < s->patterns[pattern].n)
        return KKT_ERR_ARG;
    Request *r = new (std::nothrow) Request;
    if (!r) return KKT_ERR_NOMEM;
    r->ticket = s->next_ticket++;
    r->pattern = pattern;
    r->v = d_values;
    r->b = d_b;
    r->x = d_x;
    r->nrhs = nrhs;
    r->ld = ld;
    r->t_submit = clock_type::now();
    s->reqs.emplace(r->ticket, r);
    s->queue.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return KKT_OK;
}

int kkt_server_wait(kkt_server *s, int64_t ticket, kkt_info *info, double *times_ms) {
    if (!s) return KKT_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return KKT_ERR_ARG;
    Request *r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->reqs.erase(it);
    lk.unlock();
    if (info)
        for (int32_t j = 0; j < r->nrhs; ++j)
            info[j] = j < (int32_t)r->info.size() ? r->info[j] : kkt_info{0, r->status, 0.0, 0};
    if (times_ms) {
        using ms = std::chrono::duration<double, std::milli>;
        times_ms[0] = ms(r->t_start - r->t_submit).count();   // waiting for admission
        times_ms[1] = ms(r->t_end - r->t_start).count();      // on the device
        times_ms[2] = ms(r->t_end - r->t_submit).count();     // latency
        times_ms[3] = r->new_replica ? 1.0 : 0.0;
    }
    const int rc = r->status;
    delete r;
    return rc;
}

int kkt_server_get_stats(kkt_server *s, kkt_server_stats *out) {
    if (!s || !out) return KKT_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    out->replicas = (int32_t)s->replicas.size();
    out->patterns = (int32_t)s->patterns.size();
    out->bytes_in_use = s->used;
    out->peak_bytes = s->peak;
    out->replicas_created = s->created;
    out->evictions = s->evictions;
    out->completed = s->completed;
    out->queued = (int64_t)s->queue.size();
    return KKT_OK;
}

void kkt_server_destroy(kkt_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers)
        if (t.joinable()) t.join();
    for (Replica *x : s->replicas) free_replica(x);
    for (auto &p : s->patterns) kkt_destroy(p.tmpl);
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
}

}  // extern "C"
