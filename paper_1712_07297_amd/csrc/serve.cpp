// Serving runtime: a request loop over the public C ABI (include/hs.h,
// "serving").  Worker threads, each with its own HIP stream, form batches
// from the waiting requests (continuous batching): requests on resident
// factorizations reuse them; the new operators of a batch are factored
// together by hs_factor_batch (Alg. 1 on the forest of their cluster trees)
// and stay resident; CG (symmetric) or GMRES(30) (Sec. 5) then runs on every
// factorization the batch touches with the requests' right-hand sides
// stacked by system.  Admission is by device memory: resident factorizations
// plus the estimated needs of the running batches stay under the cap, idle
// factorizations being evicted least recently used first.
#include <hip/hip_runtime.h>

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
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "hs.h"

namespace hs {
int fail_with(int code, const char* msg);  // the calling thread's error message (hs_last_error)
}

namespace {

using hs::fail_with;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    int64_t ticket = 0, key = 0;
    hs_csr A{};
    hs_geometry G{};
    hs_opts opts{};
    int nrhs = 1;
    const double* B = nullptr;
    double* X = nullptr;
    double tol = 1e-10;
    int maxit = 100;
    double t_submit = 0, t_start = 0, t_done = 0;
    hs_result res{};
    bool done = false;
};

// A resident factorization: one or several operators factored together.
struct Group {
    hs_factor_t F = nullptr;
    std::vector<int64_t> keys;      // system i of F is operator keys[i]
    std::vector<int64_t> row_off;   // rows of every system in the stacked vectors
    int64_t n = 0;
    int symmetric = 1;
    double bytes = 0;               // device bytes it holds
    double last_use = 0;
    bool busy = false;              // in use by a running batch
};

struct Plan {
    std::vector<Req*> reqs;
    std::vector<Req*> fresh;        // one request per new operator, factored together
    std::vector<Group*> groups;     // resident factorizations used
    double reserve = 0;
};

constexpr double DEFAULT_BYTES_PER_UNKNOWN = 16384.0;

// Krylov and solve vectors of a batch on n stacked unknowns: CG 4 work
// vectors, GMRES(30) 34, both about 8 for the sweep's level vectors and 2
// for the stacked right-hand sides and solutions.
double krylov_bytes(int64_t n, int nrhs, int symmetric) {
    return (symmetric ? 14.0 : 44.0) * (double)n * nrhs * sizeof(double);
}

bool same_factor_options(const hs_opts& a, const hs_opts& b) {
    return a.eps == b.eps && a.fixed_rank == b.fixed_rank && a.leaf_size == b.leaf_size &&
           a.precision == b.precision && a.symmetric == b.symmetric && a.coarse_fp64_dofs == b.coarse_fp64_dofs &&
           a.keep_levels == b.keep_levels;
}

}  // namespace

struct hs_server_s {
    hs_server_opts o{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> pending;
    std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
    std::unordered_map<int64_t, std::pair<Group*, int>> cache;  // operator -> (factorization, system)
    std::vector<std::unique_ptr<Group>> groups;
    std::unordered_set<int64_t> inflight;                       // operators being factored
    std::map<std::pair<int, int>, double> bytes_per_unknown;    // (grid dimension, precision)
    double held = 0, reserved = 0, peak = 0;
    int64_t next_ticket = 1;
    bool stop = false;
    int64_t submitted = 0, completed = 0, failed = 0, batches = 0, reused = 0, factored = 0, evictions = 0;
    std::vector<double> lat, qwait;
    double t_first = -1, t_last = 0, unknowns = 0;
    std::vector<std::thread> workers;

    double estimate_factor(const Req* r) const {
        auto it = bytes_per_unknown.find({r->G.dim, r->opts.precision});
        const double bpu = it == bytes_per_unknown.end() ? DEFAULT_BYTES_PER_UNKNOWN : it->second;
        return bpu * (double)r->A.n;
    }

    // Free least recently used idle factorizations (not in P) until `need`
    // more bytes fit under the cap; true if they do.
    bool make_room(double need, const Plan& P) {
        bool evicted = false;
        while (held + reserved + need > o.hbm_cap_bytes) {
            Group* victim = nullptr;
            for (auto& g : groups)
                if (!g->busy && std::find(P.groups.begin(), P.groups.end(), g.get()) == P.groups.end() &&
                    (!victim || g->last_use < victim->last_use))
                    victim = g.get();
            if (!victim) break;
            for (int64_t k : victim->keys) cache.erase(k);
            held -= victim->bytes;
            hs_free(victim->F);  // synchronises the device first
            ++evictions;
            evicted = true;
            groups.erase(std::find_if(groups.begin(), groups.end(), [&](auto& g) { return g.get() == victim; }));
        }
        if (evicted) trim_pool();
        return held + reserved + need <= o.hbm_cap_bytes;
    }

    // Hand the stream-ordered pool's unused memory back to the device: the
    // pool keeps freed blocks for reuse, and blocks of evicted factorizations
    // that later requests cannot reuse (other sizes) would otherwise hold
    // device memory outside the cap (and away from the caller's allocations).
    static void trim_pool() {
        int dev = 0;
        hipMemPool_t pool;
        // every free queued so far completes before the trim (an asynchronous
        // free whose completion the host has not observed may still be read)
        (void)hipDeviceSynchronize();
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess)
            (void)hipMemPoolTrimTo(pool, 0);
        (void)hipGetLastError();
    }

    // Form a batch from the waiting requests (lock held).  False: nothing
    // can start now.
    bool form(Plan& P) {
        std::unordered_set<int64_t> keys;
        std::unordered_map<Group*, std::pair<double, int>> group_tol;  // tol / maxit shared on one factorization
        double fresh_n = 0;
        int fresh_nrhs = 0;
        bool running_batches = reserved > 0;
        for (auto it = pending.begin(); it != pending.end() && (int)P.reqs.size() < o.max_batch;) {
            Req* r = *it;
            bool take = false;
            double need = 0;
            if (keys.count(r->key) || inflight.count(r->key)) {
                take = false;
            } else if (cache.count(r->key)) {
                Group* g = cache[r->key].first;
                const bool in_plan = std::find(P.groups.begin(), P.groups.end(), g) != P.groups.end();
                if (!g->busy) {
                    auto gt = group_tol.find(g);
                    take = gt == group_tol.end() || (gt->second.first == r->tol && gt->second.second == r->maxit);
                    need = in_plan ? 0.0 : krylov_bytes(g->n, r->nrhs, g->symmetric);
                    if (take && in_plan) need = krylov_bytes(g->n, r->nrhs, g->symmetric) * 0.5;
                }
            } else if ((int)P.fresh.size() < o.max_new_ops &&
                       (P.fresh.empty() || (same_factor_options(P.fresh[0]->opts, r->opts) &&
                                            P.fresh[0]->tol == r->tol && P.fresh[0]->maxit == r->maxit))) {
                take = true;
                const int nr = std::max(fresh_nrhs, r->nrhs);
                need = estimate_factor(r) + krylov_bytes((int64_t)(fresh_n + r->A.n), nr, r->opts.symmetric) -
                       krylov_bytes((int64_t)fresh_n, fresh_nrhs, r->opts.symmetric);
            }
            if (take && !make_room(P.reserve + need, P)) {
                // nothing else holds memory: start it anyway (it may fail on allocation)
                take = P.reqs.empty() && !running_batches && held + reserved == 0;
            }
            if (!take) {
                if (P.reqs.empty() && it == pending.begin() && !cache.count(r->key) && !inflight.count(r->key) &&
                    !keys.count(r->key)) {
                    // the oldest request waits for memory: keep arrival order
                    return false;
                }
                ++it;
                continue;
            }
            keys.insert(r->key);
            P.reqs.push_back(r);
            P.reserve += need;
            if (cache.count(r->key)) {
                Group* g = cache[r->key].first;
                if (std::find(P.groups.begin(), P.groups.end(), g) == P.groups.end()) P.groups.push_back(g);
                group_tol[g] = {r->tol, r->maxit};
            } else {
                P.fresh.push_back(r);
                fresh_n += (double)r->A.n;
                fresh_nrhs = std::max(fresh_nrhs, r->nrhs);
            }
            it = pending.erase(it);
        }
        if (P.reqs.empty()) return false;
        for (Group* g : P.groups) g->busy = true;
        for (Req* r : P.fresh) inflight.insert(r->key);
        reserved += P.reserve;
        peak = std::max(peak, held + reserved);
        ++batches;
        return true;
    }

    // Solve the requests on one factorization (no lock held).
    void solve_on(Group* g, const std::vector<std::pair<Req*, int>>& items, hipStream_t st) {
        int nr = 0;
        for (auto& it : items) nr = std::max(nr, it.first->nrhs);
        const int64_t n = g->n;
        const int ns = (int)g->keys.size();
        double *Bs = nullptr, *Xs = nullptr;
        int rc = HS_OK;
        // stream-ordered (no device-wide synchronisation that would stall the other workers)
        if (hipMallocAsync((void**)&Bs, (size_t)n * nr * sizeof(double), st) != hipSuccess ||
            hipMallocAsync((void**)&Xs, (size_t)n * nr * sizeof(double), st) != hipSuccess)
            rc = HS_ERR_NOMEM;
        std::vector<double> rel((size_t)ns * nr, 0.0);
        int iters = 0;
        const Req* r0 = items[0].first;
        if (rc == HS_OK) {
            (void)hipMemsetAsync(Bs, 0, (size_t)n * nr * sizeof(double), st);
            for (auto& it : items) {
                const Req* r = it.first;
                const int64_t o = g->row_off[it.second], ni = r->A.n;
                (void)hipMemcpy2DAsync(Bs + o, n * sizeof(double), r->B, ni * sizeof(double), ni * sizeof(double),
                                       r->nrhs, hipMemcpyDeviceToDevice, st);
            }
            rc = g->symmetric ? hs_pcg(g->F, nr, Bs, n, Xs, n, r0->tol, r0->maxit, &iters, rel.data(), st)
                              : hs_gmres(g->F, nr, Bs, n, Xs, n, r0->tol, r0->maxit, 30, &iters, rel.data(), st);
        }
        if (rc >= 0) {
            for (auto& it : items) {
                Req* r = it.first;
                const int64_t o = g->row_off[it.second], ni = r->A.n;
                (void)hipMemcpy2DAsync(r->X, ni * sizeof(double), Xs + o, n * sizeof(double), ni * sizeof(double),
                                       r->nrhs, hipMemcpyDeviceToDevice, st);
            }
        }
        // the solve's buffers are freed once the host has seen the stream finish
        // (a pool trim on another worker may return memory whose asynchronous
        // free is still pending)
        if (hipStreamSynchronize(st) != hipSuccess && rc >= 0) rc = HS_ERR_HIP;
        hs_factor_trim(g->F, st);  // resident between uses: only the factorization itself
        for (auto& it : items) {
            Req* r = it.first;
            r->res.iterations = iters;
            double worst = 0.0;
            for (int c = 0; c < r->nrhs; ++c) worst = std::max(worst, rel[(size_t)it.second + (size_t)ns * c]);
            r->res.relres = worst;
            r->res.status = rc < 0 ? rc : (worst <= r->tol ? HS_OK : HS_WARN_NOT_CONVERGED);
        }
        if (Bs) (void)hipFreeAsync(Bs, st);
        if (Xs) (void)hipFreeAsync(Xs, st);
    }

    // Run a batch (no lock held).  Returns the new factorization, if any.
    std::unique_ptr<Group> run(Plan& P, hipStream_t st) {
        const double t0 = now_s();
        for (Req* r : P.reqs) {
            r->t_start = t0;
            r->res.batch_size = (int)P.reqs.size();
            r->res.reused = std::find(P.fresh.begin(), P.fresh.end(), r) == P.fresh.end();
        }
        std::unique_ptr<Group> ng;
        if (!P.fresh.empty()) {
            std::vector<hs_csr> A;
            std::vector<hs_geometry> G;
            for (Req* r : P.fresh) {
                A.push_back(r->A);
                G.push_back(r->G);
            }
            hs_factor_t F = nullptr;
            const int rc = hs_factor_batch((int)P.fresh.size(), A.data(), G.data(), &P.fresh[0]->opts, st, &F);
            if (rc < 0) {
                for (Req* r : P.fresh) r->res.status = rc;
            } else {
                ng.reset(new Group());
                ng->F = F;
                ng->symmetric = P.fresh[0]->opts.symmetric;
                int32_t ns = 0;
                hs_factor_systems(F, &ns, nullptr);
                ng->row_off.resize(ns + 1);
                hs_factor_systems(F, &ns, ng->row_off.data());
                ng->n = ng->row_off[ns];
                for (Req* r : P.fresh) ng->keys.push_back(r->key);
                std::vector<std::pair<Req*, int>> items;
                for (int i = 0; i < (int)P.fresh.size(); ++i) items.push_back({P.fresh[i], i});
                solve_on(ng.get(), items, st);
            }
        }
        for (Group* g : P.groups) {
            std::vector<std::pair<Req*, int>> items;
            for (Req* r : P.reqs) {
                auto c = cache_lookup(r->key);
                if (c.first == g) items.push_back({r, c.second});
            }
            if (!items.empty()) solve_on(g, items, st);
        }
        return ng;
    }

    // The resident factorization of an operator (lock not needed: the cache
    // entries of a busy factorization do not change while its batch runs).
    std::pair<Group*, int> cache_lookup(int64_t key) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        return it == cache.end() ? std::pair<Group*, int>{nullptr, -1} : it->second;
    }

    // Bookkeeping after a batch (lock held).
    void finish(Plan& P, std::unique_ptr<Group> ng) {
        const double t = now_s();
        reserved -= P.reserve;
        for (Req* r : P.fresh) inflight.erase(r->key);
        for (Group* g : P.groups) {
            g->busy = false;
            g->last_use = t;
            hs_info info;
            if (hs_factor_info(g->F, &info) == HS_OK) {
                held += info.device_bytes - g->bytes;
                g->bytes = info.device_bytes;
            }
        }
        if (ng) {
            hs_info info;
            hs_factor_info(ng->F, &info);
            ng->bytes = info.device_bytes;
            ng->last_use = t;
            held += ng->bytes;
            factored += (int64_t)ng->keys.size();
            auto& bpu = bytes_per_unknown[{P.fresh[0]->G.dim, P.fresh[0]->opts.precision}];
            bpu = std::max(bpu, info.peak_device_bytes / (double)std::max<int64_t>(1, ng->n));
            for (int i = 0; i < (int)ng->keys.size(); ++i) cache[ng->keys[i]] = {ng.get(), i};
            groups.push_back(std::move(ng));
        }
        peak = std::max(peak, held + reserved);
        for (Req* r : P.reqs) {
            r->t_done = t;
            r->res.latency_s = r->t_done - r->t_submit;
            r->res.queue_s = r->t_start - r->t_submit;
            r->done = true;
            if (r->res.status < 0) {
                ++failed;
            } else {
                ++completed;
                reused += r->res.reused;
                lat.push_back(r->res.latency_s);
                qwait.push_back(r->res.queue_s);
                unknowns += (double)r->A.n * r->nrhs;
                t_last = std::max(t_last, t);
            }
        }
    }

    void worker() {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            Plan P;
            while (!form(P)) {
                if (stop && pending.empty()) break;
                cv_work.wait(lk);
            }
            if (P.reqs.empty()) break;
            lk.unlock();
            std::unique_ptr<Group> ng = run(P, st);
            lk.lock();
            finish(P, std::move(ng));
            cv_done.notify_all();
            cv_work.notify_all();
        }
        lk.unlock();
        (void)hipStreamDestroy(st);
    }
};

extern "C" {

int hs_server_create(const hs_server_opts* opts, hs_server_t* S_out) {
    if (!opts || !S_out || !(opts->hbm_cap_bytes > 0) || opts->workers < 0 || opts->max_batch < 0 ||
        opts->max_new_ops < 0)
        return fail_with(HS_ERR_ARG, "bad server options");
    *S_out = nullptr;
    std::unique_ptr<hs_server_s> S(new hs_server_s());
    S->o = *opts;
    if (S->o.workers == 0) S->o.workers = 2;
    if (S->o.max_batch == 0) S->o.max_batch = 32;
    if (S->o.max_new_ops == 0) S->o.max_new_ops = 8;
    if (hipGetDevice(&S->device) != hipSuccess) return fail_with(HS_ERR_NODEVICE, "no HIP device");
    hs_server_s* raw = S.get();
    for (int i = 0; i < S->o.workers; ++i) S->workers.emplace_back([raw] { raw->worker(); });
    *S_out = S.release();
    return HS_OK;
}

int hs_submit(hs_server_t S, int64_t op_key, const hs_csr* A, const hs_geometry* geom, const hs_opts* opts,
              int32_t nrhs, const double* B, double* X, double tol, int32_t maxit, int64_t* ticket) {
    if (!S || !A || !geom || !opts || !B || !X || !ticket) return fail_with(HS_ERR_ARG, "null argument");
    if (nrhs < 1 || nrhs > 64) return fail_with(HS_ERR_ARG, "nrhs must be 1..64");
    if (!(tol >= 0) || maxit < 0) return fail_with(HS_ERR_ARG, "bad tol or maxit");
    if (opts->symmetric != 0 && opts->symmetric != 1) return fail_with(HS_ERR_ARG, "opts->symmetric must be 0 or 1");
    if (A->n <= 0 || !A->row_ptr) return fail_with(HS_ERR_ARG, "bad matrix");
    if ((int64_t)geom->nx * geom->ny * geom->nz != A->n) return fail_with(HS_ERR_ARG, "n != nx*ny*nz");
    std::unique_ptr<Req> r(new Req());
    r->key = op_key;
    r->A = *A;
    r->G = *geom;
    r->opts = *opts;
    r->nrhs = nrhs;
    r->B = B;
    r->X = X;
    r->tol = tol;
    r->maxit = maxit;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail_with(HS_ERR_ARG, "server is stopping");
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    if (S->t_first < 0) S->t_first = r->t_submit;
    S->pending.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
    ++S->submitted;
    S->cv_work.notify_one();
    return HS_OK;
}

int hs_poll(hs_server_t S, int64_t ticket, int32_t* done) {
    if (!S || !done) return HS_ERR_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return HS_ERR_ARG;
    *done = it->second->done ? 1 : 0;
    return HS_OK;
}

int hs_wait(hs_server_t S, int64_t ticket, hs_result* out) {
    if (!S) return HS_ERR_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return HS_ERR_ARG;
    Req* r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->done; });
    if (out) *out = r->res;
    const int st = r->res.status;
    S->reqs.erase(it);
    return st < 0 ? st : HS_OK;
}

int hs_server_stats_get(hs_server_t S, hs_server_stats* out) {
    if (!S || !out) return HS_ERR_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    hs_server_stats s{};
    s.submitted = S->submitted;
    s.completed = S->completed;
    s.failed = S->failed;
    s.batches = S->batches;
    s.reused = S->reused;
    s.factored_ops = S->factored;
    s.evictions = S->evictions;
    std::vector<double> l = S->lat;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
        if (l.empty()) return 0.0;
        const size_t i = std::min(l.size() - 1, (size_t)std::ceil(q * l.size()) - (q * l.size() >= 1 ? 1 : 0));
        return l[i];
    };
    s.p50_latency_s = pct(0.50);
    s.p99_latency_s = pct(0.99);
    double qs = 0;
    for (double q : S->qwait) qs += q;
    s.mean_queue_s = S->qwait.empty() ? 0.0 : qs / S->qwait.size();
    const double span = S->t_last - S->t_first;
    s.unknowns_per_s = span > 0 ? S->unknowns / span : 0.0;
    s.requests_per_s = span > 0 ? S->completed / span : 0.0;
    s.held_bytes = S->held + S->reserved;
    s.peak_held_bytes = S->peak;
    *out = s;
    return HS_OK;
}

void hs_server_destroy(hs_server_t S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    for (auto& g : S->groups) hs_free(g->F);
    delete S;
}

}  // extern "C"
