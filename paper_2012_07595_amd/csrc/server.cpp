// Serving: continuous batching of BKS solves of different tensors and ranks.
//
// Requests wait in a queue in arrival order.  A free session slot takes the
// oldest waiting request whose device footprint (tensor formats when the
// server uploads them, plus the solver's basis, product and core buffers)
// fits the memory budget left by the sessions already running; a request
// that does not fit is passed over for a later one that does, but at most
// kMaxBypass times, after which nothing behind it is admitted until it is
// (so a large request is not starved by a stream of small ones).  Requests
// larger than the whole budget are refused at submit.  Each admitted session
// runs on a worker thread with its own HIP stream and workspaces, so the
// device work of different sessions overlaps on the GPU; the host-side dense
// inner solves share a bounded pool of host slots.  A slot frees its
// workspaces when its request ends, so that the device bytes it holds are
// the admitted footprint's.  A solve's arithmetic does not depend on what
// else runs (fixed-order reductions, no atomics), so a request's result is
// the same alone and in the mix.
//
// Cancellation: a waiting request leaves the queue at once; a running one
// stops at its next outer iteration and returns the point it had reached.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <thread>

#include "bks_internal.h"
#include "linalg.h"

namespace bks {

int run_bks(Ctx &c, Tensor &t, const bks_params &prm, double *U, double *W, double *F,
            bks_info *info, hipStream_t s);
size_t solve_footprint(int64_t m, int64_t n, int64_t nnz, const bks_params &prm);

namespace {

struct Request {
    uint64_t id;
    Tensor *tensor = nullptr;        // caller's tensor, or owned after upload
    bool owns_tensor = false;
    int64_t m = 0, n = 0, nnz = 0;   // COO request
    std::vector<int32_t> ci, cj, ck;
    std::vector<float> cv;
    bks_params prm;
    double *U, *W, *F;
    size_t footprint = 0;
    size_t dev_peak = 0;
    double t_submit = 0, t_start = 0, t_end = 0;
    int status = 0;
    bool done = false;
    bool running = false;
    int bypassed = 0;                 // times a later request was admitted first
    std::string error;                // message of a failed request
    std::atomic<bool> cancel{false};
    bks_info info;
};

constexpr int kMaxBypass = 16;

}  // namespace
}  // namespace bks

using namespace bks;

struct bks_server_s {
    Ctx *ctx = nullptr;
    int max_active = 8;
    int host_slots = 4;
    size_t budget = 0;
    size_t in_use = 0;
    std::mutex mu;
    std::condition_variable cv_queue, cv_done, cv_host;
    std::deque<Request *> queue;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<hipStream_t> streams;  // one per session slot, made by create
    std::vector<std::thread> workers;
    std::atomic<uint64_t> next_id{1};
    bool stop = false;
    int host_busy = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void worker(hipStream_t stream) {
        (void)hipSetDevice(ctx->device);
        // host solves run concurrently in up to host_slots workers: share the
        // host threads among them (results do not depend on the count)
        la::set_threads(std::max(1, la::threads() / std::max(1, host_slots)));
        Ctx sc;  // private workspaces and stream of this session slot
        sc.device = ctx->device;
        sc.host_acquire = [this] {
            std::unique_lock<std::mutex> g(mu);
            cv_host.wait(g, [&] { return host_busy < host_slots; });
            ++host_busy;
        };
        sc.host_release = [this] {
            {
                std::lock_guard<std::mutex> g(mu);
                --host_busy;
            }
            cv_host.notify_one();
        };
        sc.stream = stream;
        auto acct = std::make_shared<DevAccount>();
        DevAccount::current = acct;
        while (true) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> g(mu);
                cv_queue.wait(g, [&] { return stop || pick() != queue.end(); });
                if (stop && queue.empty()) break;
                auto it = pick();
                if (it == queue.end()) continue;
                r = *it;
                for (auto b = queue.begin(); b != it; ++b) ++(*b)->bypassed;
                queue.erase(it);
                in_use += r->footprint;
                r->running = true;
                r->t_start = now();
            }
            acct->peak.store(acct->live.load());
            sc.cancel = &r->cancel;
            int status = BKS_OK;
            try {
                if (!r->tensor) {
                    auto t = std::make_unique<Tensor>();
                    t->ctx = nullptr;
                    t->m = r->m;
                    t->n = r->n;
                    t->nnz = r->nnz;
                    build_formats(*t, r->ci.data(), r->cj.data(), r->ck.data(), r->cv.data(),
                                  BKS_F32, BKS_SUM_DUPLICATES);
                    r->ci.clear(); r->cj.clear(); r->ck.clear(); r->cv.clear();
                    r->ci.shrink_to_fit(); r->cj.shrink_to_fit(); r->ck.shrink_to_fit();
                    r->cv.shrink_to_fit();
                    r->tensor = t.release();
                    r->owns_tensor = true;
                }
                std::memset(&r->info, 0, sizeof(r->info));
                status = run_bks(sc, *r->tensor, r->prm, r->U, r->W, r->F, &r->info, sc.stream);
            } catch (const Error &e) {
                status = e.code;
                r->error = e.msg;
            } catch (const std::bad_alloc &) {
                status = BKS_ENOMEM;
                r->error = "host allocation failed";
            } catch (const std::exception &e) {
                status = BKS_EDEVICE;
                r->error = e.what();
            }
            sc.cancel = nullptr;
            (void)hipStreamSynchronize(sc.stream);
            const size_t peak = acct->peak.load();
            if (r->owns_tensor) {
                r->tensor->release_device();
                delete r->tensor;
                r->tensor = nullptr;
            }
            sc.release_workspaces();
            {
                std::lock_guard<std::mutex> g(mu);
                in_use -= r->footprint;
                r->dev_peak = peak;
                r->running = false;
                r->status = status;
                r->t_end = now();
                r->done = true;
            }
            cv_done.notify_all();
            cv_queue.notify_all();
        }
        sc.release_workspaces();
        DevAccount::current.reset();
        sc.stream = nullptr;  // the server's, destroyed after the workers end
    }

    // The request a free slot takes (caller holds mu): the oldest one that
    // fits the budget left, unless the head has been passed over kMaxBypass
    // times, in which case only the head may go.
    std::deque<Request *>::iterator pick() {
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            if (in_use + (*it)->footprint <= budget) return it;
            if ((*it)->bypassed >= kMaxBypass) break;
        }
        return queue.end();
    }
};

namespace {

int submit(bks_server s, std::unique_ptr<Request> r, uint64_t *id) {
    const int r1 = r->prm.r, r3 = r->prm.r3;
    const int64_t m = r->tensor ? r->tensor->m : r->m, n = r->tensor ? r->tensor->n : r->n;
    if (r1 < 1 || r3 < 1 || r1 > m || r3 > n || r3 > r1 * (r1 + 1) / 2) return BKS_EINVAL;
    const int64_t nnz = r->tensor ? r->tensor->nnz : r->nnz;
    size_t fp = solve_footprint(m, n, nnz, r->prm);
    if (!r->tensor) fp += (size_t)r->nnz * 48 + (size_t)(m + n) * 16 + 4096;
    r->footprint = fp;
    if (fp > s->budget) return BKS_ENOMEM;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return BKS_EINVAL;
    r->id = s->next_id++;
    r->t_submit = s->now();
    Request *raw = r.get();
    s->reqs[raw->id] = std::move(r);
    s->queue.push_back(raw);
    *id = raw->id;
    s->cv_queue.notify_one();
    return BKS_OK;
}

void fill(const Request &r, bks_result *res) {
    res->footprint = r.footprint;
    res->dev_peak = r.dev_peak;
    std::snprintf(res->error, sizeof(res->error), "%s", r.error.c_str());
    res->status = r.status;
    res->done = r.done ? 1 : 0;
    res->t_submit = r.t_submit;
    res->t_start = r.t_start;
    res->t_end = r.t_end;
    res->info = r.info;
}

}  // namespace

extern "C" {

int bks_server_create(bks_ctx ctx, const bks_server_params *prm, bks_server *out) {
    if (!ctx || !out) return BKS_EINVAL;
    auto s = std::make_unique<bks_server_s>();
    s->ctx = reinterpret_cast<Ctx *>(ctx);
    s->max_active = (prm && prm->max_active > 0) ? prm->max_active : 8;
    s->host_slots = (prm && prm->host_workers > 0) ? prm->host_workers : 4;
    // the ctx's device for the free-memory query and the slots' streams; the
    // caller's current device is restored before returning
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(s->ctx->device) != hipSuccess)
        return BKS_EDEVICE;
    int status = BKS_OK;
    size_t budget = prm ? prm->mem_budget_bytes : 0;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) status = BKS_EDEVICE;
        budget = fr / 4 * 3;
    }
    s->budget = budget;
    // every slot's stream before any worker starts: a slot without one
    // would leave the requests it was meant to take waiting for ever
    for (int i = 0; status == BKS_OK && i < s->max_active; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            status = BKS_EDEVICE;
        else
            s->streams.push_back(st);
    }
    if (status != BKS_OK) {
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        (void)hipSetDevice(prev);
        return status;
    }
    for (int i = 0; i < s->max_active; ++i)
        s->workers.emplace_back([p = s.get(), st = s->streams[i]] { p->worker(st); });
    (void)hipSetDevice(prev);
    *out = s.release();
    return BKS_OK;
}

int bks_server_submit(bks_server s, bks_tensor t, const bks_params *prm, double *U, double *W,
                      double *F, uint64_t *id) {
    if (!s || !t || !prm || !id) return BKS_EINVAL;
    auto r = std::make_unique<Request>();
    r->tensor = reinterpret_cast<Tensor *>(t);
    r->prm = *prm;
    r->U = U;
    r->W = W;
    r->F = F;
    return submit(s, std::move(r), id);
}

int bks_server_submit_coo(bks_server s, int64_t m, int64_t n, int64_t nnz, const int32_t *i,
                          const int32_t *j, const int32_t *k, const float *val,
                          const bks_params *prm, double *U, double *W, double *F, uint64_t *id) {
    if (!s || !prm || !id || m < 1 || n < 1 || nnz < 0) return BKS_EINVAL;
    if (nnz > 0 && (!i || !j || !k || !val)) return BKS_EINVAL;
    auto r = std::make_unique<Request>();
    r->m = m;
    r->n = n;
    r->nnz = nnz;
    r->ci.assign(i, i + nnz);
    r->cj.assign(j, j + nnz);
    r->ck.assign(k, k + nnz);
    r->cv.assign(val, val + nnz);
    r->prm = *prm;
    r->U = U;
    r->W = W;
    r->F = F;
    return submit(s, std::move(r), id);
}

int bks_server_poll(bks_server s, uint64_t id, bks_result *res) {
    if (!s || !res) return BKS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return BKS_ENOTFOUND;
    fill(*it->second, res);
    return BKS_OK;
}

int bks_server_wait(bks_server s, uint64_t id, bks_result *res) {
    if (!s || !res) return BKS_EINVAL;
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return BKS_ENOTFOUND;
    Request *r = it->second.get();
    s->cv_done.wait(g, [&] { return r->done; });
    fill(*r, res);
    return BKS_OK;
}

int bks_server_cancel(bks_server s, uint64_t id) {
    if (!s) return BKS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return BKS_ENOTFOUND;
    Request *r = it->second.get();
    if (r->done) return BKS_EINVAL;
    if (r->running) {
        r->cancel.store(true);
        return BKS_OK;
    }
    auto q = std::find(s->queue.begin(), s->queue.end(), r);
    if (q != s->queue.end()) s->queue.erase(q);
    r->ci.clear(); r->cj.clear(); r->ck.clear(); r->cv.clear();
    r->ci.shrink_to_fit(); r->cj.shrink_to_fit(); r->ck.shrink_to_fit(); r->cv.shrink_to_fit();
    r->status = BKS_ECANCELED;
    r->t_start = r->t_end = s->now();
    r->done = true;
    s->cv_done.notify_all();
    // the queue changed: a request behind this one may fit now
    s->cv_queue.notify_all();
    return BKS_OK;
}

double bks_server_now(bks_server s) { return s ? s->now() : 0.0; }

void bks_server_destroy(bks_server s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        // requests that were never admitted are cancelled
        for (Request *r : s->queue) {
            r->status = BKS_ECANCELED;
            r->done = true;
        }
        s->queue.clear();
    }
    s->cv_queue.notify_all();
    for (auto &w : s->workers) w.join();
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
}

}  // extern "C"
