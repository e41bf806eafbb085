// Serving loop with continuous batching.
//
// Requests (a resident hierarchy, or a set of equivalent replicas of one,
// nrhs right-hand sides, CG options) are queued by submit() and admitted by
// one loop thread whenever a slot is free, the request's working memory fits
// the budget, a large request would not exceed the running large ones
// allowed, and one of its hierarchies is not serving another request.  The
// queue is scanned in arrival order, or smallest expected work (fine DoFs x
// nrhs) first with an aging bound, and a request that does not fit yet does
// not hold back later ones that do.  Each
// admitted request runs as a resumable PCG task (host/hierarchy.cpp) on a
// stream of its own, so the kernels of all admitted requests overlap on the
// device; the loop advances every task whose scalars have arrived, finishes
// tasks, frees their slot and memory, and admits more.  A request's result
// is computed by exactly the launches a blocking nnmg_pcg_solve_multi makes,
// so it is the same alone and in the mix.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "../internal.hpp"

namespace nnmg {

struct Hierarchy;
struct PcgTask;
PcgTask* pcg_task_create(Hierarchy& H, const double* b, double* x, const nnmg_cg_opts& o, nnmg_cg_result* res,
                         int nr, hipStream_t s);
bool pcg_task_ready(const PcgTask* t);
bool pcg_task_step(PcgTask* t);
int pcg_task_status(const PcgTask* t);
void pcg_task_destroy(PcgTask* t);
size_t hierarchy_footprint(const Hierarchy& H, int nr);
int64_t hierarchy_fine_dofs(const Hierarchy& H);
bool hierarchy_try_acquire(Hierarchy& H);
void hierarchy_release(Hierarchy& H);

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0, Clock::time_point t1) {
    return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

struct Request {
    int64_t id = 0;
    std::vector<Hierarchy*> replicas;  // equivalent hierarchies; the request runs on an idle one
    Hierarchy* H = nullptr;            // the one it runs on
    int nr = 1;
    const double* b = nullptr;
    double* x = nullptr;
    nnmg_cg_opts o{};
    size_t bytes = 0;
    double work = 0;     // expected work: fine DoFs x nrhs
    bool large = false;  // work >= opts.large_work
    std::vector<nnmg_cg_result> res;
    int status = NNMG_OK;
    std::string error;
    bool done = false;
    Clock::time_point t_submit, t_start, t_end;
    PcgTask* task = nullptr;
    int slot = -1;
};

}  // namespace

struct Server {
    Ctx* ctx = nullptr;
    nnmg_server_opts opts{};
    std::mutex mu;
    std::condition_variable cv_loop, cv_done;
    std::deque<Request*> pending;
    std::vector<Request*> running;
    std::unordered_map<int64_t, std::unique_ptr<Request>> requests;
    std::vector<hipStream_t> streams;
    std::vector<char> slot_busy;
    size_t reserved = 0;
    int running_large = 0;
    int64_t next_id = 1;
    bool stop = false;
    nnmg_server_stats stats{};
    std::thread loop;

    void run();
    void admit(std::vector<Request*>& started);
    void finish(Request* r, Clock::time_point now);
};

void Server::admit(std::vector<Request*>& started) {
    // called with mu held
    std::vector<Request*> order(pending.begin(), pending.end());
    if (opts.policy == NNMG_ADMIT_SMALLEST) {
        // requests past the aging bound first, oldest first; then the others
        // by expected work, ties in arrival order
        const auto now = Clock::now();
        auto aged = [&](const Request* r) { return ms_since(r->t_submit, now) >= opts.aging_ms; };
        std::stable_sort(order.begin(), order.end(), [&](const Request* a, const Request* b) {
            const bool ga = aged(a), gb = aged(b);
            if (ga != gb) return ga;
            if (ga) return a->id < b->id;
            return a->work < b->work;
        });
    }
    for (Request* r : order) {
        if ((int)running.size() >= opts.max_active) break;
        if (reserved + r->bytes > opts.memory_budget && !running.empty()) continue;  // does not fit yet
        if (r->large && running_large >= opts.max_large) continue;
        r->H = nullptr;
        for (Hierarchy* h : r->replicas)
            if (hierarchy_try_acquire(*h)) {
                r->H = h;
                break;
            }
        if (!r->H) continue;  // every replica serves another request
        int slot = 0;
        while (slot_busy[(size_t)slot]) ++slot;
        slot_busy[(size_t)slot] = 1;
        r->slot = slot;
        reserved += r->bytes;
        running_large += r->large ? 1 : 0;
        running.push_back(r);
        started.push_back(r);
        pending.erase(std::find(pending.begin(), pending.end(), r));
        stats.max_running = std::max(stats.max_running, (int)running.size());
        stats.max_reserved = std::max(stats.max_reserved, reserved);
    }
}

void Server::finish(Request* r, Clock::time_point now) {
    // called with mu held
    r->t_end = now;
    r->done = true;
    if (r->task) {
        pcg_task_destroy(r->task);
        r->task = nullptr;
    }
    // a request that failed part-way may have launches in flight that still
    // use its hierarchy's buffers: drain its stream before another request
    // may take the hierarchy (a finished solve has launched nothing since the
    // event it completed on, so this costs nothing then)
    (void)hipStreamSynchronize(streams[(size_t)r->slot]);
    hierarchy_release(*r->H);
    slot_busy[(size_t)r->slot] = 0;
    reserved -= r->bytes;
    running_large -= r->large ? 1 : 0;
    running.erase(std::find(running.begin(), running.end(), r));
    ++stats.completed;
    cv_done.notify_all();
}

void Server::run() {
    (void)hipSetDevice(ctx->device);
    std::vector<Request*> started;
    while (true) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_loop.wait(lk, [&] { return stop || !running.empty() || !pending.empty(); });
            if (stop && running.empty() && pending.empty()) return;
            started.clear();
            admit(started);
        }
        // start the admitted requests (launches only; no lock held)
        for (Request* r : started) {
            r->t_start = Clock::now();
            try {
                r->task = pcg_task_create(*r->H, r->b, r->x, r->o, r->res.data(), r->nr,
                                          streams[(size_t)r->slot]);
            } catch (const Error& e) {
                std::lock_guard<std::mutex> lk(mu);
                r->status = e.code;
                r->error = e.msg;
                finish(r, Clock::now());
            } catch (const std::exception& e) {
                std::lock_guard<std::mutex> lk(mu);
                r->status = NNMG_ERR_HIP;
                r->error = e.what();
                finish(r, Clock::now());
            }
        }
        // advance every task whose scalars have arrived
        bool progressed = !started.empty();
        std::vector<Request*> snapshot;
        {
            std::lock_guard<std::mutex> lk(mu);
            snapshot = running;
        }
        for (Request* r : snapshot) {
            if (!r->task || !pcg_task_ready(r->task)) continue;
            progressed = true;
            bool fin = false;
            try {
                fin = pcg_task_step(r->task);
                if (fin) {
                    r->status = pcg_task_status(r->task);
                    // the solve's last launch (the final update of x) ends before its end time
                    NNMG_HIP(hipStreamSynchronize(streams[(size_t)r->slot]));
                }
            } catch (const Error& e) {
                fin = true;
                r->status = e.code;
                r->error = e.msg;
            } catch (const std::exception& e) {
                fin = true;
                r->status = NNMG_ERR_HIP;
                r->error = e.what();
            }
            if (fin) {
                std::lock_guard<std::mutex> lk(mu);
                finish(r, Clock::now());
            }
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
}

Server* server_create(Ctx* ctx, const nnmg_server_opts& o) {
    if (o.max_active < 1 || o.max_active > 64) fail(NNMG_ERR_INVALID_ARG, "max_active must be in 1..64");
    if (o.policy != NNMG_ADMIT_ARRIVAL && o.policy != NNMG_ADMIT_SMALLEST) fail(NNMG_ERR_INVALID_ARG, "policy");
    if (!(o.aging_ms >= 0.0) || !(o.large_work >= 0.0) || o.max_large < 1)
        fail(NNMG_ERR_INVALID_ARG, "aging_ms and large_work must be >= 0, max_large >= 1");
    auto* S = new Server();
    S->ctx = ctx;
    S->opts = o;
    try {
        NNMG_HIP(hipSetDevice(ctx->device));
        for (int i = 0; i < o.max_active; ++i) {
            hipStream_t st;
            NNMG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            S->streams.push_back(st);
        }
        S->slot_busy.assign((size_t)o.max_active, 0);
        S->loop = std::thread([S] { S->run(); });
    } catch (...) {
        for (auto st : S->streams) (void)hipStreamDestroy(st);
        delete S;
        throw;
    }
    return S;
}

void server_destroy(Server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_loop.notify_all();
    if (S->loop.joinable()) S->loop.join();  // finishes every queued request first
    for (auto st : S->streams) (void)hipStreamDestroy(st);
    delete S;
}

int64_t server_submit(Server* S, Hierarchy* const* replicas, int n_replicas, int nr, const double* b, double* x,
                      const nnmg_cg_opts& o) {
    if (n_replicas < 1) fail(NNMG_ERR_INVALID_ARG, "no hierarchy");
    if (nr < 1 || nr > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "nrhs must be in 1..8");
    if (o.max_it < 0 || !(o.rtol >= 0.0)) fail(NNMG_ERR_INVALID_ARG, "CG options");
    if (o.vcycle_prec != NNMG_FP64 && o.vcycle_prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "vcycle_prec");
    auto r = std::make_unique<Request>();
    r->replicas.assign(replicas, replicas + n_replicas);
    for (Hierarchy* h : r->replicas)
        if (!h) fail(NNMG_ERR_INVALID_ARG, "hierarchy is NULL");
    r->nr = nr;
    r->b = b;
    r->x = x;
    r->o = o;
    r->bytes = hierarchy_footprint(*replicas[0], nr);
    r->work = (double)hierarchy_fine_dofs(*replicas[0]) * nr;
    r->large = S->opts.large_work > 0.0 && r->work >= S->opts.large_work;
    r->res.assign((size_t)nr, nnmg_cg_result{0, 0.0, NNMG_OK});
    r->t_submit = Clock::now();
    int64_t id;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) fail(NNMG_ERR_INVALID_ARG, "server is shutting down");
        id = S->next_id++;
        r->id = id;
        S->pending.push_back(r.get());
        S->requests.emplace(id, std::move(r));
        ++S->stats.submitted;
    }
    S->cv_loop.notify_all();
    return id;
}

static Request* find(Server* S, int64_t id) {
    auto it = S->requests.find(id);
    if (it == S->requests.end()) fail(NNMG_ERR_INVALID_ARG, "unknown ticket");
    return it->second.get();
}

int server_wait(Server* S, int64_t id, nnmg_cg_result* res, nnmg_request_times* times, std::string* err) {
    std::unique_lock<std::mutex> lk(S->mu);
    Request* r = find(S, id);
    S->cv_done.wait(lk, [&] { return r->done; });
    if (res)
        for (int k = 0; k < r->nr; ++k) res[k] = r->res[(size_t)k];
    if (times) {
        times->queued_ms = ms_since(r->t_submit, r->t_start);
        times->run_ms = ms_since(r->t_start, r->t_end);
        times->total_ms = ms_since(r->t_submit, r->t_end);
    }
    const int st = r->status;
    if (err) *err = r->error;
    S->requests.erase(id);
    return st;
}

bool server_poll(Server* S, int64_t id) {
    std::lock_guard<std::mutex> lk(S->mu);
    return find(S, id)->done;
}

void server_stats(Server* S, nnmg_server_stats* out) {
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->running = (int)S->running.size();
    out->pending = (int)S->pending.size();
    out->reserved = S->reserved;
}

}  // namespace nnmg
