// pp_server.cpp -- persistent request loop for pressure solves of many independent cases.
//
// Each request names a case (one duct: grid, density, warm-start pressure).  A
// case's solver handle, multigrid hierarchy and last pressure stay resident on
// the device between its requests, so a request that brings no new density
// skips the set-up and every solve starts from the case's previous pressure.
//
// Scheduling: worker threads (the slots) take requests from one queue.  A free
// worker scans the queue in arrival order and takes the first request whose
// case is idle and whose device footprint fits the budget, evicting idle
// resident cases in least-recently-used order when needed.  Requests arriving
// while others run are admitted as soon as a slot and memory are free, and the
// work of different slots overlaps on the device (every case has its own HIP
// stream).  A request larger than the whole budget is rejected (PP_ERR_OOM).
//
// The device work is behind a small backend table so the scheduler can be
// exercised on the host with a fake backend; the HIP backend is in
// pp_server_hip.cpp, and this file uses no HIP itself (it builds with a plain
// host compiler, which the sanitizer builds of the scheduler rely on).
#include "../../include/pp.h"
#include "../../include/pp_server.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

// The HIP library's backend (pp_server_hip.cpp).
pp_backend ppsrv_hip_backend();

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- scheduler

struct Request {
    long long id;
    long long case_id;
    pp_config cfg;
    const double* rho;
    const double* rhs;
    double* p_out;
    double t_submit = 0, t_start = 0, t_end = 0;
    int status = PP_OK;
    pp_stats st{};
    bool done = false;
    bool new_density = false;
    std::string err;
};

struct Case {
    long long id;
    pp_config cfg;
    void* state = nullptr;
    size_t bytes = 0;
    bool busy = false;
    bool have_density = false;
    bool opening = false;
    double last_use = 0;
};

bool same_grid(const pp_config& a, const pp_config& b)
{
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.h == b.h && a.mode == b.mode;
}

}  // namespace

struct pp_server_s {
    pp_server_config cfg{};
    pp_backend be{};
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<long long, std::shared_ptr<Request>> reqs;
    std::map<long long, std::unique_ptr<Case>> cases;
    // resident: bytes of the cases in the map and of evicted cases not yet closed
    // (what the device holds); pending: bytes of admitted new cases whose
    // evictions are still being closed (not opened yet).  Admission keeps
    // resident + pending within the budget, so resident never exceeds it.
    size_t resident = 0, pending = 0, peak_resident = 0;
    long long next_id = 1;
    long long evictions = 0, rejected = 0, completed = 0;
    int running = 0, max_running = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::string err = "no error";

    // Returns the index of the first admissible request, or -1 when none can
    // start now.  When the request needs idle resident cases evicted to fit,
    // they are detached here (taken out of the case map, so nothing else picks
    // them) and moved to *evict; their bytes stay counted in `resident` until the
    // worker has closed them outside the lock.  Called with m held.
    int pick(std::vector<std::unique_ptr<Case>>* evict)
    {
        for (size_t qi = 0; qi < queue.size(); ++qi) {
            Request& r = *queue[qi];
            auto it = cases.find(r.case_id);
            if (it != cases.end()) {
                if (it->second->busy || it->second->opening) continue;
                return (int)qi;
            }
            size_t need = be.footprint(be.ctx, &r.cfg);
            if (need > cfg.budget_bytes) return (int)qi;  // rejected by the worker
            if (resident + pending + need <= cfg.budget_bytes) return (int)qi;
            // evict idle cases, least recently used first, if that makes room
            size_t idle = 0;
            for (auto& kv : cases)
                if (!kv.second->busy && !kv.second->opening) idle += kv.second->bytes;
            if (resident + pending - idle + need > cfg.budget_bytes) continue;  // must wait for running cases
            size_t freed = 0;
            while (resident + pending - freed + need > cfg.budget_bytes) {
                Case* lru = nullptr;
                for (auto& kv : cases) {
                    Case* c = kv.second.get();
                    if (c->busy || c->opening) continue;
                    if (!lru || c->last_use < lru->last_use) lru = c;
                }
                if (!lru) break;
                freed += lru->bytes;
                ++evictions;
                auto node = cases.find(lru->id);
                evict->push_back(std::move(node->second));
                cases.erase(node);
            }
            return (int)qi;
        }
        return -1;
    }

    // Closes evicted cases (m not held), then returns their bytes to the budget.
    void close_evicted(std::unique_lock<std::mutex>& lk, std::vector<std::unique_ptr<Case>>& evict)
    {
        if (evict.empty()) return;
        lk.unlock();
        size_t freed = 0;
        for (auto& c : evict) {
            if (c->state) be.close_case(be.ctx, c->state);
            freed += c->bytes;
        }
        evict.clear();
        lk.lock();
        resident -= freed;
        cv_work.notify_all();
    }

    void finish(std::shared_ptr<Request> r, int status)
    {
        r->status = status;
        r->t_end = now_s();
        r->done = true;
        ++completed;
        if (status == PP_ERR_OOM || status == PP_ERR_INVALID) ++rejected;
    }

    void worker()
    {
        std::unique_lock<std::mutex> lk(m);
        std::vector<std::unique_ptr<Case>> evict;
        for (;;) {
            int qi = -1;
            cv_work.wait(lk, [&] { return stop || (!queue.empty() && (qi = pick(&evict)) >= 0); });
            if (stop) {
                close_evicted(lk, evict);
                return;
            }
            std::shared_ptr<Request> r = queue[qi];
            queue.erase(queue.begin() + qi);
            r->t_start = now_s();
            Case* c = nullptr;
            auto it = cases.find(r->case_id);
            bool fresh = false;
            if (it == cases.end()) {
                size_t need = be.footprint(be.ctx, &r->cfg);
                if (need == 0 || need > cfg.budget_bytes) {
                    r->err = need == 0 ? "invalid configuration" : "case footprint exceeds the device budget";
                    finish(r, need == 0 ? PP_ERR_INVALID : PP_ERR_OOM);
                    cv_done.notify_all();
                    cv_work.notify_all();
                    continue;
                }
                auto nc = std::make_unique<Case>();
                nc->id = r->case_id;
                nc->cfg = r->cfg;
                nc->bytes = need;
                nc->opening = true;
                c = nc.get();
                cases[r->case_id] = std::move(nc);
                fresh = true;
                c->busy = true;
                ++running;
                max_running = std::max(max_running, running);
                // the new case is pending while the evicted ones close, so no other slot
                // can admit into memory that is not free yet
                pending += need;
                close_evicted(lk, evict);
                pending -= need;
                resident += need;
                peak_resident = std::max(peak_resident, resident);
            } else {
                c = it->second.get();
                if (!same_grid(c->cfg, r->cfg)) {
                    r->err = "case was created with a different grid or mode";
                    finish(r, PP_ERR_INVALID);
                    cv_done.notify_all();
                    cv_work.notify_all();
                    continue;
                }
            }
            if (!fresh) {
                c->busy = true;
                ++running;
                max_running = std::max(max_running, running);
            }
            lk.unlock();

            int rc = PP_OK;
            std::string msg;
            if (fresh) {
                rc = be.open_case(be.ctx, &r->cfg, &c->state);
                if (rc != PP_OK) msg = be.error(be.ctx, nullptr);
            }
            if (rc == PP_OK) {
                if (r->rho) {
                    rc = be.set_density(be.ctx, c->state, r->rho);
                    if (rc == PP_OK) c->have_density = true;
                    r->new_density = true;
                } else if (!c->have_density) {
                    rc = PP_ERR_STATE;
                    msg = "first request of a case must bring its density";
                }
                if (rc == PP_OK) rc = be.solve(be.ctx, c->state, r->rhs, r->p_out, &r->st);
                if (rc != PP_OK && msg.empty()) msg = be.error(be.ctx, c->state);
            }

            lk.lock();
            --running;
            c->busy = false;
            c->opening = false;
            c->last_use = now_s();
            if (fresh && !c->state) {  // could not open: release its reservation
                resident -= c->bytes;
                cases.erase(r->case_id);
            }
            r->err = msg;
            finish(r, rc);
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

static thread_local std::string g_srv_err = "no error";

extern "C" {

int pp_server_create(const pp_server_config* cfg, const pp_backend* backend, pp_server* out)
{
    if (out) *out = nullptr;
    if (!cfg || !out || cfg->slots < 1 || cfg->slots > 64 || cfg->budget_bytes == 0) {
        g_srv_err = "invalid server configuration";
        return PP_ERR_INVALID;
    }
    auto* s = new (std::nothrow) pp_server_s;
    if (!s) return PP_ERR_OOM;
    s->cfg = *cfg;
    if (backend) {
        s->be = *backend;
    } else {
        s->be = ppsrv_hip_backend();
    }
    for (int i = 0; i < cfg->slots; ++i) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return PP_OK;
}

int pp_server_submit(pp_server s, long long case_id, const pp_config* cfg, const double* rho, const double* rhs,
                     double* p_out, long long* req_id)
{
    if (!s || !cfg || !rhs || !req_id) { g_srv_err = "null argument"; return PP_ERR_INVALID; }
    auto r = std::make_shared<Request>();
    r->case_id = case_id;
    r->cfg = *cfg;
    r->rho = rho;
    r->rhs = rhs;
    r->p_out = p_out;
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->m);
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_all();
    *req_id = r->id;
    return PP_OK;
}

int pp_server_wait(pp_server s, long long req_id, double timeout_s, pp_request_result* out)
{
    if (!s) { g_srv_err = "null server"; return PP_ERR_INVALID; }
    std::unique_lock<std::mutex> lk(s->m);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) { g_srv_err = "unknown request"; return PP_ERR_INVALID; }
    std::shared_ptr<Request> r = it->second;
    auto pred = [&] { return r->done; };
    if (timeout_s < 0) s->cv_done.wait(lk, pred);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return 1;  // still running
    if (out) {
        out->status = r->status;
        out->stats = r->st;
        out->t_submit = r->t_submit;
        out->t_start = r->t_start;
        out->t_end = r->t_end;
        out->latency_ms = (r->t_end - r->t_submit) * 1e3;
        out->new_density = r->new_density;
        std::snprintf(out->message, sizeof(out->message), "%s", r->err.c_str());
    }
    return PP_OK;
}

int pp_server_get_stats(pp_server s, pp_server_stats* out)
{
    if (!s || !out) return PP_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->m);
    std::vector<double> lat;
    double t0 = 1e300, t1 = -1e300;
    long long ok = 0;
    for (auto& kv : s->reqs) {
        Request& r = *kv.second;
        if (!r.done) continue;
        if (r.status == PP_OK) {
            lat.push_back((r.t_end - r.t_submit) * 1e3);
            ++ok;
        }
        t0 = std::min(t0, r.t_submit);
        t1 = std::max(t1, r.t_end);
    }
    std::sort(lat.begin(), lat.end());
    auto q = [&](double f) {
        if (lat.empty()) return 0.0;
        double pos = f * (lat.size() - 1);
        size_t i = (size_t)pos;
        double w = pos - i;
        return i + 1 < lat.size() ? lat[i] * (1 - w) + lat[i + 1] * w : lat[i];
    };
    std::memset(out, 0, sizeof(*out));
    out->completed = s->completed;
    out->succeeded = ok;
    out->rejected = s->rejected;
    out->queued = (long long)s->queue.size();
    out->running = s->running;
    out->max_running = s->max_running;
    out->resident_cases = (long long)s->cases.size();
    out->resident_bytes = s->resident;
    out->peak_resident_bytes = s->peak_resident;
    out->evictions = s->evictions;
    out->latency_p50_ms = q(0.50);
    out->latency_p99_ms = q(0.99);
    out->latency_max_ms = lat.empty() ? 0.0 : lat.back();
    out->solves_per_s = (ok > 0 && t1 > t0) ? ok / (t1 - t0) : 0.0;
    return PP_OK;
}

int pp_server_destroy(pp_server s)
{
    if (!s) return PP_OK;
    {
        std::unique_lock<std::mutex> lk(s->m);
        // let queued and running work drain
        s->cv_done.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->cases)
        if (kv.second->state) s->be.close_case(s->be.ctx, kv.second->state);
    delete s;
    return PP_OK;
}

const char* pp_server_last_error(void) { return g_srv_err.c_str(); }

}  // extern "C"
