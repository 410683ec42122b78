// server_stress.cpp -- host-only stress run of the serving scheduler
// (paper_2104_01636_amd/csrc/pp_server.cpp) for sanitizer builds.
//
// A fake backend stands in for the GPU: a case is a host buffer of the grid's
// size, a solve sleeps briefly and writes a value that identifies the request,
// so results can be checked.  Several submitter threads send requests for many
// cases of uneven sizes under a budget that forces evictions, and the backend
// records whether the bytes of open cases ever exceed the budget.  Exits 0 when
// every request completed with its own result and the budget held.
#include "pp_server.h"

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

// The HIP backend is not linked into this build.
pp_backend ppsrv_hip_backend() { return pp_backend{}; }

namespace {

constexpr size_t kBytesPerCell = 64;
constexpr size_t kBudget = 64 * 32 * 32 * 64;  // room for two of the largest grids

struct FakeCase {
    std::vector<double> rho, p;
    size_t bytes = 0;
    bool have_density = false;
};

std::atomic<long long> g_live{0}, g_peak{0}, g_over{0}, g_open{0}, g_close{0};

size_t fp(void*, const pp_config* c)
{
    if (c->nz % 2 || c->nx < 2) return 0;
    return (size_t)c->nx * c->ny * c->nz * kBytesPerCell;
}

int open_case(void*, const pp_config* c, void** out)
{
    auto* fc = new FakeCase;
    fc->bytes = fp(nullptr, c);
    const long long live = g_live.fetch_add((long long)fc->bytes) + (long long)fc->bytes;
    if (live > (long long)kBudget) g_over.fetch_add(1);
    long long pk = g_peak.load();
    while (live > pk && !g_peak.compare_exchange_weak(pk, live)) {
    }
    fc->rho.assign((size_t)c->nx * c->ny * c->nz, 0.0);
    fc->p.assign(fc->rho.size(), 0.0);
    g_open.fetch_add(1);
    *out = fc;
    return PP_OK;
}

int set_density(void*, void* cs, const double* rho)
{
    auto* fc = static_cast<FakeCase*>(cs);
    std::memcpy(fc->rho.data(), rho, fc->rho.size() * sizeof(double));
    fc->have_density = true;
    return PP_OK;
}

int solve(void*, void* cs, const double* rhs, double* p_out, pp_stats* st)
{
    auto* fc = static_cast<FakeCase*>(cs);
    thread_local std::mt19937 rng(std::hash<std::thread::id>{}(std::this_thread::get_id()));
    std::this_thread::sleep_for(std::chrono::microseconds(std::uniform_int_distribution<int>(0, 1500)(rng)));
    // "solution": the request's tag (rhs[0]) plus the case's density tag; the
    // previous pressure (warm start) is kept as the case's state
    const double v = rhs[0] + fc->rho[0];
    for (double& x : fc->p) x = v;
    if (p_out) p_out[0] = v;
    std::memset(st, 0, sizeof(*st));
    st->iters = 1;
    return PP_OK;
}

void close_case(void*, void* cs)
{
    auto* fc = static_cast<FakeCase*>(cs);
    g_live.fetch_sub((long long)fc->bytes);
    g_close.fetch_add(1);
    delete fc;
}

const char* err(void*, void*) { return "fake backend"; }

}  // namespace

int main()
{
    pp_backend be{nullptr, fp, open_case, set_density, solve, close_case, err};
    pp_server_config sc{kBudget, 6};
    pp_server srv = nullptr;
    if (pp_server_create(&sc, &be, &srv) != PP_OK) { std::fprintf(stderr, "create failed\n"); return 2; }

    const int kCases = 24, kThreads = 4, kPerThread = 120;
    const int grids[3][3] = {{8, 8, 16}, {16, 16, 32}, {32, 32, 64}};
    struct Req {
        long long id = 0;
        std::vector<double> rho, rhs, out;
        double expect = 0.0;
    };
    std::vector<std::vector<Req>> reqs(kThreads);
    std::atomic<int> failures{0};

    auto submitter = [&](int t) {
        std::mt19937 rng(1234 + t);
        reqs[t].resize(kPerThread);
        for (int k = 0; k < kPerThread; ++k) {
            Req& r = reqs[t][k];
            const int cid = std::uniform_int_distribution<int>(0, kCases - 1)(rng);
            const int* g = grids[cid % 3];
            pp_config cfg{};
            cfg.nx = g[0]; cfg.ny = g[1]; cfg.nz = g[2]; cfg.h = 1.0 / g[0]; cfg.mode = PP_FP32_REFINED; cfg.tol = 1e-8;
            const size_t n = (size_t)g[0] * g[1] * g[2];
            // every request brings its case's density (a case may have been evicted
            // in between); its tag is the case id
            r.rho.assign(n, (double)cid * 1000.0);
            r.rhs.assign(n, (double)(t * 100000 + k));
            r.out.assign(1, -1.0);
            r.expect = r.rhs[0] + r.rho[0];
            if (pp_server_submit(srv, cid, &cfg, r.rho.data(), r.rhs.data(), r.out.data(), &r.id) != PP_OK)
                failures.fetch_add(1);
            if (k % 7 == 0) std::this_thread::sleep_for(std::chrono::microseconds(300));
        }
        for (int k = 0; k < kPerThread; ++k) {
            pp_request_result res{};
            // untimed wait: this toolchain's ThreadSanitizer does not intercept the clock-based
            // condition wait behind a timed one and would report the mutex as locked twice
            if (pp_server_wait(srv, reqs[t][k].id, -1.0, &res) != PP_OK || res.status != PP_OK ||
                reqs[t][k].out[0] != reqs[t][k].expect)
                failures.fetch_add(1);
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < kThreads; ++t) th.emplace_back(submitter, t);
    // concurrent statistics readers
    std::atomic<bool> done{false};
    std::thread reader([&] {
        while (!done.load()) {
            pp_server_stats st{};
            pp_server_get_stats(srv, &st);
            if (st.resident_bytes > kBudget) failures.fetch_add(1);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    for (auto& x : th) x.join();
    done = true;
    reader.join();
    pp_server_stats st{};
    pp_server_get_stats(srv, &st);
    pp_server_destroy(srv);
    std::printf("completed %lld succeeded %lld evictions %lld max_running %d peak_live %lld over_budget %lld "
                "opened %lld closed %lld failures %d\n",
                st.completed, st.succeeded, st.evictions, st.max_running, g_peak.load(), g_over.load(), g_open.load(),
                g_close.load(), failures.load());
    const bool ok = failures.load() == 0 && g_over.load() == 0 && st.completed == kThreads * kPerThread &&
                    st.evictions > 0 && g_open.load() == g_close.load() && g_live.load() == 0;
    return ok ? 0 : 1;
}
