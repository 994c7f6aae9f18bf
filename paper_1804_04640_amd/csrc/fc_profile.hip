// Opt-in launch profiling: HIP events around each kernel launch, aggregated
// per kernel instance together with the algorithmic work it performed.
#include <atomic>
#include <cstring>
#include <map>

#include "fc_internal.h"

namespace fc {

namespace {
struct Pending {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
    double bytes = 0, ops = 0;
    bool closed = false;
    bool agg = false;        // counted in the per-kernel aggregates
    double *sink = nullptr;  // device-time sum of the thread that launched it
};
struct Agg {
    int64_t launches = 0;
    double ms = 0, bytes = 0, ops = 0;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, Agg> g_agg;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// caller holds g_mu
void drain() {
    for (Pending &p : g_pending) {
        if (!p.a || !p.b || !p.closed) continue;
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            if (p.agg) {
                Agg &g = g_agg[p.name];
                g.launches += 1;
                g.ms += ms;
                g.bytes += p.bytes;
                g.ops += p.ops;
            }
            if (p.sink) *p.sink += ms;
        } else {
            (void)hipGetLastError();
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}
}  // namespace

static thread_local bool t_capturing = false;
static thread_local double *t_sink = nullptr;

bool profiling_on() { return g_on.load(std::memory_order_relaxed); }

void set_capturing(bool on) { t_capturing = on; }

void device_time_begin(double *sink) { t_sink = sink; }

void device_time_end() {
    std::lock_guard<std::mutex> lk(g_mu);
    drain();
    t_sink = nullptr;
}

ProfScope::ProfScope(const char *name, hipStream_t s, double alg_bytes, double alg_ops) {
    const bool agg = profiling_on();
    if ((!agg && !t_sink) || t_capturing) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_pending.size() > 4096) drain();
    Pending p;
    p.name = name;
    p.a = get_event();
    p.b = get_event();
    p.bytes = alg_bytes;
    p.ops = alg_ops;
    p.agg = agg;
    p.sink = t_sink;
    if (p.a) (void)hipEventRecord(p.a, s);
    g_pending.push_back(p);
    slot = (int)g_pending.size() - 1;
}

void ProfScope::end(hipStream_t s) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (slot < (int)g_pending.size()) {
        Pending &p = g_pending[(size_t)slot];
        if (p.b) (void)hipEventRecord(p.b, s);
        p.closed = true;
    }
    slot = -1;
}

}  // namespace fc

using namespace fc;

extern "C" int fc_profile_enable(int on) {
    g_on.store(on != 0);
    return FC_OK;
}

extern "C" int fc_profile_read(fc_kernel_stat *out, int32_t cap, int32_t reset) {
    std::lock_guard<std::mutex> lk(g_mu);
    drain();
    int32_t i = 0;
    for (auto &kv : g_agg) {
        if (out && i < cap) {
            fc_kernel_stat &o = out[i];
            std::memset(&o, 0, sizeof o);
            std::strncpy(o.name, kv.first.c_str(), sizeof o.name - 1);
            o.launches = kv.second.launches;
            o.ms = kv.second.ms;
            o.alg_bytes = kv.second.bytes;
            o.alg_ops = kv.second.ops;
        }
        ++i;
    }
    if (reset) g_agg.clear();
    return i;
}
