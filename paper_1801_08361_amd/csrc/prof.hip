// Optional per-kernel timing: when enabled, every library launch is
// bracketed by two HIP events recorded on the launching stream, and the
// elapsed times are summed per kernel name on request.
#include <string.h>

#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace rl {

namespace {
struct Span {
    hipEvent_t a, b;
};
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::unordered_map<std::string, std::vector<Span>> spans;
    std::vector<Span> pool;
};
Profiler &prof()
{
    static Profiler p;
    return p;
}
}  // namespace

bool prof_on() { return prof().on; }

void *prof_begin(const char *name, hipStream_t s)
{
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (!P.on) return nullptr;
    Span sp;
    if (!P.pool.empty()) {
        sp = P.pool.back();
        P.pool.pop_back();
    } else {
        if (hipEventCreate(&sp.a) != hipSuccess) return nullptr;
        if (hipEventCreate(&sp.b) != hipSuccess) {
            (void)hipEventDestroy(sp.a);
            return nullptr;
        }
    }
    if (hipEventRecord(sp.a, s) != hipSuccess) {
        P.pool.push_back(sp);
        return nullptr;
    }
    P.spans[name].push_back(sp);
    return (void *)1;
}

void prof_end(const char *name, void *tok, hipStream_t s)
{
    if (!tok) return;
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    auto &v = P.spans[name];
    if (!v.empty()) (void)hipEventRecord(v.back().b, s);
}

}  // namespace rl

using namespace rl;

extern "C" int reloc_profile_enable(int on)
{
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    P.on = on != 0;
    return RELOC_OK;
}

extern "C" int reloc_profile_reset(void)
{
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    RL_HIP(hipDeviceSynchronize());
    for (auto &kv : P.spans)
        for (auto &sp : kv.second) P.pool.push_back(sp);
    P.spans.clear();
    return RELOC_OK;
}

extern "C" int reloc_profile_read(const char *kernel, double *total_ms, int64_t *launches)
{
    if (!kernel || !total_ms || !launches) return RELOC_E_ARG;
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    *total_ms = 0.0;
    *launches = 0;
    auto it = P.spans.find(kernel);
    if (it == P.spans.end()) return RELOC_OK;
    for (auto &sp : it->second) {
        RL_HIP(hipEventSynchronize(sp.b));
        float ms = 0.0f;
        RL_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
        *total_ms += ms;
        *launches += 1;
    }
    return RELOC_OK;
}

extern "C" int reloc_profile_kernels(char *names, int32_t cap)
{
    if (!names || cap < 1) return RELOC_E_ARG;
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    std::string all;
    for (auto &kv : P.spans) {
        if (!all.empty()) all += ",";
        all += kv.first;
    }
    int n = (int)all.size() < cap - 1 ? (int)all.size() : cap - 1;
    memcpy(names, all.data(), (size_t)n);
    names[n] = 0;
    return RELOC_OK;
}
