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
    hipEvent_t a, b;   // around the launch
    hipEvent_t c, d;   // a bare pair recorded right after it: the markers' own cost
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

// A timed pass starts with one wavefront that waits a fixed wall-clock time
// (the 100 MHz real-time counter), long enough for the host to queue every
// launch of the pass behind it, so that no span includes time in which the
// GPU waited for the host to queue the next one. The loop also stops after
// ticks / 10 sleeps (each sleep lasts far more than 10 ticks), so it ends
// whatever the counter does.
__global__ void __launch_bounds__(64) k_prof_delay(uint64_t ticks)
{
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (uint64_t i = 0; i < ticks / 10 && __builtin_amdgcn_s_memrealtime() - t0 < ticks; ++i)
        __builtin_amdgcn_s_sleep(32);
}

void prof_delay(hipStream_t s, int launches)
{
    // 40 us of host time per launch and its four events, at 100 ticks per us
    const uint64_t ticks = (uint64_t)(launches < 1 ? 1 : launches) * 40ull * 100ull;
    hipLaunchKernelGGL(k_prof_delay, dim3(1), dim3(64), 0, s, ticks);
}

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
        if (hipEventCreate(&sp.c) != hipSuccess) {
            (void)hipEventDestroy(sp.a);
            (void)hipEventDestroy(sp.b);
            return nullptr;
        }
        if (hipEventCreate(&sp.d) != hipSuccess) {
            (void)hipEventDestroy(sp.a);
            (void)hipEventDestroy(sp.b);
            (void)hipEventDestroy(sp.c);
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
    if (!v.empty()) {
        (void)hipEventRecord(v.back().b, s);
        (void)hipEventRecord(v.back().c, s);
        (void)hipEventRecord(v.back().d, s);
    }
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
        RL_HIP(hipEventSynchronize(sp.d));
        float ms = 0.0f, m0 = 0.0f;
        RL_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
        RL_HIP(hipEventElapsedTime(&m0, sp.c, sp.d));
        *total_ms += (double)ms - (double)m0;
        *launches += 1;
    }
    return RELOC_OK;
}

extern "C" int reloc_profile_read_raw(const char *kernel, double *bracket_ms, double *pair_ms, int64_t *launches)
{
    if (!kernel || !bracket_ms || !pair_ms || !launches) return RELOC_E_ARG;
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    *bracket_ms = *pair_ms = 0.0;
    *launches = 0;
    auto it = P.spans.find(kernel);
    if (it == P.spans.end()) return RELOC_OK;
    for (auto &sp : it->second) {
        RL_HIP(hipEventSynchronize(sp.d));
        float ms = 0.0f, m0 = 0.0f;
        RL_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
        RL_HIP(hipEventElapsedTime(&m0, sp.c, sp.d));
        *bracket_ms += ms;
        *pair_ms += m0;
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
