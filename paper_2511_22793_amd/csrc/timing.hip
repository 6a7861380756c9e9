// Kernel timing for benchmarks: HIP event pairs recorded on the launching
// stream around each launch of the timed kernels, summed on request.
#include <mutex>

#include "common.h"

namespace gs {

namespace {
struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double total_ms = 0.0;
    int64_t launches = 0;
};
std::mutex g_mu;
bool g_on = false;
Timer g_timers[TK_COUNT];
}  // namespace

bool timing_on() { return g_on; }

void timing_begin(int kernel, hipStream_t s, void** token)
{
    *token = nullptr;
    if (!g_on) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(a, s);
    std::lock_guard<std::mutex> lk(g_mu);
    g_timers[kernel].pending.push_back({a, b});
    *token = (void*)b;
}

void timing_end(void* token, hipStream_t s)
{
    if (token) (void)hipEventRecord((hipEvent_t)token, s);
}

}  // namespace gs

using namespace gs;

extern "C" {

gs_status gs_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return GS_OK;
}

gs_status gs_timing_read(int32_t kernel, double* total_ms, int64_t* launches)
{
    if (kernel < 0 || kernel >= TK_COUNT || !total_ms || !launches) return GS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    Timer& t = g_timers[kernel];
    for (auto& p : t.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.second) != hipSuccess || hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
            return GS_ERR_HIP;
        t.total_ms += ms;
        t.launches += 1;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    t.pending.clear();
    *total_ms = t.total_ms;
    *launches = t.launches;
    t.total_ms = 0.0;
    t.launches = 0;
    return GS_OK;
}

}  // extern "C"
