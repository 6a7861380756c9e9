// Batched serving: the prepare steps of every job, spread over a few
// streams so that small jobs' launches overlap, then one persistent blend
// launch over all jobs' (query, channel group, tile) items.
#include <mutex>

#include "common.h"

namespace gs {

constexpr size_t PLAN_HEAD = 256;  // work counter, then the job table

// Prepare lanes: the caller's stream plus the LANE_SIDE side streams of the
// device, forked from the caller's stream with an event and joined back
// before the blend, so the whole run stays one capturable sequence.
constexpr int LANES_MAX_DEVICES = 64;
std::mutex g_lanes_mu;
Lanes g_lanes[LANES_MAX_DEVICES] = {};

std::mutex& lanes_mutex() { return g_lanes_mu; }

gs_status lanes_init(int dev)
{
    if (dev < 0 || dev >= LANES_MAX_DEVICES) return GS_ERR_CAPACITY;
    std::lock_guard<std::mutex> lk(g_lanes_mu);
    Lanes& l = g_lanes[dev];
    if (l.ready) return GS_OK;
    for (int i = 0; i < LANE_SIDE; ++i) {
        if (hipStreamCreateWithFlags(&l.side[i], hipStreamNonBlocking) != hipSuccess) return GS_ERR_HIP;
        if (hipEventCreateWithFlags(&l.join[i], hipEventDisableTiming) != hipSuccess) return GS_ERR_HIP;
    }
    if (hipEventCreateWithFlags(&l.fork, hipEventDisableTiming) != hipSuccess) return GS_ERR_HIP;
    l.ready = true;
    return GS_OK;
}

const Lanes* side_lanes(hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= LANES_MAX_DEVICES) return nullptr;
    {
        // (a device's lanes never change once ready)
        std::lock_guard<std::mutex> lk(g_lanes_mu);
        if (g_lanes[dev].ready) return &g_lanes[dev];
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    if (lanes_init(dev) != GS_OK) return nullptr;
    return &g_lanes[dev];
}

static gs_status build_table(const gs_batch_job* jobs, int n_jobs, std::vector<BlendJob>& table, gs_batch_info* info)
{
    if (!jobs || n_jobs < 1 || n_jobs > (1 << 16)) return GS_ERR_INVALID_ARG;
    table.resize(n_jobs);
    uint64_t items = 0;
    int64_t nq_total = 0;
    int block = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const gs_batch_job& b = jobs[j];
        Layout L;
        gs_status st = check_forward(&b.scene, &b.attrs, &b.queries, &b.grid, &b.params, b.spectrum, b.workspace,
                                     b.workspace_bytes, &L);
        if (st != GS_OK) return st;
        const int C = b.attrs.is_complex ? 2 : 1;
        const int Fc = b.attrs.n_chan * C;
        int cg = choose_chan_group(Fc, b.params.chan_group);
        if (cg > 32) cg = 32;  // the persistent kernel carries groups up to 32
        BlendJob J = make_blend_job(b.attrs, b.params, L, L.nq, (char*)b.workspace, b.spectrum);
        J.cg = cg;
        J.ncg = Fc / cg;
        J.item_begin = (uint32_t)items;
        J.query0 = (int)nq_total;
        items += (uint64_t)L.T * (uint64_t)J.ncg * (uint64_t)L.nq;
        nq_total += L.nq;
        if (items >= 0xFFFFFFFFull || nq_total > 0x7FFFFFFF) return GS_ERR_CAPACITY;
        block = std::max(block, L.tw * L.th);
        table[j] = J;
    }
    if (info) {
        info->items = (int64_t)items;
        info->n_queries = (int32_t)nq_total;
        info->block = block;
        info->workgroups = 0;
        info->reserved = 0;
    }
    return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" {

size_t gs_batch_plan_bytes(int32_t n_jobs)
{
    if (n_jobs < 1) return 0;
    return PLAN_HEAD + align256((size_t)n_jobs * sizeof(BlendJob));
}

gs_status gs_batch_plan(const gs_batch_job* jobs, int32_t n_jobs, void* plan, size_t plan_bytes, gs_batch_info* info,
                        void* stream)
{
    if (!info) return GS_ERR_INVALID_ARG;
    std::vector<BlendJob> table;
    gs_status st = build_table(jobs, n_jobs, table, info);
    if (st != GS_OK) return st;
    if (!plan || ((uintptr_t)plan & 255) || plan_bytes < gs_batch_plan_bytes(n_jobs)) return GS_ERR_WORKSPACE;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return GS_ERR_HIP;
    if (persist_occupancy(info->block, &per_cu) != hipSuccess) return GS_ERR_HIP;
    st = lanes_init(dev);
    if (st != GS_OK) return st;
    info->workgroups = std::max(1, cus * std::max(1, per_cu));
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync((char*)plan + PLAN_HEAD, table.data(), table.size() * sizeof(BlendJob),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return GS_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GS_ERR_HIP;
    return GS_OK;
}

gs_status gs_batch_run(const gs_batch_job* jobs, int32_t n_jobs, void* plan, size_t plan_bytes, int32_t workgroups,
                       uint64_t* timestamps, void* stream)
{
    std::vector<BlendJob> table;
    gs_batch_info info;
    gs_status st = build_table(jobs, n_jobs, table, &info);
    if (st != GS_OK) return st;
    if (!plan || ((uintptr_t)plan & 255) || plan_bytes < gs_batch_plan_bytes(n_jobs)) return GS_ERR_WORKSPACE;
    if (workgroups < 1 || workgroups > (1 << 20)) return GS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    uint32_t* counter = (uint32_t*)plan;
    unsigned long long* ts = (unsigned long long*)timestamps;
    launch_fill_u32(counter, 1, 0, 1, 0u, s);
    if (ts) {
        launch_fill_u32((uint32_t*)ts, 2 * ((size_t)info.n_queries + 3), 0, 1, 0u, s);
        launch_stamp(ts, s);
    }
    std::vector<Layout> lay(n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        const gs_batch_job& b = jobs[j];
        st = make_layout(b.scene.n, b.queries.count, &b.grid, &b.params, &lay[j]);
        if (st != GS_OK) return st;
    }
    const Lanes* ln = n_jobs > 1 ? side_lanes(s) : nullptr;
    if (!ln) {
        for (int j = 0; j < n_jobs; ++j) {
            const gs_batch_job& b = jobs[j];
            enqueue_prepare(&b.scene, &b.queries, &b.grid, &b.params, lay[j], (char*)b.workspace, s);
        }
    } else {
        // each job to the lane with the least projected work so far
        // (Gaussians x queries), in job order
        std::lock_guard<std::mutex> lk(g_lanes_mu);
        const int nl = std::min(n_jobs, LANE_SIDE + 1);
        double load[LANE_SIDE + 1] = {};
        if (hipEventRecord(ln->fork, s) != hipSuccess) return GS_ERR_HIP;
        for (int i = 1; i < nl; ++i)
            if (hipStreamWaitEvent(ln->side[i - 1], ln->fork, 0) != hipSuccess) return GS_ERR_HIP;
        for (int j = 0; j < n_jobs; ++j) {
            const gs_batch_job& b = jobs[j];
            int best = 0;
            for (int i = 1; i < nl; ++i)
                if (load[i] < load[best]) best = i;
            load[best] += (double)b.scene.n * (double)b.queries.count;
            enqueue_prepare(&b.scene, &b.queries, &b.grid, &b.params, lay[j], (char*)b.workspace,
                            best ? ln->side[best - 1] : s);
        }
        for (int i = 1; i < nl; ++i) {
            if (hipEventRecord(ln->join[i - 1], ln->side[i - 1]) != hipSuccess) return GS_ERR_HIP;
            if (hipStreamWaitEvent(s, ln->join[i - 1], 0) != hipSuccess) return GS_ERR_HIP;
        }
    }
    if (ts) launch_stamp(ts + 2 + info.n_queries, s);
    launch_blend_persist((const BlendJob*)((char*)plan + PLAN_HEAD), n_jobs, (uint32_t)info.items, counter,
                         ts ? ts + 1 : nullptr, workgroups, info.block, s);
    if (ts) launch_stamp(ts + 1 + info.n_queries, s);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status gs_wall_clock_khz(int32_t* khz)
{
    if (!khz) return GS_ERR_INVALID_ARG;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return GS_ERR_HIP;
    *khz = v;
    return GS_OK;
}

}  // extern "C"
