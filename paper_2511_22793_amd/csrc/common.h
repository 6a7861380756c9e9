// Internal declarations shared by the HIP translation units of libgsparc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/gsparc.h"

namespace gs {

// Per-Gaussian projected record read by the blend kernels (48 bytes).
// Centre and inverse projected covariance stay in FP64: on gfx950 an FP64
// FMA issues at the same rate as an unpacked FP32 FMA, and FP64 removes the
// centre-rounding error that an FP32 pixel coordinate near 360 would carry.
struct alignas(16) GRec {
    double px, py;      // pixel-space centre
    double ca, cb, cc;  // conic: inverse of Sigma' (a, b; b, c)
    float sigma;        // opacity
    float att;          // attenuation 1 / max(d, r_near)^p
};
static_assert(sizeof(GRec) == 48, "GRec layout");

// culling status (same codes as the public documentation)
enum : uint32_t { ST_VISIBLE = 0, ST_NEAR = 1, ST_FAINT = 2, ST_OFFGRID = 3, ST_INVALID = 4 };

// per-query flag words
enum : int { FL_NVIS = 0, FL_PAIRS = 1, FL_OVERFLOW = 2, FL_INVALID = 3, FL_PUSED = 4, FL_WORDS = 16 };

// One blend job: a prepared workspace, its attribute sets and output.
struct BlendJob {
    const GRec* rec;
    size_t s_rec;
    const uint32_t* plist;
    size_t s_plist;
    const uint2* ranges;
    size_t s_ranges;
    const float* attr;
    int64_t a_stride;
    int Fc, C, H, W, tw, th, TX, T, cg, ncg, nsets, shared_geo;
    float amin, amax, tmin;
    float* out;
    float* T_final;
    uint32_t* n_last;
    uint32_t* n_contrib;
    size_t s_pix;
    uint32_t item_begin;  // first work item of this job in a persistent launch
    int query0;           // index of the job's first query in the batch
    // training loss fused into the output stage (k_blend only; null = off):
    // reads the target at each written element, writes lscale (out - tgt)
    // to dpart (when set), and each wave stores its sums of out, of tgt and
    // of (out - tgt)^2 per (set, channel component) to
    // lpart[((set * F*c + ch) * 3 + slot) * lnp + tile * waves + wave]
    // (no atomics: a few hundred workgroups add into every channel)
    const float* tgt;
    float* dpart;
    float* lpart;
    int lnp;
    float lscale;
};

// Offset of channel component ch (0 <= ch < F*C) of pixel pix inside one
// set's spectrum [F][H][W][C], for C = 1 << cs (cs = 0: real, 1: complex).
__device__ __forceinline__ size_t spec_offset(int ch, size_t pix, int cs, size_t HW)
{
    return (size_t)(ch & ~cs) * HW + (size_t)(ch & cs) + (pix << cs);
}

// Butterfly reduce-scatter of V values over the 64 lanes of a wave.  On
// return x[0] of lane l holds the wave total of value (l >> (6 - log2 V)).
// Each stage exchanges half of the remaining values with the lane at xor
// distance M; all sizes are compile-time so the arrays stay in registers.
template <int V, int M>
__device__ __forceinline__ void reduce_scatter_step(float* x, int lane)
{
    if constexpr (M >= 1) {
        if constexpr (V > 1) {
            constexpr int half = V / 2;
            const bool up = (lane & M) != 0;
#pragma unroll
            for (int i = 0; i < half; ++i) {
                const float send = up ? x[i] : x[i + half];
                const float keep = up ? x[i + half] : x[i];
                x[i] = keep + __shfl_xor(send, M, 64);
            }
            reduce_scatter_step<half, M / 2>(x, lane);
        } else {
            x[0] += __shfl_xor(x[0], M, 64);
            reduce_scatter_step<1, M / 2>(x, lane);
        }
    }
}

template <int V>
__device__ __forceinline__ void wave_reduce_scatter(float* x, int lane)
{
    reduce_scatter_step<V, 32>(x, lane);
}

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;  // keys per sort workgroup
// Wide sort workgroups: 16 waves, so 4x the keys per block.  A block's
// output runs per digit are 4x longer (fewer partly written lines) and the
// digit-by-block count matrix 4x smaller; taken while the launch still has
// at least SORT_WIDE_MIN_BLOCKS workgroups.
constexpr int SORT_WIDE_WAVES = 16;
constexpr int SORT_WIDE_MIN_BLOCKS = 256;
// at most this many blocks per query: the depth sort's scatter scans the
// per-block counts itself instead of a separate scan launch
constexpr int SORT_FUSED_SCAN_BLOCKS = 64;
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
// tile ids up to this many bits are sorted in one counting pass
constexpr int TILE_PASS_MAX_BITS = 10;
// keys per thread of that pass: large blocks keep its digit-by-block count
// matrix (up to 1024 rows) small
constexpr int TILE_PASS_ITEMS = 32;
// keys per thread of that pass in wide workgroups (2x the keys per block
// within the 128 registers a 1024-thread workgroup allows)
constexpr int TILE_PASS_WIDE_ITEMS = 16;

// Byte layout of the caller's workspace (all sub-buffers 256-byte aligned,
// each an array over queries with the given stride).
struct Layout {
    int n, nq, H, W, tw, th, TX, TY, T;
    int64_t cap;          // pair capacity per query
    int rank_bits;        // bits of the depth rank inside a pair key
    int tile_bits;        // bits of the tile id inside a pair key
    int pair_passes;      // radix passes over pair keys
    int tile_blocks;      // workgroups of the single tile pass
    int sort_blocks;      // max sort workgroups for n keys
    int pair_blocks;      // max sort workgroups for cap keys
    int sort_wide;        // depth sort in wide workgroups
    int pair_wide;        // pair sorts (tile pass included) in wide workgroups
    size_t flags, rec, rect, status, tinfo, keys_a, keys_b, vals_a, vals_b, partial;
    size_t pkeys_a, pkeys_b, plist, ranges, counts, totals, T_final, n_last, n_contrib, g2d, live, gacc, wtot;
    size_t s_flags, s_rec, s_rect, s_status, s_tinfo, s_keys, s_partial, s_pkeys, s_plist, s_ranges,
        s_counts, s_totals, s_pix, s_g2d, s_live, s_gacc, s_wtot;
    size_t total;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
gs_status make_layout(int32_t n, int32_t nq, const gs_grid* g, const gs_params* p, Layout* L);

// kernel launchers (stream-ordered, no synchronisation)
void launch_fill_u32(uint32_t* p, size_t count, size_t q_stride, int nq, uint32_t v, hipStream_t s);
constexpr int FILL_SEGS = 8;
struct FillSegs {
    uint32_t* p[FILL_SEGS];
    size_t count[FILL_SEGS];
    int n;
};
void launch_fill_segs(const FillSegs& f, hipStream_t s);  // zero-fills f.n buffers (words)

// Side streams of a device for the library's fork/join launch sequences
// (default priority, non-blocking), created once per device and kept until
// the process ends, with the events that fork them from and join them into
// a caller's stream.  Enqueueing on them is serialised by lanes_mutex().
constexpr int LANE_SIDE = 3;
struct Lanes {
    hipStream_t side[LANE_SIDE];
    hipEvent_t fork;
    hipEvent_t join[LANE_SIDE];
    bool ready;
};
gs_status lanes_init(int dev);           // creates device dev's lanes (call outside graph capture)
const Lanes* side_lanes(hipStream_t s);  // the current device's lanes, created unless s is being
                                         // captured; null: the caller runs serially
std::mutex& lanes_mutex();
// fills [0, min(per_query * n_dev[q], max_count)) of each query, n_dev read
// on the device
void launch_fill_dev(uint32_t* p, size_t max_count, size_t q_stride, int nq, const uint32_t* n_dev, size_t n_stride,
                     uint32_t per_query, hipStream_t s);
void launch_project(const gs_scene& sc, const gs_queries& qs, const gs_grid& g, const gs_params& p,
                    const Layout& L, char* ws, hipStream_t s);
void launch_depth_sort(const Layout& L, char* ws, hipStream_t s);
void launch_binning(const Layout& L, char* ws, hipStream_t s);
gs_status launch_blend(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws, float* out,
                       hipStream_t s, const float* tgt = nullptr, float* dpart = nullptr, float* lpart = nullptr,
                       float lscale = 0.0f);
// loss accumulators [set][F*c][3] from the per-wave sums of the fused
// blend (np partials per entry), then loss, spatial means and the
// channel-mean gradient term from them (loss.hip)
void launch_loss_parts(int n_sets, int Fc, int C, int np, const float* part, float* acc, hipStream_t s);
void launch_loss_finish(int n_sets, int Fc, int C, size_t HW, float lambda, const float* acc, float* h_hat,
                        float* loss, float* mean_grad, hipStream_t s);
void launch_live(const gs_params& p, const Layout& L, char* ws, uint32_t* list, size_t s_list, uint32_t* count,
                 hipStream_t s);
gs_status check_forward(const gs_scene* sc, const gs_attrs* a, const gs_queries* qs, const gs_grid* g,
                        const gs_params* p, const float* spectrum, const void* ws, size_t ws_bytes, Layout* L);
void enqueue_prepare(const gs_scene* scene, const gs_queries* queries, const gs_grid* grid, const gs_params* prm,
                     const Layout& L, char* ws, hipStream_t s);
int choose_chan_group(int Fc, int requested);
BlendJob make_blend_job(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws, float* out);
void launch_blend_persist(const BlendJob* jobs, int njobs, uint32_t total, uint32_t* counter,
                          unsigned long long* done_ts, int workgroups, int block, hipStream_t s);
void launch_stamp(unsigned long long* ts, hipStream_t s);
hipError_t persist_occupancy(int block, int* per_cu);
// Upstream gradient of the backward: dout alone; or, with mean_grad,
// dout + mean_grad (dout = the elementwise part of the L2 loss gradient),
// or scale (out - target) + mean_grad when target is set.
struct BwdUpstream {
    const float* dout;
    const float* target;
    const float* mean_grad;
    float scale;
};
// kernel timing (timing.hip): event pairs around launches when enabled
enum { TK_BLEND = GS_TIMER_BLEND, TK_BLEND_BWD = GS_TIMER_BLEND_BWD, TK_TRAIN = GS_TIMER_TRAIN, TK_COUNT = 3 };
bool timing_on();
void timing_begin(int kernel, hipStream_t s, void** token);
void timing_end(void* token, hipStream_t s);
gs_status launch_blend_bwd(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws,
                           const float* out, const BwdUpstream& up, float* d_attr, hipStream_t s);
// the shared-geometry compositing / backward over the groups whose walk is
// longer than min_walk entries only (the long-walk part of the fused
// training pass); the per-pair geometric accumulators folded per Gaussian
void launch_blend_sg_long(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws, float* out,
                          int min_walk, hipStream_t s);
void launch_blend_bwd_sg_long(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws,
                              const float* out, const float* target, const float* mean_grad, float scale,
                              const float* gscale, float* d_attr, int min_walk, float* lacc, hipStream_t s);
void launch_geo_fold(const Layout& L, char* ws, hipStream_t s);
void launch_project_bwd(const gs_scene& sc, const gs_queries& qs, const gs_grid& g, const gs_params& p,
                        const Layout& L, char* ws, float* d_mean, float* d_log_scale, float* d_quat, float* d_opac,
                        hipStream_t s);

}  // namespace gs

#define GS_CHECK_LAUNCH()                                  \
    do {                                                   \
        if (hipGetLastError() != hipSuccess) return GS_ERR_HIP; \
    } while (0)
