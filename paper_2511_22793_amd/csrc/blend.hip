// Front-to-back compositing of the per-tile depth-ordered lists (Eq. (3),
// Sec. 4.2; the per-pixel loop of Algorithm 1).  One workgroup per
// (tile, channel group, query), one thread per pixel.  Batches of the
// tile's list are staged in LDS; every thread walks the batch in order:
//   dx, dy      pixel-centre offset, azimuth wrapped into [-W/2, W/2)  (FP64)
//   q           conic quadratic form                                  (FP64)
//   G           exp(-q/2) via v_exp_f32                               (FP32)
//   alpha       min(alpha_max, opacity G); skip when alpha < alpha_min
//   stop        before the Gaussian that would take T below T_min
//   out_f      += T alpha a_i v_{i,f} for the group's channels        (FP32)
// The whole workgroup leaves the list once every pixel has stopped.
// The attribute row of the current Gaussian is wave-uniform and is read
// through scalar loads.
#include <type_traits>

#include "common.h"

namespace gs {

constexpr double LOG2E = 1.4426950408889634;

// Attribute rows are read-only for the whole launch: reading them through a
// constant-address-space pointer lets the wave-uniform row go through the
// scalar cache (s_load) whatever the kernel stores elsewhere.
typedef __attribute__((address_space(4))) const float CFloat;
// The other buffers are global memory; naming the address space keeps the
// persistent kernel (which reads its pointers from a table) off flat
// instructions.
#define GLOBAL_AS __attribute__((address_space(1)))

// LDS batch of one tile's list (declared once per kernel, so that the
// channel-group instantiations of one kernel share it).
struct BlendLds {
    double px[256], py[256], ca[256], cb[256], cc[256];
    float sig[256], att[256];
    uint32_t g[256];
    // per wave: pixel weights of a run of 16 entries (matrix-core path), then
    // the output transpose (64 pixels x 17)
    float w[4][16][68];
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One (tile, channel group, set) of a blend job; every thread of the
// workgroup must call it (it synchronises).  Threads beyond the tile's pixel
// count idle.
// The buffers are passed as restrict parameters so that, once inlined, the
// attribute rows are known not to alias the stores and load through the
// scalar cache.
template <int CG, bool FUSE = false>
__device__ __forceinline__ void blend_tile_impl(const BlendJob& J, BlendLds& S, int tile, int cg, int set,
                                                const GRec* __restrict__ rec, const uint32_t* __restrict__ plist,
                                                const uint2* __restrict__ ranges, const float* __restrict__ attr,
                                                float* __restrict__ out, float* __restrict__ T_final,
                                                uint32_t* __restrict__ n_last, uint32_t* __restrict__ n_contrib)
{
    const int q = J.shared_geo ? 0 : set;  // geometry query
    const int nthr = J.tw * J.th;
    const int txi = tile % J.TX, tyi = tile / J.TX;
    const int lx = threadIdx.x % J.tw, ly = threadIdx.x / J.tw;
    const int col = txi * J.tw + lx, row = tyi * J.th + ly;
    const bool inside = (int)threadIdx.x < nthr && col < J.W && row < J.H;
    uint2 rg;
    {
        const unsigned long long r = ((const GLOBAL_AS unsigned long long*)ranges)[q * J.s_ranges + tile];
        rg.x = (uint32_t)r;
        rg.y = (uint32_t)(r >> 32);
    }
    const double pcx = col + 0.5, pcy = row + 0.5, halfW = 0.5 * J.W;
    const double Wd = (double)J.W;
    rec += q * J.s_rec;
    plist += q * J.s_plist;
    const int Fc = J.Fc;
    const float* A = attr + set * J.a_stride + cg * CG;
    const float amin = J.amin, amax = J.amax, tmin = J.tmin;

    float T = 1.0f;
    uint32_t last = 0, cnt = 0;
    bool done = !inside;
    const size_t HW = (size_t)J.H * J.W, pix = inside ? (size_t)row * J.W + col : 0;
    const int cs = J.C - 1;  // C is 1 or 2
    const size_t obase = (size_t)set * Fc * HW;
    // CG = 16, 32: the channel sums out[p][f] = sum_e w[p][e] v[e][f] of a
    // run of 16 entries go to the FP32 matrix cores (v_mfma_f32_16x16x4_f32,
    // A = the wave's pixel weights from LDS, B = the entries' attribute
    // rows); the walk only produces the weights.  Smaller groups
    // accumulate on the VALU with the row in SGPRs.
    constexpr bool MF = CG == 16 || CG == 32 || CG == 64;
    constexpr int NB = MF ? CG / 16 : 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float acc[MF ? 1 : CG];
    f32x4 macc[MF ? 4 : 1][NB];
    if constexpr (MF) {
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) macc[pb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    } else {
#pragma unroll
        for (int k = 0; k < CG; ++k) acc[k] = 0.0f;
    }

    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += nthr) {
        if (__syncthreads_count(done) == (int)blockDim.x) break;
        const uint32_t i = b0 + threadIdx.x;
        if ((int)threadIdx.x < nthr && i < rg.y) {
            const uint32_t g = ((const GLOBAL_AS uint32_t*)plist)[i];
            const GLOBAL_AS GRec& r = ((const GLOBAL_AS GRec*)rec)[g];
            S.px[threadIdx.x] = r.px;
            S.py[threadIdx.x] = r.py;
            S.ca[threadIdx.x] = r.ca;
            S.cb[threadIdx.x] = r.cb;
            S.cc[threadIdx.x] = r.cc;
            S.sig[threadIdx.x] = r.sigma;
            S.att[threadIdx.x] = r.att;
            S.g[threadIdx.x] = g;
        }
        __syncthreads();
        const int m = (int)min((uint32_t)nthr, rg.y - b0);
        if constexpr (MF) {
            for (int j0 = 0; j0 < m; j0 += 16) {
                if (__ballot(!done) == 0ull) break;  // wave-uniform: all its pixels stopped
                const int jn = min(16, m - j0);
                // B operands of the run, loaded ahead of the walk: lane holds
                // v[entry 4 ks + lane/16][channel 16 nb + lane%16]
                float bv[4][NB];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int e = 4 * ks + (lane >> 4);
                    const bool ev = e < jn;
                    const float* vr = A + (size_t)(ev ? S.g[j0 + e] : 0u) * Fc + (lane & 15);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) bv[ks][nb] = ev ? ((const CFloat*)vr)[16 * nb] : 0.0f;
                }
#pragma unroll 4
                for (int jj = 0; jj < 16; ++jj) {
                    const int j = j0 + jj;
                    float wgt = 0.0f;
                    if (jj < jn && !done) {
                        double dx = pcx - S.px[j];
                        dx += dx >= halfW ? -Wd : (dx < -halfW ? Wd : 0.0);
                        const double dy = pcy - S.py[j];
                        const double qv = S.ca[j] * dx * dx + 2.0 * S.cb[j] * dx * dy + S.cc[j] * dy * dy;
                        const float G = __builtin_amdgcn_exp2f((float)(-0.5 * LOG2E * qv));
                        const float alpha = fminf(amax, S.sig[j] * G);
                        const float Tn = T * (1.0f - alpha);
                        const bool stop = alpha >= amin && Tn < tmin;
                        const bool take = alpha >= amin && !stop;
                        done = stop;
                        wgt = take ? T * alpha * S.att[j] : 0.0f;
                        T = take ? Tn : T;
                        last = take ? b0 + j + 1 - rg.x : last;
                        cnt += take ? 1u : 0u;
                    }
                    S.w[wave][jj][lane] = wgt;
                }
                wave_sync_lds();
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
                    for (int pb = 0; pb < 4; ++pb) {
                        const float a = S.w[wave][4 * ks + (lane >> 4)][16 * pb + (lane & 15)];
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            macc[pb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv[ks][nb], macc[pb][nb], 0, 0, 0);
                    }
                }
                wave_sync_lds();
            }
        } else {
            for (int j = 0; j < m && !done; ++j) {
                // the attribute row is wave-uniform: issue its scalar loads
                // first so that the alpha evaluation below hides their latency
                const uint32_t g = __builtin_amdgcn_readfirstlane(S.g[j]);
                const CFloat* vp = (const CFloat*)(A + (size_t)g * Fc);
                float v[CG];
#pragma unroll
                for (int k = 0; k < CG; ++k) v[k] = vp[k];
                double dx = pcx - S.px[j];
                dx += dx >= halfW ? -Wd : (dx < -halfW ? Wd : 0.0);
                const double dy = pcy - S.py[j];
                const double qv = S.ca[j] * dx * dx + 2.0 * S.cb[j] * dx * dy + S.cc[j] * dy * dy;
                const float G = __builtin_amdgcn_exp2f((float)(-0.5 * LOG2E * qv));
                const float alpha = fminf(amax, S.sig[j] * G);
                const float Tn = T * (1.0f - alpha);
                const bool stop = alpha >= amin && Tn < tmin;
                const bool take = alpha >= amin && !stop;
                done = stop;
                // branch-free update (one basic block, so the row loads issue
                // first): a skipped pair adds zero and keeps T
                const float wgt = take ? T * alpha * S.att[j] : 0.0f;
#pragma unroll
                for (int k = 0; k < CG; ++k) acc[k] = fmaf(wgt, v[k], acc[k]);
                T = take ? Tn : T;
                last = take ? b0 + j + 1 - rg.x : last;
                cnt += take ? 1u : 0u;
            }
        }
    }
    __syncthreads();  // the LDS batch may be reused by the caller's next item
    // the fused loss (FUSE: k_blend with a target): per written element the
    // target, the elementwise gradient part and the three sums,
    // reduce-scattered over the wave (lane 4 k + 0 ends with channel k's
    // totals) and stored per wave
    constexpr bool fuse = FUSE;
    // one of the sums (slot 0: out, 1: tgt, 2: squared error) of V channels
    // from ch0 on
    auto loss_sum = [&](auto vc, float* x, int ch0, int slot) {
        constexpr int V = decltype(vc)::value;
        wave_reduce_scatter<V>(x, lane);
        constexpr int sh = V >= 64 ? 0 : (V == 32 ? 1 : (V == 16 ? 2 : (V == 8 ? 3 : (V == 4 ? 4 : (V == 2 ? 5 : 6)))));
        if ((lane & ((1 << sh) - 1)) == 0) {
            const int ch = ch0 + (lane >> sh);
            J.lpart[(((size_t)set * Fc + ch) * 3 + slot) * J.lnp + (size_t)tile * (nthr >> 6) + wave] = x[0];
        }
    };
    if constexpr (MF) {
        // lane holds out[pixel 16 pb + 4 (lane/16) + r][channel 16 nb + lane%16]:
        // transpose through LDS so that each lane writes its own pixel
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            float* tr = &S.w[wave][0][0];  // [64 pixels][17]
#pragma unroll
            for (int pb = 0; pb < 4; ++pb)
#pragma unroll
                for (int r = 0; r < 4; ++r) tr[(16 * pb + 4 * (lane >> 4) + r) * 17 + (lane & 15)] = macc[pb][nb][r];
            wave_sync_lds();
            if constexpr (fuse) {
                // two 16-value arrays at a time next to the accumulators;
                // the 16 target loads are issued before any store (the
                // buffers are not known not to alias, so a store would
                // order the loads after it)
                const int ch0 = cg * CG + 16 * nb;
                float x[16], y[16];
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    y[k] = inside ? J.tgt[obase + spec_offset(ch0 + k, pix, cs, HW)] : 0.0f;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const size_t idx = obase + spec_offset(ch0 + k, pix, cs, HW);
                    const float o = tr[lane * 17 + k];
                    if (inside) {
                        ((GLOBAL_AS float*)out)[idx] = o;
                        if (J.dpart) J.dpart[idx] = J.lscale * (o - y[k]);
                    }
                    x[k] = inside ? o : 0.0f;
                }
                loss_sum(std::integral_constant<int, 16>{}, x, ch0, 0);
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const float d = tr[lane * 17 + k] - y[k];
                    x[k] = inside ? d * d : 0.0f;
                }
                loss_sum(std::integral_constant<int, 16>{}, x, ch0, 2);
                loss_sum(std::integral_constant<int, 16>{}, y, ch0, 1);
            } else if (inside) {
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int ch = cg * CG + 16 * nb + k;
                    ((GLOBAL_AS float*)out)[obase + spec_offset(ch, pix, cs, HW)] = tr[lane * 17 + k];
                }
            }
            wave_sync_lds();
        }
    } else {
        if constexpr (fuse) {
            float x[CG], y[CG];
#pragma unroll
            for (int k = 0; k < CG; ++k) y[k] = inside ? J.tgt[obase + spec_offset(cg * CG + k, pix, cs, HW)] : 0.0f;
#pragma unroll
            for (int k = 0; k < CG; ++k) {
                const size_t idx = obase + spec_offset(cg * CG + k, pix, cs, HW);
                if (inside) {
                    ((GLOBAL_AS float*)out)[idx] = acc[k];
                    if (J.dpart) J.dpart[idx] = J.lscale * (acc[k] - y[k]);
                }
                x[k] = inside ? (acc[k] - y[k]) * (acc[k] - y[k]) : 0.0f;
            }
            loss_sum(std::integral_constant<int, CG>{}, x, cg * CG, 2);
            loss_sum(std::integral_constant<int, CG>{}, y, cg * CG, 1);
#pragma unroll
            for (int k = 0; k < CG; ++k) x[k] = inside ? acc[k] : 0.0f;
            loss_sum(std::integral_constant<int, CG>{}, x, cg * CG, 0);
        }
    }
    if (!inside) return;
    if constexpr (!MF) {
        if constexpr (!fuse) {
#pragma unroll
            for (int k = 0; k < CG; ++k) {
                const int ch = cg * CG + k;
                ((GLOBAL_AS float*)out)[obase + spec_offset(ch, pix, cs, HW)] = acc[k];
            }
        }
    }
    if (cg == 0 && set == q && T_final) {
        ((GLOBAL_AS float*)T_final)[q * J.s_pix + pix] = T;
        ((GLOBAL_AS uint32_t*)n_last)[q * J.s_pix + pix] = last;
        ((GLOBAL_AS uint32_t*)n_contrib)[q * J.s_pix + pix] = cnt;
    }
}

template <int CG>
__device__ __forceinline__ void blend_tile(const BlendJob& J, BlendLds& S, int tile, int cg, int set)
{
    blend_tile_impl<CG>(J, S, tile, cg, set, J.rec, J.plist, J.ranges, J.attr, J.out, J.T_final, J.n_last,
                        J.n_contrib);
}

template <int CG, bool FUSE>
__global__ __launch_bounds__(256) void k_blend(BlendJob J, const GRec* __restrict__ rec,
                                               const uint32_t* __restrict__ plist, const uint2* __restrict__ ranges,
                                               const float* __restrict__ attr, float* __restrict__ out,
                                               float* __restrict__ T_final, uint32_t* __restrict__ n_last,
                                               uint32_t* __restrict__ n_contrib)
{
    __shared__ BlendLds S;
    blend_tile_impl<CG, FUSE>(J, S, blockIdx.x, blockIdx.y, blockIdx.z, rec, plist, ranges, attr, out, T_final,
                              n_last, n_contrib);
}

// Persistent blend over a table of jobs (scenes of any size, grid, tile
// shape and channel count): each workgroup takes (job, tile, channel group,
// set) items from a device counter until none are left -- every workgroup
// exits once the counter passes the total -- and stamps the completion time
// of the item's query.  Items are numbered job by job, then set by set, then
// channel group, then tile, so a query's items are contiguous and the job
// order is the service order.
__global__ __launch_bounds__(256) void k_blend_persist(const BlendJob* __restrict__ jobs, int njobs, uint32_t total,
                                                       uint32_t* counter, unsigned long long* done_ts)
{
    __shared__ BlendLds S;
    __shared__ uint32_t s_item;
    __shared__ int s_job;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t item = atomicAdd(counter, 1u);
            int lo = 0, hi = njobs - 1;  // last job with item_begin <= item
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].item_begin <= item) lo = mid;
                else hi = mid - 1;
            }
            s_item = item;
            s_job = lo;
        }
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        const int j = __builtin_amdgcn_readfirstlane(s_job);
        __syncthreads();
        if (item >= total) break;
        const BlendJob& J = jobs[j];
        const uint32_t local = item - J.item_begin;
        const int tile = (int)(local % (uint32_t)J.T);
        const uint32_t rest = local / (uint32_t)J.T;
        const int cg = (int)(rest % (uint32_t)J.ncg);
        const int set = (int)(rest / (uint32_t)J.ncg);
        switch (J.cg) {
            case 1: blend_tile<1>(J, S, tile, cg, set); break;
            case 2: blend_tile<2>(J, S, tile, cg, set); break;
            case 4: blend_tile<4>(J, S, tile, cg, set); break;
            case 8: blend_tile<8>(J, S, tile, cg, set); break;
            case 16: blend_tile<16>(J, S, tile, cg, set); break;
            default: blend_tile<32>(J, S, tile, cg, set); break;
        }
        if (threadIdx.x == 0 && done_ts) atomicMax(&done_ts[J.query0 + set], (unsigned long long)wall_clock64());
    }
}

__global__ void k_stamp(unsigned long long* ts)
{
    if (threadIdx.x == 0) *ts = (unsigned long long)wall_clock64();
}

// Geometry-only walk: marks every Gaussian that reaches at least one pixel
// (alpha >= alpha_min before the pixel stops) and records the per-pixel
// state.  Its output decides which (set, Gaussian) rows the attribute
// network must evaluate: no other Gaussian can change a pixel.
// One wave per 64 pixels of a tile (the tile's pixels row-major, in groups of
// 64): the groups of a tile walk the same list independently, so every CU
// has work (a tile per workgroup left half the chip idle at 138 tiles).
constexpr int LIVE_PIX = 64;
__global__ __launch_bounds__(LIVE_PIX) void k_live(
    const GRec* __restrict__ rec, size_t s_rec, const uint32_t* __restrict__ plist, size_t s_plist,
    const uint2* __restrict__ ranges, size_t s_ranges, int H, int W, int tw, int th, int TX, float amin, float amax,
    float tmin, uint32_t* __restrict__ flags_live, size_t s_live, float* __restrict__ T_final,
    uint32_t* __restrict__ n_last, uint32_t* __restrict__ n_contrib, size_t s_pix, float* __restrict__ wtot,
    size_t s_wtot)
{
    const int tile = blockIdx.x, q = blockIdx.z;
    constexpr int nthr = LIVE_PIX;
    const int txi = tile % TX, tyi = tile / TX;
    const int k = blockIdx.y * LIVE_PIX + threadIdx.x;  // pixel of the tile
    const int lx = k % tw, ly = k / tw;
    const int col = txi * tw + lx, row = tyi * th + ly;
    const bool inside = ly < th && col < W && row < H;
    if (__syncthreads_count(inside) == 0) return;  // a group past the image
    const uint2 rg = ranges[q * s_ranges + tile];
    const double pcx = col + 0.5, pcy = row + 0.5, halfW = 0.5 * W;
    rec += q * s_rec;
    plist += q * s_plist;
    flags_live += q * s_live;
    __shared__ double s_px[LIVE_PIX], s_py[LIVE_PIX], s_ca[LIVE_PIX], s_cb[LIVE_PIX], s_cc[LIVE_PIX];
    __shared__ float s_sig[LIVE_PIX], s_att[LIVE_PIX];
    __shared__ uint32_t s_g[LIVE_PIX];
    // per-pixel weights of the batch's entries, [entry][pixel] (a row of 65
    // keeps both the per-pixel writes and the per-entry sums conflict-free)
    __shared__ float s_w[LIVE_PIX][LIVE_PIX + 1];
    if (wtot) wtot += q * s_wtot;
    float T = 1.0f;
    uint32_t last = 0, cnt = 0;
    bool done = !inside;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += nthr) {
        if (__syncthreads_count(done) == nthr) break;
        const uint32_t i = b0 + threadIdx.x;
        if (i < rg.y) {
            const uint32_t g = plist[i];
            const GRec r = rec[g];
            s_px[threadIdx.x] = r.px;
            s_py[threadIdx.x] = r.py;
            s_ca[threadIdx.x] = r.ca;
            s_cb[threadIdx.x] = r.cb;
            s_cc[threadIdx.x] = r.cc;
            s_sig[threadIdx.x] = r.sigma;
            s_att[threadIdx.x] = r.att;
            s_g[threadIdx.x] = g;
        }
        __syncthreads();
        const int m = (int)min((uint32_t)nthr, rg.y - b0);
        int jend = 0;  // entries walked by some pixel of the wave
        for (int j = 0; j < m; ++j) {
            if (__ballot(!done) == 0ull) break;
            jend = j + 1;
            float wgt = 0.0f;
            if (!done) {
                double dx = pcx - s_px[j];
                dx += dx >= halfW ? -(double)W : (dx < -halfW ? (double)W : 0.0);
                const double dy = pcy - s_py[j];
                const double qv = s_ca[j] * dx * dx + 2.0 * s_cb[j] * dx * dy + s_cc[j] * dy * dy;
                const float G = __builtin_amdgcn_exp2f((float)(-0.5 * LOG2E * qv));
                const float alpha = fminf(amax, s_sig[j] * G);
                const float Tn = T * (1.0f - alpha);
                const bool stop = alpha >= amin && Tn < tmin;
                const bool take = alpha >= amin && !stop;
                done = stop;
                if (take) flags_live[s_g[j]] = 1u;
                wgt = take ? T * alpha * s_att[j] : 0.0f;
                T = take ? Tn : T;
                last = take ? b0 + j + 1 - rg.x : last;
                cnt += take ? 1u : 0u;
            }
            if (wtot) s_w[j][threadIdx.x] = wgt;
        }
        if (wtot) {
            // thread t sums entry t's weight over the 64 pixels
            __syncthreads();
            if ((int)threadIdx.x < jend) {
                float ws = 0.0f;
#pragma unroll 8
                for (int i = 0; i < LIVE_PIX; ++i) ws += s_w[threadIdx.x][i];
                if (ws != 0.0f) unsafeAtomicAdd(&wtot[s_g[threadIdx.x]], ws);
            }
        }
    }
    if (!inside) return;
    const size_t pix = (size_t)row * W + col;
    T_final[q * s_pix + pix] = T;
    n_last[q * s_pix + pix] = last;
    n_contrib[q * s_pix + pix] = cnt;
}

// Compacts the live flags of each query into a list (order unspecified).
__global__ __launch_bounds__(256) void k_compact_live(const uint32_t* __restrict__ flags_live, size_t s_live, int n,
                                                      uint32_t* __restrict__ list, size_t s_list,
                                                      uint32_t* __restrict__ count)
{
    const int q = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool on = i < n && flags_live[q * s_live + i] != 0u;
    const unsigned long long b = __ballot(on);
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (lane == 0 && b) base = atomicAdd(&count[q], (uint32_t)__popcll(b));
    base = __shfl(base, 0, 64);
    if (on) list[q * s_list + base + __popcll(b & ((1ull << lane) - 1ull))] = (uint32_t)i;
}

void launch_live(const gs_params& p, const Layout& L, char* ws, uint32_t* list, size_t s_list, uint32_t* count,
                 hipStream_t s)
{
    uint32_t* fl = (uint32_t*)(ws + L.live);
    {
        // the live flags and weight sums of every query (their query
        // strides included: one contiguous range each) and the counts
        FillSegs f{};
        f.p[0] = fl; f.count[0] = (size_t)L.nq * (L.s_live / 4);
        f.p[1] = count; f.count[1] = (size_t)L.nq;
        f.p[2] = (uint32_t*)(ws + L.wtot); f.count[2] = (size_t)L.nq * (L.s_wtot / 4);
        f.n = 3;
        launch_fill_segs(f, s);
    }
    hipLaunchKernelGGL(k_live, dim3(L.T, (L.tw * L.th + LIVE_PIX - 1) / LIVE_PIX, L.nq), dim3(LIVE_PIX), 0, s,
                       (const GRec*)(ws + L.rec),
                       L.s_rec / sizeof(GRec), (const uint32_t*)(ws + L.plist), L.s_plist / 4,
                       (const uint2*)(ws + L.ranges), L.s_ranges / sizeof(uint2), L.H, L.W, L.tw, L.th, L.TX,
                       p.alpha_min, p.alpha_max, p.T_min, fl, L.s_live / 4, (float*)(ws + L.T_final),
                       (uint32_t*)(ws + L.n_last), (uint32_t*)(ws + L.n_contrib), L.s_pix / 4,
                       (float*)(ws + L.wtot), L.s_wtot / 4);
    hipLaunchKernelGGL(k_compact_live, dim3((L.n + 255) / 256, L.nq), dim3(256), 0, s, fl, L.s_live / 4, L.n, list,
                       s_list, count);
}

BlendJob make_blend_job(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws, float* out)
{
    const int C = a.is_complex ? 2 : 1;
    BlendJob J{};
    J.rec = (const GRec*)(ws + L.rec);
    J.s_rec = L.s_rec / sizeof(GRec);
    J.plist = (const uint32_t*)(ws + L.plist);
    J.s_plist = L.s_plist / 4;
    J.ranges = (const uint2*)(ws + L.ranges);
    J.s_ranges = L.s_ranges / sizeof(uint2);
    J.attr = a.data;
    J.a_stride = a.query_stride;
    J.Fc = a.n_chan * C;
    J.C = C;
    J.H = L.H;
    J.W = L.W;
    J.tw = L.tw;
    J.th = L.th;
    J.TX = L.TX;
    J.T = L.T;
    J.nsets = n_sets;
    J.shared_geo = (L.nq == 1 && n_sets > 1) ? 1 : 0;
    J.amin = p.alpha_min;
    J.amax = p.alpha_max;
    J.tmin = p.T_min;
    J.out = out;
    J.T_final = (float*)(ws + L.T_final);
    J.n_last = (uint32_t*)(ws + L.n_last);
    J.n_contrib = (uint32_t*)(ws + L.n_contrib);
    J.s_pix = L.s_pix / 4;
    J.tgt = nullptr;
    J.dpart = nullptr;
    J.lpart = nullptr;
    J.lnp = 0;
    J.lscale = 0.0f;
    return J;
}

// ---------------------------------------------------------------------------
// Compositing of S attribute sets over one shared geometry (the training
// batch: one receiver, S transmitters whose effect is in the attributes).
// The pixel weight w_k(p) = T_k alpha_k a_k and the walk's decisions do not
// depend on the set, so out[s][f](p) = sum_k w_k(p) v[s][k][f] is one
// product of the weights W (entries x pixels) with the attribute rows V
// (entries x S*F*c columns).  One workgroup (8 waves) takes 64 pixels of a
// tile (the tile's in-image pixels packed into groups of 64): wave 0 walks
// the list once per pixel (the same decisions, in the same order, as
// k_blend), the weights of up to SGF_BUF entries collect in LDS, and the
// eight waves then form out = W^T V on the FP32 matrix cores, each for its
// share of the columns.  A walk longer than the buffer flushes it and the
// next products add to the stored spectrum (only this workgroup writes
// these pixels).
// ---------------------------------------------------------------------------
constexpr int SGF_WAVES = 8;
constexpr int SGF_PIX = 64;
constexpr int SGF_BATCH = 64;   // entries staged per walk step
constexpr int SGF_BUF = 128;    // entries whose weights the LDS holds

template <int CS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_blend_sg(
    const GRec* __restrict__ rec, const uint32_t* __restrict__ plist, const uint2* __restrict__ ranges,
    const float* __restrict__ attr, int64_t a_stride, int S, int Fc, int H, int W, int tw, int th, int TX,
    float amin, float amax, float tmin, float* __restrict__ out, float* __restrict__ T_final,
    uint32_t* __restrict__ n_last, uint32_t* __restrict__ n_contrib, int min_walk)
{
    const int tile = blockIdx.x, pg = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j4 = lane >> 4, l16 = lane & 15;
    const int txi = tile % TX, tyi = tile / TX;
    const int vw = min(tw, W - txi * tw), vh = min(th, H - tyi * th);
    if (pg * SGF_PIX >= vw * vh) return;
    if (min_walk > 0) {
        // only groups whose walk (the stop positions a live pass recorded)
        // is longer than min_walk entries
        const int k = pg * SGF_PIX + lane;
        const uint32_t st = k < vw * vh ? n_last[(tyi * th + k / vw) * W + txi * tw + k % vw] : 0u;
        uint32_t mx = st;
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        if (mx <= (uint32_t)min_walk) return;
    }
    const uint2 rg = ranges[tile];
    const size_t HW = (size_t)H * W;
    const int F = Fc >> CS;
    const int ncb = S * Fc / 16;  // 16-column blocks (Fc % 16 == 0)
    const int cb_lo = wave * ncb / SGF_WAVES, cb_hi = (wave + 1) * ncb / SGF_WAVES;

    __shared__ float s_w[SGF_BUF][SGF_PIX + 1];         // weights of the buffered entries
    __shared__ uint32_t s_gb[SGF_BUF];                   // their Gaussians
    __shared__ float s_t[SGF_WAVES][16][SGF_PIX + 1];   // per-wave output transpose
    __shared__ double s_px[SGF_BATCH], s_py[SGF_BATCH], s_ca[SGF_BATCH], s_cb[SGF_BATCH], s_cc[SGF_BATCH];
    __shared__ float s_sig[SGF_BATCH], s_att[SGF_BATCH];
    __shared__ uint32_t s_g[SGF_BATCH];
    __shared__ int s_pix[SGF_PIX];
    __shared__ int s_walked, s_alldone;

    if (threadIdx.x < SGF_PIX) {
        const int k = pg * SGF_PIX + threadIdx.x;
        s_pix[threadIdx.x] = k < vw * vh ? (tyi * th + k / vw) * W + txi * tw + k % vw : -1;
    }
    __syncthreads();
    // the walking wave's pixel and state
    const int wpix = s_pix[lane];
    const double pcx = (wpix >= 0 ? wpix % W : 0) + 0.5, pcy = (wpix >= 0 ? wpix / W : 0) + 0.5;
    const double halfW = 0.5 * W, Wd = (double)W;
    float T = 1.0f;
    uint32_t last = 0, cnt = 0;
    bool done = wpix < 0;

    // out = W^T V over the nbuf buffered entries for this wave's columns;
    // add: add to what an earlier flush stored
    auto contract = [&](int nbuf, bool add) {
        const int nks = (nbuf + 3) >> 2;  // K-steps of 4 entries (rows past nbuf hold zero weights)
        for (int cb = cb_lo; cb < cb_hi; ++cb) {
            const int s = cb * 16 / Fc;
            const int c0 = cb * 16 - s * Fc;
            const CFloat* vb = (const CFloat*)(attr + s * a_stride + c0 + l16);
            // the B operands of every K-step first (independent loads)
            float bq[SGF_BUF / 4];
#pragma unroll
            for (int ks = 0; ks < SGF_BUF / 4; ++ks)
                if (ks < nks) bq[ks] = vb[(size_t)s_gb[4 * ks + j4] * Fc];
            f32x4 acc[4];
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) acc[pb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < SGF_BUF / 4; ++ks) {
                if (ks < nks) {
#pragma unroll
                    for (int pb = 0; pb < 4; ++pb)
                        acc[pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(s_w[4 * ks + j4][16 * pb + l16], bq[ks],
                                                                       acc[pb], 0, 0, 0);
                }
            }
            // lane holds out[pixel 16 pb + 4 j4 + r][column c0 + l16]: through
            // LDS so that each lane stores its own pixel
#pragma unroll
            for (int pb = 0; pb < 4; ++pb)
#pragma unroll
                for (int r = 0; r < 4; ++r) s_t[wave][l16][16 * pb + 4 * j4 + r] = acc[pb][r];
            wave_sync_lds();
            const int px = s_pix[lane];
            if (px >= 0) {
                float* ob = out + ((size_t)s * F * HW << CS);
                if constexpr (CS == 1) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        float2* o2 = (float2*)(ob + (((size_t)((c0 >> 1) + q) * HW + px) << 1));
                        float2 v = float2{s_t[wave][2 * q][lane], s_t[wave][2 * q + 1][lane]};
                        if (add) {
                            const float2 o = *o2;
                            v.x += o.x;
                            v.y += o.y;
                        }
                        *o2 = v;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        float* o1 = ob + (size_t)(c0 + q) * HW + px;
                        const float v = s_t[wave][q][lane];
                        *o1 = add ? *o1 + v : v;
                    }
                }
            }
            wave_sync_lds();
        }
    };

    int nbuf = 0;
    bool stored = false, alldone = false;
    for (uint32_t b0 = rg.x; b0 < rg.y && !alldone; b0 += SGF_BATCH) {
        const int m = (int)min((uint32_t)SGF_BATCH, rg.y - b0);
        if ((int)threadIdx.x < m) {
            const uint32_t g = plist[b0 + threadIdx.x];
            const GRec r = rec[g];
            s_px[threadIdx.x] = r.px;
            s_py[threadIdx.x] = r.py;
            s_ca[threadIdx.x] = r.ca;
            s_cb[threadIdx.x] = r.cb;
            s_cc[threadIdx.x] = r.cc;
            s_sig[threadIdx.x] = r.sigma;
            s_att[threadIdx.x] = r.att;
            s_g[threadIdx.x] = g;
        }
        __syncthreads();
        if (wave == 0) {
            // the walk, as in k_blend: stop before an entry that would take
            // T below T_min; entries past the group's last live pixel are
            // not buffered
            int j = 0;
            for (; j < m; ++j) {
                if (__ballot(!done) == 0ull) break;
                float wgt = 0.0f;
                if (!done) {
                    double dx = pcx - s_px[j];
                    dx += dx >= halfW ? -Wd : (dx < -halfW ? Wd : 0.0);
                    const double dy = pcy - s_py[j];
                    const double qv = s_ca[j] * dx * dx + 2.0 * s_cb[j] * dx * dy + s_cc[j] * dy * dy;
                    const float G = __builtin_amdgcn_exp2f((float)(-0.5 * LOG2E * qv));
                    const float alpha = fminf(amax, s_sig[j] * G);
                    const float Tn = T * (1.0f - alpha);
                    const bool stop = alpha >= amin && Tn < tmin;
                    const bool take = alpha >= amin && !stop;
                    done = stop;
                    wgt = take ? T * alpha * s_att[j] : 0.0f;
                    T = take ? Tn : T;
                    last = take ? b0 + j + 1 - rg.x : last;
                    cnt += take ? 1u : 0u;
                }
                s_w[nbuf + j][lane] = wgt;
                if (lane == 0) s_gb[nbuf + j] = s_g[j];
            }
            // zero weight rows up to the next multiple of 4 (valid Gaussians)
            for (int k = j; k < ((j + 3) & ~3); ++k) {
                s_w[nbuf + k][lane] = 0.0f;
                if (lane == 0) s_gb[nbuf + k] = s_g[0];
            }
            const bool ad = __ballot(!done) == 0ull;
            if (lane == 0) {
                s_walked = j;
                s_alldone = ad ? 1 : 0;
            }
        }
        __syncthreads();
        nbuf += s_walked;
        alldone = s_alldone != 0;
        const bool last_batch = alldone || b0 + SGF_BATCH >= rg.y;
        if (last_batch || nbuf + SGF_BATCH > SGF_BUF) {
            if (nbuf > 0) {
                contract(nbuf, stored);
                stored = true;
            }
            nbuf = 0;
        }
        __syncthreads();
    }
    if (!stored) {
        // no entry reached the group: its spectrum is zero
        const int px = s_pix[lane];
        if (px >= 0) {
            for (int cb = cb_lo; cb < cb_hi; ++cb) {
                const int s = cb * 16 / Fc;
                const int c0 = cb * 16 - s * Fc;
                float* ob = out + ((size_t)s * F * HW << CS);
                for (int q = 0; q < 16; ++q) ob[((size_t)((c0 + q) >> CS) * HW + px) * (1 << CS) + ((c0 + q) & CS)] = 0.0f;
            }
        }
    }
    if (wave == 0 && wpix >= 0) {
        T_final[wpix] = T;
        n_last[wpix] = last;
        n_contrib[wpix] = cnt;
    }
}

// Channel floats per workgroup: the largest power of two that divides F*c,
// at most 64, or the caller's choice (a power of two up to 64 dividing F*c).
// (The backward and the persistent batch kernel cap it at 32.)
int choose_chan_group(int Fc, int requested)
{
    if (requested > 0 && requested <= 64 && (requested & (requested - 1)) == 0 && Fc % requested == 0)
        return requested;
    int cg = 1;
    while (cg < 64 && Fc % (cg * 2) == 0) cg *= 2;
    return cg;
}

gs_status launch_blend(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws, float* out,
                       hipStream_t s, const float* tgt, float* dpart, float* lpart, float lscale)
{
    const int C = a.is_complex ? 2 : 1;
    const int Fc = a.n_chan * C;
    if (!tgt && L.nq == 1 && Fc % 16 == 0 && !(p.options & GS_OPT_BLEND_PER_GROUP)) {
        // every set over the one prepared geometry: the walk once per pixel
        void* tok;
        timing_begin(TK_BLEND, s, &tok);
        auto kern = C == 2 ? k_blend_sg<1> : k_blend_sg<0>;
        hipLaunchKernelGGL(kern, dim3(L.T, (L.tw * L.th) / SGF_PIX), dim3(64 * SGF_WAVES), 0, s,
                           (const GRec*)(ws + L.rec), (const uint32_t*)(ws + L.plist), (const uint2*)(ws + L.ranges),
                           a.data, a.query_stride, n_sets, Fc, L.H, L.W, L.tw, L.th, L.TX, p.alpha_min, p.alpha_max,
                           p.T_min, out, (float*)(ws + L.T_final), (uint32_t*)(ws + L.n_last),
                           (uint32_t*)(ws + L.n_contrib), 0);
        timing_end(tok, s);
        return GS_OK;
    }
    int cg = choose_chan_group(Fc, p.chan_group);
    if (tgt && cg > 32) cg = 32;  // the fused loss stage needs the registers of a 64-channel group
    if (Fc / cg > 65535) return GS_ERR_CAPACITY;
    BlendJob J = make_blend_job(a, p, L, n_sets, ws, out);
    J.cg = cg;
    J.ncg = Fc / cg;
    J.tgt = tgt;
    J.dpart = dpart;
    J.lpart = lpart;
    J.lnp = L.T * ((L.tw * L.th) >> 6);
    J.lscale = lscale;
    dim3 grid(L.T, Fc / cg, n_sets), block(L.tw * L.th);
#define ARGS J.rec, J.plist, J.ranges, J.attr, J.out, J.T_final, J.n_last, J.n_contrib
    void* tok;
    timing_begin(TK_BLEND, s, &tok);
    auto go = [&](auto fz) {
        constexpr bool FZ = decltype(fz)::value;
        switch (cg) {
            case 1: hipLaunchKernelGGL((k_blend<1, FZ>), grid, block, 0, s, J, ARGS); break;
            case 2: hipLaunchKernelGGL((k_blend<2, FZ>), grid, block, 0, s, J, ARGS); break;
            case 4: hipLaunchKernelGGL((k_blend<4, FZ>), grid, block, 0, s, J, ARGS); break;
            case 8: hipLaunchKernelGGL((k_blend<8, FZ>), grid, block, 0, s, J, ARGS); break;
            case 16: hipLaunchKernelGGL((k_blend<16, FZ>), grid, block, 0, s, J, ARGS); break;
            case 32: hipLaunchKernelGGL((k_blend<32, FZ>), grid, block, 0, s, J, ARGS); break;
            default: hipLaunchKernelGGL((k_blend<64, FZ>), grid, block, 0, s, J, ARGS); break;
        }
    };
    if (tgt) go(std::true_type{});
    else go(std::false_type{});
    timing_end(tok, s);
#undef ARGS
    return GS_OK;
}

// k_blend_sg over the groups whose walk (live-pass stop positions) is longer
// than min_walk entries only
void launch_blend_sg_long(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws, float* out,
                          int min_walk, hipStream_t s)
{
    auto kern = a.is_complex ? k_blend_sg<1> : k_blend_sg<0>;
    hipLaunchKernelGGL(kern, dim3(L.T, (L.tw * L.th) / SGF_PIX), dim3(64 * SGF_WAVES), 0, s,
                       (const GRec*)(ws + L.rec), (const uint32_t*)(ws + L.plist), (const uint2*)(ws + L.ranges),
                       a.data, a.query_stride, n_sets, a.n_chan * (a.is_complex ? 2 : 1), L.H, L.W, L.tw, L.th, L.TX,
                       p.alpha_min, p.alpha_max, p.T_min, out, (float*)(ws + L.T_final), (uint32_t*)(ws + L.n_last),
                       (uint32_t*)(ws + L.n_contrib), min_walk);
}

void launch_blend_persist(const BlendJob* jobs, int njobs, uint32_t total, uint32_t* counter,
                          unsigned long long* done_ts, int workgroups, int block, hipStream_t s)
{
    hipLaunchKernelGGL(k_blend_persist, dim3(workgroups), dim3(block), 0, s, jobs, njobs, total, counter, done_ts);
}

hipError_t persist_occupancy(int block, int* per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_blend_persist, block, 0);
}

void launch_stamp(unsigned long long* ts, hipStream_t s) { hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, ts); }

}  // namespace gs
