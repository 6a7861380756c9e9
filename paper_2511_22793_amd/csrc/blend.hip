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
#include "common.h"

namespace gs {

constexpr double LOG2E = 1.4426950408889634;

template <int CG>
__global__ __launch_bounds__(256) void k_blend(
    const GRec* __restrict__ rec, size_t s_rec, const uint32_t* __restrict__ plist, size_t s_plist,
    const uint2* __restrict__ ranges, size_t s_ranges, const float* __restrict__ attr, int64_t a_stride,
    int Fc, int C, int H, int W, int tw, int th, int TX, float amin, float amax, float tmin,
    float* __restrict__ out, float* __restrict__ T_final, uint32_t* __restrict__ n_last,
    uint32_t* __restrict__ n_contrib, size_t s_pix, int shared_geo)
{
    const int tile = blockIdx.x, cg = blockIdx.y, set = blockIdx.z;
    const int q = shared_geo ? 0 : set;  // geometry query
    const int nthr = tw * th;
    const int txi = tile % TX, tyi = tile / TX;
    const int lx = threadIdx.x % tw, ly = threadIdx.x / tw;
    const int col = txi * tw + lx, row = tyi * th + ly;
    const bool inside = col < W && row < H;
    const uint2 rg = ranges[q * s_ranges + tile];
    const double pcx = col + 0.5, pcy = row + 0.5, halfW = 0.5 * W;
    rec += q * s_rec;
    plist += q * s_plist;
    const float* A = attr + set * a_stride + cg * CG;

    __shared__ double s_px[256], s_py[256], s_ca[256], s_cb[256], s_cc[256];
    __shared__ float s_sig[256], s_att[256];
    __shared__ uint32_t s_g[256];

    float T = 1.0f;
    float acc[CG];
#pragma unroll
    for (int k = 0; k < CG; ++k) acc[k] = 0.0f;
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
        for (int j = 0; j < m && !done; ++j) {
            // the attribute row is wave-uniform: issue its scalar loads first
            // so that the alpha evaluation below hides their latency
            const uint32_t g = __builtin_amdgcn_readfirstlane(s_g[j]);
            const float* vp = A + (size_t)g * Fc;
            float v[CG];
#pragma unroll
            for (int k = 0; k < CG; ++k) v[k] = vp[k];
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
            // branch-free update (one basic block, so the row loads issue
            // first): a skipped pair adds zero and keeps T
            const float wgt = take ? T * alpha * s_att[j] : 0.0f;
#pragma unroll
            for (int k = 0; k < CG; ++k) acc[k] = fmaf(wgt, v[k], acc[k]);
            T = take ? Tn : T;
            last = take ? b0 + j + 1 - rg.x : last;
            cnt += take ? 1u : 0u;
        }
    }
    if (!inside) return;
    const size_t HW = (size_t)H * W, pix = (size_t)row * W + col;
    const int F = Fc / C;
#pragma unroll
    for (int k = 0; k < CG; ++k) {
        const int ch = cg * CG + k;
        const int f = ch / C, comp = ch - f * C;
        out[(((size_t)set * F + f) * HW + pix) * C + comp] = acc[k];
    }
    if (cg == 0 && set == q) {
        T_final[q * s_pix + pix] = T;
        n_last[q * s_pix + pix] = last;
        n_contrib[q * s_pix + pix] = cnt;
    }
}

// Geometry-only walk: marks every Gaussian that reaches at least one pixel
// (alpha >= alpha_min before the pixel stops) and records the per-pixel
// state.  Its output decides which (set, Gaussian) rows the attribute
// network must evaluate: no other Gaussian can change a pixel.
__global__ __launch_bounds__(256) void k_live(
    const GRec* __restrict__ rec, size_t s_rec, const uint32_t* __restrict__ plist, size_t s_plist,
    const uint2* __restrict__ ranges, size_t s_ranges, int H, int W, int tw, int th, int TX, float amin, float amax,
    float tmin, uint32_t* __restrict__ flags_live, size_t s_live, float* __restrict__ T_final,
    uint32_t* __restrict__ n_last, uint32_t* __restrict__ n_contrib, size_t s_pix)
{
    const int tile = blockIdx.x, q = blockIdx.z;
    const int nthr = tw * th;
    const int txi = tile % TX, tyi = tile / TX;
    const int lx = threadIdx.x % tw, ly = threadIdx.x / tw;
    const int col = txi * tw + lx, row = tyi * th + ly;
    const bool inside = col < W && row < H;
    const uint2 rg = ranges[q * s_ranges + tile];
    const double pcx = col + 0.5, pcy = row + 0.5, halfW = 0.5 * W;
    rec += q * s_rec;
    plist += q * s_plist;
    flags_live += q * s_live;
    __shared__ double s_px[256], s_py[256], s_ca[256], s_cb[256], s_cc[256];
    __shared__ float s_sig[256];
    __shared__ uint32_t s_g[256];
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
            s_g[threadIdx.x] = g;
        }
        __syncthreads();
        const int m = (int)min((uint32_t)nthr, rg.y - b0);
        for (int j = 0; j < m && !done; ++j) {
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
            T = take ? Tn : T;
            last = take ? b0 + j + 1 - rg.x : last;
            cnt += take ? 1u : 0u;
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
    launch_fill_u32(fl, (size_t)L.n, L.s_live / 4, L.nq, 0u, s);
    launch_fill_u32(count, 1, 1, L.nq, 0u, s);
    hipLaunchKernelGGL(k_live, dim3(L.T, 1, L.nq), dim3(L.tw * L.th), 0, s, (const GRec*)(ws + L.rec),
                       L.s_rec / sizeof(GRec), (const uint32_t*)(ws + L.plist), L.s_plist / 4,
                       (const uint2*)(ws + L.ranges), L.s_ranges / sizeof(uint2), L.H, L.W, L.tw, L.th, L.TX,
                       p.alpha_min, p.alpha_max, p.T_min, fl, L.s_live / 4, (float*)(ws + L.T_final),
                       (uint32_t*)(ws + L.n_last), (uint32_t*)(ws + L.n_contrib), L.s_pix / 4);
    hipLaunchKernelGGL(k_compact_live, dim3((L.n + 255) / 256, L.nq), dim3(256), 0, s, fl, L.s_live / 4, L.n, list,
                       s_list, count);
}

template <int CG>
static void blend_cg(dim3 grid, dim3 block, hipStream_t s, const gs_attrs& a, const gs_params& p, const Layout& L,
                     char* ws, float* out, int C, int shared_geo)
{
    hipLaunchKernelGGL(k_blend<CG>, grid, block, 0, s, (const GRec*)(ws + L.rec), L.s_rec / sizeof(GRec),
                       (const uint32_t*)(ws + L.plist), L.s_plist / 4, (const uint2*)(ws + L.ranges),
                       L.s_ranges / sizeof(uint2), a.data, a.query_stride, a.n_chan * C, C, L.H, L.W, L.tw, L.th,
                       L.TX, p.alpha_min, p.alpha_max, p.T_min, out, (float*)(ws + L.T_final),
                       (uint32_t*)(ws + L.n_last), (uint32_t*)(ws + L.n_contrib), L.s_pix / 4, shared_geo);
}

// Channel floats per workgroup: the largest power of two that divides F*c,
// at most 32, or the caller's choice (a power of two up to 64 dividing F*c).
int choose_chan_group(int Fc, int requested)
{
    if (requested > 0 && requested <= 64 && (requested & (requested - 1)) == 0 && Fc % requested == 0)
        return requested;
    int cg = 1;
    while (cg < 32 && Fc % (cg * 2) == 0) cg *= 2;
    return cg;
}

gs_status launch_blend(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws, float* out,
                       hipStream_t s)
{
    const int C = a.is_complex ? 2 : 1;
    const int Fc = a.n_chan * C;
    const int cg = choose_chan_group(Fc, p.chan_group);
    if (Fc / cg > 65535) return GS_ERR_CAPACITY;
    const int shared = (L.nq == 1 && n_sets > 1) ? 1 : 0;
    dim3 grid(L.T, Fc / cg, n_sets), block(L.tw * L.th);
    switch (cg) {
        case 1: blend_cg<1>(grid, block, s, a, p, L, ws, out, C, shared); break;
        case 2: blend_cg<2>(grid, block, s, a, p, L, ws, out, C, shared); break;
        case 4: blend_cg<4>(grid, block, s, a, p, L, ws, out, C, shared); break;
        case 8: blend_cg<8>(grid, block, s, a, p, L, ws, out, C, shared); break;
        case 16: blend_cg<16>(grid, block, s, a, p, L, ws, out, C, shared); break;
        case 32: blend_cg<32>(grid, block, s, a, p, L, ws, out, C, shared); break;
        default: blend_cg<64>(grid, block, s, a, p, L, ws, out, C, shared); break;
    }
    return GS_OK;
}

}  // namespace gs
