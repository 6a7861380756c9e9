// Adaptive densification, pruning and opacity reset (Sec. 4.2, Algorithm 1's
// densify branch).
//
// Statistics: for every Gaussian in a step's live list, grad_acc += |dL/dmu|
// and grad_cnt += 1; the criterion is grad_acc / grad_cnt >= tau_grad.
//
// Plan: per Gaussian i, in index order,
//   densify  = cnt_i > 0 and acc_i / cnt_i >= tau_grad (FP32);
//   small    = max_c exp(log_scale_i[c]) <= clone_extent (epsilon r_scene);
//   faint    = sigmoid(opacity_logit_i) < opacity_min;
//   large    = screen_radius_i > radius_max (pixels; 0 for culled ones);
//   outputs  keep:  [i]               unless faint or large
//            clone: [i], [i's copy]   i unless faint or large, the copy unless faint
//            split: N children        unless faint (i itself leaves)
// (the prune of Algorithm 1 runs after the densification over the new set;
// new Gaussians have not been rendered, so only their inherited opacity can
// prune them).  Output slot j of the new set carries src[j] (its parent) and
// kind[j] (DENS_KEEP, DENS_CLONE, or the child number k < N); slots follow
// the parents' order (an exclusive scan of the per-parent counts), so the
// plan is deterministic.
//
// Apply: children of a split take mu + R(q) (s * xi_k) with s = exp(log
// scale) and xi_k standard normals given by the caller, and log scale minus
// log(0.8 N); everything else is copied from the parent.  Gather copies any
// other per-Gaussian array (embeddings, Adam moments) to the new order,
// optionally zeroing the rows of new Gaussians (fresh optimiser state).
#include "common.h"

namespace gs {

constexpr int DENS_KEEP = -1, DENS_CLONE = -2;
constexpr int DENS_SCAN = 1024;  // counts per scan block

__global__ __launch_bounds__(256) void k_dens_stats(const float* __restrict__ d_mean, int n,
                                                    const uint32_t* __restrict__ live,
                                                    const uint32_t* __restrict__ count, float* __restrict__ acc,
                                                    uint32_t* __restrict__ cnt)
{
    const uint32_t nl = *count;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nl; t += gridDim.x * blockDim.x) {
        const uint32_t i = live[t];
        const float gx = d_mean[i], gy = d_mean[n + i], gz = d_mean[2 * n + i];
        acc[i] += sqrtf(gx * gx + gy * gy + gz * gz);  // one live entry per Gaussian: no race
        cnt[i] += 1u;
    }
}

// per-parent output count, then the block sums of the counts
__global__ __launch_bounds__(256) void k_dens_count(int n, const float* __restrict__ log_scale,
                                                    const float* __restrict__ opacity_logit,
                                                    const float* __restrict__ acc, const uint32_t* __restrict__ cnt,
                                                    const float* __restrict__ radius, gs_densify_params P,
                                                    uint32_t* __restrict__ counts, uint8_t* __restrict__ action)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool densify = cnt[i] > 0u && acc[i] / (float)cnt[i] >= P.grad_threshold;
    const float smax = expf(fmaxf(log_scale[i], fmaxf(log_scale[n + i], log_scale[2 * n + i])));
    const bool small = smax <= P.clone_extent;
    const float op = 1.0f / (1.0f + expf(-opacity_logit[i]));
    const bool faint = op < P.opacity_min;
    const bool large = radius && radius[i] > P.radius_max;
    uint32_t c;
    uint8_t a;  // 0 keep, 1 clone, 2 split
    if (!densify) {
        a = 0;
        c = (faint || large) ? 0u : 1u;
    } else if (small) {
        a = 1;
        c = faint ? 0u : (large ? 1u : 2u);
    } else {
        a = 2;
        c = faint ? 0u : (uint32_t)P.split_n;
    }
    counts[i] = c;
    action[i] = a | (uint8_t)((faint || large) ? 4 : 0);  // bit 2: the parent itself is pruned
}

// exclusive scan of counts in blocks of DENS_SCAN: block totals first
__global__ __launch_bounds__(256) void k_dens_block_sum(const uint32_t* __restrict__ counts, int n,
                                                        uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t red[256];
    const int b = blockIdx.x;
    uint32_t v = 0;
    for (int k = threadIdx.x; k < DENS_SCAN; k += 256) {
        const int i = b * DENS_SCAN + k;
        if (i < n) v += counts[i];
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[b] = red[0];
}

// the block totals' exclusive scan (one workgroup, sequential over chunks of
// 256) and the total
__global__ __launch_bounds__(256) void k_dens_top(uint32_t* __restrict__ bsum, int nb, uint32_t* __restrict__ total)
{
    __shared__ uint32_t sh[256];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 256) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {  // inclusive Hillis-Steele
            const uint32_t t = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0u;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255) carry += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// per block: the exclusive scan of its counts plus the block offset, and
// each parent's output slots
__global__ __launch_bounds__(256) void k_dens_write(const uint32_t* __restrict__ counts,
                                                    const uint8_t* __restrict__ action, int n,
                                                    const uint32_t* __restrict__ bsum, int split_n,
                                                    int32_t* __restrict__ src, int32_t* __restrict__ kind)
{
    __shared__ uint32_t sh[DENS_SCAN];
    const int b = blockIdx.x;
    for (int k = threadIdx.x; k < DENS_SCAN; k += 256) {
        const int i = b * DENS_SCAN + k;
        sh[k] = i < n ? counts[i] : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // sequential within the block: 1024 adds
        uint32_t run = bsum[b];
        for (int k = 0; k < DENS_SCAN; ++k) {
            const uint32_t c = sh[k];
            sh[k] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < DENS_SCAN; k += 256) {
        const int i = b * DENS_SCAN + k;
        if (i >= n) break;
        const uint32_t c = counts[i];
        if (c == 0u) continue;
        uint32_t j = sh[k];
        const uint8_t a = action[i];
        const bool parent_pruned = (a & 4) != 0;
        switch (a & 3) {
            case 0:
                src[j] = i;
                kind[j] = DENS_KEEP;
                break;
            case 1:
                if (!parent_pruned) {
                    src[j] = i;
                    kind[j] = DENS_KEEP;
                    ++j;
                }
                src[j] = i;
                kind[j] = DENS_CLONE;
                break;
            default:
                for (int ch = 0; ch < split_n; ++ch) {
                    src[j + ch] = i;
                    kind[j + ch] = ch;
                }
                break;
        }
    }
}

// the new scene: parents copied, split children displaced and shrunk
__global__ __launch_bounds__(256) void k_dens_apply(int n, int n_out, const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ kind, const float* __restrict__ mean,
                                                    const float* __restrict__ log_scale,
                                                    const float* __restrict__ quat,
                                                    const float* __restrict__ opacity_logit,
                                                    const float* __restrict__ xi, int split_n,
                                                    float* __restrict__ o_mean, float* __restrict__ o_log_scale,
                                                    float* __restrict__ o_quat, float* __restrict__ o_opacity_logit)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_out) return;
    const int i = src[j], k = kind[j];
    float m[3] = {mean[i], mean[n + i], mean[2 * n + i]};
    float l[3] = {log_scale[i], log_scale[n + i], log_scale[2 * n + i]};
    const float qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
    if (k >= 0) {
        // R(q) (s * xi) for the unit quaternion (w, x, y, z), the projection's convention
        const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        const float w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
        const float* e = xi + ((size_t)i * split_n + k) * 3;
        const float u0 = expf(l[0]) * e[0], u1 = expf(l[1]) * e[1], u2 = expf(l[2]) * e[2];
        m[0] += (1.0f - 2.0f * (y * y + z * z)) * u0 + 2.0f * (x * y - w * z) * u1 + 2.0f * (x * z + w * y) * u2;
        m[1] += 2.0f * (x * y + w * z) * u0 + (1.0f - 2.0f * (x * x + z * z)) * u1 + 2.0f * (y * z - w * x) * u2;
        m[2] += 2.0f * (x * z - w * y) * u0 + 2.0f * (y * z + w * x) * u1 + (1.0f - 2.0f * (x * x + y * y)) * u2;
        const float shrink = logf(0.8f * (float)split_n);
        l[0] -= shrink;
        l[1] -= shrink;
        l[2] -= shrink;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o_mean[(size_t)c * n_out + j] = m[c];
        o_log_scale[(size_t)c * n_out + j] = l[c];
    }
    o_quat[j] = qw;
    o_quat[(size_t)n_out + j] = qx;
    o_quat[2 * (size_t)n_out + j] = qy;
    o_quat[3 * (size_t)n_out + j] = qz;
    o_opacity_logit[j] = opacity_logit[i];
}

// out[c][j][w] = in[c][src[j]][w] (32-bit words), zero for new Gaussians when asked
__global__ __launch_bounds__(256) void k_dens_gather(int n, int n_out, const int32_t* __restrict__ src,
                                                     const int32_t* __restrict__ kind,
                                                     const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                     int comps, int width, int zero_new)
{
    const size_t total = (size_t)comps * n_out * width;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int w = (int)(t % width);
        const size_t r = t / width;
        const int j = (int)(r % n_out), c = (int)(r / n_out);
        const bool fresh = zero_new && kind[j] != DENS_KEEP;
        out[t] = fresh ? 0u : in[((size_t)c * n + src[j]) * width + w];
    }
}

__global__ __launch_bounds__(256) void k_dens_reset(int n, float* __restrict__ opacity_logit, float cap_logit)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) opacity_logit[i] = fminf(opacity_logit[i], cap_logit);
}

// half the larger side of the support rectangle (pixels); 0 for culled
__global__ __launch_bounds__(256) void k_dens_radius(int n, const int4* __restrict__ rect,
                                                     const uint32_t* __restrict__ status, float* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int4 r = rect[i];
    out[i] = status[i] == ST_VISIBLE ? 0.5f * (float)max(r.y - r.x + 1, r.w - r.z + 1) : 0.0f;
}

}  // namespace gs

using namespace gs;

extern "C" {

gs_status gs_densify_stats(const float* d_mean, int32_t n, const uint32_t* live_list, const uint32_t* live_count,
                           float* grad_acc, uint32_t* grad_cnt, void* stream)
{
    if (!d_mean || !live_list || !live_count || !grad_acc || !grad_cnt || n < 1) return GS_ERR_INVALID_ARG;
    (void)hipGetLastError();
    const int blocks = std::min(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_dens_stats, dim3(blocks), dim3(256), 0, (hipStream_t)stream, d_mean, n, live_list,
                       live_count, grad_acc, grad_cnt);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

size_t gs_densify_scratch_bytes(int32_t n)
{
    if (n < 1) return 0;
    const size_t nb = ((size_t)n + DENS_SCAN - 1) / DENS_SCAN;
    return align256((size_t)n * 4) + align256((size_t)n) + align256(nb * 4);
}

gs_status gs_densify_plan(int32_t n, const float* log_scale, const float* opacity_logit, const float* grad_acc,
                          const uint32_t* grad_cnt, const float* screen_radius, const gs_densify_params* prm,
                          int32_t* src, int32_t* kind, int64_t out_capacity, uint32_t* n_out, void* scratch,
                          size_t scratch_bytes, void* stream)
{
    if (!log_scale || !opacity_logit || !grad_acc || !grad_cnt || !prm || !src || !kind || !n_out || n < 1)
        return GS_ERR_INVALID_ARG;
    if (prm->split_n < 2 || prm->split_n > 64 || !(prm->grad_threshold > 0.0f) || !(prm->clone_extent >= 0.0f) ||
        !(prm->opacity_min >= 0.0f) || !(prm->radius_max > 0.0f))
        return GS_ERR_INVALID_ARG;
    if ((int64_t)n * prm->split_n > 0x7FFFFFFF) return GS_ERR_CAPACITY;
    if (out_capacity < (int64_t)n * prm->split_n) return GS_ERR_WORKSPACE;
    if (!scratch || ((uintptr_t)scratch & 255) || scratch_bytes < gs_densify_scratch_bytes(n)) return GS_ERR_WORKSPACE;
    char* sc = (char*)scratch;
    uint32_t* counts = (uint32_t*)sc;
    uint8_t* action = (uint8_t*)(sc + align256((size_t)n * 4));
    uint32_t* bsum = (uint32_t*)(sc + align256((size_t)n * 4) + align256((size_t)n));
    const int nb = (n + DENS_SCAN - 1) / DENS_SCAN;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_dens_count, dim3((n + 255) / 256), dim3(256), 0, s, n, log_scale, opacity_logit, grad_acc,
                       grad_cnt, screen_radius, *prm, counts, action);
    hipLaunchKernelGGL(k_dens_block_sum, dim3(nb), dim3(256), 0, s, counts, n, bsum);
    hipLaunchKernelGGL(k_dens_top, dim3(1), dim3(256), 0, s, bsum, nb, n_out);
    hipLaunchKernelGGL(k_dens_write, dim3(nb), dim3(256), 0, s, counts, action, n, bsum, prm->split_n, src, kind);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_densify_apply(int32_t n, int32_t n_out, const int32_t* src, const int32_t* kind,
                           const gs_scene* scene, const float* xi, int32_t split_n, float* o_mean,
                           float* o_log_scale, float* o_quat, float* o_opacity_logit, void* stream)
{
    if (!src || !kind || !scene || !scene->mean || !scene->log_scale || !scene->quat || !scene->opacity_logit ||
        !xi || !o_mean || !o_log_scale || !o_quat || !o_opacity_logit || n < 1 || n_out < 0 || split_n < 2 ||
        split_n > 64 || scene->n != n)
        return GS_ERR_INVALID_ARG;
    if (n_out == 0) return GS_OK;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_dens_apply, dim3((n_out + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, n_out, src,
                       kind, scene->mean, scene->log_scale, scene->quat, scene->opacity_logit, xi, split_n, o_mean,
                       o_log_scale, o_quat, o_opacity_logit);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_densify_gather(int32_t n, int32_t n_out, const int32_t* src, const int32_t* kind, const void* in,
                            void* out, int32_t comps, int32_t width_words, int32_t zero_new, void* stream)
{
    if (!src || !kind || !in || !out || n < 1 || n_out < 0 || comps < 1 || width_words < 1) return GS_ERR_INVALID_ARG;
    if (n_out == 0) return GS_OK;
    const size_t total = (size_t)comps * n_out * width_words;
    const size_t blocks = std::min<size_t>(4096, (total + 255) / 256);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_dens_gather, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, n, n_out, src, kind,
                       (const uint32_t*)in, (uint32_t*)out, comps, width_words, zero_new ? 1 : 0);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_opacity_reset(int32_t n, float* opacity_logit, float opacity_cap, void* stream)
{
    if (!opacity_logit || n < 1 || !(opacity_cap > 0.0f && opacity_cap < 1.0f)) return GS_ERR_INVALID_ARG;
    const float cap_logit = logf(opacity_cap / (1.0f - opacity_cap));
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_dens_reset, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, opacity_logit,
                       cap_logit);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_screen_radius(const void* workspace, size_t ws_bytes, int32_t n, int32_t n_queries,
                           const gs_grid* grid, const gs_params* prm, int32_t q, float* radius, void* stream)
{
    if (!radius || q < 0 || q >= n_queries) return GS_ERR_INVALID_ARG;
    Layout L;
    gs_status st = make_layout(n, n_queries, grid, prm, &L);
    if (st != GS_OK) return st;
    if (!workspace || ws_bytes < L.total) return GS_ERR_WORKSPACE;
    const char* ws = (const char*)workspace;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_dens_radius, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n,
                       (const int4*)(ws + L.rect + (size_t)q * L.s_rect), (const uint32_t*)(ws + L.status + (size_t)q * L.s_status),
                       radius);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

}  // extern "C"
