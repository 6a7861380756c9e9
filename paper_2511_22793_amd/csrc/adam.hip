// Fused Adam (Kingma and Ba) over several parameter segments in one launch;
// segments that feed the BF16 matrix cores also refresh their BF16 copy.
#include "common.h"

namespace gs {

constexpr int ADAM_MAX_SEGS = 16;

struct AdamSegs {
    float* p[ADAM_MAX_SEGS];
    const float* g[ADAM_MAX_SEGS];
    float* m[ADAM_MAX_SEGS];
    float* v[ADAM_MAX_SEGS];
    uint16_t* sh[ADAM_MAX_SEGS];
    int64_t start[ADAM_MAX_SEGS + 1];  // prefix of counts
    float lr[ADAM_MAX_SEGS];
    float lr_log2_ratio[ADAM_MAX_SEGS];  // log2(lr_final / lr) of a scheduled segment, else 0
    int nseg;
};

__device__ __forceinline__ uint16_t f2bf_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// step_dev (device, or null): the number of completed steps t; then the
// bias corrections use step t + 1 and a scheduled segment's rate is
// lr (lr_final / lr)^u, u = min((t + 1) / (total_steps - 1), 1) (log-linear decay),
// all formed on the device so that a captured graph replays correctly.
__global__ __launch_bounds__(256) void k_adam(AdamSegs S, float b1, float b2, float eps, float c1, float c2,
                                              const uint32_t* __restrict__ skip_if, uint32_t* __restrict__ skip_count,
                                              const uint32_t* __restrict__ step_dev, float inv_span)
{
    // a set guard word (e.g. a render's pair-overflow flag) leaves every
    // parameter and moment untouched; one thread counts the skipped step
    if (skip_if && *skip_if) {
        if (skip_count && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(skip_count, 1u);
        return;
    }
    float u = 0.0f;
    if (step_dev) {
        const uint32_t t = *step_dev;
        c1 = (float)(1.0 - pow((double)b1, (double)(t + 1)));
        c2 = (float)(1.0 - pow((double)b2, (double)(t + 1)));
        u = fminf((float)(t + 1) * inv_span, 1.0f);
    }
    const int64_t total = S.start[S.nseg];
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int k = 0;
        while (e >= S.start[k + 1]) ++k;
        const int64_t i = e - S.start[k];
        const float g = S.g[k][i];
        const float m = b1 * S.m[k][i] + (1.0f - b1) * g;
        const float v = b2 * S.v[k][i] + (1.0f - b2) * g * g;
        S.m[k][i] = m;
        S.v[k][i] = v;
        const float lr = S.lr_log2_ratio[k] != 0.0f ? S.lr[k] * exp2f(u * S.lr_log2_ratio[k]) : S.lr[k];
        const float p = S.p[k][i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
        S.p[k][i] = p;
        if (S.sh[k]) S.sh[k][i] = f2bf_rne(p);
    }
}

// one completed step more (after the update of a device-scheduled step)
__global__ void k_step_advance(uint32_t* step_dev)
{
    if (threadIdx.x == 0) *step_dev += 1u;
}

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_adam_step(const gs_adam_segment* segs, int32_t n_segs, int32_t step, float beta1,
                                  float beta2, float eps, const uint32_t* skip_if, uint32_t* skip_count,
                                  void* stream)
{
    if (!segs || n_segs < 1 || n_segs > ADAM_MAX_SEGS || step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return GS_ERR_INVALID_ARG;
    AdamSegs S{};
    S.nseg = n_segs;
    int64_t total = 0;
    for (int k = 0; k < n_segs; ++k) {
        const gs_adam_segment& a = segs[k];
        if (!a.p || !a.g || !a.m || !a.v || a.count < 0) return GS_ERR_INVALID_ARG;
        S.p[k] = a.p; S.g[k] = a.g; S.m[k] = a.m; S.v[k] = a.v; S.sh[k] = a.shadow; S.lr[k] = a.lr;
        S.start[k] = total;
        total += a.count;
    }
    S.start[n_segs] = total;
    if (total == 0) return GS_OK;
    const double c1 = 1.0 - pow((double)beta1, step), c2 = 1.0 - pow((double)beta2, step);
    (void)hipGetLastError();
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, (hipStream_t)stream,
                       S, beta1, beta2, eps, (float)c1, (float)c2, skip_if, skip_count, (const uint32_t*)nullptr,
                       0.0f);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

extern "C" gs_status gs_adam_step_scheduled(const gs_adam_segment* segs, const float* lr_final, int32_t n_segs,
                                            int32_t total_steps, uint32_t* step_counter, float beta1, float beta2,
                                            float eps, const uint32_t* skip_if, uint32_t* skip_count, void* stream)
{
    if (!segs || !step_counter || n_segs < 1 || n_segs > ADAM_MAX_SEGS || total_steps < 1 ||
        !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return GS_ERR_INVALID_ARG;
    AdamSegs S{};
    S.nseg = n_segs;
    int64_t total = 0;
    for (int k = 0; k < n_segs; ++k) {
        const gs_adam_segment& a = segs[k];
        if (!a.p || !a.g || !a.m || !a.v || a.count < 0) return GS_ERR_INVALID_ARG;
        S.p[k] = a.p; S.g[k] = a.g; S.m[k] = a.m; S.v[k] = a.v; S.sh[k] = a.shadow; S.lr[k] = a.lr;
        if (lr_final && lr_final[k] != a.lr) {
            if (!(a.lr > 0.0f) || !(lr_final[k] > 0.0f)) return GS_ERR_INVALID_ARG;
            S.lr_log2_ratio[k] = (float)log2((double)lr_final[k] / (double)a.lr);
        }
        S.start[k] = total;
        total += a.count;
    }
    S.start[n_segs] = total;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    const int64_t blocks = (total + 255) / 256;
    if (total > 0)
        hipLaunchKernelGGL(k_adam, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, S, beta1, beta2,
                           eps, 1.0f, 1.0f, skip_if, skip_count, (const uint32_t*)step_counter,
                           total_steps > 1 ? 1.0f / (float)(total_steps - 1) : 0.0f);
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step_counter);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}
