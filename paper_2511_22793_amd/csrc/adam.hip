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
    int64_t start[ADAM_MAX_SEGS + 1];  // prefix of the counts, each rounded up to a multiple of 4
    int64_t count[ADAM_MAX_SEGS];
    float lr[ADAM_MAX_SEGS];
    float lr_log2_ratio[ADAM_MAX_SEGS];  // log2(lr_final / lr) of a scheduled segment, else 0
    int vec[ADAM_MAX_SEGS];              // 1: p, g, m, v 16-byte aligned (and the shadow 8-byte)
    int nseg;
};

__device__ __forceinline__ uint16_t f2bf_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct AdamConst {
    float b1, b2, eps, c1, c2, lr;
};

__device__ __forceinline__ float adam_one(float p, float g, float& m, float& v, const AdamConst& K)
{
    m = K.b1 * m + (1.0f - K.b1) * g;
    v = K.b2 * v + (1.0f - K.b2) * g * g;
    return p - K.lr * (m / K.c1) / (sqrtf(v / K.c2) + K.eps);
}

// step_dev (device, or null): the number of completed steps t; then the
// bias corrections use step t + 1 and a scheduled segment's rate is
// lr (lr_final / lr)^u, u = min((t + 1) / (total_steps - 1), 1) (log-linear decay),
// all formed on the device (once per workgroup) so that a captured graph
// replays correctly.  Each thread takes 4 consecutive elements of one
// segment: one 16-byte load of each of p, g, m, v where the segment is
// aligned for it.
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
    __shared__ float s_c[3];
    if (step_dev) {
        if (threadIdx.x == 0) {
            const uint32_t t = *step_dev;
            s_c[0] = (float)(1.0 - pow((double)b1, (double)(t + 1)));
            s_c[1] = (float)(1.0 - pow((double)b2, (double)(t + 1)));
            s_c[2] = fminf((float)(t + 1) * inv_span, 1.0f);
        }
        __syncthreads();
    }
    AdamConst K{b1, b2, eps, step_dev ? s_c[0] : c1, step_dev ? s_c[1] : c2, 0.0f};
    const float u = step_dev ? s_c[2] : 0.0f;
    const int64_t total = S.start[S.nseg];
    for (int64_t e = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x); e < total; e += 4 * (int64_t)gridDim.x * 256) {
        int k = 0;
        while (e >= S.start[k + 1]) ++k;
        const int64_t i = e - S.start[k];  // a multiple of 4
        const int64_t cnt = S.count[k];
        K.lr = S.lr_log2_ratio[k] != 0.0f ? S.lr[k] * exp2f(u * S.lr_log2_ratio[k]) : S.lr[k];
        if (S.vec[k] && i + 4 <= cnt) {
            const float4 g = *(const float4*)(S.g[k] + i);
            float4 m = *(const float4*)(S.m[k] + i);
            float4 v = *(const float4*)(S.v[k] + i);
            float4 p = *(const float4*)(S.p[k] + i);
            p.x = adam_one(p.x, g.x, m.x, v.x, K);
            p.y = adam_one(p.y, g.y, m.y, v.y, K);
            p.z = adam_one(p.z, g.z, m.z, v.z, K);
            p.w = adam_one(p.w, g.w, m.w, v.w, K);
            *(float4*)(S.m[k] + i) = m;
            *(float4*)(S.v[k] + i) = v;
            *(float4*)(S.p[k] + i) = p;
            if (S.sh[k]) {
                const uint32_t lo = (uint32_t)f2bf_rne(p.x) | ((uint32_t)f2bf_rne(p.y) << 16);
                const uint32_t hi = (uint32_t)f2bf_rne(p.z) | ((uint32_t)f2bf_rne(p.w) << 16);
                *(uint2*)(S.sh[k] + i) = make_uint2(lo, hi);
            }
        } else {
            for (int64_t j = i; j < i + 4 && j < cnt; ++j) {
                float m = S.m[k][j], v = S.v[k][j];
                const float p = adam_one(S.p[k][j], S.g[k][j], m, v, K);
                S.m[k][j] = m;
                S.v[k][j] = v;
                S.p[k][j] = p;
                if (S.sh[k]) S.sh[k][j] = f2bf_rne(p);
            }
        }
    }
}

// fills the segment table; false on an invalid segment
static bool adam_segs(const gs_adam_segment* segs, int n_segs, AdamSegs* S)
{
    S->nseg = n_segs;
    int64_t total = 0;
    for (int k = 0; k < n_segs; ++k) {
        const gs_adam_segment& a = segs[k];
        if (!a.p || !a.g || !a.m || !a.v || a.count < 0) return false;
        S->p[k] = a.p; S->g[k] = a.g; S->m[k] = a.m; S->v[k] = a.v; S->sh[k] = a.shadow; S->lr[k] = a.lr;
        S->count[k] = a.count;
        const uintptr_t al = (uintptr_t)a.p | (uintptr_t)a.g | (uintptr_t)a.m | (uintptr_t)a.v;
        S->vec[k] = (al & 15) == 0 && ((uintptr_t)a.shadow & 7) == 0;
        S->start[k] = total;
        total += (a.count + 3) / 4 * 4;
    }
    S->start[n_segs] = total;
    return true;
}

static unsigned adam_blocks(int64_t total)
{
    const int64_t blocks = (total / 4 + 255) / 256;
    return (unsigned)(blocks < 4096 ? (blocks ? blocks : 1) : 4096);
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
    if (!adam_segs(segs, n_segs, &S)) return GS_ERR_INVALID_ARG;
    const int64_t total = S.start[n_segs];
    if (total == 0) return GS_OK;
    const double c1 = 1.0 - pow((double)beta1, step), c2 = 1.0 - pow((double)beta2, step);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_adam, dim3(adam_blocks(total)), dim3(256), 0, (hipStream_t)stream, S, beta1, beta2, eps,
                       (float)c1, (float)c2, skip_if, skip_count, (const uint32_t*)nullptr, 0.0f);
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
    if (!adam_segs(segs, n_segs, &S)) return GS_ERR_INVALID_ARG;
    for (int k = 0; k < n_segs; ++k) {
        const gs_adam_segment& a = segs[k];
        if (lr_final && lr_final[k] != a.lr) {
            if (!(a.lr > 0.0f) || !(lr_final[k] > 0.0f)) return GS_ERR_INVALID_ARG;
            S.lr_log2_ratio[k] = (float)log2((double)lr_final[k] / (double)a.lr);
        }
    }
    const int64_t total = S.start[n_segs];
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    if (total > 0)
        hipLaunchKernelGGL(k_adam, dim3(adam_blocks(total)), dim3(256), 0, s, S, beta1, beta2, eps, 1.0f, 1.0f,
                           skip_if, skip_count, (const uint32_t*)step_counter,
                           total_steps > 1 ? 1.0f / (float)(total_steps - 1) : 0.0f);
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step_counter);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}
