// Confidence head and confidence-weighted loss (Sec. 4.2, Eq. (6)).
//
// Per sample b: h = relu(W1 x_b + b1) (32 hidden units), g = w2 . h + b2,
// C = 1 + exp(g), L_conf = C L_task - alpha log C.  The gradients of the
// batch sum of L_conf: dL/dL_task = C, dL/dC = L_task - alpha / C,
// dC/dg = C - 1, then through the two layers.
//
// Workgroups of sixteen waves.  Each half of a wave (32 lanes) takes one
// sample at a time, lane j of the half owning hidden unit j; the half forms
// g with a 32-lane reduction and keeps its lane's partial weight gradients in
// registers; the 32 halves' partials are added in LDS in a fixed order.  Up
// to CONF_ONE samples one workgroup does everything; beyond, G workgroups
// (G set by n alone) take fixed chunks of CONF_CHUNK samples each, write
// their partials to the caller's scratch, and one more workgroup adds the G
// partials in workgroup order: the result does not depend on timing either
// way.
#include "common.h"

namespace gs {

constexpr int CONF_HIDDEN = 32;
constexpr int CONF_WAVES = 16;
constexpr int CONF_HALVES = 2 * CONF_WAVES;
constexpr int CONF_ONE = 4096;                  // largest n taken by one workgroup
constexpr int CONF_CHUNK = 8 * CONF_HALVES;     // samples of one chunk (eight per half)
constexpr int CONF_MAX_WG = 1024;               // workgroups of the multi-workgroup path
constexpr int CONF_MAX_N = 1 << 24;
constexpr int CONF_NPART = 6 * CONF_HIDDEN;     // partial sums per workgroup

__host__ __device__ inline int conf_groups(int n)
{
    const int c = (n + CONF_CHUNK - 1) / CONF_CHUNK;
    return c < CONF_MAX_WG ? c : CONF_MAX_WG;
}

// One sample b through the head (half-wave, lane j = hidden unit j): the
// outputs, and this lane's gradient terms added to acc[6].
__device__ __forceinline__ void conf_sample(int b, int j, const float* __restrict__ x,
                                            const float* __restrict__ task, float w10, float w11, float w12,
                                            float bj, float vj, float bias2, float alpha, float* __restrict__ conf,
                                            float* __restrict__ loss, float* acc)
{
    const float x0 = x[3 * b], x1 = x[3 * b + 1], x2 = x[3 * b + 2];
    const float z = fmaf(w10, x0, fmaf(w11, x1, fmaf(w12, x2, bj)));
    const float h = fmaxf(z, 0.0f);
    float s = vj * h;
    for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);  // within the half
    const float g = s + bias2;
    const float e = expf(g);
    const float C = 1.0f + e;
    const float L = task[b];
    if (j == 0) {
        conf[b] = C;
        loss[b] = C * L - alpha * logf(C);
    }
    const float dg = (L - alpha / C) * e;  // dL/dC * dC/dg
    const float dh = z > 0.0f ? dg * vj : 0.0f;
    acc[0] = fmaf(dh, x0, acc[0]);
    acc[1] = fmaf(dh, x1, acc[1]);
    acc[2] = fmaf(dh, x2, acc[2]);
    acc[3] += dh;
    acc[4] = fmaf(dg, h, acc[4]);
    acc[5] += dg;
}

// The workgroup's 32 halves' terms summed in LDS (half order): thread j <
// 32 ends with the workgroup totals r[6] of hidden unit j.
__device__ __forceinline__ void conf_wg_sum(const float* acc, int half, int j, float* r)
{
    __shared__ float part[CONF_HALVES][6][CONF_HIDDEN];
#pragma unroll
    for (int k = 0; k < 6; ++k) part[half][k][j] = acc[k];
    __syncthreads();
    if (threadIdx.x < CONF_HIDDEN) {
        for (int k = 0; k < 6; ++k) {
            float v = 0.0f;
            for (int w = 0; w < CONF_HALVES; ++w) v += part[w][k][j];
            r[k] = v;
        }
    }
}

__device__ __forceinline__ void conf_store(const float* r, int j, float* __restrict__ dW1, float* __restrict__ db1,
                                           float* __restrict__ dw2, float* __restrict__ db2)
{
    dW1[3 * j] = r[0];
    dW1[3 * j + 1] = r[1];
    dW1[3 * j + 2] = r[2];
    db1[j] = r[3];
    dw2[j] = r[4];
    if (j == 0) db2[0] = r[5];  // every lane of a half holds the same dg sum
}

__global__ __launch_bounds__(CONF_WAVES * 64) void k_confidence(const float* __restrict__ x,
                                                                const float* __restrict__ task, int n,
                                                                const float* __restrict__ W1,
                                                                const float* __restrict__ b1,
                                                                const float* __restrict__ w2,
                                                                const float* __restrict__ b2, float alpha,
                                                                float* __restrict__ conf, float* __restrict__ loss,
                                                                float* __restrict__ dW1, float* __restrict__ db1,
                                                                float* __restrict__ dw2, float* __restrict__ db2)
{
    const int j = threadIdx.x & 31, half = threadIdx.x >> 5;  // hidden unit, half-wave
    const float w10 = W1[3 * j], w11 = W1[3 * j + 1], w12 = W1[3 * j + 2];
    const float bj = b1[j], vj = w2[j];
    const float bias2 = b2[0];
    float acc[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int b = half; b < n; b += CONF_HALVES)
        conf_sample(b, j, x, task, w10, w11, w12, bj, vj, bias2, alpha, conf, loss, acc);
    // (the two halves of a wave may run different trip counts; the
    // reduction in conf_sample never crosses a half)
    float r[6];
    conf_wg_sum(acc, half, j, r);
    if (threadIdx.x < CONF_HIDDEN) conf_store(r, j, dW1, db1, dw2, db2);
}

// Multi-workgroup path: workgroup w takes chunks w, w + G, w + 2G, ... (in
// that order), sample b = c CONF_CHUNK + 32 i + half, i < 8, and writes its
// totals to part[w][6][32].
__global__ __launch_bounds__(CONF_WAVES * 64) void k_confidence_part(const float* __restrict__ x,
                                                                     const float* __restrict__ task, int n,
                                                                     const float* __restrict__ W1,
                                                                     const float* __restrict__ b1,
                                                                     const float* __restrict__ w2,
                                                                     const float* __restrict__ b2, float alpha,
                                                                     float* __restrict__ conf,
                                                                     float* __restrict__ loss,
                                                                     float* __restrict__ part)
{
    const int j = threadIdx.x & 31, half = threadIdx.x >> 5;
    const float w10 = W1[3 * j], w11 = W1[3 * j + 1], w12 = W1[3 * j + 2];
    const float bj = b1[j], vj = w2[j];
    const float bias2 = b2[0];
    float acc[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    const int nchunk = (n + CONF_CHUNK - 1) / CONF_CHUNK;
    for (int c = blockIdx.x; c < nchunk; c += gridDim.x)
        for (int i = 0; i < CONF_CHUNK / CONF_HALVES; ++i) {
            const int b = c * CONF_CHUNK + i * CONF_HALVES + half;
            if (b < n) conf_sample(b, j, x, task, w10, w11, w12, bj, vj, bias2, alpha, conf, loss, acc);
        }
    float r[6];
    conf_wg_sum(acc, half, j, r);
    if (threadIdx.x < CONF_HIDDEN)
        for (int k = 0; k < 6; ++k) part[((size_t)blockIdx.x * 6 + k) * CONF_HIDDEN + j] = r[k];
}

// the G workgroups' partials added in workgroup order (thread k*32 + j);
// CONF_SUM_BATCH loads in flight ahead of the additions, which keep the order
constexpr int CONF_SUM_BATCH = 16;
__global__ __launch_bounds__(CONF_NPART) void k_confidence_sum(const float* __restrict__ part, int G,
                                                               float* __restrict__ dW1, float* __restrict__ db1,
                                                               float* __restrict__ dw2, float* __restrict__ db2)
{
    __shared__ float r[6][CONF_HIDDEN];
    const int k = threadIdx.x / CONF_HIDDEN, j = threadIdx.x % CONF_HIDDEN;
    const float* p = part + (size_t)k * CONF_HIDDEN + j;
    constexpr size_t STEP = 6 * CONF_HIDDEN;  // one workgroup's partials
    float v = 0.0f;
    int w = 0;
    for (; w + CONF_SUM_BATCH <= G; w += CONF_SUM_BATCH) {
        float b[CONF_SUM_BATCH];
#pragma unroll
        for (int u = 0; u < CONF_SUM_BATCH; ++u) b[u] = p[(size_t)(w + u) * STEP];
#pragma unroll
        for (int u = 0; u < CONF_SUM_BATCH; ++u) v += b[u];
    }
    for (; w < G; ++w) v += p[(size_t)w * STEP];
    r[k][j] = v;
    __syncthreads();
    if (threadIdx.x < CONF_HIDDEN) {
        const float t[6] = {r[0][j], r[1][j], r[2][j], r[3][j], r[4][j], r[5][j]};
        conf_store(t, j, dW1, db1, dw2, db2);
    }
}

}  // namespace gs

using namespace gs;

extern "C" size_t gs_confidence_scratch_bytes(int32_t n)
{
    if (n <= CONF_ONE || n > CONF_MAX_N) return 0;
    return align256((size_t)conf_groups(n) * CONF_NPART * 4);
}

extern "C" gs_status gs_confidence_loss(const float* x_rx, const float* task_loss, int32_t n, const float* W1,
                                        const float* b1, const float* w2, const float* b2, float alpha,
                                        float* conf, float* loss, float* dW1, float* db1, float* dw2, float* db2,
                                        void* scratch, size_t scratch_bytes, void* stream)
{
    if (!x_rx || !task_loss || !W1 || !b1 || !w2 || !b2 || !conf || !loss || !dW1 || !db1 || !dw2 || !db2 ||
        n < 1 || !(alpha >= 0.0f) || !(alpha < INFINITY))
        return GS_ERR_INVALID_ARG;
    if (n > CONF_MAX_N) return GS_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    if (n <= CONF_ONE) {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_confidence, dim3(1), dim3(CONF_WAVES * 64), 0, s, x_rx, task_loss, n, W1, b1, w2, b2,
                           alpha, conf, loss, dW1, db1, dw2, db2);
        return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
    }
    if (!scratch || ((uintptr_t)scratch & 255) || scratch_bytes < gs_confidence_scratch_bytes(n))
        return GS_ERR_WORKSPACE;
    const int G = conf_groups(n);
    float* part = (float*)scratch;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_confidence_part, dim3(G), dim3(CONF_WAVES * 64), 0, s, x_rx, task_loss, n, W1, b1, w2, b2,
                       alpha, conf, loss, part);
    hipLaunchKernelGGL(k_confidence_sum, dim3(1), dim3(CONF_NPART), 0, s, part, G, dW1, db1, dw2, db2);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}
