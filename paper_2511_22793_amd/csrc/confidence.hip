// Confidence head and confidence-weighted loss (Sec. 4.2, Eq. (6)).
//
// Per sample b: h = relu(W1 x_b + b1) (32 hidden units), g = w2 . h + b2,
// C = 1 + exp(g), L_conf = C L_task - alpha log C.  The gradients of the
// batch sum of L_conf: dL/dL_task = C, dL/dC = L_task - alpha / C,
// dC/dg = C - 1, then through the two layers.
//
// One workgroup of sixteen waves.  Each half of a wave (32 lanes) takes one
// sample at a time, lane j of the half owning hidden unit j; the half forms
// g with a 32-lane reduction and keeps its lane's partial weight gradients in
// registers; the 32 halves' partials are added in LDS in a fixed order, so
// the result does not depend on timing.
#include "common.h"

namespace gs {

constexpr int CONF_HIDDEN = 32;
constexpr int CONF_WAVES = 16;
constexpr int CONF_HALVES = 2 * CONF_WAVES;

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
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, gb = 0.0f, gv = 0.0f, go = 0.0f;
    for (int b = half; b < n; b += CONF_HALVES) {
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
        g0 = fmaf(dh, x0, g0);
        g1 = fmaf(dh, x1, g1);
        g2 = fmaf(dh, x2, g2);
        gb += dh;
        gv = fmaf(dg, h, gv);
        go += dg;
    }
    // (the two halves of a wave may run different trip counts; the
    // reduction above never crosses a half)
    __shared__ float part[CONF_HALVES][6][CONF_HIDDEN];
    part[half][0][j] = g0;
    part[half][1][j] = g1;
    part[half][2][j] = g2;
    part[half][3][j] = gb;
    part[half][4][j] = gv;
    part[half][5][j] = go;
    __syncthreads();
    if (threadIdx.x < CONF_HIDDEN) {
        float r[6];
        for (int k = 0; k < 6; ++k) {
            float v = 0.0f;
            for (int w = 0; w < CONF_HALVES; ++w) v += part[w][k][j];
            r[k] = v;
        }
        dW1[3 * j] = r[0];
        dW1[3 * j + 1] = r[1];
        dW1[3 * j + 2] = r[2];
        db1[j] = r[3];
        dw2[j] = r[4];
        if (j == 0) db2[0] = r[5];  // every lane of a half holds the same dg sum
    }
}

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_confidence_loss(const float* x_rx, const float* task_loss, int32_t n, const float* W1,
                                        const float* b1, const float* w2, const float* b2, float alpha,
                                        float* conf, float* loss, float* dW1, float* db1, float* dw2, float* db2,
                                        void* stream)
{
    if (!x_rx || !task_loss || !W1 || !b1 || !w2 || !b2 || !conf || !loss || !dW1 || !db1 || !dw2 || !db2 ||
        n < 1 || !(alpha >= 0.0f) || !(alpha < INFINITY))
        return GS_ERR_INVALID_ARG;
    if (n > 65536) return GS_ERR_CAPACITY;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_confidence, dim3(1), dim3(CONF_WAVES * 64), 0, (hipStream_t)stream, x_rx, task_loss, n,
                       W1, b1, w2, b2, alpha, conf, loss, dW1, db1, dw2, db2);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}
