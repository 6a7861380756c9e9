// The paper's own emission form: one 3 -> H -> 2 network per Gaussian
// (Sec. 4.1, Eq. (1); H = 16, and 8 or 64 for the width ablation).  For
// query q (receiver rx_q, transmitter tx_q):
//   h = relu(W1_i rx_q + b1_i), f = W2_i h + b2_i,
//   d = max(|tx_q - mu_i|, r_near),  s = sigmoid(f - log d)  (Re, Im);
// the means in the scene's layout [3][n].
// Parameters are stored per parameter index, then per Gaussian
// (params[k * stride + i], k < 6H + 2: W1 [H][3], b1 [H], W2 [2][H], b2 [2]),
// so that one load instruction of a wave reads 64 consecutive Gaussians.
// One thread per Gaussian holds its 6H + 2 parameters in registers and takes
// every query, so the parameters leave HBM once per launch (a batched
// matrix-vector product: HBM-bound, not a matrix-core shape).
#include "common.h"

namespace gs {

// parameters of a width-H network: W1 at 0 (3H), b1 at 3H, W2 at 4H (2H), b2 at 6H (2)
__host__ __device__ constexpr int em_np(int H) { return 6 * H + 2; }

__device__ __forceinline__ float em_sigmoid(float u) { return 1.0f / (1.0f + expf(-u)); }

template <int H>
__global__ __launch_bounds__(256) void k_emission_fwd(const float* __restrict__ P, int64_t ps,
                                                      const float* __restrict__ mean, int n,
                                                      const float* __restrict__ rx, const float* __restrict__ tx,
                                                      int nq, float r_near, float* __restrict__ attr, int64_t as)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int NP = em_np(H);
    float p[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) p[k] = P[(size_t)k * ps + i];
    const float m0 = mean[i], m1 = mean[n + i], m2 = mean[2 * n + i];  // [3][n], as the scene
    for (int q = 0; q < nq; ++q) {
        const float x0 = rx[3 * q], x1 = rx[3 * q + 1], x2 = rx[3 * q + 2];
        float f0 = p[6 * H], f1 = p[6 * H + 1];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const float z = fmaf(p[3 * j], x0, fmaf(p[3 * j + 1], x1, fmaf(p[3 * j + 2], x2, p[3 * H + j])));
            const float h = fmaxf(z, 0.0f);
            f0 = fmaf(p[4 * H + j], h, f0);
            f1 = fmaf(p[5 * H + j], h, f1);
        }
        const float v0 = tx[3 * q] - m0, v1 = tx[3 * q + 1] - m1, v2 = tx[3 * q + 2] - m2;
        const float d = fmaxf(sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2))), r_near);
        const float ld = logf(d);
        float2* o = (float2*)(attr + q * as) + i;
        *o = float2{em_sigmoid(f0 - ld), em_sigmoid(f1 - ld)};
    }
}

template <int H>
__global__ __launch_bounds__(256) void k_emission_bwd(const float* __restrict__ P, int64_t ps,
                                                      const float* __restrict__ mean, int n,
                                                      const float* __restrict__ rx, const float* __restrict__ tx,
                                                      int nq, float r_near, const float* __restrict__ dattr,
                                                      int64_t as, float* __restrict__ dP,
                                                      float* __restrict__ dmean)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int NP = em_np(H);
    float p[NP], g[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        p[k] = P[(size_t)k * ps + i];
        g[k] = 0.0f;
    }
    const float m0 = mean[i], m1 = mean[n + i], m2 = mean[2 * n + i];  // [3][n], as the scene
    float gm0 = 0.0f, gm1 = 0.0f, gm2 = 0.0f;
    for (int q = 0; q < nq; ++q) {
        const float x0 = rx[3 * q], x1 = rx[3 * q + 1], x2 = rx[3 * q + 2];
        float z[H];
        float f0 = p[6 * H], f1 = p[6 * H + 1];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            z[j] = fmaf(p[3 * j], x0, fmaf(p[3 * j + 1], x1, fmaf(p[3 * j + 2], x2, p[3 * H + j])));
            const float h = fmaxf(z[j], 0.0f);
            f0 = fmaf(p[4 * H + j], h, f0);
            f1 = fmaf(p[5 * H + j], h, f1);
        }
        const float v0 = tx[3 * q] - m0, v1 = tx[3 * q + 1] - m1, v2 = tx[3 * q + 2] - m2;
        const float dist = sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
        const float d = fmaxf(dist, r_near);
        const float ld = logf(d);
        const float s0 = em_sigmoid(f0 - ld), s1 = em_sigmoid(f1 - ld);
        const float2 up = ((const float2*)(dattr + q * as))[i];
        const float u0 = up.x * s0 * (1.0f - s0), u1 = up.y * s1 * (1.0f - s1);
        g[6 * H] += u0;
        g[6 * H + 1] += u1;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const float h = fmaxf(z[j], 0.0f);
            g[4 * H + j] = fmaf(u0, h, g[4 * H + j]);
            g[5 * H + j] = fmaf(u1, h, g[5 * H + j]);
            const float dz = z[j] > 0.0f ? fmaf(u0, p[4 * H + j], u1 * p[5 * H + j]) : 0.0f;
            g[3 * H + j] += dz;
            g[3 * j] = fmaf(dz, x0, g[3 * j]);
            g[3 * j + 1] = fmaf(dz, x1, g[3 * j + 1]);
            g[3 * j + 2] = fmaf(dz, x2, g[3 * j + 2]);
        }
        // d(-log d)/d mu = (tx - mu) / d^2 where d is not floored
        if (dist > r_near) {
            const float c = -(u0 + u1) / (dist * dist);  // dL/dlog d times d(log d)/d mu = -v / d^2
            gm0 = fmaf(-c, v0, gm0);
            gm1 = fmaf(-c, v1, gm1);
            gm2 = fmaf(-c, v2, gm2);
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) dP[(size_t)k * ps + i] = g[k];
    dmean[i] = gm0;
    dmean[n + i] = gm1;
    dmean[2 * n + i] = gm2;
}

static gs_status em_check(const float* P, int64_t ps, const float* mean, int n, const float* rx, const float* tx,
                          int nq, float r_near, int64_t as)
{
    if (!P || !mean || !rx || !tx || n < 1 || nq < 1 || ps < n || as < 2 * (int64_t)n || (as & 1) || !(r_near > 0.0f) ||
        !(r_near < INFINITY))
        return GS_ERR_INVALID_ARG;
    if (nq > 1024) return GS_ERR_CAPACITY;
    return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_emission_forward(const float* params, int64_t param_stride, int32_t hidden, const float* mean, int32_t n,
                                         const float* rx, const float* tx, int32_t n_queries, float r_near,
                                         float* attr, int64_t attr_query_stride, void* stream)
{
    gs_status st = em_check(params, param_stride, mean, n, rx, tx, n_queries, r_near, attr_query_stride);
    if (st != GS_OK) return st;
    if (!attr || (hidden != 8 && hidden != 16 && hidden != 64)) return GS_ERR_INVALID_ARG;
    (void)hipGetLastError();
    auto kern = hidden == 8 ? k_emission_fwd<8> : (hidden == 16 ? k_emission_fwd<16> : k_emission_fwd<64>);
    hipLaunchKernelGGL(kern, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, param_stride, mean,
                       n, rx, tx, n_queries, r_near, attr, attr_query_stride);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

extern "C" gs_status gs_emission_backward(const float* params, int64_t param_stride, int32_t hidden, const float* mean, int32_t n,
                                          const float* rx, const float* tx, int32_t n_queries, float r_near,
                                          const float* d_attr, int64_t attr_query_stride, float* d_params,
                                          float* d_mean, void* stream)
{
    gs_status st = em_check(params, param_stride, mean, n, rx, tx, n_queries, r_near, attr_query_stride);
    if (st != GS_OK) return st;
    if (!d_attr || !d_params || !d_mean || (hidden != 8 && hidden != 16 && hidden != 64)) return GS_ERR_INVALID_ARG;
    (void)hipGetLastError();
    auto kern = hidden == 8 ? k_emission_bwd<8> : (hidden == 16 ? k_emission_bwd<16> : k_emission_bwd<64>);
    hipLaunchKernelGGL(kern, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, param_stride, mean,
                       n, rx, tx, n_queries, r_near, d_attr, attr_query_stride, d_params, d_mean);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}
