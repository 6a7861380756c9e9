// The paper's own emission form: one 3 -> H -> 2 network per Gaussian
// (Sec. 4.1, Eq. (1); H = 16, and 8 or 64 for the width ablation).  For
// query q (receiver rx_q, transmitter tx_q):
//   h = relu(W1_i rx_q + b1_i), f = W2_i h + b2_i,
//   d = max(|tx_q - mu_i|, r_near),  s = sigmoid(f - log d)  (Re, Im);
// the means in the scene's layout [3][n].
// Parameters are stored per parameter index, then per Gaussian
// (params[k * stride + i], k < 6H + 2: W1 [H][3], b1 [H], W2 [2][H], b2 [2]),
// so that one load instruction of a wave reads 64 consecutive Gaussians.
// One thread per Gaussian (H = 8, 16; eight lanes per Gaussian at H = 64)
// holds its parameters in registers and takes every query, so the parameters
// leave HBM once per launch (a batched matrix-vector product: HBM-bound, not
// a matrix-core shape).
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

// Width 64: one Gaussian's 386 parameters (and as many gradients) do not fit
// one lane's registers, so L lanes share a Gaussian, each owning H / L hidden
// units (W1 rows, b1, both W2 columns of those units).  Lane t of the group
// sits at lane t * (64 / L) + g of the wave (g = the Gaussian inside the
// wave), so one load instruction still reads 64 / L consecutive Gaussians of
// a parameter row; f is summed over the group with xor shuffles.  b2, the
// output and the mean gradient are formed by every lane of the group alike
// and written by slice 0.
// Parameter rows through a raw buffer resource.  A lane's rows are those of
// its slice: W1 rows 3 (t HS + jj) + c, b1 row 3H + t HS + jj, W2 rows
// 4H / 5H + t HS + jj; the per-lane part of an offset is the slice's first
// row and the Gaussian, the rest (jj, c) is uniform over the wave (scalar
// operand), so four per-lane offsets serve every load and store (the host
// bounds 6H+2 rows of ps floats below 2^31 bytes).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t em_rsrc(const float* base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, 0x7FFFFFFF, 0x00020000);
}
__device__ __forceinline__ float em_ld(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t row_off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, row_off, 0));
}
__device__ __forceinline__ void em_st(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t row_off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, lane_off, row_off, 0);
}

template <int H, int L>
__device__ __forceinline__ float em_group_sum(float v)
{
#pragma unroll
    for (int o = 64 / L; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// per-lane byte offsets of the slice's W1, b1, W2 (f0), W2 (f1) rows
template <int H, int L>
struct EmOff {
    uint32_t w1, b1, wa, wb, b2;
    __device__ EmOff(int t, int i, int64_t ps)
    {
        constexpr int HS = H / L;
        const uint32_t rs = (uint32_t)ps * 4u, li = (uint32_t)i * 4u;
        w1 = (uint32_t)(3 * t * HS) * rs + li;
        b1 = (uint32_t)(3 * H + t * HS) * rs + li;
        wa = (uint32_t)(4 * H + t * HS) * rs + li;
        wb = (uint32_t)(5 * H + t * HS) * rs + li;
        b2 = (uint32_t)(6 * H) * rs + li;
    }
};

template <int H, int L>
__global__ __launch_bounds__(256) void k_emission_fwd_split(const float* __restrict__ P, int64_t ps,
                                                            const float* __restrict__ mean, int n,
                                                            const float* __restrict__ rx,
                                                            const float* __restrict__ tx, int nq, float r_near,
                                                            float* __restrict__ attr, int64_t as)
{
    constexpr int HS = H / L, GPW = 64 / L;
    const int lane = threadIdx.x & 63;
    const int t = lane / GPW, gl = lane % GPW;
    const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * GPW + gl;
    const bool ok = i < n;  // (no early exit: the group's lanes shuffle)
    const int ii = ok ? i : 0;
    const __amdgpu_buffer_rsrc_t rp = em_rsrc(P);
    const uint32_t rs = (uint32_t)ps * 4u;
    const EmOff<H, L> off(t, ii, ps);
    float w1[HS][3], b1[HS], w2a[HS], w2b[HS];
#pragma unroll
    for (int jj = 0; jj < HS; ++jj) {
#pragma unroll
        for (int c = 0; c < 3; ++c) w1[jj][c] = em_ld(rp, off.w1, (3 * jj + c) * rs);
        b1[jj] = em_ld(rp, off.b1, jj * rs);
        w2a[jj] = em_ld(rp, off.wa, jj * rs);
        w2b[jj] = em_ld(rp, off.wb, jj * rs);
    }
    const float b20 = em_ld(rp, off.b2, 0), b21 = em_ld(rp, off.b2, rs);
    const float m0 = mean[ii], m1 = mean[n + ii], m2 = mean[2 * n + ii];
#pragma unroll 1
    for (int q = 0; q < nq; ++q) {
        const float x0 = rx[3 * q], x1 = rx[3 * q + 1], x2 = rx[3 * q + 2];
        float f0 = 0.0f, f1 = 0.0f;
#pragma unroll
        for (int jj = 0; jj < HS; ++jj) {
            const float z = fmaf(w1[jj][0], x0, fmaf(w1[jj][1], x1, fmaf(w1[jj][2], x2, b1[jj])));
            const float h = fmaxf(z, 0.0f);
            f0 = fmaf(w2a[jj], h, f0);
            f1 = fmaf(w2b[jj], h, f1);
        }
        f0 = em_group_sum<H, L>(f0) + b20;
        f1 = em_group_sum<H, L>(f1) + b21;
        if (ok && t == 0) {
            const float v0 = tx[3 * q] - m0, v1 = tx[3 * q + 1] - m1, v2 = tx[3 * q + 2] - m2;
            const float d = fmaxf(sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2))), r_near);
            const float ld = logf(d);
            float2* o = (float2*)(attr + q * as) + i;
            *o = float2{em_sigmoid(f0 - ld), em_sigmoid(f1 - ld)};
        }
    }
}

template <int H, int L>
__global__ __launch_bounds__(256) void k_emission_bwd_split(const float* __restrict__ P, int64_t ps,
                                                            const float* __restrict__ mean, int n,
                                                            const float* __restrict__ rx,
                                                            const float* __restrict__ tx, int nq, float r_near,
                                                            const float* __restrict__ dattr, int64_t as,
                                                            float* __restrict__ dP, float* __restrict__ dmean)
{
    constexpr int HS = H / L, GPW = 64 / L;
    const int lane = threadIdx.x & 63;
    const int t = lane / GPW, gl = lane % GPW;
    const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * GPW + gl;
    const bool ok = i < n;  // (no early exit: the group's lanes shuffle)
    const int ii = ok ? i : 0;
    const __amdgpu_buffer_rsrc_t rp = em_rsrc(P);
    const uint32_t rs = (uint32_t)ps * 4u;
    const EmOff<H, L> off(t, ii, ps);
    float w1[HS][3], b1[HS], w2a[HS], w2b[HS];
    float gw1[HS][3], gb1[HS], gw2a[HS], gw2b[HS];
#pragma unroll
    for (int jj = 0; jj < HS; ++jj) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w1[jj][c] = em_ld(rp, off.w1, (3 * jj + c) * rs);
            gw1[jj][c] = 0.0f;
        }
        b1[jj] = em_ld(rp, off.b1, jj * rs);
        w2a[jj] = em_ld(rp, off.wa, jj * rs);
        w2b[jj] = em_ld(rp, off.wb, jj * rs);
        gb1[jj] = gw2a[jj] = gw2b[jj] = 0.0f;
    }
    const float b20 = em_ld(rp, off.b2, 0), b21 = em_ld(rp, off.b2, rs);
    const float m0 = mean[ii], m1 = mean[n + ii], m2 = mean[2 * n + ii];
    float gb20 = 0.0f, gb21 = 0.0f, gm0 = 0.0f, gm1 = 0.0f, gm2 = 0.0f;
#pragma unroll 1
    for (int q = 0; q < nq; ++q) {
        const float x0 = rx[3 * q], x1 = rx[3 * q + 1], x2 = rx[3 * q + 2];
        float z[HS];
        float f0 = 0.0f, f1 = 0.0f;
#pragma unroll
        for (int jj = 0; jj < HS; ++jj) {
            z[jj] = fmaf(w1[jj][0], x0, fmaf(w1[jj][1], x1, fmaf(w1[jj][2], x2, b1[jj])));
            const float h = fmaxf(z[jj], 0.0f);
            f0 = fmaf(w2a[jj], h, f0);
            f1 = fmaf(w2b[jj], h, f1);
        }
        f0 = em_group_sum<H, L>(f0) + b20;
        f1 = em_group_sum<H, L>(f1) + b21;
        const float v0 = tx[3 * q] - m0, v1 = tx[3 * q + 1] - m1, v2 = tx[3 * q + 2] - m2;
        const float dist = sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
        const float d = fmaxf(dist, r_near);
        const float ld = logf(d);
        const float s0 = em_sigmoid(f0 - ld), s1 = em_sigmoid(f1 - ld);
        const float2 up = ((const float2*)(dattr + q * as))[ii];
        const float u0 = up.x * s0 * (1.0f - s0), u1 = up.y * s1 * (1.0f - s1);
        gb20 += u0;
        gb21 += u1;
#pragma unroll
        for (int jj = 0; jj < HS; ++jj) {
            const float h = fmaxf(z[jj], 0.0f);
            gw2a[jj] = fmaf(u0, h, gw2a[jj]);
            gw2b[jj] = fmaf(u1, h, gw2b[jj]);
            const float dz = z[jj] > 0.0f ? fmaf(u0, w2a[jj], u1 * w2b[jj]) : 0.0f;
            gb1[jj] += dz;
            gw1[jj][0] = fmaf(dz, x0, gw1[jj][0]);
            gw1[jj][1] = fmaf(dz, x1, gw1[jj][1]);
            gw1[jj][2] = fmaf(dz, x2, gw1[jj][2]);
        }
        // d(-log d)/d mu = (tx - mu) / d^2 where d is not floored
        if (dist > r_near) {
            const float c = -(u0 + u1) / (dist * dist);
            gm0 = fmaf(-c, v0, gm0);
            gm1 = fmaf(-c, v1, gm1);
            gm2 = fmaf(-c, v2, gm2);
        }
    }
    if (!ok) return;
    const __amdgpu_buffer_rsrc_t rg = em_rsrc(dP);
#pragma unroll
    for (int jj = 0; jj < HS; ++jj) {
#pragma unroll
        for (int c = 0; c < 3; ++c) em_st(rg, off.w1, (3 * jj + c) * rs, gw1[jj][c]);
        em_st(rg, off.b1, jj * rs, gb1[jj]);
        em_st(rg, off.wa, jj * rs, gw2a[jj]);
        em_st(rg, off.wb, jj * rs, gw2b[jj]);
    }
    if (t == 0) {
        em_st(rg, off.b2, 0, gb20);
        em_st(rg, off.b2, rs, gb21);
        dmean[i] = gm0;
        dmean[n + i] = gm1;
        dmean[2 * n + i] = gm2;
    }
}

// lanes per Gaussian of the width-64 kernels
constexpr int EM_SPLIT = 8;

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
    if (hidden == 64 && (uint64_t)em_np(64) * (uint64_t)param_stride * 4 >= (1ull << 31)) return GS_ERR_CAPACITY;
    (void)hipGetLastError();
    if (hidden == 64) {
        constexpr int per_block = 256 / EM_SPLIT;
        hipLaunchKernelGGL((k_emission_fwd_split<64, EM_SPLIT>), dim3((n + per_block - 1) / per_block), dim3(256), 0,
                           (hipStream_t)stream, params, param_stride, mean, n, rx, tx, n_queries, r_near, attr,
                           attr_query_stride);
    } else {
        auto kern = hidden == 8 ? k_emission_fwd<8> : k_emission_fwd<16>;
        hipLaunchKernelGGL(kern, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, param_stride,
                           mean, n, rx, tx, n_queries, r_near, attr, attr_query_stride);
    }
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
    if (hidden == 64 && (uint64_t)em_np(64) * (uint64_t)param_stride * 4 >= (1ull << 31)) return GS_ERR_CAPACITY;
    (void)hipGetLastError();
    if (hidden == 64) {
        constexpr int per_block = 256 / EM_SPLIT;
        hipLaunchKernelGGL((k_emission_bwd_split<64, EM_SPLIT>), dim3((n + per_block - 1) / per_block), dim3(256), 0,
                           (hipStream_t)stream, params, param_stride, mean, n, rx, tx, n_queries, r_near, d_attr,
                           attr_query_stride, d_params, d_mean);
    } else {
        auto kern = hidden == 8 ? k_emission_bwd<8> : k_emission_bwd<16>;
        hipLaunchKernelGGL(kern, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, param_stride,
                           mean, n, rx, tx, n_queries, r_near, d_attr, attr_query_stride, d_params, d_mean);
    }
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}
