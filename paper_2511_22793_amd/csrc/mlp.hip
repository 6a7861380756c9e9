// Attribute network on the BF16 matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Per (set s, Gaussian g) row, a shared form of the emission predictor of
// Eq. (1):
//   h1 = relu(Z1[g] + c[s])          Z1 = E W1e^T (query-independent),
//                                    c[s] = b1 + W1t gamma(tx_s)
//   h2 = relu(W2 h1 + b2)
//   o  = W3 h2 + b3                  (64 amplitudes, 64 phases)
//   A_f = sigmoid(o_f - ln d_sg), phi_f = o_{64+f},  attr = A e^{j phi}
// with d_sg = max(|tx_s - mu_g|, r_near).  Rows come from a list of
// Gaussians (e.g. those that reach some pixel) shared by all sets or one
// list per set.
//
// MFMA 16x16x32 operand layout (lane l of a wave):
//   A (16 x 32): row l%16, k = 8*(l/16) .. +7   (8 bf16)
//   B (32 x 16): col l%16, k = 8*(l/16) .. +7   (8 bf16)
//   C (16 x 16): col l%16, rows 4*(l/16) .. +3  (4 floats)
#include "common.h"
#include "mlp.h"

namespace gs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t f2bf(float x)  // round to nearest even
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40);  // NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p)  // 16-byte aligned
{
    const uint4 v = *(const uint4*)p;
    bf16x8 r;
    __builtin_memcpy(&r, &v, 16);
    return r;
}

// ---- Z1 = E W1e^T, one wave per 16 Gaussians -----------------------------
__global__ __launch_bounds__(256) void k_mlp_embed(const uint16_t* __restrict__ E, int n,
                                                   const uint16_t* __restrict__ W1, float* __restrict__ Z1)
{
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int r0 = tile * 16;
    if (r0 >= n) return;
    const int row = r0 + (lane & 15);
    bf16x8 a = {};
    if (row < n) a = load8(E + (size_t)row * MLP_EMB + 8 * (lane >> 4));
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const bf16x8 b = load8(W1 + (size_t)(nt * 16 + (lane & 15)) * MLP_IN + 8 * (lane >> 4));
        f32x4 c = {0, 0, 0, 0};
        c = mfma(a, b, c);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = r0 + 4 * (lane >> 4) + i;
            if (rr < n) Z1[(size_t)rr * MLP_HID + nt * 16 + (lane & 15)] = c[i];
        }
    }
}

// ---- c[s] = b1 + W1t bf16(gamma(tx_s)) -----------------------------------
__global__ __launch_bounds__(64) void k_mlp_bias(const uint16_t* __restrict__ W1, const float* __restrict__ b1,
                                                 const float* __restrict__ tx, float lo0, float lo1, float lo2,
                                                 float hi0, float hi1, float hi2, float* __restrict__ cb,
                                                 uint16_t* __restrict__ genc)
{
    const int s = blockIdx.x, j = threadIdx.x;
    __shared__ float g[MLP_ENC];
    __shared__ double su[3];
    if (j < 3) {
        const float lo = j == 0 ? lo0 : (j == 1 ? lo1 : lo2), hi = j == 0 ? hi0 : (j == 1 ? hi1 : hi2);
        const double u = 2.0 * ((double)tx[3 * s + j] - lo) / ((double)hi - lo) - 1.0;
        su[j] = u;
        g[j] = bf2f(f2bf((float)u));
    }
    __syncthreads();
    if (j < 3 * MLP_BANDS) {  // one (band, coordinate) angle per thread
        const int k = j / 3, d = j % 3;
        const double a = ldexp(M_PI, k) * su[d];
        g[3 + 6 * k + d] = bf2f(f2bf((float)sin(a)));
        g[6 + 6 * k + d] = bf2f(f2bf((float)cos(a)));
    }
    __syncthreads();
    float acc = b1[j];
    for (int k = 0; k < MLP_ENC; ++k) acc = fmaf(bf2f(W1[(size_t)j * MLP_IN + MLP_EMB + k]), g[k], acc);
    cb[s * MLP_HID + j] = acc;
    if (genc)
        for (int k = j; k < MLP_ENC; k += 64) genc[s * MLP_ENC_PAD + k] = f2bf(g[k]);
}

// one wave's 16 rows: h1 (bf16, LDS) -> h2 (bf16, LDS) -> o (C layout)
struct RowTile {
    int g[16];
};

__device__ __forceinline__ void layer_mfma(const uint16_t* __restrict__ act /*LDS [16][64]*/,
                                           const uint16_t* __restrict__ W /*[N][64] bf16*/, int ntiles,
                                           f32x4* acc, int lane)
{
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        if (nt < ntiles) {
            f32x4 c = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                const bf16x8 a = load8(act + (lane & 15) * MLP_HID + kc * 32 + 8 * (lane >> 4));
                const bf16x8 b = load8(W + (size_t)(nt * 16 + (lane & 15)) * MLP_HID + kc * 32 + 8 * (lane >> 4));
                c = mfma(a, b, c);
            }
            acc[nt] = c;
        }
    }
}

// Weights staged in LDS for the row kernels: rows of 64 bf16 padded to
// WROW (16-byte aligned rows, fewer bank conflicts in the B-operand reads).
constexpr int WROW = MLP_HID + 8;

// layer_mfma with the weights' B operands from LDS rows of `ws` bf16
__device__ __forceinline__ void layer_mfma_lds(const uint16_t* act /*LDS [16][64]*/, const uint16_t* W /*LDS [N][ws]*/,
                                               int ws, int ntiles, f32x4* acc, int lane)
{
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        if (nt < ntiles) {
            f32x4 c = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                const bf16x8 a = load8(act + (lane & 15) * MLP_HID + kc * 32 + 8 * (lane >> 4));
                const bf16x8 b = load8(W + (nt * 16 + (lane & 15)) * ws + kc * 32 + 8 * (lane >> 4));
                c = mfma(a, b, c);
            }
            acc[nt] = c;
        }
    }
}

// dst[r][k] = W[r * 64 + k] for r < rows (LDS rows of WROW), in 16-byte chunks
__device__ __forceinline__ void stage_rows(uint16_t* dst, const uint16_t* __restrict__ W, int rows)
{
    for (int c = threadIdx.x; c < rows * (MLP_HID / 8); c += blockDim.x) {
        const int r = c / (MLP_HID / 8), k = (c % (MLP_HID / 8)) * 8;
        *(uint4*)(dst + r * WROW + k) = *(const uint4*)(W + (size_t)r * MLP_HID + k);
    }
}

// 16 consecutive bf16 (32 bytes, 16-byte aligned) between global and LDS
__device__ __forceinline__ void copy16(uint16_t* dst, const uint16_t* src)
{
    ((uint4*)dst)[0] = ((const uint4*)src)[0];
    ((uint4*)dst)[1] = ((const uint4*)src)[1];
}

// Loads h1 = relu(Z1[g] + c[s]) for the wave's 16 rows into LDS (bf16).
__device__ __forceinline__ void load_h1(const float* __restrict__ Z1, const float* __restrict__ cs, const int* rows,
                                        uint16_t* h1s, int lane)
{
    const int r = lane & 15, c0 = (lane >> 4) * 16;
    const int g = rows[r];
    float z[16], c[16];
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
        const float4 zz = g >= 0 ? *(const float4*)(Z1 + (size_t)g * MLP_HID + c0 + j) : make_float4(0, 0, 0, 0);
        const float4 cc = *(const float4*)(cs + c0 + j);
        z[j] = zz.x; z[j + 1] = zz.y; z[j + 2] = zz.z; z[j + 3] = zz.w;
        c[j] = cc.x; c[j + 1] = cc.y; c[j + 2] = cc.z; c[j + 3] = cc.w;
    }
    uint16_t h[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) h[j] = f2bf(g >= 0 ? fmaxf(z[j] + c[j], 0.0f) : 0.0f);
    uint4 v[2];
    __builtin_memcpy(v, h, 32);
    ((uint4*)(h1s + r * MLP_HID + c0))[0] = v[0];
    ((uint4*)(h1s + r * MLP_HID + c0))[1] = v[1];
}

// C layout (16 x 64 as 4 tiles) + bias -> relu -> bf16 -> LDS [16][64]
__device__ __forceinline__ void store_hidden(const f32x4* acc, const float* __restrict__ b, uint16_t* hs,
                                             int lane)
{
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int col = nt * 16 + (lane & 15), row = 4 * (lane >> 4) + i;
            hs[row * MLP_HID + col] = f2bf(fmaxf(acc[nt][i] + b[col], 0.0f));
        }
}

// rows of a set: list entries [0, count); list shared (stride 0) or per set
__device__ __forceinline__ int row_gauss(const uint32_t* list, uint32_t count, int i)
{
    return i < (int)count ? (int)list[i] : -1;
}

template <int NF>
__global__ __launch_bounds__(256) void k_mlp_fwd(MlpArgs A)
{
    const int s = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t* list = A.list + (size_t)s * A.list_stride;
    const uint32_t count = A.count[A.count_stride ? s : 0];
    if (blockIdx.x * 64 >= (int)count) return;  // no rows for this workgroup
    __shared__ __attribute__((aligned(16))) uint16_t s_h1[4][16 * MLP_HID];
    __shared__ __attribute__((aligned(16))) uint16_t s_h2[4][16 * MLP_HID];
    __shared__ __attribute__((aligned(16))) uint16_t s_W2[MLP_HID * WROW];
    __shared__ __attribute__((aligned(16))) uint16_t s_W3[2 * NF * WROW];
    __shared__ int s_rows[4][16];
    stage_rows(s_W2, A.W2, MLP_HID);
    stage_rows(s_W3, A.W3, 2 * NF);
    const float* cs = A.cb + s * MLP_HID;
    const float tx0 = A.tx[3 * s], tx1 = A.tx[3 * s + 1], tx2 = A.tx[3 * s + 2];
    for (int base = blockIdx.x * 64; base < (int)count; base += gridDim.x * 64) {
        const int r0 = base + w * 16;
        if (lane < 16) s_rows[w][lane] = row_gauss(list, count, r0 + lane);
        __builtin_amdgcn_wave_barrier();
        __syncthreads();
        load_h1(A.Z1, cs, s_rows[w], s_h1[w], lane);
        __syncthreads();
        f32x4 acc[8];
        layer_mfma_lds(s_h1[w], s_W2, WROW, 4, acc, lane);
        store_hidden(acc, A.b2, s_h2[w], lane);
        __syncthreads();
        layer_mfma_lds(s_h2[w], s_W3, WROW, 2 * NF / 16, acc, lane);
        // save activations for the backward (row-compact order r = s*cap + i)
        if (A.save_h1) {
            const int r = lane & 15, c0 = (lane >> 4) * 16;
            const int i = r0 + r;
            if (i < (int)count) {
                copy16(A.save_h1 + ((size_t)s * A.row_cap + i) * MLP_HID + c0, &s_h1[w][r * MLP_HID + c0]);
                copy16(A.save_h2 + ((size_t)s * A.row_cap + i) * MLP_HID + c0, &s_h2[w][r * MLP_HID + c0]);
            }
        }
        // epilogue: amplitude / phase -> complex attribute
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = 4 * (lane >> 4) + i;
            const int g = s_rows[w][rr];
            if (g < 0) continue;
            const float e0 = A.mean[g] - tx0, e1 = A.mean[A.n + g] - tx1, e2 = A.mean[2 * A.n + g] - tx2;
            const float d = fmaxf(sqrtf(e0 * e0 + e1 * e1 + e2 * e2), A.r_near);
            const float lnd = logf(d);
            float* out = A.attr + (size_t)s * A.attr_stride + (size_t)g * (2 * NF);
#pragma unroll
            for (int nt = 0; nt < NF / 16; ++nt) {
                const int f = nt * 16 + (lane & 15);
                const float oa = acc[nt][i] + A.b3[f] - lnd;
                const float op = acc[nt + NF / 16][i] + A.b3[NF + f];
                const float amp = 1.0f / (1.0f + expf(-oa));
                float sn, cs_;
                sincosf(op, &sn, &cs_);
                *(float2*)(out + 2 * f) = make_float2(amp * cs_, amp * sn);
            }
        }
    }
}

// Backward through the epilogue and the three layers for each row.  Writes
// the rounded products' operands (d_o, dZ2, dZ1 as bf16) for the weight
// gradients, bias sums, per-set dZ1 sums and dE (atomics).
template <int NF>
__global__ __launch_bounds__(256) void k_mlp_bwd_data(MlpArgs A)
{
    const int s = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t* list = A.list + (size_t)s * A.list_stride;
    const uint32_t count = A.count[A.count_stride ? s : 0];
    __shared__ __attribute__((aligned(16))) uint16_t s_h1[4][16 * MLP_HID];
    __shared__ __attribute__((aligned(16))) uint16_t s_h2[4][16 * MLP_HID];
    __shared__ __attribute__((aligned(16))) uint16_t s_do[4][16 * 2 * NF];
    __shared__ __attribute__((aligned(16))) uint16_t s_dz[4][16 * MLP_HID];
    __shared__ int s_rows[4][16];
    __shared__ float s_db3[2 * NF], s_db2[MLP_HID], s_dc[MLP_HID];
    for (int k = threadIdx.x; k < 2 * NF; k += 256) s_db3[k] = 0.0f;
    if (threadIdx.x < MLP_HID) {
        s_db2[threadIdx.x] = 0.0f;
        s_dc[threadIdx.x] = 0.0f;
    }
    const float tx0 = A.tx[3 * s], tx1 = A.tx[3 * s + 1], tx2 = A.tx[3 * s + 2];
    __syncthreads();
    for (int base = blockIdx.x * 64; base < (int)count; base += gridDim.x * 64) {
        const int r0 = base + w * 16;
        if (lane < 16) s_rows[w][lane] = row_gauss(list, count, r0 + lane);
        __syncthreads();
        // saved h1 and h2 of the 16 rows
        {
            const int r = lane & 15, c0 = (lane >> 4) * 16;
            const int i = r0 + r;
            if (i < (int)count) {
                copy16(&s_h1[w][r * MLP_HID + c0], A.save_h1 + ((size_t)s * A.row_cap + i) * MLP_HID + c0);
                copy16(&s_h2[w][r * MLP_HID + c0], A.save_h2 + ((size_t)s * A.row_cap + i) * MLP_HID + c0);
            } else {
                const uint4 z = make_uint4(0, 0, 0, 0);
                ((uint4*)&s_h1[w][r * MLP_HID + c0])[0] = z;
                ((uint4*)&s_h1[w][r * MLP_HID + c0])[1] = z;
                ((uint4*)&s_h2[w][r * MLP_HID + c0])[0] = z;
                ((uint4*)&s_h2[w][r * MLP_HID + c0])[1] = z;
            }
        }
        __syncthreads();
        f32x4 acc[8];
        layer_mfma(s_h2[w], A.W3, 2 * NF / 16, acc, lane);  // recompute o
        // d_o from d_attr
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = 4 * (lane >> 4) + i;
            const int g = s_rows[w][rr];
            float lnd = 0.0f;
            if (g >= 0) {
                const float e0 = A.mean[g] - tx0, e1 = A.mean[A.n + g] - tx1, e2 = A.mean[2 * A.n + g] - tx2;
                lnd = logf(fmaxf(sqrtf(e0 * e0 + e1 * e1 + e2 * e2), A.r_near));
            }
            const float* dat = A.d_attr + (size_t)s * A.attr_stride + (size_t)(g < 0 ? 0 : g) * (2 * NF);
#pragma unroll
            for (int nt = 0; nt < NF / 16; ++nt) {
                const int f = nt * 16 + (lane & 15);
                float da = 0.0f, dp = 0.0f;
                if (g >= 0) {
                    const float oa = acc[nt][i] + A.b3[f] - lnd;
                    const float op = acc[nt + NF / 16][i] + A.b3[NF + f];
                    const float amp = 1.0f / (1.0f + expf(-oa));
                    float sn, cs_;
                    sincosf(op, &sn, &cs_);
                    const float2 gg = *(const float2*)(dat + 2 * f);
                    if (A.clear)
                        *(float2*)(A.clear + (size_t)s * A.attr_stride + (size_t)g * (2 * NF) + 2 * f) =
                            make_float2(0.0f, 0.0f);
                    da = (gg.x * cs_ + gg.y * sn) * amp * (1.0f - amp);
                    dp = amp * (-gg.x * sn + gg.y * cs_);
                }
                s_do[w][rr * 2 * NF + f] = f2bf(da);
                s_do[w][rr * 2 * NF + NF + f] = f2bf(dp);
                acc[nt][i] = da;
                acc[nt + NF / 16][i] = dp;
            }
        }
        // db3: FP32 sums of d_o
#pragma unroll
        for (int nt = 0; nt < 2 * NF / 16; ++nt) {
            float v = acc[nt][0] + acc[nt][1] + acc[nt][2] + acc[nt][3];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) atomicAdd(&s_db3[nt * 16 + lane], v);
        }
        __syncthreads();
        // write d_o (bf16) for the weight gradient
        {
            const int r = lane & 15;
            const int i = r0 + r;
            if (i < (int)count)
                for (int j = (lane >> 4) * (NF / 2); j < (lane >> 4) * (NF / 2) + NF / 2; j += 16)
                    copy16(A.save_do + ((size_t)s * A.row_cap + i) * 2 * NF + j, &s_do[w][r * 2 * NF + j]);
        }
        // dh2 = d_o W3  (K = 2 NF in 32-wide chunks; B from W3^T [64][2 NF])
        f32x4 dh[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 c = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 2 * NF / 32; ++kc) {
                const bf16x8 a = load8(&s_do[w][(lane & 15) * 2 * NF + kc * 32 + 8 * (lane >> 4)]);
                const bf16x8 b = load8(A.W3T + (size_t)(nt * 16 + (lane & 15)) * 2 * NF + kc * 32 + 8 * (lane >> 4));
                c = mfma(a, b, c);
            }
            dh[nt] = c;
        }
        // dZ2 = dh2 * [h2 > 0]
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int col = nt * 16 + (lane & 15), row = 4 * (lane >> 4) + i;
                const float m = bf2f(s_h2[w][row * MLP_HID + col]) > 0.0f ? 1.0f : 0.0f;
                dh[nt][i] *= m;
            }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            float v = dh[nt][0] + dh[nt][1] + dh[nt][2] + dh[nt][3];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) atomicAdd(&s_db2[nt * 16 + lane], v);
        }
        __syncthreads();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                s_dz[w][(4 * (lane >> 4) + i) * MLP_HID + nt * 16 + (lane & 15)] = f2bf(dh[nt][i]);
        __syncthreads();
        {
            const int r = lane & 15, c0 = (lane >> 4) * 16;
            const int i = r0 + r;
            if (i < (int)count)
                copy16(A.save_dz2 + ((size_t)s * A.row_cap + i) * MLP_HID + c0, &s_dz[w][r * MLP_HID + c0]);
        }
        // dh1 = dZ2 W2 (B from W2^T), dZ1 = dh1 * [h1 > 0]
        f32x4 d1[4];
        layer_mfma(s_dz[w], A.W2T, 4, d1, lane);
        __syncthreads();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int col = nt * 16 + (lane & 15), row = 4 * (lane >> 4) + i;
                const int rix = r0 + row;
                float m = 0.0f;
                if (rix < (int)count) m = bf2f(s_h1[w][row * MLP_HID + col]) > 0.0f;
                d1[nt][i] *= m;
                s_dz[w][row * MLP_HID + col] = f2bf(d1[nt][i]);
            }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            float v = d1[nt][0] + d1[nt][1] + d1[nt][2] + d1[nt][3];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) atomicAdd(&s_dc[nt * 16 + lane], v);
        }
        __syncthreads();
        {
            const int r = lane & 15, c0 = (lane >> 4) * 16;
            const int i = r0 + r;
            if (i < (int)count)
                copy16(A.save_dz1 + ((size_t)s * A.row_cap + i) * MLP_HID + c0, &s_dz[w][r * MLP_HID + c0]);
        }
        // dE[g] += dZ1 W1e  (B from W1e^T [32][64])
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            f32x4 c = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                const bf16x8 a = load8(&s_dz[w][(lane & 15) * MLP_HID + kc * 32 + 8 * (lane >> 4)]);
                const bf16x8 b = load8(A.W1eT + (size_t)(nt * 16 + (lane & 15)) * MLP_HID + kc * 32 + 8 * (lane >> 4));
                c = mfma(a, b, c);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int g = s_rows[w][4 * (lane >> 4) + i];
                if (g >= 0) unsafeAtomicAdd(A.dE + (size_t)g * MLP_EMB + nt * 16 + (lane & 15), c[i]);
            }
        }
        __syncthreads();
    }
    __syncthreads();
    // only workgroups that had rows flush (the grid is sized for the largest
    // row count; the others would add zeros into the same few addresses)
    if (blockIdx.x * 64 >= (int)count) return;
    for (int k = threadIdx.x; k < 2 * NF; k += 256) unsafeAtomicAdd(A.db3 + k, s_db3[k]);
    if (threadIdx.x < MLP_HID) {
        unsafeAtomicAdd(A.db2 + threadIdx.x, s_db2[threadIdx.x]);
        unsafeAtomicAdd(A.dc + s * MLP_HID + threadIdx.x, s_dc[threadIdx.x]);
    }
}

// Split-K weight gradient C[M][N] = sum over rows r of a[r][m] b[r][n] (bf16
// operands, FP32 accumulation).  a rows: [S][cap][M]; b rows: [S][cap][N], or
// when b_gather is set, b = E[list[i]] ([n][N]).  Each workgroup handles K
// blocks of 32 rows round-robin and writes its partial [M][N].
// LDS of one weight-gradient workgroup: A and B row blocks, [m][32 rows] padded
struct WgradLds {
    __attribute__((aligned(16))) uint16_t tA[2 * MLP_F][40];
    __attribute__((aligned(16))) uint16_t tB[MLP_HID][40];
};

// (M and N are run-time values so that one kernel carries all three
// matrices; the accumulator array is sized for the largest, 8 tiles a wave)
__device__ __forceinline__ void wgrad_body(WgradLds& L, const int M, const int N, const uint16_t* __restrict__ a,
                                           const uint16_t* __restrict__ b, const uint16_t* __restrict__ bgather,
                                           const uint32_t* __restrict__ list, size_t list_stride,
                                           const uint32_t* __restrict__ count, int count_stride, int S, size_t cap,
                                           float* __restrict__ partial)
{
    constexpr int MAXPW = (2 * MLP_F / 16) * (MLP_HID / 16) / 4;
    const int NT = N / 16, PER_WAVE = (M / 16) * NT / 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    auto& tA = L.tA;
    auto& tB = L.tB;
    f32x4 acc[MAXPW];
#pragma unroll
    for (int t = 0; t < MAXPW; ++t) acc[t] = f32x4{0, 0, 0, 0};
    // K blocks enumerate (set, 32-row block)
    int kb = blockIdx.x;
    for (int s = 0; s < S; ++s) {
        const uint32_t cnt = count[count_stride ? s : 0];
        const int nblk = (int)((cnt + 31) / 32);
        const uint32_t* lst = list + (size_t)s * list_stride;
        while (kb < nblk) {
            // stage 32 rows transposed
            for (int e = threadIdx.x; e < 32 * M; e += 256) {
                const int r = e / M, m = e % M;
                const int i = kb * 32 + r;
                tA[m][r] = i < (int)cnt ? a[((size_t)s * cap + i) * M + m] : (uint16_t)0;
            }
            for (int e = threadIdx.x; e < 32 * N; e += 256) {
                const int r = e / N, c = e % N;
                const int i = kb * 32 + r;
                uint16_t v = 0;
                if (i < (int)cnt) v = bgather ? bgather[(size_t)lst[i] * N + c] : b[((size_t)s * cap + i) * N + c];
                tB[c][r] = v;
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < MAXPW; ++t) {
                if (t < PER_WAVE) {
                    const int tile = w * PER_WAVE + t;
                    const int mt = tile / NT, nt = tile % NT;
                    const bf16x8 av = load8(&tA[mt * 16 + (lane & 15)][8 * (lane >> 4)]);
                    const bf16x8 bv = load8(&tB[nt * 16 + (lane & 15)][8 * (lane >> 4)]);
                    acc[t] = mfma(av, bv, acc[t]);
                }
            }
            __syncthreads();
            kb += gridDim.x;
        }
        kb -= nblk;
    }
    float* P = partial + (size_t)blockIdx.x * M * N;
#pragma unroll
    for (int t = 0; t < MAXPW; ++t) {
        if (t < PER_WAVE) {
            const int tile = w * PER_WAVE + t;
            const int mt = tile / NT, nt = tile % NT;
#pragma unroll
            for (int i = 0; i < 4; ++i) P[(mt * 16 + 4 * (lane >> 4) + i) * N + nt * 16 + (lane & 15)] = acc[t][i];
        }
    }
}

// The three weight gradients in one launch (blockIdx.y picks the matrix);
// their split-K partials sit one after the other in `partial`.
struct WgradArgs {
    const uint16_t *do_, *h2, *dz2, *h1, *dz1, *E;
    const uint32_t* list;
    size_t list_stride;
    const uint32_t* count;
    int count_stride, S;
    size_t cap;
    float* partial;
};

constexpr int WG3_LEN1 = MLP_HID * MLP_HID, WG3_LEN2 = MLP_HID * MLP_EMB;
__host__ __device__ constexpr int wg3_len0(int nf) { return 2 * nf * MLP_HID; }

template <int NF>
__global__ __launch_bounds__(256) void k_wgrad3(WgradArgs A)
{
    __shared__ WgradLds L;
    const int P = gridDim.x;
    constexpr int WG3_LEN0 = wg3_len0(NF);
    // y = 0: dW3 = d_o^T h2; 1: dW2 = dZ2^T h1; 2: dW1e = dZ1^T E[g]
    const int y = blockIdx.y;
    const int M = y == 0 ? 2 * NF : MLP_HID, N = y == 2 ? MLP_EMB : MLP_HID;
    const uint16_t* a = y == 0 ? A.do_ : (y == 1 ? A.dz2 : A.dz1);
    const uint16_t* b = y == 0 ? A.h2 : (y == 1 ? A.h1 : nullptr);
    float* part = A.partial + (y == 0 ? 0 : (y == 1 ? (size_t)P * WG3_LEN0 : (size_t)P * (WG3_LEN0 + WG3_LEN1)));
    wgrad_body(L, M, N, a, b, y == 2 ? A.E : nullptr, A.list, A.list_stride, A.count, A.count_stride, A.S, A.cap,
               part);
}

// Sums the partials of the three weight gradients into dW3, dW2 and the
// embedding columns of dW1.
template <int NF>
__global__ void k_reduce3(const float* __restrict__ partial, int nparts, float* __restrict__ dW3,
                          float* __restrict__ dW2, float* __restrict__ dW1)
{
    constexpr int WG3_LEN0 = wg3_len0(NF);
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    const float* base = partial;
    int len = WG3_LEN0, ncols = MLP_HID, ld = MLP_HID;
    float* out = dW3;
    if (e >= WG3_LEN0) {
        e -= WG3_LEN0;
        base += (size_t)nparts * WG3_LEN0;
        len = WG3_LEN1;
        out = dW2;
        if (e >= WG3_LEN1) {
            e -= WG3_LEN1;
            base += (size_t)nparts * WG3_LEN1;
            len = WG3_LEN2;
            ncols = MLP_EMB;
            ld = MLP_IN;
            out = dW1;
            if (e >= WG3_LEN2) return;
        }
    }
    // the partials added in order, 16 loads in flight ahead of the additions
    float acc = 0.0f;
    int p = 0;
    for (; p + 16 <= nparts; p += 16) {
        float b[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) b[u] = base[(size_t)(p + u) * len + e];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += b[u];
    }
    for (; p < nparts; ++p) acc += base[(size_t)p * len + e];
    out[(size_t)(e / ncols) * ld + e % ncols] = acc;
}

// dW1t = sum_s dc_s gamma_s^T (bf16 gamma), db1 = sum_s dc_s
__global__ void k_mlp_bias_grad(const float* __restrict__ dc, const uint16_t* __restrict__ genc, int S,
                                float* __restrict__ dW1, float* __restrict__ db1)
{
    const int j = threadIdx.x;  // hidden unit
    for (int k = blockIdx.x; k <= MLP_ENC; k += gridDim.x) {
        // the sets added in order, 16 sets' loads in flight ahead of the products
        float acc = 0.0f;
        int s = 0;
        for (; s + 16 <= S; s += 16) {
            float d[16], g[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                d[u] = dc[(s + u) * MLP_HID + j];
                g[u] = k < MLP_ENC ? bf2f(genc[(s + u) * MLP_ENC_PAD + k]) : 1.0f;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += d[u] * g[u];
        }
        for (; s < S; ++s) acc += dc[s * MLP_HID + j] * (k < MLP_ENC ? bf2f(genc[s * MLP_ENC_PAD + k]) : 1.0f);
        if (k < MLP_ENC) dW1[(size_t)j * MLP_IN + MLP_EMB + k] = acc;
        else db1[j] = acc;
    }
}

// bf16 transposes of the weights used as B operands in the backward
__global__ void k_mlp_transpose(const uint16_t* __restrict__ W1, const uint16_t* __restrict__ W2,
                                const uint16_t* __restrict__ W3, uint16_t* __restrict__ W1eT,
                                uint16_t* __restrict__ W2T, uint16_t* __restrict__ W3T, int NF)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < MLP_EMB * MLP_HID) {  // W1eT[n][k] = W1[k][n], n < 32
        const int n = e / MLP_HID, k = e % MLP_HID;
        W1eT[e] = W1[(size_t)k * MLP_IN + n];
    }
    if (e < MLP_HID * MLP_HID) {  // W2T[n][k] = W2[k][n]
        const int n = e / MLP_HID, k = e % MLP_HID;
        W2T[e] = W2[(size_t)k * MLP_HID + n];
    }
    if (e < MLP_HID * 2 * NF) {  // W3T[n][k] = W3[k][n], n < 64, k < 2 NF
        const int n = e / (2 * NF), k = e % (2 * NF);
        W3T[e] = W3[(size_t)k * MLP_HID + n];
    }
}

}  // namespace gs

using namespace gs;

extern "C" {

gs_status gs_mlp_embed(const gs_mlp* net, const uint16_t* E, int32_t n, float* Z1, void* stream)
{
    if (!net || !net->W1 || !E || !Z1 || n < 1) return GS_ERR_INVALID_ARG;
    (void)hipGetLastError();
    const int tiles = (n + 15) / 16;
    hipLaunchKernelGGL(k_mlp_embed, dim3((tiles + 3) / 4), dim3(256), 0, (hipStream_t)stream, E, n, net->W1, Z1);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

static gs_status check_rows(const gs_mlp* net, const gs_mlp_rows* rows, const float* mean, int32_t n)
{
    if (!net || !rows || !mean || n < 1) return GS_ERR_INVALID_ARG;
    if (net->n_chan != 32 && net->n_chan != 64) return GS_ERR_INVALID_ARG;
    if (!net->W1 || !net->b1 || !net->W2 || !net->b2 || !net->W3 || !net->b3) return GS_ERR_INVALID_ARG;
    if (!rows->tx || !rows->list || !rows->count || rows->n_sets < 1 || rows->n_sets > 65535) return GS_ERR_INVALID_ARG;
    if (rows->row_cap < 1 || !(net->r_near > 0.0f)) return GS_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k)
        if (!(net->box_hi[k] > net->box_lo[k])) return GS_ERR_INVALID_ARG;
    return GS_OK;
}

gs_status gs_mlp_forward(const gs_mlp* net, const float* Z1, const float* mean, int32_t n, const gs_mlp_rows* rows,
                         float* attr, int64_t attr_stride, gs_mlp_state* st, void* stream)
{
    gs_status e = check_rows(net, rows, mean, n);
    if (e != GS_OK) return e;
    const int NF = net->n_chan;
    if (!Z1 || !attr || !st || !st->cb || attr_stride < (int64_t)n * 2 * NF) return GS_ERR_INVALID_ARG;
    if ((st->save_h1 == nullptr) != (st->save_h2 == nullptr)) return GS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_mlp_bias, dim3(rows->n_sets), dim3(64), 0, s, net->W1, net->b1, rows->tx, net->box_lo[0],
                       net->box_lo[1], net->box_lo[2], net->box_hi[0], net->box_hi[1], net->box_hi[2], st->cb,
                       st->genc);
    MlpArgs A{};
    A.W2 = net->W2; A.b2 = net->b2; A.W3 = net->W3; A.b3 = net->b3;
    A.Z1 = Z1; A.cb = st->cb; A.mean = mean; A.n = n; A.tx = rows->tx; A.r_near = net->r_near;
    A.list = rows->list; A.list_stride = rows->list_stride; A.count = rows->count; A.count_stride = rows->count_stride;
    A.row_cap = rows->row_cap; A.attr = attr; A.attr_stride = attr_stride;
    A.save_h1 = st->save_h1; A.save_h2 = st->save_h2;
    const int gx = rows->grid_x > 0 ? rows->grid_x : 32;
    if (NF == 64) hipLaunchKernelGGL(k_mlp_fwd<64>, dim3(gx, rows->n_sets), dim3(256), 0, s, A);
    else hipLaunchKernelGGL(k_mlp_fwd<32>, dim3(gx, rows->n_sets), dim3(256), 0, s, A);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_mlp_backward(const gs_mlp* net, const uint16_t* E, const float* mean, int32_t n, const gs_mlp_rows* rows,
                          float* d_attr, int64_t attr_stride, int32_t clear_d_attr, gs_mlp_state* st,
                          gs_mlp_grads* gr, void* stream)
{
    gs_status e = check_rows(net, rows, mean, n);
    if (e != GS_OK) return e;
    if (!E || !d_attr || !st || !gr || !st->save_h1 || !st->save_h2 || !st->save_do || !st->save_dz2 ||
        !st->save_dz1 || !st->genc || !st->dc || !st->wT || !st->partial || st->n_partial < 1)
        return GS_ERR_INVALID_ARG;
    if (!gr->dW1 || !gr->db1 || !gr->dW2 || !gr->db2 || !gr->dW3 || !gr->db3 || !gr->dE) return GS_ERR_INVALID_ARG;
    const int NF = net->n_chan;
    if (attr_stride < (int64_t)n * 2 * NF) return GS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    uint16_t* W1eT = st->wT;
    uint16_t* W2T = W1eT + MLP_EMB * MLP_HID;
    uint16_t* W3T = W2T + MLP_HID * MLP_HID;
    hipLaunchKernelGGL(k_mlp_transpose, dim3((MLP_HID * 2 * MLP_F + 255) / 256), dim3(256), 0, s, net->W1, net->W2,
                       net->W3, W1eT, W2T, W3T, NF);
    {
        FillSegs f{};
        f.p[0] = (uint32_t*)gr->db3; f.count[0] = 2 * NF;
        f.p[1] = (uint32_t*)gr->db2; f.count[1] = MLP_HID;
        f.p[2] = (uint32_t*)gr->dW1; f.count[2] = (size_t)MLP_HID * MLP_IN;
        f.p[3] = (uint32_t*)st->dc; f.count[3] = (size_t)rows->n_sets * MLP_HID;
        f.p[4] = (uint32_t*)gr->dE; f.count[4] = (size_t)n * MLP_EMB;
        f.n = 5;
        launch_fill_segs(f, s);
    }
    MlpArgs A{};
    A.W2 = net->W2; A.b2 = net->b2; A.W3 = net->W3; A.b3 = net->b3;
    A.W2T = W2T; A.W3T = W3T; A.W1eT = W1eT;
    A.mean = mean; A.n = n; A.tx = rows->tx; A.r_near = net->r_near;
    A.list = rows->list; A.list_stride = rows->list_stride; A.count = rows->count; A.count_stride = rows->count_stride;
    A.row_cap = rows->row_cap; A.d_attr = d_attr; A.attr_stride = attr_stride;
    A.clear = clear_d_attr ? d_attr : nullptr;
    A.save_h1 = st->save_h1; A.save_h2 = st->save_h2; A.save_do = st->save_do; A.save_dz2 = st->save_dz2;
    A.save_dz1 = st->save_dz1; A.db3 = gr->db3; A.db2 = gr->db2; A.dc = st->dc; A.dE = gr->dE;
    const int gx = rows->grid_x > 0 ? rows->grid_x : 32;
    if (NF == 64) hipLaunchKernelGGL(k_mlp_bwd_data<64>, dim3(gx, rows->n_sets), dim3(256), 0, s, A);
    else hipLaunchKernelGGL(k_mlp_bwd_data<32>, dim3(gx, rows->n_sets), dim3(256), 0, s, A);
    const int P = st->n_partial;
    // dW3 = d_o^T h2, dW2 = dZ2^T h1, dW1e = dZ1^T E: one split-K launch, one reduction
    WgradArgs W{st->save_do, st->save_h2, st->save_dz2, st->save_h1, st->save_dz1, E, rows->list, (size_t)rows->list_stride,
                rows->count, rows->count_stride, rows->n_sets, (size_t)rows->row_cap, st->partial};
    const unsigned rb = (unsigned)((wg3_len0(NF) + WG3_LEN1 + WG3_LEN2 + 255) / 256);
    if (NF == 64) {
        hipLaunchKernelGGL(k_wgrad3<64>, dim3(P, 3), dim3(256), 0, s, W);
        hipLaunchKernelGGL(k_reduce3<64>, dim3(rb), dim3(256), 0, s, st->partial, P, gr->dW3, gr->dW2, gr->dW1);
    } else {
        hipLaunchKernelGGL(k_wgrad3<32>, dim3(P, 3), dim3(256), 0, s, W);
        hipLaunchKernelGGL(k_reduce3<32>, dim3(rb), dim3(256), 0, s, st->partial, P, gr->dW3, gr->dW2, gr->dW1);
    }
    hipLaunchKernelGGL(k_mlp_bias_grad, dim3(MLP_ENC + 1), dim3(MLP_HID), 0, s, st->dc, st->genc, rows->n_sets,
                       gr->dW1, gr->db1);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

}  // extern "C"
