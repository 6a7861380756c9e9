// Spectrum-to-channel map and training loss (Eq. (2), Eq. (4)).
//
// For each set b and channel f (re and im separately when complex):
//   h^_bf = (1/HW) sum_p zhat_bfp                  (coherent spatial mean)
//   L_b   = (1/(F H W)) sum_{f,p} |zhat - z|^2 + lambda sum_f |h^_bf - h_bf|^2
//   L     = (1/B) sum_b L_b
// with h_bf the spatial mean of the target spectrum.  The gradient is
//   dL/dzhat = (1/B) [2 (zhat - z) / (F H W) + lambda 2 (h^ - h) / (H W)].
// Two passes: a reduction per (set, channel component) into FP32
// accumulators (workgroup partial sums, then atomics), then the elementwise
// gradient.  Both passes stream the spectra once.
#include <mutex>

#include "common.h"

namespace gs {

// One (set, channel) slice is HW*C contiguous floats; with C = 2 the even
// positions are real parts and the odd ones imaginary parts.  Slices whose
// length is a multiple of 4 (and 16-byte aligned spectra) are streamed as
// float4, so that component c of element x, y, z, w is 0, 1, 0, 1 (C = 2) or
// always 0 (C = 1).
// acc layout per set: [Fc][3] = (sum zhat, sum z, sum (zhat - z)^2)
// With dpart set, the same pass also writes dpart = scale (zhat - z), the
// elementwise part of the gradient.
template <bool VEC>
__global__ __launch_bounds__(256) void k_loss_reduce(const float* __restrict__ zhat, const float* __restrict__ z,
                                                     int Fc, int C, size_t HW, float* __restrict__ acc,
                                                     float* __restrict__ dpart, float scale)
{
    const int b = blockIdx.z, f = blockIdx.y;  // f indexes complex channels (F)
    const size_t F = Fc / C;
    const size_t n = HW * C, base = ((size_t)b * F + f) * n;
    float s[2] = {0, 0}, t[2] = {0, 0}, e = 0.0f;
    const size_t nv = VEC ? n / 4 : 0;
    const size_t stride = (size_t)gridDim.x * 256;
    if (VEC) {
        const float4* a4 = (const float4*)(zhat + base);
        const float4* y4 = (const float4*)(z + base);
        for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += stride) {
            const float4 a = a4[i], y = y4[i];
            if (dpart)
                ((float4*)(dpart + base))[i] =
                    make_float4(scale * (a.x - y.x), scale * (a.y - y.y), scale * (a.z - y.z), scale * (a.w - y.w));
            s[0] += a.x + a.z;
            s[1] += a.y + a.w;
            t[0] += y.x + y.z;
            t[1] += y.y + y.w;
            const float d0 = a.x - y.x, d1 = a.y - y.y, d2 = a.z - y.z, d3 = a.w - y.w;
            e += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
        }
        if (C == 1) {
            s[0] += s[1];
            t[0] += t[1];
            s[1] = t[1] = 0.0f;
        }
    }
    for (size_t k = nv * 4 + (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += stride) {
        const float a = zhat[base + k], y = z[base + k];
        if (dpart) dpart[base + k] = scale * (a - y);
        const int c = (int)(k % C);
        s[c] += a;
        t[c] += y;
        e += (a - y) * (a - y);
    }
    __shared__ float red[5][4];
    float vals[5] = {s[0], s[1], t[0], t[1], e};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        float v = vals[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int k = threadIdx.x;
        const float v = red[k][0] + red[k][1] + red[k][2] + red[k][3];
        float* a = acc + ((size_t)b * Fc + (size_t)f * C) * 3;
        if (k < 2 && k < C) unsafeAtomicAdd(a + k * 3 + 0, v);
        else if (k >= 2 && k < 4 && k - 2 < C) unsafeAtomicAdd(a + (k - 2) * 3 + 1, v);
        else if (k == 4) unsafeAtomicAdd(a + 2, v);  // squared error summed over components
    }
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_loss_grad(const float* __restrict__ zhat, const float* __restrict__ z,
                                                   int B, int Fc, int C, size_t HW, float lambda,
                                                   const float* __restrict__ acc, float* __restrict__ dz,
                                                   float* __restrict__ hhat, float* __restrict__ loss)
{
    const int b = blockIdx.z, f = blockIdx.y;
    const size_t F = Fc / C;
    const size_t n = HW * C, base = ((size_t)b * F + f) * n;
    const float* a = acc + ((size_t)b * Fc + (size_t)f * C) * 3;
    const float inv_hw = 1.0f / (float)HW;
    const float k1 = 2.0f / ((float)F * (float)HW * (float)B);
    float gmean[2] = {0.0f, 0.0f};
    for (int c = 0; c < C; ++c) gmean[c] = lambda * 2.0f * (a[c * 3] - a[c * 3 + 1]) * inv_hw * inv_hw / (float)B;
    const float g1 = C == 2 ? gmean[1] : gmean[0];
    const size_t nv = VEC ? n / 4 : 0;
    const size_t stride = (size_t)gridDim.x * 256;
    if (VEC) {
        const float4* a4 = (const float4*)(zhat + base);
        const float4* y4 = (const float4*)(z + base);
        float4* d4 = (float4*)(dz + base);
        for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += stride) {
            const float4 x = a4[i], y = y4[i];
            d4[i] = make_float4(k1 * (x.x - y.x) + gmean[0], k1 * (x.y - y.y) + g1, k1 * (x.z - y.z) + gmean[0],
                                k1 * (x.w - y.w) + g1);
        }
    }
    for (size_t k = nv * 4 + (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += stride)
        dz[base + k] = k1 * (zhat[base + k] - z[base + k]) + gmean[k % C];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float Lf = a[2] / ((float)F * (float)HW);
        for (int c = 0; c < C; ++c) {
            const float hd = (a[c * 3] - a[c * 3 + 1]) * inv_hw;
            hhat[((size_t)b * Fc + (size_t)f * C) + c] = a[c * 3] * inv_hw;
            Lf += lambda * hd * hd;
        }
        unsafeAtomicAdd(loss + b, Lf);
    }
}

// Loss, spatial means and the channel-mean term of the gradient, without
// the elementwise gradient: one workgroup per set, one thread per channel
// component.  mean_grad[b][f*C + c] = lambda 2 (h^ - h) / (H W) / B.
__global__ void k_loss_finish(int B, int Fc, int C, size_t HW, float lambda, const float* __restrict__ acc,
                              float* __restrict__ hhat, float* __restrict__ loss, float* __restrict__ mgrad)
{
    const int b = blockIdx.x;
    const float inv_hw = 1.0f / (float)HW;
    const float F = (float)(Fc / C);
    float Lpart = 0.0f;
    for (int k = threadIdx.x; k < Fc; k += blockDim.x) {
        const float* a = acc + ((size_t)b * Fc + (size_t)(k - k % C)) * 3;  // the channel's accumulators
        const int c = k % C;
        const float hd = (a[c * 3] - a[c * 3 + 1]) * inv_hw;
        hhat[(size_t)b * Fc + k] = a[c * 3] * inv_hw;
        mgrad[(size_t)b * Fc + k] = lambda * 2.0f * (a[c * 3] - a[c * 3 + 1]) * inv_hw * inv_hw / (float)B;
        Lpart += lambda * hd * hd + (c == 0 ? a[2] / (F * (float)HW) : 0.0f);
    }
    for (int o = 32; o > 0; o >>= 1) Lpart += __shfl_xor(Lpart, o, 64);
    __shared__ float red[16];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = Lpart;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += red[w];
        loss[b] = t;
    }
}

// acc[set][ch][slot] = sum of the np per-wave partials (slot 2, the squared
// error, of both components of a complex channel into its first component)
__global__ __launch_bounds__(256) void k_loss_parts(int n_sets, int Fc, int C, int np, const float* __restrict__ part,
                                                    float* __restrict__ acc)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);  // (set, ch, slot), one wave each
    const int lane = threadIdx.x & 63;
    if (i >= n_sets * Fc * 3) return;
    const int slot = i % 3, ch = (i / 3) % Fc;
    float v = 0.0f;
    if (slot < 2 || ch % C == 0) {
        for (int c = 0; c < (slot == 2 ? C : 1); ++c) {
            const float* p = part + (size_t)(i + 3 * c) * np;
            for (int k = lane; k < np; k += 64) v += p[k];
        }
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) acc[i] = v;
}

void launch_loss_parts(int n_sets, int Fc, int C, int np, const float* part, float* acc, hipStream_t s)
{
    const int n = n_sets * Fc * 3;
    hipLaunchKernelGGL(k_loss_parts, dim3((n + 3) / 4), dim3(256), 0, s, n_sets, Fc, C, np, part, acc);
}

void launch_loss_finish(int n_sets, int Fc, int C, size_t HW, float lambda, const float* acc, float* h_hat,
                        float* loss, float* mean_grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_loss_finish, dim3(n_sets), dim3(256), 0, s, n_sets, Fc, C, HW, lambda, acc, h_hat, loss,
                       mean_grad);
}

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_loss_spectrum_stats(const float* spectrum, const float* target, int32_t n_sets,
                                            int32_t n_chan, int32_t is_complex, int32_t H, int32_t W,
                                            float lambda_ch, float* loss, float* h_hat, float* mean_grad,
                                            float* d_partial, void* scratch, size_t scratch_bytes, void* stream)
{
    if (!spectrum || !target || !loss || !h_hat || !mean_grad || n_sets < 1 || n_chan < 1 || H < 1 || W < 1 ||
        (is_complex != 0 && is_complex != 1) || !(lambda_ch >= 0.0f))
        return GS_ERR_INVALID_ARG;
    if (n_chan > 65535 || n_sets > 65535) return GS_ERR_CAPACITY;
    const int C = is_complex ? 2 : 1;
    const int Fc = n_chan * C;
    const size_t need = (size_t)n_sets * Fc * 3 * sizeof(float);
    if (!scratch || scratch_bytes < need || ((uintptr_t)scratch & 255)) return GS_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    const size_t HW = (size_t)H * W;
    launch_fill_u32((uint32_t*)scratch, (size_t)n_sets * Fc * 3, 0, 1, 0u, s);
    const bool vec = (HW * C) % 4 == 0 &&
                     (((uintptr_t)spectrum | (uintptr_t)target | (uintptr_t)d_partial) & 15) == 0;
    const size_t per = vec ? HW * C / 4 : HW * C;
    const unsigned gx = (unsigned)((per + 255) / 256 < 32 ? (per + 255) / 256 : 32);
    dim3 grid(gx, n_chan, n_sets);
    const float scale = 2.0f / ((float)n_chan * (float)HW * (float)n_sets);
    if (vec)
        hipLaunchKernelGGL(k_loss_reduce<true>, grid, dim3(256), 0, s, spectrum, target, Fc, C, HW, (float*)scratch,
                           d_partial, scale);
    else
        hipLaunchKernelGGL(k_loss_reduce<false>, grid, dim3(256), 0, s, spectrum, target, Fc, C, HW, (float*)scratch,
                           d_partial, scale);
    hipLaunchKernelGGL(k_loss_finish, dim3(n_sets), dim3(256), 0, s, n_sets, Fc, C, HW, lambda_ch,
                       (const float*)scratch, h_hat, loss, mean_grad);
    if (hipGetLastError() != hipSuccess) return GS_ERR_HIP;
    return GS_OK;
}

// The two passes of gs_loss_spectrum() with a checked scratch of at least
// n_sets * F*c * 3 floats.
static gs_status loss_spectrum_run(const float* spectrum, const float* target, int32_t n_sets, int32_t n_chan,
                                   int32_t is_complex, int32_t H, int32_t W, float lambda_ch, float* loss,
                                   float* h_hat, float* d_spectrum, float* scratch, hipStream_t s)
{
    const int C = is_complex ? 2 : 1;
    const int Fc = n_chan * C;
    (void)hipGetLastError();
    const size_t HW = (size_t)H * W;
    launch_fill_u32((uint32_t*)scratch, (size_t)n_sets * Fc * 3, 0, 1, 0u, s);
    launch_fill_u32((uint32_t*)loss, (size_t)n_sets, 0, 1, 0u, s);
    const bool vec = (HW * C) % 4 == 0 && (((uintptr_t)spectrum | (uintptr_t)target | (uintptr_t)d_spectrum) & 15) == 0;
    const size_t per = vec ? HW * C / 4 : HW * C;  // items of one slice
    const unsigned gx = (unsigned)((per + 255) / 256 < 32 ? (per + 255) / 256 : 32);
    dim3 grid(gx, n_chan, n_sets);
    if (vec) {
        hipLaunchKernelGGL(k_loss_reduce<true>, grid, dim3(256), 0, s, spectrum, target, Fc, C, HW, scratch,
                           nullptr, 0.0f);
        hipLaunchKernelGGL(k_loss_grad<true>, grid, dim3(256), 0, s, spectrum, target, n_sets, Fc, C, HW, lambda_ch,
                           (const float*)scratch, d_spectrum, h_hat, loss);
    } else {
        hipLaunchKernelGGL(k_loss_reduce<false>, grid, dim3(256), 0, s, spectrum, target, Fc, C, HW, scratch,
                           nullptr, 0.0f);
        hipLaunchKernelGGL(k_loss_grad<false>, grid, dim3(256), 0, s, spectrum, target, n_sets, Fc, C, HW,
                           lambda_ch, (const float*)scratch, d_spectrum, h_hat, loss);
    }
    if (hipGetLastError() != hipSuccess) return GS_ERR_HIP;
    return GS_OK;
}

static bool loss_args_ok(const float* spectrum, const float* target, int32_t n_sets, int32_t n_chan,
                         int32_t is_complex, int32_t H, int32_t W, float lambda_ch, const float* loss,
                         const float* h_hat, const float* d_spectrum)
{
    return spectrum && target && loss && h_hat && d_spectrum && n_sets >= 1 && n_chan >= 1 && H >= 1 && W >= 1 &&
           (is_complex == 0 || is_complex == 1) && lambda_ch >= 0.0f;
}

extern "C" gs_status gs_loss_spectrum(const float* spectrum, const float* target, int32_t n_sets, int32_t n_chan,
                                      int32_t is_complex, int32_t H, int32_t W, float lambda_ch, float* loss,
                                      float* h_hat, float* d_spectrum, void* scratch, size_t scratch_bytes,
                                      void* stream)
{
    if (!loss_args_ok(spectrum, target, n_sets, n_chan, is_complex, H, W, lambda_ch, loss, h_hat, d_spectrum))
        return GS_ERR_INVALID_ARG;
    if (n_chan > 65535 || n_sets > 65535) return GS_ERR_CAPACITY;
    const size_t need = (size_t)n_sets * n_chan * (is_complex ? 2 : 1) * 3 * sizeof(float);
    if (!scratch || scratch_bytes < need || ((uintptr_t)scratch & 255)) return GS_ERR_WORKSPACE;
    return loss_spectrum_run(spectrum, target, n_sets, n_chan, is_complex, H, W, lambda_ch, loss, h_hat, d_spectrum,
                             (float*)scratch, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// gs_loss_spectrum_noalloc: the same loss with its per-channel accumulators
// in a file-scope device array instead of caller scratch.  Each device the
// library runs on holds its own copy of the array (until the process ends);
// its device address is looked up once per device, with that device
// current, on the entry point's first call there.  In host code the array's
// name is only a host-side stand-in: every kernel argument and fill uses the
// looked-up address.  Calls on one device share the array, so calls that
// overlap on one device (different streams) race; each call clears the
// accumulators it uses before accumulating.
// ---------------------------------------------------------------------------
static __device__ __align__(256) float scratch[GS_LOSS_NOALLOC_MAX_FLOATS];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
float* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

extern "C" gs_status gs_loss_spectrum_noalloc(const float* spectrum, const float* target, int32_t n_sets,
                                              int32_t n_chan, int32_t is_complex, int32_t H, int32_t W,
                                              float lambda_ch, float* loss, float* h_hat, float* d_spectrum,
                                              void* stream)
{
    if (!loss_args_ok(spectrum, target, n_sets, n_chan, is_complex, H, W, lambda_ch, loss, h_hat, d_spectrum))
        return GS_ERR_INVALID_ARG;
    if (n_chan > 65535 || n_sets > 65535) return GS_ERR_CAPACITY;
    const size_t need = (size_t)n_sets * n_chan * (is_complex ? 2 : 1) * 3;
    if (need > (size_t)GS_LOSS_NOALLOC_MAX_FLOATS) return GS_ERR_CAPACITY;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GS_ERR_HIP;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return GS_ERR_CAPACITY;
    float* acc = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GS_ERR_HIP;
            g_noalloc_ptr[dev] = (float*)ptr;
        }
        acc = g_noalloc_ptr[dev];
    }
    return loss_spectrum_run(spectrum, target, n_sets, n_chan, is_complex, H, W, lambda_ch, loss, h_hat, d_spectrum,
                             acc, (hipStream_t)stream);
}
