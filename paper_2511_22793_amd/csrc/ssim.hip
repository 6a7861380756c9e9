// Magnitude-spectrum loss, Eq. (5): per set b of real spectra
// zhat, z [F][H][W],
//   L_b = (1 - lambda_1) L1_b + lambda_1 (1 - SSIM_b),
// L1_b the mean absolute error over channels and pixels, SSIM_b the mean of
// the structural-similarity map: an 11 x 11 Gaussian window (sigma 1.5,
// normalised, separable) applied as a same-size filter with zero padding,
//   s = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)),
// mx = G*x, sxx = G*x^2 - mx^2, sxy = G*(x y) - mx my, C1 = 0.01^2,
// C2 = 0.03^2; and the gradient of L = (1/S) sum_b L_b.
//
// The gradient of the mean SSIM with respect to x at pixel q is, by the chain
// rule through the filtered maps (G symmetric, zero outside the image),
//   (G*a)(q) + 2 x(q) (G*b)(q) + y(q) (G*c)(q),
// a = ds/dmx, b = ds/dsxx (through G*x^2), c = ds/dsxy (through G*(x y)),
// each map zero outside the image, divided by the pixel count.
//
// One workgroup per (32 x 16 tile, channel, set), everything in LDS: the
// inputs with a 10-pixel halo, the five filtered maps on the tile with a
// 5-pixel halo (rows, then columns), the three derivative maps there, and
// their filtered values on the tile.  Per-workgroup sums of |x - y| and of s
// go to a partial buffer summed in a fixed order by a second kernel.
#include "common.h"

namespace gs {

constexpr int SS_TW = 32, SS_TH = 16, SS_R = 5;
constexpr int SS_K = 2 * SS_R + 1;               // window taps
constexpr int SS_IW = SS_TW + 4 * SS_R;          // input columns (52)
constexpr int SS_IH = SS_TH + 4 * SS_R;          // input rows (36)
constexpr int SS_MW = SS_TW + 2 * SS_R;          // map columns (42)
constexpr int SS_MH = SS_TH + 2 * SS_R;          // map rows (26)

struct SsimWin {
    float w[SS_K];
};

__global__ __launch_bounds__(256) void k_l1_ssim(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                 int W, int tiles_x, int ntiles, SsimWin win, float C1, float C2,
                                                 float gx_l1, float gx_ssim, float* __restrict__ grad,
                                                 float* __restrict__ part)
{
    const int tx0 = blockIdx.x * SS_TW, ty0 = blockIdx.y * SS_TH;
    const size_t img = blockIdx.z;  // set * F + channel
    const size_t HW = (size_t)H * W;
    x += img * HW;
    y += img * HW;
    __shared__ float s_x[SS_IH][SS_IW], s_y[SS_IH][SS_IW];
    __shared__ float s_h[5][SS_IH][SS_MW];   // row-filtered maps; later the derivative maps
    __shared__ float s_m[5][SS_MH][SS_MW];   // filtered maps; later the row-filtered derivative maps
    __shared__ float s_red[2][4];
    const int t = threadIdx.x;

    for (int i = t; i < SS_IH * SS_IW; i += 256) {
        const int r = i / SS_IW, c = i % SS_IW;
        const int gr = ty0 - 2 * SS_R + r, gc = tx0 - 2 * SS_R + c;
        const bool in = gr >= 0 && gr < H && gc >= 0 && gc < W;
        s_x[r][c] = in ? x[(size_t)gr * W + gc] : 0.0f;
        s_y[r][c] = in ? y[(size_t)gr * W + gc] : 0.0f;
    }
    __syncthreads();
    // rows: x, y, x^2, y^2, x y filtered along the columns
    for (int i = t; i < SS_IH * SS_MW; i += 256) {
        const int r = i / SS_MW, c = i % SS_MW;
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, a4 = 0.0f;
#pragma unroll
        for (int k = 0; k < SS_K; ++k) {
            const float xv = s_x[r][c + k], yv = s_y[r][c + k], w = win.w[k];
            a0 = fmaf(w, xv, a0);
            a1 = fmaf(w, yv, a1);
            a2 = fmaf(w, xv * xv, a2);
            a3 = fmaf(w, yv * yv, a3);
            a4 = fmaf(w, xv * yv, a4);
        }
        s_h[0][r][c] = a0;
        s_h[1][r][c] = a1;
        s_h[2][r][c] = a2;
        s_h[3][r][c] = a3;
        s_h[4][r][c] = a4;
    }
    __syncthreads();
    for (int i = t; i < 5 * SS_MH * SS_MW; i += 256) {
        const int q = i / (SS_MH * SS_MW), rc = i % (SS_MH * SS_MW);
        const int r = rc / SS_MW, c = rc % SS_MW;
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < SS_K; ++k) a = fmaf(win.w[k], s_h[q][r + k][c], a);
        s_m[q][r][c] = a;
    }
    __syncthreads();
    // SSIM and its derivative maps on the tile plus the 5-pixel halo (zero
    // outside the image); the SSIM sum over the tile's own pixels
    float ssum = 0.0f, l1sum = 0.0f;
    for (int i = t; i < SS_MH * SS_MW; i += 256) {
        const int r = i / SS_MW, c = i % SS_MW;
        const int gr = ty0 - SS_R + r, gc = tx0 - SS_R + c;
        float da = 0.0f, db = 0.0f, dc = 0.0f;
        if (gr >= 0 && gr < H && gc >= 0 && gc < W) {
            const float mx = s_m[0][r][c], my = s_m[1][r][c];
            const float sxx = s_m[2][r][c] - mx * mx, syy = s_m[3][r][c] - my * my, sxy = s_m[4][r][c] - mx * my;
            const float A1 = 2.0f * mx * my + C1, A2 = 2.0f * sxy + C2;
            const float B1 = mx * mx + my * my + C1, B2 = sxx + syy + C2;
            const float s = (A1 * A2) / (B1 * B2);
            da = s * (2.0f * my / A1 - 2.0f * my / A2 - 2.0f * mx / B1 + 2.0f * mx / B2);
            db = -s / B2;
            dc = 2.0f * s / A2;
            if (r >= SS_R && r < SS_R + SS_TH && c >= SS_R && c < SS_R + SS_TW) ssum += s;
        }
        s_h[0][r][c] = da;
        s_h[1][r][c] = db;
        s_h[2][r][c] = dc;
    }
    __syncthreads();
    // the derivative maps filtered along the columns (tile columns only)
    for (int i = t; i < 3 * SS_MH * SS_TW; i += 256) {
        const int q = i / (SS_MH * SS_TW), rc = i % (SS_MH * SS_TW);
        const int r = rc / SS_TW, c = rc % SS_TW;
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < SS_K; ++k) a = fmaf(win.w[k], s_h[q][r][c + k], a);
        s_m[q][r][c] = a;
    }
    __syncthreads();
    for (int i = t; i < SS_TH * SS_TW; i += 256) {
        const int r = i / SS_TW, c = i % SS_TW;
        const int gr = ty0 + r, gc = tx0 + c;
        if (gr >= H || gc >= W) continue;
        float ga = 0.0f, gb = 0.0f, gcc = 0.0f;
#pragma unroll
        for (int k = 0; k < SS_K; ++k) {
            ga = fmaf(win.w[k], s_m[0][r + k][c], ga);
            gb = fmaf(win.w[k], s_m[1][r + k][c], gb);
            gcc = fmaf(win.w[k], s_m[2][r + k][c], gcc);
        }
        const float xv = s_x[r + 2 * SS_R][c + 2 * SS_R], yv = s_y[r + 2 * SS_R][c + 2 * SS_R];
        const float d = xv - yv;
        l1sum += fabsf(d);
        if (grad) {
            const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            const float dss = ga + 2.0f * xv * gb + yv * gcc;
            grad[img * HW + (size_t)gr * W + gc] = gx_l1 * sg - gx_ssim * dss;
        }
    }
    // workgroup sums (fixed order)
    for (int o = 32; o > 0; o >>= 1) {
        ssum += __shfl_xor(ssum, o, 64);
        l1sum += __shfl_xor(l1sum, o, 64);
    }
    if ((t & 63) == 0) {
        s_red[0][t >> 6] = l1sum;
        s_red[1][t >> 6] = ssum;
    }
    __syncthreads();
    if (t < 2) {
        const size_t slot = (blockIdx.z * (size_t)ntiles + blockIdx.y * tiles_x + blockIdx.x) * 2 + t;
        part[slot] = s_red[t][0] + s_red[t][1] + s_red[t][2] + s_red[t][3];
    }
}

// per set: L1 = sum |x - y| / N, SSIM = sum s / N, loss = (1 - l) L1 + l (1 - SSIM)
__global__ __launch_bounds__(256) void k_l1_ssim_finish(const float* __restrict__ part, int per_set, float inv_n,
                                                        float lambda_1, float* __restrict__ loss,
                                                        float* __restrict__ ssim, float* __restrict__ l1)
{
    const int s = blockIdx.x;
    float a = 0.0f, b = 0.0f;
    for (int i = threadIdx.x; i < per_set; i += 256) {
        a += part[((size_t)s * per_set + i) * 2];
        b += part[((size_t)s * per_set + i) * 2 + 1];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    __shared__ float red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const float L1 = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) * inv_n;
        const float SS = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) * inv_n;
        if (l1) l1[s] = L1;
        if (ssim) ssim[s] = SS;
        loss[s] = (1.0f - lambda_1) * L1 + lambda_1 * (1.0f - SS);
    }
}

}  // namespace gs

using namespace gs;

extern "C" {

size_t gs_loss_l1_ssim_scratch_bytes(int32_t n_sets, int32_t n_chan, int32_t H, int32_t W)
{
    if (n_sets < 1 || n_chan < 1 || H < 1 || W < 1) return 0;
    const size_t tiles = (size_t)((W + SS_TW - 1) / SS_TW) * ((H + SS_TH - 1) / SS_TH);
    return align256((size_t)n_sets * n_chan * tiles * 2 * sizeof(float));
}

gs_status gs_loss_l1_ssim(const float* spectrum, const float* target, int32_t n_sets, int32_t n_chan, int32_t H,
                          int32_t W, float lambda_1, float* loss, float* ssim, float* l1, float* d_spectrum,
                          void* scratch, size_t scratch_bytes, void* stream)
{
    if (!spectrum || !target || !loss || n_sets < 1 || n_chan < 1 || H < 1 || W < 1 ||
        !(lambda_1 >= 0.0f && lambda_1 <= 1.0f))
        return GS_ERR_INVALID_ARG;
    if ((int64_t)n_sets * n_chan > 65535) return GS_ERR_CAPACITY;
    const size_t need = gs_loss_l1_ssim_scratch_bytes(n_sets, n_chan, H, W);
    if (!scratch || ((uintptr_t)scratch & 255) || scratch_bytes < need) return GS_ERR_WORKSPACE;
    SsimWin win{};
    {
        double g[SS_K], sum = 0.0;
        for (int k = 0; k < SS_K; ++k) {
            const double d = k - SS_R;
            g[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
            sum += g[k];
        }
        for (int k = 0; k < SS_K; ++k) win.w[k] = (float)(g[k] / sum);
    }
    const int tiles_x = (W + SS_TW - 1) / SS_TW, tiles_y = (H + SS_TH - 1) / SS_TH;
    const double N = (double)n_chan * H * W;
    const float gx_l1 = (float)((1.0 - lambda_1) / (N * n_sets));
    const float gx_ssim = (float)(lambda_1 / (N * n_sets));
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_l1_ssim, dim3(tiles_x, tiles_y, n_sets * n_chan), dim3(256), 0, s, spectrum, target, H, W,
                       tiles_x, tiles_x * tiles_y, win, 0.01f * 0.01f, 0.03f * 0.03f, gx_l1, gx_ssim, d_spectrum,
                       (float*)scratch);
    hipLaunchKernelGGL(k_l1_ssim_finish, dim3(n_sets), dim3(256), 0, s, (const float*)scratch,
                       n_chan * tiles_x * tiles_y, (float)(1.0 / N), lambda_1, loss, ssim, l1);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

}  // extern "C"
