// Backward of the front-to-back compositing (Eq. (3)), one workgroup per
// (tile, channel group, attribute set), one thread per pixel.
//
// With c_k = a_k sum_f g_f v_{k,f} (g = dL/dout of the pixel, summed over
// the group's channels) and T_k the transmittance in front of entry k:
//   dL/dv_{k,f}   = T_k alpha_k a_k g_f
//   dL/dalpha_k   = T_k c_k - R_k / (1 - alpha_k),  R_k = sum_{m>k} T_m alpha_m c_m
//   dL/da_k       = T_k alpha_k sum_f g_f v_{k,f}
// R_k = D - P_k with D = sum_f g_f out_f (the forward output) and P_k the
// running prefix, so the list is re-walked front to back, recomputing alpha
// and T instead of storing them; the walk ends at the pixel's recorded stop
// position.  alpha = min(alpha_max, sigma G): a clamped pair passes no
// gradient to sigma or G.  Through G = exp(-q/2) and the conic quadratic
// form q the gradient reaches the pixel-space centre and the conic.
//
// Per list entry the per-pixel terms are summed over the wave by a
// butterfly reduce-scatter (every lane ends with one summed value) and
// added to the per-Gaussian accumulators with one vector atomic.
#include "common.h"

namespace gs {

constexpr double LOG2E_B = 1.4426950408889634;

// Butterfly reduce-scatter of V values over the 64 lanes of a wave.  On
// return x[0] of lane l holds the wave total of value (l >> (6 - log2 V)).
template <int V>
__device__ __forceinline__ void wave_reduce_scatter(float* x, int lane)
{
    int n = V;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        if (n > 1) {
            const int half = n >> 1;
            const bool up = (lane & m) != 0;
#pragma unroll
            for (int i = 0; i < V / 2; ++i) {
                if (i < half) {
                    const float send = up ? x[i] : x[i + half];
                    const float keep = up ? x[i + half] : x[i];
                    x[i] = keep + __shfl_xor(send, m, 64);
                }
            }
            n = half;
        } else {
            x[0] += __shfl_xor(x[0], m, 64);
        }
    }
}

template <int CG>
__global__ __launch_bounds__(256) void k_blend_bwd(
    const GRec* __restrict__ rec, size_t s_rec, const uint32_t* __restrict__ plist, size_t s_plist,
    const uint2* __restrict__ ranges, size_t s_ranges, const float* __restrict__ attr, int64_t a_stride,
    int Fc, int C, int H, int W, int tw, int th, int TX, float amin, float amax,
    const float* __restrict__ out, const float* __restrict__ dout, const uint32_t* __restrict__ n_last, size_t s_pix,
    float* __restrict__ g2d, size_t s_g2d, float* __restrict__ d_attr, int64_t da_stride, int shared_geo)
{
    const int tile = blockIdx.x, cg = blockIdx.y, set = blockIdx.z;
    const int q = shared_geo ? 0 : set;
    const int nthr = tw * th;
    const int txi = tile % TX, tyi = tile / TX;
    const int lx = threadIdx.x % tw, ly = threadIdx.x / tw;
    const int col = txi * tw + lx, row = tyi * th + ly;
    const bool inside = col < W && row < H;
    const int lane = threadIdx.x & 63;
    const uint2 rg = ranges[q * s_ranges + tile];
    const double pcx = col + 0.5, pcy = row + 0.5, halfW = 0.5 * W;
    rec += q * s_rec;
    plist += q * s_plist;
    g2d += q * s_g2d;
    const float* A = attr + set * a_stride + cg * CG;
    float* dA = d_attr + set * da_stride + cg * CG;
    const size_t HW = (size_t)H * W, pix = inside ? (size_t)row * W + col : 0;
    const int F = Fc / C;

    // per-pixel upstream gradient of the group's channels and D = g . out
    float gch[CG];
    float D = 0.0f;
#pragma unroll
    for (int k = 0; k < CG; ++k) {
        const int ch = cg * CG + k;
        const int f = ch / C, comp = ch - f * C;
        const size_t idx = (((size_t)set * F + f) * HW + pix) * C + comp;
        gch[k] = inside ? dout[idx] : 0.0f;
        D += inside ? gch[k] * out[idx] : 0.0f;
    }
    const uint32_t stop = inside ? n_last[q * s_pix + pix] : 0u;

    __shared__ double s_px[256], s_py[256], s_ca[256], s_cb[256], s_cc[256];
    __shared__ float s_sig[256], s_att[256];
    __shared__ uint32_t s_g[256];

    float T = 1.0f, P = 0.0f;
    // the walk of this workgroup ends at the largest stop position of its pixels
    __shared__ uint32_t s_maxstop;
    if (threadIdx.x == 0) s_maxstop = 0;
    __syncthreads();
    if (stop) atomicMax(&s_maxstop, stop);
    __syncthreads();
    const uint32_t end = rg.x + s_maxstop;

    for (uint32_t b0 = rg.x; b0 < end; b0 += nthr) {
        __syncthreads();
        const uint32_t i = b0 + threadIdx.x;
        if (i < end) {
            const uint32_t g = plist[i];
            const GRec r = rec[g];
            s_px[threadIdx.x] = r.px;
            s_py[threadIdx.x] = r.py;
            s_ca[threadIdx.x] = r.ca;
            s_cb[threadIdx.x] = r.cb;
            s_cc[threadIdx.x] = r.cc;
            s_sig[threadIdx.x] = r.sigma;
            s_att[threadIdx.x] = r.att;
            s_g[threadIdx.x] = g;
        }
        __syncthreads();
        const int m = (int)min((uint32_t)nthr, end - b0);
        for (int j = 0; j < m; ++j) {
            const uint32_t g = __builtin_amdgcn_readfirstlane(s_g[j]);
            const float* vp = A + (size_t)g * Fc;
            float v[CG];
#pragma unroll
            for (int k = 0; k < CG; ++k) v[k] = vp[k];
            double dx = pcx - s_px[j];
            dx += dx >= halfW ? -(double)W : (dx < -halfW ? (double)W : 0.0);
            const double dy = pcy - s_py[j];
            const double ca = s_ca[j], cb = s_cb[j], cc = s_cc[j];
            const double qv = ca * dx * dx + 2.0 * cb * dx * dy + cc * dy * dy;
            const float G = __builtin_amdgcn_exp2f((float)(-0.5 * LOG2E_B * qv));
            const float sig = s_sig[j], att = s_att[j];
            const float sg = sig * G;
            const float alpha = fminf(amax, sg);
            const bool take = (b0 + j - rg.x) < stop && alpha >= amin;
            if (__ballot(take) == 0ull) continue;  // wave-uniform skip
            float gv = 0.0f;
#pragma unroll
            for (int k = 0; k < CG; ++k) gv = fmaf(gch[k], v[k], gv);
            const float cA = att * gv;
            const float Ta = T * alpha;
            const float Pn = P + Ta * cA;
            const float dalpha = T * cA - (D - Pn) / (1.0f - alpha);
            const float dsg = sg < amax ? dalpha : 0.0f;  // clamp passes nothing
            const float dq = -0.5f * dsg * sig * G;
            float red[CG];
            const float w = take ? Ta * att : 0.0f;
#pragma unroll
            for (int k = 0; k < CG; ++k) red[k] = w * gch[k];
            float geo[8];
            if (take) {
                geo[0] = dq * (float)(-2.0 * (ca * dx + cb * dy));  // d/dpx
                geo[1] = dq * (float)(-2.0 * (cb * dx + cc * dy));  // d/dpy
                geo[2] = dq * (float)(dx * dx);                     // d/dA
                geo[3] = dq * (float)(2.0 * dx * dy);               // d/dB
                geo[4] = dq * (float)(dy * dy);                     // d/dC
                geo[5] = dsg * G;                             // d/dsigma
                geo[6] = Ta * gv;                             // d/da
                geo[7] = 0.0f;
                T = T * (1.0f - alpha);
                P = Pn;
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) geo[k] = 0.0f;
            }
            wave_reduce_scatter<CG>(red, lane);
            wave_reduce_scatter<8>(geo, lane);
            constexpr int shA = CG >= 64 ? 0 : (CG == 32 ? 1 : (CG == 16 ? 2 : (CG == 8 ? 3 : (CG == 4 ? 4 : (CG == 2 ? 5 : 6)))));
            if ((lane & ((1 << shA) - 1)) == 0) unsafeAtomicAdd(dA + (size_t)g * Fc + (lane >> shA), red[0]);
            if ((lane & 7) == 0) unsafeAtomicAdd(g2d + (size_t)g * 8 + (lane >> 3), geo[0]);
        }
    }
}

template <int CG>
static void bwd_cg(dim3 grid, dim3 block, hipStream_t s, const gs_attrs& a, const gs_params& p, const Layout& L,
                   char* ws, const float* out, const float* dout, float* d_attr, int64_t da_stride, int C, int shared)
{
    hipLaunchKernelGGL(k_blend_bwd<CG>, grid, block, 0, s, (const GRec*)(ws + L.rec), L.s_rec / sizeof(GRec),
                       (const uint32_t*)(ws + L.plist), L.s_plist / 4, (const uint2*)(ws + L.ranges),
                       L.s_ranges / sizeof(uint2), a.data, a.query_stride, a.n_chan * C, C, L.H, L.W, L.tw, L.th,
                       L.TX, p.alpha_min, p.alpha_max, out, dout, (const uint32_t*)(ws + L.n_last), L.s_pix / 4,
                       (float*)(ws + L.g2d), L.s_g2d / 4, d_attr, da_stride, shared);
}

int choose_chan_group(int Fc, int requested);

gs_status launch_blend_bwd(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws,
                           const float* out, const float* dout, float* d_attr, hipStream_t s)
{
    const int C = a.is_complex ? 2 : 1;
    const int Fc = a.n_chan * C;
    int cg = choose_chan_group(Fc, p.chan_group);
    if (cg > 32) cg = 32;
    if (Fc / cg > 65535) return GS_ERR_CAPACITY;
    const int shared = (L.nq == 1 && n_sets > 1) ? 1 : 0;
    dim3 grid(L.T, Fc / cg, n_sets), block(L.tw * L.th);
    const int64_t das = a.query_stride;  // d_attr mirrors the attribute layout
    switch (cg) {
        case 1: bwd_cg<1>(grid, block, s, a, p, L, ws, out, dout, d_attr, das, C, shared); break;
        case 2: bwd_cg<2>(grid, block, s, a, p, L, ws, out, dout, d_attr, das, C, shared); break;
        case 4: bwd_cg<4>(grid, block, s, a, p, L, ws, out, dout, d_attr, das, C, shared); break;
        case 8: bwd_cg<8>(grid, block, s, a, p, L, ws, out, dout, d_attr, das, C, shared); break;
        case 16: bwd_cg<16>(grid, block, s, a, p, L, ws, out, dout, d_attr, das, C, shared); break;
        default: bwd_cg<32>(grid, block, s, a, p, L, ws, out, dout, d_attr, das, C, shared); break;
    }
    return GS_OK;
}

}  // namespace gs
