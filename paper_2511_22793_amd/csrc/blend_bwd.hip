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
// butterfly reduce-scatter (every lane ends with one summed value), the
// four waves are combined in LDS, and each batch of entries is flushed once
// per workgroup: attribute gradients by atomics, geometric terms into a
// per-pair accumulator (only the workgroups of one tile share an address)
// that a second pass folds into the per-Gaussian sums.  The nearest
// Gaussians cover every tile, so per-wave atomics would serialise on a few
// addresses.
#include <type_traits>

#include "common.h"

namespace gs {

constexpr double LOG2E_B = 1.4426950408889634;

// read-only attribute rows through the scalar/constant path where uniform
typedef __attribute__((address_space(4))) const float CFloatB;

// The same reduce-scatter for 8 values without the LDS crossbar: lane
// halves and quarter rows are exchanged with v_permlane32_swap /
// v_permlane16_swap (each swap also moves the partner's half, so one add
// completes a stage), the xor-8 stage and the final sum over 8 lanes use
// DPP row rotations and quad permutations.  Lane l ends with the wave
// total of value l >> 3 in x[0].
// (every lane has a source lane in these patterns; old = 0 with bound_ctrl
// lets the compiler fold the move into the add as a DPP operand)
__device__ __forceinline__ float dpp_f(float v, int ctrl_sel)
{
    const int iv = __float_as_int(v);
    int r;
    switch (ctrl_sel) {
        case 0: r = __builtin_amdgcn_update_dpp(0, iv, 0x128, 0xF, 0xF, true); break;  // row_ror:8
        case 1: r = __builtin_amdgcn_update_dpp(0, iv, 0xB1, 0xF, 0xF, true); break;   // quad_perm [1,0,3,2]
        case 2: r = __builtin_amdgcn_update_dpp(0, iv, 0x4E, 0xF, 0xF, true); break;   // quad_perm [2,3,0,1]
        default: r = __builtin_amdgcn_update_dpp(0, iv, 0x141, 0xF, 0xF, true); break; // row_half_mirror
    }
    return __int_as_float(r);
}

__device__ __forceinline__ void wave_reduce_scatter8(float* x, int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[i + 4]), false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[i]), __float_as_uint(x[i + 2]), false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const float t0 = x[0] + dpp_f(x[0], 0), t1 = x[1] + dpp_f(x[1], 0);
    float v = (lane & 8) ? t1 : t0;
    v += dpp_f(v, 1);
    v += dpp_f(v, 2);
    v += dpp_f(v, 3);
    x[0] = v;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Entries per matrix-core step of the attribute gradient (MFMA path), and
// entries staged in LDS per batch (a small batch keeps the LDS footprint,
// and so the occupancy, reasonable).
constexpr int BWD_SUB = 16;
constexpr int BWD_BATCH = 64;

template <int CG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_blend_bwd(
    const GRec* __restrict__ rec, size_t s_rec, const uint32_t* __restrict__ plist, size_t s_plist,
    const uint2* __restrict__ ranges, size_t s_ranges, const float* __restrict__ attr, int64_t a_stride,
    int Fc, int C, int H, int W, int tw, int th, int TX, float amin, float amax,
    const float* __restrict__ out, const float* __restrict__ dout, const float* __restrict__ tgt,
    const float* __restrict__ mgrad, float gscale, const uint32_t* __restrict__ n_last, size_t s_pix,
    float* __restrict__ gacc, size_t s_gacc, float* __restrict__ d_attr, int64_t da_stride, int shared_geo)
{
    // dL/dout of the element at idx = the elementwise part (read, or formed
    // from the output and the target) + the set's channel-mean term, which
    // the callers load once per channel (mg)
    auto upstream = [&](size_t idx) -> float { return tgt ? gscale * (out[idx] - tgt[idx]) : dout[idx]; };
    // plus the channel-mean term m_f of the set (0 without mgrad).  It is
    // not added to the per-pixel operands (that costs a quarter of the kernel
    // time in register pressure) but folded in exactly by linearity:
    //   D     += sum_f m_f out_f                    (per pixel, m uniform)
    //   gv_e  += sum_f m_f v_{e,f}                  (per entry, at staging)
    //   dL/dv_{e,f} += m_f sum_p w_{p,e}            (per entry, at the flush)
    auto mean_term = [&](int ch) -> float { return mgrad ? mgrad[(size_t)blockIdx.z * Fc + ch] : 0.0f; };
    // CG >= 16: the attribute gradient of a run of BWD_SUB entries,
    // dA[e][f] = sum_p w[p][e] g[p][f], is a 16 x CG x 64 product per wave
    // on the FP32 matrix cores (v_mfma_f32_16x16x4_f32); w goes through LDS.
    // Smaller groups reduce over the wave with the butterfly.
    constexpr bool MFMA = CG >= 16;
    constexpr int NB = MFMA ? CG / 16 : 1;
    const int tile = blockIdx.x, cg = blockIdx.y, set = blockIdx.z;
    const int q = shared_geo ? 0 : set;
    const int nthr = tw * th;
    const int txi = tile % TX, tyi = tile / TX;
    const int lx = threadIdx.x % tw, ly = threadIdx.x / tw;
    const int col = txi * tw + lx, row = tyi * th + ly;
    const bool inside = col < W && row < H;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint2 rg = ranges[q * s_ranges + tile];
    const double pcx = col + 0.5, pcy = row + 0.5, halfW = 0.5 * W;
    rec += q * s_rec;
    plist += q * s_plist;
    gacc += q * s_gacc;
    const float* A = attr + set * a_stride + cg * CG;
    float* dA = d_attr + set * da_stride + cg * CG;
    const size_t HW = (size_t)H * W, pix = inside ? (size_t)row * W + col : 0;
    // (the channel split below divides by the run-time C on purpose: the
    // shift form lets the scheduler interleave these loads with the walk and
    // the kernel then spills at its 128-register cap)
    const int F = Fc / C;

    // per-pixel upstream gradient of the group's channels and D = g . out
    float gch[CG];
    float D = 0.0f;
#pragma unroll
    for (int k = 0; k < CG; ++k) {
        const int ch = cg * CG + k;
        const int f = ch / C, comp = ch - f * C;
        const size_t idx = (((size_t)set * F + f) * HW + pix) * C + comp;
        const float mk = mean_term(ch);  // uniform
        gch[k] = inside ? upstream(idx) + (MFMA ? 0.0f : mk) : 0.0f;
        D += inside ? (MFMA ? gch[k] + mk : gch[k]) * out[idx] : 0.0f;
    }
    const uint32_t stop = inside ? n_last[q * s_pix + pix] : 0u;

    // MFMA operands held for the whole kernel:
    //  gB (attribute gradient, B = g[pixel][channel]): for K-step s the lane
    //    holds g of pixel 4s + lane/16 of its wave, channel nb*16 + lane%16;
    //  gT (gv = v . g per entry and pixel, B = g^T[channel][pixel]): for
    //    K-step k and pixel block pb the lane holds g of pixel 16 pb + lane%16,
    //    channel 4k + lane/16.
    float gB[MFMA ? 16 : 1][NB];
    float gT[MFMA ? 4 : 1][MFMA ? CG / 4 : 1];
    if constexpr (MFMA) {
        // (t % tw and t / tw are computed directly: stepping them in loops
        // puts a branch between the loads and serialises their latency)
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) {
            const int t = wave * 64 + 16 * pb + (lane & 15);
            const int pc = txi * tw + t % tw, pr = tyi * th + t / tw;
            const bool in = t < nthr && pc < W && pr < H;
            const size_t pp = in ? (size_t)pr * W + pc : 0;
#pragma unroll
            for (int k = 0; k < CG / 4; ++k) {
                const int ch = cg * CG + 4 * k + (lane >> 4);
                const int f = ch / C, comp = ch - f * C;
                gT[pb][k] = in ? upstream((((size_t)set * F + f) * HW + pp) * C + comp) : 0.0f;
            }
        }
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int t = wave * 64 + 4 * st + (lane >> 4);
            const int pc = txi * tw + t % tw, pr = tyi * th + t / tw;
            const bool in = t < nthr && pc < W && pr < H;
            const size_t pp = in ? (size_t)pr * W + pc : 0;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int ch = cg * CG + nb * 16 + (lane & 15);
                const int f = ch / C, comp = ch - f * C;
                gB[st][nb] = in ? upstream((((size_t)set * F + f) * HW + pp) * C + comp) : 0.0f;
            }
        }
    }

    __shared__ double s_px[BWD_BATCH], s_py[BWD_BATCH], s_ca[BWD_BATCH], s_cb[BWD_BATCH], s_cc[BWD_BATCH];
    __shared__ float s_sig[BWD_BATCH], s_att[BWD_BATCH];
    __shared__ float s_caf[BWD_BATCH], s_cbf[BWD_BATCH], s_ccf[BWD_BATCH];
    __shared__ uint32_t s_g[BWD_BATCH];
    // per-entry sums over the workgroup's pixels, flushed once per batch
    __shared__ float s_ad[BWD_BATCH][CG];
    __shared__ float s_geo[BWD_BATCH][8];
    __shared__ float s_m[CG];              // m_f of the group's channels
    __shared__ float s_mvb[BWD_BATCH];     // sum_f m_f v_{e,f} per staged entry
    // per wave, for the current run of entries: gv = v . g from the matrix
    // cores, replaced entry by entry by the pixel weight w (rows padded)
    __shared__ float s_w[MFMA ? 4 : 1][MFMA ? BWD_SUB : 1][65];

    float T = 1.0f, P = 0.0f;
    // the walk of this workgroup ends at the largest stop position of its pixels
    __shared__ uint32_t s_maxstop;
    if (threadIdx.x == 0) s_maxstop = 0;
    if ((int)threadIdx.x < CG) s_m[threadIdx.x] = mean_term(cg * CG + threadIdx.x);
    __syncthreads();
    if (stop) atomicMax(&s_maxstop, stop);
    __syncthreads();
    const uint32_t end = rg.x + s_maxstop;
    // a wave stops walking at the largest stop position of its own pixels
    uint32_t wstop = stop;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wstop = max(wstop, (uint32_t)__shfl_xor((int)wstop, o, 64));
    const uint32_t wend = rg.x + wstop;
    constexpr int shA = CG >= 64 ? 0 : (CG == 32 ? 1 : (CG == 16 ? 2 : (CG == 8 ? 3 : (CG == 4 ? 4 : (CG == 2 ? 5 : 6)))));

    for (uint32_t b0 = rg.x; b0 < end; b0 += BWD_BATCH) {
        __syncthreads();
        const uint32_t i = b0 + threadIdx.x;
        if (threadIdx.x < BWD_BATCH && i < end) {
            const uint32_t g = plist[i];
            const GRec r = rec[g];
            s_px[threadIdx.x] = r.px;
            s_py[threadIdx.x] = r.py;
            s_ca[threadIdx.x] = r.ca;
            s_cb[threadIdx.x] = r.cb;
            s_cc[threadIdx.x] = r.cc;
            s_caf[threadIdx.x] = (float)r.ca;
            s_cbf[threadIdx.x] = (float)r.cb;
            s_ccf[threadIdx.x] = (float)r.cc;
            s_sig[threadIdx.x] = r.sigma;
            s_att[threadIdx.x] = r.att;
            s_g[threadIdx.x] = g;
        }
        for (int e = threadIdx.x; e < BWD_BATCH * CG; e += nthr) s_ad[e / CG][e % CG] = 0.0f;
        for (int e = threadIdx.x; e < BWD_BATCH * 8; e += nthr) s_geo[e / 8][e % 8] = 0.0f;
        __syncthreads();
        const int m = (int)min((uint32_t)BWD_BATCH, end - b0);
        if constexpr (MFMA) {
            // sum_f m_f v_{e,f} of the staged entries: four threads per entry
            const int e = threadIdx.x >> 2, qd = threadIdx.x & 3;
            float mv = 0.0f;
            if (e < m) {
                const float* vr = A + (size_t)s_g[e] * Fc + qd * (CG / 4);
#pragma unroll
                for (int k = 0; k < CG / 4; ++k) mv = fmaf(s_m[qd * (CG / 4) + k], vr[k], mv);
            }
            mv += __shfl_xor(mv, 1, 64);
            mv += __shfl_xor(mv, 2, 64);
            if (qd == 0 && e < m) s_mvb[e] = mv;
            __syncthreads();
        }
        for (int j0 = 0; j0 < m; j0 += (MFMA ? BWD_SUB : m)) {
            if (b0 + j0 >= wend) break;  // wave-uniform: nothing left for this wave
            const int jn = MFMA ? min(BWD_SUB, m - j0) : m;
            if constexpr (MFMA) {
                // gv[e][p] = sum_f v[e][f] g[p][f]: A = v rows of the run
                // (lane: entry lane%16, channel 4k + lane/16), B = gT
                const int e = lane & 15;
                const bool ev = e < jn;
                const CFloatB* vr = (const CFloatB*)(A + (size_t)(ev ? s_g[j0 + e] : 0u) * Fc) + (lane >> 4);
                float va[CG / 4];
#pragma unroll
                for (int k = 0; k < CG / 4; ++k) va[k] = ev ? vr[4 * k] : 0.0f;

                f32x4 gv4[4];
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) {
                    gv4[pb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int k = 0; k < CG / 4; ++k)
                        gv4[pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(va[k], gT[pb][k], gv4[pb], 0, 0, 0);
                }
                // lane holds entries 4*(lane/16) + r of pixel 16 pb + lane%16
#pragma unroll
                for (int pb = 0; pb < 4; ++pb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) s_w[wave][4 * (lane >> 4) + r][16 * pb + (lane & 15)] = gv4[pb][r];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            for (int jj = 0; jj < (MFMA ? BWD_SUB : jn); ++jj) {
                const int j = j0 + jj;
                float w = 0.0f;
                if (jj < jn && b0 + j < wend) {
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
                    if (__ballot(take) != 0ull) {  // else the whole wave skips the entry
                        float gv = 0.0f;
                        if constexpr (MFMA) {
                            gv = s_w[wave][jj][lane] + s_mvb[j];
                        } else {
                            const uint32_t g = __builtin_amdgcn_readfirstlane(s_g[j]);
                            const float* vp = A + (size_t)g * Fc;
#pragma unroll
                            for (int k = 0; k < CG; ++k) gv = fmaf(gch[k], vp[k], gv);
                        }
                        // branch-free: a lane that does not take the entry
                        // gets Ta = 0, so every term below is zero and T, P
                        // stay as they are
                        const float cA = att * gv;
                        const float Ta = take ? T * alpha : 0.0f;
                        const float Pn = P + Ta * cA;
                        // alpha <= alpha_max < 1; a one-ulp reciprocal is ample here
                        const float dalpha = T * cA - (D - Pn) * __builtin_amdgcn_rcpf(1.0f - alpha);
                        const float dsg = (take && sg < amax) ? dalpha : 0.0f;  // clamp passes nothing
                        const float dq = -0.5f * dsg * sig * G;
                        w = Ta * att;
                        // gradient factors in FP32 from the exact offsets
                        const float dxf = (float)dx, dyf = (float)dy;
                        const float dq2 = -2.0f * dq;
                        float geo[8];
                        geo[0] = dq2 * fmaf(s_caf[j], dxf, s_cbf[j] * dyf);  // d/dpx
                        geo[1] = dq2 * fmaf(s_cbf[j], dxf, s_ccf[j] * dyf);  // d/dpy
                        geo[2] = dq * (dxf * dxf);                           // d/dA
                        geo[3] = dq * (2.0f * dxf * dyf);                    // d/dB
                        geo[4] = dq * (dyf * dyf);                           // d/dC
                        geo[5] = dsg * G;                                   // d/dsigma
                        geo[6] = Ta * gv;                                   // d/da
                        geo[7] = w;                                         // sum_p w (mean term)
                        T = take ? T * (1.0f - alpha) : T;
                        P = Pn;
                        wave_reduce_scatter8(geo, lane);
                        if ((lane & 7) == 0) atomicAdd(&s_geo[j][lane >> 3], geo[0]);
                        if constexpr (!MFMA) {
                            float red[CG];
#pragma unroll
                            for (int k = 0; k < CG; ++k) red[k] = w * gch[k];
                            wave_reduce_scatter<CG>(red, lane);
                            if ((lane & ((1 << shA) - 1)) == 0) atomicAdd(&s_ad[j][lane >> shA], red[0]);
                        }
                    }
                }
                if constexpr (MFMA) s_w[wave][jj][lane] = w;
            }
            if constexpr (MFMA) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                f32x4 acc[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    const float a = s_w[wave][lane & 15][4 * st + (lane >> 4)];
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, gB[st][nb], acc[nb], 0, 0, 0);
                }
                // lane holds entries 4*(lane/16) + r, channel nb*16 + lane%16
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = 4 * (lane >> 4) + r;
                    if (e < jn) {
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            if (acc[nb][r] != 0.0f) atomicAdd(&s_ad[j0 + e][nb * 16 + (lane & 15)], acc[nb][r]);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        __syncthreads();
        // flush: attribute gradients (one atomic per entry and channel per
        // workgroup), geometric terms into the per-pair accumulator
        for (int e = threadIdx.x; e < m * CG; e += nthr) {
            const int j = e / CG, k = e % CG;
            const float val = MFMA ? s_ad[j][k] + s_m[k] * s_geo[j][7] : s_ad[j][k];
            if (val != 0.0f) unsafeAtomicAdd(dA + (size_t)s_g[j] * Fc + k, val);
        }
        for (int e = threadIdx.x; e < m * 8; e += nthr) {
            const int j = e / 8, k = e % 8;
            const float val = k < 7 ? s_geo[j][k] : 0.0f;  // slot 7 holds sum_p w
            if (val != 0.0f) unsafeAtomicAdd(gacc + (size_t)(b0 + j) * 8 + k, val);
        }
    }
}

// ---------------------------------------------------------------------------
// Backward over attribute sets that share one geometry (one prepared query,
// S attribute sets: the transmitter batch of the training step).
//
// T_k, alpha_k, G_k and a_k do not depend on the set, so the per-set terms
// above combine linearly:
//   sum over sets and channels of dL/dalpha_k
//     = T_k a_k GV_k - (D - P_k) / (1 - alpha_k),
//   GV_k = sum_{s,f} g_{s,f} v_{s,k,f},  D = sum_{s,f} g_{s,f} out_{s,f},
//   P_k = sum_{m<=k} T_m alpha_m a_m GV_m,
// and dL/dv_{s,k,f} = w_k g_{s,f} with the set-independent weight
// w_k = T_k alpha_k a_k.  One workgroup takes 64 pixels of a tile and every
// column (set, channel) at once: per batch of entries the matrix cores form
// GV (entries x pixels, contracted over all S*F*c columns), one wave walks
// the pixels' lists once for the geometric terms and the weights, and the
// matrix cores form dL/dv = W^T g (entries x columns, contracted over the
// pixels).  Eight waves split the columns; the geometry is evaluated once
// per (pixel, entry) instead of once per set and channel group.
// ---------------------------------------------------------------------------
constexpr int SG_WAVES = 8;   // column split
constexpr int SG_E = 64;      // entries per batch
constexpr int SG_PIX = 64;    // pixels per workgroup

struct SgUp {  // upstream gradient g = upstream + mean term
    const float* out;
    const float* dout;
    const float* tgt;
    const float* mgrad;
    float scale;
    const float* gscale;  // with tgt: device factor on scale (the mean term carries it already), or null
};

// Raw upstream words of one element: dout, or (out, target) with TGT.
template <bool TGT>
struct SgRaw {
    float a, b;
};
template <bool TGT>
__device__ __forceinline__ SgRaw<TGT> sg_fetch(const SgUp& u, size_t idx)
{
    if constexpr (TGT) return SgRaw<TGT>{u.out[idx], u.tgt[idx]};
    else return SgRaw<TGT>{u.dout[idx], 0.0f};
}
template <bool TGT>
__device__ __forceinline__ float sg_value(const SgUp& u, SgRaw<TGT> r)
{
    if constexpr (TGT) return u.scale * (r.a - r.b);
    else return r.a;
}
// (re, im) or two consecutive real channels at element index idx (even)
template <bool TGT>
__device__ __forceinline__ float2 sg_load2(const SgUp& u, size_t idx)
{
    if constexpr (TGT) {
        const float2 o = *(const float2*)(u.out + idx), t = *(const float2*)(u.tgt + idx);
        return float2{u.scale * (o.x - t.x), u.scale * (o.y - t.y)};
    } else {
        return *(const float2*)(u.dout + idx);
    }
}

// stands in for an absent mean-term vector (read with stride 0)
__device__ const float4 sg_zero4 = {0.0f, 0.0f, 0.0f, 0.0f};

template <int CS, bool TGT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_blend_bwd_sg(
    const GRec* __restrict__ rec, const uint32_t* __restrict__ plist, const uint2* __restrict__ ranges,
    const float* __restrict__ attr, int64_t a_stride, int S, int Fc, int H, int W, int tw_log, int th, int TX,
    float amin, float amax, SgUp up_in, const uint32_t* __restrict__ n_last, float* __restrict__ gacc,
    float* __restrict__ d_attr, int64_t da_stride, int min_walk, float* __restrict__ lacc)
{
    SgUp up = up_in;
    if (TGT && up.gscale) up.scale *= *up.gscale;
    const int tw = 1 << tw_log;
    const int tile = blockIdx.x, pg = blockIdx.y;
    // (wave-uniform values go through readfirstlane so that they live in
    // scalar registers)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j4 = lane >> 4, l16 = lane & 15;
    const int txi = tile % TX, tyi = tile / TX;
    const uint2 rg = ranges[tile];
    const size_t HW = (size_t)H * W;
    const int F = Fc >> CS;
    const int ncb = S * Fc / 16;  // 16-column blocks (Fc % 16 == 0)
    const int cb_lo = wave * ncb / SG_WAVES, cb_hi = (wave + 1) * ncb / SG_WAVES;
    // mean term m[s * Fc + c], or zeros
    const float* mg = up.mgrad ? up.mgrad : (const float*)&sg_zero4;
    const size_t mstr = up.mgrad ? 1 : 0;

    // The tile's pixels inside the image (vw x vh, row-major) are packed
    // into groups of 64: edge tiles need fewer groups, and the spare
    // workgroups leave at once.
    const int vw = min(tw, W - txi * tw), vh = min(th, H - tyi * th);
    if (pg * SG_PIX >= vw * vh) return;
    auto pixel_of = [&](int k) -> int {
        return k < vw * vh ? (tyi * th + k / vw) * W + txi * tw + k % vw : -1;
    };

    __shared__ float s_gv[SG_E][SG_PIX + 1];  // GV of the batch
    __shared__ float s_w[SG_E][SG_PIX + 1];   // weights w of the batch
    __shared__ int s_pix[SG_PIX];             // image offset of each pixel of the group (-1 outside)
    __shared__ double s_px[SG_E], s_py[SG_E], s_ca[SG_E], s_cb[SG_E], s_cc[SG_E];
    __shared__ float s_caf[SG_E], s_cbf[SG_E], s_ccf[SG_E], s_sig[SG_E], s_att[SG_E];
    __shared__ uint32_t s_g[SG_E];
    __shared__ float s_D[SG_PIX];
    __shared__ uint32_t s_maxstop;

    // the walking wave's pixel (lane) and its stop position
    const int wpix = pixel_of(pg * SG_PIX + lane);
    const uint32_t stop = (wave == 0 && wpix >= 0) ? n_last[wpix] : 0u;
    if (threadIdx.x == 0) s_maxstop = 0;
    if (threadIdx.x < SG_PIX) {
        s_D[threadIdx.x] = 0.0f;
        s_pix[threadIdx.x] = pixel_of(pg * SG_PIX + threadIdx.x);
    }
    for (int e = threadIdx.x; e < SG_E * (SG_PIX + 1); e += blockDim.x) (&s_gv[0][0])[e] = 0.0f;
    __syncthreads();
    if (stop) atomicMax(&s_maxstop, stop);
    __syncthreads();
    // (min_walk > 0: only groups whose walk is longer than min_walk entries)
    if (min_walk > 0 && s_maxstop <= (uint32_t)min_walk) return;
    const uint32_t end = __builtin_amdgcn_readfirstlane(rg.x + s_maxstop);
    // one batch holds the whole walk of the group (the common case): D is
    // then the walk's own final prefix sum_k w_k GV_k (out = sum_k w_k v_k),
    // else it is formed from the forward output first
    const bool one_batch = end - rg.x <= (uint32_t)SG_E;

    if (end > rg.x && !one_batch) {
        int pixB[4];
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) pixB[pb] = s_pix[16 * pb + l16];
        float dp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int cb = cb_lo; cb < cb_hi; ++cb) {
            const int s = cb * 16 / Fc;
            const int ch = cb * 16 - s * Fc + 4 * j4;
            float mk[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) mk[kk] = mg[((size_t)s * Fc + ch + kk) * mstr];
            float ls = 0.0f;  // squared error of the block (with lacc)
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                const int px = pixB[pb];
                if (px < 0) continue;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const size_t i = (((size_t)(s * F + ((ch + kk) >> CS)) * HW + px) << CS) + ((ch + kk) & CS);
                    const SgRaw<TGT> raw = sg_fetch<TGT>(up, i);
                    dp[pb] += (sg_value<TGT>(up, raw) + mk[kk]) * up.out[i];
                    if constexpr (TGT) {
                        const float d = raw.a - raw.b;
                        ls = fmaf(d, d, ls);
                    }
                }
            }
            if (TGT && lacc) {
                for (int o = 32; o > 0; o >>= 1) ls += __shfl_xor(ls, o, 64);
                if (lane == 0 && ls != 0.0f) atomicAdd(lacc + s, ls);
            }
        }
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) {
            float v = dp[pb];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (j4 == 0 && cb_hi > cb_lo) atomicAdd(&s_D[16 * pb + l16], v);
        }
    }

    float T = 1.0f, P = 0.0f, D = 0.0f;

    for (uint32_t b0 = rg.x; b0 < end; b0 += SG_E) {
        const int m = (int)min((uint32_t)SG_E, end - b0);
        const int neb = (m + 15) >> 4;
        const bool first = b0 == rg.x;
        if ((int)threadIdx.x < m) {
            const uint32_t g = plist[b0 + threadIdx.x];
            const GRec r = rec[g];
            s_px[threadIdx.x] = r.px;
            s_py[threadIdx.x] = r.py;
            s_ca[threadIdx.x] = r.ca;
            s_cb[threadIdx.x] = r.cb;
            s_cc[threadIdx.x] = r.cc;
            s_caf[threadIdx.x] = (float)r.ca;
            s_cbf[threadIdx.x] = (float)r.cb;
            s_ccf[threadIdx.x] = (float)r.cc;
            s_sig[threadIdx.x] = r.sigma;
            s_att[threadIdx.x] = r.att;
            s_g[threadIdx.x] = g;
        }
        __syncthreads();

        // ---- GV[e][p] = sum over this wave's columns of v[e][c] g[p][c]
        // K-step kk of a 16-column block pairs lane group j4 with channel
        // ch0 + 4 j4 + kk, so each lane reads 4 consecutive channels.
        // NEB = entry blocks of 16 in the batch (a compile-time count keeps
        // the matrix-core sequence free of branches).
        // Wave w takes pixel blocks 2 (w & 1) and 2 (w & 1) + 1 and one of
        // SG_WAVES / 2 column ranges (32 accumulator registers).
        auto gv_phase = [&](auto nebc) {
            constexpr int NEB = decltype(nebc)::value;
            const int ph = wave & 1, cq = wave >> 1;
            const int q_lo = cq * ncb / (SG_WAVES / 2), q_hi = (cq + 1) * ncb / (SG_WAVES / 2);
            int pixB[2];
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) pixB[pb] = s_pix[16 * (2 * ph + pb) + l16];
            f32x4 acc[NEB][2];
#pragma unroll
            for (int eb = 0; eb < NEB; ++eb)
#pragma unroll
                for (int pb = 0; pb < 2; ++pb) acc[eb][pb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            uint32_t ge[NEB];
#pragma unroll
            for (int eb = 0; eb < NEB; ++eb) {
                const int e = 16 * eb + l16;
                ge[eb] = e < m ? s_g[e] : 0xFFFFFFFFu;
            }
            // Operands of one 16-column block: v of 4 consecutive channels per
            // entry block, the raw upstream words of those channels per pixel
            // block, and the mean terms; the next block's are fetched while
            // this block multiplies (software pipelining).
            constexpr int NR = TGT ? 2 : 1;
            struct Ops {
                float4 a[NEB];
                float b[2][4][NR];
                float4 mm;
            };
            auto load = [&](int cb, Ops& o) {
                const int s = cb * 16 / Fc;
                const int ch = cb * 16 - s * Fc + 4 * j4;
                const float* As = attr + s * a_stride + ch;
#pragma unroll
                for (int eb = 0; eb < NEB; ++eb)
                    o.a[eb] = ge[eb] != 0xFFFFFFFFu ? *(const float4*)(As + (size_t)ge[eb] * Fc)
                                                    : float4{0.0f, 0.0f, 0.0f, 0.0f};
                o.mm = *(const float4*)(mg + ((size_t)s * Fc + ch) * mstr);
#pragma unroll
                for (int pb = 0; pb < 2; ++pb) {
                    const size_t px = pixB[pb] >= 0 ? (size_t)pixB[pb] : 0;
                    if constexpr (CS == 1) {
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const size_t i = ((size_t)(s * F + (ch >> 1) + h) * HW + px) * 2;
                            const float2 u = *(const float2*)(TGT ? up.out + i : up.dout + i);
                            o.b[pb][2 * h][0] = u.x;
                            o.b[pb][2 * h + 1][0] = u.y;
                            if constexpr (TGT) {
                                const float2 t = *(const float2*)(up.tgt + i);
                                o.b[pb][2 * h][NR - 1] = t.x;
                                o.b[pb][2 * h + 1][NR - 1] = t.y;
                            }
                        }
                    } else {
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            const size_t i = (size_t)(s * F + ch + kk) * HW + px;
                            o.b[pb][kk][0] = TGT ? up.out[i] : up.dout[i];
                            if constexpr (TGT) o.b[pb][kk][NR - 1] = up.tgt[i];
                        }
                    }
                }
            };
            Ops ops[2];
            if (q_hi > q_lo) load(q_lo, ops[0]);
            for (int cb = q_lo; cb < q_hi; cb += 2) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int cc = cb + half;
                    if (cc < q_hi) {
                        if (cc + 1 < q_hi) load(cc + 1, ops[half ^ 1]);
                        __builtin_amdgcn_sched_barrier(0);
                        const Ops& o = ops[half];
                        const float mk[4] = {o.mm.x, o.mm.y, o.mm.z, o.mm.w};
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            float bv[2];
#pragma unroll
                            for (int pb = 0; pb < 2; ++pb) {
                                const float u = TGT ? up.scale * (o.b[pb][kk][0] - o.b[pb][kk][NR - 1]) : o.b[pb][kk][0];
                                bv[pb] = pixB[pb] >= 0 ? u + mk[kk] : 0.0f;
                            }
#pragma unroll
                            for (int eb = 0; eb < NEB; ++eb) {
                                const float av = kk == 0 ? o.a[eb].x : (kk == 1 ? o.a[eb].y : (kk == 2 ? o.a[eb].z : o.a[eb].w));
#pragma unroll
                                for (int pb = 0; pb < 2; ++pb)
                                    acc[eb][pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[pb], acc[eb][pb], 0, 0, 0);
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
            // lane holds GV of entry 16 eb + 4 j4 + r, pixel 16 (2 ph + pb) + l16
            if (q_hi > q_lo) {
#pragma unroll
                for (int eb = 0; eb < NEB; ++eb)
#pragma unroll
                    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            atomicAdd(&s_gv[16 * eb + 4 * j4 + r][16 * (2 * ph + pb) + l16], acc[eb][pb][r]);
            }
        };
        switch (neb) {
            case 1: gv_phase(std::integral_constant<int, 1>{}); break;
            case 2: gv_phase(std::integral_constant<int, 2>{}); break;
            case 3: gv_phase(std::integral_constant<int, 3>{}); break;
            default: gv_phase(std::integral_constant<int, 4>{}); break;
        }
        __syncthreads();

        // ---- the walk: one lane per pixel, front to back
        if (wave == 0) {
            const double pcx = (wpix >= 0 ? wpix % W : 0) + 0.5, pcy = (wpix >= 0 ? wpix / W : 0) + 0.5;
            const double halfW = 0.5 * W;
            // offsets, G and alpha of entry e at this lane's pixel
            auto geom = [&](int e, double& dx, double& dy, float& G) -> float {
                dx = pcx - s_px[e];
                dx += dx >= halfW ? -(double)W : (dx < -halfW ? (double)W : 0.0);
                dy = pcy - s_py[e];
                const double qv = s_ca[e] * dx * dx + 2.0 * s_cb[e] * dx * dy + s_cc[e] * dy * dy;
                G = __builtin_amdgcn_exp2f((float)(-0.5 * LOG2E_B * qv));
                return s_sig[e] * G;
            };
            if (first) {
                if (one_batch) {
                    // D = the final prefix of the walk below, same operations
                    float Tq = 1.0f, Pq = 0.0f;
                    for (int e = 0; e < m; ++e) {
                        double dx, dy;
                        float G;
                        const float sg = geom(e, dx, dy, G);
                        const float alpha = fminf(amax, sg);
                        const bool take = (b0 + e - rg.x) < stop && alpha >= amin;
                        const float cA = s_att[e] * s_gv[e][lane];
                        const float Ta = take ? Tq * alpha : 0.0f;
                        Pq = Pq + Ta * cA;
                        Tq = take ? Tq * (1.0f - alpha) : Tq;
                    }
                    D = Pq;
                } else {
                    D = s_D[lane];
                }
            }
            for (int e = 0; e < m; ++e) {
                float w = 0.0f;
                double dx, dy;
                float G;
                const float sg = geom(e, dx, dy, G);
                const float sig = s_sig[e], att = s_att[e];
                const float alpha = fminf(amax, sg);
                const bool take = (b0 + e - rg.x) < stop && alpha >= amin;
                if (__ballot(take) != 0ull) {
                    const float gv = s_gv[e][lane];
                    const float cA = att * gv;
                    const float Ta = take ? T * alpha : 0.0f;
                    const float Pn = P + Ta * cA;
                    const float dalpha = T * cA - (D - Pn) * __builtin_amdgcn_rcpf(1.0f - alpha);
                    const float dsg = (take && sg < amax) ? dalpha : 0.0f;
                    const float dq = -0.5f * dsg * sig * G;
                    w = Ta * att;
                    const float dxf = (float)dx, dyf = (float)dy;
                    const float dq2 = -2.0f * dq;
                    float geo[8];
                    geo[0] = dq2 * fmaf(s_caf[e], dxf, s_cbf[e] * dyf);
                    geo[1] = dq2 * fmaf(s_cbf[e], dxf, s_ccf[e] * dyf);
                    geo[2] = dq * (dxf * dxf);
                    geo[3] = dq * (2.0f * dxf * dyf);
                    geo[4] = dq * (dyf * dyf);
                    geo[5] = dsg * G;
                    geo[6] = Ta * gv;
                    geo[7] = 0.0f;
                    T = take ? T * (1.0f - alpha) : T;
                    P = Pn;
                    wave_reduce_scatter8(geo, lane);
                    if ((lane & 7) == 0 && lane < 56 && geo[0] != 0.0f)
                        unsafeAtomicAdd(gacc + (size_t)(b0 + e) * 8 + (lane >> 3), geo[0]);
                }
                s_w[e][lane] = w;
                s_gv[e][lane] = 0.0f;  // cleared for the next batch
            }
        }
        __syncthreads();

        // ---- dL/dv[e][c] = sum_p w[e][p] g[p][c]: K-step kk pairs lane
        // group j4 with pixel 4 kk + j4.  The next block's upstream words
        // are fetched before this block's products (software pipelining).
        auto da_phase = [&](auto nebc) {
            constexpr int NEB = decltype(nebc)::value;
            uint32_t pvalid = 0;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) pvalid |= (s_pix[4 * kk + j4] >= 0 ? 1u : 0u) << kk;
            SgRaw<TGT> rb[2][16];
            // a uniform base per set and 32-bit lane offsets (one register
            // per address)
            auto fetch = [&](int cb, SgRaw<TGT>* r) {
                const int s = cb * 16 / Fc;
                const int c = cb * 16 - s * Fc + l16;
                const size_t sbase = ((size_t)s * F * HW) << CS;
                const uint32_t coff = ((uint32_t)((c >> CS) * HW) << CS) + (uint32_t)(c & CS);
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) {
                    const int px = s_pix[4 * kk + j4];
                    r[kk] = sg_fetch<TGT>(up, sbase + (coff + (px >= 0 ? ((uint32_t)px << CS) : 0u)));
                }
            };
            for (int cb = cb_lo; cb < cb_hi; cb += 2) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int cc = cb + half;
                    if (cc < cb_hi) {
                        fetch(cc, rb[half]);
                        const int s = cc * 16 / Fc;
                        const int c = cc * 16 - s * Fc + l16;
                        const float mk = mg[((size_t)s * Fc + c) * mstr];
                        f32x4 acc[NEB];
#pragma unroll
                        for (int eb = 0; eb < NEB; ++eb) acc[eb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                        // the weights in four groups of four K-steps, the
                        // next group read from LDS while this one multiplies
                        float wv[2][4][NEB];
                        auto ldw = [&](int grp, float (*w)[NEB]) {
#pragma unroll
                            for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                                for (int eb = 0; eb < NEB; ++eb) w[k4][eb] = s_w[16 * eb + l16][4 * (4 * grp + k4) + j4];
                        };
                        ldw(0, wv[0]);
#pragma unroll
                        for (int grp = 0; grp < 4; ++grp) {
                            if (grp < 3) ldw(grp + 1, wv[(grp + 1) & 1]);
                            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                            for (int k4 = 0; k4 < 4; ++k4) {
                                const int kk = 4 * grp + k4;
                                const float bvl =
                                    ((pvalid >> kk) & 1u) ? sg_value<TGT>(up, rb[half][kk]) + mk : 0.0f;
#pragma unroll
                                for (int eb = 0; eb < NEB; ++eb)
                                    acc[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[grp & 1][k4][eb], bvl, acc[eb],
                                                                                   0, 0, 0);
                            }
                            __builtin_amdgcn_sched_barrier(0);
                        }
                        // lane holds entry 16 eb + 4 j4 + r, column c
                        float* dA = d_attr + s * da_stride + c;
#pragma unroll
                        for (int eb = 0; eb < NEB; ++eb)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int e = 16 * eb + 4 * j4 + r;
                                if (e < m && acc[eb][r] != 0.0f) unsafeAtomicAdd(dA + (size_t)s_g[e] * Fc, acc[eb][r]);
                            }
                    }
                }
            }
        };
        if (cb_hi > cb_lo) {
            switch (neb) {
                case 1: da_phase(std::integral_constant<int, 1>{}); break;
                case 2: da_phase(std::integral_constant<int, 2>{}); break;
                case 3: da_phase(std::integral_constant<int, 3>{}); break;
                default: da_phase(std::integral_constant<int, 4>{}); break;
            }
        }
        __syncthreads();
    }
}

// Folds the per-pair geometric sums into the per-Gaussian accumulators and
// clears the pair accumulator for the next call.
__global__ __launch_bounds__(256) void k_geo_fold(float* __restrict__ gacc, size_t s_gacc,
                                                  const uint32_t* __restrict__ plist, size_t s_plist,
                                                  const uint32_t* __restrict__ flags, size_t s_flags,
                                                  float* __restrict__ g2d, size_t s_g2d)
{
    const int q = blockIdx.y;
    const uint32_t P = flags[q * s_flags + FL_PUSED];
    gacc += q * s_gacc;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < P * 8u; e += gridDim.x * blockDim.x) {
        const float v = gacc[e];
        if (v != 0.0f) {
            gacc[e] = 0.0f;
            unsafeAtomicAdd(g2d + q * s_g2d + (size_t)plist[q * s_plist + e / 8] * 8 + (e & 7), v);
        }
    }
}

template <int CG>
static void bwd_cg(dim3 grid, dim3 block, hipStream_t s, const gs_attrs& a, const gs_params& p, const Layout& L,
                   char* ws, const float* out, const BwdUpstream& up, float* d_attr, int64_t da_stride, int C, int shared)
{
    hipLaunchKernelGGL(k_blend_bwd<CG>, grid, block, 0, s, (const GRec*)(ws + L.rec), L.s_rec / sizeof(GRec),
                       (const uint32_t*)(ws + L.plist), L.s_plist / 4, (const uint2*)(ws + L.ranges),
                       L.s_ranges / sizeof(uint2), a.data, a.query_stride, a.n_chan * C, C, L.H, L.W, L.tw, L.th,
                       L.TX, p.alpha_min, p.alpha_max, out, up.dout, up.target, up.mean_grad, up.scale,
                       (const uint32_t*)(ws + L.n_last), L.s_pix / 4,
                       (float*)(ws + L.gacc), L.s_gacc / 4, d_attr, da_stride, shared);
}

// k_blend_bwd_sg with g = scale (out - target) + mean_grad over the groups
// whose walk is longer than min_walk entries only; the squared error of
// their pixels is added to lacc[set]
void launch_blend_bwd_sg_long(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws,
                              const float* out, const float* target, const float* mean_grad, float scale,
                              const float* gscale, float* d_attr, int min_walk, float* lacc, hipStream_t s)
{
    int tw_log = 0;
    while ((1 << tw_log) < L.tw) ++tw_log;
    const SgUp sup{out, nullptr, target, mean_grad, scale, gscale};
    const int Fc = a.n_chan * (a.is_complex ? 2 : 1);
    auto kern = a.is_complex ? k_blend_bwd_sg<1, true> : k_blend_bwd_sg<0, true>;
    hipLaunchKernelGGL(kern, dim3(L.T, (L.tw * L.th) / SG_PIX), dim3(SG_WAVES * 64), 0, s, (const GRec*)(ws + L.rec),
                       (const uint32_t*)(ws + L.plist), (const uint2*)(ws + L.ranges), a.data, a.query_stride, n_sets,
                       Fc, L.H, L.W, tw_log, L.th, L.TX, p.alpha_min, p.alpha_max, sup,
                       (const uint32_t*)(ws + L.n_last), (float*)(ws + L.gacc), d_attr, a.query_stride, min_walk,
                       lacc);
}

void launch_geo_fold(const Layout& L, char* ws, hipStream_t s)
{
    const int64_t fb = (L.cap * 8 + 255) / 256;
    hipLaunchKernelGGL(k_geo_fold, dim3((unsigned)(fb < 2048 ? fb : 2048), L.nq), dim3(256), 0, s,
                       (float*)(ws + L.gacc), L.s_gacc / 4, (const uint32_t*)(ws + L.plist), L.s_plist / 4,
                       (const uint32_t*)(ws + L.flags), L.s_flags / 4, (float*)(ws + L.g2d), L.s_g2d / 4);
}

gs_status launch_blend_bwd(const gs_attrs& a, const gs_params& p, const Layout& L, int n_sets, char* ws,
                           const float* out, const BwdUpstream& up, float* d_attr, hipStream_t s)
{
    const int C = a.is_complex ? 2 : 1;
    const int Fc = a.n_chan * C;
    // (32-bit element offsets inside one set's spectrum)
    const bool offs32 = (uint64_t)Fc * L.H * L.W < (1ull << 30);
    if (L.nq == 1 && Fc % 16 == 0 && offs32 && !(p.options & GS_OPT_BWD_PER_GROUP)) {
        // one geometry for every set: the factorised backward
        int tw_log = 0;
        while ((1 << tw_log) < L.tw) ++tw_log;
        const SgUp sup{out, up.dout, up.target, up.mean_grad, up.scale, nullptr};
        const dim3 grid(L.T, (L.tw * L.th) / SG_PIX), block(SG_WAVES * 64);
        void* tok;
        timing_begin(TK_BLEND_BWD, s, &tok);
        auto kern = C == 2 ? (up.target ? k_blend_bwd_sg<1, true> : k_blend_bwd_sg<1, false>)
                           : (up.target ? k_blend_bwd_sg<0, true> : k_blend_bwd_sg<0, false>);
        hipLaunchKernelGGL(kern, grid, block, 0, s, (const GRec*)(ws + L.rec), (const uint32_t*)(ws + L.plist),
                           (const uint2*)(ws + L.ranges), a.data, a.query_stride, n_sets, Fc, L.H, L.W, tw_log,
                           L.th, L.TX, p.alpha_min, p.alpha_max, sup, (const uint32_t*)(ws + L.n_last),
                           (float*)(ws + L.gacc), d_attr, a.query_stride, 0, (float*)nullptr);
        timing_end(tok, s);
    } else {
    int cg = choose_chan_group(Fc, p.chan_group);
    if (cg > 32) cg = 32;
    if (Fc / cg > 65535) return GS_ERR_CAPACITY;
    const int shared = (L.nq == 1 && n_sets > 1) ? 1 : 0;
    dim3 grid(L.T, Fc / cg, n_sets), block(L.tw * L.th);
    const int64_t das = a.query_stride;  // d_attr mirrors the attribute layout
    void* tok;
    timing_begin(TK_BLEND_BWD, s, &tok);
    switch (cg) {
        case 1: bwd_cg<1>(grid, block, s, a, p, L, ws, out, up, d_attr, das, C, shared); break;
        case 2: bwd_cg<2>(grid, block, s, a, p, L, ws, out, up, d_attr, das, C, shared); break;
        case 4: bwd_cg<4>(grid, block, s, a, p, L, ws, out, up, d_attr, das, C, shared); break;
        case 8: bwd_cg<8>(grid, block, s, a, p, L, ws, out, up, d_attr, das, C, shared); break;
        case 16: bwd_cg<16>(grid, block, s, a, p, L, ws, out, up, d_attr, das, C, shared); break;
        default: bwd_cg<32>(grid, block, s, a, p, L, ws, out, up, d_attr, das, C, shared); break;
    }
    timing_end(tok, s);
    }
    const int64_t fb = (L.cap * 8 + 255) / 256;
    hipLaunchKernelGGL(k_geo_fold, dim3((unsigned)(fb < 2048 ? fb : 2048), L.nq), dim3(256), 0, s,
                       (float*)(ws + L.gacc), L.s_gacc / 4, (const uint32_t*)(ws + L.plist), L.s_plist / 4,
                       (const uint32_t*)(ws + L.flags), L.s_flags / 4, (float*)(ws + L.g2d), L.s_g2d / 4);
    return GS_OK;
}

}  // namespace gs
