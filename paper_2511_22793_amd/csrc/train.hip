// One fused training pass over attribute sets that share one geometry (a
// fixed receiver, S transmitters whose effect is in the attributes):
// compositing (Eq. (3)), the training loss (the Eq. (2) spatial mean with
// the Eq. (4) channel term, and the pixel term) and the compositing backward,
// without writing the spectra or their gradient to memory.
//
// Per pixel p the weight of list entry k, w_k(p) = T_k alpha_k a_k, and the
// walk's decisions do not depend on the set, so for every column c = (set,
// channel, re/im):
//   zhat(p, c)  = sum_k w_k(p) v(k, c)                 (forward, Eq. (3))
//   g(p, c)     = e (zhat - z)(p, c) + m(c)            (dL/dzhat)
//   GV_k(p)     = sum_c v(k, c) g(p, c)                (geometric backward)
//   dL/dv(k, c) = sum_p w_k(p) g(p, c)                 (attribute gradient)
// with e = 2 / (F H W S) and m(c) = lambda 2 (hhat - h)(c) / (H W S).  m needs
// the spatial mean hhat before any pixel is formed: by linearity,
// hhat(c) = (1/HW) sum_g Wtot_g v(g, c) with Wtot_g = sum_p w_g(p), which the
// live pass accumulates per Gaussian; h, the target's channel (Eq. (2) of the
// target spectrum), is an input.
//
// Work units: (64-pixel group of a tile, column range).  A unit evaluates
// alpha for every (entry, pixel) of the group's walk (all four waves), forms
// the prefix transmittance and the weights (one wave), then walks its column
// range in rounds of four 16-column blocks, one per wave:
//   (F) zhat on the FP32 matrix cores (the product of k_blend_sg, same
//       operands and K order, so an optional spectrum store is bit-identical
//       to the compositing kernel's), the target read, g, the loss partial;
//   (D) dL/dv over the group's 64 pixels from g in registers, one atomic per
//       (entry, column) of the unit;
//   (G) g of all four blocks goes through LDS so that each wave adds GV for
//       its 16 pixels over the round's 64 columns.
// Each unit adds its GV (its columns' share) into the group's accumulator; a
// second kernel walks the backward recurrence per group (Eq. (3)
// differentiated): the running prefix P_k = sum_{m<=k} w_m GV_m, dL/dalpha_k
// = T_k a_k GV_k - (D - P_k) / (1 - alpha_k) with D = P_last, and the seven
// geometric terms of each entry reduced over the group's pixels.
// Both kernels come in variants for walks of at most 64, 128 and 256 list
// entries (the weights of the whole walk stay in LDS, so the wider variants
// hold fewer workgroups per CU); a group takes the smallest that holds its
// walk.  A classification kernel sorts the groups into those three classes
// (and clears their GV rows); each variant then runs as a persistent grid of
// the workgroups that fit the chip at once, taking units from its class's
// list through an atomic counter.  The column split R of a class is chosen
// on the device from its group count: enough units to fill that grid, so a
// class of a few long walks is spread over many CUs instead of running as a
// few long units.  Walks grow as training makes Gaussians fainter.  Groups
// whose walk is longer than 256 entries are left to the unfused kernels
// (compositing, then the backward forming g from the stored spectrum and the
// target).
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "common.h"

namespace gs {

constexpr double LOG2E_T = 1.4426950408889634;
constexpr int TR_PIX = 64;     // pixels per group
constexpr int TR_WAVES = 4;
constexpr int TR_PAD = 68;     // padded LDS row (pixels)
constexpr int TR_CH = 64;      // entries per alpha chunk
constexpr int TR_EMAX = 256;   // longest group walk the fused kernels take

typedef float f32x4t __attribute__((ext_vector_type(4)));

// pixel k (0 <= k < vw*vh, row-major inside the tile's in-image part) of
// tile (txi, tyi) as an image offset, or -1
__device__ __forceinline__ int tr_pixel(int k, int vw, int vh, int txi, int tyi, int tw, int th, int W)
{
    return k < vw * vh ? (tyi * th + k / vw) * W + txi * tw + k % vw : -1;
}

// The group's pixels, stop positions (the live pass's) and the records of
// the entries its walk reaches, for walks of at most E entries.
template <int E>
struct TrLds {
    double px[E], py[E], ca[E], cb[E], cc[E];
    float sig[E], att[E];
    uint32_t g[E];
    uint32_t voff[E];      // float offset of the entry's attribute row (g Fc; entry 0's row past the walk)
    uint32_t nzb[E / 16];  // per block of 16 entries: bit b set if one of them weighs at a pixel of block b
    int pix[TR_PIX];
    uint32_t maxstop;
};

// Shared start of both kernels: returns the walk length m of the group when
// lo < m <= E (lo = 0: 0 <= m <= E), else -1 (another variant, or the
// unfused kernels beyond TR_EMAX, takes the group).
template <int E>
__device__ __forceinline__ int tr_group(TrLds<E>& L, const GRec* __restrict__ rec,
                                        const uint32_t* __restrict__ plist, uint2 rg,
                                        const uint32_t* __restrict__ n_last, int pg, int vw, int vh, int txi, int tyi,
                                        int tw, int th, int W, int lo, uint32_t& stop)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) L.maxstop = 0;
    if (threadIdx.x < TR_PIX) L.pix[threadIdx.x] = tr_pixel(pg * TR_PIX + threadIdx.x, vw, vh, txi, tyi, tw, th, W);
    __syncthreads();
    const int mypix = L.pix[lane];
    stop = mypix >= 0 ? n_last[mypix] : 0u;
    if (wave == 0 && stop) atomicMax(&L.maxstop, stop);
    __syncthreads();
    const uint32_t ms = L.maxstop;
    if (ms > (uint32_t)E || (lo > 0 && ms <= (uint32_t)lo)) return -1;
    const int m = (int)ms;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const uint32_t g = plist[rg.x + t];
        const GRec r = rec[g];
        L.px[t] = r.px;
        L.py[t] = r.py;
        L.ca[t] = r.ca;
        L.cb[t] = r.cb;
        L.cc[t] = r.cc;
        L.sig[t] = r.sigma;
        L.att[t] = r.att;
        L.g[t] = g;
    }
    __syncthreads();
    return m;
}

// alpha of entries k0 .. k0 + 63 at the lane's pixel, with the walk's
// decisions applied (0 where the pixel does not take the entry, and beyond
// the walk), into rows row0 + (k - k0) of s_a; all four waves, no barrier
template <int E>
__device__ __forceinline__ void tr_alpha(const TrLds<E>& L, float (*s_a)[TR_PAD], int row0, int k0, int m,
                                         uint32_t stop, int W, float amin, float amax)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mypix = L.pix[lane];
    const double pcx = (mypix >= 0 ? mypix % W : 0) + 0.5, pcy = (mypix >= 0 ? mypix / W : 0) + 0.5;
    const double halfW = 0.5 * W;
    for (int kk = wave; kk < TR_CH; kk += TR_WAVES) {
        const int k = k0 + kk;
        float a = 0.0f;
        if (k < m && (uint32_t)k < stop) {
            double dx = pcx - L.px[k];
            dx += dx >= halfW ? -(double)W : (dx < -halfW ? (double)W : 0.0);
            const double dy = pcy - L.py[k];
            const double qv = L.ca[k] * dx * dx + 2.0 * L.cb[k] * dx * dy + L.cc[k] * dy * dy;
            const float G = __builtin_amdgcn_exp2f((float)(-0.5 * LOG2E_T * qv));
            const float alpha = fminf(amax, L.sig[k] * G);
            a = alpha >= amin ? alpha : 0.0f;
        }
        s_a[row0 + kk][lane] = a;
    }
}

// Raw buffer resource over `base` (32-bit byte offsets from it; no range
// check): per-lane offsets then need one 32-bit add instead of 64-bit
// address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tr_rsrc(const void* base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7FFFFFFF, 0x00020000);
}

// One float at byte offset `off` of the buffer; offsets at or past 2^31 - 1
// (beyond the resource's range) read 0.0f without touching memory.
constexpr uint32_t TR_OOB = 0x80000000u;
__device__ __forceinline__ float tr_ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// ---------------------------------------------------------------------------
// Kernel 1: forward products, loss partial, attribute gradient, GV partials.
// ---------------------------------------------------------------------------
struct TrArgs {
    const GRec* rec;
    const uint32_t* plist;
    const uint2* ranges;
    const uint32_t* n_last;
    const float* attr;
    int64_t a_stride;
    const float* tgt;
    const float* mgrad;  // m [S][Fc]
    float escale;        // e
    float* out;          // spectrum, or null
    float* d_attr;
    int64_t da_stride;
    float* gv;           // GV accumulators [group][TR_EMAX][TR_PIX] (rows of the walk cleared by the classification)
    double* lacc;        // squared-error sums [S]
    uint32_t* cls;       // group lists of the three walk classes [3][groups]
    uint32_t* ctr;       // class sizes, then the work counters of both kernels
    float* gacc;         // per-pair geometric accumulators [pairs][8]
    const float* gscale; // device scale c of every gradient, or null
    int S, Fc, H, W, tw, th, TX, gpt, groups;
    int rmin, rmax;      // bounds of a class's column split
    float amin, amax;
};

// counters: class sizes at TR_CNT + c, units taken by the forward/backward
// products at TR_WK_FB + c, groups taken by the backward walk at TR_WK_WALK + c
constexpr int TR_CNT = 0, TR_WK_FB = 4, TR_WK_WALK = 8, TR_NCTR = 16;

// shortest walk of class c (exclusive; class 0 takes empty walks too)
__device__ __forceinline__ int tr_lo(int c) { return c == 0 ? 0 : (c == 1 ? 64 : 128); }

// Column split of a class of `cnt` groups over a persistent grid of `slots`
// workgroups: enough units to fill the grid, within [rmin, rmax].
__device__ __forceinline__ int tr_split(const TrArgs& A, uint32_t cnt, int slots)
{
    const int r = cnt ? (int)((slots + cnt - 1) / cnt) : A.rmin;
    return min(A.rmax, max(A.rmin, r));
}

// One wave per group: its walk length (the largest stop position of its
// pixels), its class, and the GV rows of its walk cleared for the products'
// atomics.  Groups of no class (walks past TR_EMAX) are left alone.
__global__ __launch_bounds__(64) void k_train_classify(TrArgs A)
{
    const int grp = blockIdx.x;
    const int tile = grp / A.gpt, pg = grp % A.gpt;
    const int lane = threadIdx.x;
    const int txi = tile % A.TX, tyi = tile / A.TX;
    const int vw = min(A.tw, A.W - txi * A.tw), vh = min(A.th, A.H - tyi * A.th);
    if (pg * TR_PIX >= vw * vh) return;
    const int px = tr_pixel(pg * TR_PIX + lane, vw, vh, txi, tyi, A.tw, A.th, A.W);
    int m = px >= 0 ? (int)A.n_last[px] : 0;
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if (m > TR_EMAX) return;
    const int c = m <= 64 ? 0 : (m <= 128 ? 1 : 2);
    float4* gv = (float4*)(A.gv + (size_t)grp * TR_EMAX * TR_PIX);
    for (int i = lane; i < m * (TR_PIX / 4); i += 64) gv[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (lane == 0) A.cls[c * A.groups + atomicAdd(A.ctr + TR_CNT + c, 1u)] = (uint32_t)grp;
}

// occupancy per variant: the LDS of E = 64 fits four workgroups per CU, of
// 128 two, of 256 one
template <int E>
struct TrOcc {
    static constexpr int waves = E <= 64 ? 4 : (E <= 128 ? 2 : 1);
    // rows of s_a: the round's V block goes through it for walks of up to
    // 128 entries (E = 128 keeps two workgroups per CU with it; E = 256
    // would not fit, so it reads the other waves' columns from memory)
    static constexpr int sa_rows = E <= 128 ? E : TR_CH;
};

// One unit (group grp, column range r of R) of kernel 1.  Returns early only
// for the whole workgroup.
template <int E>
__device__ __forceinline__ void tr_fb_unit(const TrArgs& A, TrLds<E>& L, float (*s_a)[TR_PAD], float (*s_w)[TR_PAD],
                                           int grp, int r, int R, int lo)
{
    const int tile = grp / A.gpt, pg = grp % A.gpt;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j4 = lane >> 4, l16 = lane & 15;
    const int txi = tile % A.TX, tyi = tile / A.TX;
    const int vw = min(A.tw, A.W - txi * A.tw), vh = min(A.th, A.H - tyi * A.th);
    if (pg * TR_PIX >= vw * vh) return;
    const uint2 rg = A.ranges[tile];
    const size_t HW = (size_t)A.H * A.W;
    const int F = A.Fc >> 1;
    const int ncb = A.S * A.Fc / 16;
    const int cb_lo = r * ncb / R, cb_hi = (r + 1) * ncb / R;
    // e, times the gradient scale c when one is given (the mean term m
    // carries c already)
    const float escale = A.gscale ? A.escale * *A.gscale : A.escale;
    uint32_t stop;
    const int m = tr_group<E>(L, A.rec, A.plist, rg, A.n_last, pg, vw, vh, txi, tyi, A.tw, A.th, A.W, lo, stop);
    if (m < 0) return;
    const int nks = (m + 3) >> 2;  // K-steps of 4 entries
    const int mp = nks * 4;
    const int neb = (m + 15) >> 4;
    for (int t = threadIdx.x; t < 16 * neb; t += blockDim.x) L.voff[t] = (t < m ? L.g[t] : L.g[0]) * (uint32_t)A.Fc;
    __syncthreads();

    // The (F) products take the group's pixels in an interleaved order:
    // row m of output block pb is pixel 4 m + pb, so that a lane's four A
    // operands of one K-step (one entry, pixels 4 l16 .. 4 l16 + 3) are one
    // 16-byte LDS read.  A lane then holds rows 4 j4 + i of each block, i.e.
    // pixel 16 j4 + 4 i + pb (read from LDS where used).
    auto pixY = [&](int pb, int i) -> int { return L.pix[16 * j4 + 4 * i + pb]; };
    const int nrounds = (cb_hi - cb_lo + TR_WAVES - 1) / TR_WAVES;
    // Memory operations complete in issue order for the wait counter, so a
    // wait for a load also waits for every atomic issued before it.  A round
    // therefore issues the next round's (F) operands (first chain) and target
    // words before its own attribute-gradient atomics: the next round's first
    // wait leaves those atomics in flight.
    constexpr int KCH = (E < 128 ? E : 128) / 4;  // K-steps of one chain
    float bq[KCH];   // V words of the next chain
    float tcur[16];  // target words of this wave's block
    auto round_load = [&](int rd_) {
        const int cb_ = cb_lo + rd_ * TR_WAVES + wave;
        if (rd_ >= nrounds || cb_ >= cb_hi) return;
        const int s_ = cb_ * 16 / A.Fc;
        const int c_ = cb_ * 16 - s_ * A.Fc;
        const __amdgpu_buffer_rsrc_t rv_ = tr_rsrc(A.attr + s_ * A.a_stride);
#pragma unroll
        for (int q = 0; q < KCH; ++q)
            if (q < nks) bq[q] = tr_ld(rv_, (L.voff[4 * q + j4] + (uint32_t)(c_ + l16)) * 4u);
        const __amdgpu_buffer_rsrc_t rt = tr_rsrc(A.tgt + (size_t)s_ * F * HW * 2);
        const int cl = c_ + l16;
        const uint32_t plane = (uint32_t)((cl >> 1) * HW * 2 + (cl & 1));
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int px = pixY(pb, i);
                tcur[4 * pb + i] = tr_ld(rt, px >= 0 ? (plane + 2u * px) * 4u : TR_OOB);
            }
    };
    // the first round's loads fly during the weights' walk
    round_load(0);

    // prefix transmittance and weights chunk by chunk: alpha by all waves,
    // the walk by one (lane = pixel, in list order: the operations of the
    // compositing kernel); the walk also marks which (entries, 16-pixel
    // block) tiles of the weights hold a nonzero value: the products skip
    // the others (their terms are exact zeros)
    float T = 1.0f;
    for (int k0 = 0; k0 < mp; k0 += TR_CH) {
        tr_alpha<E>(L, s_a, 0, k0, m, stop, A.W, A.amin, A.amax);
        __syncthreads();
        if (wave == 0) {
            const int kn = min(TR_CH, mp - k0);
            unsigned long long nz = 0ull;
            for (int kk = 0; kk < kn; ++kk) {
                const float a = s_a[kk][lane];
                const float w = a > 0.0f ? T * a * L.att[k0 + kk] : 0.0f;
                T = a > 0.0f ? T * (1.0f - a) : T;
                s_w[k0 + kk][lane] = w;
                nz |= __ballot(w != 0.0f);
                const int k = k0 + kk;
                if ((k & 15) == 15 || k == mp - 1) {
                    if (lane == 0)
                        L.nzb[k >> 4] = ((nz & 0xFFFFull) ? 1u : 0u) | ((nz & 0xFFFF0000ull) ? 2u : 0u) |
                                        ((nz & 0xFFFF00000000ull) ? 4u : 0u) | ((nz >> 48) ? 8u : 0u);
                    nz = 0ull;
                }
            }
        }
        __syncthreads();
    }

    constexpr int NEB = E / 16;
    f32x4t gv[NEB];  // GV[16 eb + 4 j4 + i][16 wave + l16], over this unit's columns
#pragma unroll
    for (int eb = 0; eb < NEB; ++eb) gv[eb] = f32x4t{0.0f, 0.0f, 0.0f, 0.0f};
    float lsum = 0.0f;
    int lset = -1;

    for (int rd = 0; rd < nrounds; ++rd) {
        const int cb = cb_lo + rd * TR_WAVES + wave;
        const bool own = cb < cb_hi;
        const int s = own ? cb * 16 / A.Fc : 0;
        const int c0 = own ? cb * 16 - s * A.Fc : 0;
        f32x4t z[4];  // zhat, then g: [pixel 16 j4 + 4 i + pb][column c0 + l16]
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) z[pb] = f32x4t{0.0f, 0.0f, 0.0f, 0.0f};
        if (own) {
            // (F) zhat = W^T V, in chains of 128 entries added in list order
            // (the compositing kernel's buffer flushes, so that the stored
            // spectrum is bit-identical to it); the first chain's V words
            // were loaded with the previous round
            const __amdgpu_buffer_rsrc_t rv = tr_rsrc(A.attr + s * A.a_stride);
            for (int kc = 0; kc < nks; kc += KCH) {
                if (kc > 0) {
#pragma unroll
                    for (int q = 0; q < KCH; ++q)
                        if (kc + q < nks) bq[q] = tr_ld(rv, (L.voff[4 * (kc + q) + j4] + (uint32_t)(c0 + l16)) * 4u);
                }
                f32x4t zc[4];
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) zc[pb] = f32x4t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int q = 0; q < KCH; ++q) {
                    if (kc + q < nks) {
                        const int ks = kc + q;
                        const float4 wa = *(const float4*)&s_w[4 * ks + j4][4 * l16];
                        zc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.x, bq[q], zc[0], 0, 0, 0);
                        zc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.y, bq[q], zc[1], 0, 0, 0);
                        zc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.z, bq[q], zc[2], 0, 0, 0);
                        zc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.w, bq[q], zc[3], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) z[pb] = kc == 0 ? zc[pb] : zc[pb] + z[pb];
            }
            // target, g, loss partial (column c0 + l16 = channel f, re/im)
            const int c = c0 + l16;
            const float mc = A.mgrad[(size_t)s * A.Fc + c];
            if (A.out) {
                // the spectrum, on request (one set's spectrum: 32-bit offsets)
                const __amdgpu_buffer_rsrc_t ro = tr_rsrc(A.out + (size_t)s * F * HW * 2);
                const uint32_t plane = (uint32_t)((c >> 1) * HW * 2 + (c & 1));
#pragma unroll
                for (int pb = 0; pb < 4; ++pb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int px = pixY(pb, i);
                        const float zv = z[pb][i];
                        if (px >= 0)
                            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(zv), ro, (plane + 2u * px) * 4u, 0,
                                                                  0);
                    }
            }
            float ls = 0.0f;
#pragma unroll
            for (int pb = 0; pb < 4; ++pb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int px = pixY(pb, i);
                    if (px >= 0) {
                        const float d = z[pb][i] - tcur[4 * pb + i];
                        ls = fmaf(d, d, ls);
                        z[pb][i] = fmaf(escale, d, mc);
                    } else {
                        z[pb][i] = 0.0f;
                    }
                }
            if (s != lset) {
                if (lset >= 0) {
                    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
                    if (lane == 0) unsafeAtomicAdd(A.lacc + lset, (double)lsum);
                }
                lset = s;
                lsum = 0.0f;
            }
            lsum += ls;
            // g to LDS for (G): s_a[16 wave + j][p] = g(p, c0 + j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float g0 = z[0][i], g1 = z[1][i], g2 = z[2][i], g3 = z[3][i];
                *(float4*)&s_a[16 * wave + l16][16 * j4 + 4 * i] = float4{g0, g1, g2, g3};
            }
        }
        __syncthreads();
        // (G) GV[k][16 wave + l16] += sum over the round's columns of v(k, c) g(p, c)
        if constexpr (E <= 128) {
            // The round's V block is the four waves' (F) operands: it goes
            // through s_a too (after each wave has taken its g words), so
            // that no wave reads the other waves' columns from memory.
            const int nown = min(TR_WAVES, cb_hi - (cb_lo + rd * TR_WAVES));
            float bg[TR_WAVES][4];
#pragma unroll
            for (int ow = 0; ow < TR_WAVES; ++ow)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) bg[ow][kk] = s_a[16 * ow + 4 * j4 + kk][16 * wave + l16];
            __syncthreads();
            // s_a[k][16 ow + j] = v(k, column j of owner ow's block)
            if (own) {
#pragma unroll
                for (int q = 0; q < KCH; ++q)
                    if (q < nks) s_a[4 * q + j4][16 * wave + l16] = bq[q];
            }
            __syncthreads();
#pragma unroll
            for (int eb = 0; eb < NEB; ++eb) {
                if (eb < neb && (__builtin_amdgcn_readfirstlane(L.nzb[eb]) & (1u << wave))) {
#pragma unroll
                    for (int ow = 0; ow < TR_WAVES; ++ow) {
                        if (ow < nown) {
                            const float4 v4 = *(const float4*)&s_a[16 * eb + l16][16 * ow + 4 * j4];
                            gv[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(v4.x, bg[ow][0], gv[eb], 0, 0, 0);
                            gv[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(v4.y, bg[ow][1], gv[eb], 0, 0, 0);
                            gv[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(v4.z, bg[ow][2], gv[eb], 0, 0, 0);
                            gv[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(v4.w, bg[ow][3], gv[eb], 0, 0, 0);
                        }
                    }
                }
            }
        } else {
#pragma unroll 1
        for (int ow = 0; ow < TR_WAVES; ++ow) {
            const int ocb = cb_lo + rd * TR_WAVES + ow;
            if (ocb >= cb_hi) break;
            const int os = ocb * 16 / A.Fc;
            const int oc0 = ocb * 16 - os * A.Fc;
            const __amdgpu_buffer_rsrc_t rv = tr_rsrc(A.attr + os * A.a_stride);
            float bg[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) bg[kk] = s_a[16 * ow + 4 * j4 + kk][16 * wave + l16];
#pragma unroll
            for (int eb = 0; eb < NEB; ++eb) {
                if (eb < neb && (__builtin_amdgcn_readfirstlane(L.nzb[eb]) & (1u << wave))) {
                    const float4 v4 = __builtin_bit_cast(
                        float4, __builtin_amdgcn_raw_buffer_load_b128(
                                    rv, (L.voff[16 * eb + l16] + (uint32_t)(oc0 + 4 * j4)) * 4u, 0, 0));
                    __builtin_amdgcn_sched_barrier(0);
                    gv[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(v4.x, bg[0], gv[eb], 0, 0, 0);
                    gv[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(v4.y, bg[1], gv[eb], 0, 0, 0);
                    gv[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(v4.z, bg[2], gv[eb], 0, 0, 0);
                    gv[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(v4.w, bg[3], gv[eb], 0, 0, 0);
                }
            }
        }
        }
        // (D) dL/dv[k][c0 + l16] = sum_p w_k(p) g(p, c0 + l16): K-step (i, pb)
        // pairs lane group j4 with pixel 16 j4 + 4 i + pb; all entry blocks'
        // sums first, then the next round's loads, then the atomics
        f32x4t acc[NEB];
#pragma unroll
        for (int eb = 0; eb < NEB; ++eb) {
            acc[eb] = f32x4t{0.0f, 0.0f, 0.0f, 0.0f};
            if (own && eb < neb && __builtin_amdgcn_readfirstlane(L.nzb[eb])) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float4 w4 = *(const float4*)&s_w[16 * eb + l16][16 * j4 + 4 * i];
                    acc[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4.x, z[0][i], acc[eb], 0, 0, 0);
                    acc[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4.y, z[1][i], acc[eb], 0, 0, 0);
                    acc[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4.z, z[2][i], acc[eb], 0, 0, 0);
                    acc[eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4.w, z[3][i], acc[eb], 0, 0, 0);
                }
            }
        }
        round_load(rd + 1);
        if (own) {
            const __amdgpu_buffer_rsrc_t rd_attr = tr_rsrc(A.d_attr + s * A.da_stride);
#pragma unroll
            for (int eb = 0; eb < NEB; ++eb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = 16 * eb + 4 * j4 + i;
                    if (k < m && acc[eb][i] != 0.0f)
                        __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(
                            acc[eb][i], rd_attr, (L.voff[k] + (uint32_t)(c0 + l16)) * 4u, 0, 0);
                }
        }
        __syncthreads();  // before the next round's g overwrites s_a
    }
    if (lset >= 0) {
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
        if (lane == 0) unsafeAtomicAdd(A.lacc + lset, (double)lsum);
    }
    // this column range's share of GV: lane holds entries 16 eb + 4 j4 + i at
    // pixel 16 wave + l16
    // (byte offset: the entry block in the scalar offset, the entry inside
    // it as an immediate, one per-lane register)
    const __amdgpu_buffer_rsrc_t rg_gv = tr_rsrc(A.gv + (size_t)grp * TR_EMAX * TR_PIX);
    const uint32_t lane_off = (uint32_t)(4 * j4 * TR_PIX + 16 * wave + l16) * 4u;
#pragma unroll
    for (int eb = 0; eb < NEB; ++eb)
        if (eb < neb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = 16 * eb + 4 * j4 + i;
                if (k < m && gv[eb][i] != 0.0f)
                    __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(gv[eb][i], rg_gv, lane_off + i * TR_PIX * 4,
                                                                    eb * 16 * TR_PIX * 4, 0);
            }
}

// Kernel 1 as a persistent grid over the units of walk class c.
template <int E>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TrOcc<E>::waves))) void k_train_fb(TrArgs A,
                                                                                                      int c)
{
    __shared__ TrLds<E> L;
    // alpha of a chunk, then the exchange of g, then (E <= 128) the round's V block
    __shared__ __align__(16) float s_a[TrOcc<E>::sa_rows][TR_PAD];
    __shared__ __align__(16) float s_w[E][TR_PAD];      // weights w_k(p)
    __shared__ uint32_t s_item;
    const uint32_t cnt = A.ctr[TR_CNT + c];
    const int R = tr_split(A, cnt, (int)gridDim.x);
    const uint32_t total = cnt * (uint32_t)R;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.ctr + TR_WK_FB + c, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        tr_fb_unit<E>(A, L, s_a, s_w, (int)A.cls[c * A.groups + item / R], (int)(item % R), R, tr_lo(c));
        __syncthreads();  // the next unit reuses the LDS
    }
}

// ---------------------------------------------------------------------------
// Kernel 2: per group, GV summed over the column ranges, the backward walk
// and the geometric terms of each entry reduced over the group's pixels into
// the per-pair accumulators (folded per Gaussian afterwards).
// ---------------------------------------------------------------------------

// reduce-scatter of 8 values over the wave: lane l ends with the wave total
// of value l >> 3 (permlane swaps, then DPP; as in the compositing backward)
__device__ __forceinline__ float tr_dpp(float v, int sel)
{
    const int iv = __float_as_int(v);
    int rr;
    switch (sel) {
        case 0: rr = __builtin_amdgcn_update_dpp(0, iv, 0x128, 0xF, 0xF, true); break;  // row_ror:8
        case 1: rr = __builtin_amdgcn_update_dpp(0, iv, 0xB1, 0xF, 0xF, true); break;   // quad_perm [1,0,3,2]
        case 2: rr = __builtin_amdgcn_update_dpp(0, iv, 0x4E, 0xF, 0xF, true); break;   // quad_perm [2,3,0,1]
        default: rr = __builtin_amdgcn_update_dpp(0, iv, 0x141, 0xF, 0xF, true); break; // row_half_mirror
    }
    return __int_as_float(rr);
}

__device__ __forceinline__ void tr_reduce_scatter8(float* x, int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[i + 4]), false, false);
        x[i] = __uint_as_float(q[0]) + __uint_as_float(q[1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[i]), __float_as_uint(x[i + 2]), false, false);
        x[i] = __uint_as_float(q[0]) + __uint_as_float(q[1]);
    }
    const float t0 = x[0] + tr_dpp(x[0], 0), t1 = x[1] + tr_dpp(x[1], 0);
    float v = (lane & 8) ? t1 : t0;
    v += tr_dpp(v, 1);
    v += tr_dpp(v, 2);
    v += tr_dpp(v, 3);
    x[0] = v;
}

template <int E>
__device__ __forceinline__ void tr_walk_group(const TrArgs& A, TrLds<E>& L, float (*s_a)[TR_PAD],
                                              float (*s_gv)[TR_PAD], int grp, int lo)
{
    const int tile = grp / A.gpt, pg = grp % A.gpt;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int txi = tile % A.TX, tyi = tile / A.TX;
    const int vw = min(A.tw, A.W - txi * A.tw), vh = min(A.th, A.H - tyi * A.th);
    if (pg * TR_PIX >= vw * vh) return;
    const uint2 rg = A.ranges[tile];
    uint32_t stop;
    const int m = tr_group<E>(L, A.rec, A.plist, rg, A.n_last, pg, vw, vh, txi, tyi, A.tw, A.th, A.W, lo, stop);
    if (m <= 0) return;
    for (int k0 = 0; k0 < m; k0 += TR_CH) tr_alpha<E>(L, s_a, k0, k0, m, stop, A.W, A.amin, A.amax);
    const float4* gp = (const float4*)(A.gv + (size_t)grp * TR_EMAX * TR_PIX);
    for (int e = threadIdx.x; e < m * (TR_PIX / 4); e += blockDim.x)
        *(float4*)&s_gv[e / (TR_PIX / 4)][4 * (e % (TR_PIX / 4))] = gp[e];
    __syncthreads();
    if (wave == 0) {
        // D = sum_k w_k GV_k (the forward output contracted with g), then the
        // recurrence front to back
        float T = 1.0f, P = 0.0f;
        for (int k = 0; k < m; ++k) {
            const float a = s_a[k][lane];
            const float Ta = a > 0.0f ? T * a : 0.0f;
            P = P + Ta * (L.att[k] * s_gv[k][lane]);
            T = a > 0.0f ? T * (1.0f - a) : T;
        }
        const float D = P;
        T = 1.0f;
        P = 0.0f;
        for (int k = 0; k < m; ++k) {
            const float a = s_a[k][lane];
            const bool take = a > 0.0f;
            const float gvk = s_gv[k][lane];
            const float cA = L.att[k] * gvk;
            const float Ta = take ? T * a : 0.0f;
            const float Pn = P + Ta * cA;
            const float dalpha = T * cA - (D - Pn) * __builtin_amdgcn_rcpf(1.0f - a);
            s_a[k][lane] = (take && a < A.amax) ? dalpha : 0.0f;
            s_gv[k][lane] = Ta * gvk;
            T = take ? T * (1.0f - a) : T;
            P = Pn;
        }
    }
    __syncthreads();
    // geometric terms of entry k at this lane's pixel, reduced over the pixels
    const int mypix = L.pix[lane];
    const double pcx = (mypix >= 0 ? mypix % A.W : 0) + 0.5, pcy = (mypix >= 0 ? mypix / A.W : 0) + 0.5;
    const double halfW = 0.5 * A.W;
    for (int k = wave; k < m; k += TR_WAVES) {
        const float dsg = s_a[k][lane];
        const float tg = s_gv[k][lane];
        if (__ballot(dsg != 0.0f || tg != 0.0f) == 0ull) continue;
        double dx = pcx - L.px[k];
        dx += dx >= halfW ? -(double)A.W : (dx < -halfW ? (double)A.W : 0.0);
        const double dy = pcy - L.py[k];
        const double qv = L.ca[k] * dx * dx + 2.0 * L.cb[k] * dx * dy + L.cc[k] * dy * dy;
        const float G = __builtin_amdgcn_exp2f((float)(-0.5 * LOG2E_T * qv));
        const float dq = -0.5f * dsg * L.sig[k] * G;
        const float dxf = (float)dx, dyf = (float)dy;
        const float caf = (float)L.ca[k], cbf = (float)L.cb[k], ccf = (float)L.cc[k];
        const float dq2 = -2.0f * dq;
        float geo[8];
        geo[0] = dq2 * fmaf(caf, dxf, cbf * dyf);
        geo[1] = dq2 * fmaf(cbf, dxf, ccf * dyf);
        geo[2] = dq * (dxf * dxf);
        geo[3] = dq * (2.0f * dxf * dyf);
        geo[4] = dq * (dyf * dyf);
        geo[5] = dsg * G;
        geo[6] = tg;
        geo[7] = 0.0f;
        tr_reduce_scatter8(geo, lane);
        if ((lane & 7) == 0 && lane < 56 && geo[0] != 0.0f)
            unsafeAtomicAdd(A.gacc + (size_t)(rg.x + k) * 8 + (lane >> 3), geo[0]);
    }
}

// Kernel 2 as a persistent grid over the groups of walk class c.
template <int E>
__global__ __launch_bounds__(256) void k_train_walk(TrArgs A, int c)
{
    __shared__ TrLds<E> L;
    __shared__ __align__(16) float s_a[E][TR_PAD];   // alpha, then dL/d(sigma G)
    __shared__ __align__(16) float s_gv[E][TR_PAD];  // GV, then T alpha GV
    __shared__ uint32_t s_item;
    const uint32_t cnt = A.ctr[TR_CNT + c];
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.ctr + TR_WK_WALK + c, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= cnt) break;
        tr_walk_group<E>(A, L, s_a, s_gv, (int)A.cls[c * A.groups + item], tr_lo(c));
        __syncthreads();  // the next group reuses the LDS
    }
}

// ---------------------------------------------------------------------------
// hhat from the per-Gaussian weight totals, the channel-mean gradient term
// and the channel part of the loss.
// ---------------------------------------------------------------------------
// hs[s][c] += sum over live entries i = blockIdx.x + k gridDim.x of
// Wtot_g v(g, c): a fixed grid of TR_HSUM_BLOCKS per set whatever the live
// count (it is only known on the device), each thread a column, four
// entries' loads in flight at a time
constexpr int TR_HSUM_BLOCKS = 64;
__global__ __launch_bounds__(128) void k_train_hsum(const uint32_t* __restrict__ live, const uint32_t* __restrict__ count,
                                                    const float* __restrict__ wtot, const float* __restrict__ attr,
                                                    int64_t a_stride, int Fc, float* __restrict__ hs)
{
    const int s = blockIdx.y;
    const uint32_t nl = *count;
    if (blockIdx.x >= nl) return;
    const float* a = attr + s * a_stride;
    const uint32_t G = gridDim.x;
    for (int c = threadIdx.x; c < Fc; c += blockDim.x) {
        float acc = 0.0f;
        uint32_t i = blockIdx.x;
        for (; i + 3 * G < nl; i += 4 * G) {
            const uint32_t g0 = live[i], g1 = live[i + G], g2 = live[i + 2 * G], g3 = live[i + 3 * G];
            const float w0 = wtot[g0], w1 = wtot[g1], w2 = wtot[g2], w3 = wtot[g3];
            const float v0 = a[(size_t)g0 * Fc + c], v1 = a[(size_t)g1 * Fc + c];
            const float v2 = a[(size_t)g2 * Fc + c], v3 = a[(size_t)g3 * Fc + c];
            acc = fmaf(w0, v0, acc);
            acc = fmaf(w1, v1, acc);
            acc = fmaf(w2, v2, acc);
            acc = fmaf(w3, v3, acc);
        }
        for (; i < nl; i += G) {
            const uint32_t g = live[i];
            acc = fmaf(wtot[g], a[(size_t)g * Fc + c], acc);
        }
        unsafeAtomicAdd(&hs[(size_t)s * Fc + c], acc);
    }
}

// h_hat = hs / HW; m = c lambda 2 (h_hat - h) / (HW S) (c = the gradient
// scale, 1 without one); loss[s] = lambda sum_c (h_hat - h)^2 (the pixel
// term is added by k_train_loss_add)
__global__ __launch_bounds__(256) void k_train_hfinish(const float* __restrict__ hs, const float* __restrict__ h,
                                                       int S, int Fc, float inv_hw, float lambda,
                                                       const float* __restrict__ gscale,
                                                       float* __restrict__ h_hat, float* __restrict__ mgrad,
                                                       float* __restrict__ loss)
{
    const int s = blockIdx.x;
    const float cs = gscale ? *gscale : 1.0f;
    float part = 0.0f;
    for (int c = threadIdx.x; c < Fc; c += blockDim.x) {
        const size_t i = (size_t)s * Fc + c;
        const float hh = hs[i] * inv_hw;
        const float d = hh - h[i];
        h_hat[i] = hh;
        mgrad[i] = cs * (lambda * 2.0f * d * inv_hw / (float)S);
        part = fmaf(d, d, part);
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) loss[s] = lambda * (red[0] + red[1] + red[2] + red[3]);
}

// loss[s] += lscale * (squared-error sum of the fused kernels + that of the
// long-walk kernels)
__global__ __launch_bounds__(64) void k_train_loss_add(const double* __restrict__ lacc,
                                                       const float* __restrict__ llong, int S, float lscale,
                                                       float* __restrict__ loss)
{
    for (int s = threadIdx.x; s < S; s += blockDim.x)
        loss[s] += lscale * (float)(lacc[s] + (double)llong[s]);
}

// Eq. (2): h[s][c] = (1/HW) sum_p z(s, c, p); one workgroup per (set,
// channel), both components of a complex channel (summed in FP32 per thread,
// then over the workgroup; deterministic)
__global__ __launch_bounds__(256) void k_spatial_mean(const float* __restrict__ z, int Fc, int C, size_t HW,
                                                      float* __restrict__ h)
{
    const int s = blockIdx.y, f = blockIdx.x;
    const int F = Fc / C;
    const float* zb = z + ((size_t)s * F + f) * HW * C;
    float a0 = 0.0f, a1 = 0.0f;
    if (C == 2) {
        const float2* z2 = (const float2*)zb;
        for (size_t p = threadIdx.x; p < HW; p += blockDim.x) {
            const float2 v = z2[p];
            a0 += v.x;
            a1 += v.y;
        }
    } else {
        for (size_t p = threadIdx.x; p < HW; p += blockDim.x) a0 += zb[p];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
    }
    __shared__ float red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a0;
        red[1][threadIdx.x >> 6] = a1;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)C) {
        const float t = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        h[((size_t)s * F + f) * C + threadIdx.x] = t / (float)HW;
    }
}

// Scratch layout of gs_render_train (byte offsets from its start).
struct TrScratch {
    size_t gv, lacc, llong, hs, mg, cls, ctr, total;
};
TrScratch train_scratch(int groups, int S, int Fc)
{
    TrScratch t;
    t.gv = 0;
    t.lacc = t.gv + align256((size_t)groups * TR_EMAX * TR_PIX * 4);
    t.llong = t.lacc + align256((size_t)S * 8);
    t.hs = t.llong + align256((size_t)S * 4);
    t.mg = t.hs + align256((size_t)S * Fc * 4);
    t.cls = t.mg + align256((size_t)S * Fc * 4);
    t.ctr = t.cls + align256((size_t)3 * groups * 4);
    t.total = t.ctr + align256((size_t)TR_NCTR * 4);
    return t;
}

// Workgroups of each variant resident on the whole device at once (the
// persistent grids), per device.
struct TrSlots {
    int fb[3], walk[3];
};
hipError_t train_slots(TrSlots* out)
{
    static std::mutex mu;
    static int have[64] = {};
    static TrSlots cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!have[dev]) {
        int cus = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        const void* fb[3] = {(const void*)k_train_fb<64>, (const void*)k_train_fb<128>, (const void*)k_train_fb<256>};
        const void* wk[3] = {(const void*)k_train_walk<64>, (const void*)k_train_walk<128>,
                             (const void*)k_train_walk<256>};
        for (int c = 0; c < 3; ++c) {
            int a = 0, b = 0;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, fb[c], 256, 0)) != hipSuccess) return e;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, wk[c], 256, 0)) != hipSuccess) return e;
            cache[dev].fb[c] = std::max(1, a) * std::max(1, cus);
            cache[dev].walk[c] = std::max(1, b) * std::max(1, cus);
        }
        have[dev] = 1;
    }
    *out = cache[dev];
    return hipSuccess;
}

}  // namespace gs

using namespace gs;

extern "C" {

gs_status gs_spatial_mean(const float* spectrum, int32_t n_sets, int32_t n_chan, int32_t is_complex, int32_t H,
                          int32_t W, float* h, void* stream)
{
    if (!spectrum || !h || n_sets < 1 || n_chan < 1 || H < 1 || W < 1 || (is_complex != 0 && is_complex != 1))
        return GS_ERR_INVALID_ARG;
    if (n_chan > 65535 || n_sets > 65535) return GS_ERR_CAPACITY;
    const int C = is_complex ? 2 : 1;
    if (C == 2 && ((uintptr_t)spectrum & 7)) return GS_ERR_INVALID_ARG;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_spatial_mean, dim3(n_chan, n_sets), dim3(256), 0, (hipStream_t)stream, spectrum, n_chan * C,
                       C, (size_t)H * W, h);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status gs_render_train(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries, int32_t n_sets,
                          const gs_grid* grid, const gs_params* prm, const uint32_t* live_list,
                          const uint32_t* live_count, const gs_train_target* tt, float* spectrum, float* d_mean,
                          float* d_log_scale, float* d_quat, float* d_opacity_logit, float* d_attr, int32_t flags,
                          void* workspace, size_t ws_bytes, void* scratch, size_t scratch_bytes, void* stream)
{
    if (!tt || !tt->target || !tt->target_mean || !tt->loss || !tt->h_hat || !(tt->lambda_ch >= 0.0f) ||
        !live_list || !live_count || !d_mean || !d_log_scale || !d_quat || !d_opacity_logit || !d_attr)
        return GS_ERR_INVALID_ARG;
    if (flags & ~(GS_BWD_ATTR_GRAD_ZEROED | GS_TRAIN_WRITE_SPECTRUM | GS_TRAIN_DEFER_GEOMETRY))
        return GS_ERR_INVALID_ARG;
    Layout L;
    gs_status st = check_forward(scene, attrs, queries, grid, prm, spectrum, workspace, ws_bytes, &L);
    if (st != GS_OK) return st;
    if (prm->options & GS_OPT_FORWARD_ONLY) return GS_ERR_INVALID_ARG;
    // one prepared receiver shared by every set (attenuation to the receiver)
    if (queries->count != 1 || prm->atten_ref != 0 || n_sets < 1 || attrs->is_complex != 1) return GS_ERR_INVALID_ARG;
    const int Fc = attrs->n_chan * 2;
    if (Fc % 16 != 0) return GS_ERR_INVALID_ARG;
    // (one set's spectrum, target and attributes are addressed with 32-bit
    // byte offsets)
    if ((uint64_t)Fc * L.H * L.W >= (1ull << 29) || (uint64_t)scene->n * Fc >= (1ull << 29)) return GS_ERR_CAPACITY;
    if (n_sets > 1 && attrs->query_stride != 0 && attrs->query_stride < (int64_t)scene->n * Fc)
        return GS_ERR_INVALID_ARG;
    const int gpt = (L.tw * L.th) / TR_PIX;
    const int groups = L.T * gpt;
    const int ncb = n_sets * Fc / 16;
    if (groups > 0x7FFFFFFF / (TR_EMAX * TR_PIX) || (int64_t)groups * ncb > 0x7FFFFFFF) return GS_ERR_CAPACITY;
    const TrScratch ts = train_scratch(groups, n_sets, Fc);
    if (!scratch || ((uintptr_t)scratch & 255) || scratch_bytes < ts.total) return GS_ERR_WORKSPACE;
    TrSlots slots;
    if (train_slots(&slots) != hipSuccess) return GS_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    char* sc = (char*)scratch;
    (void)hipGetLastError();

    double* lacc = (double*)(sc + ts.lacc);
    float* llong = (float*)(sc + ts.llong);
    float* hs = (float*)(sc + ts.hs);
    float* mg = (float*)(sc + ts.mg);
    uint32_t* ctr = (uint32_t*)(sc + ts.ctr);
    const size_t HW = (size_t)L.H * L.W;
    const float escale = 2.0f / ((float)attrs->n_chan * (float)HW * (float)n_sets);
    const float lscale = 1.0f / ((float)attrs->n_chan * (float)HW);

    FillSegs fs{};
    fs.p[0] = (uint32_t*)lacc;  // lacc, llong, hs (adjacent)
    fs.count[0] = (ts.mg - ts.lacc) / 4;
    fs.p[1] = ctr;
    fs.count[1] = TR_NCTR;
    fs.p[2] = (uint32_t*)(ws + L.g2d);
    fs.count[2] = (size_t)L.n * 8;
    fs.n = 3;
    if (!(flags & GS_BWD_ATTR_GRAD_ZEROED)) {
        fs.p[3] = (uint32_t*)d_attr;
        fs.count[3] = (size_t)(attrs->query_stride ? n_sets : 1) * scene->n * Fc;
        fs.n = 4;
    }
    launch_fill_segs(fs, s);
    launch_fill_dev((uint32_t*)(ws + L.gacc), (size_t)L.cap * 8, L.s_gacc / 4, L.nq,
                    (const uint32_t*)(ws + L.flags) + FL_PUSED, L.s_flags / 4, 8u, s);
    // hhat, the mean term of g and the channel part of the loss
    hipLaunchKernelGGL(k_train_hsum, dim3(TR_HSUM_BLOCKS, n_sets), dim3(128), 0, s, live_list, live_count,
                       (const float*)(ws + L.wtot), attrs->data, attrs->query_stride, Fc, hs);
    hipLaunchKernelGGL(k_train_hfinish, dim3(n_sets), dim3(256), 0, s, hs, tt->target_mean, n_sets, Fc,
                       1.0f / (float)HW, tt->lambda_ch, tt->grad_scale, tt->h_hat, mg, tt->loss);

    TrArgs A{};
    A.rec = (const GRec*)(ws + L.rec);
    A.plist = (const uint32_t*)(ws + L.plist);
    A.ranges = (const uint2*)(ws + L.ranges);
    A.n_last = (const uint32_t*)(ws + L.n_last);
    A.attr = attrs->data;
    A.a_stride = attrs->query_stride;
    A.tgt = tt->target;
    A.mgrad = mg;
    A.escale = escale;
    A.out = (flags & GS_TRAIN_WRITE_SPECTRUM) ? spectrum : nullptr;
    A.d_attr = d_attr;
    A.da_stride = attrs->query_stride;
    A.gv = (float*)(sc + ts.gv);
    A.lacc = lacc;
    A.cls = (uint32_t*)(sc + ts.cls);
    A.ctr = ctr;
    A.gacc = (float*)(ws + L.gacc);
    A.gscale = tt->grad_scale;
    A.S = n_sets;
    A.Fc = Fc;
    A.H = L.H;
    A.W = L.W;
    A.tw = L.tw;
    A.th = L.th;
    A.TX = L.TX;
    A.gpt = gpt;
    A.groups = groups;
    // each wave owns a 16-column block per round: at least one round of
    // four blocks per unit, and at least four units per group where the
    // columns allow
    A.rmax = std::max(1, ncb / TR_WAVES);
    A.rmin = std::min(A.rmax, 4);
    A.amin = prm->alpha_min;
    A.amax = prm->alpha_max;
    void* tok;
    timing_begin(TK_TRAIN, s, &tok);
    // the groups sorted by walk length into the variants' lists, then each
    // variant over its list (the longest walks first)
    hipLaunchKernelGGL(k_train_classify, dim3(groups), dim3(64), 0, s, A);
    // The classes touch disjoint groups (their GV rows, work counters and
    // lists; the attribute gradients, loss partials and per-pair sums are
    // atomics), so the 256 and 128 classes run on side streams beside the
    // 64 class: their few long walks fill the 64 class's tail instead of
    // running alone.
    // Groups whose walk is longer than the fused kernels take go through
    // compositing into the spectrum, then the backward forming g from it and
    // the target (their own loss partial; attribute gradients and per-pair
    // sums are atomics): a third branch beside the classes.
    const Lanes* ln = side_lanes(s);
    if (ln) {
        std::lock_guard<std::mutex> lk(lanes_mutex());
        if (hipEventRecord(ln->fork, s) != hipSuccess) return GS_ERR_HIP;
        for (int i = 0; i < 3; ++i)
            if (hipStreamWaitEvent(ln->side[i], ln->fork, 0) != hipSuccess) return GS_ERR_HIP;
        hipLaunchKernelGGL(k_train_fb<TR_EMAX>, dim3(slots.fb[2]), dim3(256), 0, ln->side[0], A, 2);
        hipLaunchKernelGGL(k_train_walk<TR_EMAX>, dim3(slots.walk[2]), dim3(256), 0, ln->side[0], A, 2);
        hipLaunchKernelGGL(k_train_fb<128>, dim3(slots.fb[1]), dim3(256), 0, ln->side[1], A, 1);
        hipLaunchKernelGGL(k_train_walk<128>, dim3(slots.walk[1]), dim3(256), 0, ln->side[1], A, 1);
        launch_blend_sg_long(*attrs, *prm, L, n_sets, ws, spectrum, TR_EMAX, ln->side[2]);
        launch_blend_bwd_sg_long(*attrs, *prm, L, n_sets, ws, spectrum, tt->target, mg, escale, tt->grad_scale,
                                 d_attr, TR_EMAX, llong, ln->side[2]);
        hipLaunchKernelGGL(k_train_fb<64>, dim3(slots.fb[0]), dim3(256), 0, s, A, 0);
        hipLaunchKernelGGL(k_train_walk<64>, dim3(slots.walk[0]), dim3(256), 0, s, A, 0);
        for (int i = 0; i < 3; ++i) {
            if (hipEventRecord(ln->join[i], ln->side[i]) != hipSuccess) return GS_ERR_HIP;
            if (hipStreamWaitEvent(s, ln->join[i], 0) != hipSuccess) return GS_ERR_HIP;
        }
        timing_end(tok, s);
    } else {
        hipLaunchKernelGGL(k_train_fb<TR_EMAX>, dim3(slots.fb[2]), dim3(256), 0, s, A, 2);
        hipLaunchKernelGGL(k_train_fb<128>, dim3(slots.fb[1]), dim3(256), 0, s, A, 1);
        hipLaunchKernelGGL(k_train_fb<64>, dim3(slots.fb[0]), dim3(256), 0, s, A, 0);
        hipLaunchKernelGGL(k_train_walk<TR_EMAX>, dim3(slots.walk[2]), dim3(256), 0, s, A, 2);
        hipLaunchKernelGGL(k_train_walk<128>, dim3(slots.walk[1]), dim3(256), 0, s, A, 1);
        hipLaunchKernelGGL(k_train_walk<64>, dim3(slots.walk[0]), dim3(256), 0, s, A, 0);
        timing_end(tok, s);
        launch_blend_sg_long(*attrs, *prm, L, n_sets, ws, spectrum, TR_EMAX, s);
        launch_blend_bwd_sg_long(*attrs, *prm, L, n_sets, ws, spectrum, tt->target, mg, escale, tt->grad_scale,
                                 d_attr, TR_EMAX, llong, s);
    }
    hipLaunchKernelGGL(k_train_loss_add, dim3(1), dim3(64), 0, s, lacc, llong, n_sets, lscale, tt->loss);
    if (!(flags & GS_TRAIN_DEFER_GEOMETRY)) {
        launch_geo_fold(L, ws, s);
        launch_project_bwd(*scene, *queries, *grid, *prm, L, ws, d_mean, d_log_scale, d_quat, d_opacity_logit, s);
    }
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status gs_render_train_geometry(const gs_scene* scene, const gs_queries* queries, const gs_grid* grid,
                                   const gs_params* prm, float* d_mean, float* d_log_scale, float* d_quat,
                                   float* d_opacity_logit, void* workspace, size_t ws_bytes, void* stream)
{
    if (!d_mean || !d_log_scale || !d_quat || !d_opacity_logit || !queries || !prm) return GS_ERR_INVALID_ARG;
    if (queries->count != 1 || (prm->options & GS_OPT_FORWARD_ONLY)) return GS_ERR_INVALID_ARG;
    // the scene, queries, params and workspace checks of a forward (no
    // attributes or spectrum are touched here)
    gs_attrs none{};
    none.data = (const float*)workspace;
    none.n_chan = 1;
    Layout L;
    gs_status st = check_forward(scene, &none, queries, grid, prm, (const float*)workspace, workspace, ws_bytes, &L);
    if (st != GS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    char* ws = (char*)workspace;
    launch_geo_fold(L, ws, s);
    launch_project_bwd(*scene, *queries, *grid, *prm, L, ws, d_mean, d_log_scale, d_quat, d_opacity_logit, s);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

size_t gs_train_scratch_bytes(int32_t n_sets, int32_t n_chan, const gs_grid* grid)
{
    if (!grid || n_sets < 1 || n_chan < 1 || grid->H < 1 || grid->W < 1 || grid->tile_h < 1 || grid->tile_w < 1)
        return 0;
    const int TX = (grid->W + grid->tile_w - 1) / grid->tile_w, TY = (grid->H + grid->tile_h - 1) / grid->tile_h;
    const int gpt = (grid->tile_w * grid->tile_h + TR_PIX - 1) / TR_PIX;
    return train_scratch(TX * TY * gpt, n_sets, n_chan * 2).total;
}

}  // extern "C"
