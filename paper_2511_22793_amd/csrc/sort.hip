// Depth ordering and tile binning (the "directional sorting" of the method:
// Gaussians are binned to tiles and each tile's list is ordered by distance
// to the receiver, Sec. 4.2 and the per-pixel loop of Algorithm 1).
//
// 1. depth sort: stable LSD radix sort of the FP32 distance keys (index
//    order breaks ties), 8-bit digits, one pass = count + scan + scatter;
// 2. tiles-touched scan: exclusive prefix sum of the tile counts in depth
//    order, giving each Gaussian's first pair slot and the pair total;
// 3. pair emission: key = tile << rank_bits | depth_rank, unique per pair;
// 4. pair sort: the same radix sort over the tile digits only (pairs are
//    emitted in depth order, so a stable sort by tile completes the order);
// 5. tile ranges: [start, end) of each tile in the sorted pair array, and
//    the Gaussian id of every sorted pair.
// Every query of a batch is an independent segment (blockIdx.y).
#include "common.h"

namespace gs {

__global__ void k_fill_u32(uint32_t* p, size_t count, size_t q_stride, uint32_t v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[blockIdx.y * q_stride + i] = v;
}

// Zero-fills up to FILL_SEGS buffers in one launch (blockIdx.y = segment).
__global__ void k_fill_segs(FillSegs f)
{
    const int k = blockIdx.y;
    if (k >= f.n) return;
    uint32_t* p = f.p[k];
    const size_t c = f.count[k];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < c; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

void launch_fill_segs(const FillSegs& f, hipStream_t s)
{
    size_t mx = 1;
    for (int k = 0; k < f.n; ++k) mx = f.count[k] > mx ? f.count[k] : mx;
    const size_t blocks = (mx + 255) / 256;
    hipLaunchKernelGGL(k_fill_segs, dim3((unsigned)(blocks < 1024 ? blocks : 1024), f.n), dim3(256), 0, s, f);
}

void launch_fill_u32(uint32_t* p, size_t count, size_t q_stride, int nq, uint32_t v, hipStream_t s)
{
    if (count == 0) return;
    dim3 grid((unsigned)((count + 255) / 256), nq);
    hipLaunchKernelGGL(k_fill_u32, grid, dim3(256), 0, s, p, count, q_stride, v);
}

__global__ void k_fill_dev(uint32_t* p, size_t q_stride, const uint32_t* n_dev, size_t n_stride, uint32_t mult,
                           size_t max_count)
{
    size_t n = (size_t)n_dev[blockIdx.y * n_stride] * mult;
    n = n < max_count ? n : max_count;  // never past the buffer
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[blockIdx.y * q_stride + i] = 0u;
}

void launch_fill_dev(uint32_t* p, size_t max_count, size_t q_stride, int nq, const uint32_t* n_dev, size_t n_stride,
                     uint32_t per_query, hipStream_t s)
{
    const size_t blocks = (max_count + 255) / 256;
    dim3 grid((unsigned)(blocks < 2048 ? (blocks ? blocks : 1) : 2048), nq);
    hipLaunchKernelGGL(k_fill_dev, grid, dim3(256), 0, s, p, q_stride, n_dev, n_stride, per_query, max_count);
}

__device__ __forceinline__ uint32_t seg_count(const uint32_t* n_dev, size_t n_stride, uint32_t n_fixed, int q)
{
    return n_dev ? n_dev[q * n_stride] : n_fixed;
}

// Per-workgroup digit histogram (RB-bit digits) of a block of 64*WV*IT
// keys; counts laid out [digit][block] per query, or [block][digit] (BM)
// for the scatter that scans them itself.
template <int RB, int IT = SORT_ITEMS, int WV = SORT_THREADS / 64, bool BM = false>
__global__ __launch_bounds__(64 * WV) void k_sort_count(
    const uint32_t* __restrict__ keys, size_t s_keys, const uint32_t* __restrict__ n_dev, size_t n_stride,
    uint32_t n_fixed, int shift, uint32_t* __restrict__ counts, size_t s_counts, int max_blocks)
{
    constexpr int R = 1 << RB;
    constexpr int NT = 64 * WV;
    constexpr uint32_t TILE = NT * IT;
    const int q = blockIdx.y;
    const uint32_t n = seg_count(n_dev, n_stride, n_fixed, q);
    const uint32_t base = blockIdx.x * TILE;
    if (base >= n) return;
    __shared__ uint32_t hist[R];
    for (int d = threadIdx.x; d < R; d += NT) hist[d] = 0;
    __syncthreads();
    keys += q * s_keys;
    uint32_t kv[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const uint32_t e = base + i * NT + threadIdx.x;
        kv[i] = e < n ? keys[e] : 0u;
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const uint32_t e = base + i * NT + threadIdx.x;
        if (e < n) atomicAdd(&hist[(kv[i] >> shift) & (R - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += NT)
        counts[q * s_counts + (BM ? (size_t)blockIdx.x * R + d : (size_t)d * max_blocks + blockIdx.x)] = hist[d];
}

// Exclusive scan over blocks for one digit (one workgroup per digit and
// query); writes the digit total to totals[digit].
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t* __restrict__ counts, size_t s_counts,
                                                   uint32_t* __restrict__ totals, size_t s_totals,
                                                   const uint32_t* __restrict__ n_dev, size_t n_stride,
                                                   uint32_t n_fixed, int max_blocks, uint32_t tile)
{
    const int d = blockIdx.x, q = blockIdx.y;
    const uint32_t n = seg_count(n_dev, n_stride, n_fixed, q);
    const int nb = (int)((n + tile - 1) / tile);
    uint32_t* row = counts + q * s_counts + (size_t)d * max_blocks;
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? row[b] : 0u;
        // inclusive wave scan
        uint32_t x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        uint32_t wbase = carry;
        for (int k = 0; k < w; ++k) wbase += wsum[k];
        if (b < nb) row[b] = wbase + x - v;
        __syncthreads();
        if (threadIdx.x == 255) carry = wbase + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[q * s_totals + d] = carry;
}

// Stable scatter of RB-bit digits.  Wave w of the WV-wave workgroup owns
// keys [w*64*IT, (w+1)*64*IT) of the block, consumed as IT rounds of 64
// consecutive keys.  A key's rank is (digit base) + (same digit in earlier
// blocks) + (in earlier waves) + (in earlier rounds of this wave) + (lanes
// below it with the same digit in this round, from an RB-ballot match mask).
// With `order` set (the single tile pass over pair keys) the output is the
// pair's Gaussian, order[key & rank_mask], instead of the key.
template <int RB, int IT = SORT_ITEMS, bool KV = true, int WV = SORT_THREADS / 64, bool FS = false>
__global__ __launch_bounds__(64 * WV) void k_sort_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, size_t s_keys, const uint32_t* __restrict__ n_dev, size_t n_stride,
    uint32_t n_fixed, int shift, const uint32_t* __restrict__ counts, size_t s_counts,
    const uint32_t* __restrict__ totals, size_t s_totals, int max_blocks, const uint32_t* __restrict__ order,
    size_t s_order, uint32_t* __restrict__ plist, size_t s_plist, uint32_t rank_mask, uint2* __restrict__ ranges,
    size_t s_ranges, int T)
{
    constexpr int R = 1 << RB;
    constexpr int NT = 64 * WV;
    constexpr int DPT = R >= NT ? R / NT : 1;  // digits per thread in the digit scans
    constexpr int NDT = R / DPT;               // threads owning digits
    constexpr uint32_t TILE = NT * IT;
    const int q = blockIdx.y;
    const uint32_t n = seg_count(n_dev, n_stride, n_fixed, q);
    const uint32_t base = blockIdx.x * TILE;
    // (with `ranges`, block 0 always runs: it writes the tile ranges, also
    // when there are no keys)
    if (base >= n && !(ranges && blockIdx.x == 0)) return;
    __shared__ uint32_t s_goff[R];
    __shared__ uint32_t s_wcnt[WV][R];
    __shared__ uint32_t s_wsum[WV];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    kin += q * s_keys;
    if (!order) kout += q * s_keys;
    if (vin) {
        vin += q * s_keys;
        vout += q * s_keys;
    }
    // digit bases: exclusive scan of the totals over digits (thread tid <
    // NDT owns digits [tid*DPT, tid*DPT + DPT)).  FS: the counts are
    // [block][digit] and this workgroup forms its digits' totals and its
    // earlier-block prefixes itself (no scan launch; for a few blocks).
    {
        const bool own = tid < NDT;
        uint32_t t[DPT], tsum = 0;
        uint32_t pre[FS ? DPT : 1];
        if constexpr (FS) {
            const int nb = (int)((n + TILE - 1) / TILE);
            const uint32_t* cq = counts + q * s_counts + (size_t)tid * DPT;
#pragma unroll
            for (int k = 0; k < DPT; ++k) t[k] = pre[k] = 0u;
            if (own) {
                // eight blocks' loads in flight at a time
                for (int b0 = 0; b0 < nb; b0 += 8) {
                    uint32_t c[8][DPT];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
#pragma unroll
                        for (int k = 0; k < DPT; ++k) c[u][k] = b0 + u < nb ? cq[(size_t)(b0 + u) * R + k] : 0u;
#pragma unroll
                    for (int u = 0; u < 8; ++u)
#pragma unroll
                        for (int k = 0; k < DPT; ++k) {
                            t[k] += c[u][k];
                            pre[k] += b0 + u < (int)blockIdx.x ? c[u][k] : 0u;
                        }
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < DPT; ++k) t[k] = own ? totals[q * s_totals + tid * DPT + k] : 0u;
        }
#pragma unroll
        for (int k = 0; k < DPT; ++k) tsum += t[k];
        uint32_t x = tsum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_wsum[w] = x;
        for (int d = tid; d < WV * R; d += NT) s_wcnt[d / R][d % R] = 0;
        __syncthreads();
        uint32_t run = x - tsum;
        for (int k = 0; k < w; ++k) run += s_wsum[k];
        if (own) {
#pragma unroll
            for (int k = 0; k < DPT; ++k) {
                const int d = tid * DPT + k;
                if constexpr (FS)
                    s_goff[d] = run + pre[k];
                else
                    s_goff[d] = run + counts[q * s_counts + (size_t)d * max_blocks + blockIdx.x];
                // the tile pass: [start, end) of tile d is its digit range
                if (ranges && blockIdx.x == 0 && d < T) ranges[q * s_ranges + d] = make_uint2(run, run + t[k]);
                run += t[k];
            }
        }
    }
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t key[IT], val[KV ? IT : 1], pos[IT];
    // issue every load before the rank chain so that they overlap
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const uint32_t e = base + w * (TILE / WV) + j * 64 + lane;
        key[j] = e < n ? kin[e] : 0u;
        if constexpr (KV) val[j] = (e < n && vin) ? vin[e] : 0u;
    }
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const uint32_t e = base + w * (TILE / WV) + j * 64 + lane;
        const bool valid = e < n;
        const uint32_t dig = (key[j] >> shift) & (R - 1);
        // lanes whose digit differs from this lane's in some bit: per bit,
        // the ballot of the bit, inverted where this lane's bit is set
        // (bm: the bit as an all-ones or all-zeros word)
        uint32_t dlo = 0u, dhi = 0u;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int32_t bm = (int32_t)(dig << (31 - b)) >> 31;
            const unsigned long long bb = __ballot(bm != 0);
            dlo |= (uint32_t)bb ^ (uint32_t)bm;
            dhi |= (uint32_t)(bb >> 32) ^ (uint32_t)bm;
        }
        const unsigned long long m = __ballot(valid) & ~(((unsigned long long)dhi << 32) | dlo);
        const uint32_t r = (uint32_t)__popcll(m & lt);
        const uint32_t c = s_wcnt[w][dig];
        pos[j] = c + r;
        // the highest lane of each digit group advances the wave's counter
        const bool leader = valid && ((m >> lane) == 1ull);
        __builtin_amdgcn_wave_barrier();
        if (leader) s_wcnt[w][dig] = c + r + 1;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    for (int d = tid; d < R; d += NT) {
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < WV; ++k) {
            const uint32_t c = s_wcnt[k][d];
            s_wcnt[k][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const uint32_t e = base + w * (TILE / WV) + j * 64 + lane;
        if (e < n) {
            const uint32_t dig = (key[j] >> shift) & (R - 1);
            const uint32_t dst = s_goff[dig] + s_wcnt[w][dig] + pos[j];
            if (dst < n) {  // always true when the counts are consistent
                if (order) {
                    plist[q * s_plist + dst] = order[q * s_order + (key[j] & rank_mask)];
                } else {
                    kout[dst] = key[j];
                    if constexpr (KV) {
                        if (vout) vout[dst] = val[j];
                    }
                }
            }
        }
    }
}

// One counting pass over the RB-bit digits at `shift`: per-block counts,
// their scan over blocks, the stable scatter.  `blocks` is the count-row
// stride (the layout sizes the rows for it).
template <int RB, int IT, bool KV, int WV>
static void sort_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, size_t s_keys,
                      const uint32_t* n_dev, size_t n_stride, uint32_t n_fixed, int shift, int blocks,
                      const Layout& L, char* ws, const uint32_t* order, size_t s_order, uint32_t* plist,
                      size_t s_plist, uint32_t rank_mask, hipStream_t s, uint2* ranges = nullptr)
{
    uint32_t* counts = (uint32_t*)(ws + L.counts);
    uint32_t* totals = (uint32_t*)(ws + L.totals);
    const size_t sc = L.s_counts / 4, st = L.s_totals / 4;
    if (!n_dev && blocks <= SORT_FUSED_SCAN_BLOCKS) {
        // a fixed key count (the depth sort) in a few blocks: the scatter
        // scans the block-major counts itself (the digit totals are not kept)
        hipLaunchKernelGGL((k_sort_count<RB, IT, WV, true>), dim3(blocks, L.nq), dim3(64 * WV), 0, s, kin, s_keys,
                           n_dev, n_stride, n_fixed, shift, counts, sc, blocks);
        hipLaunchKernelGGL((k_sort_scatter<RB, IT, KV, WV, true>), dim3(blocks, L.nq), dim3(64 * WV), 0, s, kin, vin,
                           kout, vout, s_keys, n_dev, n_stride, n_fixed, shift, counts, sc, totals, st, blocks,
                           order, s_order, plist, s_plist, rank_mask, (uint2*)nullptr, (size_t)0, 0);
        return;
    }
    hipLaunchKernelGGL((k_sort_count<RB, IT, WV>), dim3(blocks, L.nq), dim3(64 * WV), 0, s, kin, s_keys, n_dev,
                       n_stride, n_fixed, shift, counts, sc, blocks);
    hipLaunchKernelGGL(k_sort_scan, dim3(1 << RB, L.nq), dim3(256), 0, s, counts, sc, totals, st, n_dev, n_stride,
                       n_fixed, blocks, (uint32_t)(64 * WV * IT));
    hipLaunchKernelGGL((k_sort_scatter<RB, IT, KV, WV>), dim3(blocks, L.nq), dim3(64 * WV), 0, s, kin, vin, kout,
                       vout, s_keys, n_dev, n_stride, n_fixed, shift, counts, sc, totals, st, blocks, order, s_order,
                       plist, s_plist, rank_mask, ranges, L.s_ranges / sizeof(uint2), L.T);
}

// Sorts `passes` digits starting at bit 0; returns the buffer index (0 = a,
// 1 = b) that holds the result.
static int radix_sort(uint32_t* ka, uint32_t* kb, uint32_t* va, uint32_t* vb, size_t s_keys,
                      const uint32_t* n_dev, size_t n_stride, uint32_t n_fixed, int first_bit, int passes,
                      int blocks, bool wide, const Layout& L, char* ws, hipStream_t s)
{
    uint32_t *kin = ka, *kout = kb, *vin = va, *vout = vb;
    for (int p = 0; p < passes; ++p) {
        const int shift = first_bit + p * RADIX_BITS;
        if (wide)
            sort_pass<RADIX_BITS, SORT_ITEMS, true, SORT_WIDE_WAVES>(kin, vin, kout, vout, s_keys, n_dev, n_stride,
                                                                     n_fixed, shift, blocks, L, ws, nullptr, 0,
                                                                     nullptr, 0, 0u, s);
        else
            sort_pass<RADIX_BITS, SORT_ITEMS, true, SORT_THREADS / 64>(kin, vin, kout, vout, s_keys, n_dev, n_stride,
                                                                       n_fixed, shift, blocks, L, ws, nullptr, 0,
                                                                       nullptr, 0, 0u, s);
        uint32_t* t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    return passes & 1;
}

void launch_depth_sort(const Layout& L, char* ws, hipStream_t s)
{
    // keys a -> ... -> a after 4 passes (even), values follow
    radix_sort((uint32_t*)(ws + L.keys_a), (uint32_t*)(ws + L.keys_b), (uint32_t*)(ws + L.vals_a),
               (uint32_t*)(ws + L.vals_b), L.s_keys / 4, nullptr, 0, (uint32_t)L.n, 0, 4, L.sort_blocks,
               L.sort_wide != 0, L, ws, s);
}

// ---- tiles-touched scan and pair emission -------------------------------
// Scan granularity: EMIT_RANKS consecutive depth ranks per workgroup.
constexpr int EMIT_RANKS = 64;
// up to this many blocks the emission adds up the block sums itself (each
// workgroup reads the sums before its own: quadratic, so only for a few
// thousand blocks)
constexpr int EMIT_SCAN_BLOCKS = 2048;

__device__ __forceinline__ uint32_t ntiles_at(const uint32_t* order, const uint4* tinfo, uint32_t k, uint32_t nvis)
{
    return k < nvis ? tinfo[order[k]].w : 0u;
}

// Exclusive scan within a 256-thread workgroup; returns the prefix of v.
__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t* wsum)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int k = 0; k < w; ++k) base += wsum[k];
    return base + x - v;
}

// Sum of the tile counts of each EMIT_RANKS block of the depth order (one
// wave per block).
__global__ __launch_bounds__(64) void k_scan_reduce(const uint32_t* __restrict__ order, size_t s_order,
                                                    const uint4* __restrict__ tinfo, size_t s_tinfo,
                                                    const uint32_t* __restrict__ flags, size_t s_flags,
                                                    uint32_t* __restrict__ partial, size_t s_partial)
{
    const int q = blockIdx.y;
    const uint32_t nvis = flags[q * s_flags + FL_NVIS];
    const uint32_t k = blockIdx.x * EMIT_RANKS + threadIdx.x;
    uint32_t v = ntiles_at(order + q * s_order, tinfo + q * s_tinfo, k, nvis);
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x == 0) partial[q * s_partial + blockIdx.x] = v;
}

// Exclusive scan of the block sums; records the pair count and overflow.
__global__ __launch_bounds__(256) void k_scan_top(uint32_t* __restrict__ partial, size_t s_partial, int nblocks,
                                                  uint32_t* __restrict__ flags, size_t s_flags, int64_t cap)
{
    const int q = blockIdx.x;
    partial += q * s_partial;
    flags += q * s_flags;
    __shared__ uint32_t wsum[4];
    __shared__ unsigned long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nblocks; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const uint32_t v = b < nblocks ? partial[b] : 0u;
        const uint32_t ex = block_exclusive_scan_256(v, wsum);
        const unsigned long long c = carry;
        if (b < nblocks) partial[b] = (uint32_t)(c + ex);
        __syncthreads();
        if (threadIdx.x == 255) carry = c + ex + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long P = carry;
        flags[FL_PAIRS] = (uint32_t)(P > 0xFFFFFFFFull ? 0xFFFFFFFFull : P);
        flags[FL_OVERFLOW] = P > (unsigned long long)cap ? 1u : 0u;
        flags[FL_PUSED] = (uint32_t)(P > (unsigned long long)cap ? (unsigned long long)cap : P);
    }
}

// Emits the pair keys in depth order.  A workgroup owns 64 consecutive
// ranks; their pairs are spread over its 256 lanes (pair p belongs to the
// last rank whose first pair slot is <= p; each lane walks forward through
// the 64 prefix offsets as its p grows by 256), so the stores stay coalesced
// and the work balanced however unequal the tile counts are.
// SCAN: `partial` holds the block sums (no k_scan_top): each workgroup adds
// up the sums before its own (for a few thousand blocks at most), and the
// last active one records the pair count and overflow.
template <bool SCAN>
__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ order, size_t s_order,
                                             const uint4* __restrict__ tinfo, size_t s_tinfo,
                                             uint32_t* __restrict__ flags, size_t s_flags,
                                             const uint32_t* __restrict__ partial, size_t s_partial,
                                             uint32_t* __restrict__ pkeys, size_t s_pkeys, int64_t cap,
                                             int TX, int rank_bits)
{
    const int q = blockIdx.y;
    const uint32_t nvis = flags[q * s_flags + FL_NVIS];
    const uint32_t base = blockIdx.x * EMIT_RANKS;
    if (base >= nvis) return;
    uint32_t o0 = 0;
    if constexpr (SCAN) {
        __shared__ unsigned long long s_pre;
        if (threadIdx.x == 0) s_pre = 0ull;
        __syncthreads();
        unsigned long long v = 0ull;
        for (uint32_t b = threadIdx.x; b < blockIdx.x; b += 256) v += partial[q * s_partial + b];
        if (v) atomicAdd(&s_pre, v);
        __syncthreads();
        const unsigned long long pre = s_pre;
        o0 = (uint32_t)pre;
        if (threadIdx.x == 0 && blockIdx.x == (nvis - 1) / EMIT_RANKS) {
            const unsigned long long P = pre + partial[q * s_partial + blockIdx.x];
            flags[q * s_flags + FL_PAIRS] = (uint32_t)(P > 0xFFFFFFFFull ? 0xFFFFFFFFull : P);
            flags[q * s_flags + FL_OVERFLOW] = P > (unsigned long long)cap ? 1u : 0u;
            flags[q * s_flags + FL_PUSED] = (uint32_t)(P > (unsigned long long)cap ? (unsigned long long)cap : P);
        }
    } else {
        o0 = partial[q * s_partial + blockIdx.x];
    }
    order += q * s_order;
    tinfo += q * s_tinfo;
    pkeys += q * s_pkeys;
    __shared__ uint4 s_ti[EMIT_RANKS];
    __shared__ uint32_t s_start[EMIT_RANKS + 1];
    __shared__ uint32_t s_total;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        const uint32_t k = base + lane;
        const uint4 ti = k < nvis ? tinfo[order[k]] : make_uint4(0, 0, 0, 0);
        uint32_t x = ti.w;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        s_ti[lane] = ti;
        s_start[lane] = x - ti.w;
        if (lane == 63) {
            s_start[EMIT_RANKS] = 0xFFFFFFFFu;  // sentinel
            s_total = x;
        }
    }
    __syncthreads();
    const uint32_t total = s_total;
    int j = 0;  // largest j with s_start[j] <= p; only moves forward as p grows
    for (uint32_t p = threadIdx.x; p < total; p += 256) {
        while (s_start[j + 1] <= p) ++j;
        const uint4 t = s_ti[j];
        const uint32_t e = p - s_start[j];
        const int xa0 = t.x & 0xFFFF, xa1 = t.x >> 16, xb0 = t.y & 0xFFFF, xb1 = t.y >> 16;
        const int ty0 = t.z & 0xFFFF;
        const int na = xa1 - xa0 + 1, nb = xb1 >= xb0 ? xb1 - xb0 + 1 : 0, ncols = na + nb;
        // row = e / ncols: (e + 0.5) / ncols is at least 0.5/ncols from an
        // integer and the float product's error is below that while
        // e < 2^22 (the layout caps the tile count there)
        const int r = (int)(((float)e + 0.5f) * (1.0f / (float)ncols));
        const int c = (int)e - r * ncols;
        const int tx = c < na ? xa0 + c : xb0 + (c - na);
        const uint32_t dst = o0 + p;
        if ((int64_t)dst < cap) pkeys[dst] = ((uint32_t)((ty0 + r) * TX + tx) << rank_bits) | (base + j);
    }
}

// Tile ranges from the sorted pair keys; also resolves each pair's Gaussian.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ pkeys, size_t s_pkeys,
                                                const uint32_t* __restrict__ order, size_t s_order,
                                                const uint32_t* __restrict__ flags, size_t s_flags,
                                                uint32_t* __restrict__ plist, size_t s_plist,
                                                uint2* __restrict__ ranges, size_t s_ranges, int rank_bits,
                                                uint32_t T)
{
    const int q = blockIdx.y;
    const uint32_t P = flags[q * s_flags + FL_PUSED];
    pkeys += q * s_pkeys;
    ranges += q * s_ranges;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const uint32_t key = pkeys[p];
        const uint32_t t = key >> rank_bits;
        plist[q * s_plist + p] = order[q * s_order + (key & ((1u << rank_bits) - 1u))];
        const uint32_t prev = p > 0 ? (pkeys[p - 1] >> rank_bits) : 0xFFFFFFFFu;
        if (t >= T || (p > 0 && prev >= T)) continue;  // never taken for keys written by k_emit
        if (t != prev) {
            ranges[t].x = p;
            if (p > 0) ranges[prev].y = p;
        }
        if (p == P - 1) ranges[t].y = P;
    }
}

void launch_binning(const Layout& L, char* ws, hipStream_t s)
{
    const uint32_t* order = (const uint32_t*)(ws + L.vals_a);
    const uint4* tinfo = (const uint4*)(ws + L.tinfo);
    uint32_t* flags = (uint32_t*)(ws + L.flags);
    uint32_t* partial = (uint32_t*)(ws + L.partial);
    const size_t so = L.s_keys / 4, sti = L.s_tinfo / sizeof(uint4), sf = L.s_flags / 4, sp = L.s_partial / 4;
    const int nblk = (L.n + EMIT_RANKS - 1) / EMIT_RANKS;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk, L.nq), dim3(64), 0, s, order, so, tinfo, sti, flags, sf,
                       partial, sp);
    uint32_t* pa = (uint32_t*)(ws + L.pkeys_a);
    uint32_t* pb = (uint32_t*)(ws + L.pkeys_b);
    const size_t spk = L.s_pkeys / 4;
    if (nblk <= EMIT_SCAN_BLOCKS) {
        hipLaunchKernelGGL(k_emit<true>, dim3(nblk, L.nq), dim3(256), 0, s, order, so, tinfo, sti, flags, sf,
                           partial, sp, pa, spk, L.cap, L.TX, L.rank_bits);
    } else {
        hipLaunchKernelGGL(k_scan_top, dim3(L.nq), dim3(256), 0, s, partial, sp, nblk, flags, sf, L.cap);
        hipLaunchKernelGGL(k_emit<false>, dim3(nblk, L.nq), dim3(256), 0, s, order, so, tinfo, sti, flags, sf,
                           partial, sp, pa, spk, L.cap, L.TX, L.rank_bits);
    }
    // pairs are emitted in depth-rank order, so a stable sort on the tile
    // digits alone yields (tile, depth) order
    uint2* ranges = (uint2*)(ws + L.ranges);
    if (L.tile_bits <= TILE_PASS_MAX_BITS) {
        // one counting pass over all tile digits: the scatter writes each
        // pair's Gaussian straight into the list, and the tile ranges are
        // the scan of the per-tile totals
        const uint32_t* nd = flags + FL_PUSED;
        const uint32_t rmask = (1u << L.rank_bits) - 1u;
        uint32_t* plist = (uint32_t*)(ws + L.plist);
        const size_t spl = L.s_plist / 4;
        constexpr int WN = SORT_THREADS / 64, WW = SORT_WIDE_WAVES;
        if (L.tile_bits <= RADIX_BITS) {
            // 256 digits: the usual blocks of SORT_ITEMS keys per thread
            if (L.pair_wide)
                sort_pass<RADIX_BITS, SORT_ITEMS, false, WW>(pa, nullptr, nullptr, nullptr, spk, nd, sf, 0u,
                                                             L.rank_bits, L.pair_blocks, L, ws, order, so, plist,
                                                             spl, rmask, s, ranges);
            else
                sort_pass<RADIX_BITS, SORT_ITEMS, false, WN>(pa, nullptr, nullptr, nullptr, spk, nd, sf, 0u,
                                                             L.rank_bits, L.pair_blocks, L, ws, order, so, plist,
                                                             spl, rmask, s, ranges);
        } else {
            // 1024 digits: blocks of TILE_PASS_ITEMS (TILE_PASS_WIDE_ITEMS)
            // keys per thread keep the digit-by-block count matrix small
            if (L.pair_wide)
                sort_pass<TILE_PASS_MAX_BITS, TILE_PASS_WIDE_ITEMS, false, WW>(pa, nullptr, nullptr, nullptr, spk, nd,
                                                                          sf, 0u, L.rank_bits, L.tile_blocks, L, ws,
                                                                          order, so, plist, spl, rmask, s, ranges);
            else
                sort_pass<TILE_PASS_MAX_BITS, TILE_PASS_ITEMS, false, WN>(pa, nullptr, nullptr, nullptr, spk, nd,
                                                                          sf, 0u, L.rank_bits, L.tile_blocks, L, ws,
                                                                          order, so, plist, spl, rmask, s, ranges);
        }
        // (the scatter's block 0 wrote the tile ranges: the digit ranges)
        return;
    }
    const int which = radix_sort(pa, pb, nullptr, nullptr, spk, flags + FL_PUSED, sf, 0, L.rank_bits,
                                 L.pair_passes, L.pair_blocks, L.pair_wide != 0, L, ws, s);
    uint32_t* sorted = which ? pb : pa;
    launch_fill_u32((uint32_t*)ranges, (size_t)L.T * 2, L.s_ranges / 4, L.nq, 0u, s);
    const int64_t rblocks = (L.cap + 255) / 256;
    dim3 grid((unsigned)(rblocks < 1024 ? rblocks : 1024), L.nq);
    hipLaunchKernelGGL(k_ranges, grid, dim3(256), 0, s, sorted, spk, order, so, flags, sf,
                       (uint32_t*)(ws + L.plist), L.s_plist / 4, ranges, L.s_ranges / sizeof(uint2), L.rank_bits,
                       (uint32_t)L.T);
}

}  // namespace gs
