// C ABI entry points: argument validation, workspace layout and the
// sequence of stream-ordered kernel launches.
#include <string.h>

#include "common.h"

namespace gs {

static int bits_for(uint64_t v)  // bits needed to hold values 0..v
{
    int b = 1;
    while (b < 63 && (v >> b) != 0) ++b;
    return b;
}

gs_status make_layout(int32_t n, int32_t nq, const gs_grid* g, const gs_params* p, Layout* L)
{
    if (n < 1 || nq < 1 || !g || !p) return GS_ERR_INVALID_ARG;
    if (p->options & ~(GS_OPT_FORWARD_ONLY | GS_OPT_BWD_PER_GROUP | GS_OPT_BLEND_PER_GROUP)) return GS_ERR_INVALID_ARG;
    if (g->H < 1 || g->W < 2 || g->tile_h < 1 || g->tile_w < 1) return GS_ERR_INVALID_ARG;
    const int nthr = g->tile_h * g->tile_w;
    if (nthr != 64 && nthr != 128 && nthr != 256) return GS_ERR_INVALID_ARG;
    memset(L, 0, sizeof(*L));
    L->n = n;
    L->nq = nq;
    L->H = g->H;
    L->W = g->W;
    L->tw = g->tile_w;
    L->th = g->tile_h;
    L->TX = (g->W + g->tile_w - 1) / g->tile_w;
    L->TY = (g->H + g->tile_h - 1) / g->tile_h;
    L->T = L->TX * L->TY;
    if (L->TX > 0xFFFF || L->TY > 0xFFFF || L->T >= (1 << 22)) return GS_ERR_CAPACITY;
    int64_t cap = p->pair_capacity;
    if (cap <= 0) cap = (int64_t)n * (L->T < 64 ? L->T : 64) + 4096;
    if (cap > 0x7FFFFFFFll) return GS_ERR_CAPACITY;
    L->cap = cap;
    L->rank_bits = bits_for((uint64_t)(n - 1));
    L->tile_bits = bits_for((uint64_t)(L->T - 1));
    if (L->rank_bits + L->tile_bits > 32) return GS_ERR_CAPACITY;
    L->pair_passes = L->tile_bits <= TILE_PASS_MAX_BITS ? 1 : (L->tile_bits + RADIX_BITS - 1) / RADIX_BITS;
    const int digits = L->tile_bits <= RADIX_BITS ? RADIX
                       : (L->tile_bits <= TILE_PASS_MAX_BITS ? (1 << TILE_PASS_MAX_BITS) : RADIX);
    const int64_t wide = SORT_WIDE_WAVES / (SORT_THREADS / 64);  // keys-per-block factor of a wide block
    L->sort_wide = (n + wide * SORT_TILE - 1) / (wide * SORT_TILE) * nq >= SORT_WIDE_MIN_BLOCKS;
    L->pair_wide = (cap + wide * SORT_TILE - 1) / (wide * SORT_TILE) * nq >= SORT_WIDE_MIN_BLOCKS;
    const int64_t stile = L->sort_wide ? wide * SORT_TILE : SORT_TILE;
    const int64_t ptile = L->pair_wide ? wide * SORT_TILE : SORT_TILE;
    const int64_t ttile = L->pair_wide ? (int64_t)64 * SORT_WIDE_WAVES * TILE_PASS_WIDE_ITEMS
                                       : (int64_t)SORT_THREADS * TILE_PASS_ITEMS;
    L->sort_blocks = (int)((n + stile - 1) / stile);
    L->pair_blocks = (int)((cap + ptile - 1) / ptile);
    L->tile_blocks = (int)((cap + ttile - 1) / ttile);
    const size_t HW = (size_t)g->H * g->W;

    L->s_flags = align256(FL_WORDS * 4);
    // a whole number of 48-byte records and of 256-byte blocks (lcm = 768)
    L->s_rec = ((size_t)n * sizeof(GRec) + 767) / 768 * 768;
    L->s_rect = align256((size_t)n * 16);
    L->s_status = align256((size_t)n * 4);
    L->s_tinfo = align256((size_t)n * 16);
    L->s_keys = align256((size_t)n * 4);
    L->s_partial = align256((size_t)((n + 63) / 64) * 4);
    L->s_pkeys = align256((size_t)cap * 4);
    L->s_plist = align256((size_t)cap * 4);
    L->s_ranges = align256((size_t)L->T * 8);
    {
        // depth passes: sort_blocks x 256; 8-bit or multi-pass tile sorts:
        // pair_blocks x 256; the single 10-bit tile pass: tile_blocks x 1024
        size_t rows = (size_t)L->sort_blocks * RADIX;
        if (L->pair_passes > 1 || L->tile_bits <= RADIX_BITS) rows = std::max(rows, (size_t)L->pair_blocks * RADIX);
        else rows = std::max(rows, (size_t)L->tile_blocks * digits);
        L->s_counts = align256(rows * 4);
    }
    L->s_totals = align256((size_t)(1 << TILE_PASS_MAX_BITS) * 4);
    L->s_pix = align256(HW * 4);
    const bool fwd_only = (p->options & GS_OPT_FORWARD_ONLY) != 0;
    L->s_g2d = fwd_only ? 0 : align256((size_t)n * 8 * 4);
    L->s_live = fwd_only ? 0 : align256((size_t)n * 4);
    L->s_gacc = fwd_only ? 0 : align256((size_t)cap * 8 * 4);
    L->s_wtot = fwd_only ? 0 : align256((size_t)n * 4);

    size_t off = 0;
    auto take = [&](size_t stride) {
        const size_t o = off;
        off += stride * (size_t)nq;
        return o;
    };
    L->flags = take(L->s_flags);
    L->rec = take(L->s_rec);
    L->rect = take(L->s_rect);
    L->status = take(L->s_status);
    L->tinfo = take(L->s_tinfo);
    L->keys_a = take(L->s_keys);
    L->keys_b = take(L->s_keys);
    L->vals_a = take(L->s_keys);
    L->vals_b = take(L->s_keys);
    L->partial = take(L->s_partial);
    L->pkeys_a = take(L->s_pkeys);
    // the single tile pass writes the list directly: no second key buffer
    L->pkeys_b = take(L->tile_bits <= TILE_PASS_MAX_BITS ? 0 : L->s_pkeys);
    L->plist = take(L->s_plist);
    L->ranges = take(L->s_ranges);
    L->counts = take(L->s_counts);
    L->totals = take(L->s_totals);
    L->T_final = take(L->s_pix);
    L->n_last = take(L->s_pix);
    L->n_contrib = take(L->s_pix);
    L->g2d = take(L->s_g2d);
    L->live = take(L->s_live);
    L->gacc = take(L->s_gacc);
    L->wtot = take(L->s_wtot);
    L->total = off;
    return GS_OK;
}

gs_status check_forward(const gs_scene* sc, const gs_attrs* a, const gs_queries* qs, const gs_grid* g,
                               const gs_params* p, const float* spectrum, const void* ws, size_t ws_bytes,
                               Layout* L)
{
    if (!sc || !a || !qs || !g || !p || !spectrum) return GS_ERR_INVALID_ARG;
    if (!sc->mean || !sc->log_scale || !sc->quat || !sc->opacity_logit || sc->n < 1) return GS_ERR_INVALID_ARG;
    if (!a->data || a->n_chan < 1 || a->query_stride < 0 || (a->is_complex != 0 && a->is_complex != 1))
        return GS_ERR_INVALID_ARG;
    if ((int64_t)a->n_chan * (a->is_complex ? 2 : 1) > 65536) return GS_ERR_CAPACITY;
    if (!qs->rx || qs->count < 1) return GS_ERR_INVALID_ARG;
    if (!(p->alpha_min > 0.0f) || !(p->alpha_max > p->alpha_min) || !(p->alpha_max < 1.0f) || !(p->T_min >= 0.0f) ||
        !(p->T_min < 1.0f) || !(p->dilation >= 0.0f) || !(p->r_near >= 0.0f) || !(p->margin >= 0.0f) ||
        !(p->atten_power >= 0.0f) || (p->atten_ref != 0 && p->atten_ref != 1))
        return GS_ERR_INVALID_ARG;
    const gs_status st = make_layout(sc->n, qs->count, g, p, L);
    if (st != GS_OK) return st;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < L->total) return GS_ERR_WORKSPACE;
    return GS_OK;
}

void enqueue_prepare(const gs_scene* scene, const gs_queries* queries, const gs_grid* grid,
                            const gs_params* prm, const Layout& L, char* ws, hipStream_t s)
{
    launch_fill_u32((uint32_t*)(ws + L.flags), FL_WORDS, L.s_flags / 4, L.nq, 0u, s);
    launch_project(*scene, *queries, *grid, *prm, L, ws, s);
    launch_depth_sort(L, ws, s);
    launch_binning(L, ws, s);
}

}  // namespace gs

using namespace gs;

extern "C" {

void gs_default_params(gs_params* p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->alpha_min = 1.0f / 255.0f;
    p->alpha_max = 0.99f;
    p->T_min = 1e-4f;
    p->dilation = 0.3f;
    p->r_near = 0.2f;
    p->atten_power = 2.0f;
    p->atten_ref = 0;
    p->margin = 1e-3f;
    p->pair_capacity = 0;
    p->chan_group = 0;
}

void gs_default_grid(gs_grid* g, int32_t H, int32_t W)
{
    if (!g) return;
    memset(g, 0, sizeof(*g));
    g->H = H;
    g->W = W;
    g->tile_h = 16;
    g->tile_w = 16;
    const double V[9] = {0, 1, 0, 0, 0, 1, 1, 0, 0};
    memcpy(g->view, V, sizeof(V));
}

const char* gs_status_string(gs_status s)
{
    switch (s) {
        case GS_OK: return "ok";
        case GS_ERR_INVALID_ARG: return "invalid argument";
        case GS_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case GS_ERR_CAPACITY: return "size beyond the library's limits";
        case GS_ERR_HIP: return "HIP runtime error";
        case GS_ERR_NONFINITE: return "non-finite input";
    }
    return "unknown status";
}

gs_status gs_workspace_layout(int32_t n, int32_t n_queries, const gs_grid* grid, const gs_params* prm,
                              gs_layout* out)
{
    if (!out) return GS_ERR_INVALID_ARG;
    Layout L;
    const gs_status st = make_layout(n, n_queries, grid, prm, &L);
    if (st != GS_OK) return st;
    memset(out, 0, sizeof(*out));
    out->total = L.total;
    out->flags = L.flags;
    out->rec = L.rec;
    out->rect = L.rect;
    out->status = L.status;
    out->tinfo = L.tinfo;
    out->order = L.vals_a;
    out->keys = L.keys_a;
    out->pair_keys = L.pkeys_a;
    out->pair_list = L.plist;
    out->ranges = L.ranges;
    out->T_final = L.T_final;
    out->n_last = L.n_last;
    out->n_contrib = L.n_contrib;
    out->flags_stride = L.s_flags;
    out->rec_stride = L.s_rec;
    out->rect_stride = L.s_rect;
    out->status_stride = L.s_status;
    out->tinfo_stride = L.s_tinfo;
    out->order_stride = L.s_keys;
    out->keys_stride = L.s_keys;
    out->pair_keys_stride = L.s_pkeys;
    out->pair_list_stride = L.s_plist;
    out->ranges_stride = L.s_ranges;
    out->pix_stride = L.s_pix;
    out->pair_capacity = L.cap;
    out->tiles_x = L.TX;
    out->tiles_y = L.TY;
    return GS_OK;
}

gs_status gs_render_forward(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries,
                            const gs_grid* grid, const gs_params* prm, float* spectrum, void* workspace,
                            size_t ws_bytes, void* stream)
{
    Layout L;
    gs_status st = check_forward(scene, attrs, queries, grid, prm, spectrum, workspace, ws_bytes, &L);
    if (st != GS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    (void)hipGetLastError();  // clear a stale error so that GS_CHECK_LAUNCH reports ours
    enqueue_prepare(scene, queries, grid, prm, L, ws, s);
    st = launch_blend(*attrs, *prm, L, L.nq, ws, spectrum, s);
    if (st != GS_OK) return st;
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status gs_render_prepare(const gs_scene* scene, const gs_queries* queries, const gs_grid* grid,
                            const gs_params* prm, void* workspace, size_t ws_bytes, void* stream)
{
    if (!scene || !queries || !grid || !prm) return GS_ERR_INVALID_ARG;
    gs_attrs dummy = {1, 0, (const float*)workspace, 0};
    Layout L;
    gs_status st = check_forward(scene, &dummy, queries, grid, prm, (const float*)workspace, workspace, ws_bytes, &L);
    if (st != GS_OK) return st;
    (void)hipGetLastError();
    enqueue_prepare(scene, queries, grid, prm, L, (char*)workspace, (hipStream_t)stream);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status gs_render_blend(const gs_attrs* attrs, int32_t n, int32_t n_queries, int32_t n_sets,
                          const gs_grid* grid, const gs_params* prm, float* spectrum, void* workspace,
                          size_t ws_bytes, void* stream)
{
    if (!attrs || !attrs->data || attrs->n_chan < 1 || attrs->query_stride < 0 || !spectrum || !grid || !prm)
        return GS_ERR_INVALID_ARG;
    if (attrs->is_complex != 0 && attrs->is_complex != 1) return GS_ERR_INVALID_ARG;
    if ((int64_t)attrs->n_chan * (attrs->is_complex ? 2 : 1) > 65536) return GS_ERR_CAPACITY;
    if (n_sets < 1 || n_queries < 1) return GS_ERR_INVALID_ARG;
    if (n_sets != n_queries && !(n_queries == 1 && prm->atten_ref == 0)) return GS_ERR_INVALID_ARG;
    if (n_sets > 65535) return GS_ERR_CAPACITY;
    Layout L;
    gs_status st = make_layout(n, n_queries, grid, prm, &L);
    if (st != GS_OK) return st;
    if (!workspace || ((uintptr_t)workspace & 255) || ws_bytes < L.total) return GS_ERR_WORKSPACE;
    (void)hipGetLastError();
    st = launch_blend(*attrs, *prm, L, n_sets, (char*)workspace, spectrum, (hipStream_t)stream);
    if (st != GS_OK) return st;
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status gs_render_blend_loss(const gs_attrs* attrs, int32_t n, int32_t n_queries, int32_t n_sets,
                               const gs_grid* grid, const gs_params* prm, float* spectrum, void* workspace,
                               size_t ws_bytes, const float* target, float lambda_ch, float* loss, float* h_hat,
                               float* mean_grad, float* d_partial, void* scratch, size_t scratch_bytes,
                               void* stream)
{
    if (!attrs || !attrs->data || attrs->n_chan < 1 || attrs->query_stride < 0 || !spectrum || !grid || !prm)
        return GS_ERR_INVALID_ARG;
    if (!target || !loss || !h_hat || !mean_grad || !(lambda_ch >= 0.0f)) return GS_ERR_INVALID_ARG;
    if (attrs->is_complex != 0 && attrs->is_complex != 1) return GS_ERR_INVALID_ARG;
    if ((int64_t)attrs->n_chan * (attrs->is_complex ? 2 : 1) > 65536) return GS_ERR_CAPACITY;
    if (n_sets < 1 || n_queries < 1) return GS_ERR_INVALID_ARG;
    if (n_sets != n_queries && !(n_queries == 1 && prm->atten_ref == 0)) return GS_ERR_INVALID_ARG;
    if (n_sets > 65535) return GS_ERR_CAPACITY;
    Layout L;
    gs_status st = make_layout(n, n_queries, grid, prm, &L);
    if (st != GS_OK) return st;
    if (!workspace || ((uintptr_t)workspace & 255) || ws_bytes < L.total) return GS_ERR_WORKSPACE;
    const int C = attrs->is_complex ? 2 : 1;
    const int Fc = attrs->n_chan * C;
    // scratch: the loss accumulators, then the per-wave partial sums
    const int np = L.T * ((L.tw * L.th) >> 6);
    const size_t acc_bytes = align256((size_t)n_sets * Fc * 3 * sizeof(float));
    const size_t need = acc_bytes + (size_t)n_sets * Fc * 3 * np * sizeof(float);
    if (!scratch || scratch_bytes < need || ((uintptr_t)scratch & 255)) return GS_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    const size_t HW = (size_t)L.H * L.W;
    float* acc = (float*)scratch;
    float* part = (float*)((char*)scratch + acc_bytes);
    const float scale = 2.0f / ((float)attrs->n_chan * (float)HW * (float)n_sets);
    st = launch_blend(*attrs, *prm, L, n_sets, (char*)workspace, spectrum, s, target, d_partial, part, scale);
    if (st != GS_OK) return st;
    launch_loss_parts(n_sets, Fc, C, np, part, acc, s);
    launch_loss_finish(n_sets, Fc, C, HW, lambda_ch, acc, h_hat, loss, mean_grad, s);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status gs_render_live(int32_t n, int32_t n_queries, const gs_grid* grid, const gs_params* prm, void* workspace,
                         size_t ws_bytes, uint32_t* live_list, int64_t list_stride, uint32_t* live_count,
                         void* stream)
{
    if (!live_list || !live_count || !grid || !prm) return GS_ERR_INVALID_ARG;
    if (prm->options & GS_OPT_FORWARD_ONLY) return GS_ERR_INVALID_ARG;
    Layout L;
    gs_status st = make_layout(n, n_queries, grid, prm, &L);
    if (st != GS_OK) return st;
    if (list_stride < n && n_queries > 1) return GS_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace & 255) || ws_bytes < L.total) return GS_ERR_WORKSPACE;
    (void)hipGetLastError();
    launch_live(*prm, L, (char*)workspace, live_list, (size_t)list_stride, live_count, (hipStream_t)stream);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

static gs_status render_backward(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries,
                                 int32_t n_sets, const gs_grid* grid, const gs_params* prm, const float* spectrum,
                                 const BwdUpstream& up, float* d_mean, float* d_log_scale, float* d_quat,
                                 float* d_opacity_logit, float* d_attr, int32_t flags, void* workspace,
                                 size_t ws_bytes, void* stream)
{
    if (!d_mean || !d_log_scale || !d_quat || !d_opacity_logit || !d_attr) return GS_ERR_INVALID_ARG;
    if (prm && (prm->options & GS_OPT_FORWARD_ONLY)) return GS_ERR_INVALID_ARG;
    Layout L;
    gs_status st = check_forward(scene, attrs, queries, grid, prm, spectrum, workspace, ws_bytes, &L);
    if (st != GS_OK) return st;
    if (n_sets < 1 || (n_sets != queries->count && !(queries->count == 1 && prm->atten_ref == 0)))
        return GS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    (void)hipGetLastError();
    const int C = attrs->is_complex ? 2 : 1;
    const size_t na = (size_t)(attrs->query_stride ? n_sets : 1) * scene->n * attrs->n_chan * C;
    launch_fill_u32((uint32_t*)(ws + L.g2d), (size_t)L.n * 8, L.s_g2d / 4, L.nq, 0u, s);
    // the per-pair accumulator over the used pairs (the fold clears it again)
    launch_fill_dev((uint32_t*)(ws + L.gacc), (size_t)L.cap * 8, L.s_gacc / 4, L.nq,
                    (const uint32_t*)(ws + L.flags) + FL_PUSED, L.s_flags / 4, 8u, s);
    if (!(flags & GS_BWD_ATTR_GRAD_ZEROED)) launch_fill_u32((uint32_t*)d_attr, na, 0, 1, 0u, s);
    st = launch_blend_bwd(*attrs, *prm, L, n_sets, ws, spectrum, up, d_attr, s);
    if (st != GS_OK) return st;
    launch_project_bwd(*scene, *queries, *grid, *prm, L, ws, d_mean, d_log_scale, d_quat, d_opacity_logit, s);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status gs_render_backward(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries,
                             int32_t n_sets, const gs_grid* grid, const gs_params* prm, const float* spectrum,
                             const float* d_spectrum, float* d_mean, float* d_log_scale, float* d_quat,
                             float* d_opacity_logit, float* d_attr, int32_t flags, void* workspace, size_t ws_bytes,
                             void* stream)
{
    if (!d_spectrum) return GS_ERR_INVALID_ARG;
    const BwdUpstream up{d_spectrum, nullptr, nullptr, 0.0f};
    return render_backward(scene, attrs, queries, n_sets, grid, prm, spectrum, up, d_mean, d_log_scale, d_quat,
                           d_opacity_logit, d_attr, flags, workspace, ws_bytes, stream);
}

gs_status gs_render_backward_l2(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries,
                                int32_t n_sets, const gs_grid* grid, const gs_params* prm, const float* spectrum,
                                const gs_l2_grad* lg, float* d_mean, float* d_log_scale, float* d_quat,
                                float* d_opacity_logit, float* d_attr, int32_t flags, void* workspace,
                                size_t ws_bytes, void* stream)
{
    if (!lg || !lg->mean_grad || (!lg->partial && !lg->target) || !(lg->scale == lg->scale))
        return GS_ERR_INVALID_ARG;
    const BwdUpstream up{lg->partial, lg->partial ? nullptr : lg->target, lg->mean_grad, lg->scale};
    return render_backward(scene, attrs, queries, n_sets, grid, prm, spectrum, up, d_mean, d_log_scale, d_quat,
                           d_opacity_logit, d_attr, flags, workspace, ws_bytes, stream);
}

gs_status gs_overflow_word(const void* workspace, size_t ws_bytes, int32_t n, int32_t n_queries,
                           const gs_grid* grid, const gs_params* prm, int32_t q, const uint32_t** word)
{
    if (!word || q < 0 || q >= n_queries) return GS_ERR_INVALID_ARG;
    Layout L;
    gs_status st = make_layout(n, n_queries, grid, prm, &L);
    if (st != GS_OK) return st;
    if (!workspace || ws_bytes < L.total) return GS_ERR_WORKSPACE;
    *word = (const uint32_t*)((const char*)workspace + L.flags + (size_t)q * L.s_flags) + FL_OVERFLOW;
    return GS_OK;
}

gs_status gs_read_flags(const void* workspace, size_t ws_bytes, int32_t n, int32_t n_queries, const gs_grid* grid,
                        const gs_params* prm, gs_flags* out, void* stream)
{
    if (!out) return GS_ERR_INVALID_ARG;
    Layout L;
    gs_status st = make_layout(n, n_queries, grid, prm, &L);
    if (st != GS_OK) return st;
    if (!workspace || ws_bytes < L.total) return GS_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) return GS_ERR_HIP;
    for (int q = 0; q < n_queries; ++q) {
        uint32_t w[FL_WORDS];
        if (hipMemcpy(w, (const char*)workspace + L.flags + (size_t)q * L.s_flags, sizeof(w),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return GS_ERR_HIP;
        out[q].n_visible = w[FL_NVIS];
        out[q].n_pairs = w[FL_PAIRS];
        out[q].overflow = w[FL_OVERFLOW];
        out[q].n_invalid = w[FL_INVALID];
    }
    return GS_OK;
}

gs_status gs_check(const void* workspace, size_t ws_bytes, int32_t n, int32_t n_queries, const gs_grid* grid,
                   const gs_params* prm, void* stream)
{
    if (n_queries < 1 || n_queries > (1 << 20)) return GS_ERR_INVALID_ARG;
    std::vector<gs_flags> f((size_t)n_queries);
    const gs_status st = gs_read_flags(workspace, ws_bytes, n, n_queries, grid, prm, f.data(), stream);
    if (st != GS_OK) return st;
    bool invalid = false;
    for (const gs_flags& q : f) {
        if (q.overflow) return GS_ERR_CAPACITY;
        invalid = invalid || q.n_invalid != 0;
    }
    return invalid ? GS_ERR_NONFINITE : GS_OK;
}

}  // extern "C"
