/*
 * gsparc.h -- C ABI of the MI355X hemispherical RF Gaussian-splatting renderer.
 *
 * The library renders, for each query (a receiver position, optionally a
 * transmitter position), the directional spectrum of N anisotropic 3D
 * Gaussians on a receiver-centred equirectangular azimuth x elevation grid:
 *
 *   render(gaussians, attrs, rx, grid, channels) -> spectrum[F][H][W]
 *
 * following the paper's problem statement (Sec. 3.3), the projection and
 * projected covariance of Sec. 4.2 and the compositing rule Eq. (3).  The
 * spectrum-to-channel map (spatial mean, Eq. (2)) and the losses of
 * Eq. (4) are separate calls.
 *
 * Conventions for every call
 *  - Pointers are DEVICE pointers unless a comment marks them (host).  The
 *    caller allocates and owns every buffer; the library never allocates
 *    device memory inside these calls and keeps no pointer after a call
 *    returns, except that the workspace carries state from a forward call to
 *    the matching backward call.
 *  - Calls are asynchronous and ordered on `stream` (a hipStream_t passed as
 *    void*; NULL is the default stream).  They return once the work is
 *    enqueued.  Host-side argument errors return at once and enqueue nothing.
 *  - Conditions only the device can see (pair-buffer overflow, non-finite
 *    inputs) are recorded in the workspace's per-query flags and read back
 *    with gs_read_flags(); when a query's overflow flag is set its output is
 *    undefined.
 *  - No call synchronises the stream except gs_read_flags().  Calls are not
 *    thread-safe on one workspace.
 *
 * Data layout (FP32 unless stated)
 *  - Gaussian parameters are structure-of-arrays over n Gaussians:
 *      mean[3][n] (m), log_scale[3][n], quat[4][n] (w, x, y, z; need not be
 *      normalised), opacity_logit[n].
 *    Activations are applied inside the library: scale = exp(log_scale),
 *    rotation from quat/|quat|, opacity = sigmoid(opacity_logit) (Sec. 3.2).
 *  - Attributes: attr[q][n][F][c], c = 2 (interleaved re, im) when complex,
 *    else 1; query q starts at attr + q * query_stride (floats); a stride of
 *    0 shares one attribute set between all queries.
 *  - Spectrum: out[q][F][H][W][c].  Row 0 is the horizon, row H-1 touches the
 *    zenith; column 0 starts at azimuth -pi.  Pixel centres are at
 *    (col + 1/2, row + 1/2).
 */
#ifndef GSPARC_H
#define GSPARC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARG = 1, /* a NULL pointer, a non-positive size, a bad tile shape */
    GS_ERR_WORKSPACE = 2,   /* workspace NULL, misaligned (256 B) or smaller than required */
    GS_ERR_CAPACITY = 3,    /* a size exceeds what the library supports */
    GS_ERR_HIP = 4,         /* a HIP runtime call failed (launch, copy, sync) */
    GS_ERR_NONFINITE = 5    /* gs_check(): a Gaussian with non-finite or degenerate parameters was dropped */
} gs_status;

/* N Gaussians, structure of arrays (see file header). */
typedef struct {
    int32_t n;
    const float* mean;          /* [3][n] */
    const float* log_scale;     /* [3][n] */
    const float* quat;          /* [4][n], (w, x, y, z) */
    const float* opacity_logit; /* [n] */
} gs_scene;

/* Per-Gaussian channel values (the emission s_i of Eq. (3)). */
typedef struct {
    int32_t n_chan;       /* F >= 1 */
    int32_t is_complex;   /* 0: real, 1: complex interleaved (re, im) */
    const float* data;    /* [n_queries or 1][n][F][c] */
    int64_t query_stride; /* floats between queries; 0 = shared */
} gs_attrs;

/* Queries: receiver (grid centre) and optional transmitter positions. */
typedef struct {
    int32_t count;   /* number of queries B >= 1 */
    const float* rx; /* [B][3] device */
    const float* tx; /* [B][3] device, or NULL (then tx = rx) */
} gs_queries;

/* Hemispherical grid.  `view` is V of Sec. 4.2, row-major: t = V (mu - rx),
 * azimuth atan2(t_x, t_z), elevation asin(t_y / |t|).  The default maps world
 * (x, y, z), z up, to (y, z, x). */
typedef struct {
    int32_t H, W;           /* rows (elevation 0..pi/2), columns (azimuth 2 pi) */
    int32_t tile_h, tile_w; /* tile_h * tile_w in {64, 128, 256} */
    double view[9];         /* (host value) */
} gs_grid;

/* Renderer parameters; gs_default_params() fills the defaults. */
typedef struct {
    float alpha_min;   /* a pair with alpha < alpha_min is skipped (1/255) */
    float alpha_max;   /* alpha = min(alpha_max, opacity * G) (0.99) */
    float T_min;       /* stop before a Gaussian that would take T below T_min (1e-4) */
    float dilation;    /* added to both diagonal entries of Sigma', px^2 (0.3) */
    float r_near;      /* Gaussians nearer than this to the receiver are dropped, m (0.2) */
    float atten_power; /* attenuation 1 / max(d, r_near)^p (2) */
    int32_t atten_ref; /* d measured to: 0 the receiver, 1 the transmitter (0) */
    float margin;      /* support-rectangle margin, px (1e-3) */
    int64_t pair_capacity; /* (Gaussian, tile) pairs per query; 0 = n * min(tiles, 64) + 4096 */
    int32_t chan_group;    /* channel floats per blend workgroup (a power of two dividing F*c, at most
                              64; the per-group backward and batched blends use at most 32; the
                              shared-geometry backward takes all columns at once), 0 = automatic:
                              the largest such power of two */
    int32_t options;       /* GS_OPT_* bits (0) */
} gs_params;

/* options: the workspace holds only what the forward needs (no per-pair
 * gradient accumulators, no live-set buffers); gs_render_backward() and
 * gs_render_live() then reject it.  For serving, where the pair
 * accumulators would otherwise be the largest part of the workspace. */
#define GS_OPT_FORWARD_ONLY 1
/* options: the backward takes the per-set, per-channel-group decomposition
 * even where the sets share one geometry (the default there evaluates the
 * geometry once for all sets and channels; both give the same gradients up
 * to summation order).  For comparisons and tests. */
#define GS_OPT_BWD_PER_GROUP 2
/* options: gs_render_blend() takes the per-set, per-channel-group kernel
 * even where the sets share one geometry (the default there walks each
 * pixel once for all sets and forms the channel sums on the matrix cores;
 * the spectra agree to FP32 summation order).  For comparisons and tests. */
#define GS_OPT_BLEND_PER_GROUP 4

/* Per-query device-side results, read with gs_read_flags(). */
typedef struct {
    uint32_t n_visible;  /* Gaussians that survived culling */
    uint32_t n_pairs;    /* (Gaussian, tile) pairs requested */
    uint32_t overflow;   /* 1 if n_pairs > pair_capacity (output undefined) */
    uint32_t n_invalid;  /* Gaussians dropped for non-finite or degenerate values */
} gs_flags;

/* Byte offsets of the workspace sub-buffers for query 0 and the per-query
 * stride of each (for inspection and tests). */
typedef struct {
    size_t total;
    size_t flags, rec, rect, status, tinfo, order, keys, pair_keys, pair_list, ranges;
    size_t T_final, n_last, n_contrib;
    size_t flags_stride, rec_stride, rect_stride, status_stride, tinfo_stride, order_stride,
        keys_stride, pair_keys_stride, pair_list_stride, ranges_stride, pix_stride;
    int64_t pair_capacity;
    int32_t tiles_x, tiles_y;
} gs_layout;

void gs_default_params(gs_params* p);
/* Fills H, W, 16x16 tiles and the default view. */
void gs_default_grid(gs_grid* g, int32_t H, int32_t W);
const char* gs_status_string(gs_status s);

/* Workspace size and layout for n Gaussians, B queries, a grid and params. */
gs_status gs_workspace_layout(int32_t n, int32_t n_queries, const gs_grid* grid,
                              const gs_params* prm, gs_layout* out);

/*
 * Forward render (Sec. 4.2, Eq. (3)) of every query.
 *  spectrum: [B][F][H][W][c], fully written.
 *  workspace: >= gs_layout.total bytes, 256-byte aligned, caller-owned.  It
 *  keeps the per-pixel final transmittance and stop positions, the sorted
 *  tile lists and the projected records for gs_render_backward().
 * Steps enqueued: projection + culling, depth sort, tiles-touched scan,
 * (tile, depth) pair emission, pair sort, tile ranges, tile blending.
 */
gs_status gs_render_forward(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries,
                            const gs_grid* grid, const gs_params* prm, float* spectrum,
                            void* workspace, size_t ws_bytes, void* stream);

/*
 * The two halves of gs_render_forward():
 *  gs_render_prepare: projection + culling, depth sort, tiles-touched scan,
 *    pair emission, pair sort and tile ranges for every query, into the
 *    workspace.
 *  gs_render_blend: compositing (Eq. (3)) of `n_sets` attribute sets over the
 *    prepared workspace.  n_sets == queries prepared: set q uses query q's
 *    geometry.  One prepared query and n_sets > 1: every set shares query 0's
 *    geometry (a fixed receiver seen by many transmitters whose effect is in
 *    the attributes); this requires atten_ref == 0.  `attrs->query_stride`
 *    then steps between sets.  spectrum: [n_sets][F][H][W][c].  The
 *    per-pixel state (T_final, stop position) is per prepared query.
 *  `n_queries` must equal the count passed to gs_render_prepare().
 */
gs_status gs_render_prepare(const gs_scene* scene, const gs_queries* queries, const gs_grid* grid,
                            const gs_params* prm, void* workspace, size_t ws_bytes, void* stream);
gs_status gs_render_blend(const gs_attrs* attrs, int32_t n, int32_t n_queries, int32_t n_sets,
                          const gs_grid* grid, const gs_params* prm, float* spectrum, void* workspace,
                          size_t ws_bytes, void* stream);

/*
 * Backward of gs_render_forward() / gs_render_prepare() + gs_render_blend()
 * (Eq. (3) differentiated; Sec. 4.2 projection differentiated), for the
 * workspace state that call left.  Arguments repeat the forward's (same
 * scene, attrs, queries, n_sets, grid, params) plus:
 *  spectrum    the forward output [S][F][H][W][c]
 *  d_spectrum  dL/dspectrum, same layout
 * Outputs (overwritten, not accumulated):
 *  d_mean [3][n], d_log_scale [3][n], d_quat [4][n], d_opacity_logit [n]:
 *    gradients with respect to the raw parameters, summed over all queries;
 *  d_attr: layout of attrs (one slice when attrs->query_stride == 0, then
 *    summed over sets; else [S][n][F][c]).
 * Per pixel the list is re-walked front to back up to the forward's stop
 * position, recomputing alpha and the transmittance.  Discrete decisions
 * (alpha >= alpha_min, the stop, the alpha_max clamp) are those of the
 * forward; a clamped alpha passes no gradient to opacity or footprint.
 * Where every set shares one prepared query and F*c is a multiple of 16,
 * the walk runs once per pixel for all sets and channels (the per-set terms
 * enter the geometric gradient only through sum_{s,f} g v, formed on the
 * matrix cores, and the attribute gradient only through the set-independent
 * weight T alpha a); otherwise once per set and channel group.  The option
 * GS_OPT_BWD_PER_GROUP forces the second form, and so does a set spectrum
 * of 2^30 or more floats.
 * Float atomics make the summation order, and so the last bits, vary
 * between runs.
 */
#define GS_BWD_ATTR_GRAD_ZEROED 1 /* flags: d_attr is already zero, do not clear it */
gs_status gs_render_backward(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries,
                             int32_t n_sets, const gs_grid* grid, const gs_params* prm, const float* spectrum,
                             const float* d_spectrum, float* d_mean, float* d_log_scale, float* d_quat,
                             float* d_opacity_logit, float* d_attr, int32_t flags, void* workspace,
                             size_t ws_bytes, void* stream);

/*
 * gs_render_backward() for the loss of gs_loss_spectrum() with the gradient
 * assembled inside the kernel, dL/dzhat = E + mean_grad[s][f*c + comp],
 * where the elementwise part E is either read from `partial` (d_partial of
 * gs_loss_spectrum_stats(); one pass over the spectra less than
 * gs_loss_spectrum() + gs_render_backward()) or, when partial is NULL,
 * formed as scale (zhat - z) from the forward output and `target` (no
 * gradient buffer at all; for the loss of gs_loss_spectrum(),
 * scale = 2 / (F H W n_sets)).  lg is a host struct of device pointers;
 * other arguments as for gs_render_backward().
 */
typedef struct {
    const float* partial;   /* E, layout of the spectrum, or NULL */
    const float* target;    /* z (used when partial is NULL) */
    const float* mean_grad; /* [n_sets][F*c] */
    float scale;
} gs_l2_grad;
gs_status gs_render_backward_l2(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries,
                                int32_t n_sets, const gs_grid* grid, const gs_params* prm, const float* spectrum,
                                const gs_l2_grad* lg, float* d_mean, float* d_log_scale, float* d_quat,
                                float* d_opacity_logit, float* d_attr, int32_t flags, void* workspace,
                                size_t ws_bytes, void* stream);

/*
 * Live set of a prepared workspace: walks every pixel's list without
 * attributes (alpha and transmittance only, the discrete decisions of
 * Eq. (3)) and lists, per query, the Gaussians that reach at least one pixel
 * before it stops; no other Gaussian can change the spectrum or receive a
 * gradient.  live_list: [n_queries][list_stride] (order unspecified),
 * live_count: [n_queries] (device).  Also records the per-pixel state that
 * the forward records.
 */
gs_status gs_render_live(int32_t n, int32_t n_queries, const gs_grid* grid, const gs_params* prm,
                         void* workspace, size_t ws_bytes, uint32_t* live_list, int64_t list_stride,
                         uint32_t* live_count, void* stream);

/*
 * Training loss on spectra (Eq. (2) spatial mean, Eq. (4) channel loss).
 * For each of n_sets spectra zhat [F][H][W][c] and targets z (same layout):
 *   h^_f = (1/HW) sum_p zhat_f,p      (coherent mean; re, im separately)
 *   L_b  = (1/(F H W)) sum |zhat - z|^2 + lambda_ch sum_f |h^_f - h_f|^2
 * with h_f the spatial mean of the target.  Writes loss[b] = L_b (device,
 * [n_sets]), h_hat [n_sets][F][c] and d_spectrum = dL/dzhat for
 * L = (1/n_sets) sum_b L_b.  scratch: >= n_sets*F*c*3 floats, 256-byte
 * aligned, caller-owned.
 */
gs_status gs_loss_spectrum(const float* spectrum, const float* target, int32_t n_sets, int32_t n_chan,
                           int32_t is_complex, int32_t H, int32_t W, float lambda_ch, float* loss,
                           float* h_hat, float* d_spectrum, void* scratch, size_t scratch_bytes, void* stream);

/*
 * gs_loss_spectrum() for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no scratch argument.  The per-channel accumulators live in a
 * device array inside the library, GS_LOSS_NOALLOC_MAX_FLOATS floats on each
 * device the library runs on, held until the process ends.  The caller
 * still passes inputs and outputs (as for gs_loss_spectrum()).
 * Errors: those of gs_loss_spectrum(), and GS_ERR_CAPACITY (nothing
 * enqueued) when n_sets * n_chan * c * 3 > GS_LOSS_NOALLOC_MAX_FLOATS;
 * GS_ERR_HIP if the array's device address cannot be found.  Calls share
 * the device's array and leave their sums in it: calls that overlap on one
 * device (different streams) race.  Each call clears what it accumulates.
 */
#define GS_LOSS_NOALLOC_MAX_FLOATS 65536
gs_status gs_loss_spectrum_noalloc(const float* spectrum, const float* target, int32_t n_sets, int32_t n_chan,
                                   int32_t is_complex, int32_t H, int32_t W, float lambda_ch, float* loss,
                                   float* h_hat, float* d_spectrum, void* stream);

/*
 * The loss of gs_loss_spectrum() in one pass over the spectra, for
 * gs_render_backward_l2(): writes loss [n_sets], h_hat [n_sets][F][c],
 * mean_grad [n_sets][F*c] = lambda_ch 2 (h^ - h) / (H W) / n_sets (the
 * channel-mean part of dL/dzhat) and, when d_partial is not NULL,
 * d_partial = 2 (zhat - z) / (F H W n_sets) (the elementwise part, layout
 * of the spectrum) in the same pass.  Same arguments and scratch otherwise.
 */
gs_status gs_loss_spectrum_stats(const float* spectrum, const float* target, int32_t n_sets, int32_t n_chan,
                                 int32_t is_complex, int32_t H, int32_t W, float lambda_ch, float* loss,
                                 float* h_hat, float* mean_grad, float* d_partial, void* scratch,
                                 size_t scratch_bytes, void* stream);

/*
 * Magnitude-spectrum loss, Eq. (5), for real spectra zhat, z
 * [n_sets][F][H][W] (e.g. magnitude spectra):
 *   L_b = (1 - lambda_1) L1_b + lambda_1 (1 - SSIM_b)
 * with L1_b the mean |zhat - z| over channels and pixels and SSIM_b the mean
 * structural similarity (Wang et al.): an 11 x 11 Gaussian window, sigma
 * 1.5, normalised, applied as a same-size filter with zero padding (no wrap
 * at the azimuth seam), C1 = 0.01^2, C2 = 0.03^2 (a dynamic range of 1), the
 * map averaged over channels and pixels.  The paper takes lambda_1 = 0.2.
 * Writes loss [n_sets], and when not NULL ssim [n_sets], l1 [n_sets] and
 * d_spectrum = dL/dzhat for L = (1/n_sets) sum_b L_b (layout of zhat; the
 * L1 term contributes 0 where zhat = z).  scratch: >=
 * gs_loss_l1_ssim_scratch_bytes() bytes, 256-byte aligned, caller-owned
 * (one pair of partial sums per 32 x 16 tile and channel, summed in a fixed
 * order: deterministic).  Errors: GS_ERR_INVALID_ARG (null input, a
 * non-positive size, lambda_1 outside [0, 1]), GS_ERR_CAPACITY (n_sets * F >
 * 65535), GS_ERR_WORKSPACE.
 */
size_t gs_loss_l1_ssim_scratch_bytes(int32_t n_sets, int32_t n_chan, int32_t H, int32_t W);
gs_status gs_loss_l1_ssim(const float* spectrum, const float* target, int32_t n_sets, int32_t n_chan, int32_t H,
                          int32_t W, float lambda_1, float* loss, float* ssim, float* l1, float* d_spectrum,
                          void* scratch, size_t scratch_bytes, void* stream);

/*
 * Spectrum-to-channel map, Eq. (2): h[s][f][c] = (1/(H W)) sum_p z[s][f][p][c]
 * for spectra z [n_sets][F][H][W][c] (c = 2 when complex: real and
 * imaginary parts separately).  h: [n_sets][F][c] (device, overwritten).
 * Deterministic (fixed summation order).  Errors: GS_ERR_INVALID_ARG for a
 * null pointer, a non-positive size or a complex spectrum not 8-byte
 * aligned; GS_ERR_CAPACITY for n_chan or n_sets above 65535.
 */
gs_status gs_spatial_mean(const float* spectrum, int32_t n_sets, int32_t n_chan, int32_t is_complex, int32_t H,
                          int32_t W, float* h, void* stream);

/*
 * One fused training pass over S complex attribute sets that share one
 * prepared receiver (the transmitter batch of the training step): Eq. (3)
 * compositing, the loss of gs_loss_spectrum() against targets z (pixel term
 * plus the Eq. (4) channel term on the Eq. (2) means) and its backward,
 * without materialising the spectra or their gradient.
 *
 * Preconditions: the workspace was prepared for queries->count == 1 with
 * atten_ref == 0 (gs_render_prepare) and then walked by gs_render_live()
 * (its stop positions, live list and per-Gaussian weight sums are used);
 * attrs complex with 2 F a multiple of 16; attrs->query_stride 0 (one
 * shared set) or >= n * 2F.
 * tt (host struct of device pointers):
 *   target       z [S][F][H][W][2];
 *   target_mean  h [S][F][2] = Eq. (2) of the target (gs_spatial_mean), a
 *                property of each training sample;
 *   lambda_ch    weight of the channel term;
 *   loss [S], h_hat [S][F][2]: outputs (per-set loss, Eq. (2) of the
 *                rendered spectra, formed from the live pass's per-Gaussian
 *                weight sums: h_hat = (1/HW) sum_g (sum_p w_g(p)) v_g).
 *   grad_scale   NULL, or a device float c: every gradient output is that
 *                of c L (the loss outputs stay those of L).  The
 *                confidence-weighted objective of Eq. (6) with the sets'
 *                shared receiver: c = C(x_rx) from gs_confidence_loss().
 * spectrum: [S][F][H][W][2], written in full with GS_TRAIN_WRITE_SPECTRUM
 *   (bit-identical to gs_render_blend()), else used only for the groups of
 *   64 pixels whose walk exceeds 256 list entries (those take the unfused
 *   compositing and backward kernels inside this call).
 * Gradient outputs as for gs_render_backward() for L = (1/S) sum_b L_b
 * (d_attr cleared first unless GS_BWD_ATTR_GRAD_ZEROED).
 * scratch: >= gs_train_scratch_bytes(n_sets, F, grid) bytes, 256-byte
 *   aligned, caller-owned (GV partials, loss partials, the mean term).
 * Errors: GS_ERR_INVALID_ARG (null pointer, an unsupported shape above,
 * unknown flag bits), GS_ERR_WORKSPACE, GS_ERR_CAPACITY (also when one set's
 * attributes, n 2F floats, or one set's spectrum, 2F H W floats, reach 2^29:
 * the kernels address them with 32-bit byte offsets); nothing is enqueued
 * on an argument error.  Float atomics make the last bits of the gradients
 * vary between runs.
 * Streams: the walk classes of up to 256 and 128 entries run on two of the
 * library's side streams of the device (those of gs_batch_run(), created on
 * first use outside graph capture), forked from and joined back into
 * `stream` with events inside the call; a graph capture of the call records
 * them as parallel branches.  Before the side streams exist (first call
 * under capture) everything runs on `stream`.
 */
typedef struct {
    const float* target;
    const float* target_mean;
    float lambda_ch;
    float* loss;
    float* h_hat;
    const float* grad_scale;
} gs_train_target;
#define GS_TRAIN_WRITE_SPECTRUM 2 /* flags: also store the spectra */
/* flags: leave the per-pair fold and the projection backward (the outputs
 * d_mean, d_log_scale, d_quat, d_opacity_logit) to a later
 * gs_render_train_geometry() on the same workspace, e.g. on a second stream
 * beside the network backward, which needs only d_attr and the loss. */
#define GS_TRAIN_DEFER_GEOMETRY 4
size_t gs_train_scratch_bytes(int32_t n_sets, int32_t n_chan, const gs_grid* grid);
gs_status gs_render_train(const gs_scene* scene, const gs_attrs* attrs, const gs_queries* queries, int32_t n_sets,
                          const gs_grid* grid, const gs_params* prm, const uint32_t* live_list,
                          const uint32_t* live_count, const gs_train_target* tt, float* spectrum, float* d_mean,
                          float* d_log_scale, float* d_quat, float* d_opacity_logit, float* d_attr, int32_t flags,
                          void* workspace, size_t ws_bytes, void* scratch, size_t scratch_bytes, void* stream);
/* The geometric tail of a gs_render_train() call made with
 * GS_TRAIN_DEFER_GEOMETRY (Sec. 4.2, the backward through the projection):
 * folds the per-pair geometric sums that call left in the workspace per
 * Gaussian and runs the projection backward into d_mean [3][n],
 * d_log_scale [3][n], d_quat [4][n], d_opacity_logit [n] (overwritten).
 * Same scene, queries (one receiver), grid, params and workspace as that
 * call; it must run after it (stream order or an event) and before the
 * workspace is prepared again.  Errors: GS_ERR_INVALID_ARG,
 * GS_ERR_WORKSPACE. */
gs_status gs_render_train_geometry(const gs_scene* scene, const gs_queries* queries, const gs_grid* grid,
                                   const gs_params* prm, float* d_mean, float* d_log_scale, float* d_quat,
                                   float* d_opacity_logit, void* workspace, size_t ws_bytes, void* stream);

/*
 * gs_render_blend() with the loss of gs_loss_spectrum_stats() fused into its
 * output stage (Eq. (3) compositing, then Eq. (2) spatial means and Eq. (4)
 * channel loss): as each spectrum element is written the kernel reads the
 * target element, writes the elementwise gradient part to d_partial (when
 * not NULL) and adds the per-channel sums the loss needs; a small second
 * kernel forms loss, h_hat and mean_grad.  Same results as gs_render_blend()
 * followed by gs_loss_spectrum_stats() (the spectrum and d_partial
 * bit-identical, the loss sums up to float summation order), without a
 * second pass over the spectrum.  Arguments: those of gs_render_blend(),
 * then target [n_sets][F][H][W][c] (device), lambda_ch, and the outputs of
 * gs_loss_spectrum_stats().  scratch (device, 256-byte aligned, caller-
 * owned) holds the loss sums and one partial sum per wave: at least
 * align256(n_sets*F*c*3*4) + n_sets*F*c*3 * tiles * (tile_h*tile_w/64) * 4
 * bytes (tiles = ceil(H/tile_h) * ceil(W/tile_w)).  Errors as for either
 * call; nothing is enqueued on an argument error.
 */
gs_status gs_render_blend_loss(const gs_attrs* attrs, int32_t n, int32_t n_queries, int32_t n_sets,
                               const gs_grid* grid, const gs_params* prm, float* spectrum, void* workspace,
                               size_t ws_bytes, const float* target, float lambda_ch, float* loss, float* h_hat,
                               float* mean_grad, float* d_partial, void* scratch, size_t scratch_bytes,
                               void* stream);

/* ---- attribute network (shared form of the emission predictor, Eq. (1)) ----
 * Per (set s, Gaussian g):  h1 = relu(W1 [e_g, gamma(tx_s), 0] + b1),
 * h2 = relu(W2 h1 + b2), o = W3 h2 + b3, A_f = sigmoid(o_f - ln d),
 * phi_f = o_{64+f}, attr = A e^{j phi}, d = max(|tx_s - mu_g|, r_near);
 * gamma = Fourier features (u, sin 2^k pi u, cos 2^k pi u), k = 0..7, u the
 * transmitter scaled to [-1, 1] by the box.  Shapes: embedding 32, input
 * padded to 96, hidden 64, F = n_chan complex subcarriers (32 or 64), so
 * 2F outputs.  Weights are BF16 ([out][in] row-major), biases FP32;
 * products run on BF16 matrix cores with FP32 accumulation.  Errors:
 * GS_ERR_INVALID_ARG also for n_chan not 32 or 64. */
typedef struct {
    const uint16_t* W1; /* bf16 [64][96] */
    const float* b1;    /* [64] */
    const uint16_t* W2; /* bf16 [64][64] */
    const float* b2;    /* [64] */
    const uint16_t* W3; /* bf16 [2F][64]: rows 0..F-1 amplitudes, F..2F-1 phases */
    const float* b3;    /* [2F] */
    float box_lo[3], box_hi[3]; /* (host values) encoding box */
    float r_near;               /* distance floor of the log-distance bias, m */
    int32_t n_chan;             /* F: 32 or 64 */
} gs_mlp;

/* Rows to evaluate: for set s, the Gaussians list[s*list_stride + i],
 * i < count[count_stride ? s : 0] (device count, so the list can come from a
 * device-side pass).  row_cap: rows per set the saved-activation buffers
 * hold (>= every count).  grid_x: workgroups per set, each taking 64 rows
 * per round (0 = 32). */
typedef struct {
    int32_t n_sets;
    const float* tx;        /* [S][3] */
    const uint32_t* list;   /* Gaussian indices */
    int64_t list_stride;
    const uint32_t* count;
    int32_t count_stride;
    int64_t row_cap;
    int32_t grid_x;
} gs_mlp_rows;

/* Caller-owned scratch of the network calls.  For inference only cb is
 * needed (save_* may be NULL); training needs every buffer. */
typedef struct {
    float* cb;           /* [S][64] per-set first-layer bias */
    uint16_t* genc;      /* [S][64] bf16 encodings (training) */
    uint16_t* save_h1;   /* [S][row_cap][64] bf16 */
    uint16_t* save_h2;   /* [S][row_cap][64] bf16 */
    uint16_t* save_do;   /* [S][row_cap][128] bf16 */
    uint16_t* save_dz2;  /* [S][row_cap][64] bf16 */
    uint16_t* save_dz1;  /* [S][row_cap][64] bf16 */
    float* dc;           /* [S][64] */
    uint16_t* wT;        /* 32*64 + 64*64 + 64*128 bf16 transposed weights */
    float* partial;      /* n_partial * (128*64 + 64*64 + 64*32) floats (the three weight gradients) */
    int32_t n_partial;   /* split-K workgroups of the weight gradients */
} gs_mlp_state;

typedef struct {
    float *dW1, *db1, *dW2, *db2, *dW3, *db3; /* FP32, shapes of the weights */
    float* dE;                                /* [n][32] */
} gs_mlp_grads;

/* Z1 = E W1[:, :32]^T: the query-independent part of the first layer.
 * E: bf16 [n][32]; Z1: FP32 [n][64]. */
gs_status gs_mlp_embed(const gs_mlp* net, const uint16_t* E, int32_t n, float* Z1, void* stream);
/* Attributes of the listed rows into attr[s * attr_stride + g*2F ...]
 * ([S][n][F][2] for attr_stride = n*2F); other rows untouched.  With
 * st->save_h1/save_h2 set, keeps the activations for gs_mlp_backward(). */
gs_status gs_mlp_forward(const gs_mlp* net, const float* Z1, const float* mean, int32_t n,
                         const gs_mlp_rows* rows, float* attr, int64_t attr_stride, gs_mlp_state* st,
                         void* stream);
/* Gradients of sum(d_attr * attr) over the listed rows (same rows as the
 * forward that saved the activations).  All outputs overwritten.  With
 * clear_d_attr set, the listed rows of d_attr are zeroed after use (so a
 * buffer that only those rows ever touch stays zero between steps). */
gs_status gs_mlp_backward(const gs_mlp* net, const uint16_t* E, const float* mean, int32_t n,
                          const gs_mlp_rows* rows, float* d_attr, int64_t attr_stride, int32_t clear_d_attr,
                          gs_mlp_state* st, gs_mlp_grads* grads, void* stream);

/* ---- fused Adam over parameter segments (Kingma and Ba) ----
 * For each segment: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); when shadow is
 * set, shadow = bf16(p).  Segments are described on the host (at most 16).
 * skip_if (device, or NULL): when the word it points to is non-zero at run
 * time, nothing is updated and *skip_count (device, or NULL) is incremented
 * -- e.g. the overflow word of the render workspace, so that a step whose
 * pair buffer overflowed (its spectra and gradients undefined) changes no
 * parameter, without a host synchronisation.  Errors: GS_ERR_INVALID_ARG
 * for a null segment pointer, a negative count, n_segs outside [1, 16],
 * step < 1 or beta / eps out of range. */
typedef struct {
    float* p;
    const float* g;
    float* m;
    float* v;
    uint16_t* shadow; /* optional bf16 copy of p */
    int64_t count;
    float lr;
} gs_adam_segment;
gs_status gs_adam_step(const gs_adam_segment* segs /*(host)*/, int32_t n_segs, int32_t step, float beta1,
                       float beta2, float eps, const uint32_t* skip_if, uint32_t* skip_count, void* stream);

/* gs_adam_step() with the step number and learning-rate schedule on the
 * device, so that a captured graph of a training step replays correctly:
 * *step_counter (device) holds the number of completed steps t; the update
 * uses bias corrections for step t + 1 and, for segment k with
 * lr_final[k] != segs[k].lr (lr_final a host array, or NULL for constant
 * rates), the rate lr (lr_final / lr)^u with u = min((t + 1) / (total_steps - 1), 1)
 * (the log-linear decay of the position rate, Table 2); then *step_counter
 * is incremented (also when skip_if skips the update).  Errors as for
 * gs_adam_step(), and GS_ERR_INVALID_ARG for a null step_counter,
 * total_steps < 1 or a scheduled rate that is not positive. */
gs_status gs_adam_step_scheduled(const gs_adam_segment* segs /*(host)*/, const float* lr_final /*(host)*/,
                                 int32_t n_segs, int32_t total_steps, uint32_t* step_counter, float beta1,
                                 float beta2, float eps, const uint32_t* skip_if, uint32_t* skip_count,
                                 void* stream);

/* Device address of query q's overflow word in a workspace laid out for
 * (n, n_queries, grid, prm): for gs_adam_step's skip_if.  Host-side only. */
gs_status gs_overflow_word(const void* workspace, size_t ws_bytes, int32_t n, int32_t n_queries,
                           const gs_grid* grid, const gs_params* prm, int32_t q, const uint32_t** word);

/* ---- confidence head and confidence-weighted loss (Sec. 4.2, Eq. (6)) ----
 * Per sample b (receiver position x_rx[b][3], task loss task_loss[b]):
 *   h = relu(W1 x + b1) (32 units; hidden activation: a reading, the paper
 *   names none), g = w2 . h + b2, C = 1 + exp(g) > 1,
 *   loss[b] = C task_loss[b] - alpha log C;  conf[b] = C, which is also
 *   d loss[b] / d task_loss[b] (the factor on the task loss gradient).
 * Gradients of sum_b loss[b]: dW1 [32][3], db1 [32], dw2 [32], db2 [1],
 * overwritten.  Layout: W1 row-major [32][3], all FP32 device pointers,
 * caller-owned; the paper's alpha is 0.3.  Up to 4096 samples one
 * workgroup does everything (scratch may be NULL); beyond, up to 1024
 * workgroups write partial gradient sums to `scratch` (>=
 * gs_confidence_scratch_bytes(n) bytes, 256-byte aligned, caller-owned
 * device memory, its contents not needed before or after the call) and one
 * more workgroup adds them.  Either way the weight gradients are summed in
 * an order fixed by n alone (deterministic).
 * Errors: GS_ERR_INVALID_ARG for a null pointer, n < 1 or alpha negative or
 * not finite; GS_ERR_CAPACITY for n > 2^24; GS_ERR_WORKSPACE for missing,
 * misaligned or short scratch when n > 4096. */
/* ---- the paper's own emission form: one network per Gaussian (Sec. 4.1, Eq. (1)) ----
 * Gaussian i owns a 3 -> H -> 2 network, H = hidden in {8, 16, 64} (16 in
 * the paper, 8 and 64 in its width ablation): 6H + 2 FP32 parameters, stored
 * as params[k * param_stride + i], k = W1 [H][3] row-major, b1 [H],
 * W2 [2][H] row-major, b2 [2]; param_stride >= n.  For query q (receiver rx[q][3],
 * transmitter tx[q][3], device pointers):
 *   h = relu(W1 rx + b1) (hidden activation: a reading, the paper names
 *   none), f = W2 h + b2, d = max(|tx - mean_i|, r_near),
 *   attr[q * attr_query_stride + 2 i + {0, 1}] = sigmoid(f - log d) (Re, Im),
 * i.e. one complex channel per Gaussian in the attribute layout of the
 * renderer.  mean [3][n] (the scene's layout).  All pointers are
 * caller-owned device memory.
 * The backward takes d_attr in the same layout and writes (overwrites) the
 * gradients of sum(d_attr * attr) with respect to the parameters (d_params,
 * same layout as params) and the means (d_mean [3][n]), summed over queries.
 * Errors: GS_ERR_INVALID_ARG for a null pointer, hidden not 8, 16 or 64,
 * n < 1, n_queries < 1, param_stride < n, attr_query_stride < 2 n or odd,
 * r_near not positive and finite; GS_ERR_CAPACITY for n_queries > 1024. */
gs_status gs_emission_forward(const float* params, int64_t param_stride, int32_t hidden, const float* mean, int32_t n,
                              const float* rx, const float* tx, int32_t n_queries, float r_near, float* attr,
                              int64_t attr_query_stride, void* stream);
gs_status gs_emission_backward(const float* params, int64_t param_stride, int32_t hidden, const float* mean, int32_t n,
                               const float* rx, const float* tx, int32_t n_queries, float r_near,
                               const float* d_attr, int64_t attr_query_stride, float* d_params, float* d_mean,
                               void* stream);

size_t gs_confidence_scratch_bytes(int32_t n); /* 0 when n <= 4096 or n > 2^24 */
gs_status gs_confidence_loss(const float* x_rx, const float* task_loss, int32_t n, const float* W1,
                             const float* b1, const float* w2, const float* b2, float alpha, float* conf,
                             float* loss, float* dW1, float* db1, float* dw2, float* db2, void* scratch,
                             size_t scratch_bytes, void* stream);

/* ---- adaptive densification, pruning and opacity reset (Sec. 4.2, Algorithm 1) ----
 * Statistics (gs_densify_stats, after a step's backward): for every Gaussian
 * i in the live list, grad_acc[i] += |d_mean[:, i]| (d_mean [3][n]) and
 * grad_cnt[i] += 1.  The caller zeroes both after each densification.
 *
 * Plan (gs_densify_plan): per Gaussian i (scene arrays in the scene's
 * layout; screen_radius [n] from gs_screen_radius, or NULL for no size
 * pruning), with FP32 decisions
 *   densify = grad_cnt > 0 and grad_acc / grad_cnt >= grad_threshold,
 *   small   = max_c exp(log_scale[c]) <= clone_extent (epsilon r_scene),
 *   faint   = sigmoid(opacity_logit) < opacity_min,
 *   large   = screen_radius > radius_max,
 * i yields: not densified: itself unless faint or large; small: itself
 * unless faint or large, then its clone unless faint; otherwise split_n
 * children unless faint (i leaves).  (Reading: Algorithm 1's prune runs over
 * the densified set and the new Gaussians have no screen radius yet.)
 * Output slot j: src[j] = parent, kind[j] = -1 (the parent itself), -2 (a
 * clone) or the child number; slots in parent order (deterministic).
 * n_out (device u32) = the new count.  src, kind: device int32 arrays of
 * out_capacity >= n * split_n entries; scratch >=
 * gs_densify_scratch_bytes(n), 256-byte aligned.
 *
 * Apply (gs_densify_apply, n_out read back by the caller): the new scene
 * arrays ([3][n_out], [4][n_out], [n_out]): copies of the parents, split
 * children at mean + R(q) (exp(log_scale) * xi) with xi [n][split_n][3] the
 * caller's standard normals (parent i, child k), log_scale - log(0.8
 * split_n) (the paper's Sigma / (0.8 N), read as on the scale).
 * Gather (gs_densify_gather): any per-Gaussian array [comps][n][width_words]
 * of 32-bit words to [comps][n_out][width_words] in the new order; with
 * zero_new, the rows of clones and children are zero (fresh Adam moments).
 * Opacity reset (gs_opacity_reset): opacity_logit <- min(opacity_logit,
 * logit(opacity_cap)), the paper's sigma <- min(sigma, 0.01).
 * All pointers are caller-owned device memory.  Errors: GS_ERR_INVALID_ARG
 * for a null pointer, n < 1, split_n outside [2, 64] or a threshold that is
 * not positive (grad_threshold, radius_max) or negative (clone_extent,
 * opacity_min); GS_ERR_CAPACITY when n * split_n >= 2^31; GS_ERR_WORKSPACE
 * for a short src/kind capacity or scratch. */
typedef struct {
    float grad_threshold; /* tau_grad on the mean |dL/dmu| over the steps a Gaussian was live */
    float clone_extent;   /* epsilon * r_scene */
    int32_t split_n;      /* N children of a split */
    float opacity_min;    /* sigma_min */
    float radius_max;     /* r_max, pixels */
} gs_densify_params;
gs_status gs_densify_stats(const float* d_mean, int32_t n, const uint32_t* live_list, const uint32_t* live_count,
                           float* grad_acc, uint32_t* grad_cnt, void* stream);
size_t gs_densify_scratch_bytes(int32_t n);
gs_status gs_densify_plan(int32_t n, const float* log_scale, const float* opacity_logit, const float* grad_acc,
                          const uint32_t* grad_cnt, const float* screen_radius, const gs_densify_params* prm,
                          int32_t* src, int32_t* kind, int64_t out_capacity, uint32_t* n_out, void* scratch,
                          size_t scratch_bytes, void* stream);
gs_status gs_densify_apply(int32_t n, int32_t n_out, const int32_t* src, const int32_t* kind, const gs_scene* scene,
                           const float* xi, int32_t split_n, float* o_mean, float* o_log_scale, float* o_quat,
                           float* o_opacity_logit, void* stream);
gs_status gs_densify_gather(int32_t n, int32_t n_out, const int32_t* src, const int32_t* kind, const void* in,
                            void* out, int32_t comps, int32_t width_words, int32_t zero_new, void* stream);
gs_status gs_opacity_reset(int32_t n, float* opacity_logit, float opacity_cap, void* stream);
/* Screen radius of every Gaussian for query q of a prepared workspace: half
 * the larger side of its support rectangle in pixels, 0 if culled. */
gs_status gs_screen_radius(const void* workspace, size_t ws_bytes, int32_t n, int32_t n_queries,
                           const gs_grid* grid, const gs_params* prm, int32_t q, float* radius, void* stream);

/*
 * Batched serving: many queries over several scenes of uneven size, grid,
 * tile shape and channel count in one persistent blend launch.
 *
 * A job is one scene with a group of queries (receiver positions; n_sets =
 * queries.count, set q seen from query q) and its own grid, params, output
 * and workspace, exactly as for gs_render_forward() (GS_OPT_FORWARD_ONLY is
 * allowed and saves memory); no two jobs may share a workspace.
 * gs_batch_run() enqueues the prepare steps of gs_render_prepare() for every
 * job, spread over the caller's stream and up to three side streams of the
 * library (each job to the stream with the least Gaussians x queries so far;
 * forked from and joined back into the caller's stream with events, so a
 * graph capture records them as parallel branches), then one persistent
 * blend kernel whose workgroups pull (job, query, channel group, tile) items
 * from a device counter in job order, so the job order is the service order.
 * Spectra and workspace state are those that gs_render_forward() leaves for
 * the same job, bit for bit.
 *
 *  gs_batch_plan_bytes(n_jobs): size of the plan buffer (device, 256-byte
 *    aligned, caller-owned).
 *  gs_batch_plan: validates the jobs (host array), writes the job table into
 *    the plan buffer and fills *info (host).  Synchronises `stream` (the
 *    table is copied from host memory).  Creates the side streams of the
 *    current device on its first call there (kept until the process ends).
 *    Call again whenever any job field changes; the plan holds device
 *    pointers of the jobs' buffers.
 *  gs_batch_run: enqueues the batch for a plan made from the same jobs.
 *    Enqueues kernels only (no copies, no memset, no allocation, no host
 *    synchronisation), so it can be captured into a HIP graph and replayed.
 *    workgroups: persistent workgroups (> 0; info->workgroups fills the
 *    device at the kernel's occupancy).  timestamps: NULL, or a device array
 *    of info->n_queries + 3 uint64 values written as device wall-clock ticks
 *    (gs_wall_clock_khz()): [0] batch start (before the first prepare),
 *    [1 + k] completion of the k-th query's spectrum (queries numbered job
 *    by job), [n_queries + 1] batch end, [n_queries + 2] end of the prepare
 *    steps (start of the blend).  With one job, or under a graph capture
 *    before the side streams exist, every prepare runs on `stream`.
 *  Concurrent runs of one plan race on its work counter; runs enqueued from
 *  several host threads take turns on the side streams (a lock), and runs on
 *  different caller streams of one device are ordered through them.
 */
typedef struct {
    gs_scene scene;
    gs_attrs attrs;
    gs_queries queries;
    gs_grid grid;
    gs_params params;
    float* spectrum;        /* [queries.count][F][H][W][c] */
    void* workspace;        /* >= gs_workspace_layout(...).total bytes */
    size_t workspace_bytes;
} gs_batch_job;

typedef struct {
    int64_t items;       /* blend work items of the batch */
    int32_t n_queries;   /* queries over all jobs */
    int32_t block;       /* threads per workgroup: the largest tile's pixels */
    int32_t workgroups;  /* workgroups that fill the device at full occupancy */
    int32_t reserved;
} gs_batch_info;

size_t gs_batch_plan_bytes(int32_t n_jobs);
gs_status gs_batch_plan(const gs_batch_job* jobs, int32_t n_jobs, void* plan, size_t plan_bytes,
                        gs_batch_info* info, void* stream);
gs_status gs_batch_run(const gs_batch_job* jobs, int32_t n_jobs, void* plan, size_t plan_bytes,
                       int32_t workgroups, uint64_t* timestamps, void* stream);
/*
 * Kernel timing for benchmarks.  While enabled, the library records a HIP
 * event pair on the launching stream around every launch of the timed
 * kernels: GS_TIMER_BLEND (the compositing kernel of gs_render_forward /
 * gs_render_blend) and GS_TIMER_BLEND_BWD (the compositing backward of
 * gs_render_backward*).  gs_timing_read synchronises on the recorded
 * events, returns the summed milliseconds and launch count since the last
 * read, and resets them.  Off by default; not for use under graph capture.
 */
#define GS_TIMER_BLEND 0
#define GS_TIMER_BLEND_BWD 1
#define GS_TIMER_TRAIN 2 /* the fused kernels of gs_render_train() (both, as one interval) */
gs_status gs_timing_enable(int32_t on);
gs_status gs_timing_read(int32_t kernel, double* total_ms, int64_t* launches);

/* Device wall-clock rate (kHz) of the current device, for the timestamps. */
gs_status gs_wall_clock_khz(int32_t* khz);

/*
 * Copies the per-query flags of the last forward call into `out` (host,
 * [B] entries).  Synchronises `stream`.
 */
gs_status gs_read_flags(const void* workspace, size_t ws_bytes, int32_t n, int32_t n_queries,
                        const gs_grid* grid, const gs_params* prm, gs_flags* out, void* stream);

/*
 * Synchronises `stream` and reports the device-side conditions of the last
 * prepare/forward on the workspace: GS_ERR_CAPACITY if any query's pair
 * buffer overflowed (its outputs are undefined; raise pair_capacity), else
 * GS_ERR_NONFINITE if any Gaussian was dropped for non-finite or degenerate
 * parameters (the rest rendered normally), else GS_OK.  Argument errors as
 * for gs_read_flags().
 */
gs_status gs_check(const void* workspace, size_t ws_bytes, int32_t n, int32_t n_queries, const gs_grid* grid,
                   const gs_params* prm, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GSPARC_H */
