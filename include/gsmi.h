/*
 * gsmi — differentiable 16x16-tile Gaussian-splatting rasterizer with
 * view-level active-set reduction, for AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Conventions shared by every entry point:
 *  - Array pointers are DEVICE pointers owned by the caller; the library never
 *    allocates, frees or keeps them.  Structs (gs_scene, gs_camera, ...) are
 *    HOST memory read during the call only.
 *  - Layouts are structure-of-arrays, component-major: a [C][n] array holds
 *    component c of element i at index c*n + i.  Images are [3][H][W] float32,
 *    per-pixel maps [H][W].  Bitmaps hold bit i in bit (i % 32) of 32-bit word
 *    i / 32.
 *  - Every call is asynchronous on `stream` (NULL = the null stream).  Counts
 *    the host may want (pairs, active Gaussians) are written to device int64
 *    slots; reading them is the caller's only synchronisation.
 *  - Scratch memory is a caller-owned device workspace `ws` of `ws_bytes`
 *    bytes (256-byte aligned), sized with gs_workspace_size().  Its contents
 *    are undefined between calls; calls that share one workspace must not
 *    overlap.
 *  - Return value: GS_OK or a negative GS_ERR_* code; nothing aborts or
 *    throws.  gs_last_error() returns a thread-local message for the last
 *    failing call.  Argument checks happen on the host before any launch; a
 *    call that returns an error has launched nothing.
 *
 * The rasterizer follows the paper's 3DGS preliminaries (Appendix A, the
 * Gaussian-kernel and the front-to-back alpha-compositing equations) with the
 * standard constants of the 3DGS rasterizer it keeps: 16x16 tiles, 64-bit
 * (tile | depth) keys, alpha = min(0.99, o G), Gaussians with alpha < 1/255
 * skipped, a pixel stops before its transmittance would fall below 1e-4,
 * 0.3 px^2 screen-space dilation, 3-sigma radius, SH degree 3.
 */
#ifndef GSMI_H
#define GSMI_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARG = -1, /* null/misaligned pointer, bad size or count */
    GS_ERR_CAPACITY = -2,    /* not returned by the asynchronous calls: a pair-buffer overflow is
                                only known on the device and is reported through the device count
                                (gs_bin_sort: *n_pairs_dev > capacity, every tile range empty) */
    GS_ERR_WORKSPACE = -3,   /* ws_bytes below gs_workspace_size() */
    GS_ERR_HIP = -4          /* a HIP launch failed; see gs_last_error() */
};

#define GS_TILE 16
#define GS_SH_COEFFS 16
#define GS_MAX_CAMS 8
#define GS_MAX_PAIRS ((int64_t)1 << 30)

/* Pinhole camera.  x_cam = R x_world + t (R row-major, rows = camera right,
 * down, forward).  Pixel (u, v) samples the image plane at (u+0.5, v+0.5);
 * Gaussians with camera depth <= znear are culled. */
typedef struct gs_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float znear;
} gs_camera;

/* Gaussian parameters, before activation (Sec. 3 "standard 3DGS
 * parameterization"): scale = exp(log_scale), rotation = normalised quat
 * (w, x, y, z), opacity = sigmoid(opacity_logit), colour = SH degree 3. */
typedef struct gs_scene {
    int64_t n;
    const float* mean;          /* [3][n] */
    const float* log_scale;     /* [3][n] */
    const float* quat;          /* [4][n] */
    const float* opacity_logit; /* [n] */
    const float* sh;            /* [16][3][n] (coefficient, channel, Gaussian) */
    const uint8_t* lod;         /* [n] level labels, or NULL */
} gs_scene;

/* Projection of one camera's input list (entry j = Gaussian active_idx[j]).
 * `rec` is required: the packed per-Gaussian render record, 12 floats,
 * 16-byte aligned: (mx, my, conic_a, conic_b), (conic_c, opacity, r, g),
 * (b, depth, 0, 0).  The component-major copies (mean2d .. rgb) are optional
 * (NULL = not written).  Culled entries get radius 0, tiles_touched 0,
 * depth 0, clamp bits 0 and zeros in the optional arrays; their `rec` is not
 * written. */
typedef struct gs_projected {
    float* rec;               /* [n][12] required */
    float* depth;             /* [n] required */
    int32_t* radius;          /* [n] required */
    uint32_t* tiles_touched;  /* [n] required */
    uint8_t* clamp_bits;      /* [n] required; bit c: colour channel c clamped at 0 */
    float* mean2d;            /* [2][n] optional */
    float* conic;             /* [3][n] optional */
    float* opacity;           /* [n] optional */
    float* rgb;               /* [3][n] optional */
} gs_projected;

/* Parameter gradients, same layouts as gs_scene.  overwrite = 0: the
 * backward adds (+=) into them.  overwrite = 1: the gradients of the
 * Gaussians the backward reaches (visible in some camera of the call) are
 * stored (=) instead, which saves reading them; for callers whose gradient
 * arrays hold zeros there (e.g. cleared by gs_adam_step), where both give the
 * same result.  Gaussians the call does not reach are untouched either way. */
typedef struct gs_grads {
    float* mean;
    float* log_scale;
    float* quat;
    float* opacity_logit;
    float* sh;
    int32_t overwrite;
} gs_grads;

enum { GS_LOD_NONE = 0, GS_LOD_LEVEL = 1, GS_LOD_RADIUS = 2 };

typedef struct gs_lod_params {
    int32_t mode;          /* GS_LOD_NONE | GS_LOD_LEVEL | GS_LOD_RADIUS */
    float d0;              /* level mode: reference camera-to-scene distance */
    float f;               /* level mode: ratio between levels (2) */
    int32_t l_max;         /* level mode: unlocked ceiling L_max(t) */
    float fallback_ratio;  /* skip the gate when it keeps >= this share (0.95) */
    float radius_min_px;   /* radius mode: keep r >= this (0.5) */
    float radius_sigma_k;  /* radius mode: r = k fx max_j s_j / |mu - c| (1) */
} gs_lod_params;

enum {
    GS_OP_LOD_MASK = 0,
    GS_OP_BIN_SORT = 1,
    GS_OP_RENDER_BWD = 2,
    GS_OP_IMPORTANCE = 3,
    GS_OP_SCORE_KEEP = 4,
    GS_OP_L1_LOSS = 5,
    GS_OP_SIMPLIFY = 6,
    GS_OP_PHOTO_LOSS = 7, /* n = width * 65536 + height */
    GS_OP_SCALE_REG = 8,
    GS_OP_PROJECT = 9,
    GS_OP_VOXEL_LEVELS = 10,
    GS_OP_SPAWN_GATE = 11 /* n = max(n_clone, n_split) */
};

/* Bytes of workspace `op` needs for n Gaussians (per camera), n_pairs pair
 * capacity, n_tiles tiles over all cameras and n_cams cameras.  Arguments an
 * op does not use are ignored. */
size_t gs_workspace_size(int op, int64_t n, int64_t n_pairs, int64_t n_tiles, int n_cams);

const char* gs_last_error(void);

/* Diagnostics: while `name` is set, every launch of that kernel (one of
 * "project_cull", "project", "visible_list", "project_bwd", "project_bwd_sh",
 * "export_d2", "scan_reduce", "emit", "vis_compact", "part_count", "sort_pass",
 * "tile_ranges", "seg_sort", "seg_sort_long", "render_fwd", "render_bwd",
 * "importance_blend", "importance_split", "importance_fold", "sel_hist",
 * "gate", "compact" (the gate's active-set pass), "adam", "l1_partial",
 * "l1_final", "ssim_fwd", "ssim_bwd", "voxel_codes", "voxel_label",
 * "spawn_emit", "spawn_stub") records `start`
 * and `stop` (caller-owned HIP events) immediately around the kernel on the
 * stream it is launched on; each launch overwrites the previous record.
 * name = NULL or "" turns it off.  Per calling thread. */
int gs_profile_kernel(const char* name, hipEvent_t start, hipEvent_t stop);

/* Number of 16x16 tiles of a width x height image. */
int64_t gs_num_tiles(int32_t width, int32_t height);

/*
 * View-level active set (Sec. 3.3, Eqs. 1-3).  Gate per Gaussian i:
 *  GS_LOD_LEVEL:  L_v = clamp(floor(log_f(d0 / d) + 0.5), 0, l_max) with
 *                 d = |mean_i - camera centre| (d < 1e-6 gives l_max);
 *                 keep lod_i <= L_v (Eqs. 1-2).  Needs scene->lod.
 *  GS_LOD_RADIUS: keep k * fx * max_j exp(log_scale_ij) / d >= radius_min_px.
 *  GS_LOD_NONE:   keep all.
 * If the gate keeps at least fallback_ratio * n Gaussians it is skipped (the
 * paper's fall-back to the full shard when the ratio is close to one).
 * Active set (Eq. 3) = gate AND keep_bits (NULL = all kept; e.g. the
 * complement of a view's Cull row, or a score mask), written to
 * active_idx[0 .. n_active) in ascending order; *n_active_dev = count.
 * active_idx holds n entries.  Workspace: GS_OP_LOD_MASK.
 */
int gs_lod_mask(const gs_scene* scene, const gs_camera* cam, const gs_lod_params* params,
                const uint32_t* keep_bits, int32_t* active_idx, int64_t* n_active_dev,
                void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * gs_lod_mask without a workspace, for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as gs_lod_mask.  Its scratch (gate bitmap and per-workgroup counts,
 * 2,162,688 bytes) is a fixed array inside the library, one per GPU, held
 * until the process ends; it allows n <= 16,777,216 (2^24) Gaussians and
 * returns GS_ERR_INVALID_ARG above that.  The first call on a device looks up
 * that device's copy (GS_ERR_HIP if the lookup fails).  The call allocates
 * nothing.  Every call on one GPU shares its array: calls that overlap on one
 * GPU (concurrent streams or host threads) race and must be serialised by the
 * caller.
 */
int gs_lod_mask_noalloc(const gs_scene* scene, const gs_camera* cam, const gs_lod_params* params,
                        const uint32_t* keep_bits, int32_t* active_idx, int64_t* n_active_dev,
                        hipStream_t stream);

/*
 * Projection (Appendix A: Gaussians projected to screen-space ellipses) of
 * the input list into n_cams cameras at once, reading the scene once.
 * Entry j < n_in is Gaussian active_idx[j] (active_idx NULL: Gaussian j).
 * If n_in_dev is non-NULL the list holds min(*n_in_dev, n_in) entries and the
 * remaining entries are written as culled (no host synchronisation needed).
 * Per entry and camera: scale activation, Sigma = R S S^T R^T, camera
 * transform, near cull, EWA Jacobian (off-axis clamp 1.3x the half field of
 * view), screen covariance + 0.3 I, conic, radius ceil(3 sqrt(lambda_max)),
 * 16x16 tile rectangle, SH degree-3 colour + 0.5 clamped at 0, depth.
 * out[c] receives camera c.  n_cams <= GS_MAX_CAMS.  Workspace: GS_OP_PROJECT
 * (n = n_in).
 */
int gs_project(const gs_scene* scene, const int32_t* active_idx, int64_t n_in,
               const int64_t* n_in_dev, const gs_camera* cams, int n_cams,
               const gs_projected* out, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Tile binning and depth sort (Appendix A: the depth-ordered Gaussians of each
 * pixel's tile).  Cameras are concatenated: camera c owns global tiles
 * [tile_offset_c, tile_offset_c + gs_num_tiles(c)).  For every entry j with
 * radius > 0 (in order of camera, then j) and each tile of its rectangle in
 * row-major order, a pair (key = global_tile << 32 | float bits of depth,
 * value = j) is emitted; pairs are sorted stably by key, so each tile's list
 * is ordered by (depth, j).  (Implementation: short lists, LSD radix passes
 * over the tile bits, then each tile's segment sorted by (depth bits,
 * position); long lists (capacity above 256 pairs per tile), the visible
 * entries sorted by depth first, the pairs emitted in that order, then stable
 * passes over the tile bits.  Both equal the stable full-key sort.)
 * tile_ranges [2][total_tiles]: row 0 start, row 1 end.
 * Reads rec (or, when every camera has it, the mean2d copy), depth, radius
 * and tiles_touched of the projection.
 * *n_pairs_dev = number of pairs K.  If K > capacity nothing is sorted and
 * every tile range is empty; the caller re-runs with capacity >= K.  No
 * workgroup waits for another (the radix passes take the reduce-then-scan
 * form), so the call cannot stall.
 * keys/vals hold `capacity` entries (capacity <= GS_MAX_PAIRS).
 * Workspace: GS_OP_BIN_SORT with n_pairs = capacity.
 */
int gs_bin_sort(const gs_projected* proj, const gs_camera* cams, int n_cams, int64_t n_in,
                uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* tile_ranges,
                int64_t* n_pairs_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Front-to-back compositing (Appendix A, compositing equation) of every tile.
 * Per pixel: T = 1; for the tile's list in order: alpha = min(0.99, o G);
 * skip if alpha < 1/255; if T (1 - alpha) < 1e-4 stop without compositing;
 * C += c alpha T; T *= 1 - alpha.  Finally C += T bg.
 * out_rgb[c] [3][H_c][W_c], out_T[c] [H_c][W_c] final transmittance,
 * out_last[c] [H_c][W_c] = 1 + list position of the last composited
 * Gaussian (0 if none).  bg: host float[3].
 * chain (optional, NULL = not stored): [K][256] floats, K = the pair count of
 * gs_bin_sort; entry (k, s) receives the transmittance in front of sorted
 * pair k at pixel slot s of its tile (s = lane + 64 r for the pixel at
 * column lane % 16, row lane / 16 + 4 r), written where that pair is
 * composited.  It lets gs_render_bwd read the chain instead of recomputing.
 * pair_live (optional, NULL = not written): [K] bytes; entry k is set to 1 if
 * some pixel of its tile composites sorted pair k, else 0 (entries past the
 * point where every pixel of the tile has stopped may be left unwritten:
 * they lie beyond every pixel's `last`).  gs_render_bwd skips the pairs
 * marked 0.
 */
int gs_render_fwd(const gs_projected* proj, const gs_camera* cams, int n_cams,
                  const uint32_t* vals, const uint32_t* tile_ranges, const float* bg,
                  float* const* out_rgb, float* const* out_T, uint32_t* const* out_last,
                  float* chain, uint8_t* pair_live, hipStream_t stream);

/*
 * Backward of gs_render_fwd and gs_project: given dL/dC (grad_rgb[c],
 * [3][H][W]) accumulates dL/dparameters into grads (+=) at the Gaussians
 * named by active_idx.  Per tile the list is walked back to front from each
 * pixel's `last`, the transmittance before each Gaussian is recomputed from
 * the final T (T_k = T_{k+1} / (1 - alpha_k)), and
 *   dC/dalpha_k = T_k (c_k - S_k) - T_final bg / (1 - alpha_k)
 * with S_k the colour composited behind k normalised by T_{k+1}.  Per
 * (Gaussian, tile) the 9 screen-space partials are reduced across the
 * wavefront and added to the Gaussian's record by one atomic instruction;
 * two more kernels map them to mean, log_scale, quat, opacity_logit and SH
 * (all derivatives exact, zero through culls, clamps and skip/stop
 * decisions).
 * If grads2d is non-NULL it receives the screen-space partials of camera 0
 * ([9][n_in]: d mean2d (2), d conic (3), d opacity (1), d rgb (3)).
 * chain: NULL (recompute T from the final T) or the chain the forward stored;
 * then T_k is read instead of recomputed.
 * pair_live: NULL, or the flags the forward wrote for these lists and outputs;
 * pairs marked 0 (composited by no pixel, hence contributing nothing) are
 * skipped.  The result is the same either way.
 * Workspace: GS_OP_RENDER_BWD (n = n_in, n_cams).
 */
int gs_render_bwd(const gs_scene* scene, const int32_t* active_idx, int64_t n_in,
                  const int64_t* n_in_dev, const gs_projected* proj, const gs_camera* cams,
                  int n_cams, const uint32_t* vals, const uint32_t* tile_ranges, const float* bg,
                  float* const* out_T, uint32_t* const* out_last, float* const* grad_rgb,
                  const float* chain, const uint8_t* pair_live, gs_grads* grads, float* grads2d,
                  void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * One view of the importance-scoring sweep (Sec. 3.2 "Importance score",
 * Fig. 3) over a single camera's projection of the whole shard (n entries):
 * the colour-less instrumented blend records w_i = sum_p alpha T and
 * a_i = number of pixels at which i is composited (w, a: [n], overwritten);
 * then c^rad = [radius_i > 0], c^vis = membership in the shortest prefix of
 * (w descending, i ascending) whose mass reaches mass_frac * sum(w),
 * Cull = 1 - c^vis written as bitmap row cull_row [ceil(n/32)],
 * score_i += w_i / (a_i + eps) where a_i > 0, c_rad_i += c^rad,
 * c_vis_i += c^vis.  count_mode chooses the reading of a_i ("the number of
 * pixels it touches"): GS_COUNT_COMPOSITED (the pixels at which i is
 * composited, the default reading) or GS_COUNT_FOOTPRINT (every pixel of
 * i's tiles, inside the image, whose kernel value passes the 1/255 test,
 * occluded or not; the blend then visits whole lists).  w is the same in both.
 * Workspace: GS_OP_IMPORTANCE.
 */
enum { GS_COUNT_COMPOSITED = 0, GS_COUNT_FOOTPRINT = 1 };

int gs_importance(const gs_projected* proj, const gs_camera* cam, int64_t n,
                  const uint32_t* vals, const uint32_t* tile_ranges, float mass_frac, float eps,
                  int32_t count_mode, float* w, uint32_t* a, float* score, uint32_t* c_rad,
                  uint32_t* c_vis, uint32_t* cull_row, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Score mask: keep_bits [ceil(n/32)] with the n_drop lowest scores (order:
 * score ascending, index ascending) cleared and all others set.  Scores must
 * be non-negative.  Workspace: GS_OP_SCORE_KEEP.
 */
int gs_score_keep_bits(const float* score, int64_t n, int64_t n_drop, uint32_t* keep_bits,
                       void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Second simplification pass (Sec. 3.2 "Scheduled simplification"): the
 * deterministic cumulative-mass cut keeps the smallest prefix of (score
 * descending, index ascending) whose summed score reaches mass_frac (0.99)
 * of the total, the crossing element included; zero scores are never kept.
 * keep_bits [ceil(n/32)]; *n_keep_dev = number kept.  Workspace:
 * GS_OP_SIMPLIFY.
 */
int gs_mass_keep_bits(const float* score, int64_t n, float mass_frac, uint32_t* keep_bits,
                      int64_t* n_keep_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * First simplification pass (Sec. 3.2): importance-weighted sampling without
 * replacement of n_keep Gaussians with probability proportional to the score,
 * in the exponential-race form of Efraimidis & Spirakis: keep the n_keep
 * smallest -ln(u_i) / s_i (+inf for s_i = 0), ties by index.  uniforms [n]
 * in (0, 1] are the caller's random draws.  Workspace: GS_OP_SIMPLIFY.
 */
int gs_sample_keep_bits(const float* score, const float* uniforms, int64_t n, int64_t n_keep,
                        uint32_t* keep_bits, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Compaction after a pass: for each of n_arrays component-major arrays
 * (rows[a] x n elements of elem_bytes[a] = 4 or 1 bytes; a [16][3][n] array
 * is 48 rows), dst[a] (rows[a] x n_keep) receives the kept columns in
 * ascending index order.  keep_bits: ceil(n / 32) words, bit i % 32 of word
 * i / 32 (may be null when n = 0).  n_keep must equal the number of set bits
 * (read from gs_mass_keep_bits or known); columns ranked n_keep or later are
 * not written.  1 <= n_arrays <= 16, rows[a] >= 1, n < 2^31; src, dst and
 * the keep bits are device memory the caller owns, src and dst distinct.
 * GS_ERR_INVALID_ARG for other arguments, GS_ERR_WORKSPACE for a short or
 * unaligned workspace (GS_OP_SIMPLIFY); n = 0 or n_keep = 0 launch nothing.
 */
int gs_compact(const void* const* src, void* const* dst, const int32_t* rows, const int32_t* elem_bytes,
               int n_arrays, int64_t n, int64_t n_keep, const uint32_t* keep_bits, void* ws,
               size_t ws_bytes, hipStream_t stream);

/*
 * L1 photometric term (Eq. 4 with lambda = 0): *loss_dev = mean |C - target|
 * over n_vals values, grad = s * sign(C - target) / n_vals (sign(0) = 0)
 * with s = *grad_scale (a device float, e.g. the upstream derivative of an
 * autograd graph) or 1 when grad_scale is NULL.  Either output may be NULL
 * (not computed), not both.  Deterministic two-stage reduction.  Workspace:
 * GS_OP_L1_LOSS (only used when loss_dev is non-NULL).
 */
int gs_l1_loss(const float* rgb, const float* target, int64_t n_vals, float* loss_dev,
               float* grad, const float* grad_scale, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Photometric term of the paper's objective (Sec. 3.4, Eq. 4) for one view:
 * loss = scale * [(1 - lambda) mean|C - I| + lambda (1 - mean SSIM(C, I))]
 * with SSIM over an 11x11 Gaussian window (sigma 1.5), constants (0.01)^2
 * and (0.03)^2, local statistics zero-padded at the image border; grad =
 * d loss / dC.  rgb, target, grad: [3][height][width].  Use scale = 1/B to
 * average a batch of B views.  Deterministic.  Workspace: gs_workspace_size
 * (GS_OP_PHOTO_LOSS, width * 65536 + height, ...).
 */
int gs_photo_loss(const float* rgb, const float* target, int32_t width, int32_t height, float lambda,
                  float scale, float* loss_dev, float* grad, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Scale regulariser (Sec. 3.4, Eq. 5): *loss_dev = beta * mean over the
 * visible entries (radius > 0 in `radius`, the projection of this view) of
 * the smallest scale exp(min_j log_scale_j), and grad_log_scale (+=) gets
 * beta / |V| * s_min on the arg-min axis (first axis on ties).  Entry j is
 * Gaussian active_idx[j] as in gs_project.  Workspace: GS_OP_SCALE_REG.
 */
int gs_scale_reg(const gs_scene* scene, const int32_t* active_idx, int64_t n_in, const int64_t* n_in_dev,
                 const int32_t* radius, float beta, float* loss_dev, float* grad_log_scale, void* ws,
                 size_t ws_bytes, hipStream_t stream);

/*
 * Adam with bias correction (Kingma & Ba), one fused launch over n_groups
 * parameter groups (host arrays of device pointers and counts); the paper's
 * per-rank optimizer state (Sec. 3.1) implies it:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr_k * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * The step number is `step` (>= 1), or, if step_dev is non-NULL, the device
 * counter *step_dev + 1, which the call then increments on the device (so a
 * captured HIP graph replays successive steps).  With clear_grads != 0 each
 * gradient is reset to 0 after it is read, ready for the next accumulating
 * gs_render_bwd.  n_groups <= 8.
 */
int gs_adam_step(float* const* params, float* const* grads, float* const* m,
                 float* const* v, const int64_t* counts, int n_groups, const float* lr,
                 float b1, float b2, float eps, int step, int32_t* step_dev, int clear_grads,
                 hipStream_t stream);

/*
 * LOD labels by multi-resolution voxelisation (Sec. 3.3, "Distance-based LOD
 * gate": labels attached at multi-resolution voxelisation).  Level l
 * partitions space into cubes of edge delta0 / 2^l anchored at origin[3]
 * (host floats, e.g. the per-axis minimum of the means); every occupied
 * level-l cube is represented by one Gaussian, its first in the order
 * (Z-order code of the point's finest cell, index), and lod[i] is the
 * coarsest level l in [0, n_levels) at which Gaussian i represents its cube,
 * n_levels - 1 if none.  Keeping lod <= L therefore keeps exactly one
 * Gaussian per occupied cube of edge delta0 / 2^L.  The finest cell of a point
 * is floor((mean - origin) * s) per axis in float32 with s = 2^(n_levels-1) /
 * delta0 (NaN -> 0, clamped to [0, 2^21)).  mean [3][n]; lod [n] (written).
 * n_levels in [1, 22].  Workspace: GS_OP_VOXEL_LEVELS.
 */
int gs_voxel_levels(const float* mean, int64_t n, const float* origin, float delta0, int32_t n_levels,
                    uint8_t* lod, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Coarse-to-fine ceiling L_max(t) of the level gate (Sec. 3.3, after Eq. 2:
 * levels unlock coarse to fine on a geometric schedule).  Level k unlocks at
 * iteration u_k = t0 * (t1 / t0)^(k / (n_levels - 1)) (double arithmetic), so
 * u_0 = t0, u_{n_levels-1} = t1 and consecutive unlock times have a constant
 * ratio; returns the largest k with u_k <= t (0 up to t0, n_levels - 1 from
 * t1 on).  Pass the result as gs_lod_params.l_max.  Host only; needs
 * 0 < t0 < t1.
 */
int32_t gs_lod_level_ceiling(int64_t t, int64_t t0, int64_t t1, int32_t n_levels);

/*
 * Spawn gate of one densification event (Sec. 3.2 "Spawn gate"; the veto
 * equation of Appendix E).  Clones (clone_parent[n_clone], predicted
 * survival p_clone) and splits (split_parent[n_split], p_split) are separate
 * candidate sets; in each, the ceil(rho * |C|) candidates of lowest survival
 * (rho * |C| evaluated in double) are vetoed, ties by candidate index (the
 * lower index vetoed first).  Survival scores must be non-negative and not
 * NaN (probabilities).  The instantiated candidates are written in order -
 * surviving clones in candidate order, then surviving splits - as
 * child_parent (the parent's index), child_lod (the inherited level: a clone
 * keeps lod[parent], a split gets lod[parent] + 1, clamped at n_levels - 1)
 * and child_split (0 clone, 1 split).  *n_children (HOST int64) receives
 * their number, known before any launch; outputs hold n_clone + n_split
 * entries.  rho in [0, 1] (0.6 in the paper).  Workspace: GS_OP_SPAWN_GATE.
 */
int gs_spawn_gate(const uint8_t* lod, const int32_t* clone_parent, const float* p_clone, int64_t n_clone,
                  const int32_t* split_parent, const float* p_split, int64_t n_split, double rho,
                  int32_t n_levels, int32_t* child_parent, uint8_t* child_lod, uint8_t* child_split,
                  int64_t* n_children, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Stand-in for the offline survival predictor of the spawn gate (Sec. 3.2;
 * the gradient-boosted tree is fit on lineage logs of real scenes): p[i] =
 * the opacity of Gaussian parent[i], sigmoid(opacity_logit), one of the
 * spawn-time features the paper lists.  No workspace.
 */
int gs_spawn_stub_score(const gs_scene* scene, const int32_t* parent, int64_t n, float* p, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GSMI_H */
