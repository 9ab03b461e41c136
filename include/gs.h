/*
 * gs.h - C ABI of the MI355X (gfx950) Gaussian-splatting hot path.
 *
 * One GPU's share of a Gaussian-splatting training step, as listed in
 * Section 4 of "A Scalable PyTorch Abstraction for Multi-GPU Gaussian
 * Splatting" (arXiv 2606.11390): spherical-harmonic colour and projection per
 * Gaussian for every camera of a batch, a per-camera depth sort, rasterisation
 * and an image-space loss, and the backward passes of all of them.  The paper
 * takes the mathematics from 3D Gaussian Splatting (Kerbl et al. 2023); the
 * formulas below are those.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every pointer argument is a DEVICE pointer owned by the caller unless its
 *   comment says "host".  The library never allocates, frees or retains
 *   memory: scratch space comes in through an explicit workspace argument.
 * - Every call only enqueues work on `stream` (a hipStream_t passed as void*,
 *   NULL for the default stream) and returns without synchronising; outputs
 *   are valid once the stream reaches that point.  No call reads a device
 *   value back to the host, so a whole step can be captured in a HIP graph.
 * - Return value: GS_OK (0) or a negative gs_status.  Argument errors are
 *   detected on the host before anything is enqueued; GS_ERR_HIP reports a
 *   failed launch.  No C++ exception crosses the ABI.
 * - N = number of Gaussians, V = number of views (1 <= V <= GS_MAX_VIEWS),
 *   K = (sh_degree + 1)^2 SH coefficients per channel (sh_degree in 0..3),
 *   tile = tile edge in pixels (8, 16 or 32).
 * - Per-Gaussian parameters are planar structure-of-arrays [C][N] float32.
 * - Per-(view, Gaussian) outputs are [V][N][...] with view v at offset v*N.
 * - Images of view v (W_v x H_v pixels) are packed back to back: colour
 *   images [3][H_v][W_v] starting at float offset 3 * sum_{u<v} W_u H_u,
 *   single-channel images [H_v][W_v] starting at sum_{u<v} W_u H_u.
 * - Pixel (i, j) (column i, row j) has its centre at (i + 0.5, j + 0.5).
 * - Tiles of view v are numbered row-major, TX_v = ceil(W_v / tile),
 *   TY_v = ceil(H_v / tile); the global tile id is tile_offset_v + ty*TX_v + tx
 *   with tile_offset_v = sum_{u<v} TX_u TY_u, and T_total = tile_offset_V.
 *
 * The splat record (GS_SPLAT_FLOATS = 12 float32, 48 bytes, 16-byte aligned),
 * one per (view, Gaussian), written by gs_project and read by the
 * rasterisers:
 *   [0] u, [1] v      projected mean in pixels
 *   [2] m00, [3] m10, [4] m11
 *                     lower-triangular M = [[m00, 0], [m10, m11]] with
 *                     M M^T = (log2(e) / 2) * Q, Q = [[A, B], [B, C]] the
 *                     conic (inverse of the EWA 2-D covariance).  Then
 *                     q' = |M^T d|^2 = (log2 e / 2) d^T Q d and the Gaussian
 *                     falloff exp(-d^T Q d / 2) equals 2^(-q').
 *   [5] log2(sigma)   sigma = sigmoid(opacity logit)
 *   [6] r, [7] g, [8] b   view-dependent colour (after the clamp at 0)
 *   [9] sigma
 *   [10], [11] (int32 bit patterns) conservative pixel ranges of the region
 *                     where alpha >= 1/255: x range lo | hi << 16 and y range
 *                     likewise (int16 column / row indices, inclusive); every
 *                     pixel outside the box has alpha < 1/255, so the
 *                     rasterisers may skip the splat there
 * Records of culled Gaussians are left unwritten.  Views are at most 32767
 * pixels wide and high.
 *
 * The 2-D gradient record (GS_GRAD_FLOATS = 9 float32), one per
 * (view, Gaussian): derivatives of the loss with respect to
 *   [0] u, [1] v, [2] A, [3] B, [4] C (conic entries, B counted once),
 *   [5] sigma, [6] r, [7] g, [8] b.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 5
#define GS_MAX_VIEWS 64
#define GS_SPLAT_FLOATS 12
#define GS_GRAD_FLOATS 9
#define GS_ADAM_MAX_TENSORS 8

/* flags byte per (view, Gaussian) */
#define GS_FLAG_VISIBLE 0x1u
#define GS_FLAG_CLAMP_R 0x2u
#define GS_FLAG_CLAMP_G 0x4u
#define GS_FLAG_CLAMP_B 0x8u

/* radius_mode of gs_project: the screen box that selects a splat's tiles */
#define GS_RADIUS_3SIGMA 0   /* per-axis 3-sigma box (default) */
#define GS_RADIUS_OPACITY 1  /* 3-sigma box clipped to the alpha >= 1/255 region */
#define GS_RADIUS_EIGEN 2    /* square of 3 sqrt(largest eigenvalue) (3D Gaussian Splatting) */

/* gs_bin_sort info words (device int32[4]) */
#define GS_INFO_VISIBLE 0   /* number of visible (view, Gaussian) pairs */
#define GS_INFO_ISECT 1     /* number of intersections M (saturates at INT32_MAX) */
#define GS_INFO_OVERFLOW 2  /* 1 if M > capacity: lists truncated, re-run larger */

typedef enum {
    GS_OK = 0,
    GS_ERR_ARG = -1,         /* null pointer, bad size, unsupported tile/degree */
    GS_ERR_UNSUPPORTED = -2, /* valid request this build does not implement */
    GS_ERR_HIP = -3,         /* a HIP launch or runtime call failed */
    GS_ERR_WORKSPACE = -4    /* workspace smaller than the *_workspace_size query */
} gs_status;

/* GS_ABI_VERSION of the loaded library */
int gs_abi_version(void);

/* static, human-readable text of a gs_status */
const char* gs_strerror(int code);

/*
 * gs_project - forward projection and SH colour (paper Section 4: the
 * spherical-harmonics and projection operators, per Gaussian, outputs for
 * every camera of the batch).  Reads each Gaussian's parameters once for all
 * V views.
 *
 * Inputs:
 *   means[3][N]           world-space centres mu
 *   log_scales[3][N]      per-axis log standard deviations (S = diag exp)
 *   quats[4][N]           rotation quaternion (w, x, y, z), any non-zero norm
 *   opacity_logits[N]     sigma = 1 / (1 + exp(-o))
 *   sh[K][3][N]           real SH coefficients, index l*l + l + m, Condon-
 *                         Shortley phase; colour = max(0, sum_k sh_k Y_k(d) + 0.5)
 *                         with d the unit ray from the camera centre to mu
 *   viewmats[V][12]       world-to-camera [R | t], row-major, OpenCV axes
 *                         (+x right, +y down, +z forward)
 *   intrinsics[V][4]      fx, fy, cx, cy (pixels)
 *   sizes (host)[V][2]    W, H of each view
 *   near_plane, far_plane culling planes on camera z (z <= near or z >= far)
 *   eps2d                 isotropic dilation added to the 2-D covariance (0.3)
 *   tile                  tile edge used to count tiles_touched
 *   radius_mode           GS_RADIUS_* (densification-oriented variants of the
 *                         screen box; the paper fixes none):
 *                         3SIGMA  rx, ry = ceil(3 sqrt(Sigma2_xx)), ceil(3 sqrt(Sigma2_yy));
 *                         OPACITY min of 3SIGMA and ceil(sqrt(tau' Sigma2_xx)) + 1
 *                                 (same in y), tau' = 1.001 * 2 ln(255 sigma) + 0.01:
 *                                 drops only tiles where every pixel has
 *                                 alpha < 1/255, so images and gradients are
 *                                 those of 3SIGMA with fewer intersections;
 *                         EIGEN   rx = ry = ceil(3 sqrt(m + sqrt(max(m^2 - det, 0.1)))),
 *                                 m = (Sigma2_xx + Sigma2_yy) / 2;
 *                         any other value is GS_ERR_ARG
 * Method: Sigma = R S S^T R^T; p = R_v mu + t_v; J = Jacobian of the pinhole
 * projection at p with x/z, y/z clamped to +-1.3 * (W/2)/fx, (H/2)/fy;
 * Sigma2 = J R_v Sigma R_v^T J^T + eps2d I; Q = Sigma2^-1; (u, v) = (fx x/z +
 * cx, fy y/z + cy); radii per radius_mode;
 * tile rectangle [floor((u-rx)/tile), floor((u+rx)/tile)+1) x (same in y),
 * clamped to the grid, evaluated in float32.
 * Culled (all outputs zero, record unwritten): non-finite input, z outside
 * (near, far), sigma < 1/255, det Sigma2 <= 0, empty tile rectangle.
 * Outputs ([V][N] unless stated):
 *   splats[V][N][12]      splat record (see above)
 *   depths                camera-space z (float32; sort key)
 *   radii[V][N][2]        rx, ry in pixels (int32)
 *   tiles_touched         number of tiles in the rectangle (int32)
 *   tile_rects[V][N][2]   the tile rectangle [x0, x1) x [y0, y1) in the view's tile
 *                         grid, packed as x0 | y0 << 16, x1 | y1 << 16 (int32);
 *                         all zero when culled
 *   flags                 GS_FLAG_* bits (uint8)
 *   grad2d_clear[V][N][9] optional (may be NULL): the 2-D gradient records of
 *                         the visible pairs are zeroed, so that a following
 *                         gs_rasterize_bwd / gs_rasterize_bwd_l2 of these
 *                         lists can accumulate (accumulate != 0) instead of
 *                         clearing all V N records first; records of culled
 *                         pairs are left as they are (no call reads them)
 */
int gs_project(const float* means, const float* log_scales, const float* quats,
               const float* opacity_logits, const float* sh, int64_t n, int sh_degree,
               const float* viewmats, const float* intrinsics, const int32_t* sizes, int n_views,
               float near_plane, float far_plane, float eps2d, int tile, int radius_mode,
               float* splats, float* depths, int32_t* radii, int32_t* tiles_touched,
               int32_t* tile_rects, uint8_t* flags, float* grad2d_clear, void* stream);

/*
 * gs_bin_sort_workspace_size - bytes of device workspace gs_bin_sort needs
 * for n Gaussians, V views, an intersection capacity and T_total tiles.
 */
size_t gs_bin_sort_workspace_size(int64_t n, int n_views, int64_t capacity, int64_t total_tiles);

/*
 * gs_bin_sort - tile binning and depth sort (paper Section 4: per camera,
 * the Gaussians are sorted by depth before rasterisation; one record per
 * (Gaussian, tile) intersection).
 *
 * Result: the M intersections of all views sorted stably by the 64-bit key
 * (global tile id << 32) | float32 bits of depth, where intersections are
 * enumerated per view, Gaussian index ascending and tiles row-major within
 * each rectangle; equal keys therefore keep Gaussian order.  (Depth is
 * positive, so its bit pattern orders like its value.)
 * Inputs: tile_rects and depths as written by gs_project for the same n, V,
 *   sizes and tile (a pair is binned when its rectangle is not empty);
 *   capacity = entries available in isect_tile / isect_gid
 *   (1 <= capacity < 2^31).
 * Outputs:
 *   isect_tile[capacity]  global tile id of each sorted intersection
 *   isect_gid[capacity]   Gaussian index (0..N-1) of each sorted intersection
 *   tile_ranges[T_total][2]  first and one-past-last position of each tile's
 *                         run in the sorted arrays (0, 0 when empty)
 *   info[4] (device int32) GS_INFO_* words.
 * Overflow: if M > capacity, info[GS_INFO_OVERFLOW] = 1 and only the first
 *   `capacity` intersections (in depth-sorted enumeration order) are kept;
 *   the lists are then incomplete and the caller must re-run with more room.
 * workspace: >= gs_bin_sort_workspace_size() bytes, 256-byte aligned,
 *   contents need not be initialised and are clobbered.
 */
int gs_bin_sort(const int32_t* tile_rects, const float* depths, int64_t n, int n_views, const int32_t* sizes,
                int tile, int64_t capacity, void* workspace, size_t workspace_bytes,
                int32_t* isect_tile, int32_t* isect_gid, int32_t* tile_ranges, int32_t* info,
                void* stream);

/*
 * gs_tile_schedule_size - bytes of device memory gs_tile_schedule needs for
 * T_total tiles (its `order` plus its own scratch).
 */
size_t gs_tile_schedule_size(int64_t total_tiles);

/*
 * gs_tile_schedule - order tiles so that long lists start first: by
 * decreasing list length rounded down to four significant bits (lengths
 * below 8 kept exactly, lengths above 65535 taken as 65535), ties by tile
 * id.  Writes order[T_total] (int32 global tile ids) at the start of
 * `schedule` (256-byte aligned).
 */
int gs_tile_schedule(const int32_t* tile_ranges, int64_t total_tiles, void* schedule,
                     size_t schedule_bytes, void* stream);

/*
 * gs_tile_order_xcd - a static tile order for grid launches on a GPU whose
 * workgroups are handed round-robin to n_xcd dies with private L2 caches
 * (MI355X: 8 XCDs): workgroup b gets tile x * (T/n_xcd) + min(x, T mod n_xcd)
 * + b / n_xcd with x = b mod n_xcd, so each die renders one contiguous band of
 * tiles and neighbouring tiles, which share most of their splats, share an
 * L2.  Writes order[T_total] at the start of `schedule` (same size and
 * alignment as for gs_tile_schedule).
 */
int gs_tile_order_xcd(int64_t total_tiles, int n_xcd, void* schedule, size_t schedule_bytes, void* stream);

/*
 * gs_rasterize_fwd - front-to-back alpha compositing (paper Section 4: the
 * rasterisation operator, per camera).  For each pixel, over its tile's list
 * in sorted order: alpha = min(0.99, sigma * 2^(-q')); entries with
 * alpha < 1/255 are skipped; compositing stops before the first entry that
 * would bring the transmittance T below 1e-4; colour C += alpha T c,
 * T *= 1 - alpha.  Output colour = C + T * background.
 * Inputs: splats, isect_gid and tile_ranges from gs_project / gs_bin_sort;
 *   background (host)[3].
 * block_w, px_per_lane: the pixel block one wavefront covers (block_w wide,
 *   64 * px_per_lane / block_w rows) and the adjacent pixels each lane owns;
 *   0, 0 selects the default (8, 1).  Valid pairs: tile 8: (8, 1); tile 16:
 *   (8, 1), (16, 1), (16, 2), (16, 4); tile 32: (8, 1), (16, 2), (16, 4),
 *   (32, 4).  The choice changes only speed, never a result bit.
 * schedule, queue: how tiles are assigned to workgroups.
 *   schedule NULL: one workgroup per tile, in tile order (queue must be NULL).
 *   schedule set, queue NULL: one workgroup per tile, workgroup b renders
 *     tile order[b] of the schedule buffer (gs_tile_schedule: longest lists
 *     first; gs_tile_order_xcd: one band of tiles per XCD).
 *   schedule and queue set: a persistent grid whose waves pull (view, tile)
 *     items in schedule order from the global counter *queue (device int32,
 *     reset by this call), eight items per atomic.
 *   The order entries must be tile ids in [0, T_total); others are skipped.
 *   None of this changes a result bit.
 * Outputs: images (packed [3][H][W] per view), T_final and n_contrib (packed
 *   [H][W] per view): final transmittance and one past the list position of
 *   the last composited entry.
 */
int gs_rasterize_fwd(const float* splats, const int32_t* isect_gid, const int32_t* tile_ranges,
                     int64_t n, int n_views, const int32_t* sizes, int tile, int block_w, int px_per_lane,
                     const float* background, const void* schedule, int32_t* queue, float* images,
                     float* T_final, int32_t* n_contrib, void* stream);

/*
 * gs_rasterize_bwd - backward of gs_rasterize_fwd (paper Section 4: backward
 * of the rasteriser with gradient accumulation by atomics).  Walks each
 * pixel's composited entries from the back, recovering each transmittance
 * from T_final by division by (1 - alpha) instead of storing per-pixel lists.
 * Inputs: as gs_rasterize_fwd (block_w and px_per_lane likewise only change
 *   speed) plus its T_final and n_contrib, d_images (packed
 *   like images) and d_alpha (packed [H][W] per view; gradient with respect
 *   to 1 - T_final; may be NULL).
 * Output: grad2d[V][N][9] (see the 2-D gradient record).  With accumulate = 0
 *   the call first zeroes it (with a fill kernel, so the call stays graph
 *   capturable) and then accumulates; with accumulate != 0 it adds to the
 *   existing contents.  Summation order is not deterministic.
 */
int gs_rasterize_bwd(const float* splats, const int32_t* isect_gid, const int32_t* tile_ranges,
                     int64_t n, int n_views, const int32_t* sizes, int tile, int block_w, int px_per_lane,
                     const float* background, const void* schedule, int32_t* queue, const float* T_final,
                     const int32_t* n_contrib, const float* d_images, const float* d_alpha,
                     float* grad2d, int accumulate, void* stream);

/*
 * gs_rasterize_bwd_l2_workspace_size - bytes of device workspace
 * gs_rasterize_bwd_l2 needs for these views and tile edge (8 bytes per
 * 64 pixels of tile area: one partial sum per wavefront).
 */
size_t gs_rasterize_bwd_l2_workspace_size(int n_views, const int32_t* sizes, int tile);

/*
 * gs_rasterize_bwd_l2 - the L2 image loss and the rasteriser backward in one
 * pass (paper Section 4: per camera the image loss, then the backward of the
 * rasteriser with gradient accumulation by atomics).  Equals gs_loss_l2 over
 * all packed elements (n = 3 * sum of W * H) followed by gs_rasterize_bwd
 * with d_images = 2 (images - targets) / n and no d_alpha, except that
 * d_images is never stored: each wavefront forms its pixels' gradient from
 * images and targets as gs_loss_l2 does (same float32 operations, so grad2d
 * gets the same per-pixel terms), and adds its pixels' squared errors to a
 * per-wavefront partial sum.
 * Inputs: as gs_rasterize_bwd, with images (the gs_rasterize_fwd output) and
 *   targets (packed [3][H][W] per view) instead of d_images and d_alpha.
 *   Grid dispatch only (schedule NULL or a tile order; no work queue).
 * Outputs: loss (device float[1]) = mean squared error, reduced in a fixed
 *   order (per-wavefront float sums, then in double by one workgroup), so it
 *   is deterministic; grad2d as gs_rasterize_bwd (accumulate likewise).
 * workspace: >= gs_rasterize_bwd_l2_workspace_size() bytes, 8-byte aligned,
 *   clobbered (one double per wavefront, then one per 4,096 of those).
 * unseen_grads (optional, NULL: not used): a host array of five device
 *   pointers d_means [3][N], d_log_scales [3][N], d_quats [4][N],
 *   d_opacity_logits [N] and d_sh [K][3][N] (K = (sh_degree + 1)^2), into
 *   which the call also writes what gs_project_bwd_part writes with
 *   GS_GRADS_UNSEEN: zeros for every group of 64 Gaussians that no view sees
 *   (flags, [V][N] from gs_project), leaving the other elements untouched.
 *   That part of the projection backward needs no 2-D gradient; the
 *   compositing waves write it while their arithmetic, not memory, bounds
 *   them.  gs_project_bwd_part with GS_GRADS_SEEN then completes the
 *   parameter gradients.  flags and
 *   sh_degree are read only with unseen_grads.  Errors: GS_ERR_ARG for a
 *   NULL flags or plane pointer (N > 0) or sh_degree outside 0..3.
 */
int gs_rasterize_bwd_l2(const float* splats, const int32_t* isect_gid, const int32_t* tile_ranges, int64_t n,
                        int n_views, const int32_t* sizes, int tile, int block_w, int px_per_lane,
                        const float* background, const void* schedule, const float* T_final,
                        const int32_t* n_contrib, const float* images, const float* targets, float* loss,
                        float* grad2d, int accumulate, void* workspace, size_t workspace_bytes,
                        const uint8_t* flags, int sh_degree, float* const* unseen_grads, void* stream);

/*
 * gs_project_bwd - backward of gs_project (paper Section 4: backward of the
 * SH and projection operators, partitioned per Gaussian).  One thread owns
 * one Gaussian and sums its views in registers, so no atomics are used.
 * Inputs: the gs_project inputs, its flags, and grad2d from gs_rasterize_bwd.
 * Outputs (OVERWRITTEN, not accumulated): d_means[3][N], d_log_scales[3][N],
 *   d_quats[4][N], d_opacity_logits[N], d_sh[K][3][N].  Gaussians culled in
 *   every view get zeros.  Depth is not differentiated (sort key only).
 */
int gs_project_bwd(const float* means, const float* log_scales, const float* quats,
                   const float* opacity_logits, const float* sh, int64_t n, int sh_degree,
                   const float* viewmats, const float* intrinsics, const int32_t* sizes, int n_views,
                   float eps2d, const uint8_t* flags, const float* grad2d, float* d_means,
                   float* d_log_scales, float* d_quats, float* d_opacity_logits, float* d_sh,
                   void* stream);

/* which gradients gs_project_bwd_part writes; a group is Gaussians
 * 64 k ... 64 k + 63 (the last one shorter) */
#define GS_GRADS_ALL 0    /* every Gaussian's: gs_project_bwd */
#define GS_GRADS_SEEN 1   /* every Gaussian's of the groups in which some view sees a Gaussian */
#define GS_GRADS_UNSEEN 2 /* zeros for the groups in which no view sees any Gaussian */

/*
 * gs_project_bwd_part - gs_project_bwd split by visibility (paper Section 4:
 * backward of the SH and projection operators), in groups of 64 Gaussians:
 * each part leaves the other part's groups untouched, and GS_GRADS_SEEN
 * followed (or preceded) by GS_GRADS_UNSEEN writes exactly what
 * gs_project_bwd writes.  Groups, not single Gaussians, so that each line of
 * a gradient plane is written whole by one of the two.  The unseen part
 * reads only flags, so it can run as soon as gs_project has written them;
 * the two parts write disjoint elements and may overlap in time.
 * Inputs and outputs as gs_project_bwd.  With GS_GRADS_UNSEEN the
 * parameters, cameras, eps2d and grad2d are not read and may be NULL (sizes
 * and n_views are still checked).  Errors: GS_ERR_ARG for another part value
 * and for the gs_project_bwd checks of the arguments that part reads.
 */
int gs_project_bwd_part(const float* means, const float* log_scales, const float* quats,
                        const float* opacity_logits, const float* sh, int64_t n, int sh_degree,
                        const float* viewmats, const float* intrinsics, const int32_t* sizes, int n_views,
                        float eps2d, const uint8_t* flags, const float* grad2d, float* d_means,
                        float* d_log_scales, float* d_quats, float* d_opacity_logits, float* d_sh, int part,
                        void* stream);

/*
 * gs_project_bwd_adam - gs_project_bwd followed by gs_adam over the five
 * parameter tensors, fused: the thread that forms a Gaussian's gradient
 * applies the Adam step to its parameters in place, so the gradient is never
 * written to or read back from memory (paper Section 3.2: fused optimizer
 * over the Gaussian parameters; Section 4: backward of the SH and projection
 * operators).  The update is that of gs_adam with t = *step + 1, for the
 * tensors means[3][N], log_scales[3][N], quats[4][N], opacity_logits[N] and
 * sh[K][3][N] in this order, which are READ AND OVERWRITTEN (device).
 * exp_avg and exp_avg_sq are host arrays of five device pointers to the
 * moments, each shaped like its parameter tensor; lrs is a host array of the
 * five learning rates.  Gaussians that no view sees get a zero gradient and
 * are still updated (their moments decay).  step (device int32) is
 * incremented on the stream after the update, so a captured graph replays
 * consecutive steps.  The parameters, moments, flags and grad2d must not
 * overlap one another.  N <= 2^30.  Errors: GS_ERR_ARG for null pointers
 * (when N > 0), betas outside [0, 1), eps <= 0, a non-finite rate, N above
 * 2^30 or the other gs_project_bwd argument checks.
 */
int gs_project_bwd_adam(float* means, float* log_scales, float* quats, float* opacity_logits, float* sh,
                        int64_t n, int sh_degree, const float* viewmats, const float* intrinsics,
                        const int32_t* sizes, int n_views, float eps2d, const uint8_t* flags, const float* grad2d,
                        float* const* exp_avg, float* const* exp_avg_sq, const float* lrs, float beta1,
                        float beta2, float eps, int32_t* step, void* stream);

/*
 * gs_densify_stats - per-Gaussian statistics of the adaptive density control
 * of 3D Gaussian Splatting (Kerbl et al. 2023; the paper densifies to larger
 * Gaussian counts with it, Section 5), gathered from one step's 2-D gradients.
 * For every view v in which Gaussian g is visible (flags & GS_FLAG_VISIBLE):
 *   grad_accum[g] += || (dL/du * W_v / 2, dL/dv * H_v / 2) ||_2
 * (the gradient norm with respect to the normalised device coordinates of the
 * projected mean, u = ((x_ndc + 1) W - 1) / 2), count[g] += 1 and
 * max_radius[g] = max(max_radius[g], rx, ry).
 * grad2d [V][N][9] and radii [V][N][2] as written by gs_rasterize_bwd and
 * gs_project; grad_accum (float), count and max_radius (int32) [N] are
 * accumulated, never cleared.  Deterministic: one thread per Gaussian walks
 * the views in order.
 */
int gs_densify_stats(const float* grad2d, const uint8_t* flags, const int32_t* radii, int64_t n, int n_views,
                     const int32_t* sizes, float* grad_accum, int32_t* count, int32_t* max_radius, void* stream);

/*
 * gs_raster_visits - instrumentation for the roofline numerator: runs the
 * forward compositing of gs_rasterize_fwd (zero background, one workgroup per
 * tile) and also writes visits (packed [H][W] per view, int32): the number of
 * list entries each pixel examined, i.e. up to and including the entry that
 * stopped it, or its whole tile list.
 */
int gs_raster_visits(const float* splats, const int32_t* isect_gid, const int32_t* tile_ranges, int64_t n,
                     int n_views, const int32_t* sizes, int tile, float* images, float* T_final,
                     int32_t* n_contrib, int32_t* visits, void* stream);

/*
 * gs_loss_workspace_size - bytes of device workspace gs_loss_l2 needs for
 * n_elems image elements.
 */
size_t gs_loss_workspace_size(int64_t n_elems);

/*
 * gs_loss_l2 - image-space loss (paper Section 4: per-camera image loss; L2
 * here): loss = sum((images - targets)^2) / n_elems and
 * d_images = 2 (images - targets) / n_elems over n_elems packed floats.
 * loss (device float[1]) is overwritten; the sum is reduced in a fixed order
 * (deterministic) through `workspace`.
 */
int gs_loss_l2(const float* images, const float* targets, int64_t n_elems, float* loss,
               float* d_images, void* workspace, size_t workspace_bytes, void* stream);

/*
 * gs_loss_l2_noalloc - gs_loss_l2 without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments,
 * results and determinism as gs_loss_l2, for any n_elems >= 0: the partial
 * sums (at most GS_LOSS_NOALLOC_PARTIALS doubles, 16 KiB) live in a device
 * array inside the library, one copy per GPU, held until the process ends;
 * the first call on a device looks up that copy's address.  The call never
 * allocates or frees memory.  It runs on the current device (the stream
 * must belong to it).  Calls that overlap in time on one GPU (several
 * streams or threads) share the array and race: serialise them.  Returns
 * GS_ERR_ARG for a negative n_elems or a null pointer, GS_ERR_HIP if the
 * array's address cannot be obtained or the launch fails.
 */
#define GS_LOSS_NOALLOC_PARTIALS 2048
int gs_loss_l2_noalloc(const float* images, const float* targets, int64_t n_elems, float* loss,
                       float* d_images, void* stream);

/*
 * gs_adam - fused Adam update of up to GS_ADAM_MAX_TENSORS parameter tensors
 * (paper Section 3.2: the backend's fused Adam; the rule is Kingma and Ba
 * 2015 with bias correction, as torch.optim.Adam without weight decay):
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   p -= lr_k / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps),
 * with t = *step + 1.  params, grads, exp_avg, exp_avg_sq are HOST arrays of
 * n_tensors DEVICE pointers (16-byte aligned, numel[k] float32 each, host
 * array); lrs is a host array of per-tensor learning rates.  step (device
 * int32) is read by the update and then incremented on the stream, so a
 * captured graph replays consecutive steps.
 */
int gs_adam(int n_tensors, float* const* params, const float* const* grads, float* const* exp_avg,
            float* const* exp_avg_sq, const int64_t* numel, const float* lrs, float beta1, float beta2,
            float eps, int32_t* step, void* stream);

/*
 * gs_ssim_workspace_size - bytes of device workspace gs_loss_ssim_l1 needs for
 * the given views (sizes: host [V][2]).
 */
size_t gs_ssim_workspace_size(int n_views, const int32_t* sizes);

/*
 * gs_loss_ssim_l1 - the image-space loss the paper's per-camera fused SSIM
 * operator computes (Section 4; SSIM of Wang et al. 2004 with the 3D Gaussian
 * Splatting settings): per channel an 11x11 Gaussian window (std 1.5) applied
 * as a zero-padded "same" correlation, C1 = 0.01^2, C2 = 0.03^2;
 *   loss = (1 - lambda) mean|img - target| + lambda (1 - mean SSIM)
 * over every element of the packed [3][H][W] images of all views, and
 * d_images = d loss / d images (same layout; sign(0) = 0 for the L1 term).
 * loss (device float[1]) is reduced in a fixed order.  workspace holds three
 * partial-derivative maps and per-tile partial sums.
 */
int gs_loss_ssim_l1(const float* images, const float* targets, int n_views, const int32_t* sizes, float lambda,
                    float* loss, float* d_images, void* workspace, size_t workspace_bytes, void* stream);

/*
 * gs_morton_workspace_size - bytes of device workspace gs_morton_order needs.
 */
size_t gs_morton_workspace_size(int64_t n);

/*
 * gs_morton_order - 3-D Morton order of the Gaussians (paper Section 5.2:
 * the Gaussians are Morton-sorted in 3-D during densification to improve the
 * locality of rasterisation).  Each mean is quantised per axis to a 10-bit
 * cell c_k = clamp(floor((mu_k - origin_k) * inv_cell_k), 0, 1023), computed
 * in float32 as one subtraction then one multiplication (non-finite values
 * land in cell 0); the 30-bit code has bit 3b + k equal to bit b of c_k
 * (x: k = 0, y: 1, z: 2).  order[i] (int32, [N]) is the index of the Gaussian
 * with the i-th smallest code, equal codes in index order (stable).
 * origin, inv_cell are host float[3]; means is the planar [3][N] array.
 */
int gs_morton_order(const float* means, int64_t n, const float* origin, const float* inv_cell, void* workspace,
                    size_t workspace_bytes, int32_t* order, void* stream);

/*
 * gs_gather_columns - dst[c][i] = src[c][order[i]] for a planar [C][N]
 * float32 array: applies a permutation such as the Morton order to a
 * parameter (or gradient, or optimiser state) tensor.  src and dst must not
 * overlap.
 */
int gs_gather_columns(const float* src, int channels, int64_t n, const int32_t* order, float* dst,
                      void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
