// extern "C" entry points of include/gs.h: host-side argument checks, the
// per-launch view table, and kernel launches on the caller's stream.
#include <cmath>

#include "gs_device.h"

namespace gs {
hipError_t launch_project(int deg, const float* means, const float* log_scales, const float* quats,
                          const float* opac, const float* sh, long long N, const float* viewmats,
                          const float* intr, const ViewTable& vt, float near_plane, float far_plane,
                          float eps2d, int tile, int radius_mode, float* splats, float* depths, int2* radii,
                          int* tiles, int2* rects, uint8_t* flags, float* g2clear, hipStream_t stream);
hipError_t launch_densify_stats(const float* grad2d, const uint8_t* flags, const int2* radii, long long N,
                                const ViewTable& vt, float* grad_accum, int* count, int* max_radius,
                                hipStream_t st);
hipError_t launch_project_bwd(int deg, const float* means, const float* log_scales,
                              const float* quats, const float* opac, const float* sh, long long N,
                              const float* viewmats, const float* intr, const ViewTable& vt,
                              float eps2d, const uint8_t* flags, const float* grad2d,
                              float* d_means, float* d_log_scales, float* d_quats, float* d_opac,
                              float* d_sh, int part, hipStream_t stream);
hipError_t launch_project_bwd_adam(int deg, float* means, float* log_scales, float* quats, float* opac, float* sh,
                                   long long N, const float* viewmats, const float* intr, const ViewTable& vt,
                                   float eps2d, const uint8_t* flags, const float* grad2d, float* const* exp_avg,
                                   float* const* exp_avg_sq, const float* lrs, float beta1, float beta2, float eps,
                                   int* step_dev, hipStream_t stream);
size_t bin_sort_workspace_size(unsigned long long vn, unsigned long long cap);
hipError_t launch_bin_sort(const int2* rects, const float* depths, long long N, const ViewTable& vt,
                           unsigned long long cap, void* workspace, uint32_t* isect_tile,
                           uint32_t* isect_gid, int2* ranges, int* info, hipStream_t st);
size_t tile_schedule_size(long long total_tiles);
hipError_t launch_tile_schedule(const int2* ranges, long long total_tiles, void* schedule,
                                hipStream_t st);
bool raster_cfg_ok(int tile, int bw, int ppl);
hipError_t launch_raster_fwd(int tile, int bw, int ppl, const ViewTable& vt, const float* splats,
                             const int* gids, const int2* ranges, long long N, const float* bg,
                             const int* order, int* queue, float* img, float* Tout, int* lastout, int* visits,
                             hipStream_t st);
hipError_t launch_raster_bwd(int tile, int bw, int ppl, const ViewTable& vt, const float* splats,
                             const int* gids, const int2* ranges, long long N, const float* bg,
                             const int* order, int* queue, const float* Tfin, const int* nlast,
                             const float* dimg, const float* dalpha, float* grad2d, hipStream_t st);
size_t raster_bwd_l2_workspace_size(const ViewTable& vt, int tile);
hipError_t launch_raster_bwd_l2(int tile, int bw, int ppl, const ViewTable& vt, const float* splats,
                                const int* gids, const int2* ranges, long long N, const float* bg,
                                const int* order, const float* Tfin, const int* nlast, const float* img,
                                const float* tgt, long long n_elems, float* loss, void* part, float* grad2d,
                                const uint8_t* flags, int sh_degree, float* const* unseen_grads, hipStream_t st);
size_t loss_workspace_size(long long n);
hipError_t launch_fill_i32(int* p, int value, long long n, hipStream_t st);
size_t morton_workspace_size(long long n);
hipError_t launch_tile_order_xcd(long long total_tiles, int n_xcd, void* schedule, hipStream_t st);
size_t ssim_workspace_size(const ViewTable& vt);
hipError_t launch_ssim_l1(const ViewTable& vt, const float* img, const float* tgt, float lam, float* loss,
                          float* dimg, void* workspace, hipStream_t st);
hipError_t launch_morton_order(const float* means, long long n, const float* org, const float* inv_cell,
                               void* workspace, int* order, hipStream_t st);
hipError_t launch_gather_columns(const float* src, int C, long long n, const int* order, float* dst,
                                 hipStream_t st);
hipError_t launch_adam(int n_tensors, float* const* params, const float* const* grads, float* const* exp_avg,
                       float* const* exp_avg_sq, const int64_t* numel, const float* lrs, float beta1,
                       float beta2, float eps, int* step_dev, hipStream_t st);
hipError_t launch_loss_l2(const float* img, const float* tgt, long long n, float* loss, float* dimg,
                          void* ws, hipStream_t st);
hipError_t launch_loss_l2_noalloc(const float* img, const float* tgt, long long n, float* loss, float* dimg,
                                  hipStream_t st);
}  // namespace gs

namespace {

using gs::ViewTable;

bool tile_ok(int tile) { return tile == 8 || tile == 16 || tile == 32; }

// Fills the view table from host sizes; returns false on a bad size list.
bool make_views(const int32_t* sizes, int n_views, int tile, ViewTable& vt)
{
    if (!sizes || n_views < 1 || n_views > GS_MAX_VIEWS) return false;
    vt.n_views = n_views;
    vt.tile_off[0] = 0;
    vt.pix_off[0] = 0;
    long long tiles = 0, pix = 0;
    for (int v = 0; v < n_views; v++) {
        const int W = sizes[2 * v], H = sizes[2 * v + 1];
        if (W <= 0 || H <= 0 || W > 32767 || H > 32767) return false;
        const int TX = (W + tile - 1) / tile, TY = (H + tile - 1) / tile;
        vt.W[v] = W;
        vt.H[v] = H;
        vt.tiles_x[v] = TX;
        tiles += (long long)TX * TY;
        pix += (long long)W * H;
        if (tiles > 0x3FFFFFFFll) return false;
        vt.tile_off[v + 1] = (int)tiles;
        vt.pix_off[v + 1] = pix;
    }
    vt.total_tiles = (int)tiles;
    return true;
}

int status(hipError_t e) { return e == hipSuccess ? GS_OK : GS_ERR_HIP; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// The checks and launch of gs_project_bwd and gs_project_bwd_part: the
// parameters and the 2-D gradients are needed unless only the gradients of
// unseen Gaussians (zeros) are written.
int project_bwd_checked(const float* means, const float* log_scales, const float* quats,
                        const float* opacity_logits, const float* sh, int64_t n, int sh_degree,
                        const float* viewmats, const float* intrinsics, const int32_t* sizes, int n_views,
                        float eps2d, const uint8_t* flags, const float* grad2d, float* d_means,
                        float* d_log_scales, float* d_quats, float* d_opacity_logits, float* d_sh, int part,
                        void* stream)
{
    ViewTable vt;
    if (n < 0 || n > 0x7FFFFFFFll || sh_degree < 0 || sh_degree > 3 || !make_views(sizes, n_views, 16, vt))
        return GS_ERR_ARG;
    if (part != GS_GRADS_ALL && part != GS_GRADS_SEEN && part != GS_GRADS_UNSEEN) return GS_ERR_ARG;
    const bool inputs = part != GS_GRADS_UNSEEN;
    if (inputs && !(eps2d >= 0.0f)) return GS_ERR_ARG;
    if (n == 0) return GS_OK;
    if (!flags || !d_means || !d_log_scales || !d_quats || !d_opacity_logits || !d_sh) return GS_ERR_ARG;
    if (inputs && (!means || !log_scales || !quats || !opacity_logits || !sh || !viewmats || !intrinsics || !grad2d))
        return GS_ERR_ARG;
    return status(gs::launch_project_bwd(sh_degree, means, log_scales, quats, opacity_logits, sh, n, viewmats,
                                         intrinsics, vt, eps2d, flags, grad2d, d_means, d_log_scales, d_quats,
                                         d_opacity_logits, d_sh, part, as_stream(stream)));
}

}  // namespace

extern "C" {

int gs_abi_version(void) { return GS_ABI_VERSION; }

const char* gs_strerror(int code)
{
    switch (code) {
    case GS_OK: return "ok";
    case GS_ERR_ARG: return "invalid argument";
    case GS_ERR_UNSUPPORTED: return "unsupported request";
    case GS_ERR_HIP: return "HIP launch or runtime error";
    case GS_ERR_WORKSPACE: return "workspace too small";
    default: return "unknown gs_status";
    }
}

int gs_project(const float* means, const float* log_scales, const float* quats,
               const float* opacity_logits, const float* sh, int64_t n, int sh_degree,
               const float* viewmats, const float* intrinsics, const int32_t* sizes, int n_views,
               float near_plane, float far_plane, float eps2d, int tile, int radius_mode, float* splats,
               float* depths, int32_t* radii, int32_t* tiles_touched, int32_t* tile_rects, uint8_t* flags,
               float* grad2d_clear, void* stream)
{
    ViewTable vt;
    if (n < 0 || n > 0x7FFFFFFFll || sh_degree < 0 || sh_degree > 3 || !tile_ok(tile) ||
        !make_views(sizes, n_views, tile, vt))
        return GS_ERR_ARG;
    if (radius_mode != GS_RADIUS_3SIGMA && radius_mode != GS_RADIUS_OPACITY && radius_mode != GS_RADIUS_EIGEN)
        return GS_ERR_ARG;
    if ((unsigned long long)n * (unsigned long long)n_views > 0xFFFFFFFFull) return GS_ERR_ARG;
    if (!(eps2d >= 0.0f) || !(near_plane > 0.0f) || !(far_plane > near_plane)) return GS_ERR_ARG;
    if (n == 0) return GS_OK;
    if (!means || !log_scales || !quats || !opacity_logits || !sh || !viewmats || !intrinsics ||
        !splats || !depths || !radii || !tiles_touched || !tile_rects || !flags || !aligned16(splats))
        return GS_ERR_ARG;
    return status(gs::launch_project(sh_degree, means, log_scales, quats, opacity_logits, sh, n, viewmats,
                                     intrinsics, vt, near_plane, far_plane, eps2d, tile, radius_mode, splats,
                                     depths, reinterpret_cast<int2*>(radii), tiles_touched,
                                     reinterpret_cast<int2*>(tile_rects), flags, grad2d_clear,
                                     as_stream(stream)));
}

size_t gs_bin_sort_workspace_size(int64_t n, int n_views, int64_t capacity, int64_t total_tiles)
{
    (void)total_tiles;
    if (n < 0 || n_views < 1 || capacity < 1) return 0;
    return gs::bin_sort_workspace_size((unsigned long long)n * (unsigned long long)n_views,
                                       (unsigned long long)capacity);
}

int gs_bin_sort(const int32_t* tile_rects, const float* depths, int64_t n, int n_views, const int32_t* sizes,
                int tile, int64_t capacity, void* workspace, size_t workspace_bytes, int32_t* isect_tile,
                int32_t* isect_gid, int32_t* tile_ranges, int32_t* info, void* stream)
{
    ViewTable vt;
    if (n < 0 || n > 0x7FFFFFFFll || !tile_ok(tile) || !make_views(sizes, n_views, tile, vt))
        return GS_ERR_ARG;
    if ((unsigned long long)n * (unsigned long long)n_views > 0xFFFFFFFFull) return GS_ERR_ARG;
    if (capacity < 1 || capacity > 0x7FFFFFFFll) return GS_ERR_ARG;
    if (!isect_tile || !isect_gid || !tile_ranges || !info || !workspace) return GS_ERR_ARG;
    if (n > 0 && (!tile_rects || !depths)) return GS_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return GS_ERR_ARG;
    if (workspace_bytes < gs_bin_sort_workspace_size(n, n_views, capacity, vt.total_tiles))
        return GS_ERR_WORKSPACE;
    return status(gs::launch_bin_sort(reinterpret_cast<const int2*>(tile_rects), depths, n, vt,
                                      (unsigned long long)capacity, workspace,
                                      reinterpret_cast<uint32_t*>(isect_tile),
                                      reinterpret_cast<uint32_t*>(isect_gid),
                                      reinterpret_cast<int2*>(tile_ranges), info, as_stream(stream)));
}

size_t gs_tile_schedule_size(int64_t total_tiles)
{
    if (total_tiles < 1 || total_tiles > 0x3FFFFFFFll) return 0;
    return gs::tile_schedule_size(total_tiles);
}

int gs_tile_schedule(const int32_t* tile_ranges, int64_t total_tiles, void* schedule,
                     size_t schedule_bytes, void* stream)
{
    if (!tile_ranges || !schedule || total_tiles < 1 || total_tiles > 0x3FFFFFFFll) return GS_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(schedule) & 255u) != 0) return GS_ERR_ARG;
    if (schedule_bytes < gs::tile_schedule_size(total_tiles)) return GS_ERR_WORKSPACE;
    return status(gs::launch_tile_schedule(reinterpret_cast<const int2*>(tile_ranges), total_tiles, schedule,
                                           as_stream(stream)));
}

int gs_tile_order_xcd(int64_t total_tiles, int n_xcd, void* schedule, size_t schedule_bytes, void* stream)
{
    if (total_tiles < 1 || total_tiles > 0x3FFFFFFFll || n_xcd < 1 || n_xcd > 64 || !schedule) return GS_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(schedule) & 255u) != 0) return GS_ERR_ARG;
    if (schedule_bytes < gs::tile_schedule_size(total_tiles)) return GS_ERR_WORKSPACE;
    return status(gs::launch_tile_order_xcd(total_tiles, n_xcd, schedule, as_stream(stream)));
}

int gs_rasterize_fwd(const float* splats, const int32_t* isect_gid, const int32_t* tile_ranges,
                     int64_t n, int n_views, const int32_t* sizes, int tile, int block_w, int px_per_lane,
                     const float* background, const void* schedule, int32_t* queue, float* images,
                     float* T_final, int32_t* n_contrib, void* stream)
{
    ViewTable vt;
    if (n < 0 || n > 0x7FFFFFFFll || !tile_ok(tile) || !make_views(sizes, n_views, tile, vt))
        return GS_ERR_ARG;
    if (!gs::raster_cfg_ok(tile, block_w, px_per_lane)) return GS_ERR_ARG;
    if (!tile_ranges || !images || !T_final || !n_contrib || !background) return GS_ERR_ARG;
    if (!isect_gid || (n > 0 && (!splats || !aligned16(splats)))) return GS_ERR_ARG;
    if (queue && !schedule) return GS_ERR_ARG;
    for (int c = 0; c < 3; c++)
        if (!std::isfinite(background[c])) return GS_ERR_ARG;
    return status(gs::launch_raster_fwd(tile, block_w, px_per_lane, vt, splats, isect_gid,
                                        reinterpret_cast<const int2*>(tile_ranges), n, background,
                                        static_cast<const int*>(schedule), queue, images, T_final, n_contrib,
                                        nullptr, as_stream(stream)));
}

int gs_rasterize_bwd(const float* splats, const int32_t* isect_gid, const int32_t* tile_ranges,
                     int64_t n, int n_views, const int32_t* sizes, int tile, int block_w, int px_per_lane,
                     const float* background, const void* schedule, int32_t* queue, const float* T_final,
                     const int32_t* n_contrib, const float* d_images, const float* d_alpha,
                     float* grad2d, int accumulate, void* stream)
{
    ViewTable vt;
    if (n < 0 || n > 0x7FFFFFFFll || !tile_ok(tile) || !make_views(sizes, n_views, tile, vt))
        return GS_ERR_ARG;
    if (!tile_ranges || !T_final || !n_contrib || !d_images || !grad2d || !background || !isect_gid)
        return GS_ERR_ARG;
    if (!gs::raster_cfg_ok(tile, block_w, px_per_lane)) return GS_ERR_ARG;
    if (n > 0 && (!splats || !aligned16(splats))) return GS_ERR_ARG;
    if (queue && !schedule) return GS_ERR_ARG;
    for (int c = 0; c < 3; c++)
        if (!std::isfinite(background[c])) return GS_ERR_ARG;
    if (!accumulate) {
        const hipError_t e = gs::launch_fill_i32(reinterpret_cast<int*>(grad2d), 0,
                                                 n * n_views * GS_GRAD_FLOATS, as_stream(stream));
        if (e != hipSuccess) return GS_ERR_HIP;
    }
    return status(gs::launch_raster_bwd(tile, block_w, px_per_lane, vt, splats, isect_gid,
                                        reinterpret_cast<const int2*>(tile_ranges), n, background,
                                        static_cast<const int*>(schedule), queue, T_final, n_contrib, d_images,
                                        d_alpha, grad2d, as_stream(stream)));
}

size_t gs_rasterize_bwd_l2_workspace_size(int n_views, const int32_t* sizes, int tile)
{
    ViewTable vt;
    if (!tile_ok(tile) || !make_views(sizes, n_views, tile, vt)) return 0;
    return gs::raster_bwd_l2_workspace_size(vt, tile);
}

int gs_rasterize_bwd_l2(const float* splats, const int32_t* isect_gid, const int32_t* tile_ranges, int64_t n,
                        int n_views, const int32_t* sizes, int tile, int block_w, int px_per_lane,
                        const float* background, const void* schedule, const float* T_final,
                        const int32_t* n_contrib, const float* images, const float* targets, float* loss,
                        float* grad2d, int accumulate, void* workspace, size_t workspace_bytes,
                        const uint8_t* flags, int sh_degree, float* const* unseen_grads, void* stream)
{
    ViewTable vt;
    if (n < 0 || n > 0x7FFFFFFFll || !tile_ok(tile) || !make_views(sizes, n_views, tile, vt))
        return GS_ERR_ARG;
    if (!tile_ranges || !T_final || !n_contrib || !images || !targets || !loss || !grad2d || !background ||
        !isect_gid || !workspace)
        return GS_ERR_ARG;
    if (unseen_grads) {
        if (!flags || sh_degree < 0 || sh_degree > 3) return GS_ERR_ARG;
        for (int k = 0; k < 5; k++)
            if (n > 0 && !unseen_grads[k]) return GS_ERR_ARG;
    }
    if (!gs::raster_cfg_ok(tile, block_w, px_per_lane)) return GS_ERR_ARG;
    if (n > 0 && (!splats || !aligned16(splats))) return GS_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(workspace) & 7u) != 0) return GS_ERR_ARG;
    for (int c = 0; c < 3; c++)
        if (!std::isfinite(background[c])) return GS_ERR_ARG;
    if (workspace_bytes < gs::raster_bwd_l2_workspace_size(vt, tile)) return GS_ERR_WORKSPACE;
    if (!accumulate) {
        const hipError_t e = gs::launch_fill_i32(reinterpret_cast<int*>(grad2d), 0,
                                                 n * n_views * GS_GRAD_FLOATS, as_stream(stream));
        if (e != hipSuccess) return GS_ERR_HIP;
    }
    return status(gs::launch_raster_bwd_l2(tile, block_w, px_per_lane, vt, splats, isect_gid,
                                           reinterpret_cast<const int2*>(tile_ranges), n, background,
                                           static_cast<const int*>(schedule), T_final, n_contrib, images, targets,
                                           3ll * vt.pix_off[n_views], loss, workspace, grad2d,
                                           unseen_grads ? flags : nullptr, sh_degree, unseen_grads,
                                           as_stream(stream)));
}

int gs_project_bwd(const float* means, const float* log_scales, const float* quats,
                   const float* opacity_logits, const float* sh, int64_t n, int sh_degree,
                   const float* viewmats, const float* intrinsics, const int32_t* sizes, int n_views,
                   float eps2d, const uint8_t* flags, const float* grad2d, float* d_means,
                   float* d_log_scales, float* d_quats, float* d_opacity_logits, float* d_sh,
                   void* stream)
{
    return project_bwd_checked(means, log_scales, quats, opacity_logits, sh, n, sh_degree, viewmats, intrinsics,
                               sizes, n_views, eps2d, flags, grad2d, d_means, d_log_scales, d_quats,
                               d_opacity_logits, d_sh, GS_GRADS_ALL, stream);
}

int gs_project_bwd_part(const float* means, const float* log_scales, const float* quats,
                        const float* opacity_logits, const float* sh, int64_t n, int sh_degree,
                        const float* viewmats, const float* intrinsics, const int32_t* sizes, int n_views,
                        float eps2d, const uint8_t* flags, const float* grad2d, float* d_means,
                        float* d_log_scales, float* d_quats, float* d_opacity_logits, float* d_sh, int part,
                        void* stream)
{
    return project_bwd_checked(means, log_scales, quats, opacity_logits, sh, n, sh_degree, viewmats, intrinsics,
                               sizes, n_views, eps2d, flags, grad2d, d_means, d_log_scales, d_quats,
                               d_opacity_logits, d_sh, part, stream);
}

int gs_project_bwd_adam(float* means, float* log_scales, float* quats, float* opacity_logits, float* sh,
                        int64_t n, int sh_degree, const float* viewmats, const float* intrinsics,
                        const int32_t* sizes, int n_views, float eps2d, const uint8_t* flags, const float* grad2d,
                        float* const* exp_avg, float* const* exp_avg_sq, const float* lrs, float beta1,
                        float beta2, float eps, int32_t* step, void* stream)
{
    ViewTable vt;
    // N <= 2^30: the kernel addresses a parameter plane with a 32-bit byte
    // offset (4 N bytes)
    if (n < 0 || n > (1ll << 30) || sh_degree < 0 || sh_degree > 3 || !make_views(sizes, n_views, 16, vt))
        return GS_ERR_ARG;
    if (!(eps2d >= 0.0f) || !exp_avg || !exp_avg_sq || !lrs || !step) return GS_ERR_ARG;
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) return GS_ERR_ARG;
    float* const params[5] = {means, log_scales, quats, opacity_logits, sh};
    for (int k = 0; k < 5; k++) {
        if (!std::isfinite(lrs[k])) return GS_ERR_ARG;
        if (n > 0 && (!params[k] || !exp_avg[k] || !exp_avg_sq[k])) return GS_ERR_ARG;
    }
    if (n > 0 && (!viewmats || !intrinsics || !flags || !grad2d)) return GS_ERR_ARG;
    return status(gs::launch_project_bwd_adam(sh_degree, means, log_scales, quats, opacity_logits, sh, n, viewmats,
                                              intrinsics, vt, eps2d, flags, grad2d, exp_avg, exp_avg_sq, lrs, beta1,
                                              beta2, eps, step, as_stream(stream)));
}

int gs_raster_visits(const float* splats, const int32_t* isect_gid, const int32_t* tile_ranges, int64_t n,
                     int n_views, const int32_t* sizes, int tile, float* images, float* T_final,
                     int32_t* n_contrib, int32_t* visits, void* stream)
{
    ViewTable vt;
    if (n < 0 || n > 0x7FFFFFFFll || !tile_ok(tile) || !make_views(sizes, n_views, tile, vt))
        return GS_ERR_ARG;
    if (!tile_ranges || !images || !T_final || !n_contrib || !visits || !isect_gid) return GS_ERR_ARG;
    if (n > 0 && (!splats || !aligned16(splats))) return GS_ERR_ARG;
    const float bg[3] = {0.0f, 0.0f, 0.0f};
    return status(gs::launch_raster_fwd(tile, 0, 0, vt, splats, isect_gid,
                                        reinterpret_cast<const int2*>(tile_ranges), n, bg, nullptr, nullptr, images,
                                        T_final, n_contrib, visits, as_stream(stream)));
}

size_t gs_loss_workspace_size(int64_t n_elems)
{
    if (n_elems < 0) return 0;
    return gs::loss_workspace_size(n_elems);
}

int gs_loss_l2(const float* images, const float* targets, int64_t n_elems, float* loss, float* d_images,
               void* workspace, size_t workspace_bytes, void* stream)
{
    if (n_elems < 0 || !loss || !workspace) return GS_ERR_ARG;
    if (n_elems > 0 && (!images || !targets || !d_images)) return GS_ERR_ARG;
    if (workspace_bytes < gs::loss_workspace_size(n_elems)) return GS_ERR_WORKSPACE;
    return status(gs::launch_loss_l2(images, targets, n_elems, loss, d_images, workspace, as_stream(stream)));
}

int gs_loss_l2_noalloc(const float* images, const float* targets, int64_t n_elems, float* loss, float* d_images,
                       void* stream)
{
    if (n_elems < 0 || !loss) return GS_ERR_ARG;
    if (n_elems > 0 && (!images || !targets || !d_images)) return GS_ERR_ARG;
    return status(gs::launch_loss_l2_noalloc(images, targets, n_elems, loss, d_images, as_stream(stream)));
}

int gs_adam(int n_tensors, float* const* params, const float* const* grads, float* const* exp_avg,
            float* const* exp_avg_sq, const int64_t* numel, const float* lrs, float beta1, float beta2,
            float eps, int32_t* step, void* stream)
{
    if (n_tensors < 1 || n_tensors > GS_ADAM_MAX_TENSORS || !params || !grads || !exp_avg || !exp_avg_sq ||
        !numel || !lrs || !step)
        return GS_ERR_ARG;
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) return GS_ERR_ARG;
    for (int k = 0; k < n_tensors; k++) {
        if (numel[k] < 0 || !std::isfinite(lrs[k])) return GS_ERR_ARG;
        if (numel[k] > 0 && (!params[k] || !grads[k] || !exp_avg[k] || !exp_avg_sq[k])) return GS_ERR_ARG;
        if (numel[k] > 0 && (!aligned16(params[k]) || !aligned16(grads[k]) || !aligned16(exp_avg[k]) ||
                             !aligned16(exp_avg_sq[k])))
            return GS_ERR_ARG;
    }
    return status(gs::launch_adam(n_tensors, params, grads, exp_avg, exp_avg_sq, numel, lrs, beta1, beta2, eps, step,
                                  as_stream(stream)));
}

size_t gs_morton_workspace_size(int64_t n)
{
    if (n < 1 || n > 0x7FFFFFFFll) return 0;
    return gs::morton_workspace_size(n);
}

int gs_morton_order(const float* means, int64_t n, const float* origin, const float* inv_cell, void* workspace,
                    size_t workspace_bytes, int32_t* order, void* stream)
{
    if (n < 1 || n > 0x7FFFFFFFll || !means || !origin || !inv_cell || !workspace || !order) return GS_ERR_ARG;
    for (int k = 0; k < 3; k++)
        if (!std::isfinite(origin[k]) || !std::isfinite(inv_cell[k])) return GS_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return GS_ERR_ARG;
    if (workspace_bytes < gs::morton_workspace_size(n)) return GS_ERR_WORKSPACE;
    return status(gs::launch_morton_order(means, n, origin, inv_cell, workspace, order, as_stream(stream)));
}

int gs_gather_columns(const float* src, int channels, int64_t n, const int32_t* order, float* dst, void* stream)
{
    if (channels < 0 || n < 0 || n > 0x7FFFFFFFll) return GS_ERR_ARG;
    if (channels > 0 && n > 0 && (!src || !order || !dst || src == dst)) return GS_ERR_ARG;
    return status(gs::launch_gather_columns(src, channels, n, order, dst, as_stream(stream)));
}

size_t gs_ssim_workspace_size(int n_views, const int32_t* sizes)
{
    ViewTable vt;
    if (!make_views(sizes, n_views, 16, vt)) return 0;
    return gs::ssim_workspace_size(vt);
}

int gs_loss_ssim_l1(const float* images, const float* targets, int n_views, const int32_t* sizes, float lambda,
                    float* loss, float* d_images, void* workspace, size_t workspace_bytes, void* stream)
{
    ViewTable vt;
    if (!make_views(sizes, n_views, 16, vt)) return GS_ERR_ARG;
    if (!images || !targets || !loss || !d_images || !workspace || !(lambda >= 0.0f && lambda <= 1.0f))
        return GS_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return GS_ERR_ARG;
    if (workspace_bytes < gs::ssim_workspace_size(vt)) return GS_ERR_WORKSPACE;
    return status(gs::launch_ssim_l1(vt, images, targets, lambda, loss, d_images, workspace, as_stream(stream)));
}

int gs_densify_stats(const float* grad2d, const uint8_t* flags, const int32_t* radii, int64_t n, int n_views,
                     const int32_t* sizes, float* grad_accum, int32_t* count, int32_t* max_radius, void* stream)
{
    ViewTable vt;
    if (n < 0 || n > 0x7FFFFFFFll || !make_views(sizes, n_views, 16, vt)) return GS_ERR_ARG;
    if ((unsigned long long)n * (unsigned long long)n_views > 0xFFFFFFFFull) return GS_ERR_ARG;
    if (n == 0) return GS_OK;
    if (!grad2d || !flags || !radii || !grad_accum || !count || !max_radius) return GS_ERR_ARG;
    return status(gs::launch_densify_stats(grad2d, flags, reinterpret_cast<const int2*>(radii), n, vt, grad_accum,
                                           count, max_radius, as_stream(stream)));
}

}  // extern "C"
