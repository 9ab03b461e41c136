// Front-to-back alpha compositing, forward and backward (gfx950).
//
// Paper Section 4: the rasterisation operator renders one camera (or a tile
// of it) after the depth sort, and its backward accumulates gradients into
// the Gaussians with atomics.  The compositing rule is that of 3D Gaussian
// Splatting: per pixel, over its tile's depth-sorted list,
//   alpha = min(0.99, sigma * exp(-d^T Q d / 2)), skip alpha < 1/255,
//   stop before T would drop below 1e-4, C += alpha T c, T *= 1 - alpha.
//
// GPU organisation.  A work unit is one wavefront covering a band of a tile;
// lane l owns P horizontally adjacent pixels.  Every lane of a wave walks the
// same list position at the same time, so each splat record is fetched with
// wave-uniform addresses: the compiler issues scalar (SMEM) loads through the
// scalar cache and the VALU reads the record from SGPRs.  This replaces the
// usual LDS staging: a broadcast LDS read still returns 64 copies of the data
// through the LDS return path, while an SGPR operand costs nothing extra.
// Waves of a tile never synchronise; each stops as soon as all of its pixels
// have terminated (ballot).  The backward walks the same list from the back,
// recovers T before each entry by dividing by (1 - alpha), and pre-reduces the
// nine per-Gaussian gradient values across the wave with DPP before one lane
// per value issues a float atomic.
#include "gs_device.h"

namespace gs {
namespace {

struct Rec {
    float u, v, m00, m10, m11, ls, r, g, b;
};

__device__ __forceinline__ Rec load_rec(const float* __restrict__ base, int gid)
{
    const float4* p = reinterpret_cast<const float4*>(base + (size_t)gid * GS_SPLAT_FLOATS);
    const float4 a = p[0], b = p[1];
    const float c = base[(size_t)gid * GS_SPLAT_FLOATS + 8];
    return Rec{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c};
}

template <int TS, int P>
struct Layout {
    static constexpr int LPR = TS / P;          // lanes per pixel row
    static constexpr int ROWS = GS_WAVE / LPR;  // pixel rows per wave
    static constexpr int WPT = TS / ROWS;       // waves per tile
    static_assert(TS % P == 0 && GS_WAVE % LPR == 0 && TS % ROWS == 0, "bad raster layout");
};

template <int TS, int P>
__device__ __forceinline__ void unit_pixels(const ViewTable& vt, int gt, int wit, int& v, int& px0,
                                            int& py)
{
    using L = Layout<TS, P>;
    v = view_of_tile(vt, gt);
    const int lt = gt - vt.tile_off[v];
    const int TX = vt.tiles_x[v];
    const int ty = lt / TX, tx = lt - ty * TX;
    const int lane = __lane_id();
    px0 = tx * TS + (lane % L::LPR) * P;
    py = ty * TS + wit * L::ROWS + lane / L::LPR;
}

template <int TS, int P, bool COUNT>
__device__ __forceinline__ void fwd_unit(const ViewTable& vt, int gt, int wit,
                                         const float* __restrict__ splats,
                                         const int* __restrict__ gids,
                                         const int2* __restrict__ ranges, long long N, float bg0,
                                         float bg1, float bg2, float* __restrict__ img,
                                         float* __restrict__ Tout, int* __restrict__ lastout,
                                         int* __restrict__ visits)
{
    int v, px0, py;
    unit_pixels<TS, P>(vt, gt, wit, v, px0, py);
    const int W = vt.W[v], H = vt.H[v];
    const float fy = (float)py + 0.5f;
    float fx[P], T[P], C0[P], C1[P], C2[P];
    int last[P], nvis[P];
    bool done[P];
#pragma unroll
    for (int p = 0; p < P; p++) {
        fx[p] = (float)(px0 + p) + 0.5f;
        nvis[p] = 0;
        T[p] = 1.0f;
        C0[p] = C1[p] = C2[p] = 0.0f;
        last[p] = 0;
        done[p] = !(px0 + p < W && py < H);
    }
    const int2 r = ranges[gt];
    const float* base = splats + (size_t)v * (size_t)N * GS_SPLAT_FLOATS;
    for (int k = r.x; k < r.y; k++) {
        bool all_done = true;
#pragma unroll
        for (int p = 0; p < P; p++) all_done = all_done && done[p];
        if (__ballot(!all_done) == 0ull) break;
        const Rec s = load_rec(base, gids[k]);
        const float dy = s.v - fy;
        const int k1 = k - r.x + 1;
#pragma unroll
        for (int p = 0; p < P; p++) {
            const Falloff f = falloff(s.u - fx[p], dy, s.m00, s.m10, s.m11, s.ls);
            const float al = fminf(f.araw, kAlphaMax);
            if (COUNT) nvis[p] += done[p] ? 0 : 1;
            bool ok = !done[p] && al >= kAlphaMin;
            const float Tn = __builtin_fmaf(-T[p], al, T[p]);
            const bool stop = ok && Tn < kTMin;
            done[p] = done[p] || stop;
            ok = ok && !stop;
            const float wgt = ok ? al * T[p] : 0.0f;
            C0[p] = __builtin_fmaf(wgt, s.r, C0[p]);
            C1[p] = __builtin_fmaf(wgt, s.g, C1[p]);
            C2[p] = __builtin_fmaf(wgt, s.b, C2[p]);
            T[p] = ok ? Tn : T[p];
            last[p] = ok ? k1 : last[p];
        }
    }
    const long long po = vt.pix_off[v];
    const long long plane = (long long)W * H;
#pragma unroll
    for (int p = 0; p < P; p++) {
        if (px0 + p < W && py < H) {
            const long long pix = (long long)py * W + px0 + p;
            img[3 * po + pix] = __builtin_fmaf(T[p], bg0, C0[p]);
            img[3 * po + plane + pix] = __builtin_fmaf(T[p], bg1, C1[p]);
            img[3 * po + 2 * plane + pix] = __builtin_fmaf(T[p], bg2, C2[p]);
            Tout[po + pix] = T[p];
            lastout[po + pix] = last[p];
            if (COUNT) visits[po + pix] = nvis[p];
        }
    }
}

template <int TS, int P, bool HAS_DA>
__device__ __forceinline__ void bwd_unit(const ViewTable& vt, int gt, int wit,
                                         const float* __restrict__ splats,
                                         const int* __restrict__ gids,
                                         const int2* __restrict__ ranges, long long N, float bg0,
                                         float bg1, float bg2, const float* __restrict__ Tfin,
                                         const int* __restrict__ nlast,
                                         const float* __restrict__ dimg,
                                         const float* __restrict__ dalpha,
                                         float* __restrict__ grad2d)
{
    int v, px0, py;
    unit_pixels<TS, P>(vt, gt, wit, v, px0, py);
    const int W = vt.W[v], H = vt.H[v];
    const long long po = vt.pix_off[v];
    const long long plane = (long long)W * H;
    const float fy = (float)py + 0.5f;
    float fx[P], T[P], TN[P], S0[P], S1[P], S2[P], g0[P], g1[P], g2[P], gA[P];
    int last[P];
    int kmax = 0;
#pragma unroll
    for (int p = 0; p < P; p++) {
        fx[p] = (float)(px0 + p) + 0.5f;
        const bool in = px0 + p < W && py < H;
        const long long pix = (long long)py * W + px0 + p;
        T[p] = in ? Tfin[po + pix] : 1.0f;
        TN[p] = T[p];
        last[p] = in ? nlast[po + pix] : 0;
        g0[p] = in ? dimg[3 * po + pix] : 0.0f;
        g1[p] = in ? dimg[3 * po + plane + pix] : 0.0f;
        g2[p] = in ? dimg[3 * po + 2 * plane + pix] : 0.0f;
        gA[p] = (HAS_DA && in) ? dalpha[po + pix] * TN[p] : 0.0f;
        S0[p] = bg0;
        S1[p] = bg1;
        S2[p] = bg2;
        kmax = max(kmax, last[p]);
    }
    kmax = wave_max_i(kmax);
    const int2 r = ranges[gt];
    kmax = min(kmax, r.y - r.x);
    const float* base = splats + (size_t)v * (size_t)N * GS_SPLAT_FLOATS;
    float* gbase = grad2d + (size_t)v * (size_t)N * GS_GRAD_FLOATS;
    const int lane = __lane_id();
    for (int k = r.x + kmax - 1; k >= r.x; k--) {
        const int gid = gids[k];
        const Rec s = load_rec(base, gid);
        const float inv_sig = 1.0f / splats[(size_t)v * (size_t)N * GS_SPLAT_FLOATS +
                                            (size_t)gid * GS_SPLAT_FLOATS + 9];
        const float dy = s.v - fy;
        const int kk = k - r.x;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f, a6 = 0.f, a7 = 0.f, a8 = 0.f;
        bool any = false;
#pragma unroll
        for (int p = 0; p < P; p++) {
            const float dx = s.u - fx[p];
            const Falloff f = falloff(dx, dy, s.m00, s.m10, s.m11, s.ls);
            const float al = fminf(f.araw, kAlphaMax);
            const bool ok = kk < last[p] && al >= kAlphaMin;
            any = any || ok;
            const float om = 1.0f - al;
            const float rom = __builtin_amdgcn_rcpf(om);
            const float Tk = T[p] * rom;
            const float wgt = al * Tk;
            const float d0 = s.r - S0[p], d1 = s.g - S1[p], d2 = s.b - S2[p];
            float ga = Tk * (d0 * g0[p] + d1 * g1[p] + d2 * g2[p]);
            if (HAS_DA) ga = __builtin_fmaf(gA[p], rom, ga);
            const bool unc = ok && f.araw < kAlphaMax;
            const float gq = unc ? -kLn2 * al * ga : 0.0f;
            a6 += ok ? wgt * g0[p] : 0.0f;
            a7 += ok ? wgt * g1[p] : 0.0f;
            a8 += ok ? wgt * g2[p] : 0.0f;
            a5 += unc ? f.araw * inv_sig * ga : 0.0f;
            // q' = |M^T d|^2:  dq'/du = 2 (M w)_x, dq'/dv = 2 (M w)_y
            a0 += 2.0f * gq * (s.m00 * f.w0);
            a1 += 2.0f * gq * (s.m10 * f.w0 + s.m11 * f.w1);
            // q' = c0 (A dx^2 + 2 B dx dy + C dy^2)
            a2 += gq * kC0 * dx * dx;
            a3 += gq * (2.0f * kC0) * dx * dy;
            a4 += gq * kC0 * dy * dy;
            S0[p] = ok ? __builtin_fmaf(al, d0, S0[p]) : S0[p];
            S1[p] = ok ? __builtin_fmaf(al, d1, S1[p]) : S1[p];
            S2[p] = ok ? __builtin_fmaf(al, d2, S2[p]) : S2[p];
            T[p] = ok ? Tk : T[p];
        }
        if (__ballot(any) == 0ull) continue;
        const float r0 = wave_sum(a0), r1 = wave_sum(a1), r2 = wave_sum(a2);
        const float r3 = wave_sum(a3), r4 = wave_sum(a4), r5 = wave_sum(a5);
        const float r6 = wave_sum(a6), r7 = wave_sum(a7), r8 = wave_sum(a8);
        if (lane < GS_GRAD_FLOATS) {
            float x = r0;
            x = lane == 1 ? r1 : x;
            x = lane == 2 ? r2 : x;
            x = lane == 3 ? r3 : x;
            x = lane == 4 ? r4 : x;
            x = lane == 5 ? r5 : x;
            x = lane == 6 ? r6 : x;
            x = lane == 7 ? r7 : x;
            x = lane == 8 ? r8 : x;
            unsafeAtomicAdd(gbase + (size_t)gid * GS_GRAD_FLOATS + lane, x);
        }
    }
}

template <int TS, int P, bool COUNT>
__global__ __launch_bounds__((GS_WAVE * Layout<TS, P>::WPT)) void k_raster_fwd(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    float* __restrict__ img, float* __restrict__ Tout, int* __restrict__ lastout,
    int* __restrict__ visits)
{
    fwd_unit<TS, P, COUNT>(vt, blockIdx.x, threadIdx.x / GS_WAVE, splats, gids, ranges, N, bg0, bg1, bg2,
                           img, Tout, lastout, visits);
}

template <int TS, int P>
__global__ __launch_bounds__(GS_WAVE) void k_raster_fwd_persistent(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    const int* __restrict__ order, int* __restrict__ queue, float* __restrict__ img,
    float* __restrict__ Tout, int* __restrict__ lastout)
{
    using L = Layout<TS, P>;
    const int n_items = vt.total_tiles * L::WPT;
    for (;;) {
        int item = 0;
        if (__lane_id() == 0) item = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n_items) break;
        const int gt = order[item / L::WPT];
        fwd_unit<TS, P, false>(vt, gt, item % L::WPT, splats, gids, ranges, N, bg0, bg1, bg2, img, Tout,
                               lastout, nullptr);
    }
}

template <int TS, int P, bool HAS_DA>
__global__ __launch_bounds__((GS_WAVE * Layout<TS, P>::WPT)) void k_raster_bwd(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    const float* __restrict__ Tfin, const int* __restrict__ nlast, const float* __restrict__ dimg,
    const float* __restrict__ dalpha, float* __restrict__ grad2d)
{
    bwd_unit<TS, P, HAS_DA>(vt, blockIdx.x, threadIdx.x / GS_WAVE, splats, gids, ranges, N, bg0, bg1,
                            bg2, Tfin, nlast, dimg, dalpha, grad2d);
}

template <int TS, int P, bool HAS_DA>
__global__ __launch_bounds__(GS_WAVE) void k_raster_bwd_persistent(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    const int* __restrict__ order, int* __restrict__ queue, const float* __restrict__ Tfin,
    const int* __restrict__ nlast, const float* __restrict__ dimg, const float* __restrict__ dalpha,
    float* __restrict__ grad2d)
{
    using L = Layout<TS, P>;
    const int n_items = vt.total_tiles * L::WPT;
    for (;;) {
        int item = 0;
        if (__lane_id() == 0) item = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n_items) break;
        const int gt = order[item / L::WPT];
        bwd_unit<TS, P, HAS_DA>(vt, gt, item % L::WPT, splats, gids, ranges, N, bg0, bg1, bg2, Tfin,
                                nlast, dimg, dalpha, grad2d);
    }
}

__global__ void k_zero_queue(int* q) { q[0] = 0; }

int persistent_blocks()
{
    static int n = 0;
    if (n == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        n = cus * 32;
    }
    return n;
}

}  // namespace

// pixels per lane for each tile edge: the whole 8x8 tile is one wave at P=1,
// 16x16 and 32x32 tiles put four adjacent pixels of a row in each lane
template <int TS> struct RasterCfg;
template <> struct RasterCfg<8> { static constexpr int P = 1; };
template <> struct RasterCfg<16> { static constexpr int P = 4; };
template <> struct RasterCfg<32> { static constexpr int P = 4; };

template <int TS>
static hipError_t fwd_ts(const ViewTable& vt, const float* splats, const int* gids, const int2* ranges,
                         long long N, const float* bg, const int* order, int* queue, float* img,
                         float* Tout, int* lastout, int* visits, hipStream_t st)
{
    constexpr int P = RasterCfg<TS>::P;
    using L = Layout<TS, P>;
    if (visits) {
        hipLaunchKernelGGL((k_raster_fwd<TS, P, true>), dim3(vt.total_tiles), dim3(GS_WAVE * L::WPT), 0, st,
                           vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], img, Tout, lastout, visits);
    } else if (order) {
        hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(1), 0, st, queue);
        hipLaunchKernelGGL((k_raster_fwd_persistent<TS, P>), dim3(persistent_blocks()), dim3(GS_WAVE), 0,
                           st, vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], order, queue, img, Tout,
                           lastout);
    } else {
        hipLaunchKernelGGL((k_raster_fwd<TS, P, false>), dim3(vt.total_tiles), dim3(GS_WAVE * L::WPT), 0, st,
                           vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], img, Tout, lastout, nullptr);
    }
    return hipGetLastError();
}

template <int TS, bool DA>
static hipError_t bwd_ts(const ViewTable& vt, const float* splats, const int* gids, const int2* ranges,
                         long long N, const float* bg, const int* order, int* queue, const float* Tfin,
                         const int* nlast, const float* dimg, const float* dalpha, float* grad2d,
                         hipStream_t st)
{
    constexpr int P = RasterCfg<TS>::P;
    using L = Layout<TS, P>;
    if (order) {
        hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(1), 0, st, queue);
        hipLaunchKernelGGL((k_raster_bwd_persistent<TS, P, DA>), dim3(persistent_blocks()), dim3(GS_WAVE),
                           0, st, vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], order, queue, Tfin,
                           nlast, dimg, dalpha, grad2d);
    } else {
        hipLaunchKernelGGL((k_raster_bwd<TS, P, DA>), dim3(vt.total_tiles), dim3(GS_WAVE * L::WPT), 0, st,
                           vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], Tfin, nlast, dimg, dalpha,
                           grad2d);
    }
    return hipGetLastError();
}

hipError_t launch_raster_fwd(int tile, const ViewTable& vt, const float* splats, const int* gids,
                             const int2* ranges, long long N, const float* bg, const int* order,
                             int* queue, float* img, float* Tout, int* lastout, int* visits,
                             hipStream_t st)
{
    if (vt.total_tiles == 0) return hipSuccess;
    switch (tile) {
    case 8: return fwd_ts<8>(vt, splats, gids, ranges, N, bg, order, queue, img, Tout, lastout, visits, st);
    case 16: return fwd_ts<16>(vt, splats, gids, ranges, N, bg, order, queue, img, Tout, lastout, visits, st);
    default: return fwd_ts<32>(vt, splats, gids, ranges, N, bg, order, queue, img, Tout, lastout, visits, st);
    }
}

hipError_t launch_raster_bwd(int tile, const ViewTable& vt, const float* splats, const int* gids,
                             const int2* ranges, long long N, const float* bg, const int* order,
                             int* queue, const float* Tfin, const int* nlast, const float* dimg,
                             const float* dalpha, float* grad2d, hipStream_t st)
{
    if (vt.total_tiles == 0) return hipSuccess;
    const bool da = dalpha != nullptr;
#define GS_BWD(TS)                                                                                   \
    return da ? bwd_ts<TS, true>(vt, splats, gids, ranges, N, bg, order, queue, Tfin, nlast, dimg,   \
                                 dalpha, grad2d, st)                                                 \
              : bwd_ts<TS, false>(vt, splats, gids, ranges, N, bg, order, queue, Tfin, nlast, dimg,  \
                                  dalpha, grad2d, st)
    switch (tile) {
    case 8: GS_BWD(8);
    case 16: GS_BWD(16);
    default: GS_BWD(32);
    }
#undef GS_BWD
}

}  // namespace gs
