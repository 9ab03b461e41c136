// SSIM + L1 image loss and its gradient (gfx950).
//
// Paper Section 4: each camera's rendered image is scored by a fused SSIM
// loss operator (SSIM of Wang et al. 2004, fused as in Mallick et al. 2024).
// Settings of 3D Gaussian Splatting: per channel, an 11x11 Gaussian window of
// standard deviation 1.5 applied as a zero-padded "same" correlation,
// C1 = 0.01^2, C2 = 0.03^2, and loss = (1 - lam) mean|x - y| +
// lam (1 - mean SSIM) over every element of every view.
//
// GPU organisation: one 256-thread workgroup per (16x16 output tile,
// channel).  The 26x26 input tile (5-pixel halo) is staged in LDS once, the
// window is applied separably (rows, then columns) to the five moments x, y,
// x^2, y^2, xy, and each pixel's SSIM and its partial derivatives with
// respect to (mu_x, E[x^2], E[xy]) are formed in registers.  The backward
// stages those three partial maps with the same halo and correlates them
// with the (symmetric) window again:
//   dL/dx = w * dmu + 2 x (w * dExx) + y (w * dExy) + (1 - lam) sign(x - y) / n.
#include <cmath>

#include "gs_device.h"

namespace gs {
namespace {

constexpr int ST = 16;            // output tile edge
constexpr int SR = 5;             // window radius
constexpr int SW = ST + 2 * SR;   // staged tile edge (26)
constexpr float C1 = 0.0001f;     // 0.01^2
constexpr float C2 = 0.0009f;     // 0.03^2

struct Window {
    float w[2 * SR + 1];
};

struct TileOf {
    int v, x0, y0, W, H;
    long long base;   // float offset of channel 0 of this view in the packed images
};

__device__ __forceinline__ TileOf tile_of(const ViewTable& vt, int gt)
{
    TileOf t;
    t.v = view_of_tile(vt, gt);
    const int lt = gt - vt.tile_off[t.v];
    const int TX = vt.tiles_x[t.v];
    t.y0 = (lt / TX) * ST;
    t.x0 = (lt - (lt / TX) * TX) * ST;
    t.W = vt.W[t.v];
    t.H = vt.H[t.v];
    t.base = 3 * vt.pix_off[t.v];
    return t;
}

__global__ __launch_bounds__(256) void k_ssim_fwd(ViewTable vt, Window win, const float* __restrict__ img,
                                                  const float* __restrict__ tgt, float lam, float inv_count,
                                                  float* __restrict__ dmu, float* __restrict__ dexx,
                                                  float* __restrict__ dexy, double* __restrict__ part)
{
    __shared__ float sx[SW][SW + 1], sy[SW][SW + 1];
    __shared__ float h[5][SW][ST + 1];
    __shared__ double s_red[4];
    const int c = blockIdx.y, t = threadIdx.x;
    const TileOf T = tile_of(vt, blockIdx.x);
    const long long plane = (long long)T.W * T.H;
    const float* X = img + T.base + c * plane;
    const float* Y = tgt + T.base + c * plane;
    for (int i = t; i < SW * SW; i += 256) {
        const int r = i / SW, q = i - r * SW;
        const int gy = T.y0 + r - SR, gx = T.x0 + q - SR;
        const bool in = gx >= 0 && gx < T.W && gy >= 0 && gy < T.H;
        sx[r][q] = in ? X[(long long)gy * T.W + gx] : 0.0f;
        sy[r][q] = in ? Y[(long long)gy * T.W + gx] : 0.0f;
    }
    __syncthreads();
    for (int i = t; i < SW * ST; i += 256) {
        const int r = i / ST, q = i - r * ST;
        float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
        for (int k = 0; k <= 2 * SR; k++) {
            const float x = sx[r][q + k], y = sy[r][q + k], w = win.w[k];
            a += w * x;
            b += w * y;
            aa += w * x * x;
            bb += w * y * y;
            ab += w * x * y;
        }
        h[0][r][q] = a; h[1][r][q] = b; h[2][r][q] = aa; h[3][r][q] = bb; h[4][r][q] = ab;
    }
    __syncthreads();
    const int ty = t / ST, tx = t - (t / ST) * ST;
    float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * SR; k++) {
        const float w = win.w[k];
        mx += w * h[0][ty + k][tx];
        my += w * h[1][ty + k][tx];
        exx += w * h[2][ty + k][tx];
        eyy += w * h[3][ty + k][tx];
        exy += w * h[4][ty + k][tx];
    }
    const int gx = T.x0 + tx, gy = T.y0 + ty;
    const bool in = gx < T.W && gy < T.H;
    float contrib = 0.0f;
    if (in) {
        const float A = 2.0f * mx * my + C1;
        const float B = 2.0f * (exy - mx * my) + C2;
        const float C = mx * mx + my * my + C1;
        const float D = (exx - mx * mx) + (eyy - my * my) + C2;
        const float iCD = 1.0f / (C * D);
        const float S = A * B * iCD;
        const float gS = -lam * inv_count;
        const long long o = T.base + c * plane + (long long)gy * T.W + gx;
        dmu[o] = gS * ((2.0f * my * (B - A)) * iCD - S * (2.0f * mx / C - 2.0f * mx / D));
        dexx[o] = gS * (-S / D);
        dexy[o] = gS * (2.0f * A * iCD);
        const float x = sx[ty + SR][tx + SR], y = sy[ty + SR][tx + SR];
        contrib = (1.0f - lam) * fabsf(x - y) + lam * (1.0f - S);
    }
    const float ws = wave_sum(contrib);
    if (__lane_id() == 0) s_red[t / GS_WAVE] = (double)ws;
    __syncthreads();
    if (t == 0) part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

__global__ __launch_bounds__(256) void k_ssim_bwd(ViewTable vt, Window win, const float* __restrict__ img,
                                                  const float* __restrict__ tgt, float lam, float inv_count,
                                                  const float* __restrict__ dmu, const float* __restrict__ dexx,
                                                  const float* __restrict__ dexy, float* __restrict__ dimg)
{
    __shared__ float sp[3][SW][SW + 1];
    __shared__ float h[3][SW][ST + 1];
    const int c = blockIdx.y, t = threadIdx.x;
    const TileOf T = tile_of(vt, blockIdx.x);
    const long long plane = (long long)T.W * T.H;
    const long long cb = T.base + c * plane;
    for (int i = t; i < SW * SW; i += 256) {
        const int r = i / SW, q = i - r * SW;
        const int gy = T.y0 + r - SR, gx = T.x0 + q - SR;
        const bool in = gx >= 0 && gx < T.W && gy >= 0 && gy < T.H;
        const long long o = cb + (long long)gy * T.W + gx;
        sp[0][r][q] = in ? dmu[o] : 0.0f;
        sp[1][r][q] = in ? dexx[o] : 0.0f;
        sp[2][r][q] = in ? dexy[o] : 0.0f;
    }
    __syncthreads();
    for (int i = t; i < SW * ST; i += 256) {
        const int r = i / ST, q = i - r * ST;
        float a = 0.f, b = 0.f, e = 0.f;
#pragma unroll
        for (int k = 0; k <= 2 * SR; k++) {
            const float w = win.w[k];
            a += w * sp[0][r][q + k];
            b += w * sp[1][r][q + k];
            e += w * sp[2][r][q + k];
        }
        h[0][r][q] = a; h[1][r][q] = b; h[2][r][q] = e;
    }
    __syncthreads();
    const int ty = t / ST, tx = t - (t / ST) * ST;
    const int gx = T.x0 + tx, gy = T.y0 + ty;
    if (gx >= T.W || gy >= T.H) return;
    float a = 0.f, b = 0.f, e = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * SR; k++) {
        const float w = win.w[k];
        a += w * h[0][ty + k][tx];
        b += w * h[1][ty + k][tx];
        e += w * h[2][ty + k][tx];
    }
    const long long o = cb + (long long)gy * T.W + gx;
    const float x = img[o], y = tgt[o];
    const float d = x - y;
    const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    dimg[o] = a + 2.0f * x * b + y * e + (1.0f - lam) * inv_count * sgn;
}

__global__ __launch_bounds__(256) void k_ssim_final(const double* __restrict__ part, long long nb, double inv_n,
                                                    float* __restrict__ loss)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < nb; i += 256) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(s[0] * inv_n);
}

Window make_window()
{
    Window w;
    double s = 0.0, v[2 * SR + 1];
    for (int k = -SR; k <= SR; k++) {
        v[k + SR] = std::exp(-(double)(k * k) / (2.0 * 1.5 * 1.5));
        s += v[k + SR];
    }
    for (int k = 0; k <= 2 * SR; k++) w.w[k] = (float)(v[k] / s);
    return w;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t ssim_workspace_size(const ViewTable& vt)
{
    const size_t n = 3 * (size_t)vt.pix_off[vt.n_views];
    return 3 * align256(4 * n) + align256(8ull * 3 * (size_t)vt.total_tiles);
}

hipError_t launch_ssim_l1(const ViewTable& vt, const float* img, const float* tgt, float lam, float* loss,
                          float* dimg, void* workspace, hipStream_t st)
{
    const size_t n = 3 * (size_t)vt.pix_off[vt.n_views];
    char* b = (char*)workspace;
    float* dmu = (float*)b;
    float* dexx = (float*)(b + align256(4 * n));
    float* dexy = (float*)(b + 2 * align256(4 * n));
    double* part = (double*)(b + 3 * align256(4 * n));
    const Window w = make_window();
    const float inv_count = (float)(1.0 / (double)n);
    const dim3 grid((unsigned)vt.total_tiles, 3);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, st, vt, w, img, tgt, lam, inv_count, dmu, dexx, dexy, part);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, st, vt, w, img, tgt, lam, inv_count, dmu, dexx, dexy, dimg);
    hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(256), 0, st, part, 3ll * vt.total_tiles, 1.0 / (double)n, loss);
    return hipGetLastError();
}

}  // namespace gs
