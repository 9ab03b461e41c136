// SSIM + L1 image loss and its gradient (gfx950).
//
// Paper Section 4: each camera's rendered image is scored by a fused SSIM
// loss operator (SSIM of Wang et al. 2004, fused as in Mallick et al. 2024).
// Settings of 3D Gaussian Splatting: per channel, an 11x11 Gaussian window of
// standard deviation 1.5 applied as a zero-padded "same" correlation,
// C1 = 0.01^2, C2 = 0.03^2, and loss = (1 - lam) mean|x - y| +
// lam (1 - mean SSIM) over every element of every view.
//
// GPU organisation: one 256-thread workgroup per (32x54 output tile,
// channel), two kernels.
//   forward: the 42x64 input region (5-pixel halo) of x and y is staged in
//     LDS; the window is applied separably to the five moments x, y, x^2,
//     y^2, xy.  Each thread filters one row segment of 8 outputs (the
//     products of its 18 inputs formed once) and then one column segment of
//     7 outputs (its 17 filtered rows held in registers), so every output
//     costs about 110 multiply-adds, not the 11 x 16 of a per-output window.
//     Each pixel's SSIM and its partial derivatives with respect to
//     (mu_x, E[x^2], E[xy]) are written out.
//   backward: the three partial maps are staged with the same halo and
//     correlated with the (symmetric) window again, the same way:
//       dL/dx = w * dmu + 2 x (w * dExx) + y (w * dExy)
//               + (1 - lam) sign(x - y) / n;
//     its first workgroup also adds up the forward's partial losses.
// Staging issues all of a thread's loads before storing any, and the staged
// inputs and the filtered rows share one LDS array, so that enough
// workgroups stay resident to cover the memory latency.
// A tile's 64 staged rows by 4 row segments and its 32 columns by 8 column
// segments (7 rows each, the last 5) give every thread one task per pass.
#include <cmath>

#include "gs_device.h"

namespace gs {
namespace {

constexpr int TW = 32;              // output tile width
constexpr int TH = 54;              // output tile height
constexpr int SR = 5;               // window radius
constexpr int NT = 2 * SR + 1;      // taps
constexpr int RW = TW + 2 * SR;     // staged region width (42)
constexpr int RH = TH + 2 * SR;     // staged region height (64)
constexpr int XP = RW + 3;          // staged row pitch (45 floats: odd, so rows start in different banks)
constexpr int HP = TW + 1;          // filtered row pitch (33 floats)
constexpr int HSEG = 8;             // outputs per row segment
constexpr int VSEG = 7;             // outputs per column segment
constexpr int THREADS = 256;
static_assert(RH * (TW / HSEG) == THREADS, "one row segment per thread");
static_assert(TW * ((TH + VSEG - 1) / VSEG) == THREADS, "one column segment per thread");
constexpr float C1 = 0.0001f;       // 0.01^2
constexpr float C2 = 0.0009f;       // 0.03^2

struct Window {
    float w[NT];
};

// per-launch tiling of the views into TW x TH output tiles
struct SsimTiles {
    int n_views;
    int W[GS_MAX_VIEWS], H[GS_MAX_VIEWS], tx[GS_MAX_VIEWS];
    int off[GS_MAX_VIEWS + 1];             // prefix of tile counts
    long long base[GS_MAX_VIEWS];          // float offset of channel 0 of the view in the packed images
};

struct TileOf {
    int x0, y0, W, H;
    long long base;
};

__device__ __forceinline__ TileOf tile_of(const SsimTiles& st, int b)
{
    int v = 0;
    while (v + 1 < st.n_views && st.off[v + 1] <= b) v++;
    TileOf t;
    const int lt = b - st.off[v];
    const int ty = lt / st.tx[v];
    t.x0 = (lt - ty * st.tx[v]) * TW;
    t.y0 = ty * TH;
    t.W = st.W[v];
    t.H = st.H[v];
    t.base = st.base[v];
    return t;
}

// stages the RH x RW region of one plane around the tile (zero outside the
// image): all of a thread's loads are issued before any is stored, so that
// they are in flight together.  The loads are unconditional, from the
// position clamped into the image, and masked afterwards (a load guarded by
// the position test becomes a branch with a wait of its own).
constexpr int STAGE_PER_THREAD = (RH * RW + THREADS - 1) / THREADS;
__device__ __forceinline__ void stage(const float* __restrict__ p, const TileOf& T, float (*s)[XP])
{
    float val[STAGE_PER_THREAD];
#pragma unroll
    for (int u = 0; u < STAGE_PER_THREAD; u++) {
        const int i = threadIdx.x + u * THREADS;
        const int r = i / RW, q = i - r * RW;
        const int gy = T.y0 + r - SR, gx = T.x0 + q - SR;
        const bool in = i < RH * RW && gx >= 0 && gx < T.W && gy >= 0 && gy < T.H;
        const int cy = min(max(gy, 0), T.H - 1), cx = min(max(gx, 0), T.W - 1);
        const float x = p[(long long)cy * T.W + cx];
        val[u] = in ? x : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < STAGE_PER_THREAD; u++) {
        const int i = threadIdx.x + u * THREADS;
        if (i < RH * RW) s[i / RW][i % RW] = val[u];
    }
}

__global__ __launch_bounds__(THREADS) void k_ssim_fwd(SsimTiles st, Window win, const float* __restrict__ img,
                                                      const float* __restrict__ tgt, float lam, float inv_count,
                                                      float* __restrict__ dmu, float* __restrict__ dexx,
                                                      float* __restrict__ dexy, double* __restrict__ part)
{
    // the staged inputs and, once every thread holds what it needs of them,
    // the filtered rows share one LDS array (more workgroups per CU)
    __shared__ float lds[5 * RH * HP];
    __shared__ double s_red[THREADS / GS_WAVE];
    float (*sx)[XP] = reinterpret_cast<float (*)[XP]>(lds);
    float (*sy)[XP] = reinterpret_cast<float (*)[XP]>(lds + RH * XP);
    float (*hm)[RH][HP] = reinterpret_cast<float (*)[RH][HP]>(lds);
    static_assert(2 * RH * XP <= 5 * RH * HP, "staged inputs fit the shared array");
    const int c = blockIdx.y, t = threadIdx.x;
    const TileOf T = tile_of(st, blockIdx.x);
    const long long plane = (long long)T.W * T.H;
    const long long cb = T.base + c * plane;
    stage(img + cb, T, sx);
    stage(tgt + cb, T, sy);
    __syncthreads();

    // row task: staged row r, outputs c0 .. c0 + HSEG - 1 (taps at staged
    // columns c0 + j .. c0 + j + 10); a wave takes 64 consecutive rows
    const int r = t % RH, c0 = (t / RH) * HSEG;
    // column task: column q, output rows j0 .. j0 + VSEG - 1
    const int q = t % TW, j0 = (t / TW) * VSEG;
    const int nj = min(VSEG, TH - j0);
    float x[HSEG + NT - 1], y[HSEG + NT - 1], cx[VSEG], cy[VSEG];
#pragma unroll
    for (int i = 0; i < HSEG + NT - 1; i++) {
        x[i] = sx[r][c0 + i];
        y[i] = sy[r][c0 + i];
    }
#pragma unroll
    for (int j = 0; j < VSEG; j++) {
        const int rr = min(j0 + j + SR, RH - 1);
        cx[j] = sx[rr][q + SR];
        cy[j] = sy[rr][q + SR];
    }
    __syncthreads();
    {
        float xx[HSEG + NT - 1], yy[HSEG + NT - 1], xy[HSEG + NT - 1];
#pragma unroll
        for (int i = 0; i < HSEG + NT - 1; i++) {
            xx[i] = x[i] * x[i];
            yy[i] = y[i] * y[i];
            xy[i] = x[i] * y[i];
        }
#pragma unroll
        for (int j = 0; j < HSEG; j++) {
            float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
            for (int k = 0; k < NT; k++) {
                const float w = win.w[k];
                a = __builtin_fmaf(w, x[j + k], a);
                b = __builtin_fmaf(w, y[j + k], b);
                aa = __builtin_fmaf(w, xx[j + k], aa);
                bb = __builtin_fmaf(w, yy[j + k], bb);
                ab = __builtin_fmaf(w, xy[j + k], ab);
            }
            hm[0][r][c0 + j] = a;
            hm[1][r][c0 + j] = b;
            hm[2][r][c0 + j] = aa;
            hm[3][r][c0 + j] = bb;
            hm[4][r][c0 + j] = ab;
        }
    }
    __syncthreads();

    float v[5][VSEG + NT - 1];
#pragma unroll
    for (int m = 0; m < 5; m++)
#pragma unroll
        for (int i = 0; i < VSEG + NT - 1; i++) v[m][i] = hm[m][min(j0 + i, RH - 1)][q];
    float contrib = 0.0f;
    const int gx = T.x0 + q;
    const float gS = -lam * inv_count;
#pragma unroll
    for (int j = 0; j < VSEG; j++) {
        float mom[5];
#pragma unroll
        for (int m = 0; m < 5; m++) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < NT; k++) s = __builtin_fmaf(win.w[k], v[m][j + k], s);
            mom[m] = s;
        }
        const int gy = T.y0 + j0 + j;
        if (j < nj && gx < T.W && gy < T.H) {
            const float mx = mom[0], my = mom[1], exx = mom[2], eyy = mom[3], exy = mom[4];
            const float A = 2.0f * mx * my + C1;
            const float B = 2.0f * (exy - mx * my) + C2;
            const float C = mx * mx + my * my + C1;
            const float D = (exx - mx * mx) + (eyy - my * my) + C2;
            // hardware reciprocals (about 1 ulp) instead of four divisions
            const float iC = __builtin_amdgcn_rcpf(C), iD = __builtin_amdgcn_rcpf(D);
            const float iCD = iC * iD;
            const float S = A * B * iCD;
            const long long o = cb + (long long)gy * T.W + gx;
            dmu[o] = gS * ((2.0f * my * (B - A)) * iCD - S * (2.0f * mx * (iC - iD)));
            dexx[o] = gS * (-S * iD);
            dexy[o] = gS * (2.0f * A * iCD);
            contrib += (1.0f - lam) * fabsf(cx[j] - cy[j]) + lam * (1.0f - S);
        }
    }
    const float ws = wave_sum(contrib);
    if (__lane_id() == 0) s_red[t / GS_WAVE] = (double)ws;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < THREADS / GS_WAVE; i++) s += s_red[i];
        part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// the loss: the forward's per-(tile, channel) partial sums added in a fixed
// order (eight running sums per thread, then a tree), by one workgroup
__device__ __forceinline__ void final_sum(const double* __restrict__ part, long long nb, double inv_n,
                                          float* __restrict__ loss, double* s)
{
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long i0 = threadIdx.x; i0 < nb; i0 += 8 * THREADS)
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const long long i = i0 + (long long)THREADS * u;
            const double x = part[i < nb ? i : nb - 1];
            acc[u] += i < nb ? x : 0.0;
        }
    s[threadIdx.x] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    for (int o = THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(s[0] * inv_n);
}

// the forward has finished when this kernel starts (same stream), so its
// first workgroup also adds up the loss
__global__ __launch_bounds__(THREADS) void k_ssim_bwd(SsimTiles st, Window win, const float* __restrict__ img,
                                                      const float* __restrict__ tgt, float lam, float inv_count,
                                                      const float* __restrict__ dmu, const float* __restrict__ dexx,
                                                      const float* __restrict__ dexy, float* __restrict__ dimg,
                                                      const double* __restrict__ part, double inv_n,
                                                      float* __restrict__ loss)
{
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        __shared__ double s_sum[THREADS];
        final_sum(part, 3ll * gridDim.x, inv_n, loss, s_sum);
    }
    // staged partial maps, then (after every thread has read its row) the filtered rows
    __shared__ float lds[3 * RH * XP];
    float (*sp)[RH][XP] = reinterpret_cast<float (*)[RH][XP]>(lds);
    float (*hb)[RH][HP] = reinterpret_cast<float (*)[RH][HP]>(lds);
    static_assert(3 * RH * HP <= 3 * RH * XP, "filtered rows fit the shared array");
    const int c = blockIdx.y, t = threadIdx.x;
    const TileOf T = tile_of(st, blockIdx.x);
    const long long plane = (long long)T.W * T.H;
    const long long cb = T.base + c * plane;
    stage(dmu + cb, T, sp[0]);
    stage(dexx + cb, T, sp[1]);
    stage(dexy + cb, T, sp[2]);

    const int r = t % RH, c0 = (t / RH) * HSEG;
    const int q = t % TW, j0 = (t / TW) * VSEG;
    const int nj = min(VSEG, TH - j0);
    const int gx = T.x0 + q;
    // this thread's output pixels of x and y, loaded while the maps are staged
    float px[VSEG], py[VSEG];
#pragma unroll
    for (int j = 0; j < VSEG; j++) {
        const int gy = T.y0 + j0 + j;
        const bool in = j < nj && gx < T.W && gy < T.H;
        const long long o = cb + (long long)(in ? gy : 0) * T.W + (in ? gx : 0);
        const float a = img[o], b = tgt[o];
        px[j] = in ? a : 0.0f;
        py[j] = in ? b : 0.0f;
    }
    __syncthreads();
    float p[3][HSEG + NT - 1];
#pragma unroll
    for (int m = 0; m < 3; m++)
#pragma unroll
        for (int i = 0; i < HSEG + NT - 1; i++) p[m][i] = sp[m][r][c0 + i];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < HSEG; j++)
#pragma unroll
        for (int m = 0; m < 3; m++) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < NT; k++) s = __builtin_fmaf(win.w[k], p[m][j + k], s);
            hb[m][r][c0 + j] = s;
        }
    __syncthreads();

    float v[3][VSEG + NT - 1];
#pragma unroll
    for (int m = 0; m < 3; m++)
#pragma unroll
        for (int i = 0; i < VSEG + NT - 1; i++) v[m][i] = hb[m][min(j0 + i, RH - 1)][q];
#pragma unroll
    for (int j = 0; j < VSEG; j++) {
        float g[3];
#pragma unroll
        for (int m = 0; m < 3; m++) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < NT; k++) s = __builtin_fmaf(win.w[k], v[m][j + k], s);
            g[m] = s;
        }
        const int gy = T.y0 + j0 + j;
        if (j < nj && gx < T.W && gy < T.H) {
            const long long o = cb + (long long)gy * T.W + gx;
            const float x = px[j], y = py[j];
            const float d = x - y;
            const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            dimg[o] = g[0] + 2.0f * x * g[1] + y * g[2] + (1.0f - lam) * inv_count * sgn;
        }
    }
}

Window make_window()
{
    Window w;
    double s = 0.0, v[NT];
    for (int k = -SR; k <= SR; k++) {
        v[k + SR] = std::exp(-(double)(k * k) / (2.0 * 1.5 * 1.5));
        s += v[k + SR];
    }
    for (int k = 0; k < NT; k++) w.w[k] = (float)(v[k] / s);
    return w;
}

SsimTiles make_tiles(const ViewTable& vt)
{
    SsimTiles st;
    st.n_views = vt.n_views;
    st.off[0] = 0;
    for (int v = 0; v < vt.n_views; v++) {
        st.W[v] = vt.W[v];
        st.H[v] = vt.H[v];
        st.tx[v] = (vt.W[v] + TW - 1) / TW;
        st.off[v + 1] = st.off[v] + st.tx[v] * ((vt.H[v] + TH - 1) / TH);
        st.base[v] = 3 * vt.pix_off[v];
    }
    return st;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// the three partial-derivative maps and one partial sum per (tile, channel);
// sized with the 16-pixel tiles of the view table, which outnumber the
// 32x54 tiles of the kernels
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
    const SsimTiles tiles = make_tiles(vt);
    const int nt = tiles.off[vt.n_views];
    const float inv_count = (float)(1.0 / (double)n);
    const dim3 grid((unsigned)nt, 3);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(THREADS), 0, st, tiles, w, img, tgt, lam, inv_count, dmu, dexx, dexy,
                       part);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(THREADS), 0, st, tiles, w, img, tgt, lam, inv_count, dmu, dexx, dexy,
                       dimg, part, 1.0 / (double)n, loss);
    return hipGetLastError();
}

}  // namespace gs
