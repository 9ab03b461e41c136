// Device-side helpers shared by the gfx950 kernels of the splatting path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs.h"

#define GS_WAVE 64

namespace gs {

// Per-launch description of the views, passed by value as a kernel argument.
struct ViewTable {
    int n_views;
    int total_tiles;
    int W[GS_MAX_VIEWS];
    int H[GS_MAX_VIEWS];
    int tiles_x[GS_MAX_VIEWS];
    int tile_off[GS_MAX_VIEWS + 1];   // prefix of TX*TY
    long long pix_off[GS_MAX_VIEWS + 1];  // prefix of W*H
};

// Non-temporal (streaming) loads and stores, for whole coalesced lines that
// no later kernel of the step reads from cache.
template <class T>
__device__ __forceinline__ void nt_store(T v, T* p)
{
    __builtin_nontemporal_store(v, p);
}

template <class T>
__device__ __forceinline__ T nt_load(const T* p)
{
    return __builtin_nontemporal_load(p);
}

// Constants of the method (3D Gaussian Splatting compositing), float32.
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kClip = 1.3f;
// log2(e) / 2: M M^T = kC0 * conic
constexpr float kC0 = 0.72134752044448170368f;
constexpr float kLn2 = 0.69314718055994530942f;

__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int t)
{
    int v = 0;
    // views are few (<= 64); binary search over the tile prefix
    int lo = 0, hi = vt.n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (vt.tile_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    v = lo;
    return v;
}

// Tile rectangle of a splat, float32 arithmetic without contraction so that
// the projection (tiles_touched) and the binning (emission) agree bit for bit.
__device__ __forceinline__ void tile_rect(float u, float v, int rx, int ry, int tile, int W, int H,
                                          int& x0, int& y0, int& x1, int& y1)
{
#pragma clang fp contract(off)
    const int TX = (W + tile - 1) / tile, TY = (H + tile - 1) / tile;
    const float ts = (float)tile;
    float fx0 = floorf((u - (float)rx) / ts);
    float fx1 = floorf((u + (float)rx) / ts) + 1.0f;
    float fy0 = floorf((v - (float)ry) / ts);
    float fy1 = floorf((v + (float)ry) / ts) + 1.0f;
    fx0 = fminf(fmaxf(fx0, 0.0f), (float)TX);
    fx1 = fminf(fmaxf(fx1, 0.0f), (float)TX);
    fy0 = fminf(fmaxf(fy0, 0.0f), (float)TY);
    fy1 = fminf(fmaxf(fy1, 0.0f), (float)TY);
    x0 = (int)fx0; x1 = (int)fx1; y0 = (int)fy0; y1 = (int)fy1;
}

// Splat falloff in the record's factor form.  Both rasterisers call this same
// function so that their skip decisions agree: w = M^T d, q' = |w|^2,
// alpha_raw = 2^(log2 sigma - q').  Explicit fma calls fix the rounding.
struct Falloff {
    float w0, w1, araw;
};

__device__ __forceinline__ Falloff falloff(float dx, float dy, float m00, float m10, float m11,
                                           float ls)
{
#pragma clang fp contract(off)
    Falloff f;
    f.w1 = m11 * dy;
    f.w0 = __builtin_fmaf(m00, dx, m10 * dy);
    float e = __builtin_fmaf(-f.w1, f.w1, ls);
    e = __builtin_fmaf(-f.w0, f.w0, e);
    f.araw = __builtin_amdgcn_exp2f(e);
    return f;
}

// Sum of x over the 64 lanes of the wave, returned uniformly (gfx9 DPP).
__device__ __forceinline__ float wave_sum(float x)
{
    // xor 1, xor 2 within quads
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
    // row half mirror (8 lanes), row mirror (16 lanes)
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false));
    // row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xA, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xC, 0xF, false));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// One butterfly step of a reduce-scatter: lanes with `hi` keep the odd member
// of the pair and send the even one, their DPP partner does the opposite, so
// each lane ends with the pair-sum of the member it kept.
template <int CTRL>
__device__ __forceinline__ float bfly(float even, float odd, bool hi)
{
    const float keep = hi ? odd : even;
    const float send = hi ? even : odd;
    return keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xF, 0xF, false));
}

// bfly(x, 0, hi): the lane without `hi` gets the pair-sum of x, the other 0
template <int CTRL>
__device__ __forceinline__ float bfly0(float x, bool hi)
{
    const float s = x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
    return hi ? 0.0f : s;
}

// Wave-wide sums of nine values, scattered: afterwards lane l (l < 16) holds
// the total of value j(l) = b3 + 2 b2 + 4 b0 + 8 b1 (b_k = bit k of l), a
// permutation of 0..15 in which 9..15 carry zeros.  The four in-row steps
// pair lanes across bit 3 (row mirror, bank-masked adds), bit 2 (half-row
// mirror, bank-masked adds), bit 0 and bit 1 (quad permutes, selects); two
// shuffles then add the four rows.  About 24 vector operations and two
// shuffles instead of nine full reductions.
// the value index j(l) whose total lane l holds after wave_sum9_scatter
__device__ __forceinline__ int wave_sum9_slot(int l)
{
    return ((l & 8) ? 1 : 0) | ((l & 4) ? 2 : 0) | ((l & 1) ? 4 : 0) | ((l & 2) ? 8 : 0);
}

// Butterfly steps across lane bit 3 (row mirror) and bit 2 (half-row mirror)
// written as two bank-masked DPP adds per pair: a DPP bank is lane bits 2-3,
// so the lanes that keep the even member are written by one add and the
// others by the second, and no selects are needed (two instructions per pair
// instead of three).  The compiler has no form for a bank-masked add that
// keeps the other lanes, hence the asm; it reads and writes registers only.
// Each DPP read waits two cycles after the last vector write of its source
// (the gfx9 DPP hazard; s_nop 1), since the compiler does not see inside.
#define GS_DPP_ADD_FIRST(t, x, CTRL, BANK)                                                          \
    asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 " CTRL " row_mask:0xf bank_mask:" BANK " bound_ctrl:1" \
        : "=&v"(t)                                                                               \
        : "v"(x))
#define GS_DPP_ADD_REST(t, x, CTRL, BANK)                                                           \
    asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 " CTRL " row_mask:0xf bank_mask:" BANK " bound_ctrl:1" \
        : "+v"(t)                                                                                \
        : "v"(x))

// t = x + x[partner] on the lanes with the bit clear, y + y[partner] on the others
__device__ __forceinline__ float bfly_mirror(float x, float y)
{
    float t;
    GS_DPP_ADD_FIRST(t, x, "row_mirror", "0x3");
    GS_DPP_ADD_REST(t, y, "row_mirror", "0xc");
    return t;
}

__device__ __forceinline__ float bfly_half_mirror(float x, float y)
{
    float t;
    GS_DPP_ADD_FIRST(t, x, "row_half_mirror", "0x5");
    GS_DPP_ADD_REST(t, y, "row_half_mirror", "0xa");
    return t;
}

__device__ __forceinline__ float wave_sum9_scatter(const float* a, int& j)
{
    const int l = __lane_id();
    const bool h1 = l & 8, h2 = l & 4, h3 = l & 1, h4 = l & 2;
    const float b0 = bfly_mirror(a[0], a[1]), b1 = bfly_mirror(a[2], a[3]);
    const float b2 = bfly_mirror(a[4], a[5]), b3 = bfly_mirror(a[6], a[7]);
    const float b4 = bfly0<0x140>(a[8], h1);
    const float c0 = bfly_half_mirror(b0, b1), c1 = bfly_half_mirror(b2, b3);
    const float c2 = bfly0<0x141>(b4, h2);
    const float d0 = bfly<0xB1>(c0, c1, h3), d1 = bfly0<0xB1>(c2, h3);
    float e = bfly<0x4E>(d0, d1, h4);
    e += __shfl_xor(e, 16);
    e += __shfl_xor(e, 32);
    j = wave_sum9_slot(l);
    return e;
}

// Adam (Kingma and Ba 2015) with bias correction, one element; shared by the
// stand-alone update and the one fused into the projection backward, so the
// two give the same bits.  Every multiply-add is written out as an fma, so no
// file's contraction setting changes the result.
struct AdamCoef {
    float step_scale;   // 1 / (1 - b1^t), multiplied by the tensor's rate
    float rbc2;         // 1 / sqrt(1 - b2^t)
};

// t = step + 1.  1 - b^t = -expm1(t log1p(b - 1)): b - 1 is exact for b in
// [0.5, 1], and the form keeps full relative precision for b near 1.
__device__ __forceinline__ AdamCoef adam_coef(int step, float b1, float b2)
{
    const float t = (float)(step + 1);
    AdamCoef c;
    c.step_scale = 1.0f / -expm1f(t * log1pf(b1 - 1.0f));
    c.rbc2 = 1.0f / sqrtf(-expm1f(t * log1pf(b2 - 1.0f)));
    return c;
}

// m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
// p <- p - lr / (1 - b1^t) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
// The square root and the reciprocal are the hardware's (v_sqrt_f32,
// v_rcp_f32: about 1 ulp each) instead of the correctly rounded expansions,
// which cost some 25 more instructions per element; the update's relative
// error stays a few ulp.
__device__ __forceinline__ void adam_elem(float& p, float g, float& m, float& v, float b1, float b2, float step,
                                          float rbc2, float eps)
{
    m = __builtin_fmaf(b1, m, (1.0f - b1) * g);
    v = __builtin_fmaf(b2, v, ((1.0f - b2) * g) * g);
    const float den = __builtin_fmaf(__builtin_amdgcn_sqrtf(v), rbc2, eps);
    p = __builtin_fmaf(-(step * m), __builtin_amdgcn_rcpf(den), p);
}

// Maximum of x over the 64 lanes of the wave, returned uniformly (DPP steps
// as in wave_sum; a lane a step does not write keeps its own value)
__device__ __forceinline__ int wave_max_i(int x)
{
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x141, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x140, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x142, 0xA, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

}  // namespace gs
