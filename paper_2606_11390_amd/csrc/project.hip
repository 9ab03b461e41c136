// Projection + spherical-harmonic colour, forward and backward (gfx950).
//
// Paper Section 4: the SH and projection operators are partitioned per
// Gaussian and emit colours and projected quantities for every camera of the
// batch; their backward is partitioned the same way.  The formulas are those
// of 3D Gaussian Splatting (EWA splatting of a 3-D Gaussian through the local
// affine approximation of the pinhole projection).
//
// GPU organisation: one thread owns one Gaussian and loops over the views, so
// each parameter is read from HBM once per step whatever the number of views,
// and the backward sums a Gaussian's views in registers without atomics.
// Parameters are planar [C][N] (coalesced 256-byte wave reads per component);
// the splat record is written with three 16-byte stores per (view, Gaussian).
//
// Numerics: the 2-D covariance is formed as Sigma2 = F F^T + eps I with the
// 2x3 factor F = J W R S, so det Sigma2 = |F0 x F1|^2 + eps (|F0|^2 + |F1|^2)
// + eps^2 (Lagrange identity) carries no cancellation, and the record stores
// the Cholesky factor of the conic computed from it:
//   m00 = sqrt(c0 c / D), m10 = -b sqrt(c0 / (c D)), m11 = sqrt(c0 / c)
// for Sigma2 = [[a, b], [b, c]], D = det Sigma2, c0 = log2(e)/2.
#include <type_traits>

#include "gs_device.h"

namespace gs {
namespace {

// Real spherical harmonics, orthonormal with the Condon-Shortley phase,
// index l*l + l + m, evaluated at a unit direction.
constexpr float SH_C0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float SH_C1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
constexpr float SH_C2A = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float SH_C2B = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float SH_C2C = 0.54627421529603959f;  // sqrt(15 / pi) / 4
constexpr float SH_C3A = 0.59004358992664352f;  // sqrt(35 / (2 pi)) / 4
constexpr float SH_C3B = 2.8906114426405538f;   // sqrt(105 / pi) / 2
constexpr float SH_C3C = 0.45704579946446572f;  // sqrt(21 / (2 pi)) / 4
constexpr float SH_C3D = 0.37317633259011540f;  // sqrt(7 / pi) / 4
constexpr float SH_C3E = 1.4453057213202769f;   // sqrt(105 / pi) / 4

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y)
{
    Y[0] = SH_C0;
    if (DEG >= 1) {
        Y[1] = -SH_C1 * y;
        Y[2] = SH_C1 * z;
        Y[3] = -SH_C1 * x;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = SH_C2A * x * y;
        Y[5] = -SH_C2A * y * z;
        Y[6] = SH_C2B * (2.0f * zz - xx - yy);
        Y[7] = -SH_C2A * x * z;
        Y[8] = SH_C2C * (xx - yy);
        if (DEG >= 3) {
            Y[9] = -SH_C3A * y * (3.0f * xx - yy);
            Y[10] = SH_C3B * x * y * z;
            Y[11] = -SH_C3C * y * (4.0f * zz - xx - yy);
            Y[12] = SH_C3D * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -SH_C3C * x * (4.0f * zz - xx - yy);
            Y[14] = SH_C3E * z * (xx - yy);
            Y[15] = -SH_C3A * x * (xx - 3.0f * yy);
        }
    }
}

// sum_j s_j grad Y_j (partials of the polynomial forms above)
template <int DEG>
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, const float* s, float& gx,
                                            float& gy, float& gz)
{
    gx = gy = gz = 0.0f;
    if (DEG >= 1) {
        gy -= SH_C1 * s[1];
        gz += SH_C1 * s[2];
        gx -= SH_C1 * s[3];
    }
    if (DEG >= 2) {
        gx += SH_C2A * y * s[4];
        gy += SH_C2A * x * s[4];
        gy -= SH_C2A * z * s[5];
        gz -= SH_C2A * y * s[5];
        gx -= 2.0f * SH_C2B * x * s[6];
        gy -= 2.0f * SH_C2B * y * s[6];
        gz += 4.0f * SH_C2B * z * s[6];
        gx -= SH_C2A * z * s[7];
        gz -= SH_C2A * x * s[7];
        gx += 2.0f * SH_C2C * x * s[8];
        gy -= 2.0f * SH_C2C * y * s[8];
        if (DEG >= 3) {
            const float xx = x * x, yy = y * y, zz = z * z;
            gx -= 6.0f * SH_C3A * x * y * s[9];
            gy -= 3.0f * SH_C3A * (xx - yy) * s[9];
            gx += SH_C3B * y * z * s[10];
            gy += SH_C3B * x * z * s[10];
            gz += SH_C3B * x * y * s[10];
            gx += 2.0f * SH_C3C * x * y * s[11];
            gy -= SH_C3C * (4.0f * zz - xx - 3.0f * yy) * s[11];
            gz -= 8.0f * SH_C3C * y * z * s[11];
            gx -= 6.0f * SH_C3D * x * z * s[12];
            gy -= 6.0f * SH_C3D * y * z * s[12];
            gz += SH_C3D * (6.0f * zz - 3.0f * xx - 3.0f * yy) * s[12];
            gx -= SH_C3C * (4.0f * zz - 3.0f * xx - yy) * s[13];
            gy += 2.0f * SH_C3C * x * y * s[13];
            gz -= 8.0f * SH_C3C * x * z * s[13];
            gx += 2.0f * SH_C3E * x * z * s[14];
            gy -= 2.0f * SH_C3E * y * z * s[14];
            gz += SH_C3E * (xx - yy) * s[14];
            gx -= 3.0f * SH_C3A * (xx - yy) * s[15];
            gy += 6.0f * SH_C3A * x * y * s[15];
        }
    }
}

// rotation matrix (row-major) of a unit quaternion (w, x, y, z)
__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float* R)
{
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// [lo, hi] pixel indices whose centres (i + 0.5) may lie within e of c,
// widened by one pixel, clamped to int16, packed lo | hi << 16
__device__ __forceinline__ int pack_range(float c, float e)
{
    const float lo = fminf(fmaxf(floorf(c - e - 0.5f) - 1.0f, -32768.0f), 32767.0f);
    const float hi = fminf(fmaxf(ceilf(c + e - 0.5f) + 1.0f, -32768.0f), 32767.0f);
    return ((int)lo & 0xFFFF) | ((int)hi << 16);
}

struct Camera {
    float r[9];   // world-to-camera rotation, row-major
    float t[3];
    float fx, fy, cx, cy;
    float limx, limy;   // clamp of x/z, y/z in the Jacobian
    int W, H;
};

__device__ __forceinline__ Camera load_camera(const float* __restrict__ viewmats,
                                              const float* __restrict__ intr, const ViewTable& vt,
                                              int v)
{
    Camera c;
    const float* m = viewmats + v * 12;
    c.r[0] = m[0]; c.r[1] = m[1]; c.r[2] = m[2]; c.t[0] = m[3];
    c.r[3] = m[4]; c.r[4] = m[5]; c.r[5] = m[6]; c.t[1] = m[7];
    c.r[6] = m[8]; c.r[7] = m[9]; c.r[8] = m[10]; c.t[2] = m[11];
    c.fx = intr[v * 4 + 0]; c.fy = intr[v * 4 + 1];
    c.cx = intr[v * 4 + 2]; c.cy = intr[v * 4 + 3];
    c.W = vt.W[v]; c.H = vt.H[v];
    c.limx = kClip * (0.5f * (float)c.W / c.fx);
    c.limy = kClip * (0.5f * (float)c.H / c.fy);
    return c;
}

// Geometry of one Gaussian in one view, shared by the forward and backward.
struct Geo {
    float px, py, pz;        // camera-space mean
    float xr, yr;            // clamped x/z, y/z
    bool clx, cly;
    float T0[3], T1[3];      // T = J R_v (2x3)
    float F0[3], F1[3];      // F = T M (2x3), M = R_q S
    float a, b, c, D;        // Sigma2 = [[a, b], [b, c]], D = det
};

__device__ __forceinline__ void geometry(const Camera& cam, const float* mu, const float* M, float eps2d,
                                         Geo& g)
{
    g.px = cam.r[0] * mu[0] + cam.r[1] * mu[1] + cam.r[2] * mu[2] + cam.t[0];
    g.py = cam.r[3] * mu[0] + cam.r[4] * mu[1] + cam.r[5] * mu[2] + cam.t[1];
    g.pz = cam.r[6] * mu[0] + cam.r[7] * mu[1] + cam.r[8] * mu[2] + cam.t[2];
    const float iz = 1.0f / g.pz;
    const float xr0 = g.px * iz, yr0 = g.py * iz;
    g.clx = (xr0 < -cam.limx) || (xr0 > cam.limx);
    g.cly = (yr0 < -cam.limy) || (yr0 > cam.limy);
    g.xr = fminf(fmaxf(xr0, -cam.limx), cam.limx);
    g.yr = fminf(fmaxf(yr0, -cam.limy), cam.limy);
    // J = [[fx/z, 0, -fx xr/z], [0, fy/z, -fy yr/z]];  T = J R_v
    const float jx = cam.fx * iz, jy = cam.fy * iz;
    for (int k = 0; k < 3; k++) {
        g.T0[k] = jx * (cam.r[k] - g.xr * cam.r[6 + k]);
        g.T1[k] = jy * (cam.r[3 + k] - g.yr * cam.r[6 + k]);
    }
    for (int j = 0; j < 3; j++) {
        g.F0[j] = g.T0[0] * M[j] + g.T0[1] * M[3 + j] + g.T0[2] * M[6 + j];
        g.F1[j] = g.T1[0] * M[j] + g.T1[1] * M[3 + j] + g.T1[2] * M[6 + j];
    }
    const float aa = g.F0[0] * g.F0[0] + g.F0[1] * g.F0[1] + g.F0[2] * g.F0[2];
    const float cc = g.F1[0] * g.F1[0] + g.F1[1] * g.F1[1] + g.F1[2] * g.F1[2];
    g.b = g.F0[0] * g.F1[0] + g.F0[1] * g.F1[1] + g.F0[2] * g.F1[2];
    const float x0 = g.F0[1] * g.F1[2] - g.F0[2] * g.F1[1];
    const float x1 = g.F0[2] * g.F1[0] - g.F0[0] * g.F1[2];
    const float x2 = g.F0[0] * g.F1[1] - g.F0[1] * g.F1[0];
    g.a = aa + eps2d;
    g.c = cc + eps2d;
    g.D = (x0 * x0 + x1 * x1 + x2 * x2) + eps2d * (aa + cc) + eps2d * eps2d;
}

// SV (one view): the SH coefficients are read where the colour sum uses
// them instead of being kept for later views, which frees ~100 VGPRs at
// degree 3 (occupancy 2 -> 6 waves per SIMD for this HBM-bound kernel).
template <int DEG, bool SV>
__global__ __launch_bounds__(256) void k_project(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ opac, const float* __restrict__ sh,
    long long N, const float* __restrict__ viewmats, const float* __restrict__ intr, ViewTable vt,
    float near_plane, float far_plane, float eps2d, int tile, int radius_mode, float* __restrict__ splats,
    float* __restrict__ depths, int2* __restrict__ radii, int* __restrict__ tiles,
    int2* __restrict__ rects, uint8_t* __restrict__ flags, float* __restrict__ g2clear)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const float mu[3] = {nt_load(&means[g]), nt_load(&means[N + g]), nt_load(&means[2 * N + g])};
    const float ls[3] = {nt_load(&log_scales[g]), nt_load(&log_scales[N + g]), nt_load(&log_scales[2 * N + g])};
    const float q[4] = {nt_load(&quats[g]), nt_load(&quats[N + g]), nt_load(&quats[2 * N + g]), nt_load(&quats[3 * N + g])};
    const float o = nt_load(&opac[g]);
    bool finite = isfinite(mu[0]) && isfinite(mu[1]) && isfinite(mu[2]) && isfinite(ls[0]) &&
                  isfinite(ls[1]) && isfinite(ls[2]) && isfinite(q[0]) && isfinite(q[1]) &&
                  isfinite(q[2]) && isfinite(q[3]) && isfinite(o);
    const float qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    finite = finite && qn2 > 0.0f;
    const float sigma = 1.0f / (1.0f + expf(-o));
    const float lsig = log2f(sigma);
    // widened tau = 2 ln(255 sigma) of the region alpha >= 1/255 (d^T Q d <= tau),
    // inflated so that float32 rounding of the per-pixel alpha stays inside
    const float tau = fmaxf(1.38629436f * (7.99435344f + lsig), 0.0f) * 1.001f + 0.01f;
    const float iq = 1.0f / sqrtf(qn2);
    float R[9], M[9];
    quat_to_rot(q[0] * iq, q[1] * iq, q[2] * iq, q[3] * iq, R);
    const float s[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[3 * i + j] = R[3 * i + j] * s[j];

    float coef[SV ? 1 : 3 * K];
    bool have_sh = false;
    for (int v = 0; v < (SV ? 1 : vt.n_views); v++) {
        const Camera cam = load_camera(viewmats, intr, vt, v);
        const long long o_vg = (long long)v * N + g;
        Geo ge;
        geometry(cam, mu, M, eps2d, ge);
        bool vis = finite && ge.pz > near_plane && ge.pz < far_plane && sigma >= kAlphaMin &&
                   ge.D > 0.0f;
        int rx = 0, ry = 0, tt = 0;
        int2 rc = make_int2(0, 0);
        float u = 0.0f, vv = 0.0f;
        if (vis) {
            u = cam.fx * ge.px / ge.pz + cam.cx;
            vv = cam.fy * ge.py / ge.pz + cam.cy;
            if (radius_mode == GS_RADIUS_EIGEN) {
                const float m = 0.5f * (ge.a + ge.c);
                const float lam = m + sqrtf(fmaxf(m * m - ge.D, 0.1f));
                rx = ry = (int)fminf(ceilf(3.0f * sqrtf(lam)), 1073741824.0f);
            } else {
                rx = (int)fminf(ceilf(3.0f * sqrtf(ge.a)), 1073741824.0f);
                ry = (int)fminf(ceilf(3.0f * sqrtf(ge.c)), 1073741824.0f);
            }
            if (radius_mode == GS_RADIUS_OPACITY) {
                const int qx = (int)fminf(ceilf(sqrtf(tau * ge.a)), 1073741823.0f) + 1;
                const int qy = (int)fminf(ceilf(sqrtf(tau * ge.c)), 1073741823.0f) + 1;
                rx = min(rx, qx);
                ry = min(ry, qy);
            }
            int x0, y0, x1, y1;
            tile_rect(u, vv, rx, ry, tile, cam.W, cam.H, x0, y0, x1, y1);
            tt = (x1 - x0) * (y1 - y0);
            vis = tt > 0;
            rc = make_int2(x0 | (y0 << 16), x1 | (y1 << 16));
        }
        uint8_t fl = 0;
        if (vis) {
            // record: Cholesky factor of c0 * conic
            const float sc = sqrtf(ge.c), sD = sqrtf(ge.D);
            const float rc0 = 0.84932180028801904272f;   // sqrt(c0)
            const float m00 = rc0 * sc / sD;
            const float m11 = rc0 / sc;
            const float m10 = -ge.b * (rc0 / (sc * sD));
            // colour along the unit ray from the camera centre c = -R^T t
            const float camc[3] = {
                -(cam.r[0] * cam.t[0] + cam.r[3] * cam.t[1] + cam.r[6] * cam.t[2]),
                -(cam.r[1] * cam.t[0] + cam.r[4] * cam.t[1] + cam.r[7] * cam.t[2]),
                -(cam.r[2] * cam.t[0] + cam.r[5] * cam.t[1] + cam.r[8] * cam.t[2])};
            float d0 = mu[0] - camc[0], d1 = mu[1] - camc[1], d2 = mu[2] - camc[2];
            const float idn = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
            d0 *= idn; d1 *= idn; d2 *= idn;
            float Y[K];
            sh_basis<DEG>(d0, d1, d2, Y);
            if constexpr (!SV) {
                if (!have_sh) {
                    for (int j = 0; j < K; j++)
                        for (int ch = 0; ch < 3; ch++) coef[3 * j + ch] = nt_load(&sh[((long long)j * 3 + ch) * N + g]);
                    have_sh = true;
                }
            }
            // the three channels' sums run side by side over the basis
            // functions (each in the same order as alone), so that all 3 K
            // coefficient loads can be in flight together
            float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int j = 0; j < K; j++)
#pragma unroll
                for (int ch = 0; ch < 3; ch++)
                    acc[ch] += (SV ? nt_load(&sh[((long long)j * 3 + ch) * N + g]) : coef[SV ? 0 : 3 * j + ch]) * Y[j];
            float col[3];
            for (int ch = 0; ch < 3; ch++) {
                const float a = acc[ch] + 0.5f;
                if (a < 0.0f) fl |= (uint8_t)(GS_FLAG_CLAMP_R << ch);
                col[ch] = fmaxf(a, 0.0f);
            }
            fl |= GS_FLAG_VISIBLE;
            float4* rec = reinterpret_cast<float4*>(splats + o_vg * GS_SPLAT_FLOATS);
            rec[0] = make_float4(u, vv, m00, m10);
            rec[1] = make_float4(m11, lsig, col[0], col[1]);
            // conservative pixel box of the region where alpha >= 1/255:
            // half-widths sqrt(tau a), sqrt(tau c), padded by one pixel
            const float ex = sqrtf(tau * ge.a), ey = sqrtf(tau * ge.c);
            rec[2] = make_float4(col[2], sigma, __int_as_float(pack_range(u, ex)),
                                 __int_as_float(pack_range(vv, ey)));
        }
        // the visible pairs' 2-D gradient records, zeroed for a backward that
        // accumulates.  In a full wave the 64 consecutive records are one run
        // of 576 floats, written by 9 coalesced stores in which lane l takes
        // float 64 k + l if its record's pair is visible; the last wave of the
        // grid, whose lanes past N have exited and cannot take their share,
        // writes each visible record from its own lane.
        if (g2clear) {
            const uint64_t vm = __ballot(vis);
            const int lane = __lane_id();
            if (__ballot(true) == ~0ull) {
                float* run = g2clear + (o_vg - lane) * GS_GRAD_FLOATS;
#pragma unroll
                for (int k = 0; k < GS_GRAD_FLOATS; k++) {
                    const int f = k * GS_WAVE + lane;
                    if ((vm >> (f / GS_GRAD_FLOATS)) & 1ull) run[f] = 0.0f;
                }
            } else if (vis) {
                float* rec2 = g2clear + o_vg * GS_GRAD_FLOATS;
#pragma unroll
                for (int k = 0; k < GS_GRAD_FLOATS; k++) rec2[k] = 0.0f;
            }
        }
        depths[o_vg] = ge.pz;
        radii[o_vg] = vis ? make_int2(rx, ry) : make_int2(0, 0);
        tiles[o_vg] = vis ? tt : 0;
        rects[o_vg] = vis ? rc : make_int2(0, 0);
        flags[o_vg] = fl;
    }
}

// SV (one view): the SH gradient is the basis times the colour gradient, so
// only the 16 basis values and 3 colour gradients are kept (not 48 sums), and
// the coefficients are read where they are used instead of being cached
// across views.
//
// ADAM: instead of storing the gradients, the same thread applies the Adam
// step to its Gaussian's parameters in place (the gradient never reaches
// HBM); the parameters are then read and written through the same pointers.
template <bool ADAM>
using ParamPtr = typename std::conditional<ADAM, float*, const float*>::type;

// Adam hyperparameters; the moments of the five parameter tensors (means,
// log-scales, quaternions, opacity logits, SH coefficients) are kernel
// arguments of their own, declared non-aliasing, so that the moment loads of
// later elements may be issued before the stores of earlier ones.
struct AdamState {
    float lr[5];
    float b1, b2, eps;
    const int* step;
};

// Element at byte offset boff of a plane whose base is uniform: the address is
// a scalar base plus one 32-bit lane offset that every plane shares, so the
// Adam variant does not keep a 64-bit address per parameter plane live in
// vector registers (it needs N <= 2^30, which its entry point checks).
template <class T>
__device__ __forceinline__ T* at(T* plane, uint32_t boff)
{
    return reinterpret_cast<T*>(reinterpret_cast<typename std::conditional<std::is_const<T>::value, const char, char>::type*>(plane) + boff);
}

// one parameter element (plane c): gradient gr, either stored or applied by
// Adam to the parameter value p
template <bool ADAM>
__device__ __forceinline__ void emit_grad(float gr, float p, float* p_base, float* d_base, float* m_base,
                                          float* v_base, long long c, long long N, long long g, uint32_t boff,
                                          float step, float rbc2, const AdamState& as)
{
    if constexpr (ADAM) {
        float* const mp = at(m_base + c * N, boff);
        float* const vp = at(v_base + c * N, boff);
        float m = nt_load(mp), v = nt_load(vp);
        adam_elem(p, gr, m, v, as.b1, as.b2, step, rbc2, as.eps);
        nt_store(p, at(p_base + c * N, boff));
        nt_store(m, mp);
        nt_store(v, vp);
    } else {
        nt_store(gr, &d_base[c * N + g]);
    }
}

template <int DEG, bool SV, bool ADAM>
__global__ __launch_bounds__(256) void k_project_bwd(
    ParamPtr<ADAM> __restrict__ means, ParamPtr<ADAM> __restrict__ log_scales,
    ParamPtr<ADAM> __restrict__ quats, ParamPtr<ADAM> __restrict__ opac, ParamPtr<ADAM> __restrict__ sh,
    long long N, const float* __restrict__ viewmats, const float* __restrict__ intr, ViewTable vt,
    float eps2d, const uint8_t* __restrict__ flags, const float* __restrict__ grad2d,
    float* __restrict__ d_means, float* __restrict__ d_log_scales, float* __restrict__ d_quats,
    float* __restrict__ d_opac, float* __restrict__ d_sh, AdamState as, float* __restrict__ m0,
    float* __restrict__ m1, float* __restrict__ m2, float* __restrict__ m3, float* __restrict__ m4,
    float* __restrict__ v0, float* __restrict__ v1, float* __restrict__ v2, float* __restrict__ v3,
    float* __restrict__ v4, int seen_only)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    // coefficients held in registers: several views, or the Adam update
    constexpr bool CACHE = !SV || ADAM;
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;

    float gmu[3] = {0.0f, 0.0f, 0.0f};
    float gM[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    float gsig = 0.0f;
    float gsh[SV ? 1 : 3 * K];
    for (int j = 0; j < (SV ? 1 : 3 * K); j++) gsh[j] = 0.0f;
    // one view: the SH basis and colour gradient, kept for one store of the
    // SH gradient by every lane after the view loop (zero where unseen)
    float Ysv[SV ? K : 1], gcsv[3] = {0.0f, 0.0f, 0.0f};
    for (int j = 0; j < (SV ? K : 1); j++) Ysv[j] = 0.0f;

    bool any = false;
    uint8_t fl0 = 0;   // the flags of the first view (the only one when SV)
    for (int v = 0; v < vt.n_views; v++) {
        const uint8_t f = flags[(long long)v * N + g];
        if (v == 0) fl0 = f;
        any |= (f & GS_FLAG_VISIBLE) != 0;
    }
    // the gradients of a group of 64 Gaussians (one wave) that no view sees
    // are left to the unseen part; a group with a seen Gaussian is written
    // whole here (zeros included), so each line is written once, in full
    if (seen_only && __ballot(any) == 0ull) return;

    // a Gaussian no view sees gets zero gradients without reading its
    // parameters (whole cache lines are skipped when such Gaussians are
    // contiguous, e.g. in Morton order)
    // (the Adam update needs every parameter whatever the gradient)
    uint32_t boff = ADAM ? (uint32_t)g * 4u : 0u;
    auto ldp = [&](const float* base, long long c) {
        return ADAM ? nt_load(at(base + c * N, boff)) : nt_load(&base[c * N + g]);
    };
    // The loads of one wave are issued together where possible: a load under
    // a condition becomes a branch with a wait of its own, and a loop of
    // loads each used at once waits once per iteration.
    float mu[3] = {0.0f, 0.0f, 0.0f}, ls[3] = {0.0f, 0.0f, 0.0f}, q[4] = {1.0f, 0.0f, 0.0f, 0.0f};
    float ologit = 0.0f;
    // one view: the pair's whole 2-D gradient record, read with the parameters
    float gr1[GS_GRAD_FLOATS];
    for (int k = 0; k < GS_GRAD_FLOATS; k++) gr1[k] = 0.0f;
    if (ADAM || any) {
        for (int i = 0; i < 3; i++) mu[i] = ldp(means, i);
        for (int i = 0; i < 3; i++) ls[i] = ldp(log_scales, i);
        for (int i = 0; i < 4; i++) q[i] = ldp(quats, i);
        ologit = ldp(opac, 0);
        if (SV && any)
            for (int k = 0; k < GS_GRAD_FLOATS; k++) gr1[k] = nt_load(&grad2d[g * GS_GRAD_FLOATS + k]);
    }
    const float qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const float iq = any ? 1.0f / sqrtf(qn2) : 0.0f;
    const float qh[4] = {q[0] * iq, q[1] * iq, q[2] * iq, q[3] * iq};
    float R[9], M[9];
    quat_to_rot(qh[0], qh[1], qh[2], qh[3], R);
    const float s[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[3 * i + j] = R[3 * i + j] * s[j];

    float coef[CACHE ? 3 * K : 1];
    if (CACHE && (ADAM || any)) {
        for (int j = 0; j < K; j++)
            for (int ch = 0; ch < 3; ch++) coef[3 * j + ch] = ldp(sh, j * 3 + ch);
    }
    // coefficient j, channel ch
    auto cf = [&](int j, int ch) {
        return CACHE ? coef[CACHE ? 3 * j + ch : 0] : nt_load(&sh[((long long)j * 3 + ch) * N + g]);
    };

    for (int v = 0; any && v < (SV ? 1 : vt.n_views); v++) {
        const long long o_vg = (long long)v * N + g;
        const uint8_t fl = SV ? fl0 : flags[o_vg];
        if (!(fl & GS_FLAG_VISIBLE)) continue;
        const float* gr = grad2d + o_vg * GS_GRAD_FLOATS;
        float grv[GS_GRAD_FLOATS];
        for (int k = 0; k < GS_GRAD_FLOATS; k++) grv[k] = SV ? gr1[k] : nt_load(&gr[k]);
        const float gu = grv[0], gv = grv[1], gA = grv[2], gB = grv[3], gC = grv[4];
        gsig += grv[5];
        const Camera cam = load_camera(viewmats, intr, vt, v);
        Geo ge;
        geometry(cam, mu, M, eps2d, ge);

        // conic Q = [[A, B], [B, C]] = Sigma2^-1;  dL/dSigma2 = -Q G Q
        const float iD = 1.0f / ge.D;
        const float A = ge.c * iD, B = -ge.b * iD, C = ge.a * iD;
        const float hB = 0.5f * gB;
        const float p00 = A * gA + B * hB, p01 = A * hB + B * gC;
        const float p10 = B * gA + C * hB, p11 = B * hB + C * gC;
        const float s00 = -(p00 * A + p01 * B);
        const float s01 = -(p00 * B + p01 * C);
        const float s11 = -(p10 * B + p11 * C);
        // Sigma2 = F F^T + eps I:  dF = 2 dSigma2 F
        float gF0[3], gF1[3];
        for (int j = 0; j < 3; j++) {
            gF0[j] = 2.0f * (s00 * ge.F0[j] + s01 * ge.F1[j]);
            gF1[j] = 2.0f * (s01 * ge.F0[j] + s11 * ge.F1[j]);
        }
        // F = T M:  dT = dF M^T,  dM += T^T dF
        float gT0[3], gT1[3];
        for (int k = 0; k < 3; k++) {
            gT0[k] = gF0[0] * M[3 * k] + gF0[1] * M[3 * k + 1] + gF0[2] * M[3 * k + 2];
            gT1[k] = gF1[0] * M[3 * k] + gF1[1] * M[3 * k + 1] + gF1[2] * M[3 * k + 2];
            for (int j = 0; j < 3; j++) gM[3 * k + j] += ge.T0[k] * gF0[j] + ge.T1[k] * gF1[j];
        }
        // T = J R_v:  dJ_ik = dT_i . (row k of R_v)
        const float gJ00 = gT0[0] * cam.r[0] + gT0[1] * cam.r[1] + gT0[2] * cam.r[2];
        const float gJ02 = gT0[0] * cam.r[6] + gT0[1] * cam.r[7] + gT0[2] * cam.r[8];
        const float gJ11 = gT1[0] * cam.r[3] + gT1[1] * cam.r[4] + gT1[2] * cam.r[5];
        const float gJ12 = gT1[0] * cam.r[6] + gT1[1] * cam.r[7] + gT1[2] * cam.r[8];
        // J(p) and (u, v)(p)
        const float z = ge.pz, iz = 1.0f / z, iz2 = iz * iz;
        float gx = 0.0f, gy = 0.0f, gz = 0.0f;
        gz -= cam.fx * iz2 * gJ00 + cam.fy * iz2 * gJ11;
        if (!ge.clx) { gx -= cam.fx * iz2 * gJ02; gz += 2.0f * cam.fx * ge.px * iz2 * iz * gJ02; }
        else gz += cam.fx * ge.xr * iz2 * gJ02;
        if (!ge.cly) { gy -= cam.fy * iz2 * gJ12; gz += 2.0f * cam.fy * ge.py * iz2 * iz * gJ12; }
        else gz += cam.fy * ge.yr * iz2 * gJ12;
        gx += gu * cam.fx * iz;
        gz -= gu * cam.fx * ge.px * iz2;
        gy += gv * cam.fy * iz;
        gz -= gv * cam.fy * ge.py * iz2;
        // p = R_v mu + t
        for (int i = 0; i < 3; i++) gmu[i] += cam.r[i] * gx + cam.r[3 + i] * gy + cam.r[6 + i] * gz;

        // colour
        const float camc[3] = {
            -(cam.r[0] * cam.t[0] + cam.r[3] * cam.t[1] + cam.r[6] * cam.t[2]),
            -(cam.r[1] * cam.t[0] + cam.r[4] * cam.t[1] + cam.r[7] * cam.t[2]),
            -(cam.r[2] * cam.t[0] + cam.r[5] * cam.t[1] + cam.r[8] * cam.t[2])};
        float d0 = mu[0] - camc[0], d1 = mu[1] - camc[1], d2 = mu[2] - camc[2];
        const float idn = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
        d0 *= idn; d1 *= idn; d2 *= idn;
        float Y[K], sdot[K];
        sh_basis<DEG>(d0, d1, d2, Y);
        const float gc[3] = {(fl & GS_FLAG_CLAMP_R) ? 0.0f : grv[6], (fl & GS_FLAG_CLAMP_G) ? 0.0f : grv[7],
                             (fl & GS_FLAG_CLAMP_B) ? 0.0f : grv[8]};
        // coefficients read from memory in batches of SH_BATCH basis functions,
        // the batch's three channels all in flight before any is used
        constexpr int SH_BATCH = 8;
        for (int j0 = 0; j0 < K; j0 += SH_BATCH) {
            float cb[SH_BATCH][3];
#pragma unroll
            for (int jj = 0; jj < SH_BATCH; jj++)
#pragma unroll
                for (int ch = 0; ch < 3; ch++) cb[jj][ch] = j0 + jj < K ? cf(j0 + jj, ch) : 0.0f;
#pragma unroll
            for (int jj = 0; jj < SH_BATCH; jj++) {
                const int j = j0 + jj;
                if (j >= K) break;
                sdot[j] = cb[jj][0] * gc[0] + cb[jj][1] * gc[1] + cb[jj][2] * gc[2];
                if constexpr (SV) {
                    Ysv[j] = Y[j];
                } else {
                    gsh[3 * j] += Y[j] * gc[0];
                    gsh[3 * j + 1] += Y[j] * gc[1];
                    gsh[3 * j + 2] += Y[j] * gc[2];
                }
            }
        }
        if constexpr (SV)
            for (int ch = 0; ch < 3; ch++) gcsv[ch] = gc[ch];
        if (DEG > 0) {
            float gdx, gdy, gdz;
            sh_grad_dot<DEG>(d0, d1, d2, sdot, gdx, gdy, gdz);
            const float dg = d0 * gdx + d1 * gdy + d2 * gdz;
            gmu[0] += (gdx - d0 * dg) * idn;
            gmu[1] += (gdy - d1 * dg) * idn;
            gmu[2] += (gdz - d2 * dg) * idn;
        }
    }

    float a_step[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, rbc2 = 0.0f;
    if constexpr (ADAM) {
        // the update's addresses are formed afresh from the lane offset (an
        // opaque copy), instead of the compiler keeping the 64-bit address of
        // every coefficient plane live from the loads above
        asm volatile("" : "+v"(boff));
        const AdamCoef ac = adam_coef(*as.step, as.b1, as.b2);
        for (int k = 0; k < 5; k++) a_step[k] = as.lr[k] * ac.step_scale;
        rbc2 = ac.rbc2;
    }

    // every lane of the wave stores each SH plane at once: whole lines, not
    // two partial writes (seen and unseen lanes) that may each reach HBM
    if constexpr (SV)
        for (int j = 0; j < K; j++)
            for (int ch = 0; ch < 3; ch++)
                emit_grad<ADAM>(Ysv[j] * gcsv[ch], CACHE ? coef[CACHE ? 3 * j + ch : 0] : 0.0f, (float*)sh, d_sh,
                                m4, v4, j * 3 + ch, N, g, boff, a_step[4], rbc2, as);

    // M = R diag(s), s = exp(l):  dl_j = s_j sum_i dM_ij R_ij;  dR_ij = dM_ij s_j
    float gR[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) gR[3 * i + j] = gM[3 * i + j] * s[j];
    float gl[3];
    for (int j = 0; j < 3; j++) gl[j] = s[j] * (gM[j] * R[j] + gM[3 + j] * R[3 + j] + gM[6 + j] * R[6 + j]);
    const float w = qh[0], x = qh[1], y = qh[2], zq = qh[3];
    float gq[4];
    gq[0] = 2.0f * (-zq * gR[1] + y * gR[2] + zq * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    gq[1] = 2.0f * (y * gR[1] + zq * gR[2] + y * gR[3] - 2.0f * x * gR[4] - w * gR[5] + zq * gR[6] +
                    w * gR[7] - 2.0f * x * gR[8]);
    gq[2] = 2.0f * (-2.0f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + zq * gR[5] - w * gR[6] +
                    zq * gR[7] - 2.0f * y * gR[8]);
    gq[3] = 2.0f * (-2.0f * zq * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0f * zq * gR[4] +
                    y * gR[5] + x * gR[6] + y * gR[7]);
    const float qd = w * gq[0] + x * gq[1] + y * gq[2] + zq * gq[3];
    const float sigma = any ? 1.0f / (1.0f + expf(-ologit)) : 0.0f;

    for (int i = 0; i < 3; i++)
        emit_grad<ADAM>(any ? gmu[i] : 0.0f, mu[i], (float*)means, d_means, m0, v0, i, N, g, boff, a_step[0], rbc2,
                        as);
    for (int i = 0; i < 3; i++)
        emit_grad<ADAM>(any ? gl[i] : 0.0f, ls[i], (float*)log_scales, d_log_scales, m1, v1, i, N, g, boff,
                        a_step[1], rbc2, as);
    for (int k = 0; k < 4; k++)
        emit_grad<ADAM>(any ? (gq[k] - qh[k] * qd) * iq : 0.0f, q[k], (float*)quats, d_quats, m2, v2, k, N, g, boff,
                        a_step[2], rbc2, as);
    emit_grad<ADAM>(any ? gsig * sigma * (1.0f - sigma) : 0.0f, ologit, (float*)opac, d_opac, m3, v3, 0, N, g, boff,
                    a_step[3], rbc2, as);
    if constexpr (!SV)
        for (int j = 0; j < K; j++)
            for (int ch = 0; ch < 3; ch++)
                emit_grad<ADAM>(gsh[3 * j + ch], coef[3 * j + ch], (float*)sh, d_sh, m4, v4, j * 3 + ch, N, g, boff,
                                a_step[4], rbc2, as);
}

constexpr long long kZeroUnseenBlocks = 256;

// Zero gradients of every group of 64 Gaussians (one wave) that no view
// sees: the part of the projection backward that needs no 2-D gradient.  A
// grid-stride loop over Gaussians; each plane is written by consecutive
// lanes, whole lines.
__global__ __launch_bounds__(256) void k_zero_unseen(const uint8_t* __restrict__ flags, long long N, int n_views,
                                                     int sh_planes, float* __restrict__ d_means,
                                                     float* __restrict__ d_log_scales, float* __restrict__ d_quats,
                                                     float* __restrict__ d_opac, float* __restrict__ d_sh)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) {
        bool any = false;
        for (int v = 0; v < n_views; v++) any |= (flags[(long long)v * N + g] & GS_FLAG_VISIBLE) != 0;
        if (__ballot(any) != 0ull) continue;
        for (int i = 0; i < 3; i++) nt_store(0.0f, &d_means[i * N + g]);
        for (int i = 0; i < 3; i++) nt_store(0.0f, &d_log_scales[i * N + g]);
        for (int i = 0; i < 4; i++) nt_store(0.0f, &d_quats[i * N + g]);
        nt_store(0.0f, &d_opac[g]);
        for (int c = 0; c < sh_planes; c++) nt_store(0.0f, &d_sh[c * N + g]);
    }
}

}  // namespace

#define GS_PROJ_LAUNCH(DEG)                                                                            \
    if (vt.n_views == 1)                                                                               \
        hipLaunchKernelGGL((k_project<DEG, true>), dim3(blocks), dim3(256), 0, stream, means, log_scales, \
                           quats, opac, sh, N, viewmats, intr, vt, near_plane, far_plane, eps2d, tile,   \
                           radius_mode, splats, depths, radii, tiles, rects, flags, g2clear);            \
    else                                                                                               \
        hipLaunchKernelGGL((k_project<DEG, false>), dim3(blocks), dim3(256), 0, stream, means,            \
                           log_scales, quats, opac, sh, N, viewmats, intr, vt, near_plane, far_plane,     \
                           eps2d, tile, radius_mode, splats, depths, radii, tiles, rects, flags, g2clear)

hipError_t launch_project(int deg, const float* means, const float* log_scales, const float* quats,
                          const float* opac, const float* sh, long long N, const float* viewmats,
                          const float* intr, const ViewTable& vt, float near_plane, float far_plane,
                          float eps2d, int tile, int radius_mode, float* splats, float* depths, int2* radii,
                          int* tiles, int2* rects, uint8_t* flags, float* g2clear, hipStream_t stream)
{
    if (N == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((N + 255) / 256);
    switch (deg) {
    case 0: GS_PROJ_LAUNCH(0); break;
    case 1: GS_PROJ_LAUNCH(1); break;
    case 2: GS_PROJ_LAUNCH(2); break;
    default: GS_PROJ_LAUNCH(3); break;
    }
    return hipGetLastError();
}

namespace {

template <bool ADAM>
hipError_t launch_bwd(int deg, ParamPtr<ADAM> means, ParamPtr<ADAM> log_scales, ParamPtr<ADAM> quats,
                      ParamPtr<ADAM> opac, ParamPtr<ADAM> sh, long long N, const float* viewmats, const float* intr,
                      const ViewTable& vt, float eps2d, const uint8_t* flags, const float* grad2d, float* d_means,
                      float* d_log_scales, float* d_quats, float* d_opac, float* d_sh, const AdamState& as,
                      float* const* mo, float* const* vo, int seen_only, hipStream_t stream)
{
    if (N == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((N + 255) / 256);
#define GS_PROJ_BWD_LAUNCH(DEG)                                                                         \
    if (vt.n_views == 1)                                                                                \
        hipLaunchKernelGGL((k_project_bwd<DEG, true, ADAM>), dim3(blocks), dim3(256), 0, stream, means,    \
                           log_scales, quats, opac, sh, N, viewmats, intr, vt, eps2d, flags, grad2d,      \
                           d_means, d_log_scales, d_quats, d_opac, d_sh, as, mo[0], mo[1], mo[2], mo[3], mo[4], \
                           vo[0], vo[1], vo[2], vo[3], vo[4], seen_only);                                \
    else                                                                                                \
        hipLaunchKernelGGL((k_project_bwd<DEG, false, ADAM>), dim3(blocks), dim3(256), 0, stream, means,   \
                           log_scales, quats, opac, sh, N, viewmats, intr, vt, eps2d, flags, grad2d,      \
                           d_means, d_log_scales, d_quats, d_opac, d_sh, as, mo[0], mo[1], mo[2], mo[3], mo[4], \
                           vo[0], vo[1], vo[2], vo[3], vo[4], seen_only)
    switch (deg) {
    case 0: GS_PROJ_BWD_LAUNCH(0); break;
    case 1: GS_PROJ_BWD_LAUNCH(1); break;
    case 2: GS_PROJ_BWD_LAUNCH(2); break;
    default: GS_PROJ_BWD_LAUNCH(3); break;
    }
#undef GS_PROJ_BWD_LAUNCH
    return hipGetLastError();
}

}  // namespace

hipError_t launch_project_bwd(int deg, const float* means, const float* log_scales,
                              const float* quats, const float* opac, const float* sh, long long N,
                              const float* viewmats, const float* intr, const ViewTable& vt,
                              float eps2d, const uint8_t* flags, const float* grad2d,
                              float* d_means, float* d_log_scales, float* d_quats, float* d_opac,
                              float* d_sh, int part, hipStream_t stream)
{
    if (N == 0) return hipSuccess;
    if (part == 2) {
        // a few workgroups per CU, so that the kernels it runs beside keep
        // room on every CU
        const long long need = (N + 255) / 256;
        const unsigned blocks = (unsigned)(need < kZeroUnseenBlocks ? need : kZeroUnseenBlocks);
        hipLaunchKernelGGL(k_zero_unseen, dim3(blocks), dim3(256), 0, stream, flags, N, vt.n_views,
                           3 * (deg + 1) * (deg + 1), d_means, d_log_scales, d_quats, d_opac, d_sh);
        return hipGetLastError();
    }
    const AdamState none = {};
    float* const no_moments[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    return launch_bwd<false>(deg, means, log_scales, quats, opac, sh, N, viewmats, intr, vt, eps2d, flags, grad2d,
                             d_means, d_log_scales, d_quats, d_opac, d_sh, none, no_moments, no_moments,
                             part == 1 ? 1 : 0, stream);
}

hipError_t launch_step_advance(int* step_dev, hipStream_t st);

hipError_t launch_project_bwd_adam(int deg, float* means, float* log_scales, float* quats, float* opac, float* sh,
                                   long long N, const float* viewmats, const float* intr, const ViewTable& vt,
                                   float eps2d, const uint8_t* flags, const float* grad2d, float* const* exp_avg,
                                   float* const* exp_avg_sq, const float* lrs, float beta1, float beta2, float eps,
                                   int* step_dev, hipStream_t stream)
{
    AdamState as;
    for (int k = 0; k < 5; k++) as.lr[k] = lrs[k];
    as.b1 = beta1;
    as.b2 = beta2;
    as.eps = eps;
    as.step = step_dev;
    const hipError_t e = launch_bwd<true>(deg, means, log_scales, quats, opac, sh, N, viewmats, intr, vt, eps2d,
                                          flags, grad2d, nullptr, nullptr, nullptr, nullptr, nullptr, as, exp_avg,
                                          exp_avg_sq, 0, stream);
    return e != hipSuccess ? e : launch_step_advance(step_dev, stream);
}

}  // namespace gs
