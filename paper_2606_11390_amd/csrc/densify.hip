// Per-Gaussian statistics of adaptive density control (gfx950).
//
// 3D Gaussian Splatting (Kerbl et al. 2023), which the paper uses to densify
// to larger Gaussian counts (Section 5), clones or splits a Gaussian when the
// running mean, over the views that saw it, of the norm of its projected
// mean's gradient in normalised device coordinates exceeds a threshold, and
// prunes by screen size.  This kernel gathers those running sums from one
// step's 2-D gradient records: one thread per Gaussian walks the views in
// order (deterministic, no atomics).  Reads 9 x 4 + 1 + 8 bytes per
// (view, Gaussian) and 12 bytes per Gaussian, writes 12 bytes per Gaussian.
#include "gs_device.h"

namespace gs {
namespace {

__global__ __launch_bounds__(256) void k_densify_stats(const float* __restrict__ grad2d,
                                                       const uint8_t* __restrict__ flags,
                                                       const int2* __restrict__ radii, long long N, ViewTable vt,
                                                       float* __restrict__ grad_accum, int* __restrict__ count,
                                                       int* __restrict__ max_radius)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    float acc = grad_accum[g];
    int cnt = count[g], mr = max_radius[g];
    for (int v = 0; v < vt.n_views; v++) {
        const long long o = (long long)v * N + g;
        if (!(flags[o] & GS_FLAG_VISIBLE)) continue;
        // du/dx_ndc = W / 2, dv/dy_ndc = H / 2
        const float gx = grad2d[o * GS_GRAD_FLOATS + 0] * (0.5f * (float)vt.W[v]);
        const float gy = grad2d[o * GS_GRAD_FLOATS + 1] * (0.5f * (float)vt.H[v]);
        acc += sqrtf(gx * gx + gy * gy);
        cnt += 1;
        const int2 r = radii[o];
        mr = max(mr, max(r.x, r.y));
    }
    grad_accum[g] = acc;
    count[g] = cnt;
    max_radius[g] = mr;
}

}  // namespace

hipError_t launch_densify_stats(const float* grad2d, const uint8_t* flags, const int2* radii, long long N,
                                const ViewTable& vt, float* grad_accum, int* count, int* max_radius,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_densify_stats, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, grad2d, flags, radii,
                       N, vt, grad_accum, count, max_radius);
    return hipGetLastError();
}

}  // namespace gs
