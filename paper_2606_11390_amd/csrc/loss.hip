// L2 image loss and its gradient (gfx950).
//
// Paper Section 4: after rasterising a camera the image-space loss is
// evaluated per camera.  loss = mean((img - target)^2) over every packed image
// element; d_img = 2 (img - target) / n.  The sum is reduced in a fixed order
// (per-block partials in double, then one block) so the loss is deterministic.
#include <mutex>

#include "gs_device.h"

namespace gs {
namespace {

constexpr int L_THREADS = 256;
typedef float lf4 __attribute__((ext_vector_type(4)));

// VEC: the three arrays are 16-byte aligned; four elements per thread and
// step as one 16-byte load or store, the last n mod 4 by the first threads
template <bool VEC>
__global__ __launch_bounds__(L_THREADS) void k_l2_partial(const float* __restrict__ img,
                                                          const float* __restrict__ tgt,
                                                          long long n, float scale,
                                                          float* __restrict__ dimg,
                                                          double* __restrict__ part)
{
    __shared__ double s_w[L_THREADS / GS_WAVE];
    const long long stride = (long long)gridDim.x * L_THREADS;
    const long long first = (long long)blockIdx.x * L_THREADS + threadIdx.x;
    float acc = 0.0f;
    if (VEC) {
        const long long n4 = n / 4;
        const lf4* __restrict__ a4 = reinterpret_cast<const lf4*>(img);
        const lf4* __restrict__ b4 = reinterpret_cast<const lf4*>(tgt);
        lf4* __restrict__ g4 = reinterpret_cast<lf4*>(dimg);
        for (long long i = first; i < n4; i += stride) {
            const lf4 d = a4[i] - b4[i];
            __builtin_nontemporal_store(scale * d, &g4[i]);
            acc = __builtin_fmaf(d.x, d.x, acc);
            acc = __builtin_fmaf(d.y, d.y, acc);
            acc = __builtin_fmaf(d.z, d.z, acc);
            acc = __builtin_fmaf(d.w, d.w, acc);
        }
        if (first < n - 4 * n4) {
            const long long i = 4 * n4 + first;
            const float d = img[i] - tgt[i];
            dimg[i] = scale * d;
            acc = __builtin_fmaf(d, d, acc);
        }
    } else {
        for (long long i = first; i < n; i += stride) {
            const float d = img[i] - tgt[i];
            nt_store(scale * d, &dimg[i]);
            acc = __builtin_fmaf(d, d, acc);
        }
    }
    const float ws = wave_sum(acc);
    if (__lane_id() == 0) s_w[threadIdx.x / GS_WAVE] = (double)ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < L_THREADS / GS_WAVE; i++) s += s_w[i];
        part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(L_THREADS) void k_l2_final(const double* __restrict__ part, int nb,
                                                        double inv_n, float* __restrict__ loss)
{
    __shared__ double s[L_THREADS];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += L_THREADS) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = L_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(s[0] * inv_n);
}

constexpr int L_MAX_BLOCKS = 2048;

int loss_blocks(long long n)
{
    long long nb = (n + L_THREADS * 16 - 1) / (L_THREADS * 16);
    if (nb < 1) nb = 1;
    if (nb > L_MAX_BLOCKS) nb = L_MAX_BLOCKS;
    return (int)nb;
}

}  // namespace

// Partial sums of the allocation-free entry point: one double per block of
// k_l2_partial (at most L_MAX_BLOCKS, whatever the element count).  Every GPU
// the library runs on holds its own copy for the life of the process.
static __device__ __align__(256) double scratch[L_MAX_BLOCKS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (the array's name in host code is only a stand-in for the
// symbol, never an address a kernel may use).
hipError_t scratch_of_current_device(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

size_t loss_workspace_size(long long n) { return sizeof(double) * (size_t)loss_blocks(n); }

hipError_t launch_loss_l2(const float* img, const float* tgt, long long n, float* loss, float* dimg,
                          void* ws, hipStream_t st)
{
    const int nb = loss_blocks(n);
    const float scale = n > 0 ? (float)(2.0 / (double)n) : 0.0f;
    const bool vec = ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(tgt) |
                       reinterpret_cast<uintptr_t>(dimg)) & 15u) == 0;
    if (vec)
        hipLaunchKernelGGL(k_l2_partial<true>, dim3(nb), dim3(L_THREADS), 0, st, img, tgt, n, scale, dimg,
                           (double*)ws);
    else
        hipLaunchKernelGGL(k_l2_partial<false>, dim3(nb), dim3(L_THREADS), 0, st, img, tgt, n, scale, dimg,
                           (double*)ws);
    hipLaunchKernelGGL(k_l2_final, dim3(1), dim3(L_THREADS), 0, st, (const double*)ws, nb,
                       n > 0 ? 1.0 / (double)n : 0.0, loss);
    return hipGetLastError();
}

hipError_t launch_loss_l2_noalloc(const float* img, const float* tgt, long long n, float* loss, float* dimg,
                                  hipStream_t st)
{
    if (loss_blocks(n) > L_MAX_BLOCKS) return hipErrorInvalidValue;
    double* ws = nullptr;
    const hipError_t e = scratch_of_current_device(&ws);
    if (e != hipSuccess) return e;
    return launch_loss_l2(img, tgt, n, loss, dimg, ws, st);
}

}  // namespace gs
