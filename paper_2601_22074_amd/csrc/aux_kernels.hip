// Small helper kernels of the runtime: world reset, buffer fill and tiling.
#include <hip/hip_runtime.h>

#include "rb_internal.h"

namespace {

// Reset listed worlds: clear the status word and load (or zero) the warm start.
// ids outside [0, capacity) are ignored.
__global__ void reset_kernel(int nv, const int32_t* ids, int n, const float* qacc_ws, DevWorlds W, int capacity) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int i = t / RB_WAVE, lane = t % RB_WAVE;
    if (i >= n) return;
    int id = ids[i];
    if (id < 0 || id >= capacity) return;
    for (int k = lane; k < nv; k += RB_WAVE) W.qacc_ws[(size_t)id * nv + k] = qacc_ws ? qacc_ws[(size_t)i * nv + k] : 0.f;
    if (lane == 0) W.status[id] = 0u;
}

__global__ void tile_kernel(float* dst, const float* src, size_t k, size_t total) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) dst[i] = src[i % k];
}

__global__ void fill_kernel(float* dst, float value, size_t count) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = value;
}

}  // namespace

hipError_t rb_launch_reset(int nv, const int32_t* ids, int n, const float* qacc_ws, DevWorlds W, int capacity,
                           hipStream_t stream) {
    size_t threads = (size_t)n * RB_WAVE;
    dim3 block(256), grid((unsigned)((threads + 255) / 256));
    hipLaunchKernelGGL(reset_kernel, grid, block, 0, stream, nv, ids, n, qacc_ws, W, capacity);
    return hipGetLastError();
}

hipError_t rb_launch_fill(float* dst, float value, size_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    dim3 block(256), grid((unsigned)((count + 255) / 256));
    hipLaunchKernelGGL(fill_kernel, grid, block, 0, stream, dst, value, count);
    return hipGetLastError();
}

// dst[c * k + i] = src[i] for every copy c < copies (per-world expansion of a model field)
hipError_t rb_launch_tile(float* dst, const float* src, size_t k, size_t copies, hipStream_t stream) {
    const size_t total = k * copies;
    if (total == 0) return hipSuccess;
    dim3 block(256), grid((unsigned)((total + 255) / 256));
    hipLaunchKernelGGL(tile_kernel, grid, block, 0, stream, dst, src, k, total);
    return hipGetLastError();
}
