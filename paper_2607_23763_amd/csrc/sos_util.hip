// Small stream-ordered helper kernels (graph-capture safe: no memset nodes).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// dst[i] = src ? src[i] : 0 for i < count
__global__ void __launch_bounds__(256) fill_kernel(float *dst, const float *src, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = src ? src[i] : 0.0f;
}

}  // namespace

extern "C" hipError_t sos_launch_fill(float *dst, const float *src, int64_t count,
                                      hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, dst, src, count);
    return hipGetLastError();
}
