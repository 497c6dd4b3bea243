// Small stream-ordered helper kernels (graph-capture safe: no memset nodes).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// dst[i] = src ? src[i] : 0 for i < count
__global__ void __launch_bounds__(256) fill_kernel(float *dst, const float *src, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = src ? src[i] : 0.0f;
}

// Plain streaming copy y = x with the same 128-bit nontemporal accesses the
// filter uses: 8 bytes of HBM traffic per sample and no arithmetic. It is the
// achievable memory floor t_mem = b_s / BW of the cost model (Eq. (28)) and
// the reference for scaling the HBM byte counters.
// One 128-bit element per thread, one wave of blocks over the whole array
// (measured faster on MI355X than a grid-stride loop).
__global__ void __launch_bounds__(256) copy_kernel(const f4 *x, f4 *y, int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(x + i), y + i);
}

// End of a server step: the launch's error bits and its B per-signal error
// words to the step's host result words (pinned, coherent host memory); the
// launch's bits are then cleared for the next launch (the per-signal words
// are rewritten by the next work table).
__global__ void __launch_bounds__(256)
report_err_kernel(unsigned *ctrl_err, unsigned *host_err, const unsigned *sig_err,
                  unsigned *host_sig_err, int B)
{
    for (int i = threadIdx.x; i < B; i += blockDim.x) host_sig_err[i] = sig_err[i];
    if (threadIdx.x == 0) {
        *host_err = *ctrl_err;
        *ctrl_err = 0u;
    }
}

}  // namespace

extern "C" hipError_t sos_launch_report_err(unsigned *ctrl_err, unsigned *host_err,
                                            const unsigned *sig_err, unsigned *host_sig_err,
                                            int B, hipStream_t stream)
{
    if (B > 0 && (!sig_err || !host_sig_err)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(report_err_kernel, dim3(1), dim3(256), 0, stream, ctrl_err, host_err,
                       sig_err, host_sig_err, B);
    return hipGetLastError();
}

extern "C" hipError_t sos_launch_fill(float *dst, const float *src, int64_t count,
                                      hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, dst, src, count);
    return hipGetLastError();
}

extern "C" hipError_t sos_launch_copy(const float *x, float *y, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const bool vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15u) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    if (n4 > 0) {
        const int64_t blocks = (n4 + 255) / 256;
        if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                           reinterpret_cast<const f4 *>(x), reinterpret_cast<f4 *>(y), n4);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n4 * 4 < n) return sos_launch_fill(y + n4 * 4, x + n4 * 4, n - n4 * 4, stream);
    return hipSuccess;
}
