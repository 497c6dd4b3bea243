// Work table of an uneven batch, built on the device so that a batched launch
// can be captured in a HIP graph and replayed with new per-signal data.
//
// Signal i (samples [sig_off[i], sig_off[i+1]), K[i] sections at sec_off[i])
// is cut into G_i = ceil(n_i / C) groups of C samples. gpre is the exclusive
// prefix of the G_i, so tickets gpre[i] .. gpre[i+1]-1 are the groups of
// signal i in order, and sigmap[t] names the signal of ticket t. A signal
// whose arguments are inconsistent is given no groups and reported through the
// handle's error bits; a signal with no samples gets zf = zi here.
#include "sos_device.h"

using namespace sosdev;

namespace {

constexpr int kScanThreads = 1024;

__device__ inline bool signal_ok(int i, int kmax, int64_t rows, int64_t total_samples,
                                 const int32_t *Ks, const int32_t *sec_off,
                                 const int64_t *sig_off)
{
    return batch_signal_ok(i, kmax, rows, total_samples, Ks, sec_off, sig_off);
}

// zf := zi (zeros without zi) for a consistent signal with no samples.
__device__ inline void empty_signal_state(int i, const int32_t *Ks, const int32_t *sec_off,
                                          const float *zi, float *zf, int k0, int dk)
{
    const int64_t so = sec_off[i];
    for (int k = k0; k < 2 * Ks[i]; k += dk) zf[2 * so + k] = zi ? zi[2 * so + k] : 0.0f;
}

// One block of kScanThreads threads: group counts and their exclusive prefix.
// Optionally it first copies `stage_bytes` of arguments from host memory
// (pinned, coherent) to device memory and arms the filter launch (ticket 0, a
// fresh epoch), which saves a step of the server a copy and a launch.
// fuse != 0 (B <= kScanThreads, few groups): it also fills the ticket map and
// the empty signals' final states, which saves the fill kernel's launch; the
// inclusive prefix is still in LDS, so each ticket finds its signal there by
// binary search.
__global__ void __launch_bounds__(kScanThreads)
worktable_scan_kernel(int B, int kmax, int64_t rows, int64_t C, int64_t total_samples,
                      int64_t max_groups,
                      const int32_t *Ks, const int32_t *sec_off, const int64_t *sig_off,
                      int64_t *gpre, int64_t *total_dev, unsigned *ctrl,
                      const unsigned *stage_src, unsigned *stage_dst, int64_t stage_words,
                      int fuse, int32_t *sigmap, const float *zi, float *zf, unsigned *sig_err)
{
    __shared__ int64_t part[kScanThreads];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (stage_src) {
        // 8-byte words, four per thread in flight: a full step's arguments
        // (32 KB at 1024 chunks) cost one round trip to host memory, not eight
        const uint2 *src8 = reinterpret_cast<const uint2 *>(stage_src);
        uint2 *dst8 = reinterpret_cast<uint2 *>(stage_dst);
        const int64_t n8 = stage_words / 2;
        for (int64_t base = 0; base < n8; base += 4 * kScanThreads) {
            uint2 v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t w = base + r * kScanThreads + tid;
                if (w < n8) v[r] = src8[w];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t w = base + r * kScanThreads + tid;
                if (w < n8) dst8[w] = v[r];
            }
        }
        if ((stage_words & 1) && tid == 0) stage_dst[stage_words - 1] = stage_src[stage_words - 1];
        if (tid == 0) {
            ctrl[CTRL_TICKET] = 0u;
            ctrl[CTRL_DONE] = 0u;
            const unsigned e = ctrl[CTRL_EPOCH] + 1u;
            ctrl[CTRL_EPOCH] = (e == 0u) ? 1u : e;
        }
        __threadfence_block();
    }
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < B; base += kScanThreads) {
        const int i = base + tid;
        int64_t gi = 0;
        if (i < B) {
            const bool ok = signal_ok(i, kmax, rows, total_samples, Ks, sec_off, sig_off);
            if (ok) {
                const int64_t n = sig_off[i + 1] - sig_off[i];
                gi = (n + C - 1) / C;
            } else {
                atomicOr(&ctrl[CTRL_ERR], ERRBIT_BADARG);
            }
            // this launch's per-signal error words start here (the filter adds
            // its lookback timeouts)
            if (sig_err) sig_err[i] = ok ? 0u : ERRBIT_BADARG;
        }
        part[tid] = gi;
        __syncthreads();
        // Hillis-Steele inclusive scan over the block
        for (int d = 1; d < kScanThreads; d <<= 1) {
            const int64_t v = tid >= d ? part[tid - d] : 0;
            __syncthreads();
            part[tid] += v;
            __syncthreads();
        }
        if (i < B) gpre[i] = carry + part[tid] - gi;
        __syncthreads();
        if (tid == kScanThreads - 1) carry += part[tid];
        __syncthreads();
    }
    if (tid == 0) {
        int64_t tot = carry;
        if (tot > max_groups) {          // cannot happen when total_samples is honest
            atomicOr(&ctrl[CTRL_ERR], ERRBIT_BADARG);
            tot = 0;
        }
        gpre[B] = tot;
        *total_dev = tot;
    }
    if (!fuse) return;
    // single scan round: part[i] is the inclusive prefix of signal i's groups
    const int64_t tot = carry > max_groups ? 0 : carry;   // 0: the table was rejected
    for (int64_t t = tid; t < tot; t += kScanThreads) {
        int lo = 0, hi = B - 1;                            // first i with part[i] > t
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (part[mid] > t) hi = mid; else lo = mid + 1;
        }
        sigmap[t] = lo;
    }
    if (zf && tid < B && sig_off[tid + 1] == sig_off[tid] &&
        signal_ok(tid, kmax, rows, total_samples, Ks, sec_off, sig_off))
        empty_signal_state(tid, Ks, sec_off, zi, zf, 0, 1);
}

// Block i: sigmap for the tickets of signal i; zf := zi for empty signals
// (consistent ones only: an inconsistent sec_off must not address zf).
__global__ void __launch_bounds__(256)
worktable_fill_kernel(int B, int kmax, int64_t rows, int64_t total_samples, const int64_t *gpre,
                      const int64_t *total_dev, int32_t *sigmap, const int32_t *Ks,
                      const int32_t *sec_off, const int64_t *sig_off, const float *zi, float *zf)
{
    const int i = blockIdx.x;
    if (i >= B) return;
    const int64_t a = gpre[i], b = gpre[i + 1];
    if (*total_dev == 0 && b > a) return;   // the table was rejected as a whole
    for (int64_t t = a + threadIdx.x; t < b; t += blockDim.x) sigmap[t] = i;
    if (zf && a == b && sig_off[i + 1] == sig_off[i] &&
        signal_ok(i, kmax, rows, total_samples, Ks, sec_off, sig_off))
        empty_signal_state(i, Ks, sec_off, zi, zf, threadIdx.x, blockDim.x);
}

}  // namespace

static hipError_t launch_worktable(int B, int kmax, int64_t rows, int64_t C,
                                   int64_t total_samples, int64_t max_groups, const int32_t *Ks,
                                   const int32_t *sec_off, const int64_t *sig_off, int64_t *gpre,
                                   int32_t *sigmap, int64_t *total_dev, const float *zi,
                                   float *zf, unsigned *ctrl, const void *stage_src,
                                   void *stage_dst, int64_t stage_bytes, unsigned *sig_err,
                                   hipStream_t stream)
{
    // one kernel when the scan takes one round and the ticket map is short
    // (at most four binary searches per thread)
    const int fuse = B <= kScanThreads && max_groups <= 4 * (int64_t)kScanThreads;
    hipLaunchKernelGGL(worktable_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, B, kmax,
                       rows, C, total_samples, max_groups, Ks, sec_off, sig_off, gpre, total_dev,
                       ctrl, static_cast<const unsigned *>(stage_src),
                       static_cast<unsigned *>(stage_dst), stage_bytes / 4, fuse, sigmap, zi, zf,
                       sig_err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (B > 0 && !fuse)
        hipLaunchKernelGGL(worktable_fill_kernel, dim3(B), dim3(256), 0, stream, B, kmax, rows,
                           total_samples, gpre, total_dev, sigmap, Ks, sec_off, sig_off, zi, zf);
    return hipGetLastError();
}

extern "C" hipError_t sos_launch_worktable(int B, int kmax, int64_t rows, int64_t C,
                                           int64_t total_samples,
                                           int64_t max_groups, const int32_t *Ks,
                                           const int32_t *sec_off, const int64_t *sig_off,
                                           int64_t *gpre, int32_t *sigmap, int64_t *total_dev,
                                           const float *zi, float *zf, unsigned *ctrl,
                                           hipStream_t stream)
{
    return launch_worktable(B, kmax, rows, C, total_samples, max_groups, Ks, sec_off, sig_off,
                            gpre, sigmap, total_dev, zi, zf, ctrl, nullptr, nullptr, 0, nullptr,
                            stream);
}

// The same, first copying stage_bytes (a multiple of 4; both buffers 8-byte
// aligned) from pinned coherent host memory to device memory (where Ks,
// sec_off and sig_off point) and arming the launch that follows.
extern "C" hipError_t sos_launch_worktable_staged(int B, int kmax, int64_t rows, int64_t C,
                                                  int64_t total_samples, int64_t max_groups,
                                                  const int32_t *Ks, const int32_t *sec_off,
                                                  const int64_t *sig_off, int64_t *gpre,
                                                  int32_t *sigmap, int64_t *total_dev,
                                                  const float *zi, float *zf, unsigned *ctrl,
                                                  const void *stage_src, void *stage_dst,
                                                  int64_t stage_bytes, unsigned *sig_err,
                                                  hipStream_t stream)
{
    if (!stage_src || !stage_dst || stage_bytes < 0 || (stage_bytes & 3) ||
        ((reinterpret_cast<uintptr_t>(stage_src) | reinterpret_cast<uintptr_t>(stage_dst)) & 7))
        return hipErrorInvalidValue;
    return launch_worktable(B, kmax, rows, C, total_samples, max_groups, Ks, sec_off, sig_off,
                            gpre, sigmap, total_dev, zi, zf, ctrl, stage_src, stage_dst,
                            stage_bytes, sig_err, stream);
}
