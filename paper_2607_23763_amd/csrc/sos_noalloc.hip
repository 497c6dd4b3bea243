// The plain filter without any allocation (sos_filter_noalloc): the same
// preparation and filter kernels as sos_filter, with their workspace (the
// control words, the coefficient tables and the lookback descriptors) in one
// file-scope device array instead of a handle's allocations.
//
// The array is a device symbol: host code never uses its name as an address.
// The first call on a device takes the array's device address there with
// hipGetSymbolAddress (once per device, that device current) and every later
// call uses that address. All calls on one device share the array, which
// keeps the last call's contents; calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "sos_internal.h"

using namespace sosdev;
using namespace sosint;

namespace {

// Layout of the scratch array: control words, the tables of up to
// SOS_MAX_SECTIONS sections, then the lookback descriptors (four 64-bit words
// per group and section).
constexpr size_t kNaCtrlBytes = 256;
constexpr size_t kNaTabBytes = (size_t)SOS_MAX_SECTIONS * TAB_BYTES;
constexpr size_t kNaDescWords = (size_t)1 << 21;
constexpr size_t kNaBytes = kNaCtrlBytes + kNaTabBytes + kNaDescWords * 8;
static_assert(kNaCtrlBytes >= CTRL_WORDS * sizeof(unsigned), "control words");
static_assert((kNaCtrlBytes % 256) == 0 && (kNaTabBytes % 256) == 0, "alignment");

// Zero at load: descriptor tag 0 never matches a launch epoch, and every call
// arms the control words itself.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kMaxDevices = 64;
std::mutex g_na_mu;
unsigned char *g_na_ptr[kMaxDevices] = {};
unsigned long long g_na_ticks[kMaxDevices] = {};

// The device address of the array on the current device `dev` (taken once),
// and the lookback wait bound there: 2000 ms of the device wall clock, or
// SOS_TIMEOUT_MS, as for a new handle.
int scratch_of(int dev, unsigned char **out, unsigned long long *ticks)
{
    if (dev < 0 || dev >= kMaxDevices) return SOS_EINVAL;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SOS_EHIP;
        }
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
            khz <= 0)
            khz = 100000;
        double ms = 2000.0;
        if (const char *e = std::getenv("SOS_TIMEOUT_MS")) ms = std::atof(e);
        const double tk = ms * (double)khz;
        g_na_ticks[dev] = tk < 1.0 ? 1ull : (unsigned long long)tk;
        g_na_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_na_ptr[dev];
    *ticks = g_na_ticks[dev];
    return SOS_OK;
}

// Start of a call: ticket 0, no workgroup done, no error bits, a fresh epoch
// (tag 0 is never used). A kernel rather than a memset, so that the call can
// be captured into a graph.
__global__ void noalloc_arm_kernel(unsigned *ctrl)
{
    ctrl[CTRL_TICKET] = 0u;
    ctrl[CTRL_DONE] = 0u;
    ctrl[CTRL_ERR] = 0u;
    const unsigned e = ctrl[CTRL_EPOCH] + 1u;
    ctrl[CTRL_EPOCH] = (e == 0u) ? 1u : e;
}

// The group shape sos_filter takes for an FP32 signal of n samples when no
// tile is set (fewer samples per lane for short signals).
Tile noalloc_tile(int64_t n)
{
    if (n <= ((int64_t)1 << 20)) return Tile{512, 16};
    if (n <= ((int64_t)1 << 22)) return Tile{512, 32};
    return Tile{kDefaultL, kDefaultN};
}

}  // namespace

extern "C" {

int sos_filter_noalloc(const float *sections, int K, const float *x, float *y, int64_t n,
                       const float *zi, float *zf, unsigned *err, hipStream_t stream)
{
    if (K < 0 || K > SOS_MAX_SECTIONS || n < 0) return SOS_EINVAL;
    if (K > 0 && !sections) return SOS_EINVAL;
    if (n > 0 && (!x || !y)) return SOS_EINVAL;
    if (n > 0 && x != y) {
        const uintptr_t xa = (uintptr_t)x, ya = (uintptr_t)y, bytes = (uintptr_t)n * 4u;
        if (xa < ya + bytes && ya < xa + bytes) return SOS_EINVAL;
    }
    const Tile t = noalloc_tile(n);
    const int64_t C = (int64_t)t.L * t.N;
    const int64_t groups = (n + C - 1) / C;
    if (groups * (int64_t)K * 4 > (int64_t)kNaDescWords) return SOS_ELIMIT;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SOS_EHIP;
    unsigned char *base = nullptr;
    unsigned long long ticks = 0;
    int rc = scratch_of(dev, &base, &ticks);
    if (rc) return rc;
    unsigned *ctrl = reinterpret_cast<unsigned *>(base);
    unsigned char *tabs = base + kNaCtrlBytes;
    unsigned long long *desc =
        reinterpret_cast<unsigned long long *>(base + kNaCtrlBytes + kNaTabBytes);

    hipLaunchKernelGGL(noalloc_arm_kernel, dim3(1), dim3(1), 0, stream, ctrl);
    if (hipGetLastError() != hipSuccess) return SOS_EHIP;
    if (n == 0) {
        if (zf && K > 0 && sos_launch_fill(zf, zi, 2 * (int64_t)K, stream) != hipSuccess)
            return SOS_EHIP;
    } else if (K == 0) {
        if (x != y && sos_launch_fill(y, x, n, stream) != hipSuccess) return SOS_EHIP;
    } else {
        const int bits = 32;
        if (sos_launch_prep(bits, sections, K, __builtin_ctz((unsigned)t.N),
                            __builtin_ctz((unsigned)(t.L / 64)), tabs, ctrl, 0, kAutoRhoMax,
                            stream) != hipSuccess)
            return SOS_EHIP;
        const int alg = launch_alg(bits, SOS_ALG_AUTO, kAutoRhoMax);
        if (sos_launch_fwd(bits, alg, t.L, t.N, x, y, n, groups, tabs, K, zi, zf, desc, ctrl,
                           ticks, grid_of(bits, alg, t.L, t.N), nullptr, nullptr,
                           stream) != hipSuccess)
            return SOS_EHIP;
    }
    if (err && sos_launch_report_err(ctrl + CTRL_ERR, err, nullptr, nullptr, 0, stream) !=
                   hipSuccess)
        return SOS_EHIP;
    return SOS_OK;
}

}  // extern "C"
