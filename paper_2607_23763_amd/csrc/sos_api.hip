// Host side of the C ABI declared in include/sosfilt.h: handle, workspace,
// argument checks and kernel launches. No exception or abort crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "sos_internal.h"

using namespace sosdev;
using namespace sosint;

namespace {

// Grow a device buffer to hold `need` elements (contents not preserved). The
// previous buffer may still be read by queued work on `stream`: wait first.
template <typename T>
int ensure_buf(T *&p, size_t &cap, size_t need, hipStream_t stream, bool zero = false)
{
    if (need <= cap) return SOS_OK;
    if (p) {
        if (hipStreamSynchronize(stream) != hipSuccess) return SOS_EHIP;
        (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    const size_t c = need + need / 4 + 64;
    if (hipMalloc(&p, c * sizeof(T)) != hipSuccess) return SOS_ENOMEM;
    // descriptors: tag 0 never matches a launch epoch, so zeroed words read as
    // "not published"
    if (zero && hipMemset(p, 0, c * sizeof(T)) != hipSuccess) return SOS_EHIP;
    cap = c;
    return SOS_OK;
}

int ensure_desc(sos_ctx *h, size_t words, hipStream_t stream)
{
    return ensure_buf(h->desc, h->desc_cap, words, stream, true);
}

size_t tab_bytes(int sections, int bits)
{
    (void)bits;   // one layout for both compute types
    return (size_t)sections * TAB_BYTES;
}

int check_signal(const float *x, const float *y, int64_t n)
{
    if (n < 0) return SOS_EINVAL;
    if (n > 0 && (!x || !y)) return SOS_EINVAL;
    if (n > 0 && x != y) {
        // in place or disjoint only
        const uintptr_t xa = (uintptr_t)x, ya = (uintptr_t)y, bytes = (uintptr_t)n * 4u;
        if (xa < ya + bytes && ya < xa + bytes) return SOS_EINVAL;
    }
    return SOS_OK;
}

// Shortest signal a plain launch of `solver` filters by the whole-cascade path
// for K sections.
int64_t toep_min_n(int solver, int K)
{
    return solver == SOS_ALG_TOEPLITZ ? 1 : toep_auto_min_n(K);
}

// Tables for `sections` at the handle's shape (or, without one, the shape for
// a signal of n samples; n < 0: unknown) and type (caller holds the lock).
int prepare_locked(sos_ctx *h, const float *sections, int K, hipStream_t stream, int64_t n = -1,
                   bool plain = true)
{
    const Tile t = tile_for_length(h, K, n);
    const int bits = bits_of(h);
    int rc = ensure_buf(h->tabs, h->tabs_cap, tab_bytes(K > 8 ? K : 8, bits), stream);
    if (rc) return rc;
    const double rho_max = rho_max_of(h);
    if (sos_launch_prep(bits, sections, K, __builtin_ctz((unsigned)t.N),
                        __builtin_ctz((unsigned)(t.L / 64)), h->tabs, h->ctrl, 0, rho_max,
                        stream) != hipSuccess)
        return SOS_EHIP;
    h->prep_K = K;
    h->prep_alg = solver_of(h);
    h->prep_rho = rho_max;
    h->prep_L = t.L;
    h->prep_N = t.N;
    h->prep_bits = bits;
    h->prep_toep = false;
    // the whole-cascade tables, when a plain launch may take that path; the
    // preparation decides on the device whether it does (gate word)
    const int s = h->prep_alg;
    if (plain && bits == 32 && K >= 1 && K <= kToepMaxK &&
        (s == SOS_ALG_TOEPLITZ || (s == SOS_ALG_AUTO && toep_auto_min_n(K) != INT64_MAX)) &&
        (n < 0 || n >= toep_min_n(s, K))) {
        rc = ensure_buf(h->ttab, h->ttab_cap, (size_t)sos_toep_table_floats(), stream);
        if (rc) return rc;
        const int ng = toep_chunk_groups(n);
        if (sos_launch_toep_prep(sections, K, ng, s == SOS_ALG_TOEPLITZ ? HUGE_VAL : kToepRhoMax,
                                 h->ttab, stream) != hipSuccess)
            return SOS_EHIP;
        h->prep_toep = true;
        h->toep_ng = ng;
    }
    return SOS_OK;
}

// Whether work enqueued on `stream` is being captured into a graph (a failed
// query counts as capturing).
bool capturing(hipStream_t stream)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return st != hipStreamCaptureStatusNone;
}

// Filter with the prepared tables (caller holds the lock).
int filter_locked(sos_ctx *h, const float *x, float *y, int64_t n, const float *zi, float *zf,
                  hipStream_t stream, float *saved)
{
    const int K = h->prep_K;
    if (n == 0) {
        if (zf && K > 0 && sos_launch_fill(zf, zi, 2 * (int64_t)K, stream) != hipSuccess)
            return SOS_EHIP;
        return SOS_OK;
    }
    if (K == 0) {
        if (x != y && sos_launch_fill(y, x, n, stream) != hipSuccess) return SOS_EHIP;
        return SOS_OK;
    }
    const int L = h->prep_L, N = h->prep_N, bits = h->prep_bits;
    const int64_t C = (int64_t)L * N;
    const int64_t groups = (n + C - 1) / C;
    if (groups >= (int64_t)1 << 31) return SOS_EINVAL;
    // the whole-cascade kernel first when its tables are there: it filters
    // the signal unless the preparation's gate sent it to the per-section
    // kernels, which then skip it (and otherwise filter it as before)
    const bool toep = h->prep_toep && !saved && n >= toep_min_n(h->prep_alg, K);
    const int64_t tchunk = (int64_t)sos_toep_group_samples() * h->toep_ng;
    const int64_t tchunks = toep ? (n + tchunk - 1) / tchunk : 0;
    size_t words = (size_t)groups * (size_t)K * 4u;
    if (toep) words = std::max(words, (size_t)tchunks * (size_t)sos_toep_desc_words());
    const int rc = ensure_desc(h, words, stream);
    if (rc) return rc;
    // Ticket 0 and a fresh epoch: left by the previous plain or adjoint launch
    // on this workspace (their last workgroup re-arms) or by its creation,
    // else armed here. A launch being captured into a graph carries its own
    // arm step, so that every replay is self-contained.
    const bool cap = capturing(stream);
    if ((!h->armed || cap || h->batch_captured) && sos_launch_arm(h->ctrl, stream) != hipSuccess)
        return SOS_EHIP;
    if (toep) {
        const int64_t g = grid_override();
        if (sos_launch_toep(x, y, n, h->ttab, K, h->toep_ng, zi, zf, h->desc, h->ctrl,
                            h->timeout_ticks, g ? g : sos_toep_capacity(), stream) != hipSuccess)
            return SOS_EHIP;
    }
    const int alg = launch_alg(bits, h->prep_alg, h->prep_rho);
    if (sos_launch_fwd(bits, alg, L, N, x, y, n, groups, h->tabs, K, zi, zf, h->desc, h->ctrl,
                       h->timeout_ticks, grid_of(bits, alg, L, N), saved,
                       toep ? h->ttab : nullptr, stream) != hipSuccess)
        return SOS_EHIP;
    h->last_groups = groups;
    h->last_K = K;
    if (!cap) h->armed = true;
    return SOS_OK;
}

// Lookback wait bound: ms milliseconds of the device wall clock, at least one
// tick.
void set_timeout_ms(sos_ctx *h, double ms)
{
    const double t = ms * (double)h->wall_khz;
    h->timeout_ticks = t < 1.0 ? 1ull : (unsigned long long)t;
}

void mark_degenerate(sos_ctx *h, int K)
{
    const Tile t = tile_of(h, K);   // degenerate calls need no tables
    h->prep_K = K;
    h->prep_L = t.L;
    h->prep_N = t.N;
    h->prep_bits = bits_of(h);
    h->prep_alg = solver_of(h);
    h->prep_rho = rho_max_of(h);
    h->prep_toep = false;
}

}  // namespace

namespace sosint {

int batch_check(const BatchArgs &ba)
{
    if (ba.B < 0 || ba.kmax < 0 || ba.kmax > SOS_MAX_SECTIONS || ba.total_samples < 0 ||
        ba.total_rows < 0)
        return SOS_EINVAL;
    if (ba.B == 0) return SOS_OK;
    if (!ba.K || !ba.sec_off || !ba.sig_off) return SOS_EINVAL;
    if (ba.total_rows > 0 && !ba.sections) return SOS_EINVAL;
    return check_signal(ba.x, ba.y, ba.total_samples);
}

int batch_reserve(sos_ctx *h, Tile t, int bits, const BatchArgs &ba, hipStream_t stream)
{
    const int64_t C = (int64_t)t.L * t.N;
    const int64_t max_groups = ba.total_samples / C + ba.B;
    if (max_groups >= (int64_t)1 << 31 || ba.total_rows >= (int64_t)1 << 31) return SOS_EINVAL;
    const int kd = ba.kmax > 0 ? ba.kmax : 1;   // descriptor stride
    int rc = ensure_buf(h->tabs, h->tabs_cap,
                        tab_bytes((int)(ba.total_rows > 8 ? ba.total_rows : 8), bits), stream);
    if (rc) return rc;
    rc = ensure_desc(h, (size_t)max_groups * (size_t)kd * 4u, stream);
    if (rc) return rc;
    rc = ensure_buf(h->gpre, h->gpre_cap, (size_t)ba.B + 1, stream);
    if (rc) return rc;
    rc = ensure_buf(h->sigmap, h->sigmap_cap, (size_t)max_groups, stream);
    if (rc) return rc;
    if (!h->total_dev && hipMalloc(&h->total_dev, sizeof(int64_t)) != hipSuccess)
        return SOS_ENOMEM;
    return SOS_OK;
}

int batch_enqueue(sos_ctx *h, Tile t, int bits, const BatchArgs &ba, hipStream_t stream)
{
    h->armed = false;   // a batched launch leaves the ticket counter advanced
    if (capturing(stream)) h->batch_captured = true;
    const int64_t C = (int64_t)t.L * t.N;
    const int64_t max_groups = ba.total_samples / C + ba.B;
    const int kd = ba.kmax > 0 ? ba.kmax : 1;
    const int log2n = __builtin_ctz((unsigned)t.N), log2w = __builtin_ctz((unsigned)(t.L / 64));
    if (ba.total_rows > 0 &&
        sos_launch_prep_batched(bits, ba.sections, ba.B, ba.kmax, ba.total_rows, ba.K,
                                ba.sec_off, log2n, log2w, h->tabs, h->ctrl, 0, rho_max_of(h),
                                stream) != hipSuccess)
        return SOS_EHIP;
    if (sos_launch_worktable(ba.B, ba.kmax, ba.total_rows, C, ba.total_samples, max_groups, ba.K,
                             ba.sec_off, ba.sig_off, h->gpre, h->sigmap, h->total_dev, ba.zi,
                             ba.zf, h->ctrl, stream) != hipSuccess)
        return SOS_EHIP;
    if (sos_launch_arm(h->ctrl, stream) != hipSuccess) return SOS_EHIP;
    const int alg = launch_alg(bits, solver_of(h), rho_max_of(h));
    int64_t grid = grid_of(bits, alg, t.L, t.N);
    if (grid <= 0 || grid > max_groups) grid = max_groups;
    if (sos_launch_fwd_batched(bits, alg, t.L, t.N, ba.B, kd, ba.K, ba.sec_off, ba.sig_off, h->gpre,
                               h->sigmap, h->total_dev, ba.x, ba.y, h->tabs, ba.zi, ba.zf,
                               h->desc, h->ctrl, h->timeout_ticks, grid, nullptr, nullptr,
                               ba.saved, ba.total_samples, max_groups, nullptr,
                               stream) != hipSuccess)
        return SOS_EHIP;
    h->prep_K = -1;        // the batch overwrote the plain tables
    h->last_groups = 0;
    h->last_K = 0;
    return SOS_OK;
}

}  // namespace sosint

extern "C" {

const char *sos_strerror(int code)
{
    switch (code) {
    case SOS_OK: return "ok";
    case SOS_EINVAL: return "invalid argument";
    case SOS_EA0: return "a section has a0 == 0";
    case SOS_EUNSTABLE: return "a section is outside the stability triangle";
    case SOS_ENOMEM: return "device allocation failed";
    case SOS_EHIP: return "HIP runtime error";
    case SOS_ETIMEOUT: return "lookback wait timed out";
    case SOS_ECLOSED: return "closed";
    case SOS_EBUSY: return "busy";
    case SOS_ELIMIT: return "beyond the fixed workspace of the no-allocation entry point";
    default: return "unknown status";
    }
}

int sos_create(sos_handle_t *out, int hip_device)
{
    if (!out) return SOS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
        return SOS_EINVAL;
    DeviceGuard g(hip_device);
    if (!g.ok) return SOS_EHIP;
    sos_ctx *h = new (std::nothrow) sos_ctx();
    if (!h) return SOS_ENOMEM;
    h->device = hip_device;
    if (hipMalloc(&h->ctrl, sizeof(unsigned) * CTRL_WORDS) != hipSuccess) {
        delete h;
        return SOS_ENOMEM;
    }
    unsigned init[CTRL_WORDS] = {};
    init[CTRL_EPOCH] = 1u;   // descriptor tag 0 is reserved for "never written"
    if (hipMemcpy(h->ctrl, init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(h->ctrl);
        delete h;
        return SOS_EHIP;
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, hip_device) != hipSuccess ||
        khz <= 0)
        khz = 100000;
    h->wall_khz = khz;
    double ms = 2000.0;
    if (const char *e = std::getenv("SOS_TIMEOUT_MS")) ms = std::atof(e);
    set_timeout_ms(h, ms);
    *out = h;
    return SOS_OK;
}

int sos_set_timeout(sos_handle_t h, double ms)
{
    if (!h || !(ms >= 0.0) || ms > 3.6e6) return SOS_EINVAL;
    set_timeout_ms(h, ms == 0.0 ? 2000.0 : ms);
    return SOS_OK;
}

int sos_wall_clock_khz(sos_handle_t h)
{
    if (!h) return SOS_EINVAL;
    return h->wall_khz;
}

int sos_destroy(sos_handle_t h)
{
    if (!h) return SOS_EINVAL;
    {
        DeviceGuard g(h->device);
        (void)hipDeviceSynchronize();
        for (void *p : {(void *)h->desc, (void *)h->tabs, (void *)h->ctrl, (void *)h->gpre,
                        (void *)h->sigmap, (void *)h->total_dev, (void *)h->tabs_bwd,
                        (void *)h->partials, (void *)h->grow, (void *)h->ttab})
            if (p) (void)hipFree(p);
    }
    delete h;
    return SOS_OK;
}

int sos_last_error(sos_handle_t h)
{
    if (!h) return SOS_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    if (hipDeviceSynchronize() != hipSuccess) return SOS_EHIP;
    unsigned bits = 0;
    if (hipMemcpy(&bits, h->ctrl + CTRL_ERR, sizeof(unsigned), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return SOS_EHIP;
    if (bits && hipMemset(h->ctrl + CTRL_ERR, 0, sizeof(unsigned)) != hipSuccess) return SOS_EHIP;
    if (bits & ERRBIT_A0) return SOS_EA0;
    if (bits & ERRBIT_UNSTABLE) return SOS_EUNSTABLE;
    if (bits & ERRBIT_TIMEOUT) return SOS_ETIMEOUT;
    if (bits & ERRBIT_BADARG) return SOS_EINVAL;
    return SOS_OK;
}

int sos_set_tile(sos_handle_t h, int L, int N)
{
    if (!h) return SOS_EINVAL;
    if (L == 0 && N == 0) {
        h->tile_L = h->tile_N = 0;
        return SOS_OK;
    }
    if (!sos_fwd_shape_supported(L, N)) return SOS_EINVAL;
    h->tile_L = L;
    h->tile_N = N;
    return SOS_OK;
}

int sos_get_tile(sos_handle_t h, int *L, int *N)
{
    if (!h) return SOS_EINVAL;
    const Tile t = tile_of(h);
    if (L) *L = t.L;
    if (N) *N = t.N;
    return SOS_OK;
}

int sos_set_precision(sos_handle_t h, int bits)
{
    if (!h || (bits != 0 && bits != 32 && bits != 64)) return SOS_EINVAL;
    h->bits = bits;
    return SOS_OK;
}

int sos_get_precision(sos_handle_t h)
{
    if (!h) return SOS_EINVAL;
    return bits_of(h);
}

int sos_set_algorithm(sos_handle_t h, int alg)
{
    if (!h || (alg != SOS_ALG_DEFAULT && alg != SOS_ALG_DCCR && alg != SOS_ALG_PH &&
               alg != SOS_ALG_AUTO && alg != SOS_ALG_TOEPLITZ))
        return SOS_EINVAL;
    h->alg = alg;
    return SOS_OK;
}

int sos_get_algorithm(sos_handle_t h)
{
    if (!h) return SOS_EINVAL;
    return solver_of(h);
}

int sos_prepare(sos_handle_t h, const float *sections, int K, hipStream_t stream)
{
    if (!h || K < 0 || K > SOS_MAX_SECTIONS) return SOS_EINVAL;
    if (K > 0 && !sections) return SOS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    return prepare_locked(h, sections, K, stream);
}

int sos_filter_prepared(sos_handle_t h, const float *x, float *y, int64_t n, const float *zi,
                        float *zf, hipStream_t stream)
{
    if (!h) return SOS_EINVAL;
    int rc = check_signal(x, y, n);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(h->mu);
    // Without a tile set, whatever shape the tables were prepared at is valid
    // (sos_filter picks it from the signal length).
    const Tile t = tile_of(h, h->prep_K);
    if (h->prep_K < 0 || h->prep_bits != bits_of(h) || h->prep_alg != solver_of(h) ||
        (tile_is_set(h) && (h->prep_N != t.N || h->prep_L != t.L)))
        return SOS_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    return filter_locked(h, x, y, n, zi, zf, stream, nullptr);
}

int sos_filter(sos_handle_t h, const float *sections, int K, const float *x, float *y, int64_t n,
               const float *zi, float *zf, hipStream_t stream)
{
    if (!h || K < 0 || K > SOS_MAX_SECTIONS) return SOS_EINVAL;
    if (K > 0 && !sections) return SOS_EINVAL;
    int rc = check_signal(x, y, n);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    if (n > 0 && K > 0) {
        rc = prepare_locked(h, sections, K, stream, n);
        if (rc) return rc;
    } else {
        mark_degenerate(h, K);
    }
    return filter_locked(h, x, y, n, zi, zf, stream, nullptr);
}

int sos_filter_batched(sos_handle_t h, int B, int kmax, int64_t total_rows,
                       int64_t total_samples, const int32_t *K, const int32_t *sec_off,
                       const float *sections, const int64_t *sig_off, const float *x, float *y,
                       const float *zi, float *zf, hipStream_t stream)
{
    if (!h) return SOS_EINVAL;
    BatchArgs ba{B, kmax, total_rows, total_samples, K, sec_off, sections, sig_off, x, y, zi, zf};
    int rc = batch_check(ba);
    if (rc || B == 0) return rc;
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    const Tile t = tile_of(h, kmax);
    const int bits = bits_of(h);
    rc = batch_reserve(h, t, bits, ba, stream);
    if (rc) return rc;
    return batch_enqueue(h, t, bits, ba, stream);
}

int sos_filter_train(sos_handle_t h, const float *sections, int K, const float *x, float *y,
                     int64_t n, const float *zi, float *zf, float *saved, hipStream_t stream)
{
    if (!h || K < 0 || K > SOS_MAX_SECTIONS) return SOS_EINVAL;
    if (K > 0 && !sections) return SOS_EINVAL;
    if (K > 1 && n > 0 && !saved) return SOS_EINVAL;
    if (n > 0 && x == y) return SOS_EINVAL;   // the adjoint needs the forward input
    int rc = check_signal(x, y, n);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    if (n > 0 && K > 0) {
        rc = prepare_locked(h, sections, K, stream, n, false);
        if (rc) return rc;
    } else {
        mark_degenerate(h, K);
    }
    return filter_locked(h, x, y, n, zi, zf, stream, K > 1 ? saved : nullptr);
}

int sos_filter_vjp(sos_handle_t h, const float *sections, int K, const float *x, const float *y,
                   const float *saved, int64_t n, const float *gy, const float *gzf, float *gx,
                   float *gzi, float *gsections, hipStream_t stream)
{
    if (!h || K < 0 || K > SOS_MAX_SECTIONS || n < 0) return SOS_EINVAL;
    if (K > 0 && !sections) return SOS_EINVAL;
    if (n > 0 && (!x || !y || !gy || !gx)) return SOS_EINVAL;
    if (K > 1 && n > 0 && !saved) return SOS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    if (K == 0) {
        if (n > 0 && gx != gy && sos_launch_fill(gx, gy, n, stream) != hipSuccess)
            return SOS_EHIP;
        return SOS_OK;
    }
    if (n == 0) {
        // zf = zi: the adjoint of zi is gzf; no samples, no coefficient gradient
        if (gzi && sos_launch_fill(gzi, gzf, 2 * (int64_t)K, stream) != hipSuccess) return SOS_EHIP;
        if (gsections && sos_launch_fill(gsections, nullptr, 6 * (int64_t)K, stream) != hipSuccess)
            return SOS_EHIP;
        return SOS_OK;
    }
    Tile t = tile_of(h);
    if (!sos_bwd_shape_supported(t.L, t.N)) t = Tile{512, 32};   // fastest adjoint shape measured
    const int bits = bits_of(h);
    const int64_t C = (int64_t)t.L * t.N;
    const int64_t groups = (n + C - 1) / C;
    if (groups >= (int64_t)1 << 31) return SOS_EINVAL;
    int rc = ensure_buf(h->tabs_bwd, h->tabs_bwd_cap, tab_bytes(K, bits), stream);
    if (rc) return rc;
    rc = ensure_buf(h->partials, h->partials_cap, (size_t)groups * K * 5, stream);
    if (rc) return rc;
    rc = ensure_desc(h, (size_t)groups * (size_t)K * 4u, stream);
    if (rc) return rc;
    if (sos_launch_prep(bits, sections, K, __builtin_ctz((unsigned)t.N),
                        __builtin_ctz((unsigned)(t.L / 64)), h->tabs_bwd, h->ctrl, 1,
                        rho_max_of(h), stream) != hipSuccess)
        return SOS_EHIP;
    if (sos_launch_arm(h->ctrl, stream) != hipSuccess) return SOS_EHIP;
    if (sos_launch_bwd(bits, launch_alg(bits, solver_of(h), rho_max_of(h)), t.L, t.N, gy, gx, n, groups,
                       h->tabs_bwd, K, x, y, saved,
                       gzf, gzi, h->partials, h->desc, h->ctrl, h->timeout_ticks, grid_override(),
                       stream) != hipSuccess)
        return SOS_EHIP;
    if (gsections &&
        sos_launch_bwd_reduce(h->partials, groups, K, sections, gsections, stream) != hipSuccess)
        return SOS_EHIP;
    h->last_groups = 0;
    h->last_K = 0;
    return SOS_OK;
}

int sos_filter_train_batched(sos_handle_t h, int B, int kmax, int64_t total_rows,
                             int64_t total_samples, const int32_t *K, const int32_t *sec_off,
                             const float *sections, const int64_t *sig_off, const float *x,
                             float *y, const float *zi, float *zf, float *saved,
                             hipStream_t stream)
{
    if (!h) return SOS_EINVAL;
    BatchArgs ba{B, kmax, total_rows, total_samples, K, sec_off, sections, sig_off, x, y, zi, zf};
    int rc = batch_check(ba);
    if (rc || B == 0) return rc;
    if (total_samples > 0 && x == y) return SOS_EINVAL;   // the adjoint needs the input
    if (kmax > 1 && total_samples > 0 && !saved) return SOS_EINVAL;
    ba.saved = kmax > 1 ? saved : nullptr;
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    const Tile t = tile_of(h, kmax);
    const int bits = bits_of(h);
    rc = batch_reserve(h, t, bits, ba, stream);
    if (rc) return rc;
    return batch_enqueue(h, t, bits, ba, stream);
}

namespace {

// The batched adjoint; coefficient gradients per signal row (gsections) or,
// for a shared cascade, summed over the signals (gsum, kmax x 6).
int vjp_batched(sos_handle_t h, int B, int kmax, int64_t total_rows, int64_t total_samples,
                const int32_t *K, const int32_t *sec_off, const float *sections,
                const int64_t *sig_off, const float *x, const float *y, const float *saved,
                const float *gy, const float *gzf, float *gx, float *gzi, float *gsections,
                float *gsum, hipStream_t stream)
{
    if (!h || B < 0 || kmax < 0 || kmax > SOS_MAX_SECTIONS || total_samples < 0 ||
        total_rows < 0)
        return SOS_EINVAL;
    if (B == 0) return SOS_OK;
    if (!K || !sec_off || !sig_off || (total_rows > 0 && !sections)) return SOS_EINVAL;
    if (total_samples > 0 && (!x || !y || !gy || !gx)) return SOS_EINVAL;
    if (kmax > 1 && total_samples > 0 && !saved) return SOS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    Tile t = tile_of(h, kmax);
    if (!sos_bwd_shape_supported(t.L, t.N)) t = Tile{512, 32};   // fastest adjoint shape measured
    const int bits = bits_of(h);
    const int64_t C = (int64_t)t.L * t.N;
    const int64_t max_groups = total_samples / C + B;
    if (max_groups >= (int64_t)1 << 31 || total_rows >= (int64_t)1 << 31) return SOS_EINVAL;
    const int kd = kmax > 0 ? kmax : 1;
    int rc = ensure_buf(h->tabs_bwd, h->tabs_bwd_cap,
                        tab_bytes((int)(total_rows > 1 ? total_rows : 1), bits), stream);
    if (rc) return rc;
    rc = ensure_buf(h->partials, h->partials_cap, (size_t)max_groups * kd * 5, stream);
    if (rc) return rc;
    rc = ensure_desc(h, (size_t)max_groups * (size_t)kd * 4u, stream);
    if (rc) return rc;
    rc = ensure_buf(h->gpre, h->gpre_cap, (size_t)B + 1, stream);
    if (rc) return rc;
    rc = ensure_buf(h->sigmap, h->sigmap_cap, (size_t)max_groups, stream);
    if (rc) return rc;
    if (!h->total_dev && hipMalloc(&h->total_dev, sizeof(int64_t)) != hipSuccess)
        return SOS_ENOMEM;
    const int log2n = __builtin_ctz((unsigned)t.N), log2w = __builtin_ctz((unsigned)(t.L / 64));
    if (total_rows > 0 &&
        sos_launch_prep_batched(bits, sections, B, kmax, total_rows, K, sec_off, log2n, log2w,
                                h->tabs_bwd, h->ctrl, 1, rho_max_of(h), stream) != hipSuccess)
        return SOS_EHIP;
    // work table over the adjoint's groups; an empty signal gets gzi = gzf
    if (sos_launch_worktable(B, kmax, total_rows, C, total_samples, max_groups, K, sec_off,
                             sig_off, h->gpre, h->sigmap, h->total_dev, gzf, gzi, h->ctrl,
                             stream) != hipSuccess)
        return SOS_EHIP;
    if (sos_launch_arm(h->ctrl, stream) != hipSuccess) return SOS_EHIP;
    if (sos_launch_bwd_batched(bits, launch_alg(bits, solver_of(h), rho_max_of(h)), t.L, t.N, B, kd, K, sec_off,
                               sig_off, h->gpre,
                               h->sigmap, h->total_dev, max_groups, gy, gx, h->tabs_bwd, x, y, saved,
                               total_samples, gzf, gzi, h->partials, h->desc, h->ctrl,
                               h->timeout_ticks, stream) != hipSuccess)
        return SOS_EHIP;
    if (gsum) {
        rc = ensure_buf(h->grow, h->grow_cap, (size_t)B * kd * 6, stream);
        if (rc) return rc;
    }
    if ((gsections || gsum) &&
        sos_launch_bwd_reduce_batched(h->partials, B, kmax, total_rows, total_samples, K,
                                      sec_off, sig_off, h->gpre, sections, gsections,
                                      gsum ? h->grow : nullptr, gsum, stream) != hipSuccess)
        return SOS_EHIP;
    h->prep_K = -1;
    h->last_groups = 0;
    h->last_K = 0;
    return SOS_OK;
}

}  // namespace

int sos_filter_vjp_batched(sos_handle_t h, int B, int kmax, int64_t total_rows,
                           int64_t total_samples, const int32_t *K, const int32_t *sec_off,
                           const float *sections, const int64_t *sig_off, const float *x,
                           const float *y, const float *saved, const float *gy,
                           const float *gzf, float *gx, float *gzi, float *gsections,
                           hipStream_t stream)
{
    return vjp_batched(h, B, kmax, total_rows, total_samples, K, sec_off, sections, sig_off, x, y,
                       saved, gy, gzf, gx, gzi, gsections, nullptr, stream);
}

int sos_filter_vjp_batched_sum(sos_handle_t h, int B, int kmax, int64_t total_rows,
                               int64_t total_samples, const int32_t *K, const int32_t *sec_off,
                               const float *sections, const int64_t *sig_off, const float *x,
                               const float *y, const float *saved, const float *gy,
                               const float *gzf, float *gx, float *gzi, float *gsum,
                               hipStream_t stream)
{
    if (!gsum) return SOS_EINVAL;
    return vjp_batched(h, B, kmax, total_rows, total_samples, K, sec_off, sections, sig_off, x, y,
                       saved, gy, gzf, gx, gzi, nullptr, gsum, stream);
}

int sos_bench_copy(const float *x, float *y, int64_t n, hipStream_t stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) return SOS_EINVAL;
    return sos_launch_copy(x, y, n, stream) == hipSuccess ? SOS_OK : SOS_EHIP;
}

int sos_debug_carries(sos_handle_t h, float *out, int64_t capacity_floats, int64_t *groups,
                      int *K)
{
    if (!h) return SOS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    if (groups) *groups = h->last_groups;
    if (K) *K = h->last_K;
    if (!out) return SOS_OK;
    const int64_t need = h->last_groups * h->last_K * 2;
    if (need == 0 || capacity_floats < need) return SOS_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return SOS_EHIP;
    if (hipDeviceSynchronize() != hipSuccess) return SOS_EHIP;
    std::vector<unsigned long long> w((size_t)need * 2);
    if (hipMemcpy(w.data(), h->desc, w.size() * sizeof(unsigned long long),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return SOS_EHIP;
    // descriptors are section-major: section s of group g at (s * groups + g) * 4
    const int64_t G = h->last_groups;
    for (int64_t g = 0; g < G; ++g)
        for (int s = 0; s < h->last_K; ++s) {
            const size_t wi = ((size_t)s * G + g) * 4;
            const uint32_t v1 = (uint32_t)(w[wi + 2] & 0xffffffffu);
            const uint32_t v2 = (uint32_t)(w[wi + 3] & 0xffffffffu);
            std::memcpy(out + 2 * (g * h->last_K + s), &v1, 4);
            std::memcpy(out + 2 * (g * h->last_K + s) + 1, &v2, 4);
        }
    return SOS_OK;
}

}  // extern "C"
