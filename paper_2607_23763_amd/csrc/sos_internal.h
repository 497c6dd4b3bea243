// Internal declarations shared by the host-side sources of the library: the
// kernel launchers, the handle structure and its shape/precision helpers.
// Not part of the public ABI (include/sosfilt.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "sosfilt.h"
#include "sos_device.h"

extern "C" {
hipError_t sos_launch_prep(int bits, const float *sections, int K, int log2n, int log2w,
                           void *tabs, unsigned *ctrl, int pair, double rho_max,
                           hipStream_t stream);
hipError_t sos_launch_prep_batched(int bits, const float *sections, int B, int kmax, int64_t rows,
                                   const int32_t *Ks, const int32_t *sec_off, int log2n,
                                   int log2w, void *tabs, unsigned *ctrl, int pair,
                                   double rho_max, hipStream_t stream);
hipError_t sos_launch_arm(unsigned *ctrl, hipStream_t stream);
hipError_t sos_launch_fwd(int bits, int alg, int L, int N, const float *x, float *y, int64_t n,
                          int64_t groups, const void *tabs, int K, const float *zi, float *zf,
                          unsigned long long *desc, unsigned *ctrl,
                          unsigned long long timeout_ticks, int64_t grid, float *saved,
                          const float *skip_gate, hipStream_t stream);
hipError_t sos_launch_toep_prep(const float *sections, int K, int ng, double rho_gate, float *tt,
                                hipStream_t stream);
hipError_t sos_launch_toep(const float *x, float *y, int64_t n, const float *tt, int K, int ng,
                           const float *zi, float *zf, unsigned long long *desc, unsigned *ctrl,
                           unsigned long long timeout_ticks, int64_t grid, hipStream_t stream);
int sos_toep_capacity(void);
int sos_toep_group_samples(void);
int sos_toep_desc_words(void);
int sos_toep_table_floats(void);
hipError_t sos_launch_fwd_batched(int bits, int alg, int L, int N, int B, int kmax,
                                  const int32_t *Ks, const int32_t *sec_off, const int64_t *sig_off,
                                  const int64_t *gpre, const int32_t *sigmap,
                                  const int64_t *total_dev, const float *x, float *y,
                                  const void *tabs, const float *zi, float *zf,
                                  unsigned long long *desc, unsigned *ctrl,
                                  unsigned long long timeout_ticks, int64_t grid,
                                  const float *const *xp, float *const *yp, float *saved,
                                  int64_t saved_stride, int64_t max_groups, unsigned *sig_err,
                                  hipStream_t stream);
hipError_t sos_launch_bwd_batched(int bits, int alg, int L, int N, int B, int kmax,
                                  const int32_t *Ks, const int32_t *sec_off, const int64_t *sig_off,
                                  const int64_t *gpre, const int32_t *sigmap,
                                  const int64_t *total_dev, int64_t max_groups, const float *gy,
                                  float *gx, const void *tabs, const float *x, const float *y,
                                  const float *saved, int64_t saved_stride, const float *gzf,
                                  float *gzi, double *partials, unsigned long long *desc,
                                  unsigned *ctrl, unsigned long long timeout_ticks,
                                  hipStream_t stream);
hipError_t sos_launch_bwd_reduce_batched(const double *partials, int B, int kmax, int64_t rows,
                                         int64_t total_samples, const int32_t *Ks,
                                         const int32_t *sec_off, const int64_t *sig_off,
                                         const int64_t *gpre, const float *sections,
                                         float *gsections, double *grow, float *gsum,
                                         hipStream_t stream);
hipError_t sos_launch_worktable(int B, int kmax, int64_t rows, int64_t C, int64_t total_samples,
                                int64_t max_groups, const int32_t *Ks, const int32_t *sec_off,
                                const int64_t *sig_off, int64_t *gpre, int32_t *sigmap,
                                int64_t *total_dev, const float *zi, float *zf, unsigned *ctrl,
                                hipStream_t stream);
hipError_t sos_launch_worktable_staged(int B, int kmax, int64_t rows, int64_t C,
                                       int64_t total_samples, int64_t max_groups,
                                       const int32_t *Ks, const int32_t *sec_off,
                                       const int64_t *sig_off, int64_t *gpre, int32_t *sigmap,
                                       int64_t *total_dev, const float *zi, float *zf,
                                       unsigned *ctrl, const void *stage_src, void *stage_dst,
                                       int64_t stage_bytes, unsigned *sig_err,
                                       hipStream_t stream);
hipError_t sos_launch_report_err(unsigned *ctrl_err, unsigned *host_err, const unsigned *sig_err,
                                 unsigned *host_sig_err, int B, hipStream_t stream);
hipError_t sos_launch_bwd(int bits, int alg, int L, int N, const float *gy, float *gx, int64_t n,
                          int64_t groups, const void *tabs, int K, const float *x,
                          const float *y, const float *saved, const float *gzf, float *gzi,
                          double *partials, unsigned long long *desc, unsigned *ctrl,
                          unsigned long long timeout_ticks, int64_t grid, hipStream_t stream);
hipError_t sos_launch_bwd_reduce(const double *partials, int64_t groups, int K,
                                 const float *sections, float *gsections, hipStream_t stream);
hipError_t sos_launch_fill(float *dst, const float *src, int64_t count, hipStream_t stream);
hipError_t sos_launch_copy(const float *x, float *y, int64_t n, hipStream_t stream);
int sos_fwd_shape_supported(int L, int N);
int sos_fwd_capacity(int bits, int alg, int L, int N);
int sos_fwd_kernel_attrs(int bits, int alg, int L, int N, int *regs, int *lds);
int sos_bwd_shape_supported(int L, int N);
}

struct sos_ctx {
    int device = 0;
    int tile_L = 0;                       // lanes per group L = 64 W; 0 = default
    int tile_N = 0;                       // samples per lane N; 0 = default
    int bits = 0;                         // compute type: 32, 64; 0 = default
    int alg = 0;                          // section solver: SOS_ALG_*; 0 = default
    unsigned *ctrl = nullptr;             // CTRL_WORDS
    unsigned char *tabs = nullptr;        // coefficient tables (bytes)
    size_t tabs_cap = 0;
    unsigned long long *desc = nullptr;   // lookback descriptors
    size_t desc_cap = 0;                  // 64-bit words
    unsigned long long timeout_ticks = 0;  // lookback wait bound, in wall-clock ticks
    int wall_khz = 0;                     // device wall clock (s_memrealtime) rate
    int64_t last_groups = 0;
    int last_K = 0;
    bool armed = true;   // ctrl holds ticket 0 and an unused epoch once the enqueued
                         // work has run (fresh, or last launch plain or adjoint)
    bool batch_captured = false;   // a batched launch was captured into a graph on
                                   // this handle: its replays advance the ticket
                                   // whenever they run, so plain launches always arm
    int prep_K = -1;                      // tables currently prepared (K, shape, type)
    int prep_L = 0;
    int prep_N = 0;
    int prep_bits = 0;
    int prep_alg = 0;                     // solver the tables were prepared for
    double prep_rho = 0.0;                // and their peak-gain threshold
    bool prep_toep = false;               // block-Toeplitz tables prepared too
    int toep_ng = 0;                      //   for chunks of this many groups
    float *ttab = nullptr;                // block-Toeplitz tables (sos_toep.hip)
    size_t ttab_cap = 0;
    // uneven-batch work table
    int64_t *gpre = nullptr;
    size_t gpre_cap = 0;
    int32_t *sigmap = nullptr;
    size_t sigmap_cap = 0;
    int64_t *total_dev = nullptr;
    // adjoint
    unsigned char *tabs_bwd = nullptr;
    size_t tabs_bwd_cap = 0;
    double *partials = nullptr;
    size_t partials_cap = 0;
    double *grow = nullptr;               // FP64 per-signal coefficient gradients
    size_t grow_cap = 0;                  // (summed over a shared cascade)
    std::mutex mu;
};

namespace sosint {

constexpr int kDefaultL = 512;   // default group shape
constexpr int kDefaultN = 64;
constexpr int kDefaultBits = 32;

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard()
    {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};

struct Tile {
    int L, N;
};

// The handle's tile, else SOS_TILE_L / SOS_TILE_N, else the default
// (L = 512, N = 64): one resident group of 32 K samples per CU, whose next
// group's samples are loaded while it is corrected and stored, beat two
// resident groups of 16 K at every order measured on MI355X (2^28 samples,
// orders 2-16), and 8 waves of N = 64 beat 16 waves of N = 32 (L = 1024) by
// 7-8 % at order 2 and more at higher orders. K is kept for shape choices
// that depend on the cascade.
inline Tile tile_of(const sos_ctx *h, int K = 1)
{
    (void)K;
    Tile t{kDefaultL, kDefaultN};
    if (const char *e = std::getenv("SOS_TILE_L")) {
        const int v = std::atoi(e);
        if (sos_fwd_shape_supported(v, t.N)) t.L = v;
    }
    if (const char *e = std::getenv("SOS_TILE_N")) {
        const int v = std::atoi(e);
        if (sos_fwd_shape_supported(t.L, v)) t.N = v;
    }
    if (h->tile_L) t = Tile{h->tile_L, h->tile_N};
    return t;
}

inline int bits_of(const sos_ctx *h)
{
    if (h->bits) return h->bits;
    if (const char *e = std::getenv("SOS_PRECISION")) {
        const int v = std::atoi(e);
        if (v == 32 || v == 64) return v;
    }
    return kDefaultBits;
}

// True when the group shape comes from the handle or the environment rather
// than from the defaults.
inline bool tile_is_set(const sos_ctx *h)
{
    return h->tile_L || std::getenv("SOS_TILE_L") || std::getenv("SOS_TILE_N");
}

// Group shape for one FP32 signal of n samples when no tile is set: fewer
// samples per lane for shorter signals, which shortens every group's
// per-section chain while there are too few groups to fill the device
// (measured on MI355X, one call including table preparation: 15-26 % less
// time at orders 8-16 up to 2^20 samples with (512, 16), 8-10 % at 2^21-2^22
// with (512, 32), which at 2^23 is already 8 % slower than the default).
// n < 0: unknown, the default tile.
inline Tile tile_for_length(const sos_ctx *h, int K, int64_t n)
{
    const Tile t = tile_of(h, K);
    if (n < 0 || tile_is_set(h) || bits_of(h) != 32) return t;
    if (n <= ((int64_t)1 << 20)) return Tile{512, 16};
    if (n <= ((int64_t)1 << 22)) return Tile{512, 32};
    return t;
}

// Section solver in effect (SOS_ALG_AUTO, SOS_ALG_DCCR or SOS_ALG_PH): the
// handle's choice, else SOS_ALG in the environment ("auto", "dccr" or "ph"),
// else SOS_ALG_AUTO.
inline int solver_of(const sos_ctx *h)
{
    if (h->alg != SOS_ALG_DEFAULT) return h->alg;
    if (const char *e = std::getenv("SOS_ALG")) {
        if (!std::strcmp(e, "ph") || !std::strcmp(e, "PH")) return SOS_ALG_PH;
        if (!std::strcmp(e, "dccr") || !std::strcmp(e, "DCCR")) return SOS_ALG_DCCR;
        if (!std::strcmp(e, "toeplitz")) return SOS_ALG_TOEPLITZ;
    }
    return SOS_ALG_AUTO;
}

// Per-section solver behind a handle's solver: the block-Toeplitz choice
// runs PH wherever the whole-cascade form does not apply.
inline bool ph_sections(int solver)
{
    return solver == SOS_ALG_PH || solver == SOS_ALG_TOEPLITZ;
}

// Whole-cascade block-Toeplitz path (sos_toep.hip): at most 8 sections (a
// 16-dimensional state), for cascades whose sections all peak at most
// kToepRhoMax. The automatic choice takes it where it was measured faster
// than the faster per-section solver (MI355X, per call, tables included):
// K = 8 from 2^25 samples (+14 / +25 / +32 / +37 % at 2^25 / 2^26 / 2^27 /
// 2^28; -3 % at 2^24), K = 7 from 2^25 (+4 / +14 / +19 %; -13 % at 2^24)
// and K = 6 from 2^26 (+1 / +6 %, and +5 / +12 % over DC-CR, which the
// automatic choice runs otherwise; -7 % at 2^25); K = 5 stays on the
// section kernels (-7 % at 2^27, -4 % at 2^28). A call takes at least about
// 0.07 ms (the tables, and chunks of 16384-sample groups that must fill the
// device), which is what shorter signals cannot amortise.
constexpr int kToepMaxK = 8;

// Shortest signal the automatic choice filters by the block-Toeplitz path for
// K sections (none: INT64_MAX).
inline int64_t toep_auto_min_n(int K)
{
    if (K == kToepMaxK || K == 7) return (int64_t)1 << 25;
    if (K == 6) return (int64_t)1 << 26;
    return INT64_MAX;
}
constexpr double kToepRhoMax = 128.0;

// Groups of 16384 samples per block-Toeplitz chunk (one ticket, one lookback)
// for a signal of n samples (n < 0: unknown). A workgroup takes a chunk's
// groups one after the other, so a chunk of 8 groups keeps one workgroup busy
// for about 0.1 ms: below 2^25 samples most workgroups would get one chunk or
// none, and chunks of 2 groups are faster (MI355X, per call, tables included:
// 57 / 94 / 139 GS/s at 2^22 / 2^23 / 2^24 against 33 / 63 / 112). From 2^25
// on, 8 groups are (193 against 188 at 2^25, 300 against 270 at 2^28); 4
// groups were never the fastest at 2^22-2^28. SOS_TOEP_CHUNK (2, 4 or 8)
// overrides.
inline int toep_chunk_groups(int64_t n)
{
    if (const char *e = std::getenv("SOS_TOEP_CHUNK")) {
        const int g = std::atoi(e);
        if (g == 2 || g == 4 || g == 8) return g;
    }
    return (n < 0 || n >= ((int64_t)1 << 25)) ? 8 : 2;
}

// Kernel of the filter launches: ALG_PH for the PH solver, ALG_DCCR for
// DC-CR and for the automatic choice (signals whose tables took the accurate
// layout are solved by PH in any launch).
inline int alg_of(const sos_ctx *h)
{
    return ph_sections(solver_of(h)) ? sosdev::ALG_PH : sosdev::ALG_DCCR;
}

// Peak gain of a section's recursive part, 1 / min |A(e^{jw})|, above which
// a signal's tables take the accurate layout (FP32 compute): its state work
// runs in FP64, its correction uses an orthonormal basis, and its sections
// are solved by PH. With poles close to the unit circle the FP32 powers of
// the state map, and DC-CR's fold B(z)A(-z) near the poles' mirror
// frequencies, amplify rounding. Measured on MI355X (2^20 samples, cascades
// of 4 and 8 sections, against a sequential FP32 filter's error): the fast
// DC-CR layout already reaches 3-6x that error at peak gains of 120-360,
// the fast PH layout stays within 3x up to 128 and reaches 3-18x from about
// 800 on (the lightly damped order-16 cascade, pole radius 0.995, peak gain
// 5673: 18x), the accurate layout stays within 2x throughout.
//   automatic choice: DC-CR's fast layout up to 32, else the accurate one
//                     (Butterworth designs up to order 16 at cutoff 0.2*pi
//                     peak at 15.7);
//   PH:               PH's fast layout up to 128, else the accurate one.
// An explicit DC-CR handle keeps DC-CR and the compute type everywhere.
constexpr double kAutoRhoMax = 32.0;
constexpr double kPhRhoMax = 128.0;

// The threshold of the handle's solver (DC-CR: none); SOS_ACCURATE_GAIN in
// the environment (a positive number, "inf" for none) overrides it for the
// automatic choice and PH.
inline double rho_max_of(const sos_ctx *h)
{
    const int s = solver_of(h);
    if (s == SOS_ALG_DCCR) return HUGE_VAL;
    if (const char *e = std::getenv("SOS_ACCURATE_GAIN")) {
        const double v = std::strtod(e, nullptr);
        if (v > 0.0) return v;
    }
    return ph_sections(s) ? kPhRhoMax : kAutoRhoMax;
}

// Solver argument of the kernel launchers for tables prepared for `solver`
// (SOS_ALG_*) at compute type `bits` with peak-gain threshold `rho_max`: the
// kernel's solver, plus ALG_MAYBE_ACC when those tables may use the accurate
// layout (FP32 with a finite threshold).
inline int launch_alg(int bits, int solver, double rho_max)
{
    const int a = ph_sections(solver) ? sosdev::ALG_PH : sosdev::ALG_DCCR;
    return (bits == 32 && std::isfinite(rho_max)) ? (a | sosdev::ALG_MAYBE_ACC) : a;
}

// SOS_GRID: exactly this many workgroups for every persistent launch, or 0
// (tests: many groups per workgroup).
inline int64_t grid_override()
{
    if (const char *e = std::getenv("SOS_GRID")) {
        const long long g = std::atoll(e);
        if (g > 0) return (int64_t)g;
    }
    return 0;
}

inline int64_t grid_of(int bits, int alg, int L, int N)
{
    // persistent grid: as many workgroups as can be resident, drawing tickets
    // until the groups run out (measured faster than one workgroup per group)
    if (const int64_t g = grid_override()) return g;
    int64_t grid = sos_fwd_capacity(bits, alg, L, N);
    if (const char *e = std::getenv("SOS_PERSISTENT")) {
        const int f = std::atoi(e);
        grid = f > 0 ? (int64_t)f * grid : 0;   // 0: one workgroup per group
    }
    return grid;
}

// Arguments of one uneven batch (see sos_filter_batched).
struct BatchArgs {
    int B, kmax;
    int64_t total_rows, total_samples;
    const int32_t *K, *sec_off;
    const float *sections;
    const int64_t *sig_off;
    const float *x;
    float *y;
    const float *zi;
    float *zf;
    float *saved = nullptr;   // training: outputs of sections 0..kmax-2, stride total_samples
};
// Argument checks (no device work).
int batch_check(const BatchArgs &ba);
// Grow the handle's workspace for the batch at tile t (may allocate and
// synchronise `stream`; never called under graph capture).
int batch_reserve(sos_ctx *h, Tile t, int bits, const BatchArgs &ba, hipStream_t stream);
// Enqueue prep, work table, arm and filter launches only (graph-capturable).
int batch_enqueue(sos_ctx *h, Tile t, int bits, const BatchArgs &ba, hipStream_t stream);


// A batch as the cost model sees it: signal lengths, sections, total samples.
struct ModelBatch {
    std::vector<int64_t> len;
    std::vector<int> K;
    int64_t total = 0;
};
double model_batch_ms(const sos_model_device &d, const ModelBatch &b, int L, int N, int pad,
                      int regs, double ops, double F_us);

}  // namespace sosint
