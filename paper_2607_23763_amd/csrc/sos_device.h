// Device-side definitions shared by the HIP kernels of libsosfilt:
// the per-section coefficient table layout, control words and small helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sosdev {

// Native 128-bit vector (usable with the nontemporal builtins).
typedef float f4 __attribute__((ext_vector_type(4)));

// Read-only view of a table in the constant address space: wave-uniform
// indexes compile to scalar (SMEM) loads into SGPRs instead of vector loads.
typedef const __attribute__((address_space(4))) float ctab_t;
__device__ __forceinline__ ctab_t *ctab(const float *p) { return (ctab_t *)p; }

// A group is L = 64*W lanes held by W wavefronts of one workgroup; lane l of
// the group owns samples [l*N, l*N + N).
constexpr int kLanes = 64;

// Control words in device memory (one block per workspace).
enum : int {
    CTRL_TICKET = 0,   // next group ticket of the running launch
    CTRL_EPOCH = 1,    // launch counter: tag of valid lookback descriptors
    CTRL_ERR = 2,      // sticky device-side error bits (ERRBIT_*)
    CTRL_DONE = 3,     // workgroups of the running launch that have left it
    CTRL_WORDS = 16
};
enum : unsigned { ERRBIT_A0 = 1u, ERRBIT_UNSTABLE = 2u, ERRBIT_TIMEOUT = 4u, ERRBIT_BADARG = 8u };

// Per-section solver of the filter kernel: divide-and-conquer cyclic
// reduction, or PH (particular solution + homogeneous correction). A launch's
// solver may carry ALG_MAYBE_ACC: its tables may use the accurate layout
// (FP32 compute only), so the launch must hold that path too.
enum : int { ALG_DCCR = 0, ALG_PH = 1, ALG_MAYBE_ACC = 4 };

// Per-section coefficient table, computed in FP64 on the device for one group
// shape (L = 64*W lanes in W waves, N samples per lane, C = L*N samples per
// group): a 16-byte header, then one of two layouts, the same for every
// section of a signal (its preparation chooses).
//
// Fast layout: TAB_FLOATS entries of the compute type T (the state-map
// powers rounded to T, the correction through the impulse response g).
//
// Accurate layout (FP32 per-sample work only): an FP64 state part, then an
// FP32 per-sample part. Powers of the state map of a section whose poles lie
// close to the unit circle are badly conditioned in TDF-II coordinates (their
// entries grow like 1/sin(theta) while the states they act on cancel), and
// rounding them to FP32, or composing states with them in FP32, is amplified
// into every sample of a group; so everything that acts on carried states
// (the lanes' terminal states, the scans over lanes, waves and groups, the
// lanes' incoming states) runs in FP64 with FP64 powers. That work is O(1)
// per lane and section. The incoming state reaches the samples through two
// orthonormal columns spanning its free responses over a lane, after an FP64
// change of basis R, so the two correction terms cannot cancel.
enum : int {
    TAB_HDR = 16,           // bytes: two 64-bit words
    HDR_STATUS = 0,         // word: 0 = usable, else ERRBIT_* of the section
    HDR_MODE = 1            // word: the layout (MODE_*), the same for the whole signal
};
enum : unsigned { MODE_FAST = 0u, MODE_ACCURATE = 1u };

enum : int {                // fast layout: entries of T after the header
    OFF_FIR = 1,            // [3] adjoint tables only: b0, b1, b2 of the section
    OFF_TAPS = 4,           // [5] taps of B(z) A(-z): the level-1 right-hand side
    OFF_B1 = 9, OFF_B2 = 10, OFF_A1 = 11, OFF_A2 = 12,
    OFF_E = 16,             // [8] e_i, level-i coefficient of w^1 (e_0 = a1)
    OFF_F = 24,             // [8] f_i, level-i coefficient of w^2 (f_0 = a2)
    OFF_KS = 32,            // [6][4] T^(N*2^k), k = 0..5 (in-row scan steps use k < 4)
    OFF_TC = 56,            // [4] T^C: state map across a whole group
    OFF_TW = 60,            // [4] T^(64*C): across one lookback window
    OFF_TWAVE = 64,         // [4] T^(64*N): across one wave's 64 lanes
    OFF_WPOW = 68,          // [16][4] T^(64*N*w): group state -> incoming state of wave w
    OFF_G = 132,            // [kMaxN + 1] g[-1..kMaxN-1], impulse response of 1/A
    OFF_LANEPOW = 264,      // [64][4] T^(N*l): wave state -> incoming state of lane l
    OFF_GRPPOW = 520,       // [64][4] T^(C*j): state j groups back -> this group
    OFF_SCANPOW = 776,      // [64][8] T^(N*((l%16)+1)), T^(N*(l-31)): cross-row scan steps
    TAB_FLOATS = 1296
};
constexpr int kMaxN = 128;
constexpr int kMaxWaves = 16;

enum : int {                // accurate layout, state part: doubles after the header
    SD_KS = 0, SD_TC = 24, SD_TW = 28, SD_TWAVE = 32,   // as OFF_KS .. OFF_TWAVE
    SD_R = 36,              // [4] R of [g[m], g[m-1]] = [q0[m], q1[m]] R (row-major, R[1][0] = 0)
    SD_B1 = 40, SD_B2 = 41, SD_A1 = 42, SD_A2 = 43,
    SD_RHO = 44,            // peak gain 1 / min |A(e^{jw})| of the recursive part
    SD_WPOW = 48, SD_LANEPOW = 112, SD_GRPPOW = 368, SD_SCANPOW = 624,   // as OFF_*
    SD_DOUBLES = 1136
};
enum : int {                // accurate layout, per-sample part: floats after the state part
    AP_FIR = 0, AP_TAPS = 4, AP_B1 = 9, AP_B2 = 10, AP_A1 = 11, AP_A2 = 12, AP_E = 16,
    AP_F = 24,
    AP_Q0 = 32,             // [kMaxN] orthonormal columns spanning the free responses
    AP_Q1 = 32 + kMaxN,     //   g[m] s1 + g[m-1] s2 over a lane (m < N)
    AP_ENTRIES = 32 + 2 * kMaxN
};
constexpr int kAccSampleOff = TAB_HDR + SD_DOUBLES * 8;
constexpr int TAB_BYTES = 10496;
static_assert(OFF_G + kMaxN + 1 <= OFF_LANEPOW && OFF_GRPPOW + 256 <= OFF_SCANPOW &&
                  OFF_SCANPOW + 512 <= TAB_FLOATS,
              "fast layout overlap");
static_assert(SD_WPOW + 4 * kMaxWaves <= SD_LANEPOW && SD_SCANPOW + 512 <= SD_DOUBLES,
              "accurate layout overlap");
static_assert(TAB_HDR + TAB_FLOATS * 8 <= TAB_BYTES && kAccSampleOff + AP_ENTRIES * 4 <= TAB_BYTES &&
                  (TAB_BYTES % 128) == 0,
              "table size");
static_assert((TAB_HDR + 4 * OFF_LANEPOW) % 16 == 0 && (TAB_HDR + 4 * OFF_GRPPOW) % 16 == 0 &&
                  (TAB_HDR + 4 * OFF_SCANPOW) % 16 == 0 && (kAccSampleOff % 16) == 0,
              "per-lane tables must be 16-byte aligned");

// Whether signal i of an uneven batch is consistent: 0 <= K <= kmax, its
// section rows inside [0, rows), its samples inside [0, total_samples). Every
// batched kernel skips an inconsistent signal (the work table reports it).
__device__ inline bool batch_signal_ok(int i, int kmax, int64_t rows, int64_t total_samples,
                                       const int32_t *Ks, const int32_t *sec_off,
                                       const int64_t *sig_off)
{
    const int K = Ks[i];
    const int64_t so = sec_off[i], a = sig_off[i], b = sig_off[i + 1];
    return K >= 0 && K <= kmax && so >= 0 && so + K <= rows && a >= 0 && b >= a &&
           b <= total_samples;
}

// Whether the recursive part of section `row` ([b0 b1 b2 a0 a1 a2]) has peak
// gain 1 / min |A(e^{jw})| at most rho_max (always, for rho_max = inf), without
// a square root or a reciprocal: min |A|^2 rho_max^2 >= 1, with
// |A|^2 = 4 a2 c^2 + l c + q on c = cos(w) in [-1, 1] after dividing by a0.
__device__ inline bool gain_within(const float *row, double rho_max)
{
    if (isinf(rho_max)) return true;
    const double a0 = row[3];
    if (a0 == 0.0) return false;
    const double a1 = row[4] / a0, a2 = row[5] / a0;
    const double q = 1.0 + a1 * a1 + a2 * a2 - 2.0 * a2, l = 2.0 * a1 * (1.0 + a2);
    auto f = [&](double c) { return (4.0 * a2 * c + l) * c + q; };
    double m = fmin(f(-1.0), f(1.0));
    if (a2 > 0.0) {
        const double cv = -l / (8.0 * a2);
        if (cv > -1.0 && cv < 1.0) m = fmin(m, f(cv));
    }
    return m > 0.0 && m * rho_max * rho_max >= 1.0;
}

// 2x2 row-major matrices (T acts on TDF-II states (z1, z2)).
struct m2 {
    double a, b, c, d;
};
__device__ inline m2 mmul(const m2 &x, const m2 &y)
{
    return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d,
            x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
__device__ inline m2 mident() { return {1.0, 0.0, 0.0, 1.0}; }

}  // namespace sosdev
