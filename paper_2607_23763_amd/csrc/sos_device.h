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
// reduction, or PH (particular solution + homogeneous correction).
enum : int { ALG_DCCR = 0, ALG_PH = 1 };

// Per-section coefficient table (FP32 values computed in FP64 on the device)
// for one group shape: L = 64*W lanes in W waves, N samples per lane,
// C = L*N samples per group. Uniform entries are read with scalar loads; the
// two per-lane arrays with one 128-bit load per lane.
enum : int {
    OFF_STATUS = 0,         // 0 = usable, else ERRBIT_* (stored as a number)
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
static_assert(OFF_G + kMaxN + 1 <= OFF_LANEPOW, "table overlap");
static_assert(OFF_GRPPOW + 256 <= OFF_SCANPOW && OFF_SCANPOW + 512 <= TAB_FLOATS,
              "table overlap");
static_assert((OFF_LANEPOW % 4) == 0 && (OFF_GRPPOW % 4) == 0 && (OFF_SCANPOW % 4) == 0 &&
                  (TAB_FLOATS % 16) == 0,
              "per-lane tables must be 16-byte aligned");

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
