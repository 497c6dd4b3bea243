// Single-kernel multi-block cascade filter for gfx950, and its adjoint.
//
// Mapping (Zhai & Paris Part II, Sec. IV-A): one workgroup of W wavefronts
// owns one group of C = L*N samples, L = 64*W lanes; lane l holds the N
// consecutive samples [l*N, l*N + N) in registers -- the stride-N permuted
// block layout of Sec. II-B. The group is read from HBM once (coalesced
// 128-bit loads, then an LDS transpose into rows), filtered by all K sections
// in registers, and written once. Groups are handed out by an atomic ticket,
// so every group's predecessors are already running (Sec. IV-A).
//
// Per section (Sec. II-D/E/F, Sec. IV-B):
//   1. level-1 right-hand side r1 = B(z) A(-z) u on every lane at zero state
//      (the divide-and-conquer fold, Eq. (23) generalised to b0 != 1);
//   2. one-sided cyclic reduction on both parity chains, log2(N)-1 levels:
//      r_{i+1}[n] = r_i[n] - e_i r_i[n-2^i] + f_i r_i[n-2^{i+1}] on the
//      positions that stay (odd chain n = -1, even chain n = -2 mod 2^{i+1}),
//      which exposes the lane's zero-state terminal pair y[N-2], y[N-1];
//   3. that pair becomes the lane's zero-state terminal state; a scan over the
//      wave's 64 lanes (DPP row shifts and row broadcasts with powers of the
//      state map) gives every lane's zero-state state and the wave's total,
//      and the W wave totals are combined through LDS (one barrier) into every
//      wave's zero-state incoming state and the group's local carry;
//   4. decoupled lookback (last wave): publish the local carry, walk the
//      predecessors' descriptors (64 per round, one per lane) until a resolved
//      carry is found, compose through T^(C j), publish this group's resolved
//      carry and hand the group state to all waves (second barrier);
//   5. each lane's true incoming state = T^(N l) (T^(64 N w) s_group + wave
//      prefix) + lane prefix; back substitution level by level, the single
//      initial-condition row per level and parity receiving g[n] s1 +
//      g[n-1] s2 (no divisions).
// The section output stays in registers as the next section's input.
//
// The PH variant (Sec. II-C, Sec. IV-E) replaces steps 1-2 by the lane's
// particular solution (the section run over the lane's samples from rest,
// whose end state is directly the lane's zero-state terminal state) and the
// back substitution of step 5 by the homogeneous correction y[m] += g[m] s1 +
// g[m-1] s2 on every sample; steps 3-4 are shared. About 7 operations per
// sample and section instead of about 9, and one lane-sequential chain of N
// dependent FMAs instead of the reduction's log-depth levels.
//
// Compute type T of the per-sample work: float, or double. In FP32 each
// signal's tables take one of two layouts (chosen by the preparation kernel
// from its sections' peak gains): the fast layout, where everything runs in
// T, or the accurate layout, where everything that acts on carried states
// (the lanes' terminal states, the scans, the wave combination, the lookback
// composition, the lanes' incoming states and zf) runs in FP64 with FP64
// tables, and each lane's incoming state reaches its samples through two
// orthonormal columns spanning the free responses, after the FP64 change of
// basis R, so that the two correction terms do not cancel. FP32 powers of the
// state map of a lightly damped section lose accuracy in proportion to its
// peak gain; the state path is O(1) per lane and section, and MI355X issues
// FP64 FMAs at the unpacked FP32 rate. Accurate-layout signals are solved by
// PH: DC-CR's fold B(z)A(-z) amplifies rounding near the mirror frequency of
// a pole close to the unit circle. Launch modes: fast-layout tables only,
// accurate-layout tables only, or per group (batched launches). Data in HBM,
// LDS staging and descriptor values are FP32 in every layout.
//
// Descriptors: per (group, section) four 64-bit words {agg.z1, agg.z2,
// inc.z1, inc.z2}, each {float value | 32-bit epoch tag}, stored
// section-major (section s, group h at s * dstride + h), so the window of
// consecutive predecessors a lookback reads spans few cache lines. A word is valid when
// its tag equals the launch epoch, so words are self-validating: no fences, no
// clearing between launches, and the agent-scope relaxed atomics keep them
// coherent across the XCDs' separate L2 caches. The last workgroup to leave a
// plain or adjoint launch zeroes the ticket and advances the epoch for the
// next launch on the same control block (a fresh block starts in that state),
// so consecutive plain launches need no kernel in between. Batched launches
// are armed by their work-table kernel and skip this (it would lengthen every
// served step).
#include "sos_device.h"
#include "sosfilt.h"

using namespace sosdev;

namespace {

struct FwdArgs {
    // plain mode (B == 0): one signal x/y of n samples, K sections at tabs
    const float *x;
    float *y;
    int64_t n;
    const void *tabs;       // K tables of TAB_BYTES (sos_device.h)
    const float *zi;
    float *zf;
    int K;                  // plain: sections; batched: descriptor stride (max sections)
    // batched mode (B > 0): per-signal arrays (device) and the work table
    int B;
    const int32_t *Ks;      // sections per signal
    const int32_t *sec_off; // B+1 section offsets (tables, zi, zf)
    const int64_t *sig_off; // B+1 sample offsets
    const int64_t *gpre;    // B+1 prefix of group counts
    const int32_t *sigmap;  // ticket -> signal
    const int64_t *total_dev;  // number of work items (batched)
    const float *const *xp; // batched, optional: per-signal input pointers (else x + sig_off)
    float *const *yp;       //   and output pointers (else y + sig_off)
    unsigned *sig_err;      // batched, optional: per-signal error bits (ERRBIT_*)
    // both modes
    float *saved;           // optional: outputs of sections 0..K-2, section s of a signal at
                            // saved + s * saved_stride (+ its sample offset when batched)
    int64_t saved_stride;
    int64_t total;          // number of work items (plain)
    unsigned long long *desc;
    int64_t dstride;        // descriptor slots per section (>= the number of work items)
    unsigned *ctrl;
    unsigned long long timeout_ticks;
    const float *skip_gate;  // plain, optional: a nonzero word here means the
                             // whole-cascade kernel filtered this signal
};

// One unit of work: group g of one signal, drawn as ticket t.
template <typename T>
struct Item {
    const float *x;
    float *y;
    int64_t n;              // samples in the signal
    int64_t g;              // group index within the signal
    int64_t t;              // ticket (descriptor row)
    const unsigned char *tabs;   // tables of the signal's sections
    const float *zi;
    float *zf;
    float *saved;           // the signal's intermediate outputs (or null)
    int K;
    int sig;                // signal of a batch (0 in plain mode)
};

// ----------------------------------------------------------------- lane ops

enum : int {
    DPP_ROW_SHR = 0x110,    // + d, d = 1..15: lane l reads l-d inside its 16-lane row
    DPP_WAVE_SHR1 = 0x138,  // lane l reads l-1 across the whole wave
    DPP_BCAST15 = 0x142,    // lane 15 of row r -> every lane of row r+1
    DPP_BCAST31 = 0x143     // lane 31 -> every lane of rows 2 and 3
};

// DPP move across lanes; lanes whose source is outside the row (or whose row
// is masked off by ROWS) read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp0(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp0(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float readlane(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }

// A per-lane 2x2 matrix (4 consecutive entries of the compute type).
template <typename T>
struct M2 {
    T a, b, c, d;
};
__device__ __forceinline__ M2<float> load_m2(const float *p)
{
    const float4 v = *reinterpret_cast<const float4 *>(p);
    return {v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ M2<double> load_m2(const double *p)
{
    const double2 u = *reinterpret_cast<const double2 *>(p);
    const double2 v = *reinterpret_cast<const double2 *>(p + 2);
    return {u.x, u.y, v.x, v.y};
}

// Read-only constant-space view of a table of the compute type (uniform
// indexes become scalar loads).
template <typename T>
using ctabT = const __attribute__((address_space(4))) T;
template <typename T>
__device__ __forceinline__ ctabT<T> *ctabp(const T *p) { return (ctabT<T> *)p; }

// 2x2 (row-major, 4 entries at p) times vector, plus addend.
template <typename T>
__device__ __forceinline__ void mv_add(ctabT<T> *p, T v1, T v2, T &o1, T &o2)
{
    const T n1 = fmaT(p[0], v1, fmaT(p[1], v2, o1));
    const T n2 = fmaT(p[2], v1, fmaT(p[3], v2, o2));
    o1 = n1;
    o2 = n2;
}

// The two table layouts (sos_device.h) as seen by the kernels. S is the type
// of the state arithmetic and of the state tables, X that of a lane's
// zero-state incoming state kept across the lookback, and the *_ entries are
// indexes into the state part (st) and the per-sample part (sp).
template <typename T, bool ACC>
struct Lay;
template <typename T>
struct Lay<T, false> {   // fast: one array of the compute type
    using S = T;
    using X = T;
    enum : int {
        KS = OFF_KS, TC = OFF_TC, TW = OFF_TW, TWAVE = OFF_TWAVE, WPOW = OFF_WPOW,
        LANEPOW = OFF_LANEPOW, GRPPOW = OFF_GRPPOW, SCANPOW = OFF_SCANPOW, B1 = OFF_B1,
        B2 = OFF_B2, A1 = OFF_A1, A2 = OFF_A2,
        P_FIR = OFF_FIR, P_TAPS = OFF_TAPS, P_B1 = OFF_B1, P_B2 = OFF_B2, P_A1 = OFF_A1,
        P_A2 = OFF_A2, P_E = OFF_E, P_F = OFF_F
    };
    static __device__ __forceinline__ const S *st(const unsigned char *tb)
    {
        return reinterpret_cast<const S *>(tb + TAB_HDR);
    }
    static __device__ __forceinline__ const T *sp(const unsigned char *tb)
    {
        return reinterpret_cast<const T *>(tb + TAB_HDR);
    }
};
template <>
struct Lay<float, true> {   // accurate: FP64 state part, FP32 per-sample part
    using S = double;
    using X = float;
    enum : int {
        KS = SD_KS, TC = SD_TC, TW = SD_TW, TWAVE = SD_TWAVE, WPOW = SD_WPOW,
        LANEPOW = SD_LANEPOW, GRPPOW = SD_GRPPOW, SCANPOW = SD_SCANPOW, B1 = SD_B1,
        B2 = SD_B2, A1 = SD_A1, A2 = SD_A2,
        P_FIR = AP_FIR, P_TAPS = AP_TAPS, P_B1 = AP_B1, P_B2 = AP_B2, P_A1 = AP_A1,
        P_A2 = AP_A2, P_E = AP_E, P_F = AP_F
    };
    static __device__ __forceinline__ const S *st(const unsigned char *tb)
    {
        return reinterpret_cast<const S *>(tb + TAB_HDR);
    }
    static __device__ __forceinline__ const float *sp(const unsigned char *tb)
    {
        return reinterpret_cast<const float *>(tb + kAccSampleOff);
    }
};

// Inclusive affine scan over the 64 lanes of a wave:
//   P[l] = t[l] + S P[l-1]   (P[-1] = 0),  S = the state map across one lane,
// the cross-lane terminal-state recurrence (role of Eq. (13)). Within each
// 16-lane row a Kogge-Stone ladder with the uniform powers S^(2^k), k < 4;
// then rows 1 and 3 add lane 15 / 47 through S^((l%16)+1) and rows 2 and 3
// add lane 31 through S^(l-31) (per-lane powers from the table).
template <typename LY, typename S>
__device__ __forceinline__ void wave_scan(S &p1, S &p2, const S *stv, int lane)
{
    using T = S;
    ctabT<T> *tab = ctabp(stv);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T q1, q2;
        switch (k) {
        case 0: q1 = dpp0<DPP_ROW_SHR + 1, 0xF>(p1); q2 = dpp0<DPP_ROW_SHR + 1, 0xF>(p2); break;
        case 1: q1 = dpp0<DPP_ROW_SHR + 2, 0xF>(p1); q2 = dpp0<DPP_ROW_SHR + 2, 0xF>(p2); break;
        case 2: q1 = dpp0<DPP_ROW_SHR + 4, 0xF>(p1); q2 = dpp0<DPP_ROW_SHR + 4, 0xF>(p2); break;
        default: q1 = dpp0<DPP_ROW_SHR + 8, 0xF>(p1); q2 = dpp0<DPP_ROW_SHR + 8, 0xF>(p2); break;
        }
        mv_add<T>(tab + LY::KS + 4 * k, q1, q2, p1, p2);
    }
    const M2<T> pa = load_m2(stv + LY::SCANPOW + 8 * lane);
    const M2<T> pb = load_m2(stv + LY::SCANPOW + 8 * lane + 4);
    {
        const T q1 = dpp0<DPP_BCAST15, 0xA>(p1), q2 = dpp0<DPP_BCAST15, 0xA>(p2);
        const T n1 = fmaT(pa.a, q1, fmaT(pa.b, q2, p1));
        const T n2 = fmaT(pa.c, q1, fmaT(pa.d, q2, p2));
        p1 = n1;
        p2 = n2;
    }
    {
        const T q1 = dpp0<DPP_BCAST31, 0xC>(p1), q2 = dpp0<DPP_BCAST31, 0xC>(p2);
        const T n1 = fmaT(pb.a, q1, fmaT(pb.b, q2, p1));
        const T n2 = fmaT(pb.c, q1, fmaT(pb.d, q2, p2));
        p1 = n1;
        p2 = n2;
    }
}

// Sum over the 64 lanes of a wave (result valid in every lane).
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    v += dpp0<DPP_ROW_SHR + 1, 0xF>(v);
    v += dpp0<DPP_ROW_SHR + 2, 0xF>(v);
    v += dpp0<DPP_ROW_SHR + 4, 0xF>(v);
    v += dpp0<DPP_ROW_SHR + 8, 0xF>(v);
    v += dpp0<DPP_BCAST15, 0xA>(v);
    v += dpp0<DPP_BCAST31, 0xC>(v);
    return readlane(v, 63);
}

// Sample memory is global memory; saying so makes its loads and stores
// global rather than flat instructions, which count only against the vector
// memory counter, so waits for LDS and scalar loads do not also wait for them
// (the signal pointers of a batch are loaded from memory, which hides their
// address space from the compiler).
template <typename P>
__device__ __forceinline__ __attribute__((address_space(1))) P *gptr(P *p)
{
    return (__attribute__((address_space(1))) P *)p;
}

// Workgroup barrier that orders LDS only. __syncthreads() also waits for all
// of the wave's outstanding global memory operations (vmcnt 0), which would
// make every barrier wait for the next group's prefetch and the previous
// group's stores; no barrier here protects global memory.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------- descriptors

__device__ __forceinline__ unsigned long long pack(float v, unsigned tag)
{
    return ((unsigned long long)tag << 32) | (unsigned long long)__float_as_uint(v);
}

__device__ __forceinline__ void store_word(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long load_word(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lane `zl` (only) writes its N registers to scratch LDS and reads back
// positions zp and zp-1 (0 if zp == 0). tl must hold 2N floats.
template <typename T, int N>
__device__ __forceinline__ void pick_two(const T (&u)[N], float *tl, int lane, int zl, int zp,
                                         T &v0, T &v1)
{
    T *sc = reinterpret_cast<T *>(tl);
    if (lane == zl) {
#pragma unroll
        for (int k = 0; k < N; ++k) sc[k] = u[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane == zl) {
        v0 = sc[zp];
        v1 = zp >= 1 ? sc[zp - 1] : T(0);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Resolve the incoming state of group it.g (> 0) of a signal for section s by
// decoupled lookback; executed by one whole wave. Returns wave-uniform values.
//
// Each round the wave reads the kSpan newest predecessors not yet consumed
// (lane l < kSpan reads predecessor l; kWin windows of them, one here) and
// consumes the longest prefix that is ready: if a resolved carry (inclusive)
// lies in that prefix at lane j*, the result is inc[j*] propagated over j*
// groups plus the local carries (aggregates) of the j* groups in front of it,
// and the walk ends; otherwise the prefix's aggregates are added and the walk
// slides past them, into the next window of the same round when the whole
// window was consumed. When the newest unconsumed predecessor is not ready,
// the wave polls that single descriptor, one request per poll, with a short
// fixed sleep between polls (an exponential backoff up to 16 times as long
// overslept the publication: order 16 and the uneven batch ran 0.6-1.5 %
// slower, same-box A/B on MI355X). On timeout it returns NaNs and sets the
// error bit (the caller still publishes, so successors terminate).
template <int kSpan, typename LY, typename It, typename T>
__device__ void lookback(const FwdArgs &a, const It &it, const T *stv, int s,
                         unsigned epoch, int lane, T &r1, T &r2)
{
    // One window of kSpan predecessors per round. Every descriptor read is an
    // agent-scope load served beyond the XCD's L2, competing with the sample
    // stream, so a window far wider than the walk loses: measured on MI355X,
    // 64 loses to 16 (order 2: 8-11 %; order 16 at 4 K-sample groups: 35 %);
    // with the fixed sleep between polls, 32 beats 16 at order 2 (+2.1 / +0.9
    // / +0.3 % at 2^24 / 2^25 / 2^28 samples; order 8: +1.2 % at 2^24, -0.4 %
    // at 2^28; order 16 and the uneven batch level) and 8 loses 3-4 %; two or
    // four windows per round lose.
    constexpr int kWin = 1;
    const M2<T> gp = load_m2(stv + LY::GRPPOW + 4 * lane);   // T^(C lane)
    T acc1 = 0, acc2 = 0;
    T m00 = 1, m01 = 0, m10 = 0, m11 = 1;   // transform from the newest unconsumed group
    const int64_t first = it.t - it.g;      // ticket of the signal's first group
    int64_t base = it.t - 1;                // newest unconsumed predecessor
    bool single = false;                    // waiting on the newest one only
    const unsigned long long t0 = wall_clock64();
    while (true) {
        unsigned long long w[kWin][4];
#pragma unroll
        for (int r = 0; r < kWin; ++r) {
            const int64_t h = base - lane - kLanes * r;
#pragma unroll
            for (int i = 0; i < 4; ++i) w[r][i] = 0ull;
            if (h >= first && (single ? (r == 0 && lane == 0) : lane < kSpan)) {
                const unsigned long long *d = a.desc + ((size_t)s * a.dstride + h) * 4;
#pragma unroll
                for (int i = 0; i < 4; ++i) w[r][i] = load_word(d + i);
            }
        }
        bool done = false, progressed = false;
#pragma unroll
        for (int r = 0; r < kWin; ++r) {
            if (single && r > 0) break;
            const bool inc_ok =
                (unsigned)(w[r][2] >> 32) == epoch && (unsigned)(w[r][3] >> 32) == epoch;
            const bool agg_ok =
                (unsigned)(w[r][0] >> 32) == epoch && (unsigned)(w[r][1] >> 32) == epoch;
            const unsigned long long incm = __ballot(inc_ok);
            const unsigned long long rdym = __ballot(inc_ok || agg_ok);
            const int span = single ? 1 : kSpan;
            const unsigned long long spanm = span == 64 ? ~0ull : ((1ull << span) - 1ull);
            const unsigned long long notr = ~rdym & spanm;
            const int nr = notr ? __builtin_ctzll(notr) : span;               // ready prefix
            const int jstar = incm ? __builtin_ctzll(incm) : 64;
            done = jstar < nr;
            const int c = done ? jstar : nr;                                 // aggregates consumed
            if (c == 0 && !done) break;
            progressed = true;
            T v1 = 0, v2 = 0;
            if (lane < c) {
                v1 = __uint_as_float((unsigned)w[r][0]);
                v2 = __uint_as_float((unsigned)w[r][1]);
            } else if (done && lane == jstar) {
                v1 = __uint_as_float((unsigned)w[r][2]);
                v2 = __uint_as_float((unsigned)w[r][3]);
            }
            const T s1 = wave_sum<T>(gp.a * v1 + gp.b * v2);
            const T s2 = wave_sum<T>(gp.c * v1 + gp.d * v2);
            acc1 += m00 * s1 + m01 * s2;
            acc2 += m10 * s1 + m11 * s2;
            if (done) break;
            // slide past the c consumed groups: m <- m T^(C c)
            T p00, p01, p10, p11;
            if (c == 64) {
                ctabT<T> *tab = ctabp(stv);
                p00 = tab[LY::TW + 0]; p01 = tab[LY::TW + 1];
                p10 = tab[LY::TW + 2]; p11 = tab[LY::TW + 3];
            } else {
                p00 = readlane(gp.a, c); p01 = readlane(gp.b, c);
                p10 = readlane(gp.c, c); p11 = readlane(gp.d, c);
            }
            const T n00 = m00 * p00 + m01 * p10, n01 = m00 * p01 + m01 * p11;
            const T n10 = m10 * p00 + m11 * p10, n11 = m10 * p01 + m11 * p11;
            m00 = n00; m01 = n01; m10 = n10; m11 = n11;
            base -= c;
            if (c < kSpan || kSpan < 64) break;   // the next window was read from the old base
        }
        if (done) break;
        if (progressed) {
            single = false;
            continue;
        }
        if (wall_clock64() - t0 > a.timeout_ticks) {
            if (lane == 0) {
                atomicOr(&a.ctrl[CTRL_ERR], ERRBIT_TIMEOUT);
                if (a.sig_err) atomicOr(&a.sig_err[it.sig], ERRBIT_TIMEOUT);
            }
            r1 = r2 = T(__builtin_nanf(""));
            return;
        }
        __builtin_amdgcn_s_sleep(2);
        single = true;
    }
    r1 = acc1;
    r2 = acc2;
}

// Exchange area of one workgroup in LDS.
template <typename T, int W>
struct Xch {
    T wave_tot[W][2];        // zero-state totals of the waves (fast layout)
    T grp[2];                // resolved incoming state of the group (fast layout)
    double wave_tot_d[W][2]; //   the same for the accurate layout's FP64 state work
    double grp_d[2];
    int64_t nxt;             // ticket drawn once the last section's state is resolved
    T zx[2];                 // a section's inputs at samples n-1, n-2 (lane that holds n-1)
    template <typename S>
    __device__ __forceinline__ S (&tot())[W][2]
    {
        if constexpr (sizeof(S) == sizeof(T)) return wave_tot;
        else return wave_tot_d;
    }
    template <typename S>
    __device__ __forceinline__ S (&group())[2]
    {
        if constexpr (sizeof(S) == sizeof(T)) return grp;
        else return grp_d;
    }
};

// A value all lanes of a wave hold alike, made visibly uniform (a scalar
// register instead of a vector one).
__device__ __forceinline__ float wave_uniform(float v)
{
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}
__device__ __forceinline__ double wave_uniform(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Hook run by every wave right after the group state is broadcast, given the
// ticket drawn at that point (see run_section).
struct NoNext {
    __device__ void operator()(int64_t) const {}
};

// Exit of a ticketed launch (thread 0 of every workgroup, after its last draw):
// the workgroup that leaves last re-arms the control block for the next
// launch. Every ticket of this launch has been drawn by then: each workgroup's
// final draw is a returning device-scope atomic whose value decided the exit,
// so it had been performed before that workgroup counted itself out, and the
// count is one atomic order. The epoch was read by every workgroup at its
// start. No release is needed (one would write back the L2 at every exit).
__device__ __forceinline__ void rearm_on_exit(unsigned *ctrl, unsigned epoch)
{
    const unsigned d = __hip_atomic_fetch_add(&ctrl[CTRL_DONE], 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    if (d + 1u == gridDim.x) {
        const unsigned e = epoch + 1u;
        __hip_atomic_store(&ctrl[CTRL_TICKET], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl[CTRL_EPOCH], e == 0u ? 1u : e, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl[CTRL_DONE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------- one section

// One section of the cascade on the group held by the workgroup, in two
// halves: section_zs solves the section at zero group state (steps 1-3) and
// publishes the group's local carry; section_corr resolves the group's
// incoming state (step 4) and corrects the samples (step 5). What the first
// half leaves for the second is small and mostly wave-uniform.
// PAIR = false: the forward filter; carries are TDF-II states.
// PAIR = true: a pure recursive section 1/A(z) (the adjoint's reversed-time
//   pass); carries are the last two outputs (y[-2], y[-1]), and the tables hold
//   the matching state map.
// ACC: the table layout (sos_device.h). Fast: the state work in the compute
//   type, the correction through g. Accurate (FP32 only): the state work in
//   FP64, the correction through the orthonormal columns after R.

// What the zero-state half leaves for the correction half of one section.
template <typename S, typename X>
struct SecState {
    X x1, x2;     // the lane's zero-state incoming state (the scan's exclusive prefix);
                  // FP32 in the accurate layout, rounded once like a sequential
                  // filter's state, which keeps the FP64 values off the registers
                  // that the lookback and the next group's prefetch need
    S e1w, e2w;   // the wave's incoming state at zero group state (wave-uniform)
    S g1, g2;     // the group's local carry (lookback wave, wave-uniform)
};

template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

// The 64-bit header word i of table tb (scalar load).
__device__ __forceinline__ unsigned long long tab_word(const unsigned char *tb, int i)
{
    return ((const __attribute__((address_space(4))) unsigned long long *)tb)[i];
}

template <typename T, bool ACC, int N, int W, bool PAIR, int ALG>
__device__ __forceinline__ void section_zs(T (&u)[N], Xch<T, W> &xch, float *tl,
                                           const FwdArgs &a, const Item<T> &it,
                                           const unsigned char *tb, int s, unsigned epoch, int wv,
                                           int lane, bool has_last, int zl, int zp,
                                           SecState<typename Lay<T, ACC>::S,
                                                    typename Lay<T, ACC>::X> &st)
{
    using LY = Lay<T, ACC>;
    using S = typename LY::S;
    using X = typename LY::X;
    constexpr int LOG = __builtin_ctz(N);
    ctabT<T> *tab = ctabp(LY::sp(tb));
    ctabT<S> *sd = ctabp(LY::st(tb));

    // --- inputs kept for the terminal state (and, in LDS, for zf at sample n-1)
    const T xl1 = u[N - 1], xl2 = u[N - 2];
    if (!PAIR && has_last) {
        T zx1 = 0, zx2 = 0;
        pick_two<T, N>(u, tl, lane, zl, zp, zx1, zx2);
        if (lane == zl) {
            xch.zx[0] = zx1;
            xch.zx[1] = zx2;
        }
    }

    if (ALG == ALG_PH) {
        // --- 1-2 (PH). Particular solution (Sec. II-C, Eq. (9)): the lane's
        // own samples through the section from rest, feedforward B(z) (in
        // place from the end), then the recursion 1/A(z) (in place from the
        // start; one FMA of dependency per sample). Nothing crosses lanes;
        // the lane's incoming state enters only in the correction.
        const T a1 = tab[LY::P_A1], a2 = tab[LY::P_A2];
        if (!PAIR) {
            const T b0 = tab[LY::P_TAPS + 0], b1 = tab[LY::P_B1], b2 = tab[LY::P_B2];
#pragma unroll
            for (int m = N - 1; m >= 0; --m) {
                T r = b0 * u[m];
                if (m >= 1) r = fmaT(b1, u[m - 1], r);
                if (m >= 2) r = fmaT(b2, u[m - 2], r);
                u[m] = r;
            }
        }
        u[1] = fmaT(-a1, u[0], u[1]);
#pragma unroll
        for (int m = 2; m < N; ++m) u[m] = fmaT(-a1, u[m - 1], fmaT(-a2, u[m - 2], u[m]));
    } else {
        // --- 1. level-1 right-hand side, in place from the end
        const T c0 = tab[LY::P_TAPS + 0], c1 = tab[LY::P_TAPS + 1], c2 = tab[LY::P_TAPS + 2];
        const T c3 = tab[LY::P_TAPS + 3], c4 = tab[LY::P_TAPS + 4];
#pragma unroll
        for (int m = N - 1; m >= 0; --m) {
            T r = c0 * u[m];
            if (m >= 1) r = fmaT(c1, u[m - 1], r);
            if (m >= 2) r = fmaT(c2, u[m - 2], r);
            if (m >= 3) r = fmaT(c3, u[m - 3], r);
            if (m >= 4) r = fmaT(c4, u[m - 4], r);
            u[m] = r;
        }

        // --- 2. reduction of both parity chains (positions that stay, descending)
#pragma unroll
        for (int i = 1; i < LOG; ++i) {
            const int st2 = 1 << i;
            const T e = tab[LY::P_E + i], f = tab[LY::P_F + i];
#pragma unroll
            for (int m = N - 1; m >= 0; --m) {
                if (((m + 1) % (2 * st2)) == 0 || ((m + 2) % (2 * st2)) == 0) {
                    T r = u[m];
                    if (m - st2 >= 0) r = fmaT(-e, u[m - st2], r);
                    if (m - 2 * st2 >= 0) r = fmaT(f, u[m - 2 * st2], r);
                    u[m] = r;
                }
            }
        }
    }

    // --- 3. zero-state terminal state of the lane, scan over the wave
    S p1, p2;
    if (PAIR) {
        p1 = (S)u[N - 2];
        p2 = (S)u[N - 1];
    } else {
        const S b1 = sd[LY::B1], b2 = sd[LY::B2], a1 = sd[LY::A1], a2 = sd[LY::A2];
        const S y1 = (S)u[N - 1], y2 = (S)u[N - 2], x1 = (S)xl1, x2 = (S)xl2;
        p1 = b1 * x1 + b2 * x2 - a1 * y1 - a2 * y2;
        p2 = b2 * x1 - a2 * y1;
    }
    wave_scan<LY>(p1, p2, LY::st(tb), lane);

    //     ... and over the W waves of the group (zero group state)
    S e1w = 0, e2w = 0;      // zero-state incoming state of this wave
    if (W > 1) {
        if (lane == 63) {
            xch.template tot<S>()[wv][0] = p1;
            xch.template tot<S>()[wv][1] = p2;
        }
        lds_barrier();
        for (int v = 0; v < wv; ++v) {
            S o1 = xch.template tot<S>()[v][0], o2 = xch.template tot<S>()[v][1];
            mv_add<S>(sd + LY::TWAVE, e1w, e2w, o1, o2);
            e1w = o1;
            e2w = o2;
        }
    }
    st.x1 = (X)dpp0<DPP_WAVE_SHR1, 0xF>(p1);
    st.x2 = (X)dpp0<DPP_WAVE_SHR1, 0xF>(p2);
    st.e1w = wave_uniform(e1w);
    st.e2w = wave_uniform(e2w);
    st.g1 = st.g2 = 0;
    if (wv == W - 1) {
        // group local carry = state after the last wave at zero group state
        S g1 = readlane(p1, 63), g2 = readlane(p2, 63);
        if (W > 1) mv_add<S>(sd + LY::TWAVE, st.e1w, st.e2w, g1, g2);
        st.g1 = wave_uniform(g1);
        st.g2 = wave_uniform(g2);
        // --- 4a. publish the local carry (the first group of a signal has none)
        if (it.g != 0 && lane == 0) {
            unsigned long long *dsc = a.desc + ((size_t)s * a.dstride + it.t) * 4;
            store_word(dsc + 0, pack((float)g1, epoch));
            store_word(dsc + 1, pack((float)g2, epoch));
        }
    }
}

// draw: the lookback wave draws the workgroup's next ticket as soon as the
//   group state is resolved (not earlier: a ticket drawn before the wait would
//   carry the wait's jitter into the next group's aggregate), and every wave
//   passes it to on_next right after the broadcast, so that the next group's
//   loads overlap this group's correction and store.
template <typename T, bool ACC, int N, int W, bool PAIR, int ALG, typename OnNext = NoNext>
__device__ __forceinline__ void section_corr(T (&u)[N], Xch<T, W> &xch, float *tl,
                                             const FwdArgs &a, const Item<T> &it,
                                             const unsigned char *tb, int s, unsigned epoch,
                                             int wv, int lane, bool has_last, int zl, int zp,
                                             const SecState<typename Lay<T, ACC>::S,
                                                            typename Lay<T, ACC>::X> &st,
                                             T &q1, T &q2, bool draw = false,
                                             const OnNext &on_next = OnNext())
{
    using LY = Lay<T, ACC>;
    using S = typename LY::S;
    constexpr int LOG = __builtin_ctz(N);
    ctabT<T> *tab = ctabp(LY::sp(tb));
    ctabT<S> *sd = ctabp(LY::st(tb));
    const S *stv = LY::st(tb);
    // The lane power of step 5 is read before the lookback, not at its use: a
    // vector load issued after on_next's loads would wait for all of them. The
    // empty asm (which the compiler must assume rewrites the values) keeps it
    // from sinking or re-issuing the load at the use.
    M2<S> lp = load_m2(stv + LY::LANEPOW + 4 * lane);
    asm volatile("" : "+v"(lp.a), "+v"(lp.b), "+v"(lp.c), "+v"(lp.d));
    if (wv == W - 1) {
        // --- 4b. decoupled lookback for the group's incoming state
        unsigned long long *dsc = a.desc + ((size_t)s * a.dstride + it.t) * 4;
        S sg1, sg2;
        if (it.g == 0) {
            // PAIR: the initial carry arrives as (y[-1], y[-2]) (the adjoint of zf)
            sg1 = it.zi ? (S)ctab(it.zi)[2 * s + (PAIR ? 1 : 0)] : S(0);
            sg2 = it.zi ? (S)ctab(it.zi)[2 * s + (PAIR ? 0 : 1)] : S(0);
        } else {
            lookback<32, LY>(a, it, stv, s, epoch, lane, sg1, sg2);
        }
        unsigned tk = 0;
        if (draw && lane == 0) tk = atomicAdd(&a.ctrl[CTRL_TICKET], 1u);
        S i1 = st.g1, i2 = st.g2;
        mv_add<S>(sd + LY::TC, sg1, sg2, i1, i2);
        if (lane == 0) {
            store_word(dsc + 2, pack((float)i1, epoch));
            store_word(dsc + 3, pack((float)i2, epoch));
            xch.template group<S>()[0] = sg1;
            xch.template group<S>()[1] = sg2;
            if (draw) xch.nxt = (int64_t)tk;
        }
    }
    lds_barrier();
    const S sg1 = xch.template group<S>()[0], sg2 = xch.template group<S>()[1];

    // --- 5. incoming state of every lane, then back substitution
    S sw1 = st.e1w, sw2 = st.e2w;
    mv_add<S>(sd + LY::WPOW + 4 * wv, sg1, sg2, sw1, sw2);
    const S r1 = fmaT(lp.a, sw1, fmaT(lp.b, sw2, (S)st.x1));
    const S r2 = fmaT(lp.c, sw1, fmaT(lp.d, sw2, (S)st.x2));
    q1 = (T)r1;
    q2 = (T)r2;
    // TDF-II injection (s1, s2) of the lane's incoming carry
    const S a1 = sd[LY::A1], a2 = sd[LY::A2];
    const S s1 = PAIR ? -(a1 * r2 + a2 * r1) : r1;
    const S s2 = PAIR ? -a2 * r2 : r2;
    // its free response, g[m] s1 + g[m-1] s2, is added through (c0t, c1t) with
    // coefficients (k1, k2): g itself (fast), or the orthonormal columns after
    // (k1, k2) = R (s1, s2) in FP64 (accurate)
    T k1, k2;
    ctabT<T> *c0t;
    ctabT<T> *c1t;
    if constexpr (ACC) {
        k1 = (T)fma(sd[SD_R + 0], s1, sd[SD_R + 1] * s2);
        k2 = (T)(sd[SD_R + 3] * s2);
        c0t = tab + AP_Q0;
        c1t = tab + AP_Q1;
    } else {
        k1 = (T)s1;
        k2 = (T)s2;
        c0t = tab + OFF_G + 1;   // g[-1] is readable and 0
        c1t = tab + OFF_G;
    }
    T s2z = (T)s2;   // for zf only
    if (draw) {
        // tickets are below 2^31 (the host bounds the groups of a launch)
        int nxt = __builtin_amdgcn_readfirstlane((int)xch.nxt);
        // In the accurate layout the next group's prefetch must not be hoisted
        // above the FP64 state work (its 4N registers would be live beside the
        // state temporaries): its addresses are made to depend on the results.
        if constexpr (ACC) asm volatile("" : "+v"(k1), "+v"(k2), "+v"(s2z), "+s"(nxt));
        on_next((int64_t)nxt);
    }

    if (ALG == ALG_PH) {
        // homogeneous correction (Eq. (11)): the incoming state's free
        // response, added to every sample independently
#pragma unroll
        for (int m = 0; m < N; ++m) u[m] = fmaT(c0t[m], k1, fmaT(c1t[m], k2, u[m]));
    } else {
        u[N - 1] = fmaT(c0t[N - 1], k1, fmaT(c1t[N - 1], k2, u[N - 1]));
        u[N - 2] = fmaT(c0t[N - 2], k1, fmaT(c1t[N - 2], k2, u[N - 2]));
#pragma unroll
        for (int i = LOG - 1; i >= 1; --i) {
            const int st2 = 1 << i;
            const T e = tab[LY::P_E + i], f = tab[LY::P_F + i];
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                const int m0 = st2 - 1 - par;                 // odd chain, then even chain
                u[m0] = fmaT(c0t[m0], k1, fmaT(c1t[m0], k2, u[m0]));
#pragma unroll
                for (int m = m0 + 2 * st2; m < N; m += 2 * st2)
                    u[m] = fmaT(-e, u[m - st2], fmaT(-f, u[m - 2 * st2], u[m]));
            }
        }
    }

    // --- final state after sample n-1 (only the lane that holds it)
    if (!PAIR && has_last && it.zf) {
        T yo1 = 0, yo2 = 0;
        pick_two<T, N>(u, tl, lane, zl, zp, yo1, yo2);
        if (lane == zl) {
            const S b1 = sd[LY::B1], b2 = sd[LY::B2];
            const S zx1 = (S)xch.zx[0], zx2 = (S)xch.zx[1], y1 = (S)yo1, y2 = (S)yo2;
            S z1;
            if (zp >= 1)
                z1 = b1 * zx1 + b2 * zx2 - a1 * y1 - a2 * y2;
            else
                z1 = b1 * zx1 - a1 * y1 + (S)s2z;   // this lane's incoming state
            gptr(it.zf)[2 * s] = (float)z1;
            gptr(it.zf)[2 * s + 1] = (float)(b2 * zx1 - a2 * y1);
        }
    }
}

// Both halves back to back. On return (q1, q2) is the lane's incoming carry.
template <typename T, bool ACC, int N, int W, bool PAIR, int ALG, typename OnNext = NoNext>
__device__ __forceinline__ void run_section(T (&u)[N], Xch<T, W> &xch, float *tl,
                                            const FwdArgs &a, const Item<T> &it,
                                            const unsigned char *tb, int s, unsigned epoch,
                                            int wv, int lane, bool has_last, int zl, int zp,
                                            T &q1, T &q2, bool draw = false,
                                            const OnNext &on_next = OnNext())
{
    SecState<typename Lay<T, ACC>::S, typename Lay<T, ACC>::X> st;
    section_zs<T, ACC, N, W, PAIR, ALG>(u, xch, tl, a, it, tb, s, epoch, wv, lane, has_last, zl,
                                        zp, st);
    section_corr<T, ACC, N, W, PAIR, ALG>(u, xch, tl, a, it, tb, s, epoch, wv, lane, has_last,
                                          zl, zp, st, q1, q2, draw, on_next);
}

// ---------------------------------------------------------------- wave tile
// A wave's part of a group (64 N consecutive samples) staged in LDS as 64 rows
// of N floats, row l holding lane l's samples, with row stride RS = N + 4 so
// that the 128-bit row accesses of 64 lanes are free of bank conflicts.
// Coalesced slot j of lane l is float4 number v = 64 j + l of the part, i.e.
// row v / Q, column 4 (v % Q) with Q = N / 4; since Q divides 64 this is a
// per-lane base plus the compile-time offset j (64 / Q) RS, so the addresses
// are one register and immediates.
template <int N>
struct WaveTile {
    static constexpr int Q = N / 4;
    static constexpr int RS = N + 4;
    static constexpr int STEP = (kLanes / Q) * RS;
    static __device__ __forceinline__ int slot_base(int lane)
    {
        return (lane / Q) * RS + (lane % Q) * 4;
    }
};

// Four samples in global memory, which need only be 4-byte aligned: a signal
// of a batch starts at any sample. gfx950 serves a dword-aligned 128-bit
// global access in one instruction (at worst one extra cache line), so the
// whole-tile path never falls back to single-sample accesses.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef __attribute__((address_space(1))) f4u gf4u;

__device__ __forceinline__ const gf4u *gptr4(const float *p)
{
    return (const gf4u *)p;
}
__device__ __forceinline__ gf4u *gptr4(float *p)
{
    return (gf4u *)p;
}

// src[0 .. 64N) -> the lane's coalesced slots t[0 .. N/4); `rem` samples are
// valid (zeros past them).
template <int N>
__device__ __forceinline__ void tile_fetch(f4 (&t)[N / 4], const float *src, int64_t rem,
                                           int lane)
{
    if (rem >= kLanes * N) {
        const gf4u *s4 = gptr4(src) + lane;
#pragma unroll
        for (int j = 0; j < N / 4; ++j) t[j] = __builtin_nontemporal_load(s4 + kLanes * j);
    } else {
        const auto g = gptr(src);
        int r = rem <= 0 ? 0 : (rem >= kLanes * N ? kLanes * N : (int)rem);
        // The per-element bounds of a partial tile depend only on r; the
        // empty asm keeps them in this (rare) branch. Otherwise the compiler
        // merges them with tile_store's identical bounds and computes all of
        // them for every group, parking the masks in spilled registers.
        asm volatile("" : "+v"(r));
#pragma unroll
        for (int j = 0; j < N / 4; ++j) {
            const int q = 4 * (kLanes * j + lane);
            t[j].x = q + 0 < r ? g[q + 0] : 0.0f;
            t[j].y = q + 1 < r ? g[q + 1] : 0.0f;
            t[j].z = q + 2 < r ? g[q + 2] : 0.0f;
            t[j].w = q + 3 < r ? g[q + 3] : 0.0f;
        }
    }
}

// the lane's coalesced slots -> the wave's LDS rows
template <int N>
__device__ __forceinline__ void tile_put(const f4 (&t)[N / 4], float *tl, int lane)
{
    using TT = WaveTile<N>;
    float *p = tl + TT::slot_base(lane);
#pragma unroll
    for (int j = 0; j < TT::Q; ++j) *reinterpret_cast<f4 *>(p + j * TT::STEP) = t[j];
}

// src[0 .. 64N) -> tile; all loads of a lane are issued before the first LDS
// write.
template <int N>
__device__ __forceinline__ void tile_load(const float *src, int64_t rem, float *tl, int lane)
{
    f4 t[N / 4];
    tile_fetch<N>(t, src, rem, lane);
    tile_put<N>(t, tl, lane);
}

// tile -> dst[0 .. min(rem, 64N)). NT: nontemporal stores, all LDS reads
// first (for the final output, when the lane's registers are free); otherwise
// each slot is stored as it is read, holding 4 registers instead of N (for
// the intermediate outputs kept for the adjoint, while the lane's N
// registers are live).
template <int N, bool NT>
__device__ __forceinline__ void tile_store(float *dst, int64_t rem, const float *tl, int lane)
{
    using TT = WaveTile<N>;
    const float *p = tl + TT::slot_base(lane);
    if (rem >= kLanes * N) {
        gf4u *d4 = gptr4(dst) + lane;
        if (NT) {
            f4 t[TT::Q];
#pragma unroll
            for (int j = 0; j < TT::Q; ++j) t[j] = *reinterpret_cast<const f4 *>(p + j * TT::STEP);
#pragma unroll
            for (int j = 0; j < TT::Q; ++j) __builtin_nontemporal_store(t[j], d4 + kLanes * j);
        } else {
#pragma unroll
            for (int j = 0; j < TT::Q; ++j) d4[kLanes * j] = *reinterpret_cast<const f4 *>(p + j * TT::STEP);
        }
    } else {
        const auto g = gptr(dst);
        int r = rem <= 0 ? 0 : (rem >= kLanes * N ? kLanes * N : (int)rem);
        asm volatile("" : "+v"(r));   // bounds stay in this branch (see tile_fetch)
#pragma unroll
        for (int j = 0; j < TT::Q; ++j) {
            const int q = 4 * (kLanes * j + lane);
            const f4 t = *reinterpret_cast<const f4 *>(p + j * TT::STEP);
            if (q + 0 < r) g[q + 0] = t.x;
            if (q + 1 < r) g[q + 1] = t.y;
            if (q + 2 < r) g[q + 2] = t.z;
            if (q + 3 < r) g[q + 3] = t.w;
        }
    }
}

// lane rows of the tile <-> the lane's N registers
template <typename T, int N>
__device__ __forceinline__ void regs_from_rows(T (&u)[N], const float *tl, int lane)
{
    const float *row = tl + lane * WaveTile<N>::RS;
#pragma unroll
    for (int k = 0; k < N / 4; ++k) {
        const f4 v = *reinterpret_cast<const f4 *>(row + 4 * k);
        u[4 * k + 0] = v.x;
        u[4 * k + 1] = v.y;
        u[4 * k + 2] = v.z;
        u[4 * k + 3] = v.w;
    }
}
template <typename T, int N>
__device__ __forceinline__ void rows_from_regs(const T (&u)[N], float *tl, int lane)
{
    float *row = tl + lane * WaveTile<N>::RS;
#pragma unroll
    for (int k = 0; k < N / 4; ++k) {
        const f4 v = {(float)u[4 * k + 0], (float)u[4 * k + 1], (float)u[4 * k + 2],
                      (float)u[4 * k + 3]};
        *reinterpret_cast<f4 *>(row + 4 * k) = v;
    }
}

// Write the wave's registers (lane rows) to dst[g0 .. g0 + 64N) through the
// wave's LDS rows with coalesced stores, masked at the signal end n.
template <typename T, int N>
__device__ __forceinline__ void store_rows(const T (&u)[N], float *tl, int lane, int64_t n,
                                           int64_t g0, float *dst)
{
    rows_from_regs<T, N>(u, tl, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    tile_store<N, false>(dst + g0, n - g0, tl, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// --------------------------------------------------------- forward kernel

// The work item of ticket t (plain signal or one signal of a batch).
template <typename T>
__device__ __forceinline__ Item<T> make_item(const FwdArgs &a, const unsigned char *tabs,
                                             int64_t t)
{
    Item<T> it;
    it.t = t;
    if (a.B == 0) {
        it.x = a.x;
        it.y = a.y;
        it.n = a.n;
        it.g = t;
        it.tabs = tabs;
        it.zi = a.zi;
        it.zf = a.zf;
        it.saved = a.saved;
        it.K = a.K;
        it.sig = 0;
    } else {
        const int i = a.sigmap[t];
        it.sig = i;
        const int64_t so = a.sig_off[i];
        const int32_t sc = a.sec_off[i];
        it.x = a.xp ? a.xp[i] : a.x + so;
        it.y = a.yp ? a.yp[i] : a.y + so;
        it.n = a.sig_off[i + 1] - so;
        it.g = t - a.gpre[i];
        it.tabs = tabs + (size_t)sc * TAB_BYTES;
        it.zi = a.zi ? a.zi + 2 * (int64_t)sc : nullptr;
        it.zf = a.zf ? a.zf + 2 * (int64_t)sc : nullptr;
        it.saved = a.saved ? a.saved + so : nullptr;
        it.K = a.Ks[i];
    }
    return it;
}


// Everything after the wave's samples are in registers: the K sections, then
// registers -> the wave's LDS rows -> coalesced 128-bit global stores. With
// draw set, the last section draws the next ticket and calls on_next with it.
template <typename T, bool ACC, int N, int W, int ALG, typename OnNext>
__device__ __forceinline__ void finish_group(const FwdArgs &a, const Item<T> &it, T (&u)[N],
                                             float *tl, Xch<T, W> &xch, unsigned epoch, int wv,
                                             int lane, bool draw, const OnNext &on_next)
{
    constexpr int CW = kLanes * N;   // samples per wave
    constexpr int C = CW * W;        // samples per group
    const int64_t g0 = it.g * C + (int64_t)wv * CW;   // first sample of this wave
    const int64_t rem = it.n - g0;                    // may be <= 0 in the last group

    // --- sections (an unusable section poisons its signal)
    bool bad = false;
    for (int s = 0; s < it.K; ++s)
        bad |= tab_word(it.tabs + (size_t)s * TAB_BYTES, HDR_STATUS) != 0ull;
    // position of the last real sample n-1 if this wave holds it
    const int64_t lp = (it.n - 1) - g0;
    const bool has_last = lp >= 0 && lp < CW;
    const int zl = has_last ? (int)(lp / N) : 0, zp = has_last ? (int)(lp % N) : 0;
    if (!bad) {
        // with draw, the last section is peeled off the loop so that the
        // next group's registers are live only from its draw on
        const int kl = draw ? it.K - 1 : it.K;
        for (int s = 0; s < kl; ++s) {
            T q1, q2;
            run_section<T, ACC, N, W, false, ALG>(u, xch, tl, a, it,
                                                  it.tabs + (size_t)s * TAB_BYTES, s, epoch, wv,
                                                  lane, has_last, zl, zp, q1, q2);
            if (it.saved && s + 1 < it.K)
                store_rows<T, N>(u, tl, lane, it.n, g0, it.saved + (size_t)s * a.saved_stride);
        }
        if (draw && it.K > 0) {
            const int s = it.K - 1;
            T q1, q2;
            run_section<T, ACC, N, W, false, ALG>(u, xch, tl, a, it,
                                                  it.tabs + (size_t)s * TAB_BYTES, s, epoch, wv,
                                                  lane, has_last, zl, zp, q1, q2, true, on_next);
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) u[k] = T(__builtin_nanf(""));
        if (has_last && lane == 0 && it.zf)
            for (int s = 0; s < it.K; ++s) it.zf[2 * s] = it.zf[2 * s + 1] = __builtin_nanf("");
    }

    // --- store: the tile is the wave's own, so wave-scope ordering suffices
    rows_from_regs<T, N>(u, tl, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    tile_store<N, true>(it.y + g0, rem, tl, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Minimum waves per SIMD the register allocation must allow, chosen so that
// two workgroups fit on a CU where LDS allows it (W = 4: 2 waves of <= 256
// registers; W = 8: 4 waves of <= 128); otherwise the compiler's choice.
// With one workgroup per CU, its load, lookback and store phases leave the
// CU idle; a second resident group fills them.
template <typename T, int N, int W>
constexpr int min_waves_per_simd()
{
    if (sizeof(T) != 4) return 1;
    if (W == 4) return 2;
    if (W == 8 && N <= 32) return 4;
    return 1;
}

// The filter kernel: every workgroup draws tickets until the work runs out.
// A ticket names one group of one signal; within a signal, tickets ascend with
// the group index, so a group's predecessors were drawn (and are being worked
// on) before it, which guarantees forward progress of the lookback whatever
// the grid size (Sec. IV-A).
// Which table layouts a launch serves: KM_FAST the fast one only, KM_ACC the
// accurate one only (plain launches: the host launches both and the one that
// does not match the signal's layout leaves at once), KM_MIX either, chosen
// per group (batched launches, whose signals may differ). A kernel holding one
// path has the register file to itself; per-group choice costs registers.
enum : int { KM_FAST = 0, KM_ACC = 1, KM_MIX = 2 };

// Whether a plain launch of mode KM serves the signal of tables `tabs`.
template <int KM>
__device__ __forceinline__ bool plain_launch_serves(const FwdArgs &a)
{
    if (a.B == 0 && a.skip_gate && ctab(a.skip_gate)[0] != 0.0f) return false;
    if (KM == KM_MIX || a.B != 0 || a.K <= 0) return true;
    const bool acc = tab_word(reinterpret_cast<const unsigned char *>(a.tabs), HDR_MODE) ==
                     MODE_ACCURATE;
    return acc == (KM == KM_ACC);
}

template <typename T, int N, int W, int ALG, int KM>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(min_waves_per_simd<T, N, W>())))
    sos_fwd_kernel(FwdArgs a)
{
    if (!plain_launch_serves<KM>(a)) return;   // before anything: no ticket, no exit count
    constexpr int RS = N + 4;
    constexpr int CW = kLanes * N;
    constexpr int C = CW * W;
    __shared__ float tile[W][kLanes * RS];
    __shared__ Xch<T, W> xch;
    __shared__ int64_t ticket;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar addressing
    const unsigned epoch = __hip_atomic_load(&a.ctrl[CTRL_EPOCH], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    const int64_t total = a.B > 0 ? *a.total_dev : a.total;
    float *tl = tile[wv];
    const unsigned char *tabs = reinterpret_cast<const unsigned char *>(a.tabs);
    // Software pipeline over groups (FP32 compute): the next ticket is drawn
    // when the current group's last state is resolved, and its samples are
    // loaded into registers while this group is corrected and stored.
    constexpr bool kPrefetch = sizeof(T) == 4;
    const bool draw = kPrefetch && (int64_t)gridDim.x < total;
    f4 pf[N / 4];     // coalesced slots of ticket tn
    int64_t tn = -1;  // ticket drawn by the previous group, or -1

    for (;;) {
        int64_t t = tn;
        if (t < 0) {
            if (threadIdx.x == 0) ticket = (int64_t)atomicAdd(&a.ctrl[CTRL_TICKET], 1u);
            lds_barrier();
            t = ticket;
            lds_barrier();
        }
        if (t >= total) break;
        const Item<T> it = make_item<T>(a, tabs, t);
        const int64_t g0 = it.g * C + (int64_t)wv * CW;
        // load: coalesced 128-bit global loads -> the wave's LDS rows -> registers
        if (tn < 0) tile_fetch<N>(pf, it.x + g0, it.n - g0, lane);
        tile_put<N>(pf, tl, lane);
        tn = -1;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        T u[N];
        regs_from_rows<T, N>(u, tl, lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // The next group's slots live in a buffer of this iteration that starts
        // unspecified and is copied to pf unconditionally at the end, so that
        // pf holds no registers while the group is filtered.
        f4 nf[N / 4];
#pragma unroll
        for (int j = 0; j < N / 4; ++j) nf[j] = __builtin_nondeterministic_value(f4{});
        auto on_next = [&](int64_t nx) {
            tn = nx;
            if (nx < total) {
                const Item<T> ni = make_item<T>(a, tabs, nx);
                const int64_t h0 = ni.g * C + (int64_t)wv * CW;
                tile_fetch<N>(nf, ni.x + h0, ni.n - h0, lane);
            }
        };
        // The signal's table layout picks the path, once per group: the
        // accurate layout (FP32 compute only) runs PH with its state work in
        // FP64, the fast one the launch's solver in the compute type. FAST and
        // ACC launches hold one path only (each has the registers to itself);
        // MIX launches pick per group.
        if constexpr (sizeof(T) == 4 && KM != KM_FAST) {
            if (KM == KM_ACC || (it.K > 0 && tab_word(it.tabs, HDR_MODE) == MODE_ACCURATE))
                finish_group<T, true, N, W, ALG_PH>(a, it, u, tl, xch, epoch, wv, lane, draw,
                                                    on_next);
            else
                finish_group<T, false, N, W, ALG>(a, it, u, tl, xch, epoch, wv, lane, draw,
                                                  on_next);
        } else {
            finish_group<T, false, N, W, ALG>(a, it, u, tl, xch, epoch, wv, lane, draw, on_next);
        }
#pragma unroll
        for (int j = 0; j < N / 4; ++j) pf[j] = nf[j];
        if ((int64_t)gridDim.x >= total) break;   // one group per workgroup: no extra draw
    }
    if (a.B == 0 && threadIdx.x == 0) rearm_on_exit(a.ctrl, epoch);
}

// ---------------------------------------------------------------------------
// Adjoint (vector-Jacobian product) of the cascade.
//
// For section k (last to first), in reversed time r = n-1-t:
//   lam'[r]  = g'[r] - a1 lam'[r-1] - a2 lam'[r-2]    (lam'[-1], lam'[-2]) = gzf[k]
//   g_prev'[r] = b0 lam'[r] + b1 lam'[r-1] + b2 lam'[r-2]
//   d/db_i  = sum_r lam'[r-i] u'[r],  d/da_i = -sum_r lam'[r-i] v'[r]
//   d/dzi   = (lam'[n-1], lam'[n-2])
// with u, v the section's forward input and output. The first line is a plain
// recursive section run by the same multi-block machinery (PAIR carries) on
// groups aligned to the end of the signal, so the initial carry enters at the
// last real sample and the zero padding falls before sample 0.
struct BwdArgs {
    const float *gy;
    float *gx;
    int64_t n;
    const void *tabs;        // PAIR tables of the K sections (compute type)
    const float *x;          // forward input
    const float *y;          // forward output
    const float *saved;      // outputs of sections 0..K-2, (K-1) x n
    const float *gzf;        // K x 2 or null
    float *gzi;              // K x 2 or null
    double *partials;        // total x K x 5 per-group coefficient sums
    unsigned long long *desc;
    int64_t dstride;         // descriptor slots per section
    unsigned *ctrl;
    int K;                   // plain: sections; batched: stride (max sections)
    int64_t total;
    unsigned long long timeout_ticks;
    // batched mode (B > 0): per-signal arrays and the work table (reversed groups)
    int B;
    const int32_t *Ks;
    const int32_t *sec_off;
    const int64_t *sig_off;
    const int64_t *gpre;
    const int32_t *sigmap;
    const int64_t *total_dev;
    int64_t saved_stride;    // distance between the saved outputs of two sections
};

// One reversed-time group of one signal.
template <typename T>
struct BItem {
    Item<T> it;              // t, g, n, K, tabs, zi = the final-state cotangent
    const float *gy, *x, *y, *saved;
    float *gx, *gzi;
};

template <typename T>
__device__ __forceinline__ BItem<T> make_bwd_item(const BwdArgs &b, const unsigned char *tabs,
                                                  int64_t t)
{
    BItem<T> r{};
    r.it.t = t;
    if (b.B == 0) {
        r.it.n = b.n;
        r.it.g = t;
        r.it.K = b.K;
        r.it.tabs = tabs;
        r.it.zi = b.gzf;
        r.gy = b.gy;
        r.gx = b.gx;
        r.x = b.x;
        r.y = b.y;
        r.saved = b.saved;
        r.gzi = b.gzi;
    } else {
        const int i = b.sigmap[t];
        r.it.sig = i;
        const int64_t so = b.sig_off[i];
        const int32_t sc = b.sec_off[i];
        r.it.n = b.sig_off[i + 1] - so;
        r.it.g = t - b.gpre[i];
        r.it.K = b.Ks[i];
        r.it.tabs = tabs + (size_t)sc * TAB_BYTES;
        r.it.zi = b.gzf ? b.gzf + 2 * (int64_t)sc : nullptr;
        r.gy = b.gy + so;
        r.gx = b.gx + so;
        r.x = b.x + so;
        r.y = b.y + so;
        r.saved = b.saved ? b.saved + so : nullptr;
        r.gzi = b.gzi ? b.gzi + 2 * (int64_t)sc : nullptr;
    }
    return r;
}

// Reversed time without reversed memory traffic. The wave's part in reversed
// time, reversed indices [r0, r0 + 64N), is the forward window
// [n - r0 - 64N, n - r0); lane l's reversed samples l N .. l N + N - 1 are
// forward row 63 - l of that window read backwards. So the window moves with
// the same coalesced 128-bit accesses and padded LDS rows as the forward
// filter, and only the row read is mirrored. Samples before forward index 0
// (the padding of the last reversed group) read as 0 and are not written.

// src[start .. start + 64N) -> tile, zero outside [0, n).
template <int N>
__device__ __forceinline__ void window_load(const float *src, int64_t start, int64_t n, float *tl,
                                            int lane)
{
    if (start >= 0) {
        tile_load<N>(src + start, n - start, tl, lane);
        return;
    }
    using TT = WaveTile<N>;
    float *p = tl + TT::slot_base(lane);
#pragma unroll
    for (int j = 0; j < TT::Q; ++j) {
        const int64_t q = start + 4 * (int64_t)(kLanes * j + lane);
        f4 t;
        t.x = q + 0 >= 0 && q + 0 < n ? gptr(src)[q + 0] : 0.0f;
        t.y = q + 1 >= 0 && q + 1 < n ? gptr(src)[q + 1] : 0.0f;
        t.z = q + 2 >= 0 && q + 2 < n ? gptr(src)[q + 2] : 0.0f;
        t.w = q + 3 >= 0 && q + 3 < n ? gptr(src)[q + 3] : 0.0f;
        *reinterpret_cast<f4 *>(p + j * TT::STEP) = t;
    }
}

// tile -> dst[start .. start + 64N) restricted to [0, n).
template <int N>
__device__ __forceinline__ void window_store(float *dst, int64_t start, int64_t n,
                                             const float *tl, int lane)
{
    if (start >= 0) {
        tile_store<N, true>(dst + start, n - start, tl, lane);
        return;
    }
    using TT = WaveTile<N>;
    const float *p = tl + TT::slot_base(lane);
#pragma unroll
    for (int j = 0; j < TT::Q; ++j) {
        const int64_t q = start + 4 * (int64_t)(kLanes * j + lane);
        const f4 t = *reinterpret_cast<const f4 *>(p + j * TT::STEP);
        if (q + 0 >= 0 && q + 0 < n) gptr(dst)[q + 0] = t.x;
        if (q + 1 >= 0 && q + 1 < n) gptr(dst)[q + 1] = t.y;
        if (q + 2 >= 0 && q + 2 < n) gptr(dst)[q + 2] = t.z;
        if (q + 3 >= 0 && q + 3 < n) gptr(dst)[q + 3] = t.w;
    }
}

// Lane l's N registers <-> forward row 63 - l of the tile, mirrored.
template <typename T, int N>
__device__ __forceinline__ void regs_from_rows_rev(T (&u)[N], const float *tl, int lane)
{
    const float *row = tl + (kLanes - 1 - lane) * WaveTile<N>::RS;
#pragma unroll
    for (int k = 0; k < N / 4; ++k) {
        const f4 v = *reinterpret_cast<const f4 *>(row + 4 * k);
        u[N - 1 - 4 * k] = v.x;
        u[N - 2 - 4 * k] = v.y;
        u[N - 3 - 4 * k] = v.z;
        u[N - 4 - 4 * k] = v.w;
    }
}
template <typename T, int N>
__device__ __forceinline__ void rows_from_regs_rev(const T (&u)[N], float *tl, int lane)
{
    float *row = tl + (kLanes - 1 - lane) * WaveTile<N>::RS;
#pragma unroll
    for (int k = 0; k < N / 4; ++k) {
        const f4 v = {(float)u[N - 1 - 4 * k], (float)u[N - 2 - 4 * k], (float)u[N - 3 - 4 * k],
                      (float)u[N - 4 - 4 * k]};
        *reinterpret_cast<f4 *>(row + 4 * k) = v;
    }
}

template <typename T, int N, int W, int ALG, int KM>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && W >= 4 ? 2 : 1)))
    sos_bwd_kernel(BwdArgs b)
{
    if (KM != KM_MIX && b.B == 0 && b.K > 0 &&
        (tab_word(reinterpret_cast<const unsigned char *>(b.tabs), HDR_MODE) == MODE_ACCURATE) !=
            (KM == KM_ACC))
        return;   // a plain launch for the other layout: before anything
    constexpr int RS = N + 4;
    constexpr int CW = kLanes * N;
    constexpr int C = CW * W;
    __shared__ float tile[W][kLanes * RS];
    __shared__ float tile2[W][kLanes * RS];
    __shared__ Xch<T, W> xch;
    __shared__ int64_t ticket;
    __shared__ double red[W][5];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar addressing
    const unsigned epoch = __hip_atomic_load(&b.ctrl[CTRL_EPOCH], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    const int64_t total = b.B > 0 ? *b.total_dev : b.total;
    float *tl = tile[wv];
    float *tl2 = tile2[wv];
    const unsigned char *tabs = reinterpret_cast<const unsigned char *>(b.tabs);
    FwdArgs a{};                 // the fields the section step and lookback use
    a.K = b.K;
    a.desc = b.desc;
    a.dstride = b.dstride;
    a.ctrl = b.ctrl;
    a.timeout_ticks = b.timeout_ticks;

    for (;;) {
        if (threadIdx.x == 0) ticket = (int64_t)atomicAdd(&b.ctrl[CTRL_TICKET], 1u);
        lds_barrier();
        const int64_t t = ticket;
        lds_barrier();
        if (t >= total) break;
        const BItem<T> bi = make_bwd_item<T>(b, tabs, t);
        const Item<T> &it = bi.it;
        const int64_t n = it.n;
        bool bad = false;
        for (int k = 0; k < it.K; ++k)
            bad |= tab_word(it.tabs + (size_t)k * TAB_BYTES, HDR_STATUS) != 0ull;
        const int64_t r0 = it.g * C + (int64_t)wv * CW;   // reversed index of the wave's start
        const int64_t f0 = n - r0 - CW;                   // forward index of the window's start

        window_load<N>(bi.gy, f0, n, tl, lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        T u[N];
        regs_from_rows_rev<T, N>(u, tl, lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // lane / position of reversed index n-1 (forward sample 0) if this wave holds it
        const int64_t pz = (n - 1) - r0;
        const bool has_first = pz >= 0 && pz < CW;
        const int zl = has_first ? (int)(pz / N) : 0, zp = has_first ? (int)(pz % N) : 0;
        const int64_t sst = b.B > 0 ? b.saved_stride : n;

        // The section's forward input and output over the window, in the
        // wave's two tiles. The input of section k is the output of section
        // k - 1, so it stays staged for the next (lower) section, whose
        // output tile it becomes: each signal is read from HBM once.
        // The last section's two windows are loaded back to back, so that
        // their global loads are in flight together.
        float *tin = tl, *tout = tl2;
        if (!bad && it.K > 0) {
            const int k = it.K - 1;
            window_load<N>(k == 0 ? bi.x : bi.saved + (size_t)(k - 1) * sst, f0, n, tin, lane);
            window_load<N>(bi.y, f0, n, tout, lane);
        }
        // the sections, last to first, in the signal's table layout (see the
        // forward kernel)
        auto cascade = [&](auto acc_tag) {
            constexpr bool ACC = decltype(acc_tag)::value;
            using LY = Lay<T, ACC>;
            for (int k = it.K - 1; k >= 0 && !bad; --k) {
                const unsigned char *tb = it.tabs + (size_t)k * TAB_BYTES;
                ctabT<T> *tab = ctabp(LY::sp(tb));
                if (k < it.K - 1)
                    window_load<N>(k == 0 ? bi.x : bi.saved + (size_t)(k - 1) * sst, f0, n, tin, lane);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                T q1, q2;   // lam'[-2], lam'[-1] of this lane
                // (the pair section reads and writes no tile)
                run_section<T, ACC, N, W, true, ACC ? ALG_PH : ALG>(u, xch, tout, a, it, tb, k, epoch,
                                                                     wv, lane, false, 0, 0, q1, q2);
                // coefficient sums over the lane (reversed position m = forward column N-1-m)
                T s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
                const float *ru = tin + (kLanes - 1 - lane) * RS;
                const float *rv = tout + (kLanes - 1 - lane) * RS;
    #pragma unroll
                for (int k4 = 0; k4 < N / 4; ++k4) {
                    const f4 U = *reinterpret_cast<const f4 *>(ru + 4 * k4);
                    const f4 V = *reinterpret_cast<const f4 *>(rv + 4 * k4);
                    const float uq[4] = {U.w, U.z, U.y, U.x};
                    const float vq[4] = {V.w, V.z, V.y, V.x};
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int m = N - 4 - 4 * k4 + i;
                        const T L0 = u[m];
                        const T L1 = m >= 1 ? u[m - 1] : q2;
                        const T L2 = m >= 2 ? u[m - 2] : (m == 1 ? q2 : q1);
                        const T uu = uq[i], vv = vq[i];
                        s0 = fmaT(L0, uu, s0);
                        s1 = fmaT(L1, uu, s1);
                        s2 = fmaT(L2, uu, s2);
                        s3 = fmaT(-L1, vv, s3);
                        s4 = fmaT(-L2, vv, s4);
                    }
                }
                // d/dzi = (lam'[n-1], lam'[n-2]); scratch: the output tile, already
                // consumed (the input tile is kept for the next section)
                if (has_first && bi.gzi) {
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    T l1 = 0, l2 = 0;
                    pick_two<T, N>(u, tout, lane, zl, zp, l1, l2);
                    if (lane == zl) {
                        gptr(bi.gzi)[2 * k] = (float)l1;
                        gptr(bi.gzi)[2 * k + 1] = (float)(zp >= 1 ? l2 : q2);
                    }
                }
                // gradient for the section below: 3-tap FIR of lam' (descending, in place)
                const T f0c = tab[LY::P_FIR + 0], f1c = tab[LY::P_FIR + 1], f2c = tab[LY::P_FIR + 2];
    #pragma unroll
                for (int m = N - 1; m >= 0; --m) {
                    const T L1 = m >= 1 ? u[m - 1] : q2;
                    const T L2 = m >= 2 ? u[m - 2] : (m == 1 ? q2 : q1);
                    u[m] = fmaT(f0c, u[m], fmaT(f1c, L1, f2c * L2));
                }
                // group partial sums (waves combined in FP64); in the accurate
                // layout FP64 from the lanes' partials on: the sums cancel heavily
                // for lightly damped sections, and FP32 sums over whole waves
                // lose what the FP32 samples still hold
                using SS = typename LY::S;
                const double w0 = wave_sum<SS>((SS)s0), w1 = wave_sum<SS>((SS)s1);
                const double w2 = wave_sum<SS>((SS)s2), w3 = wave_sum<SS>((SS)s3);
                const double w4 = wave_sum<SS>((SS)s4);
                if (lane == 0) {
                    red[wv][0] = w0;
                    red[wv][1] = w1;
                    red[wv][2] = w2;
                    red[wv][3] = w3;
                    red[wv][4] = w4;
                }
                lds_barrier();
                if (threadIdx.x < 5) {
                    double acc = 0.0;
                    for (int v = 0; v < W; ++v) acc += red[v][threadIdx.x];
                    b.partials[((size_t)t * b.K + k) * 5 + threadIdx.x] = acc;
                }
                // this section's input tile is the next section's output tile;
                // the other one is re-staged with the next input (wave-local, ordered)
                float *const tsw = tin;
                tin = tout;
                tout = tsw;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        };
        if constexpr (sizeof(T) == 4 && KM != KM_FAST) {
            if (KM == KM_ACC || (!bad && it.K > 0 && tab_word(it.tabs, HDR_MODE) == MODE_ACCURATE))
                cascade(BoolTag<true>{});
            else
                cascade(BoolTag<false>{});
        } else {
            cascade(BoolTag<false>{});
        }
        if (bad) {
#pragma unroll
            for (int m = 0; m < N; ++m) u[m] = T(__builtin_nanf(""));
            for (int i = threadIdx.x; i < 5 * it.K; i += blockDim.x)
                b.partials[(size_t)t * b.K * 5 + i] = __builtin_nan("");
        }
        // store dL/dx in forward order through the wave's rows
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        rows_from_regs_rev<T, N>(u, tl, lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        window_store<N>(bi.gx, f0, n, tl, lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if ((int64_t)gridDim.x >= total) break;
    }
    if (threadIdx.x == 0) rearm_on_exit(b.ctrl, epoch);
}

// Sum the per-group coefficient partials of section k in FP64 (fixed order)
// and apply the chain rule through the division by a0. Grid = (K), block 256.
__global__ void __launch_bounds__(256)
sos_bwd_reduce_kernel(const double *partials, int64_t total, int K, const float *sections,
                      float *gsections)
{
    __shared__ double sh[256][5];
    const int k = blockIdx.x;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t t = threadIdx.x; t < total; t += 256)
        for (int i = 0; i < 5; ++i) acc[i] += partials[((size_t)t * K + k) * 5 + i];
    for (int i = 0; i < 5; ++i) sh[threadIdx.x][i] = acc[i];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d)
            for (int i = 0; i < 5; ++i) sh[threadIdx.x][i] += sh[threadIdx.x + d][i];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float *row = sections + 6 * k;
        const double a0 = row[3];
        const double bn0 = row[0] / a0, bn1 = row[1] / a0, bn2 = row[2] / a0;
        const double an1 = row[4] / a0, an2 = row[5] / a0;
        const double *g = sh[0];
        float *o = gsections + 6 * k;
        o[0] = (float)(g[0] / a0);
        o[1] = (float)(g[1] / a0);
        o[2] = (float)(g[2] / a0);
        o[4] = (float)(g[3] / a0);
        o[5] = (float)(g[4] / a0);
        o[3] = (float)(-(g[0] * bn0 + g[1] * bn1 + g[2] * bn2 + g[3] * an1 + g[4] * an2) / a0);
    }
}

// Batched form: block (i, k) sums section k of signal i over the signal's
// tickets gpre[i] .. gpre[i+1]-1 (fixed order) and applies the a0 chain rule.
// Signals the work table skipped are skipped here too: inconsistent ones
// (their section rows may lie outside the arrays), and every signal of a
// table rejected as a whole (its groups then run past gpre[B], which is 0).
__global__ void __launch_bounds__(256)
sos_bwd_reduce_batched_kernel(const double *partials, int B, int kmax, int64_t rows,
                              int64_t total_samples, const int32_t *Ks, const int32_t *sec_off,
                              const int64_t *sig_off, const int64_t *gpre, const float *sections,
                              float *gsections, double *grow)
{
    __shared__ double sh[256][5];
    const int i = blockIdx.x, k = blockIdx.y;
    // uniform per block; a (signal, section) pair without a gradient leaves
    // zeros in the FP64 rows, which are summed over signals afterwards
    bool ok = i < B && batch_signal_ok(i, kmax, rows, total_samples, Ks, sec_off, sig_off) &&
              k < Ks[i];
    const int64_t t0 = ok ? gpre[i] : 0, t1 = ok ? gpre[i + 1] : 0;
    ok = ok && t0 <= t1 && t1 <= gpre[B];
    if (!ok) {
        if (grow && threadIdx.x < 6 && i < B) grow[((size_t)i * kmax + k) * 6 + threadIdx.x] = 0.0;
        return;
    }
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256)
        for (int c = 0; c < 5; ++c) acc[c] += partials[((size_t)t * kmax + k) * 5 + c];
    for (int c = 0; c < 5; ++c) sh[threadIdx.x][c] = acc[c];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d)
            for (int c = 0; c < 5; ++c) sh[threadIdx.x][c] += sh[threadIdx.x + d][c];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t row_i = (int64_t)sec_off[i] + k;
        const float *row = sections + 6 * row_i;
        const double a0 = row[3];
        const double bn0 = row[0] / a0, bn1 = row[1] / a0, bn2 = row[2] / a0;
        const double an1 = row[4] / a0, an2 = row[5] / a0;
        const double *g = sh[0];
        const double v[6] = {g[0] / a0, g[1] / a0, g[2] / a0,
                             -(g[0] * bn0 + g[1] * bn1 + g[2] * bn2 + g[3] * an1 + g[4] * an2) /
                                 a0,
                             g[3] / a0, g[4] / a0};
        if (gsections)
            for (int c = 0; c < 6; ++c) gsections[6 * row_i + c] = (float)v[c];
        if (grow)
            for (int c = 0; c < 6; ++c) grow[((size_t)i * kmax + k) * 6 + c] = v[c];
    }
}

// Sum over the signals of each section's coefficient gradient, for a batch
// whose signals share one cascade: block k adds the FP64 rows of every signal
// in a fixed order (strided partial sums, then a tree) and rounds once.
__global__ void __launch_bounds__(256)
sos_bwd_sum_rows_kernel(const double *grow, int B, int kmax, float *gsum)
{
    __shared__ double sh[256][6];
    const int k = blockIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < B; i += 256)
        for (int c = 0; c < 6; ++c) acc[c] += grow[((size_t)i * kmax + k) * 6 + c];
    for (int c = 0; c < 6; ++c) sh[threadIdx.x][c] = acc[c];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d)
            for (int c = 0; c < 6; ++c) sh[threadIdx.x][c] += sh[threadIdx.x + d][c];
        __syncthreads();
    }
    if (threadIdx.x < 6) gsum[6 * k + threadIdx.x] = (float)sh[0][threadIdx.x];
}

// ------------------------------------------------------------------ launch

// The forward kernel of a launch: the solver, and whether the tables may use
// the accurate layout (FP32 only): plain launches of at least kMixPlainGroups
// groups then take the fast kernel and the accurate one back to back (the one
// not needed leaves at once), batched and shorter plain launches the kernel
// that chooses per group.
constexpr int64_t kMixPlainGroups = 512;   // plain launches of fewer groups: per-group kernel

template <typename T, int N, int W>
hipError_t launch_fwd(int alg, const FwdArgs &a, int64_t grid, hipStream_t stream)
{
    const bool maybe_acc = sizeof(T) == 4 && (alg & ALG_MAYBE_ACC);
    const bool ph = (alg & ~ALG_MAYBE_ACC) == ALG_PH;
    const dim3 g((unsigned)grid), blk(64 * W);
    // short plain launches too: the second kernel's launch and exit cost more
    // than the per-group choice there (same-box A/B, order 2: 8.8 -> 7.3 us
    // per call at 2^16 samples, 11.6 -> 10.2 at 2^20, equal at 2^24, 3 %
    // slower at 2^28)
    if (maybe_acc && (a.B > 0 || a.total < kMixPlainGroups)) {
        if (ph)
            hipLaunchKernelGGL((sos_fwd_kernel<T, N, W, ALG_PH, KM_MIX>), g, blk, 0, stream, a);
        else
            hipLaunchKernelGGL((sos_fwd_kernel<T, N, W, ALG_DCCR, KM_MIX>), g, blk, 0, stream, a);
        return hipGetLastError();
    }
    if (ph)
        hipLaunchKernelGGL((sos_fwd_kernel<T, N, W, ALG_PH, KM_FAST>), g, blk, 0, stream, a);
    else
        hipLaunchKernelGGL((sos_fwd_kernel<T, N, W, ALG_DCCR, KM_FAST>), g, blk, 0, stream, a);
    if (maybe_acc) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((sos_fwd_kernel<T, N, W, ALG_PH, KM_ACC>), g, blk, 0, stream, a);
    }
    return hipGetLastError();
}

// The forward kernel a launch of `alg` runs (for batched launches: the one
// that chooses the layout per group when the tables may be accurate).
template <typename T, int N, int W>
const void *kernel_of(int alg)
{
    const bool mix = sizeof(T) == 4 && (alg & ALG_MAYBE_ACC);
    const bool ph = (alg & ~ALG_MAYBE_ACC) == ALG_PH;
    return mix ? (ph ? (const void *)sos_fwd_kernel<T, N, W, ALG_PH, KM_MIX>
                     : (const void *)sos_fwd_kernel<T, N, W, ALG_DCCR, KM_MIX>)
               : (ph ? (const void *)sos_fwd_kernel<T, N, W, ALG_PH, KM_FAST>
                     : (const void *)sos_fwd_kernel<T, N, W, ALG_DCCR, KM_FAST>);
}

template <typename T, int N, int W>
int attrs_of(int alg, int *regs, int *lds)
{
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, kernel_of<T, N, W>(alg)) != hipSuccess) return SOS_EHIP;
    if (regs) *regs = fa.numRegs;
    if (lds) *lds = (int)fa.sharedSizeBytes;
    return SOS_OK;
}

template <typename T, int N, int W>
int capacity_of(int alg)
{
    int per_cu = 0, dev = 0, cus = 0;
    const void *kern = kernel_of<T, N, W>(alg);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * W, 0) != hipSuccess)
        per_cu = 1;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    return (per_cu > 0 ? per_cu : 1) * cus;
}

// Group shapes compiled into the library (N samples per lane, W waves).
#define SOS_SHAPES(X)                                                                     \
    X(16, 1) X(32, 1) X(64, 1) X(16, 4) X(32, 4) X(64, 4) X(16, 8) X(32, 8) X(64, 8)    \
        X(16, 16) X(32, 16)

hipError_t dispatch_fwd(int bits, int alg, int L, int N, const FwdArgs &a, int64_t grid,
                        hipStream_t stream)
{
    const int W = L / 64;
#define SOS_CASE(NN, WW)                                                                  \
    if (N == NN && W == WW)                                                               \
        return bits == 64 ? launch_fwd<double, NN, WW>(alg, a, grid, stream)              \
                          : launch_fwd<float, NN, WW>(alg, a, grid, stream);
    SOS_SHAPES(SOS_CASE)
#undef SOS_CASE
    return hipErrorInvalidValue;
}

}  // namespace

extern "C" int sos_fwd_shape_supported(int L, int N)
{
    if (L % 64) return 0;
    const int W = L / 64;
#define SOS_CASE(NN, WW)                                                                  \
    if (N == NN && W == WW) return 1;
    SOS_SHAPES(SOS_CASE)
#undef SOS_CASE
    return 0;
}

// Vector registers per lane and static LDS bytes of the forward kernel of
// shape (L, N).
extern "C" int sos_fwd_kernel_attrs(int bits, int alg, int L, int N, int *regs, int *lds)
{
    if (L <= 0 || (L % 64)) return SOS_EINVAL;
    const int W = L / 64;
#define SOS_CASE(NN, WW)                                                                  \
    if (N == NN && W == WW) return bits == 64 ? attrs_of<double, NN, WW>(alg, regs, lds)   \
                                              : attrs_of<float, NN, WW>(alg, regs, lds);
    SOS_SHAPES(SOS_CASE)
#undef SOS_CASE
    return SOS_EINVAL;
}

// Workgroups of shape (L, N) that can be resident on the whole device at once.
extern "C" int sos_fwd_capacity(int bits, int alg, int L, int N)
{
    const int W = L / 64;
#define SOS_CASE(NN, WW)                                                                  \
    if (N == NN && W == WW) return bits == 64 ? capacity_of<double, NN, WW>(alg)           \
                                              : capacity_of<float, NN, WW>(alg);
    SOS_SHAPES(SOS_CASE)
#undef SOS_CASE
    return 0;
}

// Plain filter of one signal; grid <= 0 means one workgroup per group.
extern "C" hipError_t sos_launch_fwd(int bits, int alg, int L, int N, const float *x, float *y,
                                     int64_t n, int64_t groups, const void *tabs, int K,
                                     const float *zi, float *zf, unsigned long long *desc,
                                     unsigned *ctrl,
                                     unsigned long long timeout_ticks, int64_t grid, float *saved,
                                     const float *skip_gate, hipStream_t stream)
{
    FwdArgs a{};
    a.skip_gate = skip_gate;
    a.saved = saved;
    a.saved_stride = n;
    a.x = x;
    a.y = y;
    a.n = n;
    a.tabs = tabs;
    a.zi = zi;
    a.zf = zf;
    a.K = K;
    a.B = 0;
    a.total = groups;
    a.desc = desc;
    a.dstride = groups;
    a.ctrl = ctrl;
    a.timeout_ticks = timeout_ticks;
    if (grid <= 0 || grid > groups) grid = groups;
    return dispatch_fwd(bits, alg, L, N, a, grid, stream);
}

// Uneven batch in one persistent launch. The work table (gpre, sigmap,
// *total_dev) is produced on the device by sos_launch_worktable.
extern "C" hipError_t sos_launch_fwd_batched(int bits, int alg, int L, int N, int B, int kmax,
                                             const int32_t *Ks, const int32_t *sec_off,
                                             const int64_t *sig_off, const int64_t *gpre,
                                             const int32_t *sigmap, const int64_t *total_dev,
                                             const float *x, float *y, const void *tabs,
                                             const float *zi, float *zf,
                                             unsigned long long *desc, unsigned *ctrl,
                                             unsigned long long timeout_ticks, int64_t grid,
                                             const float *const *xp, float *const *yp,
                                             float *saved, int64_t saved_stride,
                                             int64_t max_groups, unsigned *sig_err,
                                             hipStream_t stream)
{
    FwdArgs a{};
    a.x = x;
    a.y = y;
    a.xp = xp;
    a.yp = yp;
    a.sig_err = sig_err;
    a.saved = saved;
    a.saved_stride = saved_stride;
    a.tabs = tabs;
    a.zi = zi;
    a.zf = zf;
    a.K = kmax;
    a.B = B;
    a.Ks = Ks;
    a.sec_off = sec_off;
    a.sig_off = sig_off;
    a.gpre = gpre;
    a.sigmap = sigmap;
    a.total_dev = total_dev;
    a.desc = desc;
    a.dstride = max_groups;
    a.ctrl = ctrl;
    a.timeout_ticks = timeout_ticks;
    return dispatch_fwd(bits, alg, L, N, a, grid, stream);
}

// Launch the adjoint kernel of shape (L, N) in the compute type; grid <= 0:
// persistent (as many workgroups as can be resident), at most `groups`.
static hipError_t launch_bwd_args(int bits, int alg, int L, int N, const BwdArgs &b,
                                  int64_t groups, int64_t grid, hipStream_t stream)
{
    const int W = L / 64;
    // grid <= 0: persistent, as many workgroups as can be resident
    auto resident = [&](const void *kern, int threads) -> int64_t {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        return (int64_t)per_cu * cus;
    };
    auto launch = [&](auto kern, int threads) {
        if (grid <= 0) grid = resident((const void *)kern, threads);
        if (grid > groups) grid = groups;
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), 0, stream, b);
        return hipGetLastError();
    };
    // the same choice of kernels as the forward launch (launch_fwd)
    const bool maybe_acc = bits != 64 && (alg & ALG_MAYBE_ACC);
    const bool ph = (alg & ~ALG_MAYBE_ACC) == ALG_PH;
    auto launch3 = [&](auto kfast_dccr, auto kfast_ph, auto kmix_dccr, auto kmix_ph, auto kacc,
                       int threads) {
        if (maybe_acc && b.B > 0) return ph ? launch(kmix_ph, threads) : launch(kmix_dccr, threads);
        const int64_t grid0 = grid;
        hipError_t e = ph ? launch(kfast_ph, threads) : launch(kfast_dccr, threads);
        if (e != hipSuccess || !maybe_acc) return e;
        grid = grid0;
        return launch(kacc, threads);
    };
#define SOS_BWD_CASE(NN, WW)                                                                   \
    if (N == NN && W == WW) {                                                                  \
        if (bits == 64)                                                                        \
            return ph ? launch(sos_bwd_kernel<double, NN, WW, ALG_PH, KM_FAST>, 64 * WW)       \
                      : launch(sos_bwd_kernel<double, NN, WW, ALG_DCCR, KM_FAST>, 64 * WW);    \
        return launch3(sos_bwd_kernel<float, NN, WW, ALG_DCCR, KM_FAST>,                       \
                       sos_bwd_kernel<float, NN, WW, ALG_PH, KM_FAST>,                         \
                       sos_bwd_kernel<float, NN, WW, ALG_DCCR, KM_MIX>,                        \
                       sos_bwd_kernel<float, NN, WW, ALG_PH, KM_MIX>,                          \
                       sos_bwd_kernel<float, NN, WW, ALG_PH, KM_ACC>, 64 * WW);                \
    }
    SOS_BWD_CASE(16, 1)
    SOS_BWD_CASE(32, 1)
    SOS_BWD_CASE(16, 4)
    SOS_BWD_CASE(32, 4)
    SOS_BWD_CASE(16, 8)
    SOS_BWD_CASE(32, 8)
#undef SOS_BWD_CASE
    return hipErrorInvalidValue;
}

// Adjoint of the plain filter: grid <= 0 means a persistent grid.
extern "C" hipError_t sos_launch_bwd(int bits, int alg, int L, int N, const float *gy, float *gx,
                                     int64_t n, int64_t groups, const void *tabs, int K,
                                     const float *x, const float *y, const float *saved,
                                     const float *gzf, float *gzi, double *partials,
                                     unsigned long long *desc, unsigned *ctrl,
                                     unsigned long long timeout_ticks, int64_t grid,
                                     hipStream_t stream)
{
    BwdArgs b{};
    b.gy = gy;
    b.gx = gx;
    b.n = n;
    b.tabs = tabs;
    b.x = x;
    b.y = y;
    b.saved = saved;
    b.gzf = gzf;
    b.gzi = gzi;
    b.partials = partials;
    b.desc = desc;
    b.dstride = groups;
    b.ctrl = ctrl;
    b.K = K;
    b.total = groups;
    b.timeout_ticks = timeout_ticks;
    return launch_bwd_args(bits, alg, L, N, b, groups, grid, stream);
}

// Batched adjoint: one persistent launch over the reversed groups of every
// signal (work table built by sos_launch_worktable with the adjoint's C).
extern "C" hipError_t sos_launch_bwd_batched(int bits, int alg, int L, int N, int B, int kmax,
                                             const int32_t *Ks, const int32_t *sec_off,
                                             const int64_t *sig_off, const int64_t *gpre,
                                             const int32_t *sigmap, const int64_t *total_dev,
                                             int64_t max_groups, const float *gy, float *gx,
                                             const void *tabs, const float *x, const float *y,
                                             const float *saved, int64_t saved_stride,
                                             const float *gzf, float *gzi, double *partials,
                                             unsigned long long *desc, unsigned *ctrl,
                                             unsigned long long timeout_ticks,
                                             hipStream_t stream)
{
    BwdArgs b{};
    b.gy = gy;
    b.gx = gx;
    b.tabs = tabs;
    b.x = x;
    b.y = y;
    b.saved = saved;
    b.gzf = gzf;
    b.gzi = gzi;
    b.partials = partials;
    b.desc = desc;
    b.dstride = max_groups;
    b.ctrl = ctrl;
    b.K = kmax;
    b.timeout_ticks = timeout_ticks;
    b.B = B;
    b.Ks = Ks;
    b.sec_off = sec_off;
    b.sig_off = sig_off;
    b.gpre = gpre;
    b.sigmap = sigmap;
    b.total_dev = total_dev;
    b.saved_stride = saved_stride;
    return launch_bwd_args(bits, alg, L, N, b, max_groups, 0, stream);
}

extern "C" hipError_t sos_launch_bwd_reduce_batched(const double *partials, int B, int kmax,
                                                    int64_t rows, int64_t total_samples,
                                                    const int32_t *Ks, const int32_t *sec_off,
                                                    const int64_t *sig_off, const int64_t *gpre,
                                                    const float *sections, float *gsections,
                                                    double *grow, float *gsum,
                                                    hipStream_t stream)
{
    if (B <= 0 || kmax <= 0) return hipSuccess;
    if (gsum && !grow) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sos_bwd_reduce_batched_kernel, dim3((unsigned)B, (unsigned)kmax),
                       dim3(256), 0, stream, partials, B, kmax, rows, total_samples, Ks, sec_off,
                       sig_off, gpre, sections, gsections, gsum ? grow : nullptr);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    if (gsum)
        hipLaunchKernelGGL(sos_bwd_sum_rows_kernel, dim3((unsigned)kmax), dim3(256), 0, stream,
                           grow, B, kmax, gsum);
    return hipGetLastError();
}

extern "C" int sos_bwd_shape_supported(int L, int N)
{
    return (L == 64 || L == 256 || L == 512) && (N == 16 || N == 32);
}

extern "C" hipError_t sos_launch_bwd_reduce(const double *partials, int64_t groups, int K,
                                            const float *sections, float *gsections,
                                            hipStream_t stream)
{
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(sos_bwd_reduce_kernel, dim3(K), dim3(256), 0, stream, partials, groups, K,
                       sections, gsections);
    return hipGetLastError();
}
