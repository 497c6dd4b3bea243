// Single-kernel multi-block cascade filter for gfx950.
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
//   3. that pair becomes the lane's zero-state terminal TDF-II state; a
//      Kogge-Stone scan over the wave's 64 lanes (constant matrices
//      T^(N 2^k)) gives every lane's zero-state state and the wave's total,
//      and the W wave totals are combined through LDS (one barrier) into
//      every wave's zero-state incoming state and the group's local carry;
//   4. decoupled lookback (last wave): publish the local carry, walk the
//      predecessors' descriptors (64 per round, one per lane) until a
//      resolved carry is found, compose through T^(C j), publish this group's
//      resolved carry and hand the group state to all waves (second barrier);
//   5. each lane's true incoming state = T^(N l) (T^(64 N w) s_group + wave
//      prefix) + lane prefix; back substitution level by level, the single
//      initial-condition row per level and parity receiving g[n] s1 +
//      g[n-1] s2 (no divisions).
// The section output stays in registers as the next section's input.
//
// Descriptors: per (group, section) four 64-bit words {agg.z1, agg.z2,
// inc.z1, inc.z2}, each {float value | 32-bit epoch tag}. A word is valid when
// its tag equals the launch epoch, so words are self-validating: no fences, no
// clearing between launches, and the agent-scope relaxed atomics keep them
// coherent across the XCDs' separate L2 caches. A one-thread kernel before
// each launch zeroes the ticket and advances the epoch.
#include "sos_device.h"

using namespace sosdev;

namespace {

struct FwdArgs {
    // plain mode (B == 0): one signal x/y of n samples, K sections at tabs
    const float *x;
    float *y;
    int64_t n;
    const float *tabs;
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
    // both modes
    int64_t total;          // number of work items (plain)
    unsigned long long *desc;
    unsigned *ctrl;
    unsigned long long timeout_ticks;
};

// One unit of work: group g of one signal, drawn as ticket t.
struct Item {
    const float *x;
    float *y;
    int64_t n;              // samples in the signal
    int64_t g;              // group index within the signal
    int64_t t;              // ticket (descriptor row)
    const float *tabs;      // tables of the signal's sections
    const float *zi;
    float *zf;
    int K;
};

// DPP move of a 32-bit value across lanes; lanes whose source is outside the
// row (or whose row is masked off by ROWS) read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp0(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
enum : int {
    DPP_ROW_SHR = 0x110,    // + d, d = 1..15: lane l reads l-d inside its 16-lane row
    DPP_WAVE_SHR1 = 0x138,  // lane l reads l-1 across the whole wave
    DPP_BCAST15 = 0x142,    // lane 15 of row r -> every lane of row r+1
    DPP_BCAST31 = 0x143     // lane 31 -> every lane of rows 2 and 3
};

// Inclusive affine scan over the 64 lanes of a wave:
//   P[l] = t[l] + T^N P[l-1]   (P[-1] = 0),
// the cross-lane terminal-state recurrence (role of Eq. (13)). Within each
// 16-lane row a Kogge-Stone ladder with the uniform powers T^(N 2^k), k < 4;
// then rows 1 and 3 add lane 15 / 47 through T^(N((l%16)+1)) and rows 2 and 3
// add lane 31 through T^(N(l-31)) (per-lane powers from the table).
__device__ __forceinline__ void wave_scan(float &p1, float &p2, ctab_t *tab, const float *tabv,
                                          int lane)
{
#define SOS_ROW_STEP(K)                                                                     \
    {                                                                                       \
        const float q1 = dpp0<DPP_ROW_SHR + (1 << K), 0xF>(p1);                             \
        const float q2 = dpp0<DPP_ROW_SHR + (1 << K), 0xF>(p2);                             \
        const float n1 = fmaf(tab[OFF_KS + 4 * K + 0], q1, fmaf(tab[OFF_KS + 4 * K + 1], q2, p1)); \
        const float n2 = fmaf(tab[OFF_KS + 4 * K + 2], q1, fmaf(tab[OFF_KS + 4 * K + 3], q2, p2)); \
        p1 = n1;                                                                            \
        p2 = n2;                                                                            \
    }
    SOS_ROW_STEP(0)
    SOS_ROW_STEP(1)
    SOS_ROW_STEP(2)
    SOS_ROW_STEP(3)
#undef SOS_ROW_STEP
    const float4 pa = *reinterpret_cast<const float4 *>(tabv + OFF_SCANPOW + 8 * lane);
    const float4 pb = *reinterpret_cast<const float4 *>(tabv + OFF_SCANPOW + 8 * lane + 4);
    {
        const float q1 = dpp0<DPP_BCAST15, 0xA>(p1), q2 = dpp0<DPP_BCAST15, 0xA>(p2);
        const float n1 = fmaf(pa.x, q1, fmaf(pa.y, q2, p1));
        const float n2 = fmaf(pa.z, q1, fmaf(pa.w, q2, p2));
        p1 = n1;
        p2 = n2;
    }
    {
        const float q1 = dpp0<DPP_BCAST31, 0xC>(p1), q2 = dpp0<DPP_BCAST31, 0xC>(p2);
        const float n1 = fmaf(pb.x, q1, fmaf(pb.y, q2, p1));
        const float n2 = fmaf(pb.z, q1, fmaf(pb.w, q2, p2));
        p1 = n1;
        p2 = n2;
    }
}

// Sum over the 64 lanes of a wave (result valid in every lane).
__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp0<DPP_ROW_SHR + 1, 0xF>(v);
    v += dpp0<DPP_ROW_SHR + 2, 0xF>(v);
    v += dpp0<DPP_ROW_SHR + 4, 0xF>(v);
    v += dpp0<DPP_ROW_SHR + 8, 0xF>(v);
    v += dpp0<DPP_BCAST15, 0xA>(v);
    v += dpp0<DPP_BCAST31, 0xC>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

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

// Lane `zl` reads samples zp and zp-1 of its row after the whole wave has
// written its registers to its LDS rows (only the wave holding sample n-1
// does this, once per section; LDS operations of one wave complete in order).
template <int N>
__device__ __forceinline__ void pick_two(const float (&u)[N], float *tl, int lane, int zl, int zp,
                                         float &v0, float &v1)
{
    constexpr int RS = N + 4;
#pragma unroll
    for (int k = 0; k < N / 4; ++k)
        *reinterpret_cast<float4 *>(&tl[lane * RS + 4 * k]) =
            make_float4(u[4 * k + 0], u[4 * k + 1], u[4 * k + 2], u[4 * k + 3]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    v0 = tl[zl * RS + zp];
    v1 = zp >= 1 ? tl[zl * RS + zp - 1] : 0.0f;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// 2x2 (row-major, 4 floats at p) times vector, plus addend.
__device__ __forceinline__ float2 mv_add(ctab_t *p, float v1, float v2, float a1, float a2)
{
    return make_float2(fmaf(p[0], v1, fmaf(p[1], v2, a1)), fmaf(p[2], v1, fmaf(p[3], v2, a2)));
}

// Resolve the incoming state of group c (> 0) for section s by decoupled
// lookback; executed by one whole wave. Returns a wave-uniform pair. On
// timeout returns NaNs and sets the error bit (the caller still publishes, so
// successors terminate).
__device__ float2 lookback(const FwdArgs &a, const Item &it, const float *tabv, int s,
                           unsigned epoch, int lane)
{
    ctab_t *tab = ctab(tabv);
    const float4 gp = *reinterpret_cast<const float4 *>(tabv + OFF_GRPPOW + 4 * lane);
    const float w00 = tab[OFF_TW + 0], w01 = tab[OFF_TW + 1];
    const float w10 = tab[OFF_TW + 2], w11 = tab[OFF_TW + 3];
    float acc1 = 0.0f, acc2 = 0.0f;
    float m00 = 1.0f, m01 = 0.0f, m10 = 0.0f, m11 = 1.0f;   // window transform
    const int64_t first = it.t - it.g;   // ticket of the signal's first group
    int64_t base = it.t - 1;
    const unsigned long long t0 = wall_clock64();
    while (true) {
        const int64_t h = base - lane;
        unsigned long long w[4] = {0ull, 0ull, 0ull, 0ull};
        if (h >= first) {
            const unsigned long long *d = a.desc + ((size_t)h * a.K + s) * 4;
#pragma unroll
            for (int i = 0; i < 4; ++i) w[i] = load_word(d + i);
        }
        const bool inc_ok = (unsigned)(w[2] >> 32) == epoch && (unsigned)(w[3] >> 32) == epoch;
        const bool agg_ok = (unsigned)(w[0] >> 32) == epoch && (unsigned)(w[1] >> 32) == epoch;
        const unsigned long long incm = __ballot(inc_ok);
        const unsigned long long rdym = __ballot(inc_ok || agg_ok);
        int jstar = 64;
        unsigned long long need;
        if (incm) {
            jstar = __builtin_ctzll(incm);
            need = (jstar == 63) ? ~0ull : ((2ull << jstar) - 1ull);
        } else {
            // no resolved carry in this window: all 64 must hold local carries
            need = ~0ull;
        }
        if ((rdym & need) != need) {
            if (wall_clock64() - t0 > a.timeout_ticks) {
                if (lane == 0) atomicOr(&a.ctrl[CTRL_ERR], ERRBIT_TIMEOUT);
                return make_float2(__builtin_nanf(""), __builtin_nanf(""));
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        float v1 = 0.0f, v2 = 0.0f;
        if (lane < jstar) {
            v1 = __uint_as_float((unsigned)w[0]);
            v2 = __uint_as_float((unsigned)w[1]);
        } else if (lane == jstar) {
            v1 = __uint_as_float((unsigned)w[2]);
            v2 = __uint_as_float((unsigned)w[3]);
        }
        const float s1 = wave_sum(gp.x * v1 + gp.y * v2);
        const float s2 = wave_sum(gp.z * v1 + gp.w * v2);
        acc1 += m00 * s1 + m01 * s2;
        acc2 += m10 * s1 + m11 * s2;
        if (jstar < 64) break;
        // slide the window 64 groups further back
        const float n00 = m00 * w00 + m01 * w10, n01 = m00 * w01 + m01 * w11;
        const float n10 = m10 * w00 + m11 * w10, n11 = m10 * w01 + m11 * w11;
        m00 = n00; m01 = n01; m10 = n10; m11 = n11;
        base -= 64;
    }
    return make_float2(acc1, acc2);
}

// Exchange area of one workgroup in LDS.
template <int W>
struct Xch {
    float wave_tot[W][2];   // zero-state totals of the waves
    float grp[2];           // resolved incoming state of the group
};

template <int N, int W>
__device__ __forceinline__ void run_section(float (&u)[N], Xch<W> &xch, float *tl,
                                            const FwdArgs &a, const Item &it, const float *tabv,
                                            int s, unsigned epoch, int wv, int lane, bool has_last,
                                            int zl, int zp)
{
    constexpr int LOG = __builtin_ctz(N);
    ctab_t *tab = ctab(tabv);

    // --- inputs kept for the terminal state (and for zf at sample n-1)
    const float xl1 = u[N - 1], xl2 = u[N - 2];
    float zx1 = 0.0f, zx2 = 0.0f;
    if (has_last) pick_two(u, tl, lane, zl, zp, zx1, zx2);

    // --- 1. level-1 right-hand side, in place from the end
    const float c0 = tab[OFF_TAPS + 0], c1 = tab[OFF_TAPS + 1], c2 = tab[OFF_TAPS + 2];
    const float c3 = tab[OFF_TAPS + 3], c4 = tab[OFF_TAPS + 4];
#pragma unroll
    for (int m = N - 1; m >= 0; --m) {
        float r = c0 * u[m];
        if (m >= 1) r = fmaf(c1, u[m - 1], r);
        if (m >= 2) r = fmaf(c2, u[m - 2], r);
        if (m >= 3) r = fmaf(c3, u[m - 3], r);
        if (m >= 4) r = fmaf(c4, u[m - 4], r);
        u[m] = r;
    }

    // --- 2. reduction of both parity chains (positions that stay, descending)
#pragma unroll
    for (int i = 1; i < LOG; ++i) {
        const int st = 1 << i;
        const float e = tab[OFF_E + i], f = tab[OFF_F + i];
#pragma unroll
        for (int m = N - 1; m >= 0; --m) {
            if (((m + 1) % (2 * st)) == 0 || ((m + 2) % (2 * st)) == 0) {
                float r = u[m];
                if (m - st >= 0) r = fmaf(-e, u[m - st], r);
                if (m - 2 * st >= 0) r = fmaf(f, u[m - 2 * st], r);
                u[m] = r;
            }
        }
    }

    // --- 3. zero-state terminal TDF-II state of the lane, scan over the wave
    const float b1 = tab[OFF_B1], b2 = tab[OFF_B2], a1 = tab[OFF_A1], a2 = tab[OFF_A2];
    float p1 = b1 * xl1 + b2 * xl2 - a1 * u[N - 1] - a2 * u[N - 2];
    float p2 = b2 * xl1 - a2 * u[N - 1];
    wave_scan(p1, p2, tab, tabv, lane);

    //     ... and over the W waves of the group (zero group state)
    float e1w = 0.0f, e2w = 0.0f;      // zero-state incoming state of this wave
    if (W > 1) {
        if (lane == 63) {
            xch.wave_tot[wv][0] = p1;
            xch.wave_tot[wv][1] = p2;
        }
        __syncthreads();
        for (int v = 0; v < wv; ++v) {
            const float2 r = mv_add(tab + OFF_TWAVE, e1w, e2w, xch.wave_tot[v][0],
                                    xch.wave_tot[v][1]);
            e1w = r.x;
            e2w = r.y;
        }
    }
    if (wv == W - 1) {
        // group local carry = state after the last wave at zero group state
        const float t1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p1), 63));
        const float t2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p2), 63));
        float g1 = t1, g2 = t2;
        if (W > 1) {
            const float2 r = mv_add(tab + OFF_TWAVE, e1w, e2w, t1, t2);
            g1 = r.x;
            g2 = r.y;
        }

        // --- 4. decoupled lookback for the group's incoming state
        unsigned long long *dsc = a.desc + ((size_t)it.t * a.K + s) * 4;
        float sg1, sg2;
        if (it.g == 0) {
            sg1 = it.zi ? ctab(it.zi)[2 * s] : 0.0f;
            sg2 = it.zi ? ctab(it.zi)[2 * s + 1] : 0.0f;
        } else {
            if (lane == 0) {
                store_word(dsc + 0, pack(g1, epoch));
                store_word(dsc + 1, pack(g2, epoch));
            }
            const float2 sg = lookback(a, it, tabv, s, epoch, lane);
            sg1 = sg.x;
            sg2 = sg.y;
        }
        const float2 inc = mv_add(tab + OFF_TC, sg1, sg2, g1, g2);
        if (lane == 0) {
            store_word(dsc + 2, pack(inc.x, epoch));
            store_word(dsc + 3, pack(inc.y, epoch));
            xch.grp[0] = sg1;
            xch.grp[1] = sg2;
        }
    }
    __syncthreads();
    const float sg1 = xch.grp[0], sg2 = xch.grp[1];

    // --- 5. incoming state of every lane, then back substitution
    const float2 sw = mv_add(tab + OFF_WPOW + 4 * wv, sg1, sg2, e1w, e2w);
    const float4 lp = *reinterpret_cast<const float4 *>(tabv + OFF_LANEPOW + 4 * lane);
    const float e1 = dpp0<DPP_WAVE_SHR1, 0xF>(p1), e2 = dpp0<DPP_WAVE_SHR1, 0xF>(p2);
    const float s1 = fmaf(lp.x, sw.x, fmaf(lp.y, sw.y, e1));
    const float s2 = fmaf(lp.z, sw.x, fmaf(lp.w, sw.y, e2));
    ctab_t *g = tab + OFF_G + 1;   // g[-1] is readable and 0

    u[N - 1] = fmaf(g[N - 1], s1, fmaf(g[N - 2], s2, u[N - 1]));
    u[N - 2] = fmaf(g[N - 2], s1, fmaf(g[N - 3], s2, u[N - 2]));
#pragma unroll
    for (int i = LOG - 1; i >= 1; --i) {
        const int st = 1 << i;
        const float e = tab[OFF_E + i], f = tab[OFF_F + i];
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            const int m0 = st - 1 - par;                 // odd chain, then even chain
            u[m0] = fmaf(g[m0], s1, fmaf(g[m0 - 1], s2, u[m0]));
#pragma unroll
            for (int m = m0 + 2 * st; m < N; m += 2 * st)
                u[m] = fmaf(-e, u[m - st], fmaf(-f, u[m - 2 * st], u[m]));
        }
    }

    // --- final state after sample n-1 (only the lane that holds it)
    if (has_last && it.zf) {
        float yo1, yo2;
        pick_two(u, tl, lane, zl, zp, yo1, yo2);
        if (lane == zl) {
            float z1;
            if (zp >= 1)
                z1 = b1 * zx1 + b2 * zx2 - a1 * yo1 - a2 * yo2;
            else
                z1 = b1 * zx1 - a1 * yo1 + s2;   // s2: this lane's incoming state
            it.zf[2 * s] = z1;
            it.zf[2 * s + 1] = b2 * zx1 - a2 * yo1;
        }
    }
}

template <int N, int W>
__device__ __forceinline__ void process_group(const FwdArgs &a, const Item &it, float *tl,
                                              Xch<W> &xch, unsigned epoch, int wv, int lane)
{
    constexpr int CW = kLanes * N;   // samples per wave
    constexpr int C = CW * W;        // samples per group
    constexpr int RS = N + 4;        // LDS row stride: conflict-free 128-bit row reads
    constexpr int Q = N / 4;         // float4 per lane row

    const int64_t g0 = it.g * C + (int64_t)wv * CW;   // first sample of this wave
    const int64_t rem = it.n - g0;                    // may be <= 0 in the last group
    const bool full = rem >= CW;
    const bool vec = ((reinterpret_cast<uintptr_t>(it.x) | reinterpret_cast<uintptr_t>(it.y)) &
                      15u) == 0;

    // --- load: coalesced 128-bit global loads -> LDS rows (transpose)
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int v = kLanes * j + lane;           // float4 index inside the wave's part
        const int64_t q = 4 * (int64_t)v;
        float4 val;
        if (full && vec) {
            const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(it.x + g0) + v);
            val = make_float4(t.x, t.y, t.z, t.w);
        } else {
            val.x = q + 0 < rem ? it.x[g0 + q + 0] : 0.0f;
            val.y = q + 1 < rem ? it.x[g0 + q + 1] : 0.0f;
            val.z = q + 2 < rem ? it.x[g0 + q + 2] : 0.0f;
            val.w = q + 3 < rem ? it.x[g0 + q + 3] : 0.0f;
        }
        *reinterpret_cast<float4 *>(&tl[(v / Q) * RS + (v % Q) * 4]) = val;
    }
    __syncthreads();
    float u[N];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const float4 v = *reinterpret_cast<const float4 *>(&tl[lane * RS + 4 * k]);
        u[4 * k + 0] = v.x;
        u[4 * k + 1] = v.y;
        u[4 * k + 2] = v.z;
        u[4 * k + 3] = v.w;
    }

    // --- sections (an unusable section poisons its signal)
    bool bad = false;
    for (int s = 0; s < it.K; ++s)
        bad |= __float_as_uint(ctab(it.tabs)[(size_t)s * TAB_FLOATS + OFF_STATUS]) != 0u;
    // position of the last real sample n-1 if this wave holds it
    const int64_t lp = (it.n - 1) - g0;
    const bool has_last = lp >= 0 && lp < CW;
    const int zl = has_last ? (int)(lp / N) : 0, zp = has_last ? (int)(lp % N) : 0;
    if (!bad) {
        for (int s = 0; s < it.K; ++s)
            run_section<N, W>(u, xch, tl, a, it, it.tabs + (size_t)s * TAB_FLOATS, s, epoch, wv,
                              lane, has_last, zl, zp);
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) u[k] = __builtin_nanf("");
        if (has_last && lane == 0 && it.zf)
            for (int s = 0; s < it.K; ++s) it.zf[2 * s] = it.zf[2 * s + 1] = __builtin_nanf("");
    }

    // --- store: registers -> LDS rows -> coalesced 128-bit global stores
    __syncthreads();
#pragma unroll
    for (int k = 0; k < Q; ++k)
        *reinterpret_cast<float4 *>(&tl[lane * RS + 4 * k]) =
            make_float4(u[4 * k + 0], u[4 * k + 1], u[4 * k + 2], u[4 * k + 3]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int v = kLanes * j + lane;
        const int64_t q = 4 * (int64_t)v;
        const float4 val = *reinterpret_cast<const float4 *>(&tl[(v / Q) * RS + (v % Q) * 4]);
        if (full && vec) {
            const f4 t = {val.x, val.y, val.z, val.w};
            __builtin_nontemporal_store(t, reinterpret_cast<f4 *>(it.y + g0) + v);
        } else {
            if (q + 0 < rem) it.y[g0 + q + 0] = val.x;
            if (q + 1 < rem) it.y[g0 + q + 1] = val.y;
            if (q + 2 < rem) it.y[g0 + q + 2] = val.z;
            if (q + 3 < rem) it.y[g0 + q + 3] = val.w;
        }
    }
}

// The filter kernel: every workgroup draws tickets until the work runs out.
// A ticket names one group of one signal; within a signal, tickets ascend with
// the group index, so a group's predecessors were drawn (and are being worked
// on) before it, which guarantees forward progress of the lookback whatever
// the grid size (Sec. IV-A).
template <int N, int W>
__global__ void __launch_bounds__(64 * W) sos_fwd_kernel(FwdArgs a)
{
    constexpr int RS = N + 4;
    __shared__ float tile[W][kLanes * RS];
    __shared__ Xch<W> xch;
    __shared__ int64_t ticket;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const unsigned epoch = __hip_atomic_load(&a.ctrl[CTRL_EPOCH], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    const int64_t total = a.B > 0 ? *a.total_dev : a.total;
    float *tl = tile[wv];

    for (;;) {
        if (threadIdx.x == 0) ticket = (int64_t)atomicAdd(&a.ctrl[CTRL_TICKET], 1u);
        __syncthreads();
        const int64_t t = ticket;
        __syncthreads();
        if (t >= total) break;
        Item it;
        it.t = t;
        if (a.B == 0) {
            it.x = a.x;
            it.y = a.y;
            it.n = a.n;
            it.g = t;
            it.tabs = a.tabs;
            it.zi = a.zi;
            it.zf = a.zf;
            it.K = a.K;
        } else {
            const int i = a.sigmap[t];
            const int64_t so = a.sig_off[i];
            const int32_t sc = a.sec_off[i];
            it.x = a.x + so;
            it.y = a.y + so;
            it.n = a.sig_off[i + 1] - so;
            it.g = t - a.gpre[i];
            it.tabs = a.tabs + (size_t)sc * TAB_FLOATS;
            it.zi = a.zi ? a.zi + 2 * (int64_t)sc : nullptr;
            it.zf = a.zf ? a.zf + 2 * (int64_t)sc : nullptr;
            it.K = a.Ks[i];
        }
        process_group<N, W>(a, it, tl, xch, epoch, wv, lane);
        if ((int64_t)gridDim.x >= total) break;   // one group per workgroup: no extra draw
    }
}

template <int N, int W>
hipError_t launch(const FwdArgs &a, int64_t grid, hipStream_t stream)
{
    hipLaunchKernelGGL((sos_fwd_kernel<N, W>), dim3((unsigned)grid), dim3(64 * W), 0, stream, a);
    return hipGetLastError();
}

template <int N, int W>
int capacity_of()
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sos_fwd_kernel<N, W>, 64 * W, 0) !=
        hipSuccess)
        per_cu = 1;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    return (per_cu > 0 ? per_cu : 1) * cus;
}

#define SOS_SHAPES(X)                                                                     \
    X(16, 1) X(32, 1) X(64, 1) X(16, 4) X(32, 4) X(64, 4) X(16, 8) X(32, 8) X(64, 8)    \
        X(16, 16) X(32, 16)

hipError_t dispatch(int L, int N, const FwdArgs &a, int64_t grid, hipStream_t stream)
{
    const int W = L / 64;
#define SOS_CASE(NN, WW)                                                                  \
    if (N == NN && W == WW) return launch<NN, WW>(a, grid, stream);
    SOS_SHAPES(SOS_CASE)
#undef SOS_CASE
    return hipErrorInvalidValue;
}

}  // namespace

// Group shapes compiled into the library: L = 64 W lanes, N samples per lane.
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

// Workgroups of shape (L, N) that can be resident on the whole device at once.
extern "C" int sos_fwd_capacity(int L, int N)
{
    const int W = L / 64;
#define SOS_CASE(NN, WW)                                                                  \
    if (N == NN && W == WW) return capacity_of<NN, WW>();
    SOS_SHAPES(SOS_CASE)
#undef SOS_CASE
    return 0;
}

// Plain filter of one signal; grid <= 0 means one workgroup per group.
extern "C" hipError_t sos_launch_fwd(int L, int N, const float *x, float *y, int64_t n,
                                     int64_t groups, const float *tabs, int K, const float *zi,
                                     float *zf, unsigned long long *desc, unsigned *ctrl,
                                     unsigned long long timeout_ticks, int64_t grid,
                                     hipStream_t stream)
{
    FwdArgs a{};
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
    a.ctrl = ctrl;
    a.timeout_ticks = timeout_ticks;
    if (grid <= 0 || grid > groups) grid = groups;
    return dispatch(L, N, a, grid, stream);
}

// Uneven batch in one persistent launch. The work table (gpre, sigmap,
// *total_dev) is produced on the device by sos_launch_worktable.
extern "C" hipError_t sos_launch_fwd_batched(int L, int N, int B, int kmax, const int32_t *Ks,
                                             const int32_t *sec_off, const int64_t *sig_off,
                                             const int64_t *gpre, const int32_t *sigmap,
                                             const int64_t *total_dev, const float *x, float *y,
                                             const float *tabs, const float *zi, float *zf,
                                             unsigned long long *desc, unsigned *ctrl,
                                             unsigned long long timeout_ticks, int64_t grid,
                                             hipStream_t stream)
{
    FwdArgs a{};
    a.x = x;
    a.y = y;
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
    a.ctrl = ctrl;
    a.timeout_ticks = timeout_ticks;
    return dispatch(L, N, a, grid, stream);
}
