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
    const float *x;
    float *y;
    int64_t n;
    int64_t groups;
    const float *tabs;
    const float *zi;
    float *zf;
    unsigned long long *desc;
    unsigned *ctrl;
    int K;
    int vec;   // x and y 16-byte aligned
    unsigned long long timeout_ticks;
};

__device__ __forceinline__ float lane_up(float v, int d, int lane)
{
    // value of lane (lane - d), 0 for lane < d
    const float r = __shfl_up(v, d, 64);
    return lane >= d ? r : 0.0f;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
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
__device__ float2 lookback(const FwdArgs &a, const float *tabv, int64_t c, int s, unsigned epoch,
                           int lane)
{
    ctab_t *tab = ctab(tabv);
    const float4 gp = *reinterpret_cast<const float4 *>(tabv + OFF_GRPPOW + 4 * lane);
    const float w00 = tab[OFF_TW + 0], w01 = tab[OFF_TW + 1];
    const float w10 = tab[OFF_TW + 2], w11 = tab[OFF_TW + 3];
    float acc1 = 0.0f, acc2 = 0.0f;
    float m00 = 1.0f, m01 = 0.0f, m10 = 0.0f, m11 = 1.0f;   // window transform
    int64_t base = c - 1;
    const unsigned long long t0 = wall_clock64();
    while (true) {
        const int64_t h = base - lane;
        unsigned long long w[4] = {0ull, 0ull, 0ull, 0ull};
        if (h >= 0) {
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
                                            const FwdArgs &a, const float *tabv, int64_t c, int s,
                                            unsigned epoch, int wv, int lane, bool has_last, int zl,
                                            int zp)
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
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int d = 1 << k;
        const float q1 = lane_up(p1, d, lane), q2 = lane_up(p2, d, lane);
        const float2 r = mv_add(tab + OFF_KS + 4 * k, q1, q2, p1, p2);
        p1 = r.x;
        p2 = r.y;
    }

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
        const float t1 = __shfl(p1, 63, 64), t2 = __shfl(p2, 63, 64);
        float g1 = t1, g2 = t2;
        if (W > 1) {
            const float2 r = mv_add(tab + OFF_TWAVE, e1w, e2w, t1, t2);
            g1 = r.x;
            g2 = r.y;
        }

        // --- 4. decoupled lookback for the group's incoming state
        unsigned long long *dsc = a.desc + ((size_t)c * a.K + s) * 4;
        float sg1, sg2;
        if (c == 0) {
            sg1 = a.zi ? ctab(a.zi)[2 * s] : 0.0f;
            sg2 = a.zi ? ctab(a.zi)[2 * s + 1] : 0.0f;
        } else {
            if (lane == 0) {
                store_word(dsc + 0, pack(g1, epoch));
                store_word(dsc + 1, pack(g2, epoch));
            }
            const float2 sg = lookback(a, tabv, c, s, epoch, lane);
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
    const float e1 = lane_up(p1, 1, lane), e2 = lane_up(p2, 1, lane);
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
    if (has_last && a.zf) {
        float yo1, yo2;
        pick_two(u, tl, lane, zl, zp, yo1, yo2);
        if (lane == zl) {
            float z1;
            if (zp >= 1)
                z1 = b1 * zx1 + b2 * zx2 - a1 * yo1 - a2 * yo2;
            else
                z1 = b1 * zx1 - a1 * yo1 + s2;   // s2: this lane's incoming state
            a.zf[2 * s] = z1;
            a.zf[2 * s + 1] = b2 * zx1 - a2 * yo1;
        }
    }
}

template <int N, int W>
__global__ void __launch_bounds__(64 * W) sos_fwd_kernel(FwdArgs a)
{
    constexpr int CW = kLanes * N;   // samples per wave
    constexpr int C = CW * W;        // samples per group
    constexpr int RS = N + 4;        // LDS row stride: conflict-free 128-bit row reads
    constexpr int Q = N / 4;         // float4 per lane row
    __shared__ float tile[W][kLanes * RS];
    __shared__ Xch<W> xch;
    __shared__ unsigned ticket;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;

    if (threadIdx.x == 0) ticket = atomicAdd(&a.ctrl[CTRL_TICKET], 1u);
    __syncthreads();
    const int64_t c = (int64_t)ticket;
    if (c >= a.groups) return;
    const unsigned epoch = __hip_atomic_load(&a.ctrl[CTRL_EPOCH], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);

    const int64_t g0 = c * C + (int64_t)wv * CW;   // first sample of this wave
    const int64_t rem = a.n - g0;                  // may be <= 0 in the last group
    const bool full = rem >= CW;
    float *tl = tile[wv];

    // --- load: coalesced 128-bit global loads -> LDS rows (transpose)
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int v = kLanes * j + lane;           // float4 index inside the wave's part
        const int64_t q = 4 * (int64_t)v;
        float4 val;
        if (full && a.vec) {
            const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(a.x + g0) + v);
            val = make_float4(t.x, t.y, t.z, t.w);
        } else {
            val.x = q + 0 < rem ? a.x[g0 + q + 0] : 0.0f;
            val.y = q + 1 < rem ? a.x[g0 + q + 1] : 0.0f;
            val.z = q + 2 < rem ? a.x[g0 + q + 2] : 0.0f;
            val.w = q + 3 < rem ? a.x[g0 + q + 3] : 0.0f;
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

    // --- sections (any unusable section poisons the whole call)
    bool bad = false;
    for (int s = 0; s < a.K; ++s)
        bad |= __float_as_uint(ctab(a.tabs)[(size_t)s * TAB_FLOATS + OFF_STATUS]) != 0u;
    // position of the last real sample n-1 if this wave holds it
    const int64_t lp = (a.n - 1) - g0;
    const bool has_last = lp >= 0 && lp < CW;
    const int zl = has_last ? (int)(lp / N) : 0, zp = has_last ? (int)(lp % N) : 0;
    if (!bad) {
        for (int s = 0; s < a.K; ++s)
            run_section<N, W>(u, xch, tl, a, a.tabs + (size_t)s * TAB_FLOATS, c, s, epoch, wv,
                              lane, has_last, zl, zp);
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) u[k] = __builtin_nanf("");
        if (has_last && lane == 0 && a.zf)
            for (int s = 0; s < a.K; ++s) a.zf[2 * s] = a.zf[2 * s + 1] = __builtin_nanf("");
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
        if (full && a.vec) {
            const f4 t = {val.x, val.y, val.z, val.w};
            __builtin_nontemporal_store(t, reinterpret_cast<f4 *>(a.y + g0) + v);
        } else {
            if (q + 0 < rem) a.y[g0 + q + 0] = val.x;
            if (q + 1 < rem) a.y[g0 + q + 1] = val.y;
            if (q + 2 < rem) a.y[g0 + q + 2] = val.z;
            if (q + 3 < rem) a.y[g0 + q + 3] = val.w;
        }
    }
}

template <int N, int W>
hipError_t launch(const FwdArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL((sos_fwd_kernel<N, W>), dim3((unsigned)a.groups), dim3(64 * W), 0, stream,
                       a);
    return hipGetLastError();
}

}  // namespace

// Host-side launcher (C linkage inside the library only). L = 64 * W lanes per
// group, N samples per lane.
extern "C" hipError_t sos_launch_fwd(int L, int N, const float *x, float *y, int64_t n,
                                     int64_t groups, const float *tabs, int K, const float *zi,
                                     float *zf, unsigned long long *desc, unsigned *ctrl,
                                     unsigned long long timeout_ticks, hipStream_t stream)
{
    const int vec =
        ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15u) == 0 ? 1 : 0;
    FwdArgs a{x, y, n, groups, tabs, zi, zf, desc, ctrl, K, vec, timeout_ticks};
    const int W = L / 64;
    switch (W * 1000 + N) {
    case 1016: return launch<16, 1>(a, stream);
    case 1032: return launch<32, 1>(a, stream);
    case 1064: return launch<64, 1>(a, stream);
    case 4016: return launch<16, 4>(a, stream);
    case 4032: return launch<32, 4>(a, stream);
    case 4064: return launch<64, 4>(a, stream);
    case 8016: return launch<16, 8>(a, stream);
    case 8032: return launch<32, 8>(a, stream);
    case 8064: return launch<64, 8>(a, stream);
    case 16016: return launch<16, 16>(a, stream);
    case 16032: return launch<32, 16>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

// Group shapes compiled into the library.
extern "C" int sos_fwd_shape_supported(int L, int N)
{
    if (L % 64) return 0;
    switch ((L / 64) * 1000 + N) {
    case 1016: case 1032: case 1064: case 4016: case 4032: case 4064:
    case 8016: case 8032: case 8064: case 16016: case 16032:
        return 1;
    default: return 0;
    }
}
