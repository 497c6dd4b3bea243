// Coefficient preparation on the device (FP64 arithmetic).
//
// The paper notes that every coefficient of the reduction, the terminal scan
// and the state correction depends only on the filter and is precomputed
// (Sec. II-D, after Eq. (17)). This kernel does that once per coefficient set:
// block s normalises section s by a0, checks it, and writes its table in the
// layout its signal needs (sos_device.h).
#include "sos_device.h"

using namespace sosdev;

namespace {

__device__ inline m2 mpow_pow2(m2 m, int log2e)
{
    for (int i = 0; i < log2e; ++i) m = mmul(m, m);
    return m;
}

template <typename T>
__device__ inline void put(T *t, int off, const m2 &m)
{
    t[off + 0] = (T)m.a;
    t[off + 1] = (T)m.b;
    t[off + 2] = (T)m.c;
    t[off + 3] = (T)m.d;
}

// T^e by binary expansion, given the powers p2[k] = T^(2^k), k < bits.
__device__ inline m2 mpow_bits(const m2 *p2, int bits, int e)
{
    m2 r = mident();
    for (int k = 0; k < bits; ++k)
        if ((e >> k) & 1) r = mmul(r, p2[k]);
    return r;
}

// Sum over the 64 lanes of a wave in FP64 (every lane gets the total).
__device__ inline double wave_total(double v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Peak gain of the recursive part of a row [b0 b1 b2 a0 a1 a2]: 1 / min over
// the unit circle of |A(e^{jw})|, A(z) = 1 + a1 z^-1 + a2 z^-2 after
// normalisation. With c = cos(w), |A|^2 = 4 a2 c^2 + 2 a1 (1 + a2) c +
// (1 + a1^2 + a2^2 - 2 a2), a quadratic in c on [-1, 1]: its minimum is at
// an end or at the vertex. Infinite for a0 = 0 or a zero on the circle.
__device__ inline double peak_gain(const float *row)
{
    const double a0 = row[3];
    if (a0 == 0.0) return INFINITY;
    const double a1 = row[4] / a0, a2 = row[5] / a0;
    auto f = [&](double c) {
        return 4.0 * a2 * c * c + 2.0 * a1 * (1.0 + a2) * c + (1.0 + a1 * a1 + a2 * a2 - 2.0 * a2);
    };
    double m = fmin(f(-1.0), f(1.0));
    if (a2 > 0.0) {
        const double cv = -a1 * (1.0 + a2) / (4.0 * a2);
        if (cv > -1.0 && cv < 1.0) m = fmin(m, f(cv));
    }
    return m > 0.0 ? 1.0 / sqrt(m) : INFINITY;
}

// Layout of a signal's tables: accurate when the compute type is FP32 and a
// section's peak gain exceeds rho_max (the FP32 state path and, in DC-CR
// launches, the fold B(z)A(-z) lose accuracy with such poles), else fast.
// rows: the signal's K rows. Each block of the signal decides alike.
template <typename T>
__device__ inline unsigned signal_mode(const float *rows, int K, double rho_max)
{
    if (sizeof(T) != 4) return MODE_FAST;
    for (int k = 0; k < K; ++k)
        if (!gain_within(rows + 6 * k, rho_max)) return MODE_ACCURATE;
    return MODE_FAST;
}

// Normalised coefficients and stability status of one row.
struct Norm {
    double inv, b0, b1, b2, a1, a2;
    unsigned status;
};
__device__ inline Norm normalise(const float *row, bool pair)
{
    Norm c;
    const double a0 = (double)row[3];
    c.status = 0u;
    if (a0 == 0.0) c.status |= ERRBIT_A0;
    c.inv = (a0 == 0.0) ? 0.0 : 1.0 / a0;
    c.b0 = pair ? 1.0 : row[0] * c.inv;
    c.b1 = pair ? 0.0 : row[1] * c.inv;
    c.b2 = pair ? 0.0 : row[2] * c.inv;
    c.a1 = row[4] * c.inv;
    c.a2 = row[5] * c.inv;
    // open stability triangle of z^2 + a1 z + a2: both poles strictly inside
    // the unit circle (NaN fails the test). On its boundary the state-map
    // powers do not decay across groups.
    if (!(fabs(c.a2) < 1.0 && fabs(c.a1) < 1.0 + c.a2)) c.status |= ERRBIT_UNSTABLE;
    return c;
}

// The state-map powers every layout holds, and this lane's per-lane ones.
struct Powers {
    m2 ks[6];     // T^(N 2^k)
    m2 twv, tc, tw;
    m2 lane, grp, wave, scan_a, scan_b;
};
__device__ inline Powers powers(const Norm &c, bool pair, int log2n, int log2w, int l)
{
    Powers P;
    // T maps the state before a sample to the state after it at zero input:
    // TDF-II states, or (pair) the last two outputs of 1/A(z).
    const m2 T1 = pair ? m2{0.0, 1.0, -c.a2, -c.a1} : m2{-c.a1, 1.0, -c.a2, 0.0};
    P.ks[0] = mpow_pow2(T1, log2n);          // across one lane (N samples)
    for (int k = 1; k < 6; ++k) P.ks[k] = mmul(P.ks[k - 1], P.ks[k - 1]);
    P.twv = mmul(P.ks[5], P.ks[5]);          // across one wave
    P.tc = mpow_pow2(P.twv, log2w);          // across one group of W waves
    m2 tcp[6];
    tcp[0] = P.tc;
    for (int k = 1; k < 6; ++k) tcp[k] = mmul(tcp[k - 1], tcp[k - 1]);
    P.tw = mmul(tcp[5], tcp[5]);             // across one lookback window
    // per-lane powers by binary expansion of the lane index
    P.lane = mident();
    P.grp = mident();
    P.wave = mident();
    m2 wk = P.twv;
    for (int k = 0; k < 6; ++k) {
        if ((l >> k) & 1) {
            P.lane = mmul(P.lane, P.ks[k]);
            P.grp = mmul(P.grp, tcp[k]);
            P.wave = mmul(P.wave, wk);
        }
        wk = mmul(wk, wk);
    }
    // cross-row steps of the in-wave scan: distance (l%16)+1 from the end of
    // the previous row, and l-31 from lane 31 (used by rows 2 and 3)
    P.scan_a = mpow_bits(P.ks, 6, (l & 15) + 1);
    P.scan_b = mpow_bits(P.ks, 6, l >= 32 ? l - 31 : 0);
    return P;
}

// Fast layout (entries of T): the state-map powers and the impulse response g
// of 1/A(z) rounded to the compute type.
template <typename T>
__device__ void prep_fast(const Norm &c, const float *row, T *t, int log2n, int log2w, int l,
                          bool pair)
{
    const int N = 1 << log2n;
    const Powers P = powers(c, pair, log2n, log2w, l);
    put(t, OFF_LANEPOW + 4 * l, P.lane);
    put(t, OFF_GRPPOW + 4 * l, P.grp);
    if (l < kMaxWaves) put(t, OFF_WPOW + 4 * l, P.wave);
    put(t, OFF_SCANPOW + 8 * l, P.scan_a);
    put(t, OFF_SCANPOW + 8 * l + 4, P.scan_b);
    // impulse response of 1/A(z), stored with g[-1] = 0 first: lane l writes
    // g[l] and g[l + 64] = (T^m)[0][0] of the TDF-II state map T (binary
    // powers, so that no lane runs the length-N recursion)
    {
        m2 p2[7];
        p2[0] = m2{-c.a1, 1.0, -c.a2, 0.0};
        for (int k = 1; k < 7; ++k) p2[k] = mmul(p2[k - 1], p2[k - 1]);
        for (int h = 0; h < 2; ++h) {
            const int m = l + 64 * h;
            t[OFF_G + 1 + m] = (m < N) ? (T)mpow_bits(p2, 7, m).a : T(0);
        }
        if (l == 0) t[OFF_G] = T(0);
    }
    if (l != 0) return;
    if (pair) {
        t[OFF_FIR + 0] = (T)(row[0] * c.inv);
        t[OFF_FIR + 1] = (T)(row[1] * c.inv);
        t[OFF_FIR + 2] = (T)(row[2] * c.inv);
    }
    // level-1 right-hand side taps: B(z) A(-z) (Eq. (23) with a general b0)
    t[OFF_TAPS + 0] = (T)c.b0;
    t[OFF_TAPS + 1] = (T)(c.b1 - c.a1 * c.b0);
    t[OFF_TAPS + 2] = (T)(c.b2 - c.a1 * c.b1 + c.a2 * c.b0);
    t[OFF_TAPS + 3] = (T)(c.a2 * c.b1 - c.a1 * c.b2);
    t[OFF_TAPS + 4] = (T)(c.a2 * c.b2);
    t[OFF_B1] = (T)c.b1;
    t[OFF_B2] = (T)c.b2;
    t[OFF_A1] = (T)c.a1;
    t[OFF_A2] = (T)c.a2;
    // reduction levels: A_{i+1}(w^2) = A_i(w) A_i(-w)
    double e = c.a1, f = c.a2;
    for (int i = 0; i < 8; ++i) {
        t[OFF_E + i] = (T)e;
        t[OFF_F + i] = (T)f;
        const double en = 2.0 * f - e * e;
        f = f * f;
        e = en;
    }
    for (int k = 0; k < 6; ++k) put(t, OFF_KS + 4 * k, P.ks[k]);
    put(t, OFF_TC, P.tc);
    put(t, OFF_TW, P.tw);
    put(t, OFF_TWAVE, P.twv);
}

// Accurate layout: FP64 powers and scalars; FP32 taps, levels and correction
// columns. The free response of a lane's incoming TDF-II state (s1, s2) at
// sample m is g[m] s1 + g[m-1] s2 with g[m] = (T^m)[0][0], g[m-1] =
// (T^m)[0][1] (for the pair carry, the same after its injection into TDF-II
// coordinates). For poles near the real axis the two sequences are nearly
// parallel, so the terms cancel and their rounding is amplified. Instead the
// N x 2 matrix G = [g[m], g[m-1]] is factored as G = Q R (Gram-Schmidt in
// FP64, with one re-orthogonalisation): the kernel applies R to the state in
// FP64 and the orthonormal columns of Q to the samples.
__device__ void prep_accurate(const Norm &c, const float *row, unsigned char *tab, int log2n,
                              int log2w, int l, bool pair)
{
    double *sd = reinterpret_cast<double *>(tab + TAB_HDR);
    float *sp = reinterpret_cast<float *>(tab + kAccSampleOff);
    const int N = 1 << log2n;
    const Powers P = powers(c, pair, log2n, log2w, l);
    put(sd, SD_LANEPOW + 4 * l, P.lane);
    put(sd, SD_GRPPOW + 4 * l, P.grp);
    if (l < kMaxWaves) put(sd, SD_WPOW + 4 * l, P.wave);
    put(sd, SD_SCANPOW + 8 * l, P.scan_a);
    put(sd, SD_SCANPOW + 8 * l + 4, P.scan_b);

    const m2 Tt = m2{-c.a1, 1.0, -c.a2, 0.0};
    m2 p2[7];
    p2[0] = Tt;
    for (int k = 1; k < 7; ++k) p2[k] = mmul(p2[k - 1], p2[k - 1]);
    double c0[2], c1[2];                  // entries m = l and m = l + 64
    for (int h = 0; h < 2; ++h) {
        const int m = l + 64 * h;
        const m2 tm = mpow_bits(p2, 7, m);
        c0[h] = m < N ? tm.a : 0.0;
        c1[h] = m < N ? tm.b : 0.0;
    }
    const double r00 = sqrt(wave_total(c0[0] * c0[0] + c0[1] * c0[1]));   // >= g[0] = 1
    const double q0[2] = {c0[0] / r00, c0[1] / r00};
    const double r01 = wave_total(q0[0] * c1[0] + q0[1] * c1[1]);
    double v[2] = {c1[0] - r01 * q0[0], c1[1] - r01 * q0[1]};
    const double d = wave_total(q0[0] * v[0] + q0[1] * v[1]);
    v[0] -= d * q0[0];
    v[1] -= d * q0[1];
    // > 0 for N >= 2: the rows m = 0, 1 of G are (1, 0) and (-a1, 1)
    const double r11 = sqrt(wave_total(v[0] * v[0] + v[1] * v[1]));
    for (int h = 0; h < 2; ++h) {
        const int m = l + 64 * h;
        sp[AP_Q0 + m] = (float)q0[h];
        sp[AP_Q1 + m] = (float)(v[h] / r11);
    }
    if (l != 0) return;
    sd[SD_R + 0] = r00;
    sd[SD_R + 1] = r01 + d;
    sd[SD_R + 2] = 0.0;
    sd[SD_R + 3] = r11;
    sd[SD_RHO] = peak_gain(row);
    sd[SD_B1] = c.b1;
    sd[SD_B2] = c.b2;
    sd[SD_A1] = c.a1;
    sd[SD_A2] = c.a2;
    for (int k = 0; k < 6; ++k) put(sd, SD_KS + 4 * k, P.ks[k]);
    put(sd, SD_TC, P.tc);
    put(sd, SD_TW, P.tw);
    put(sd, SD_TWAVE, P.twv);
    if (pair) {
        sp[AP_FIR + 0] = (float)(row[0] * c.inv);
        sp[AP_FIR + 1] = (float)(row[1] * c.inv);
        sp[AP_FIR + 2] = (float)(row[2] * c.inv);
    }
    sp[AP_TAPS + 0] = (float)c.b0;
    sp[AP_TAPS + 1] = (float)(c.b1 - c.a1 * c.b0);
    sp[AP_TAPS + 2] = (float)(c.b2 - c.a1 * c.b1 + c.a2 * c.b0);
    sp[AP_TAPS + 3] = (float)(c.a2 * c.b1 - c.a1 * c.b2);
    sp[AP_TAPS + 4] = (float)(c.a2 * c.b2);
    sp[AP_B1] = (float)c.b1;
    sp[AP_B2] = (float)c.b2;
    sp[AP_A1] = (float)c.a1;
    sp[AP_A2] = (float)c.a2;
    double e = c.a1, f = c.a2;
    for (int i = 0; i < 8; ++i) {
        sp[AP_E + i] = (float)e;
        sp[AP_F + i] = (float)f;
        const double en = 2.0 * f - e * e;
        f = f * f;
        e = en;
    }
}

}  // namespace

// Table of section k of a signal whose K rows start at `rows`: row = rows +
// 6 k, tab = its table, log2n = log2(N) samples per lane, log2w = log2(W)
// waves per group (C = 64 W N).
// pair = false: the section itself, carries are TDF-II states (state map T).
// pair = true: the pure recursive part 1/A(z) with the last two outputs as the
// carry (state map Phi = [[0, 1], [-a2, -a1]] on (y[-2], y[-1])), used by the
// adjoint. rho_max: the signal's layout bound (signal_mode). Called by all 64
// lanes of one wave (lane l fills per-lane entries).
template <typename T>
__device__ void prep_section(const float *rows, int K, int k, unsigned char *tab, int log2n,
                             int log2w, unsigned *ctrl, int l, bool pair, double rho_max)
{
    const float *row = rows + 6 * k;
    const Norm c = normalise(row, pair);
    const unsigned mode = signal_mode<T>(rows, K, rho_max);
    if (mode == MODE_ACCURATE)
        prep_accurate(c, row, tab, log2n, log2w, l, pair);
    else
        prep_fast<T>(c, row, reinterpret_cast<T *>(tab + TAB_HDR), log2n, log2w, l, pair);
    if (l == 0) {
        unsigned long long *hdr = reinterpret_cast<unsigned long long *>(tab);
        hdr[HDR_STATUS] = c.status;   // 0 = usable
        hdr[HDR_MODE] = mode;
        if (c.status) atomicOr(&ctrl[CTRL_ERR], c.status);
    }
}

// Plain filter: sections K x 6 -> tabs K x TAB_BYTES. Grid = (K), block = 64.
template <typename T>
__global__ void __launch_bounds__(64)
sos_prep_kernel(const float *__restrict__ sections, int K, int log2n, int log2w,
                unsigned char *__restrict__ tabs, unsigned *__restrict__ ctrl, int pair,
                double rho_max)
{
    const int s = blockIdx.x;
    if (s >= K) return;
    prep_section<T>(sections, K, s, tabs + (size_t)s * TAB_BYTES, log2n, log2w, ctrl,
                    threadIdx.x, pair != 0, rho_max);
}

// Uneven batch: block (i, k) prepares section k of signal i (row and table at
// sec_off[i] + k), so the kernel takes one section's time however long the
// cascades are; signals with inconsistent entries are skipped. Grid =
// (B, max(kmax, 1)), block = 64.
template <typename T>
__global__ void __launch_bounds__(64)
sos_prep_batched_kernel(const float *__restrict__ sections, int B, int kmax, int64_t rows,
                        const int32_t *__restrict__ Ks, const int32_t *__restrict__ sec_off,
                        int log2n, int log2w, unsigned char *__restrict__ tabs,
                        unsigned *__restrict__ ctrl, int pair, double rho_max)
{
    const int i = blockIdx.x;
    const int k = blockIdx.y;
    if (i >= B) return;
    const int K = Ks[i];
    const int64_t so = sec_off[i];
    if (K < 0 || K > kmax || so < 0 || so + K > rows || k >= K) return;
    prep_section<T>(sections + 6 * so, K, k, tabs + (size_t)(so + k) * TAB_BYTES, log2n, log2w,
                    ctrl, threadIdx.x, pair != 0, rho_max);
}

// K sections -> tables for the compute type `bits` (32 or 64). pair != 0: the
// adjoint's tables (recursive parts with output-pair carries). rho_max: see
// signal_mode.
extern "C" hipError_t sos_launch_prep(int bits, const float *sections, int K, int log2n,
                                      int log2w, void *tabs, unsigned *ctrl, int pair,
                                      double rho_max, hipStream_t stream)
{
    if (K <= 0) return hipSuccess;
    if (bits == 64)
        hipLaunchKernelGGL(sos_prep_kernel<double>, dim3(K), dim3(64), 0, stream, sections, K,
                           log2n, log2w, (unsigned char *)tabs, ctrl, pair, rho_max);
    else
        hipLaunchKernelGGL(sos_prep_kernel<float>, dim3(K), dim3(64), 0, stream, sections, K,
                           log2n, log2w, (unsigned char *)tabs, ctrl, pair, rho_max);
    return hipGetLastError();
}

extern "C" hipError_t sos_launch_prep_batched(int bits, const float *sections, int B, int kmax,
                                              int64_t rows, const int32_t *Ks,
                                              const int32_t *sec_off, int log2n, int log2w,
                                              void *tabs, unsigned *ctrl, int pair,
                                              double rho_max, hipStream_t stream)
{
    if (B <= 0) return hipSuccess;
    if (kmax > 65535) return hipErrorInvalidValue;   // grid y limit (callers cap kmax at 64)
    const dim3 grid((unsigned)B, (unsigned)(kmax > 0 ? kmax : 1));
    if (bits == 64)
        hipLaunchKernelGGL(sos_prep_batched_kernel<double>, grid, dim3(64), 0, stream, sections,
                           B, kmax, rows, Ks, sec_off, log2n, log2w, (unsigned char *)tabs, ctrl,
                           pair, rho_max);
    else
        hipLaunchKernelGGL(sos_prep_batched_kernel<float>, grid, dim3(64), 0, stream, sections,
                           B, kmax, rows, Ks, sec_off, log2n, log2w, (unsigned char *)tabs, ctrl,
                           pair, rho_max);
    return hipGetLastError();
}

// Start of a filter launch: ticket counter to 0 and a fresh epoch tag for the
// launch's lookback descriptors (tag 0 is never used). One thread. The filter
// kernels leave the block in this state themselves; this re-establishes it.
extern "C" __global__ void sos_arm_kernel(unsigned *ctrl)
{
    ctrl[CTRL_TICKET] = 0u;
    ctrl[CTRL_DONE] = 0u;
    const unsigned e = ctrl[CTRL_EPOCH] + 1u;
    ctrl[CTRL_EPOCH] = (e == 0u) ? 1u : e;
}

extern "C" hipError_t sos_launch_arm(unsigned *ctrl, hipStream_t stream)
{
    hipLaunchKernelGGL(sos_arm_kernel, dim3(1), dim3(1), 0, stream, ctrl);
    return hipGetLastError();
}
