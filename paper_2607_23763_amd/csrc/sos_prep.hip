// Coefficient preparation on the device (FP64 arithmetic, FP32 tables).
//
// The paper notes that every coefficient of the reduction, the terminal scan
// and the state correction depends only on the filter and is precomputed
// (Sec. II-D, after Eq. (17)). This kernel does that once per coefficient set:
// block s normalises section s by a0, checks it, and writes its table (layout
// in sos_device.h).
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

}  // namespace

// Table of one section: row = [b0 b1 b2 a0 a1 a2], t = its table, log2n =
// log2(N) samples per lane, log2w = log2(W) waves per group (C = 64 W N).
// pair = false: the section itself, carries are TDF-II states (state map T).
// pair = true: the pure recursive part 1/A(z) with the last two outputs as the
// carry (state map Phi = [[0, 1], [-a2, -a1]] on (y[-2], y[-1])), used by the
// adjoint. Called by all 64 lanes of one wave (lane l fills per-lane entries).
template <typename T>
__device__ void prep_section(const float *row, T *t, int log2n, int log2w, unsigned *ctrl, int l,
                             bool pair)
{
    const int N = 1 << log2n;
    const double a0 = (double)row[3];
    unsigned status = 0u;
    if (a0 == 0.0) status |= ERRBIT_A0;
    const double inv = (a0 == 0.0) ? 0.0 : 1.0 / a0;
    const double b0 = pair ? 1.0 : row[0] * inv, b1 = pair ? 0.0 : row[1] * inv;
    const double b2 = pair ? 0.0 : row[2] * inv;
    const double a1 = row[4] * inv, a2 = row[5] * inv;
    // closed stability triangle of z^2 + a1 z + a2 (NaN fails the test)
    if (!(fabs(a2) <= 1.0 && fabs(a1) <= 1.0 + a2)) status |= ERRBIT_UNSTABLE;

    // T maps the TDF-II state before a sample to the state after it at zero input.
    const m2 T1 = pair ? m2{0.0, 1.0, -a2, -a1} : m2{-a1, 1.0, -a2, 0.0};
    const m2 TN = mpow_pow2(T1, log2n);     // across one lane (N samples)
    m2 ks[6];
    ks[0] = TN;
    for (int k = 1; k < 6; ++k) ks[k] = mmul(ks[k - 1], ks[k - 1]);
    const m2 TWV = mmul(ks[5], ks[5]);       // TN^64: across one wave
    const m2 TC = mpow_pow2(TWV, log2w);     // across one group of W waves
    m2 tcp[6];
    tcp[0] = TC;
    for (int k = 1; k < 6; ++k) tcp[k] = mmul(tcp[k - 1], tcp[k - 1]);
    const m2 TW = mmul(tcp[5], tcp[5]);      // TC^64: across one lookback window

    // per-lane powers by binary expansion of the lane index
    m2 lp = mident(), gp = mident(), wp = mident(), wk = TWV;
    for (int k = 0; k < 6; ++k) {
        if ((l >> k) & 1) {
            lp = mmul(lp, ks[k]);
            gp = mmul(gp, tcp[k]);
            wp = mmul(wp, wk);
        }
        wk = mmul(wk, wk);
    }
    put(t, OFF_LANEPOW + 4 * l, lp);
    put(t, OFF_GRPPOW + 4 * l, gp);
    if (l < kMaxWaves) put(t, OFF_WPOW + 4 * l, wp);
    // cross-row steps of the in-wave scan: distance (l%16)+1 from the end of
    // the previous row, and l-31 from lane 31 (used by rows 2 and 3)
    {
        const int ea = (l & 15) + 1, eb = l >= 32 ? l - 31 : 0;
        m2 pa = mident(), pb = mident();
        for (int k = 0; k < 6; ++k) {
            if ((ea >> k) & 1) pa = mmul(pa, ks[k]);
            if ((eb >> k) & 1) pb = mmul(pb, ks[k]);
        }
        put(t, OFF_SCANPOW + 8 * l, pa);
        put(t, OFF_SCANPOW + 8 * l + 4, pb);
    }

    if (l == 0) {
        t[OFF_STATUS] = (T)status;   // 0 = usable
        if (pair) {
            t[OFF_FIR + 0] = (T)(row[0] * inv);
            t[OFF_FIR + 1] = (T)(row[1] * inv);
            t[OFF_FIR + 2] = (T)(row[2] * inv);
        }
        // level-1 right-hand side taps: B(z) A(-z) (Eq. (23) with a general b0)
        t[OFF_TAPS + 0] = (T)b0;
        t[OFF_TAPS + 1] = (T)(b1 - a1 * b0);
        t[OFF_TAPS + 2] = (T)(b2 - a1 * b1 + a2 * b0);
        t[OFF_TAPS + 3] = (T)(a2 * b1 - a1 * b2);
        t[OFF_TAPS + 4] = (T)(a2 * b2);
        t[OFF_B1] = (T)b1;
        t[OFF_B2] = (T)b2;
        t[OFF_A1] = (T)a1;
        t[OFF_A2] = (T)a2;
        // reduction levels: A_{i+1}(w^2) = A_i(w) A_i(-w)
        double e = a1, f = a2;
        for (int i = 0; i < 8; ++i) {
            t[OFF_E + i] = (T)e;
            t[OFF_F + i] = (T)f;
            const double en = 2.0 * f - e * e;
            f = f * f;
            e = en;
        }
        // impulse response of 1/A(z), stored with g[-1] = 0 first
        t[OFF_G] = T(0);
        double gm2 = 0.0, gm1 = 0.0;
        for (int m = 0; m < kMaxN; ++m) {
            const double g = (m == 0) ? 1.0 : (-a1 * gm1 - a2 * gm2);
            t[OFF_G + 1 + m] = (m < N) ? (T)g : T(0);
            gm2 = gm1;
            gm1 = g;
        }
        for (int k = 0; k < 6; ++k) put(t, OFF_KS + 4 * k, ks[k]);
        put(t, OFF_TC, TC);
        put(t, OFF_TW, TW);
        put(t, OFF_TWAVE, TWV);
        if (status) atomicOr(&ctrl[CTRL_ERR], status);
    }
}

// Plain filter: sections K x 6 -> tabs K x TAB_FLOATS. Grid = (K), block = 64.
template <typename T>
__global__ void __launch_bounds__(64)
sos_prep_kernel(const float *__restrict__ sections, int K, int log2n, int log2w,
                T *__restrict__ tabs, unsigned *__restrict__ ctrl, int pair)
{
    const int s = blockIdx.x;
    if (s >= K) return;
    prep_section<T>(sections + 6 * s, tabs + (size_t)s * TAB_FLOATS, log2n, log2w, ctrl,
                    threadIdx.x, pair != 0);
}

// Uneven batch: block (i, k) prepares section k of signal i (row and table at
// sec_off[i] + k), so the kernel takes one section's time however long the
// cascades are; signals with inconsistent entries are skipped. Grid =
// (B, max(kmax, 1)), block = 64.
template <typename T>
__global__ void __launch_bounds__(64)
sos_prep_batched_kernel(const float *__restrict__ sections, int B, int kmax, int64_t rows,
                        const int32_t *__restrict__ Ks, const int32_t *__restrict__ sec_off,
                        int log2n, int log2w, T *__restrict__ tabs, unsigned *__restrict__ ctrl,
                        int pair)
{
    const int i = blockIdx.x;
    const int k = blockIdx.y;
    if (i >= B) return;
    const int K = Ks[i];
    const int64_t so = sec_off[i];
    if (K < 0 || K > kmax || so < 0 || so + K > rows || k >= K) return;
    prep_section<T>(sections + 6 * (so + k), tabs + (size_t)(so + k) * TAB_FLOATS, log2n, log2w,
                    ctrl, threadIdx.x, pair != 0);
}

// K sections -> tables of the compute type `bits` (32 or 64). pair != 0: the
// adjoint's tables (recursive parts with output-pair carries).
extern "C" hipError_t sos_launch_prep(int bits, const float *sections, int K, int log2n,
                                      int log2w, void *tabs, unsigned *ctrl, int pair,
                                      hipStream_t stream)
{
    if (K <= 0) return hipSuccess;
    if (bits == 64)
        hipLaunchKernelGGL(sos_prep_kernel<double>, dim3(K), dim3(64), 0, stream, sections, K,
                           log2n, log2w, (double *)tabs, ctrl, pair);
    else
        hipLaunchKernelGGL(sos_prep_kernel<float>, dim3(K), dim3(64), 0, stream, sections, K,
                           log2n, log2w, (float *)tabs, ctrl, pair);
    return hipGetLastError();
}

extern "C" hipError_t sos_launch_prep_batched(int bits, const float *sections, int B, int kmax,
                                              int64_t rows, const int32_t *Ks,
                                              const int32_t *sec_off, int log2n, int log2w,
                                              void *tabs, unsigned *ctrl, int pair,
                                              hipStream_t stream)
{
    if (B <= 0) return hipSuccess;
    if (kmax > 65535) return hipErrorInvalidValue;   // grid y limit (callers cap kmax at 64)
    const dim3 grid((unsigned)B, (unsigned)(kmax > 0 ? kmax : 1));
    if (bits == 64)
        hipLaunchKernelGGL(sos_prep_batched_kernel<double>, grid, dim3(64), 0, stream, sections,
                           B, kmax, rows, Ks, sec_off, log2n, log2w, (double *)tabs, ctrl, pair);
    else
        hipLaunchKernelGGL(sos_prep_batched_kernel<float>, grid, dim3(64), 0, stream, sections,
                           B, kmax, rows, Ks, sec_off, log2n, log2w, (float *)tabs, ctrl, pair);
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
