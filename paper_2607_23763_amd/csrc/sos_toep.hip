// Whole-cascade block-Toeplitz filter on gfx950's matrix cores.
//
// Sec. II-B splits the multi-block system of one section into a
// non-recursive stage (a block-Toeplitz product with the input) and a
// recursive stage that couples consecutive blocks only through two carried
// values. Applied to the whole cascade at once, with the K sections' TDF-II
// states stacked into one state s of dimension 2K <= 16 (zero-padded to 16),
// the same split over a column of M = 64 consecutive samples x reads
//     y  = T x + O s            (T: M x M lower-triangular Toeplitz matrix of
//                                the cascade's impulse response h; O: rows
//                                c Phi^i, the response to each state entry)
//     s' = A s + Gam x          (A = Phi^M; Gam: columns Phi^(M-1-k) gamma)
// for the one-sample state map Phi, input vector gamma, output row c and
// feedthrough d of the cascade. All three products are dense FP32
// contractions, done with v_mfma_f32_16x16x4_f32: a tile of 16 columns (1024
// consecutive samples) is one MFMA operand, the columns being the MFMA's N
// dimension. The per-sample cost no longer grows with K (about 40 MACs per
// sample for T and 16 each for Gam and O, against about 8 FMAs per sample and
// section for the per-section recurrences), which is why this path serves the
// highest orders.
//
// Group structure (one workgroup of 8 waves, two tiles per wave, CG = 16384
// samples per group, NG = 2, 4 or 8 groups per chunk, one chunk per ticket;
// the host takes 8 for long signals and fewer where 8-group chunks would not
// give every workgroup several chunks):
//   1. Each wave forms T x and Gam x for its tiles straight from the 128-bit
//      loads: lane l holds samples 16b + 4(l/16) + {0..3} of column l%16
//      for blocks b = 0..3, which is exactly the MFMA's B operand for the
//      k-steps of block b (the reduction order of k is free, so the k index
//      of a step is permuted to match what a lane loaded). The output has
//      the same per-lane layout, so no sample passes through LDS.
//   2. A Kogge-Stone scan over the tile's 16 columns composes the columns'
//      end states from rest: each level shifts the 16 x 16 state matrix by
//      2^j columns with one DPP row shift per register (the 16 columns are
//      the 16 lanes of a DPP row) and adds A^(2^j) times it with four MFMAs.
//   3. Wave 0 scans each group's 16 tile totals the same way (powers of
//      Phi^1024), chains the chunk's groups into its end state from rest,
//      publishes that aggregate (16 words), resolves the chunk's incoming
//      state by decoupled lookback over 16-word descriptors (Sec. IV-B; one
//      lookback per chunk instead of one per group and section), publishes
//      the chunk's inclusive state and derives every tile's incoming state.
//   4. Every column's incoming state follows from its tile's through powers
//      of Phi^64; y += O s with four MFMAs per 16 output rows, and the tile
//      is stored.
// Conditioning: the state is scaled by a power-of-two diagonal D (exact) that
// balances Gam's rows against O's columns, so every table entry is O(1)
// whatever the scaling of the TDF-II states. The tables are built in FP64 by
// sos_toep_prep_kernel and rounded once to FP32.
#include "sos_device.h"
#include "sosfilt.h"

using namespace sosdev;

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef __attribute__((address_space(1))) f4u gf4u;

constexpr int S = 16;            // state dimension (2K <= 16)
constexpr int M = 64;            // samples per column
constexpr int TC = 16;           // columns per tile
constexpr int TS = M * TC;       // samples per tile
constexpr int WT = 8;            // waves per workgroup
constexpr int TPW = 2;           // tiles per wave
constexpr int NT = WT * TPW;     // tiles per group
constexpr int CG = TS * NT;      // samples per group
constexpr int kMaxNG = 8;        // groups per chunk (one ticket, one lookback): 2, 4 or 8
constexpr int kMaxDist = 32;     // lookback reach in chunks: powers H^d, d < kMaxDist
constexpr int kDescWords = 32;   // per chunk: 16 aggregate words, 16 inclusive words
constexpr int kPowStride = 260;  // LDS stride of a 16 x 16 power (bank-spread across lanes)
static_assert(NT == 16, "the group-level scan covers one 16-column MFMA tile");

// Table layout (floats). The operand blocks are stored per lane, four k-steps
// per lane, so that every lane loads its A operands with one 128-bit load.
enum : int {
    TT_GATE = 0,          // 1.0f when this path filters the signal, else 0.0f
    TT_K = 1,             // sections (as a float)
    TT_NG = 2,            // groups per chunk the chunk map H was formed for (as a float)
    TT_D = 16,            // [16] state scale: TDF-II state = D * kernel state
    TT_DINV = 32,         // [16]
    TT_TOP = 64,          // [4 delta][64 lanes][4 s]: T operands, block pair r - b = delta
    TT_GOP = TT_TOP + 1024,    // [4 b][64][4]: Gam operands of block b
    TT_OOP = TT_GOP + 1024,    // [4 r][64][4]: O operands of output rows 16r..16r+15
    TT_AOP = TT_OOP + 1024,    // [4 j][64][4]: A^(2^j) operands (column scan)
    TT_BOP = TT_AOP + 1024,    // [4 j][64][4]: (Phi^1024)^(2^j) operands (tile scan)
    TT_PHI = TT_BOP + 1024,    // [16][16] Phi (row-major): final state of a ragged end
    TT_GAM = TT_PHI + 256,     // [16] gamma
    TT_ACOL = TT_GAM + 16,     // [16 c][16][16] A^c: tile state -> column c
    TT_BTILE = TT_ACOL + 4096, // [16 t][16][16] (Phi^1024)^t: group state -> tile t
    TT_G1 = TT_BTILE + 4096,   // [16][16] G = Phi^C: across one group
    TT_HPOW = TT_G1 + 256,     // [kMaxDist d][16][16] H^d, H = G^NG: d chunks back
    TT_FLOATS = TT_HPOW + kMaxDist * 256
};
constexpr int kLdsMats = TC + NT + 1 + kMaxDist;   // matrices staged into LDS
static_assert((TT_ACOL % 4) == 0 && (TT_HPOW % 4) == 0, "128-bit rows");
static_assert(TT_BTILE == TT_ACOL + 16 * 256 && TT_G1 == TT_BTILE + 16 * 256 &&
                  TT_HPOW == TT_G1 + 256 && TT_FLOATS == TT_ACOL + kLdsMats * 256,
              "the power tables are contiguous (staged into LDS in one pass)");

// ------------------------------------------------------------ preparation

// FP64 16 x 16 matrices in LDS are stored with a row stride of 17 doubles,
// so that the 16 rows a product reads at once fall in different banks.
constexpr int RS = 17;
constexpr int MSZ = 16 * RS;
__device__ __forceinline__ int ent(int tid) { return (tid >> 4) * RS + (tid & 15); }

typedef double v4d __attribute__((ext_vector_type(4)));

// Z = X Y by one wave on the FP64 matrix cores (v_mfma_f64_16x16x4f64, four
// k-steps): lane l supplies X[l%16][4s + l/16] and Y[4s + l/16][l%16] at step
// s and receives Z[4 r + l/16][l%16] in register r (the FP64 instruction's
// result layout, unlike the FP32 one's 4 (l/16) + r); each lane reads 8
// doubles from LDS instead of the 32 a product per thread reads.
__device__ inline v4d mm16m_acc(const double *X, const double *Y, int lane)
{
    const int n = lane & 15, g = lane >> 4;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[n * RS + 4 * s + g], Y[(4 * s + g) * RS + n],
                                                   acc, 0, 0, 0);
    return acc;
}

__device__ inline void mm16m(const double *X, const double *Y, double *Z, int lane)
{
    const v4d acc = mm16m_acc(X, Y, lane);
    const int n = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) Z[(4 * r + g) * RS + n] = acc[r];
}

// The same product with the operands read through accessors x(row, k) and
// y(k, column).
template <typename FX, typename FY>
__device__ inline v4d mm16f_acc(FX x, FY y, int lane)
{
    const int n = lane & 15, g = lane >> 4;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x(n, 4 * s + g), y(4 * s + g, n), acc, 0, 0, 0);
    return acc;
}

__device__ inline void ident16(double *Z, int tid)
{
    Z[ent(tid)] = (tid >> 4) == (tid & 15) ? 1.0 : 0.0;
}

struct PrepLds {
    double co[8][5];          // b0 b1 b2 a1 a2 per section (normalised)
    double phi[MSZ];          // one-sample state map
    double gam[16], crow[16], dd;
    double q[7][MSZ];         // Phi^(2^j), j = 0..6
    double v[64][17];         // Phi^i gamma (rows padded: 16 rows at once hit distinct banks)
    double o[64][17];         // c Phi^i
    double dsc[16];           // state scale D
    double h[64];             // the cascade's impulse response
    double pw[9][MSZ];        // A^(1,2,4,8), B^(1,2,4,8), G (scaled basis)
    double work[32][MSZ];     // power tables, reused
    int gate;
};

// One block of 256 threads: every table of the path for one cascade of K
// sections (K <= 8) and chunks of ng groups, in FP64, rounded once to FP32.
__global__ void __launch_bounds__(256) sos_toep_prep_kernel(const float *sections, int K, int ng,
                                                            double rho_gate, float *tt)
{
    __shared__ PrepLds sh;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;   // 16 x 16 products: one wave each
    if (tid == 0) sh.gate = (K >= 1 && K <= 8) ? 1 : 0;
    for (int e = tid; e < MSZ; e += 256) sh.phi[e] = 0.0;
    if (tid < 16) { sh.gam[tid] = 0.0; sh.crow[tid] = 0.0; }
    __syncthreads();
    if (!sh.gate) {
        if (tid == 0) { tt[TT_GATE] = 0.0f; tt[TT_K] = (float)K; }
        return;
    }
    // sections: normalise; an unusable or (for the automatic choice) too
    // resonant section leaves the signal to the per-section kernels, which
    // also report it
    if (tid < K) {
        const float *r = sections + 6 * tid;
        const double a0 = r[3];
        const double a1 = r[4] / a0, a2 = r[5] / a0;
        const bool stable = a0 != 0.0 && fabs(a2) < 1.0 && fabs(a1) < 1.0 + a2;
        if (!stable || !gain_within(r, rho_gate)) atomicAnd(&sh.gate, 0);
        sh.co[tid][0] = r[0] / a0;
        sh.co[tid][1] = r[1] / a0;
        sh.co[tid][2] = r[2] / a0;
        sh.co[tid][3] = a1;
        sh.co[tid][4] = a2;
    }
    __syncthreads();
    if (!sh.gate) {
        if (tid == 0) { tt[TT_GATE] = 0.0f; tt[TT_K] = (float)K; }
        return;
    }
    const int n2 = 2 * K;
    // Phi, gamma, c, d: one sample of the cascade from state e_j (j < 2K) or
    // from input 1 (j = 2K)
    if (tid <= n2) {
        double s[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) s[i] = (i == tid && tid < n2) ? 1.0 : 0.0;
        double v = tid == n2 ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {   // constant indices into s (K <= 8)
            if (k < K) {
                const double y = sh.co[k][0] * v + s[2 * k];
                const double z1 = sh.co[k][1] * v - sh.co[k][3] * y + s[2 * k + 1];
                const double z2 = sh.co[k][2] * v - sh.co[k][4] * y;
                s[2 * k] = z1;
                s[2 * k + 1] = z2;
                v = y;
            }
        }
        if (tid < n2) {
            for (int i = 0; i < 16; ++i) sh.phi[i * RS + tid] = s[i];
            sh.crow[tid] = v;
        } else {
            for (int i = 0; i < 16; ++i) sh.gam[i] = s[i];
            sh.dd = v;
        }
    }
    __syncthreads();
    // v_i = Phi^i gamma and o_i = c Phi^i, i < 64, by doubling with
    // Q_j = Phi^(2^j): v_(h+c) = Q_j v_c and o_(h+c) = o_c Q_j for c < h = 2^j,
    // as 16-column blocks on the FP64 matrix cores, while one wave squares
    // Q_j into Q_(j+1)
    sh.q[0][ent(tid)] = sh.phi[ent(tid)];
    if (tid < 16) {
        sh.v[0][tid] = sh.gam[tid];
        sh.o[0][tid] = sh.crow[tid];
    }
    __syncthreads();
    for (int j = 0; j < 6; ++j) {
        const int half = 1 << j;
        const int nb = half < 16 ? 1 : half / 16;   // 16-column blocks
        const double *Q = sh.q[j];
        const int n = lane & 15, g = lane >> 4;
        // products of this step: the square, nb blocks of v, nb blocks of o
        for (int p = wv; p < 1 + 2 * nb; p += 4) {
            if (p == 0) {
                mm16m(sh.q[j], sh.q[j], sh.q[j + 1], lane);
            } else if (p <= nb) {
                const int b = 16 * (p - 1);   // Z[i][c] = (Q_j v_(b+c))[i]
                const v4d acc = mm16f_acc(
                    [&](int i, int k) { return Q[i * RS + k]; },
                    [&](int k, int c) {
                        const double e = sh.v[(b + c) & 63][k];
                        return b + c < half ? e : 0.0;
                    },
                    lane);
                if (b + n < half) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) sh.v[half + b + n][4 * r + g] = acc[r];
                }
            } else {
                const int b = 16 * (p - 1 - nb);   // Z[c][m] = (o_(b+c) Q_j)[m]
                const v4d acc = mm16f_acc(
                    [&](int c, int k) {
                        const double e = sh.o[(b + c) & 63][k];
                        return b + c < half ? e : 0.0;
                    },
                    [&](int k, int m) { return Q[k * RS + m]; }, lane);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (b + 4 * r + g < half) sh.o[half + b + 4 * r + g][n] = acc[r];
            }
        }
        __syncthreads();
    }
    // impulse response h[0] = d, h[m] = c Phi^(m-1) gamma
    if (tid < 64) {
        double acc = tid == 0 ? sh.dd : 0.0;
        if (tid > 0)
            for (int k = 0; k < 16; ++k) acc = fma(sh.o[tid - 1][k], sh.gam[k], acc);
        sh.h[tid] = acc;
    }
    // balancing scale: a power of two per state entry equalising the energy
    // of its Gam row and O column over one column (exact in every format);
    // each energy is summed in 16 parts (work[0..1] hold them) and then added
    {
        const int e = tid & 15, part = tid >> 4;
        double sv = 0.0, so = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = part + 16 * q;
            sv = fma(sh.v[i][e], sh.v[i][e], sv);
            so = fma(sh.o[i][e], sh.o[i][e], so);
        }
        static_assert(MSZ >= 256, "one partial sum per thread");
        sh.work[0][tid] = sv;
        sh.work[1][tid] = so;
    }
    __syncthreads();
    if (tid < 16) {
        double sv = 0.0, so = 0.0;
        for (int part = 0; part < 16; ++part) {
            sv += sh.work[0][16 * part + tid];
            so += sh.work[1][16 * part + tid];
        }
        double d = 1.0;
        if (sv > 0.0 && so > 0.0 && isfinite(sv) && isfinite(so)) {
            int e = (int)rint(0.25 * log2(sv / so));
            e = e < -60 ? -60 : (e > 60 ? 60 : e);
            d = ldexp(1.0, e);
        }
        sh.dsc[tid] = d;
    }
    __syncthreads();
    // scaled basis: Phi' = D^-1 Phi D (all powers alike), gamma' = D^-1 gamma,
    // c' = c D; A = Phi'^64
    {
        const int i = tid >> 4, j = tid & 15;
        const double f = sh.dsc[j] / sh.dsc[i];
        sh.pw[0][ent(tid)] = sh.q[6][ent(tid)] * f;       // A
        tt[TT_PHI + tid] = (float)(sh.phi[ent(tid)] * f);
        if (tid < 16) {
            tt[TT_GAM + tid] = (float)(sh.gam[tid] / sh.dsc[tid]);
            tt[TT_D + tid] = (float)sh.dsc[tid];
            tt[TT_DINV + tid] = (float)(1.0 / sh.dsc[tid]);
        }
    }
    __syncthreads();
    // per-lane MFMA operands (TT_TOP order): lane l = 16 g + n, k-step s
    auto operand = [&](int e) {
        const int blk = e >> 10, r = e & 1023;
        const int idx = r >> 8, ln = (r >> 2) & 63, s = r & 3;
        const int n = ln & 15, g = ln >> 4;
        double val;
        if (blk == 0) {            // T: h[16 delta + n - 4g - s]
            const int m = 16 * idx + n - 4 * g - s;
            val = m < 0 ? 0.0 : sh.h[m];
        } else if (blk == 1) {     // Gam'[n][16 b + 4 g + s] = (Phi^(63-k) gamma)[n] / D[n]
            const int k = 16 * idx + 4 * g + s;
            val = sh.v[63 - k][n] / sh.dsc[n];
        } else if (blk == 2) {     // O'[16 r + n][4 g + s] = (c Phi^i)[state] D[state]
            const int st = 4 * g + s;
            val = sh.o[16 * idx + n][st] * sh.dsc[st];
        } else {                   // A^(2^j) or B^(2^j): [n][4 g + s]
            const double *Pm = sh.pw[(blk == 3 ? 0 : 4) + idx];
            val = Pm[n * RS + 4 * g + s];
        }
        tt[TT_TOP + e] = (float)val;
    };
    // A^2, A^4, A^8, B = A^16, B^2, B^4, B^8, G = B^16 = Phi'^C by wave 0
    // alone (a wave's LDS accesses complete in order), while the other
    // three waves write the T, Gam and O operands, which need none of them
    if (wv == 0) {
        for (int j = 0; j < 8; ++j) {
            mm16m(sh.pw[j], sh.pw[j], sh.pw[j + 1], lane);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    } else {
        static_assert(3 * 1024 % 192 == 0, "T, Gam and O operands over waves 1-3");
#pragma unroll 4
        for (int i = 0; i < 3 * 1024 / 192; ++i) operand(tid - 64 + 192 * i);
    }
    __syncthreads();
    // column powers A^c (work[0..15]) and tile powers B^t (work[16..31])
    ident16(sh.work[0], tid);
    ident16(sh.work[16], tid);
    sh.work[1][ent(tid)] = sh.pw[0][ent(tid)];
    sh.work[17][ent(tid)] = sh.pw[4][ent(tid)];
    __syncthreads();
    for (int j = 1; j < 4; ++j) {
        const int half = 1 << j;
        for (int p = wv; p < 2 * half; p += 4) {   // products spread over the waves
            const int c = p >> 1;
            if (p & 1)
                mm16m(sh.pw[4 + j], sh.work[16 + c], sh.work[16 + half + c], lane);
            else
                mm16m(sh.pw[j], sh.work[c], sh.work[half + c], lane);
        }
        __syncthreads();
    }
    for (int c = 0; c < 16; ++c) {
        tt[TT_ACOL + c * 256 + tid] = (float)sh.work[c][ent(tid)];
        tt[TT_BTILE + c * 256 + tid] = (float)sh.work[16 + c][ent(tid)];
    }
    __syncthreads();
    tt[TT_G1 + tid] = (float)sh.pw[8][ent(tid)];
    // chunk map H = G^NG by squaring (work[18]), then its powers H^d,
    // d < kMaxDist, as (H^8)^a H^b: low factors work[0..7], high factors
    // work[8..11]
    sh.work[18][ent(tid)] = sh.pw[8][ent(tid)];
    __syncthreads();
    for (int k = 1; k < ng; k <<= 1) {
        if (wv == 0) mm16m(sh.work[18], sh.work[18], sh.work[19], lane);
        __syncthreads();
        sh.work[18][ent(tid)] = sh.work[19][ent(tid)];
        __syncthreads();
    }
    ident16(sh.work[0], tid);
    ident16(sh.work[8], tid);
    sh.work[1][ent(tid)] = sh.work[18][ent(tid)];
    __syncthreads();
    if (wv == 0) mm16m(sh.work[18], sh.work[18], sh.work[16], lane);      // H^2
    __syncthreads();
    if (wv == 0) mm16m(sh.work[16], sh.work[16], sh.work[17], lane);      // H^4
    if (wv == 1) mm16m(sh.work[16], sh.work[1], sh.work[3], lane);        // H^3
    sh.work[2][ent(tid)] = sh.work[16][ent(tid)];
    __syncthreads();
    mm16m(sh.work[17], sh.work[wv], sh.work[4 + wv], lane);               // H^4..7
    __syncthreads();
    if (wv == 0) mm16m(sh.work[17], sh.work[17], sh.work[9], lane);       // H^8
    __syncthreads();
    if (wv == 0) mm16m(sh.work[9], sh.work[9], sh.work[10], lane);        // H^16
    __syncthreads();
    if (wv == 0) mm16m(sh.work[10], sh.work[9], sh.work[11], lane);       // H^24
    __syncthreads();
    static_assert(kMaxDist <= 32, "high factors H^0, H^8, H^16, H^24");
    static_assert(kMaxDist % 8 == 0, "two independent products per wave and pass");
    for (int d = wv; d < kMaxDist; d += 8) {
        const v4d a0 = mm16m_acc(sh.work[8 + (d >> 3)], sh.work[d & 7], lane);
        const v4d a1 = mm16m_acc(sh.work[8 + ((d + 4) >> 3)], sh.work[(d + 4) & 7], lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int at = (4 * r + (lane >> 4)) * 16 + (lane & 15);
            tt[TT_HPOW + d * 256 + at] = (float)a0[r];
            tt[TT_HPOW + (d + 4) * 256 + at] = (float)a1[r];
        }
    }
    // the scan operands (powers of A and B)
#pragma unroll
    for (int i = 0; i < 2 * 1024 / 256; ++i) operand(3 * 1024 + tid + 256 * i);
    if (tid == 0) {
        tt[TT_K] = (float)K;
        tt[TT_NG] = (float)ng;
        tt[TT_GATE] = 1.0f;
    }
}

// ------------------------------------------------------------------ filter

struct ToepArgs {
    const float *x;
    float *y;
    int64_t n;
    const float *tt;
    const float *zi;           // K x 2 TDF-II states, or null
    float *zf;                 // K x 2, or null
    int K;
    int64_t groups;            // groups of CG samples (the last may be partial)
    int64_t total;             // chunks of NG groups (tickets)
    unsigned long long *desc;  // kDescWords per chunk
    unsigned *ctrl;
    unsigned long long timeout_ticks;
};

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// DPP row shift right by D inside each 16-lane row; lanes whose source lies
// before the row start read 0.
template <int D>
__device__ __forceinline__ v4f row_shr(v4f v)
{
    v4f r;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        r[j] = __int_as_float(
            __builtin_amdgcn_update_dpp(0, __float_as_int(v[j]), 0x110 + D, 0xF, 0xF, true));
    return r;
}

// Inclusive scan over the 16 columns of P (state 4 (l/16) + j, column l % 16
// in lane l, register j): P[:, c] <- sum_{i <= c} X^(c-i) P[:, i], with
// op[j] the A operands of X^(2^j).
__device__ __forceinline__ v4f scan16(v4f P, const v4f (&op)[4])
{
    {
        const v4f sh = row_shr<1>(P);
#pragma unroll
        for (int s = 0; s < 4; ++s) P = mfma4(op[0][s], sh[s], P);
    }
    {
        const v4f sh = row_shr<2>(P);
#pragma unroll
        for (int s = 0; s < 4; ++s) P = mfma4(op[1][s], sh[s], P);
    }
    {
        const v4f sh = row_shr<4>(P);
#pragma unroll
        for (int s = 0; s < 4; ++s) P = mfma4(op[2][s], sh[s], P);
    }
    {
        const v4f sh = row_shr<8>(P);
#pragma unroll
        for (int s = 0; s < 4; ++s) P = mfma4(op[3][s], sh[s], P);
    }
    return P;
}

__device__ __forceinline__ v4f ld4(const float *p)
{
    return *reinterpret_cast<const v4f *>(p);
}

// Sum over the wave of z[m] for m = lane / 4, in every lane of that quad
// (reduce-scatter over lane bits 5..2, then a sum over bits 1..0).
__device__ __forceinline__ float reduce16(const float (&z)[16], int lane)
{
    float a8[8], a4[4], a2[2];
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float send = b5 ? z[i] : z[8 + i];
        a8[i] = (b5 ? z[8 + i] : z[i]) + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float send = b4 ? a8[i] : a8[4 + i];
        a4[i] = (b4 ? a8[4 + i] : a8[i]) + __shfl_xor(send, 16);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float send = b3 ? a4[i] : a4[2 + i];
        a2[i] = (b3 ? a4[2 + i] : a4[i]) + __shfl_xor(send, 8);
    }
    float a1 = (b2 ? a2[1] : a2[0]) + __shfl_xor(b2 ? a2[0] : a2[1], 4);
    a1 += __shfl_xor(a1, 1);
    a1 += __shfl_xor(a1, 2);
    return a1;
}

__device__ __forceinline__ unsigned long long pack_word(float v, unsigned tag)
{
    return ((unsigned long long)tag << 32) | (unsigned long long)__float_as_uint(v);
}
__device__ __forceinline__ void put_word(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long get_word(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled lookback of chunk t (t > 0) over 16-word descriptors, by one
// whole wave; leaves the chunk's incoming state in sg[16].
//
// Each round lane p reads the unconsumed predecessor p places back (up to
// kMaxDist chunks back; its 16 aggregate and 16 inclusive words); the wave
// takes the longest
// ready prefix and, when an inclusive state lies in it, ends with that state.
// A consumed state at distance d reaches this chunk through H^d (H the state
// map across a chunk), from the LDS copy of the table: each lane forms H^d v
// for its predecessor and the wave sums the 64 vectors. The aggregate of the
// predecessor at distance kMaxDist - 1 is never consumed, so a walk that far
// waits for that predecessor's inclusive state, which every chunk publishes.
// On timeout the state is NaN and the error bit is set.
__device__ void toep_lookback(const ToepArgs &a, const float *hpow, int64_t t, unsigned epoch,
                              int lane, float *sg)
{
    float acc = 0.0f;
    int dbase = 0;
    const unsigned long long t0 = wall_clock64();
    for (;;) {
        const int dist = dbase + lane;
        const bool valid = dist < kMaxDist && (int64_t)dist < t;
        unsigned long long wa[16], wi[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) wa[i] = wi[i] = 0ull;
        if (valid) {
            const unsigned long long *d = a.desc + (size_t)(t - 1 - dist) * kDescWords;
#pragma unroll
            for (int i = 0; i < 16; ++i) wa[i] = get_word(d + i);
#pragma unroll
            for (int i = 0; i < 16; ++i) wi[i] = get_word(d + 16 + i);
        }
        bool aok = valid && dist < kMaxDist - 1, iok = valid;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            aok = aok && (unsigned)(wa[i] >> 32) == epoch;
            iok = iok && (unsigned)(wi[i] >> 32) == epoch;
        }
        const unsigned long long ra = __ballot(aok), ri = __ballot(iok);
        const unsigned long long rdy = ra | ri;
        const int nr = ~rdy ? __builtin_ctzll(~rdy) : 64;
        const int js = ri ? __builtin_ctzll(ri) : 64;
        const bool done = js < nr;
        const int c = done ? js : nr;
        if (c > 0 || done) {
            const bool use_a = lane < c, use_i = done && lane == js;
            float z[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) z[m] = 0.0f;
            if (use_a || use_i) {
                float v[16];
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    v[i] = __uint_as_float((unsigned)(use_a ? wa[i] : wi[i]));
                const float *gm = hpow + dist * kPowStride;
#pragma unroll
                for (int m = 0; m < 16; ++m) {
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) {
                        const v4f r = ld4(gm + 16 * m + 4 * k4);
                        z[m] += r.x * v[4 * k4] + r.y * v[4 * k4 + 1] + r.z * v[4 * k4 + 2] +
                                r.w * v[4 * k4 + 3];
                    }
                }
            }
            acc += reduce16(z, lane);
            if (done) break;
            dbase += c;
            continue;
        }
        if (wall_clock64() - t0 > a.timeout_ticks) {
            if (lane == 0) atomicOr(&a.ctrl[CTRL_ERR], ERRBIT_TIMEOUT);
            acc = __builtin_nanf("");
            break;
        }
        __builtin_amdgcn_s_sleep(2);   // a short fixed sleep between polls
    }
    if ((lane & 3) == 0) sg[lane >> 2] = acc;
}

// The tile starting at signal sample t0: lane l's four blocks (samples
// 64 (l%16) + 16 b + 4 (l/16) + {0..3} of the tile), zero past n.
__device__ __forceinline__ void load_tile(v4f (&xb)[4], const float *x, int64_t n, int64_t t0,
                                          int lane)
{
    const int64_t q0 = t0 + 64 * (lane & 15) + 4 * (lane >> 4);
    if (t0 + TS <= n) {
        const gf4u *p = (const gf4u *)(x + q0);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const f4u v = __builtin_nontemporal_load(p + 4 * b);
            xb[b] = v4f{v.x, v.y, v.z, v.w};
        }
    } else {
        const __attribute__((address_space(1))) float *g =
            (const __attribute__((address_space(1))) float *)x;
        int64_t r = n - q0;
        asm volatile("" : "+v"(r));   // keep the element bounds in this branch
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int s = 0; s < 4; ++s) xb[b][s] = 16 * b + s < r ? g[q0 + 16 * b + s] : 0.0f;
    }
}

__device__ __forceinline__ void store_tile(const v4f (&yr)[4], float *y, int64_t n, int64_t t0,
                                           int lane)
{
    const int64_t q0 = t0 + 64 * (lane & 15) + 4 * (lane >> 4);
    if (t0 + TS <= n) {
        gf4u *p = (gf4u *)(y + q0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const f4u v = {yr[r].x, yr[r].y, yr[r].z, yr[r].w};
            __builtin_nontemporal_store(v, p + 4 * r);
        }
    } else {
        __attribute__((address_space(1))) float *g = (__attribute__((address_space(1))) float *)y;
        int64_t r = n - q0;
        asm volatile("" : "+v"(r));
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (16 * b + s < r) g[q0 + 16 * b + s] = yr[b][s];
    }
}

__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void rearm(unsigned *ctrl, unsigned epoch)
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

// y = T x + O s for one tile, given the scan P of its columns' end states
// from rest and the tile's incoming state st (LDS, 16 floats): the columns'
// incoming states are P shifted by one column plus A^c st.
__device__ __forceinline__ v4f column_states(v4f P, const float *st_lds, const float *acol,
                                             int n16, int g4)
{
    v4f st[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) st[k] = *reinterpret_cast<const v4f *>(st_lds + 4 * k);
    v4f Q;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float *ar = acol + n16 * kPowStride + (4 * g4 + j) * 16;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const v4f r = ld4(ar + 4 * k);
            acc += r.x * st[k].x + r.y * st[k].y + r.z * st[k].z + r.w * st[k].w;
        }
        Q[j] = acc;
    }
    return row_shr<1>(P) + Q;
}

// Row block r of matrix M (16 x 16, LDS, stride kPowStride) times the
// wave-uniform vector v (LDS, 16 floats), for lanes holding rows 4 g4 + j.
__device__ __forceinline__ v4f mat_rows(const float *Mx, const float *v_lds, int g4)
{
    v4f vv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) vv[k] = *reinterpret_cast<const v4f *>(v_lds + 4 * k);
    v4f out;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float *mr = Mx + (4 * g4 + j) * 16;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const v4f r = ld4(mr + 4 * k);
            acc += r.x * vv[k].x + r.y * vv[k].y + r.z * vv[k].z + r.w * vv[k].w;
        }
        out[j] = acc;
    }
    return out;
}

// One chunk of NG groups per ticket, in two sweeps with no barrier inside a
// sweep:
//   sweep 1: per group and tile, the columns' end states from rest (Gam x,
//     column scan); each tile's total is kept in LDS and each column scan in
//     registers for the whole chunk;
//   one barrier; then wave 0 alone: the tile scans of the chunk's groups,
//     the chunk's end state from rest (its aggregate), the lookback for its
//     incoming state, the inclusive state, and every tile's incoming state
//     (LDS), then a flag; meanwhile the other waves already start sweep 2;
//   sweep 2: per group, T x (it needs no state), then, once the flag is set,
//     the columns' incoming states, y += O s, store.
// The input is read twice, the output written once; the next group's samples
// are always in flight while the current one is processed, and wave 0's
// serial work overlaps the MFMA work of the wave sharing its SIMD.
template <int NG>
__global__ void __launch_bounds__(64 * WT) __attribute__((amdgpu_waves_per_eu(2)))
    sos_toep_kernel(ToepArgs a)
{
    if (ctab(a.tt)[TT_GATE] == 0.0f) return;   // the per-section kernels take the signal
    __shared__ float aggs[NG][NT][S];   // tile end states from rest, per group of the chunk
    __shared__ float stls[NG][NT][S];   // tile incoming states, per group of the chunk
    __shared__ float srun[S];           // wave 0: running state
    __shared__ float sgl[S];            // wave 0: lookback result
    __shared__ float chain[S];          // ragged end: state entering the last column
    __shared__ int64_t ticket;
    __shared__ int ready;               // chunks of this workgroup whose states are in stls
    // the power tables, read per lane at lane-dependent matrices: staged once
    __shared__ __attribute__((aligned(16))) float mats[kLdsMats * kPowStride];
    // per-lane MFMA operands (T, Gam, O, column and tile scans)
    __shared__ __attribute__((aligned(16))) float ops[5 * 1024];
    const float *acol = mats;
    const float *btile = mats + TC * kPowStride;
    const float *g1 = mats + (TC + NT) * kPowStride;
    const float *hpow = mats + (TC + NT + 1) * kPowStride;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n16 = lane & 15, g4 = lane >> 4;
    const unsigned epoch = __hip_atomic_load(&a.ctrl[CTRL_EPOCH], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    for (int e = threadIdx.x; e < kLdsMats * 64; e += 64 * WT) {
        const int mtx = e >> 6, q4 = e & 63;   // matrix, 128-bit piece
        *reinterpret_cast<v4f *>(mats + mtx * kPowStride + 4 * q4) =
            ld4(a.tt + TT_ACOL + mtx * 256 + 4 * q4);
    }
    for (int e = threadIdx.x; e < 5 * 256; e += 64 * WT)
        *reinterpret_cast<v4f *>(ops + 4 * e) = ld4(a.tt + TT_TOP + 4 * e);
    if (threadIdx.x == 0) ready = 0;
    // operand block o (TT_TOP order), entry i, of this lane
    auto opnd = [&](int o, int i) {
        return *reinterpret_cast<const v4f *>(ops + ((o * 4 + i) * 64 + lane) * 4);
    };
    const bool draw = (int64_t)gridDim.x < a.total;
    const bool ragged = (a.n % CG) != 0;
    auto tile0 = [&](int64_t grp, int tw) { return grp * CG + (int64_t)(wv * TPW + tw) * TS; };
    v4f xb[TPW][4];

    if (threadIdx.x == 0) ticket = (int64_t)atomicAdd(&a.ctrl[CTRL_TICKET], 1u);
    lds_sync();
    int64_t t = ticket;
    lds_sync();
    if (t < a.total) {
#pragma unroll
        for (int tw = 0; tw < TPW; ++tw) load_tile(xb[tw], a.x, a.n, tile0(t * NG, tw), lane);
    }
    int seq = 0;
    while (t < a.total) {
        const int64_t gfirst = t * NG;
        const int ng = (int)(a.groups - gfirst < NG ? a.groups - gfirst : NG);
        // ---- sweep 1: tile totals from rest; the columns' scans are kept
        // for the second sweep
        v4f Pk[NG][TPW];
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            if (j >= ng) break;
            v4f gop[4], aop[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                gop[i] = opnd(1, i);
                aop[i] = opnd(3, i);
            }
            v4f U[TPW];
#pragma unroll
            for (int tw = 0; tw < TPW; ++tw) {
                U[tw] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int s = 0; s < 4; ++s) U[tw] = mfma4(gop[b][s], xb[tw][b][s], U[tw]);
            }
            // next: the following group of this sweep, else the chunk's first
            // group again (sweep 2)
            const int64_t nxt = j + 1 < ng ? gfirst + j + 1 : gfirst;
#pragma unroll
            for (int tw = 0; tw < TPW; ++tw) load_tile(xb[tw], a.x, a.n, tile0(nxt, tw), lane);
#pragma unroll
            for (int tw = 0; tw < TPW; ++tw) {
                Pk[j][tw] = scan16(U[tw], aop);
                if (n16 == 15) *reinterpret_cast<v4f *>(&aggs[j][wv * TPW + tw][4 * g4]) = Pk[j][tw];
            }
        }
        lds_sync();
        // ---- wave 0: the chunk's states
        if (wv == 0) {
            v4f bop[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) bop[i] = opnd(4, i);
            v4f GP[NG];
#pragma unroll
            for (int j = 0; j < NG; ++j)
                if (j < ng) GP[j] = scan16(*reinterpret_cast<const v4f *>(&aggs[j][n16][4 * g4]), bop);
            // the chunk's end state from rest: s <- GP[:, 15] + G s over its groups
            if (lane < S) srun[lane] = 0.0f;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int j = 0; j < NG; ++j) {
                if (j < ng) {
                    const v4f gs = mat_rows(g1, srun, g4);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    if (n16 == 15) *reinterpret_cast<v4f *>(&srun[4 * g4]) = GP[j] + gs;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                }
            }
            unsigned long long *dsc = a.desc + (size_t)t * kDescWords;
            const bool full = ng == NG;
            if (t > 0 && full && lane < S) put_word(dsc + lane, pack_word(srun[lane], epoch));
            if (t == 0) {
                if (lane < S)
                    sgl[lane] = (a.zi && lane < 2 * a.K) ? a.zi[lane] * a.tt[TT_DINV + lane] : 0.0f;
            } else {
                toep_lookback(a, hpow, t, epoch, lane, sgl);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            // inclusive: aggregate + H s_in (a partial chunk is the last one:
            // nobody reads its descriptor)
            if (full) {
                const v4f hs = mat_rows(hpow + kPowStride, sgl, g4);
                if (n16 == 0) {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        put_word(dsc + 16 + 4 * g4 + j, pack_word(srun[4 * g4 + j] + hs[j], epoch));
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (lane < S) srun[lane] = sgl[lane];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            // every tile's incoming state: GP[:, t-1] + B^t s (lane column n16
            // = t), then s <- GP[:, 15] + G s
#pragma unroll
            for (int j = 0; j < NG; ++j) {
                if (j < ng) {
                    const v4f bs = mat_rows(btile + n16 * kPowStride, srun, g4);
                    *reinterpret_cast<v4f *>(&stls[j][n16][4 * g4]) = row_shr<1>(GP[j]) + bs;
                    const v4f gs = mat_rows(g1, srun, g4);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    if (n16 == 15) {
                        const v4f sn = GP[j] + gs;
                        *reinterpret_cast<v4f *>(&srun[4 * g4]) = sn;
                        if (gfirst + j == a.groups - 1 && !ragged && a.zf) {
#pragma unroll
                            for (int jj = 0; jj < 4; ++jj) {
                                const int m = 4 * g4 + jj;
                                if (m < 2 * a.K) a.zf[m] = sn[jj] * a.tt[TT_D + m];
                            }
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                }
            }
            if (lane == 0) {
                ticket = draw ? (int64_t)atomicAdd(&a.ctrl[CTRL_TICKET], 1u) : a.total;
                __hip_atomic_store(&ready, seq + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        // ---- sweep 2: outputs
        int64_t tn = a.total;
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            if (j >= ng) break;
            const int64_t grp = gfirst + j;
            v4f Y[TPW][4];
            {
                v4f top[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) top[i] = opnd(0, i);
#pragma unroll
                for (int tw = 0; tw < TPW; ++tw) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) Y[tw][r] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int b = 0; b <= r; ++b)
#pragma unroll
                            for (int s = 0; s < 4; ++s)
                                Y[tw][r] = mfma4(top[r - b][s], xb[tw][b][s], Y[tw][r]);
                }
                if (j == 0) {
                    // the chunk's states (and the next ticket) from wave 0
                    while (__hip_atomic_load(&ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <=
                           seq)
                        __builtin_amdgcn_s_sleep(1);
                    tn = ticket;
                }
                // next: the following group, else the next chunk's first group
                const int64_t nxt = j + 1 < ng ? grp + 1 : (tn < a.total ? tn * NG : -1);
                if (nxt >= 0) {
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw)
                        load_tile(xb[tw], a.x, a.n, tile0(nxt, tw), lane);
                }
            }
            const v4f (&P)[TPW] = Pk[j];
            v4f oop[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) oop[i] = opnd(2, i);
#pragma unroll
            for (int tw = 0; tw < TPW; ++tw) {
                const int ti = wv * TPW + tw;
                const v4f Sin = column_states(P[tw], stls[j][ti], acol, n16, g4);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int s = 0; s < 4; ++s) Y[tw][r] = mfma4(oop[r][s], Sin[s], Y[tw][r]);
                const int64_t t0 = grp * CG + (int64_t)ti * TS;
                // final state of a signal ending inside a column: the state
                // entering that column, advanced sample by sample over its valid
                // part (before the tile is stored: the input may be filtered in
                // place)
                if (ragged && a.zf && grp == a.groups - 1) {
                    const int64_t o = a.n - 1 - t0;
                    if (o >= 0 && o < TS) {
                        const int cs = (int)(o / M), rr = (int)(o % M) + 1;
                        if (n16 == cs) *reinterpret_cast<v4f *>(&chain[4 * g4]) = Sin;
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        const int m = lane & 15;
                        float phr[16];
#pragma unroll
                        for (int k = 0; k < 16; ++k) phr[k] = a.tt[TT_PHI + m * 16 + k];
                        const float gm = a.tt[TT_GAM + m];
                        float sv = chain[m];
                        const float *xc = a.x + t0 + (int64_t)cs * M;
                        for (int i = 0; i < rr; ++i) {
                            float nv = gm * xc[i];
#pragma unroll
                            for (int k = 0; k < 16; ++k)
                                nv += phr[k] * __int_as_float(__builtin_amdgcn_readlane(
                                                   __float_as_int(sv), k));
                            sv = nv;
                        }
                        if (lane < 2 * a.K) a.zf[lane] = sv * a.tt[TT_D + lane];
                    }
                }
                store_tile(Y[tw], a.y, a.n, t0, lane);
            }
        }
        ++seq;
        t = tn;
    }
    if (threadIdx.x == 0) rearm(a.ctrl, epoch);
}

}  // namespace

extern "C" {

int sos_toep_group_samples(void) { return CG; }   // samples per group (a chunk is ng groups)
int sos_toep_desc_words(void) { return kDescWords; }
int sos_toep_table_floats(void) { return TT_FLOATS; }

static bool chunk_ok(int ng) { return ng == 2 || ng == 4 || ng == kMaxNG; }

hipError_t sos_launch_toep_prep(const float *sections, int K, int ng, double rho_gate, float *tt,
                                hipStream_t stream)
{
    if (!chunk_ok(ng)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sos_toep_prep_kernel, dim3(1), dim3(256), 0, stream, sections, K, ng,
                       rho_gate, tt);
    return hipGetLastError();
}

int sos_toep_capacity(void)
{
    // LDS and registers allow one 8-wave workgroup per CU at every chunk size
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                     (const void *)sos_toep_kernel<kMaxNG>,
                                                     64 * WT, 0) != hipSuccess)
        per_cu = 1;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    return (per_cu > 0 ? per_cu : 1) * cus;
}

hipError_t sos_launch_toep(const float *x, float *y, int64_t n, const float *tt, int K, int ng,
                           const float *zi, float *zf, unsigned long long *desc, unsigned *ctrl,
                           unsigned long long timeout_ticks, int64_t grid, hipStream_t stream)
{
    if (!chunk_ok(ng)) return hipErrorInvalidValue;
    ToepArgs a{};
    a.x = x;
    a.y = y;
    a.n = n;
    a.tt = tt;
    a.zi = zi;
    a.zf = zf;
    a.K = K;
    a.groups = (n + CG - 1) / CG;
    a.total = (a.groups + ng - 1) / ng;
    a.desc = desc;
    a.ctrl = ctrl;
    a.timeout_ticks = timeout_ticks;
    if (grid <= 0 || grid > a.total) grid = a.total;
    const dim3 g((unsigned)grid), b(64 * WT);
    if (ng == 2)
        hipLaunchKernelGGL(sos_toep_kernel<2>, g, b, 0, stream, a);
    else if (ng == 4)
        hipLaunchKernelGGL(sos_toep_kernel<4>, g, b, 0, stream, a);
    else
        hipLaunchKernelGGL(sos_toep_kernel<kMaxNG>, g, b, 0, stream, a);
    return hipGetLastError();
}

}  // extern "C"
