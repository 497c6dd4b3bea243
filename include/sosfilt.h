/*
 * sosfilt.h -- C ABI of the MI355X (gfx950) cascaded-biquad filter library.
 *
 * The library filters FP32 signals through a cascade of K second-order
 * sections (biquads) with the multi-block method of Zhai & Paris, "Parallel
 * Cascaded Recursive Filtering on Multi-Core CPUs and GPUs" (Part II):
 *   - each group of C = N*L samples is viewed in the stride-N permuted
 *     (multi-block) form of Sec. II-B, Eqs. (2)-(5): lane l of a group holds
 *     the N consecutive samples [l*N, l*N + N);
 *   - every lane is solved at zero incoming state by one divide-and-conquer
 *     level followed by one-sided cyclic reduction per parity (Sec. II-D/E,
 *     Eqs. (14)-(23)), which exposes both terminal samples of the lane before
 *     any back substitution (or, selected per handle, by the PH
 *     factorization's particular solution, Sec. II-C; sos_set_algorithm);
 *   - the lanes' zero-state terminal states are combined by a cross-lane scan
 *     (the role of Eq. (13)), the group's incoming state arrives over a
 *     decoupled lookback between groups (Sec. IV-B, Eq. (25)), and the
 *     homogeneous correction is folded into the back substitution (Sec.
 *     II-F, Eq. (24); for PH it is added to every sample, Eq. (11)); all K
 *     sections run in registers inside one kernel launch per call (Sec. IV-A).
 *
 * Conventions shared by every entry point
 *   sections : K x 6 FP32 rows [b0 b1 b2 a0 a1 a2] (scipy "sos" layout),
 *              row-major, DEVICE memory. Each row is divided by its a0 in FP64
 *              on the device before use. b0 is kept in the feed-forward part,
 *              so b0 == 0 is allowed. Eq. (1) of the paper is the b0 = 1 case.
 *   zi, zf   : K x 2 FP32 transposed-direct-form-II states (z1, z2) per
 *              section, DEVICE memory: the scipy sosfilt convention. zi == NULL
 *              means zero initial state; zf == NULL means "do not write".
 *              zf is the state after the last real sample n-1.
 *   x, y     : n FP32 samples, DEVICE memory. y may equal x (in place);
 *              partial overlap is not allowed.
 *   stream   : the HIP stream all work is enqueued on; every call returns
 *              as soon as the work is enqueued. Buffers must stay valid until
 *              the stream has executed the work.
 *
 * Ownership: the caller owns every data buffer. The handle owns its workspace
 * (coefficient tables, lookback descriptors, ticket/epoch words); it grows on
 * the first call of a larger shape and is reused afterwards. Calls that share
 * one handle must be ordered (same stream, or synchronised): the workspace is
 * not shared safely between concurrently running calls. Use one handle per
 * concurrently used stream. A HIP graph that captures calls of a handle
 * holds pointers into its workspace: while such a graph may still be
 * replayed, make no call of a larger shape on that handle (it would replace
 * the workspace), or give the graph a handle of its own. A captured plain
 * filter carries its own re-arm step, so eager calls of any kind between
 * replays are otherwise fine.
 *
 * Errors: every function returns an int status and never aborts across the
 * ABI. Argument errors are detected synchronously. Problems found on the
 * device (a0 == 0, a section outside the stability triangle, a lookback that
 * did not resolve in time) make the affected outputs NaN and are reported by
 * sos_last_error().
 */
#ifndef SOSFILT_H
#define SOSFILT_H

#include <stdint.h>
#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SOS_OK = 0,
    SOS_EINVAL = -1,      /* bad argument (null pointer, negative size, K out of range ...) */
    SOS_EA0 = -2,         /* a section has a0 == 0                                          */
    SOS_EUNSTABLE = -3,   /* |a2| >= 1 or |a1| >= 1 + a2 after normalisation (a pole on or  */
                          /* outside the unit circle)                                       */
    SOS_ENOMEM = -4,      /* device allocation failed                                        */
    SOS_EHIP = -5,        /* a HIP runtime call failed                                       */
    SOS_ETIMEOUT = -6,    /* a lookback wait exceeded its bound (outputs poisoned with NaN)  */
    SOS_ECLOSED = -7,     /* object already destroyed / stream closed                        */
    SOS_EBUSY = -8,       /* resource temporarily exhausted                                  */
    SOS_ELIMIT = -9       /* beyond the fixed workspace of sos_filter_noalloc                */
};

#define SOS_MAX_SECTIONS 64

typedef struct sos_ctx *sos_handle_t;

/* Create a handle bound to HIP device `hip_device` (the device must be the
 * current device whenever the handle is used). Returns SOS_OK or an error. */
int sos_create(sos_handle_t *h, int hip_device);

/* Free the handle and its workspace. Synchronises the device first. */
int sos_destroy(sos_handle_t h);

/* Static text for a status code. */
const char *sos_strerror(int code);

/* Synchronises the handle's device, returns the first device-side error
 * (SOS_EA0, SOS_EUNSTABLE, SOS_ETIMEOUT) raised since the previous call of
 * sos_last_error on this handle, or SOS_OK, and clears it. */
int sos_last_error(sos_handle_t h);

/* The paper's two tuning parameters (Sec. IV-D): L lanes (threads) per group
 * and N samples per lane; a group holds C = L*N samples and one workgroup of
 * L/64 wavefronts processes it. Compiled shapes: L in {64, 256, 512} with
 * N in {16, 32, 64}, and L = 1024 with N in {16, 32}. sos_set_tile(h, 0, 0)
 * restores the default, (512, 64), which sos_get_tile reports (with no tile
 * set, sos_filter and sos_filter_train may pick a smaller shape for short
 * FP32 signals). Applies to later calls (tables prepared for another shape
 * must be prepared again). Unsupported shapes return SOS_EINVAL. */
int sos_set_tile(sos_handle_t h, int L, int N);
int sos_get_tile(sos_handle_t h, int *L, int *N);

/* Arithmetic type of the per-sample work of the filter kernels: 32 (FP32,
 * the default) or 64 (FP64; 0 restores the default). Data in memory stay FP32
 * either way. In FP32 each signal's tables take one of two layouts, chosen by
 * the preparation kernel from the peak gain 1 / min |A(e^{jw})| of its
 * sections (thresholds under sos_set_algorithm): the fast layout (everything
 * in FP32) or the accurate one, where everything that acts on carried states
 * (the lanes' and groups' terminal states, the scans over lanes, waves and
 * groups through powers of the state map, the lanes' incoming states and zf)
 * runs in FP64 and the homogeneous correction uses an orthonormal basis of
 * the lane's free responses: with poles near the unit circle those powers
 * are badly conditioned and FP32 rounding of them would be amplified into
 * every sample of a group. With FP32, a cascade is about as accurate as a
 * sequential FP32 filter; FP64 goes further where a cascade's own FP32 error
 * floor is too high. MI355X issues FP64 FMAs at the unpacked-FP32 rate, so
 * the cost of FP64 is register pressure. Applies to later calls. */
int sos_set_precision(sos_handle_t h, int bits);
int sos_get_precision(sos_handle_t h);

/* Section solver of the filter kernels (Sec. IV-E compares the candidates):
 *   SOS_ALG_DCCR  divide-and-conquer cyclic reduction (Sec. II-E): both
 *                 terminal blocks of every lane from a log-depth reduction of
 *                 each parity chain, then back substitution; about 9 FMAs per
 *                 sample and section.
 *   SOS_ALG_PH    PH factorization (Sec. II-C): the lane's particular
 *                 solution (its samples through the section from rest,
 *                 Eq. (9)), then the homogeneous correction of every sample
 *                 from the lane's incoming state (Eq. (11)); about 7 FMAs per
 *                 sample and section and a lane-sequential chain of N FMAs.
 *   SOS_ALG_AUTO  per signal, in FP32: DC-CR on the fast layout when every
 *                 section's recursive part has a peak gain 1 / min
 *                 |A(e^{jw})| of at most 32, else PH on the accurate layout
 *                 (see sos_set_precision), in the same launch. DC-CR's fold
 *                 multiplies by A(-z), which amplifies rounding near the
 *                 mirror frequency of poles close to the unit circle; PH
 *                 applies no such factor. Butterworth designs up to order 16
 *                 at cutoff 0.2*pi peak at 15.7 and stay on DC-CR. In FP64:
 *                 DC-CR.
 * In FP32, SOS_ALG_PH takes the accurate layout for signals with a section
 * of peak gain above 128 (its fast layout stays within about 3x of a
 * sequential FP32 filter's error up to there); SOS_ALG_DCCR always takes the
 * fast layout. SOS_ACCURATE_GAIN in the environment (a positive number, or
 * "inf" for never) replaces the thresholds of SOS_ALG_AUTO and SOS_ALG_PH.
 * All share the cross-lane scan, the decoupled lookback, the tables and the
 * state conventions, and accept every tile and compute type. SOS_ALG_DEFAULT
 * (0) restores the default: SOS_ALG in the environment ("auto", "dccr",
 * "ph" or "toeplitz"), else SOS_ALG_AUTO. Applies to later launches of the handle: plain,
 * batched, captured batches, servers created afterwards, and both passes of
 * the adjoint (the training forward and the reversed-time recursion of the
 * VJP). Tables prepared by sos_prepare belong to the solver in effect then.
 * sos_set_algorithm returns SOS_EINVAL for an unknown value or a null
 * handle; sos_get_algorithm returns the solver in effect (SOS_ALG_AUTO,
 * SOS_ALG_DCCR, SOS_ALG_PH or SOS_ALG_TOEPLITZ), or SOS_EINVAL for a null
 * handle.
 *
 * Whole-cascade block-Toeplitz form (Sec. II-B taken over the whole cascade):
 * for a plain FP32 forward filter (sos_filter, sos_filter_prepared) of a
 * cascade of at most 8 sections, the cascade's 2K TDF-II states are stacked
 * into one state, and every 64-sample column is filtered as y = T x + O s,
 * s' = A s + Gam x with T the lower-triangular Toeplitz matrix of the
 * cascade's impulse response, on the matrix cores (FP32 MFMA), with one
 * 16-word lookback per chunk (8 groups of 16384 samples from 2^25 samples
 * on, 2 groups below; SOS_TOEP_CHUNK = 2, 4 or 8 in the environment
 * overrides) instead of one per group and section.
 * Its cost per sample does not grow with K, but a call takes at least about
 * 0.07 ms (its tables, and chunks that must fill the device).
 * SOS_ALG_AUTO takes it for plain FP32 forward calls with K = 7 or 8 on at
 * least 2^25 samples, or K = 6 on at least 2^26, when
 * every section's peak gain is at most 128 (decided on the device by the
 * table preparation; other signals run as before, in the same call). Tables
 * from sos_prepare, whose signal length is not known, use 8-group chunks.
 * SOS_ALG_TOEPLITZ takes it for every plain FP32 forward call with K <= 8,
 * whatever the gains; its batched, training, adjoint and served launches,
 * and FP64 ones, run PH. Results follow the same conventions (zi, zf, in
 * place); the error is about that of a sequential FP32 filter. */
enum {
    SOS_ALG_DEFAULT = 0,
    SOS_ALG_DCCR = 1,
    SOS_ALG_PH = 2,
    SOS_ALG_AUTO = 3,
    SOS_ALG_TOEPLITZ = 4
};
int sos_set_algorithm(sos_handle_t h, int alg);
int sos_get_algorithm(sos_handle_t h);

/* Bound on each lookback wait (Sec. IV-B's decoupled lookback spins on its
 * predecessors' descriptors): `ms` milliseconds of the device wall clock
 * (0 restores the default, 2000 ms, or SOS_TIMEOUT_MS at sos_create). A wait
 * that exceeds it poisons the group's outputs with NaN, still publishes so
 * successors terminate, and makes sos_last_error report SOS_ETIMEOUT.
 * Returns SOS_EINVAL for a negative or non-finite value or more than one hour. */
int sos_set_timeout(sos_handle_t h, double ms);
/* The device wall-clock rate in kHz the timeout is converted with. */
int sos_wall_clock_khz(sos_handle_t h);

/*
 * Plain filter, one signal (Sec. IV-A/B; Eqs. (1)-(25)).
 *   y[0..n) = cascade(sections[0..K))(x[0..n)) starting from zi; zf receives
 *   the final states. 0 <= K <= SOS_MAX_SECTIONS, n >= 0.
 *   n == 0: y is not touched and zf := zi (zeros if zi == NULL).
 *   K == 0: y := x.
 * Enqueues: the coefficient-preparation kernel (FP64 tables) and the filter
 * kernel (ticketed groups, register-resident cascade, decoupled lookback),
 * whose last workgroup to finish re-arms the ticket counter and the
 * descriptor epoch for the next launch on the handle. In FP32 with no tile set (sos_set_tile, SOS_TILE_L/N), the group
 * shape follows n: (512, 16) up to 2^20 samples, (512, 32) up to 2^22, else
 * the default (512, 64); shorter signals leave the device partly idle, and
 * fewer samples per lane shorten each group's chain. sos_filter_train does
 * the same.
 */
int sos_filter(sos_handle_t h, const float *sections, int K, const float *x, float *y,
               int64_t n, const float *zi, float *zf, hipStream_t stream);

/*
 * Uneven batch in one persistent launch (Sec. IV-A/B applied per signal).
 * B independent signals; signal i is x[sig_off[i] .. sig_off[i+1]) -> y at the
 * same offsets, filtered by K[i] sections whose rows start at row sec_off[i]
 * of `sections` (so rows sec_off[i] .. sec_off[i]+K[i]-1), with TDF-II states
 * zi/zf at 2*sec_off[i] .. 2*(sec_off[i]+K[i]) - 1. Rows of different signals
 * need not be contiguous or ordered (a server can keep one row table for all
 * its streams), but two signals must not share zf rows.
 *   K, sec_off (B entries), sig_off (B+1 entries) are DEVICE int arrays;
 *   sections, x, y, zi, zf are DEVICE float arrays (zi/zf nullable).
 *   kmax (host) bounds every K[i] (0 <= kmax <= SOS_MAX_SECTIONS);
 *   total_rows (host) = rows in `sections` (and pairs in zi/zf);
 *   total_samples (host) = the size of x and y (sig_off[B] <= total_samples).
 *   zi may equal zf (state updated in place).
 * The work table (groups per signal, ticket -> signal) is built on the device,
 * so a sequence of calls with changing device-side contents can be captured
 * in a HIP graph. Groups of all signals are drawn as tickets by a grid sized
 * to the device's resident capacity. A signal whose entries are inconsistent
 * (K[i] outside [0, kmax], offsets out of range or decreasing) is skipped and
 * reported by sos_last_error() as SOS_EINVAL; sections that are invalid
 * (a0 == 0, unstable) poison only their own signal. Signals with no samples
 * get zf = zi. Calls on one handle must be ordered, as for sos_filter.
 */
int sos_filter_batched(sos_handle_t h, int B, int kmax, int64_t total_rows,
                       int64_t total_samples, const int32_t *K, const int32_t *sec_off,
                       const float *sections, const int64_t *sig_off, const float *x, float *y,
                       const float *zi, float *zf, hipStream_t stream);

/* Two-step form of sos_filter for repeated calls with the same coefficients
 * (Sec. II-D: every table depends only on the filter and is precomputed).
 * sos_prepare enqueues the coefficient-preparation kernel for `sections`
 * (K x 6, device) at the handle's current tile; sos_filter_prepared then
 * enqueues only the filter kernel, with the same conventions as sos_filter.
 * sos_filter_prepared returns SOS_EINVAL if nothing was prepared, the
 * precision changed since, or a tile set on the handle differs from the one
 * prepared at (with no tile set, the shape the tables were prepared at is
 * used, including one that sos_filter picked from the signal length). The sections buffer is read by the preparation kernel only. */
int sos_prepare(sos_handle_t h, const float *sections, int K, hipStream_t stream);
int sos_filter_prepared(sos_handle_t h, const float *x, float *y, int64_t n, const float *zi,
                        float *zf, hipStream_t stream);

/*
 * Differentiable form. sos_filter_train is sos_filter that also writes the
 * outputs of sections 0..K-2 to `saved` ((K-1) x n floats, device; unused
 * when K <= 1); x and y must be distinct buffers.
 *
 * sos_filter_vjp: vector-Jacobian product of that forward call. Given the
 * upstream gradients gy (n) and gzf (K x 2, nullable = zeros) it writes
 *   gx        (n)      d<gy,y>+<gzf,zf> / dx        (may alias gy)
 *   gzi       (K x 2)  ... / dzi                   (nullable)
 *   gsections (K x 6)  ... / d[b0 b1 b2 a0 a1 a2]  (nullable; raw rows,
 *                      through the division by a0)
 * from x, y and saved of the forward call (zi is not needed). Per section, last
 * to first: the recursive part 1/A(z) runs in reversed time with the same
 * multi-block machinery (carries = last two outputs), a 3-tap FIR of its
 * output gives the gradient of the section input, and per-group correlations
 * of that output with the section's input and output give the coefficient
 * gradients, reduced over groups in FP64 in a fixed order. The paper does not
 * treat gradients; this is the adjoint of its Eq. (1) cascade. The adjoint
 * uses the handle's tile when it is one of its shapes (L in {64, 256, 512},
 * N in {16, 32}), else (512, 32).
 */
int sos_filter_train(sos_handle_t h, const float *sections, int K, const float *x, float *y,
                     int64_t n, const float *zi, float *zf, float *saved, hipStream_t stream);
int sos_filter_vjp(sos_handle_t h, const float *sections, int K, const float *x, const float *y,
                   const float *saved, int64_t n, const float *gy, const float *gzf, float *gx,
                   float *gzi, float *gsections, hipStream_t stream);

/* Batched training pair: sos_filter_batched's arguments (same layouts and
 * rules) plus, for the forward, `saved`: DEVICE (kmax-1) x total_samples
 * floats receiving the outputs of sections 0..K[i]-2 of signal i at
 * saved + s * total_samples + sig_off[i] (NULL allowed when kmax <= 1;
 * x != y). The adjoint takes the same batch description, the forward's x, y
 * and saved, the cotangents gy (like y) and gzf (like zf, nullable), and
 * writes gx (like x), gzi (like zi, nullable) and gsections (like sections,
 * nullable: the rows of the batch's signals). Empty signals get gzi = gzf and
 * zero coefficient gradients. One persistent launch of the adjoint over the
 * reversed groups of every signal, then a per-(signal, section) FP64
 * reduction of the coefficient partials. */
int sos_filter_train_batched(sos_handle_t h, int B, int kmax, int64_t total_rows,
                             int64_t total_samples, const int32_t *K, const int32_t *sec_off,
                             const float *sections, const int64_t *sig_off, const float *x,
                             float *y, const float *zi, float *zf, float *saved,
                             hipStream_t stream);
int sos_filter_vjp_batched(sos_handle_t h, int B, int kmax, int64_t total_rows,
                           int64_t total_samples, const int32_t *K, const int32_t *sec_off,
                           const float *sections, const int64_t *sig_off, const float *x,
                           const float *y, const float *saved, const float *gy,
                           const float *gzf, float *gx, float *gzi, float *gsections,
                           hipStream_t stream);

/* The batched adjoint for a batch whose signals share one cascade (the rows
 * of every signal hold the same sections, as when one filter is trained on a
 * batch): sos_filter_vjp_batched's arguments, with gsections replaced by
 * `gsum`, DEVICE kmax x 6 floats (required): row k receives the sum over the
 * signals i with K[i] > k of the gradient of signal i's row k. Each signal's
 * gradient is formed in FP64, the sum over signals runs in FP64 in a fixed
 * order and is rounded once. With B = 0 nothing is written. For callers
 * that differentiate a shared filter; the paper does not treat gradients. */
int sos_filter_vjp_batched_sum(sos_handle_t h, int B, int kmax, int64_t total_rows,
                               int64_t total_samples, const int32_t *K, const int32_t *sec_off,
                               const float *sections, const int64_t *sig_off, const float *x,
                               const float *y, const float *saved, const float *gy,
                               const float *gzf, float *gx, float *gzi, float *gsum,
                               hipStream_t stream);

/* Memory-floor reference (the t_mem = b_s / BW term of the cost model,
 * Eq. (28), with b_s = 8 bytes per sample): a plain streaming copy y = x of n
 * FP32 samples with the same 128-bit nontemporal accesses as the filter.
 * Device pointers; x and y must not overlap. Used to measure the achievable
 * copy bandwidth and to calibrate hardware byte counters. */
int sos_bench_copy(const float *x, float *y, int64_t n, hipStream_t stream);

/* Debug/inspection: after a completed sos_filter call on this handle, copy the
 * resolved state at the end of every (group, section) -- the "global carry" of
 * Sec. II-F that the decoupled lookback publishes, as a TDF-II pair -- to host
 * memory `out` (groups x K x 2 floats, group-major) and return the number of
 * groups and sections through *groups and *K. For a full group g this is the
 * state after sample (g+1)*C - 1; for a zero-padded last group it is the state
 * after the padding. out may be NULL to query the sizes; capacity_floats is
 * the size of out. Synchronises the device. Returns SOS_EINVAL if out is too
 * small or no call was made. */
int sos_debug_carries(sos_handle_t h, float *out, int64_t capacity_floats, int64_t *groups,
                      int *K);

/* ------------------------------------------------------- graph and tuning
 * An uneven batch (sos_filter_batched's arguments) captured once into a HIP
 * graph: coefficient preparation, the device-built work table, the arm step
 * and the persistent filter launch, with no memset nodes. Creation allocates
 * a private workspace (the graph pins it) at the tile, compute type and
 * lookback bound of `h`, and captures on a private stream. A launch replays
 * the same four kernels on `stream` with the same pointers: the contents of
 * every input array (samples, sections, K, sec_off, sig_off, zi) may change
 * between launches as long as B, kmax, total_rows and total_samples stay the
 * bounds they were at creation (the work table is rebuilt on the device each
 * launch). Device errors of the last finished launch: sos_graph_last_error. */
typedef struct sos_graph *sos_graph_t;
int sos_graph_create_batched(sos_graph_t *g, sos_handle_t h, int B, int kmax,
                             int64_t total_rows, int64_t total_samples, const int32_t *K,
                             const int32_t *sec_off, const float *sections,
                             const int64_t *sig_off, const float *x, float *y, const float *zi,
                             float *zf);
int sos_graph_launch(sos_graph_t g, hipStream_t stream);
int sos_graph_last_error(sos_graph_t g);
int sos_graph_destroy(sos_graph_t g);

/* The cost model of Sec. IV-C, on a device described by its per-SM (per-CU)
 * budgets. Host arithmetic only: no device is touched, so these run anywhere.
 *   sos_model_floors: Eq. (28)'s throughput roof BW / 8 bytes per sample
 *     (GS/s) and Eq. (29)'s hiding floor W_min = ceil(I lambda / ILP) (warps
 *     per SM; the paper's ILP is 3).
 *   sos_model_config: a tile of L lanes x N samples per lane: Eq. (26)'s
 *     staging buffer 4 L (N + pad) bytes (pad: the row padding in words; the
 *     paper's kernels pad by 1, these by 4 for 128-bit rows), the resident
 *     groups per SM under every budget (shared memory / LDS, group slots,
 *     threads and warps, registers at `regs_per_thread`, 0 = not counted),
 *     the warps that makes (Eq. (30)), which budget binds
 *     (SOS_MODEL_LIMIT_*), whether the buffer fits one group's cap and at
 *     least one group is resident (feasible), and whether the warps fall
 *     below W_min (starved).
 *   sos_model_device_gfx950: MI355X's budgets (256 CUs, 160 KiB LDS per CU
 *     and per workgroup, 4 SIMDs of 512 VGPRs per lane, 32 wave64 slots,
 *     one wave instruction per cycle per CU with an 8-cycle dependent FMA,
 *     8 TB/s, 2.4 GHz, 78.6 TFLOP/s unpacked FP32).
 * All return SOS_EINVAL for null pointers or non-positive sizes. */
typedef struct {
    int sms;                    /* SMs / CUs */
    double smem_per_sm;         /* bytes of shared memory (LDS) per SM */
    double smem_per_tb;         /* bytes one thread block (workgroup) may take */
    int regs_per_sm;            /* 32-bit registers per SM */
    int regs_per_simd_lane;     /* AMD: registers per lane of one SIMD (0: NVIDIA-style pool) */
    int simds;                  /* AMD: SIMDs per CU */
    int reg_granule;            /* per-thread register allocation granule */
    int max_threads_per_sm;
    int max_warps_per_sm;
    int max_tbs_per_sm;
    int warp;                   /* threads per warp / wavefront */
    double issue_rate;          /* I: warp instructions issued per cycle per SM */
    double fma_latency;         /* lambda: cycles of a dependent FMA */
    double bandwidth_gbs;       /* DRAM bandwidth, GB/s */
    double clock_ghz;
    double fp32_tflops;         /* FP32 FMA rate the kernels can use */
} sos_model_device;
typedef struct {
    double roof_gss;            /* GS/s at 8 bytes per sample */
    int w_min;                  /* warps per SM */
} sos_model_floors_t;
enum { SOS_MODEL_LIMIT_SMEM = 1, SOS_MODEL_LIMIT_TBS = 2, SOS_MODEL_LIMIT_THREADS = 3,
       SOS_MODEL_LIMIT_REGS = 4 };
typedef struct {
    double s_buf;               /* bytes of staging per group */
    int tbs_per_sm;             /* resident groups per SM */
    int warps_per_sm;
    int limit;                  /* SOS_MODEL_LIMIT_* that binds */
    int feasible;
    int starved;
} sos_model_config_t;
int sos_model_floors(const sos_model_device *d, double ilp, sos_model_floors_t *out);
int sos_model_config(const sos_model_device *d, int L, int N, int pad, int regs_per_thread,
                     double ilp, sos_model_config_t *out);
int sos_model_device_gfx950(sos_model_device *out);
/* The compiled forward kernels: whether a tile (L lanes, N samples per lane)
 * is compiled in (1) or not (0); a tile's kernel's vector registers per lane
 * and static LDS bytes as its code object records them (SOS_EINVAL for a
 * tile not compiled in, SOS_EHIP if the runtime cannot say); and the
 * workgroups of that shape resident on the whole device at once (the
 * runtime's occupancy count times the CUs; 0 for a tile not compiled in).
 * bits: 32 or 64; alg: the solver kernel (0 DC-CR, 1 PH; +4 for the kernel
 * that picks the table layout per group). */
int sos_fwd_shape_supported(int L, int N);
int sos_fwd_kernel_attrs(int bits, int alg, int L, int N, int *regs, int *lds);
int sos_fwd_capacity(int bits, int alg, int L, int N);

/* Autotuner for the two parameters of the multi-block layout (Sec. IV-A/C):
 * lanes per group L and samples per lane N (group size C = N L). Runs the
 * batch on its own buffers. Each compiled (L, N) shape and candidate solver
 * is first priced by the cost model on this device's budgets (the kernel's
 * own register count, the staging buffer, residency): shapes the budgets
 * exclude or that fall below the hiding floor are dropped, as are shapes
 * whose padded work (a signal of n samples costs ceil(n / C) groups of C)
 * exceeds 1.5x the best shape's. The rest are ranked by the model's
 * predicted time: the larger of the memory floor (8 bytes per sample at the
 * HBM bandwidth) and the FMAs of the padded work at the FP32 rate, plus a
 * fixed 1.5 us per round of resident groups (the per-group overhead F of
 * Eq. (27), measured on MI355X as the 2^28-sample filter's excess over the
 * copy kernel spread over its rounds). Only the 6 best-ranked (shape,
 * solver) pairs are timed (one warm-up, `reps` timed runs, median, HIP events
 * on `stream`); SOS_TUNE_EXHAUSTIVE=1 in the environment times every pair
 * the budgets admit (for checking the ranking). When h has no section
 * solver set (SOS_ALG_DEFAULT), the pairs span SOS_ALG_AUTO and SOS_ALG_PH
 * and the winning solver becomes h's too; otherwise only h's solver is
 * priced. The fastest tile
 * becomes h's tile and is cached per (compute type, requested solver, kmax,
 * B, floor(log2 total_samples)) for sos_tune_lookup (a default request is
 * also cached under the winning solver); y and zf end up holding the
 * winner's result. The batch runs several times, so it cannot be filtered in
 * place: x == y (with samples) and zi == zf return SOS_EINVAL. Synchronises
 * `stream`. */
int sos_tune_batched(sos_handle_t h, int B, int kmax, int64_t total_rows, int64_t total_samples,
                     const int32_t *K, const int32_t *sec_off, const float *sections,
                     const int64_t *sig_off, const float *x, float *y, const float *zi,
                     float *zf, hipStream_t stream, int reps, int *L, int *N, float *ms);
/* A cached tuning result for the key above, or SOS_EINVAL if none. */
int sos_tune_lookup(sos_handle_t h, int B, int kmax, int64_t total_samples, int *L, int *N);

/* Plain filter that allocates nothing: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation). Same arguments, conventions and result as
 * sos_filter on a default handle (FP32 compute, the automatic solver choice,
 * the group shape chosen from n), without a handle: its workspace (control
 * words, coefficient tables, lookback descriptors) is a fixed device array of
 * about 16.6 MiB in the library, one per device, kept until the process ends.
 * No hipMalloc, hipFree or allocating library routine is called.
 * Limits: K <= SOS_MAX_SECTIONS, and ceil(n / C) * K <= 2^19 group-sections
 * (C = 8192 samples per group up to 2^20 samples, 16384 up to 2^22, else
 * 32768: for example n = 2^28 with K up to 64 would need 2^19 at K = 64);
 * beyond them it returns SOS_ELIMIT and enqueues nothing.
 * err (nullable, DEVICE, one unsigned): receives the call's device-side error
 * bits in stream order (0 = none; 1 a0 == 0, 2 unstable section, 4 lookback
 * timeout), as sos_last_error reports them for a handle.
 * All calls on one device share the array, which keeps the last call's
 * contents: calls that overlap on one device (other streams, other host
 * threads) race and must be serialised by the caller. Stream-ordered on
 * `stream`; SOS_EINVAL / SOS_EHIP as sos_filter. */
int sos_filter_noalloc(const float *sections, int K, const float *x, float *y, int64_t n,
                       const float *zi, float *zf, unsigned *err, hipStream_t stream);

/* ------------------------------------------------------------------ serving
 * Many long signals ("streams") that arrive in chunks, each filtered by its
 * own cascade as one continuous signal (the problem of Sec. II per stream;
 * chunked filtering with carried state is exact by the superposition of
 * Sec. II-F: a chunk's output is its zero-state response plus the response to
 * the state the previous chunk left). A server keeps every open stream's
 * sections, their prepared tables and its K TDF-II states in device memory
 * between chunks, and batches pending chunks continuously: one scheduler
 * thread forms steps of at most one chunk per stream (oldest first), each
 * step one persistent launch of the uneven-batch path. Streams are dealt to
 * two lanes, each with its own HIP stream and workspace and at most two
 * steps in flight: a stream's chunks run in its lane's stream order (FIFO),
 * the lanes' steps over disjoint streams overlap on the device, and chunks
 * that arrive during a step join their lane's next one.
 *
 * Chunk and output buffers are DEVICE pointers owned by the caller, who keeps
 * them alive until sos_stream_wait returns for that chunk; out may equal
 * chunk. Operations on one server may come from any host thread. */
typedef struct sos_srv *sos_server_t;

/* Create a server on the device of `h`, with h's tile (L, N), compute type
 * and lookback bound (h itself is not used afterwards; the server has its own
 * workspaces). device_mem_budget bytes (0 = 256 MiB) are split between
 * stream rows (sections, states and tables: K rows per stream) and, in equal
 * parts, the two lanes' work tables and descriptors, which bound the samples
 * of a step and of a chunk (sos_server_limits). max_slots (>= 1) bounds the chunks of one step.
 * When h's tile has fewer than 16384 samples per group, every stream's
 * tables are also prepared for the throughput tile (512, 32), and steps of
 * at least 2^22 samples (a loaded server's) run at that tile.
 * Allocates everything up front; no device allocation happens while serving. */
int sos_server_create(sos_server_t *s, sos_handle_t h, size_t device_mem_budget, int max_slots);
/* Stop the scheduler, let steps on the device finish, fail chunks not yet in
 * a step with SOS_ECLOSED, free everything. */
int sos_server_destroy(sos_server_t s);
/* Capacity: stream rows in total, largest chunk (samples), and the tile. */
int sos_server_limits(sos_server_t s, int64_t *max_rows, int64_t *max_chunk, int *L, int *N);

/* Open a stream with K sections (HOST array K x 6, same layout and
 * normalisation as sos_filter) and initial TDF-II states zi (HOST K x 2, NULL
 * = zeros). Synchronous: copies and prepares the tables and checks them;
 * returns SOS_EA0 / SOS_EUNSTABLE for unusable sections, SOS_EBUSY when the
 * stream rows are used up. *stream_id receives the stream's id. */
int sos_stream_open(sos_server_t s, const float *sections_host, int K, const float *zi_host,
                    int64_t *stream_id);
/* Enqueue the next chunk of a stream: n samples at `chunk`, output to `out`.
 * Returns at once with a ticket for sos_stream_wait. SOS_EINVAL for n < 0 or
 * n above the largest chunk, SOS_ECLOSED for an unknown or closing stream,
 * and the stream's failure status for a failed stream (below). */
int sos_stream_push(sos_server_t s, int64_t stream_id, const float *chunk, int64_t n, float *out,
                    uint64_t *ticket);
/* The same for `count` chunks at once (one lock; arrays of count entries). */
int sos_stream_push_many(sos_server_t s, int count, const int64_t *stream_ids,
                         const float *const *chunks, const int64_t *n, float *const *outs,
                         uint64_t *tickets);
/* Block until the chunk is filtered; returns its own status and, if
 * latency_s is not NULL, the time in seconds from its push to the host's
 * observation that its step completed. A ticket can be waited on once.
 * Statuses are per chunk: SOS_ETIMEOUT when a lookback wait of this chunk's
 * groups ran out (its outputs from there on are NaN), SOS_EINVAL when its
 * step's work table rejected it, SOS_EHIP when its step could not be
 * launched, SOS_ECLOSED when the server was destroyed first. The other
 * chunks of the same step are not affected. A failed chunk leaves its
 * stream's device state invalid (the state is updated in place), so the
 * stream fails from then on: its chunks that finish later report the same
 * status, later pushes return it at once, and sos_stream_state returns it
 * instead of a state. Close the stream and open it again (from a
 * checkpoint) to continue. */
int sos_stream_wait(sos_server_t s, uint64_t ticket, double *latency_s);
/* After all chunks pushed so far on the stream are finished, copy its K x 2
 * TDF-II state to HOST memory zf_host (a checkpoint: reopening a stream with
 * these states continues it exactly). Returns a failed stream's status
 * without copying. */
int sos_stream_state(sos_server_t s, int64_t stream_id, float *zf_host);
/* Wait for the stream's outstanding chunks, then release its rows. */
int sos_stream_close(sos_server_t s, int64_t stream_id);
/* Load driver for measurement: push chunk r (n = lens[r] samples at
 * x + offs[r], output at y + offs[r], DEVICE memory) of stream stream_ids[r]
 * at arrival_s[r] seconds after the call (arrival times ascending), from
 * the calling thread, then wait for all; latency_s[r] (nullable) receives each
 * chunk's latency and *wall_s the time from the start to the last completion.
 * Returns the first failing status. */
int sos_server_replay(sos_server_t s, int64_t R, const int64_t *stream_ids, const int64_t *offs,
                      const int64_t *lens, const double *arrival_s, const float *x, float *y,
                      double *latency_s, double *wall_s);

#ifdef __cplusplus
}
#endif

#endif /* SOSFILT_H */
