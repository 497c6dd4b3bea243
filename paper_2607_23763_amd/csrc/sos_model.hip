// The cost model of the multi-block filter on a GPU (Sec. IV-C): the memory
// floor of Eq. (28), the latency-hiding floor of Eq. (29), the staging
// buffer of Eq. (26) and the residency of a (L, N) configuration against a
// device's per-SM budgets (Eq. (30) and Table II), and the prediction the
// autotuner ranks its candidate tiles by. Host code only.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sos_internal.h"

extern "C" {

int sos_model_floors(const sos_model_device *d, double ilp, sos_model_floors_t *out)
{
    if (!d || !out || !(ilp > 0.0) || !(d->bandwidth_gbs > 0.0)) return SOS_EINVAL;
    // Eq. (28): 8 bytes per sample (4 in, 4 out) against the DRAM bandwidth
    out->roof_gss = d->bandwidth_gbs / 8.0;
    // Eq. (29): instructions in flight needed, I lambda, over what one warp
    // keeps in flight
    out->w_min = (int)std::ceil(d->issue_rate * d->fma_latency / ilp - 1e-9);
    return SOS_OK;
}

int sos_model_config(const sos_model_device *d, int L, int N, int pad, int regs_per_thread,
                     double ilp, sos_model_config_t *out)
{
    if (!d || !out || L <= 0 || N <= 0 || pad < 0 || regs_per_thread < 0 || d->warp <= 0)
        return SOS_EINVAL;
    sos_model_floors_t f;
    int rc = sos_model_floors(d, ilp, &f);
    if (rc) return rc;
    sos_model_config_t c{};
    // Eq. (26): one FP32 staging row of N + pad words per lane
    c.s_buf = 4.0 * L * (double)(N + pad);
    const int warps_per_tb = (L + d->warp - 1) / d->warp;
    // each budget's bound on resident groups per SM; the smallest binds
    long lim[4];
    lim[0] = c.s_buf > 0.0 ? (long)std::floor(d->smem_per_sm / c.s_buf) : 1L << 30;
    lim[1] = d->max_tbs_per_sm;
    lim[2] = std::min<long>(d->max_threads_per_sm / L, d->max_warps_per_sm / warps_per_tb);
    lim[3] = 1L << 30;
    if (regs_per_thread > 0) {
        const int g = d->reg_granule > 0 ? d->reg_granule : 1;
        const long r = (long)((regs_per_thread + g - 1) / g) * g;
        if (d->regs_per_simd_lane > 0) {
            // register files per SIMD (AMD): waves per SIMD from the lane's
            // registers, the group's waves spread over the SIMDs
            const long waves = (long)(d->regs_per_simd_lane / r) * d->simds;
            lim[3] = waves / warps_per_tb;
        } else {
            lim[3] = (long)d->regs_per_sm / (r * (long)warps_per_tb * d->warp);
        }
    }
    int bind = 0;
    for (int i = 1; i < 4; ++i)
        if (lim[i] < lim[bind]) bind = i;
    c.tbs_per_sm = (int)std::max<long>(lim[bind], 0);
    c.warps_per_sm = c.tbs_per_sm * warps_per_tb;
    c.limit = bind + 1;   // SOS_MODEL_LIMIT_*
    c.feasible = c.s_buf <= d->smem_per_tb && c.tbs_per_sm >= 1;
    c.starved = c.warps_per_sm < f.w_min;
    *out = c;
    return SOS_OK;
}

int sos_model_device_gfx950(sos_model_device *out)
{
    if (!out) return SOS_EINVAL;
    sos_model_device d{};
    d.sms = 256;                       // compute units, 8 XCDs of 32
    d.smem_per_sm = 160.0 * 1024.0;    // LDS per CU
    d.smem_per_tb = 160.0 * 1024.0;    // a workgroup may take the whole LDS
    d.regs_per_sm = 4 * 512 * 64;      // 4 SIMDs x 512 VGPRs x 64 lanes
    d.regs_per_simd_lane = 512;
    d.simds = 4;
    d.reg_granule = 8;
    d.max_threads_per_sm = 2048;
    d.max_warps_per_sm = 32;           // 8 wave64 slots per SIMD
    d.max_tbs_per_sm = 32;
    d.warp = 64;
    // a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles, so the
    // CU issues one wave instruction per cycle over its 4 SIMDs; a dependent
    // FP32 FMA is ready 8 cycles after issue (4 issue cycles + pipeline)
    d.issue_rate = 1.0;
    d.fma_latency = 8.0;
    d.bandwidth_gbs = 8000.0;          // HBM3E
    d.clock_ghz = 2.4;
    d.fp32_tflops = 78.6;              // unpacked FP32 FMA rate
    *out = d;
    return SOS_OK;
}

}  // extern "C"

namespace sosint {

// Predicted time (ms) of one uneven-batch launch at tile (L, N) (Eq. (27)
// with the arithmetic term that MI355X brings back at high orders):
//   max(memory floor, arithmetic over the padded work) + F per round of
//   resident groups,
// where a round is one group on every resident slot (CUs x groups per CU),
// the padded work is sum_i ceil(n_i / C) C samples times the signal's
// sections, and F is the fixed per-group cost (ticket draw, carry exchange,
// staging synchronisations). `ops` is the solver's FMAs per sample and
// section. Returns a negative value for a configuration the budgets exclude
// or below the hiding floor.
double model_batch_ms(const sos_model_device &d, const ModelBatch &b, int L, int N, int pad,
                      int regs, double ops, double F_us)
{
    sos_model_config_t c;
    if (sos_model_config(&d, L, N, pad, regs, 3.0, &c) != SOS_OK || !c.feasible || c.starved)
        return -1.0;
    const int64_t C = (int64_t)L * N;
    double groups = 0.0, work = 0.0;
    for (size_t i = 0; i < b.len.size(); ++i) {
        const int64_t g = (b.len[i] + C - 1) / C;
        groups += (double)g;
        work += (double)(g * C) * b.K[i];
    }
    const double t_mem = 8.0 * (double)b.total / (d.bandwidth_gbs * 1e9);
    const double t_alu = work * ops * 2.0 / (d.fp32_tflops * 1e12);
    const double slots = (double)d.sms * c.tbs_per_sm;
    const double rounds = std::ceil(groups / slots);
    return 1e3 * (std::max(t_mem, t_alu) + rounds * F_us * 1e-6);
}

}  // namespace sosint
