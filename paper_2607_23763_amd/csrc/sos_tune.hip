// Uneven batches as a replayable HIP graph, and an autotuner for the two
// tuning parameters of the multi-block filter: lanes per group L (group size
// C = N L) and samples per lane N (Sec. IV-A/C).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "sos_internal.h"

using namespace sosdev;
using namespace sosint;

struct sos_graph {
    sos_ctx *h = nullptr;          // private workspace, pinned by the graph
    hipStream_t cs = nullptr;      // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

namespace {

// Tuner cache: (compute type and requested section solver, kmax, batch size,
// log2 of total samples) -> tile.
using TuneKey = std::tuple<int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, Tile> g_tune_cache;

TuneKey key_of(const sos_ctx *h, const BatchArgs &ba)
{
    int lg = 0;
    while (lg < 62 && ((int64_t)1 << (lg + 1)) <= ba.total_samples) ++lg;
    return TuneKey{bits_of(h) * 4 + h->alg, ba.kmax, ba.B, lg};   // the solver as requested
}

void destroy_graph(sos_graph *g)
{
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cs) (void)hipStreamDestroy(g->cs);
    if (g->h) (void)sos_destroy(g->h);
    delete g;
}

// Candidate tiles: every compiled forward shape, minus FP64 shapes whose
// registers spill (N = 64 holds 128 registers of samples per lane).
std::vector<Tile> candidates(int bits)
{
    std::vector<Tile> c;
    for (int L : {64, 256, 512, 1024})
        for (int N : {16, 32, 64}) {
            if (!sos_fwd_shape_supported(L, N)) continue;
            if (bits == 64 && N == 64) continue;
            c.push_back(Tile{L, N});
        }
    return c;
}

}  // namespace

extern "C" {

int sos_graph_create_batched(sos_graph_t *out, sos_handle_t hu, int B, int kmax,
                             int64_t total_rows, int64_t total_samples, const int32_t *K,
                             const int32_t *sec_off, const float *sections,
                             const int64_t *sig_off, const float *x, float *y, const float *zi,
                             float *zf)
{
    if (!out || !hu) return SOS_EINVAL;
    *out = nullptr;
    BatchArgs ba{B, kmax, total_rows, total_samples, K, sec_off, sections, sig_off, x, y, zi, zf};
    int rc = batch_check(ba);
    if (rc) return rc;
    if (B == 0) return SOS_EINVAL;
    sos_graph *g = new (std::nothrow) sos_graph();
    if (!g) return SOS_ENOMEM;
    g->device = hu->device;
    DeviceGuard dg(g->device);
    if (!dg.ok) {
        delete g;
        return SOS_EHIP;
    }
    rc = sos_create(&g->h, g->device);
    if (rc) {
        delete g;
        return rc;
    }
    const Tile t = tile_of(hu, kmax);
    const int bits = bits_of(hu);
    g->h->tile_L = t.L;
    g->h->tile_N = t.N;
    g->h->bits = bits;
    g->h->alg = hu->alg;
    g->h->timeout_ticks = hu->timeout_ticks;
    if (hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking) != hipSuccess) {
        destroy_graph(g);
        return SOS_EHIP;
    }
    rc = batch_reserve(g->h, t, bits, ba, g->cs);
    if (!rc && hipStreamSynchronize(g->cs) != hipSuccess) rc = SOS_EHIP;
    if (rc) {
        destroy_graph(g);
        return rc;
    }
    if (hipStreamBeginCapture(g->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        destroy_graph(g);
        return SOS_EHIP;
    }
    rc = batch_enqueue(g->h, t, bits, ba, g->cs);
    const hipError_t e = hipStreamEndCapture(g->cs, &g->graph);
    if (!rc && (e != hipSuccess || !g->graph)) rc = SOS_EHIP;
    if (!rc && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = SOS_EHIP;
    if (rc) {
        destroy_graph(g);
        return rc;
    }
    *out = g;
    return SOS_OK;
}

int sos_graph_launch(sos_graph_t g, hipStream_t stream)
{
    if (!g) return SOS_EINVAL;
    DeviceGuard dg(g->device);
    if (!dg.ok) return SOS_EHIP;
    return hipGraphLaunch(g->exec, stream) == hipSuccess ? SOS_OK : SOS_EHIP;
}

int sos_graph_last_error(sos_graph_t g)
{
    if (!g) return SOS_EINVAL;
    return sos_last_error(g->h);
}

int sos_graph_destroy(sos_graph_t g)
{
    if (!g) return SOS_EINVAL;
    {
        DeviceGuard dg(g->device);
        (void)hipDeviceSynchronize();
    }
    destroy_graph(g);
    return SOS_OK;
}

int sos_tune_batched(sos_handle_t h, int B, int kmax, int64_t total_rows, int64_t total_samples,
                     const int32_t *K, const int32_t *sec_off, const float *sections,
                     const int64_t *sig_off, const float *x, float *y, const float *zi,
                     float *zf, hipStream_t stream, int reps, int *L_out, int *N_out,
                     float *ms_out)
{
    if (!h || reps < 1 || reps > 1000) return SOS_EINVAL;
    BatchArgs ba{B, kmax, total_rows, total_samples, K, sec_off, sections, sig_off, x, y, zi, zf};
    int rc = batch_check(ba);
    if (rc) return rc;
    if (B == 0) return SOS_EINVAL;
    // repeated runs must neither move the state nor re-filter their own output
    if (zi && zi == zf) return SOS_EINVAL;
    if (total_samples > 0 && x == y) return SOS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceGuard dg(h->device);
    if (!dg.ok) return SOS_EHIP;
    const int bits = bits_of(h);

    // model pruning: padding. A group is C samples whatever the signal's
    // length, so the padded work sum_i ceil(n_i / C) C decides short-signal
    // batches; drop tiles whose padded work exceeds 1.5x the best tile's.
    std::vector<int64_t> off((size_t)B + 1);
    if (hipMemcpy(off.data(), sig_off, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return SOS_EHIP;
    std::vector<Tile> cand = candidates(bits);
    std::vector<double> padded(cand.size(), 0.0);
    double best_pad = 1e300;
    for (size_t c = 0; c < cand.size(); ++c) {
        const int64_t C = (int64_t)cand[c].L * cand[c].N;
        double w = 0.0;
        for (int i = 0; i < B; ++i) {
            const int64_t n = std::max<int64_t>(off[(size_t)i + 1] - off[(size_t)i], 0);
            w += (double)((n + C - 1) / C * C);
        }
        padded[c] = w;
        best_pad = std::min(best_pad, w);
    }

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SOS_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SOS_EHIP;
    }
    // the section solvers to try: the handle's, or both when it has none set
    const int requested = h->alg;
    const TuneKey key_req = key_of(h, ba);
    std::vector<int> algs;
    if (requested == SOS_ALG_DEFAULT) {
        algs.push_back(SOS_ALG_AUTO);
        algs.push_back(SOS_ALG_PH);
    } else {
        algs.push_back(requested);
    }
    Tile best{0, 0};
    int best_alg = requested;
    float best_ms = 1e30f;
    for (size_t k = 0; k < cand.size() * algs.size() && rc == SOS_OK; ++k) {
        const size_t c = k / algs.size();
        if (padded[c] > 1.5 * best_pad) continue;
        const Tile t = cand[c];
        h->alg = algs[k % algs.size()];
        rc = batch_reserve(h, t, bits, ba, stream);
        if (rc) break;
        rc = batch_enqueue(h, t, bits, ba, stream);   // warm-up
        if (rc) break;
        std::vector<float> ms;
        for (int r = 0; r < reps && rc == SOS_OK; ++r) {
            if (hipEventRecord(e0, stream) != hipSuccess) rc = SOS_EHIP;
            if (!rc) rc = batch_enqueue(h, t, bits, ba, stream);
            if (!rc && hipEventRecord(e1, stream) != hipSuccess) rc = SOS_EHIP;
            float v = 0.0f;
            if (!rc && (hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&v, e0, e1) != hipSuccess))
                rc = SOS_EHIP;
            ms.push_back(v);
        }
        if (rc) break;
        std::sort(ms.begin(), ms.end());
        const float med = ms[ms.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = t;
            best_alg = h->alg;
        }
        if (std::getenv("SOS_TUNE_VERBOSE"))
            std::fprintf(stderr, "sos_tune: L=%d N=%d %s padded=%.3f %.4f ms\n", t.L, t.N,
                         h->alg == SOS_ALG_PH ? "ph" : (h->alg == SOS_ALG_AUTO ? "auto" : "dccr"),
                         padded[c] / std::max(1.0, (double)total_samples), med);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->alg = requested;
    if (rc) return rc;
    if (best.L == 0) return SOS_EINVAL;
    // the caller's outputs: the winning tile's (and solver's) result
    h->alg = best_alg;
    rc = batch_reserve(h, best, bits, ba, stream);
    if (!rc) rc = batch_enqueue(h, best, bits, ba, stream);
    if (rc) {
        h->alg = requested;
        return rc;
    }
    h->tile_L = best.L;
    h->tile_N = best.N;
    {
        std::lock_guard<std::mutex> tl(g_tune_mu);
        g_tune_cache[key_req] = best;
        g_tune_cache[key_of(h, ba)] = best;
    }
    if (L_out) *L_out = best.L;
    if (N_out) *N_out = best.N;
    if (ms_out) *ms_out = best_ms;
    return SOS_OK;
}

int sos_tune_lookup(sos_handle_t h, int B, int kmax, int64_t total_samples, int *L_out,
                    int *N_out)
{
    if (!h) return SOS_EINVAL;
    BatchArgs ba{B, kmax, 0, total_samples, nullptr, nullptr, nullptr, nullptr,
                 nullptr, nullptr, nullptr, nullptr};
    std::lock_guard<std::mutex> tl(g_tune_mu);
    auto it = g_tune_cache.find(key_of(h, ba));
    if (it == g_tune_cache.end()) return SOS_EINVAL;
    if (L_out) *L_out = it->second.L;
    if (N_out) *N_out = it->second.N;
    return SOS_OK;
}

}  // extern "C"
