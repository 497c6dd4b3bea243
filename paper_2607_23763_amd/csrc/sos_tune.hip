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

// Model-ranked (shape, solver) pairs timed per tuning call, and the fixed
// per-group cost F of the model's prediction (the 2^28-sample order-2
// filter's excess over the copy kernel on MI355X, 374 - 330 us, over its 32
// rounds of resident groups).
constexpr size_t kTuneTimed = 6;
constexpr double kTuneGroupUs = 1.5;

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

    // the batch as the cost model sees it
    std::vector<int64_t> off((size_t)B + 1);
    std::vector<int32_t> kh((size_t)B);
    if (hipMemcpy(off.data(), sig_off, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(kh.data(), K, kh.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return SOS_EHIP;
    ModelBatch mb;
    mb.total = total_samples;
    for (int i = 0; i < B; ++i) {
        mb.len.push_back(std::max<int64_t>(off[(size_t)i + 1] - off[(size_t)i], 0));
        mb.K.push_back(std::min(std::max(kh[(size_t)i], 0), kmax));
    }
    sos_model_device md;
    (void)sos_model_device_gfx950(&md);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) ==
            hipSuccess && cus > 0)
        md.sms = cus;

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
    // price every (shape, solver) pair; drop what the budgets exclude, what
    // falls below the hiding floor, and shapes whose padded work exceeds 1.5x
    // the best shape's (a group is C samples whatever the signal's length)
    struct Pair {
        Tile t;
        int alg;
        double pred, pad;
    };
    const std::vector<Tile> shapes = candidates(bits);
    std::vector<double> padded(shapes.size(), 0.0);
    double best_pad = 1e300;
    for (size_t c = 0; c < shapes.size(); ++c) {
        const int64_t C = (int64_t)shapes[c].L * shapes[c].N;
        for (int64_t n : mb.len) padded[c] += (double)((n + C - 1) / C * C);
        best_pad = std::min(best_pad, padded[c]);
    }
    std::vector<Pair> pairs;
    for (size_t c = 0; c < shapes.size(); ++c) {
        if (padded[c] > 1.5 * best_pad) continue;
        for (int a : algs) {
            h->alg = a;
            const int la = launch_alg(bits, solver_of(h), rho_max_of(h));
            int regs = 0, lds = 0;
            if (sos_fwd_kernel_attrs(bits, la, shapes[c].L, shapes[c].N, &regs, &lds) != SOS_OK)
                continue;
            // the kernel's whole LDS (staging rows plus the wave exchange) as
            // row padding of the model's staging buffer
            const int pad = std::max(0, (lds + 4 * shapes[c].L - 1) / (4 * shapes[c].L) -
                                            shapes[c].N);
            const double ops = ph_sections(solver_of(h)) ? 7.0 : 9.0;
            const double pred = model_batch_ms(md, mb, shapes[c].L, shapes[c].N, pad, regs, ops,
                                               kTuneGroupUs);
            if (pred >= 0.0) pairs.push_back(Pair{shapes[c], a, pred, padded[c]});
        }
    }
    h->alg = requested;
    std::stable_sort(pairs.begin(), pairs.end(),
                     [](const Pair &p, const Pair &q) { return p.pred < q.pred; });
    const char *ex = std::getenv("SOS_TUNE_EXHAUSTIVE");
    const size_t timed = (ex && std::atoi(ex) == 1) ? pairs.size()
                                                    : std::min<size_t>(pairs.size(), kTuneTimed);
    const bool verbose = std::getenv("SOS_TUNE_VERBOSE") != nullptr;

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SOS_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SOS_EHIP;
    }
    Tile best{0, 0};
    int best_alg = requested;
    float best_ms = 1e30f;
    for (size_t k = 0; k < pairs.size() && rc == SOS_OK; ++k) {
        const Tile t = pairs[k].t;
        h->alg = pairs[k].alg;
        const char *an =
            h->alg == SOS_ALG_PH ? "ph"
                                 : (h->alg == SOS_ALG_AUTO
                                        ? "auto"
                                        : (h->alg == SOS_ALG_TOEPLITZ ? "toeplitz" : "dccr"));
        if (k >= timed) {
            if (verbose)
                std::fprintf(stderr, "sos_tune: L=%d N=%d %s predicted %.4f ms (not timed)\n",
                             t.L, t.N, an, pairs[k].pred);
            continue;
        }
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
        if (verbose)
            std::fprintf(stderr, "sos_tune: L=%d N=%d %s padded=%.3f predicted %.4f ms, %.4f ms\n",
                         t.L, t.N, an, pairs[k].pad / std::max(1.0, (double)total_samples),
                         pairs[k].pred, med);
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
