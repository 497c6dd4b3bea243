// Serving layer: continuous batching of per-stream filtering requests.
//
// A stream is one long signal that arrives in chunks, filtered by its own
// cascade (Sec. II's problem per stream). Its sections, their coefficient
// tables and its K TDF-II states live in device tables for the life of the
// stream, so a chunk is filtered from the state the previous chunk left, in
// place (zi = zf = the stream's state rows).
//
// One scheduler thread forms steps. A step is one persistent batched launch
// (the uneven-batch path: work table, arm, filter) over at most one chunk of
// each stream with work pending, taken in arrival order of the streams, up
// to `max_slots` chunks and a sample budget derived from the device memory
// budget. The streams are dealt to two lanes; a lane queues its steps on its
// own HIP stream with its own workspace, so a stream's next chunk may enter
// its lane's next step while the current one runs (HIP stream order keeps
// each stream's chunks in FIFO order), and the two lanes' steps, over
// disjoint sets of streams, overlap on the device: one lane's small kernels
// and launch gaps run under the other lane's filter. Chunks that arrive
// while steps are on the device join their lane's next step as soon as a
// step slot frees up. Chunk buffers are the caller's device memory,
// addressed through per-signal pointer tables (no gather copies).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <new>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>
#include <vector>

#include "sos_internal.h"

using namespace sosdev;
using namespace sosint;
using Clock = std::chrono::steady_clock;

namespace {

// Steps in flight per lane. Same-box A/B at 0.5 / 2 / 4 / 5.2 M chunks/s
// (100000 chunks each, tile (256, 16)): two lanes of two steps gave p50
// 84 / 175 / 1000 / 2500 us, one lane of three 134 / 180 / 480 / 1650 us
// and two lanes of three 104-111 / 290-560 / 780-1360 / 1700-2700 us, the
// achieved rates within 10 % of each other (75-89 GS/s at 5.2 M/s).
constexpr int kSteps = 2;

// A step of at least this many samples runs at the throughput tile (512, 32)
// when the server's own tile is smaller: a saturated server forms steps of
// hundreds of chunks, where a smaller tile's per-group costs dominate, while
// steps under light load stay on the latency tile. Same-box sweep of whole
// servers, 100000 chunks queued at once: (256, 16) 97 GS/s, (512, 32) 132;
// p50 at 50 k chunks/s: 82 and 102 us.
constexpr int64_t kBigStepSamples = (int64_t)1 << 22;
constexpr size_t kDefaultBudget = 256ull << 20;  // bytes
constexpr int kPending = 1;                      // request status while not finished

// First-fit allocator of contiguous row ranges [0, n).
struct RowPool {
    std::vector<std::pair<int64_t, int64_t>> free_;   // (offset, length), sorted
    void init(int64_t n)
    {
        free_.clear();
        if (n > 0) free_.push_back({0, n});
    }
    int64_t alloc(int64_t k)
    {
        for (size_t i = 0; i < free_.size(); ++i) {
            if (free_[i].second >= k) {
                const int64_t off = free_[i].first;
                free_[i].first += k;
                free_[i].second -= k;
                if (free_[i].second == 0) free_.erase(free_.begin() + (long)i);
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t k)
    {
        if (k <= 0) return;
        auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (int64_t)0));
        it = free_.insert(it, {off, k});
        size_t i = (size_t)(it - free_.begin());
        if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
            free_[i].second += free_[i + 1].second;
            free_.erase(free_.begin() + (long)i + 1);
        }
        if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
            free_[i - 1].second += free_[i].second;
            free_.erase(free_.begin() + (long)i);
        }
    }
};

struct Request {
    int64_t stream;
    const float *x;
    float *y;
    int64_t n;
    Clock::time_point t_push;
    int status = kPending;
    double latency = 0.0;
};

struct Stream {
    int K = 0;
    int lane = 0;                   // the lane whose steps run its chunks
    int64_t row = 0;
    std::deque<uint64_t> pending;   // pushed, not yet in a step
    int64_t outstanding = 0;        // pushed, not yet retired
    bool in_ready = false;
    bool closing = false;
    int err = SOS_OK;               // sticky: a chunk failed, the state is no longer valid
};

// Per-step argument arrays, laid out identically in pinned host memory and
// in the device copy: K | sec_off | sig_off | xp | yp. A step packs its B
// chunks with ArgLayout(B); the buffers are sized for ArgLayout(max_slots),
// whose end holds the host-only result words: the launch's error bits (8
// bytes), then one error word per chunk (max_slots words).
struct ArgLayout {
    size_t k, sec, sig, xp, yp, bytes, err;
    explicit ArgLayout(int slots = 0)
    {
        auto up8 = [](size_t v) { return (v + 7) & ~(size_t)7; };
        k = 0;
        sec = up8(k + 4 * (size_t)slots);
        sig = up8(sec + 4 * (size_t)slots);
        xp = sig + 8 * ((size_t)slots + 1);
        yp = xp + 8 * (size_t)slots;
        bytes = yp + 8 * (size_t)slots;
        err = bytes;
    }
};

struct Step {
    bool busy = false;
    uint64_t seq = 0;                // launch order (steps retire in it)
    hipEvent_t done = nullptr;
    unsigned char *host = nullptr;   // pinned, ArgLayout::bytes + 8 + 4 max_slots
    std::vector<uint64_t> tickets;
};

// An independent step pipeline: its HIP stream, its workspace (control
// block, descriptors, work table), the device copy of a step's arguments and
// per-chunk error words, its step slots and its ready streams.
constexpr int kStepLanes = 2;
struct Lane {
    sos_ctx *h = nullptr;
    hipStream_t stream = nullptr;
    unsigned char *dargs = nullptr;
    unsigned *derr = nullptr;
    Step steps[kSteps];
    std::deque<int64_t> ready;        // its streams with pending chunks
};

}  // namespace

struct sos_srv {
    Lane lanes[kStepLanes];               // step pipelines over disjoint streams
    hipStream_t ostream = nullptr;    // stream opening (table preparation)
    unsigned *octrl = nullptr;        // error word of the preparation launches
    int device = 0, L = 0, N = 0, bits = 32, alg = 0;
    int L2 = 0, N2 = 0;               // throughput tile of large steps (0: none)
    int64_t C2 = 0;
    unsigned char *tabs2 = nullptr;   // max_rows x tab_row_bytes, prepared for (L2, N2)
    double rho_max = 0.0;             // tables' PH bound (automatic solver choice)
    int64_t C = 0;
    int max_slots = 0;
    int64_t max_rows = 0, max_groups = 0, max_step_samples = 0;
    size_t tab_row_bytes = 0;
    float *sections = nullptr;        // max_rows x 6
    float *state = nullptr;           // max_rows x 2
    unsigned char *tabs = nullptr;    // max_rows x tab_row_bytes
    uint64_t next_seq = 1;            // launch order of steps
    ArgLayout lay;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::unordered_map<int64_t, Stream> streams;
    int64_t next_stream = 1;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    RowPool rows;
};

namespace {

int status_of_bits(unsigned b)
{
    if (b & ERRBIT_TIMEOUT) return SOS_ETIMEOUT;
    if (b & ERRBIT_BADARG) return SOS_EINVAL;
    if (b & ERRBIT_A0) return SOS_EA0;
    if (b & ERRBIT_UNSTABLE) return SOS_EUNSTABLE;
    return SOS_OK;
}

// Finish a step: every chunk gets its own status. step_status != SOS_OK (a
// failed launch) applies to all of them; otherwise a chunk's status comes
// from its own error word (a lookback timeout in its signal, or its entry
// rejected by the work table), and a table rejected as a whole (the launch's
// bits say so, no chunk's word does) fails all of them. A failed chunk
// leaves its stream's state invalid (the step updates it in place): the
// stream keeps that status, and its chunks retired after it report it too.
void retire(sos_srv *s, Step &st, int step_status, unsigned launch_bits,
            const unsigned *chunk_bits)
{
    const Clock::time_point now = Clock::now();
    unsigned any = 0;
    for (size_t i = 0; i < st.tickets.size(); ++i) any |= chunk_bits ? chunk_bits[i] : 0u;
    const bool table_rejected = (launch_bits & ERRBIT_BADARG) && !(any & ERRBIT_BADARG);
    for (size_t i = 0; i < st.tickets.size(); ++i) {
        auto it = s->reqs.find(st.tickets[i]);
        if (it == s->reqs.end()) continue;
        Request &rq = it->second;
        int status = step_status;
        if (status == SOS_OK)
            status = table_rejected ? SOS_EINVAL
                                    : status_of_bits(chunk_bits ? chunk_bits[i] : 0u);
        auto si = s->streams.find(rq.stream);
        if (si != s->streams.end()) {
            Stream &str = si->second;
            if (str.err == SOS_OK && status != SOS_OK) str.err = status;
            if (str.err != SOS_OK) status = str.err;
            --str.outstanding;
        }
        rq.status = status;
        rq.latency = std::chrono::duration<double>(now - rq.t_push).count();
    }
    st.tickets.clear();
    st.busy = false;
    s->cv_done.notify_all();
}

// Form a step from a lane's ready streams and enqueue it on the lane (lock
// held).
void launch_step(sos_srv *s, Lane &ln, Step &st)
{
    unsigned char *hb = st.host;
    unsigned *err = reinterpret_cast<unsigned *>(hb + s->lay.err);
    struct Pick {
        int32_t K, row;
        const float *x;
        float *y;
        int64_t n;
    };
    std::vector<Pick> pick;
    int B = 0, kmax = 0;
    int64_t total = 0;
    std::deque<int64_t> deferred;
    while (!ln.ready.empty() && B < s->max_slots) {
        const int64_t sid = ln.ready.front();
        ln.ready.pop_front();
        Stream &str = s->streams[sid];
        str.in_ready = false;
        if (str.pending.empty()) continue;
        const uint64_t tk = str.pending.front();
        Request &rq = s->reqs[tk];
        if (B > 0 && total + rq.n > s->max_step_samples) {
            deferred.push_back(sid);        // does not fit this step
            continue;
        }
        str.pending.pop_front();
        pick.push_back(Pick{str.K, (int32_t)str.row, rq.x, rq.y, rq.n});
        total += rq.n;
        kmax = std::max(kmax, str.K);
        st.tickets.push_back(tk);
        ++B;
        if (!str.pending.empty()) deferred.push_back(sid);   // its next chunk: a later step
    }
    for (int64_t sid : deferred) {
        Stream &str = s->streams[sid];
        if (!str.in_ready) {
            str.in_ready = true;
            ln.ready.push_back(sid);
        }
    }
    if (B == 0) return;
    // this step's arrays, packed for its B chunks, so that the device copy
    // (made by the work-table kernel) moves only what is used
    const ArgLayout lb(B);
    int32_t *K = reinterpret_cast<int32_t *>(hb + lb.k);
    int32_t *sec = reinterpret_cast<int32_t *>(hb + lb.sec);
    int64_t *sig = reinterpret_cast<int64_t *>(hb + lb.sig);
    const float **xp = reinterpret_cast<const float **>(hb + lb.xp);
    float **yp = reinterpret_cast<float **>(hb + lb.yp);
    int64_t off = 0;
    for (int i = 0; i < B; ++i) {
        K[i] = pick[i].K;
        sec[i] = pick[i].row;
        sig[i] = off;
        xp[i] = pick[i].x;
        yp[i] = pick[i].y;
        off += pick[i].n;
    }
    sig[B] = total;
    *err = 0;
    unsigned *chunk_err = err + 2;
    st.busy = true;
    st.seq = s->next_seq++;
    sos_ctx *h = ln.h;
    unsigned char *d = ln.dargs;
    const int32_t *dK = reinterpret_cast<const int32_t *>(d + lb.k);
    const int32_t *dsec = reinterpret_cast<const int32_t *>(d + lb.sec);
    const int64_t *dsig = reinterpret_cast<const int64_t *>(d + lb.sig);
    const float *const *dxp = reinterpret_cast<const float *const *>(d + lb.xp);
    float *const *dyp = reinterpret_cast<float *const *>(d + lb.yp);
    // persistent grid, but no more workgroups than the step has groups (each
    // chunk adds at most one partial group): a step of a few chunks launches
    // a few workgroups, not a device-filling grid that mostly exits at once
    const bool big = s->tabs2 && total >= kBigStepSamples;
    const int L = big ? s->L2 : s->L, N = big ? s->N2 : s->N;
    const int64_t C = big ? s->C2 : s->C;
    const unsigned char *tabs = big ? s->tabs2 : s->tabs;
    const int64_t step_groups = total / C + B;
    int64_t grid = grid_of(s->bits, s->alg, L, N);
    if (grid <= 0 || grid > s->max_groups) grid = s->max_groups;
    if (grid > step_groups) grid = step_groups;
    // Three or four launches, no copy operations: the work-table kernel copies
    // the arguments from the step's pinned host buffer and arms the filter
    // (and, for a step of at most 1024 chunks and 4096 groups, also fills the
    // ticket map), and the last kernel reports the error bits into that
    // buffer and clears them. The step's own group bound (each chunk adds at
    // most one partial group) sizes the work table.
    bool ok =
        sos_launch_worktable_staged(B, kmax, s->max_rows, C, total,
                                    std::min(step_groups, s->max_groups), dK, dsec,
                                    dsig, h->gpre, h->sigmap, h->total_dev, s->state, s->state,
                                    h->ctrl, hb, d, (int64_t)lb.bytes, ln.derr,
                                    ln.stream) == hipSuccess &&
        sos_launch_fwd_batched(s->bits, s->alg, L, N, B, std::max(kmax, 1), dK, dsec, dsig, h->gpre,
                               h->sigmap, h->total_dev, nullptr, nullptr, tabs, s->state,
                               s->state, h->desc, h->ctrl, h->timeout_ticks, grid, dxp, dyp,
                               nullptr, 0, s->max_groups, ln.derr, ln.stream) == hipSuccess &&
        sos_launch_report_err(h->ctrl + CTRL_ERR, err, ln.derr, chunk_err, B, ln.stream) ==
            hipSuccess &&
        hipEventRecord(st.done, ln.stream) == hipSuccess;
    if (!ok) retire(s, st, SOS_EHIP, 0u, nullptr);
}

void worker_main(sos_srv *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool busy = false;
        // retire each lane's finished steps oldest first (a stream's failure
        // must reach its later chunks, which run in the same lane)
        for (Lane &ln : s->lanes)
            for (;;) {
                Step *oldest = nullptr;
                for (Step &st : ln.steps)
                    if (st.busy && (!oldest || st.seq < oldest->seq)) oldest = &st;
                if (!oldest) break;
                const hipError_t q = hipEventQuery(oldest->done);
                if (q == hipErrorNotReady) {
                    busy = true;
                    break;
                }
                const unsigned *res =
                    reinterpret_cast<const unsigned *>(oldest->host + s->lay.err);
                retire(s, *oldest, q == hipSuccess ? SOS_OK : SOS_EHIP, res[0], res + 2);
            }
        if (s->stop && !busy) break;
        bool launched = false;
        if (!s->stop)
            for (Lane &ln : s->lanes) {
                if (ln.ready.empty()) continue;
                for (Step &st : ln.steps)
                    if (!st.busy) {
                        launch_step(s, ln, st);
                        launched = true;
                        break;
                    }
            }
        if (launched) continue;
        if (busy)
            s->cv_work.wait_for(lk, std::chrono::microseconds(5));
        else
            s->cv_work.wait(lk);
    }
}

void free_server(sos_srv *s)
{
    for (Lane &ln : s->lanes) {
        for (Step &st : ln.steps) {
            if (st.done) (void)hipEventDestroy(st.done);
            if (st.host) (void)hipHostFree(st.host);
        }
        for (void *p : {(void *)ln.dargs, (void *)ln.derr})
            if (p) (void)hipFree(p);
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
        if (ln.h) (void)sos_destroy(ln.h);
    }
    for (void *p : {(void *)s->sections, (void *)s->state, (void *)s->tabs, (void *)s->tabs2,
                    (void *)s->octrl})
        if (p) (void)hipFree(p);
    if (s->ostream) (void)hipStreamDestroy(s->ostream);
    delete s;
}

// Push `count` chunks (lock not held). Returns the first failing code.
int push_many(sos_srv *s, int count, const int64_t *ids, const float *const *x,
              float *const *y, const int64_t *n, uint64_t *tickets)
{
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return SOS_ECLOSED;
    for (int r = 0; r < count; ++r) {
        auto it = s->streams.find(ids[r]);
        if (it == s->streams.end() || it->second.closing) return SOS_ECLOSED;
        if (it->second.err != SOS_OK) return it->second.err;
        if (n[r] < 0 || n[r] > s->max_step_samples || (n[r] > 0 && (!x[r] || !y[r])))
            return SOS_EINVAL;
    }
    for (int r = 0; r < count; ++r) {
        Stream &str = s->streams[ids[r]];
        const uint64_t tk = s->next_ticket++;
        Request rq;
        rq.stream = ids[r];
        rq.x = x[r];
        rq.y = y[r];
        rq.n = n[r];
        rq.t_push = now;
        s->reqs.emplace(tk, rq);
        str.pending.push_back(tk);
        ++str.outstanding;
        if (!str.in_ready) {
            str.in_ready = true;
            s->lanes[str.lane].ready.push_back(ids[r]);
        }
        tickets[r] = tk;
    }
    s->cv_work.notify_one();
    return SOS_OK;
}

}  // namespace

extern "C" {

int sos_server_create(sos_server_t *out, sos_handle_t hu, size_t device_mem_budget,
                      int max_slots)
{
    if (!out || !hu || max_slots < 1 || max_slots > (1 << 20)) return SOS_EINVAL;
    *out = nullptr;
    sos_srv *s = new (std::nothrow) sos_srv();
    if (!s) return SOS_ENOMEM;
    s->device = hu->device;
    DeviceGuard g(s->device);
    if (!g.ok) {
        delete s;
        return SOS_EHIP;
    }
    for (Lane &ln : s->lanes) {
        const int rc = sos_create(&ln.h, s->device);
        if (rc) {
            free_server(s);
            return rc;
        }
        ln.h->timeout_ticks = hu->timeout_ticks;
    }
    const Tile t = tile_of(hu);
    s->L = t.L;
    s->N = t.N;
    s->bits = bits_of(hu);
    s->rho_max = rho_max_of(hu);
    s->alg = launch_alg(s->bits, solver_of(hu), s->rho_max);
    s->C = (int64_t)t.L * t.N;
    if (s->C < 512 * 32 && sos_fwd_shape_supported(512, 32)) {
        s->L2 = 512;
        s->N2 = 32;
        s->C2 = 512 * 32;
    }
    s->max_slots = max_slots;
    s->lay = ArgLayout(max_slots);
    s->tab_row_bytes = (size_t)TAB_BYTES;
    const size_t budget = device_mem_budget ? device_mem_budget : kDefaultBudget;
    // half for per-stream rows (sections, state, tables), half for the
    // lanes' work tables and descriptors (stride up to SOS_MAX_SECTIONS)
    const size_t row_bytes = 6 * 4 + 2 * 4 + s->tab_row_bytes * (s->L2 ? 2 : 1);
    s->max_rows = (int64_t)((budget / 2) / row_bytes);
    const size_t group_bytes = (size_t)SOS_MAX_SECTIONS * 4 * 8 + 4;
    s->max_groups = (int64_t)((budget / 2) / kStepLanes / group_bytes);
    s->max_step_samples = (s->max_groups - max_slots) * s->C;
    if (s->max_rows < 1 || s->max_step_samples < s->C || s->max_rows >= ((int64_t)1 << 31) ||
        s->max_groups >= ((int64_t)1 << 31)) {
        free_server(s);
        return SOS_EINVAL;
    }
    s->rows.init(s->max_rows);
    bool ok =
        hipStreamCreateWithFlags(&s->ostream, hipStreamNonBlocking) == hipSuccess &&
        hipMalloc(&s->sections, (size_t)s->max_rows * 6 * 4) == hipSuccess &&
        hipMalloc(&s->state, (size_t)s->max_rows * 2 * 4) == hipSuccess &&
        hipMalloc(&s->tabs, (size_t)s->max_rows * s->tab_row_bytes) == hipSuccess &&
        (!s->L2 ||
         hipMalloc(&s->tabs2, (size_t)s->max_rows * s->tab_row_bytes) == hipSuccess) &&
        hipMalloc(&s->octrl, sizeof(unsigned) * CTRL_WORDS) == hipSuccess &&
        hipMemset(s->octrl, 0, sizeof(unsigned) * CTRL_WORDS) == hipSuccess;
    const size_t desc_bytes = (size_t)s->max_groups * SOS_MAX_SECTIONS * 4 * 8;
    for (Lane &ln : s->lanes) {
        sos_ctx *h = ln.h;
        ok = ok && hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) == hipSuccess &&
             hipMalloc(&ln.dargs, s->lay.bytes) == hipSuccess &&
             hipMalloc(&ln.derr, sizeof(unsigned) * (size_t)max_slots) == hipSuccess &&
             hipMalloc(&h->gpre, sizeof(int64_t) * ((size_t)max_slots + 1)) == hipSuccess &&
             hipMalloc(&h->sigmap, sizeof(int32_t) * (size_t)s->max_groups) == hipSuccess &&
             hipMalloc(&h->total_dev, sizeof(int64_t)) == hipSuccess &&
             hipMalloc(&h->desc, desc_bytes) == hipSuccess &&
             hipMemset(h->desc, 0, desc_bytes) == hipSuccess;
        for (Step &st : ln.steps) {
            ok = ok && hipEventCreateWithFlags(&st.done, hipEventDisableTiming) == hipSuccess &&
                 // coherent: kernels read the step's arguments from it and write
                 // the step's error word into it
                 hipHostMalloc(&st.host, s->lay.bytes + 8 + 4 * (size_t)max_slots,
                               hipHostMallocCoherent) == hipSuccess;
        }
        if (!ok) break;
        h->gpre_cap = (size_t)max_slots + 1;
        h->sigmap_cap = (size_t)s->max_groups;
        h->desc_cap = (size_t)s->max_groups * SOS_MAX_SECTIONS * 4;
    }
    if (!ok) {
        free_server(s);
        return SOS_ENOMEM;
    }
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        free_server(s);
        return SOS_ENOMEM;
    }
    *out = s;
    return SOS_OK;
}

int sos_server_destroy(sos_server_t s)
{
    if (!s) return SOS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // chunks not yet in a step are not run
        for (auto &kv : s->streams) {
            for (uint64_t tk : kv.second.pending) {
                auto it = s->reqs.find(tk);
                if (it != s->reqs.end()) it->second.status = SOS_ECLOSED;
            }
            kv.second.pending.clear();
        }
        for (Lane &ln : s->lanes) ln.ready.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    DeviceGuard g(s->device);
    for (Lane &ln : s->lanes) (void)hipStreamSynchronize(ln.stream);
    free_server(s);
    return SOS_OK;
}

int sos_server_limits(sos_server_t s, int64_t *max_rows, int64_t *max_chunk, int *L, int *N)
{
    if (!s) return SOS_EINVAL;
    if (max_rows) *max_rows = s->max_rows;
    if (max_chunk) *max_chunk = s->max_step_samples;
    if (L) *L = s->L;
    if (N) *N = s->N;
    return SOS_OK;
}

int sos_stream_open(sos_server_t s, const float *sections_host, int K, const float *zi_host,
                    int64_t *stream_id)
{
    if (!s || !stream_id || K < 0 || K > SOS_MAX_SECTIONS || (K > 0 && !sections_host))
        return SOS_EINVAL;
    *stream_id = 0;
    int64_t row = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return SOS_ECLOSED;
        if (K > 0) {
            row = s->rows.alloc(K);
            if (row < 0) return SOS_EBUSY;
        }
    }
    int rc = SOS_OK;
    if (K > 0) {
        DeviceGuard g(s->device);
        std::vector<float> st(2 * (size_t)K, 0.0f);
        if (zi_host) std::memcpy(st.data(), zi_host, st.size() * sizeof(float));
        std::vector<unsigned char> tab(s->tab_row_bytes * (size_t)K);
        const bool ok =
            g.ok &&
            hipMemcpyAsync(s->sections + 6 * row, sections_host, 6 * sizeof(float) * (size_t)K,
                           hipMemcpyHostToDevice, s->ostream) == hipSuccess &&
            hipMemcpyAsync(s->state + 2 * row, st.data(), st.size() * sizeof(float),
                           hipMemcpyHostToDevice, s->ostream) == hipSuccess &&
            sos_launch_prep(s->bits, s->sections + 6 * row, K, __builtin_ctz((unsigned)s->N),
                            __builtin_ctz((unsigned)(s->L / 64)),
                            s->tabs + (size_t)row * s->tab_row_bytes, s->octrl, 0, s->rho_max,
                            s->ostream) == hipSuccess &&
            (!s->tabs2 ||
             sos_launch_prep(s->bits, s->sections + 6 * row, K, __builtin_ctz((unsigned)s->N2),
                             __builtin_ctz((unsigned)(s->L2 / 64)),
                             s->tabs2 + (size_t)row * s->tab_row_bytes, s->octrl, 0, s->rho_max,
                             s->ostream) == hipSuccess) &&
            hipMemcpyAsync(tab.data(), s->tabs + (size_t)row * s->tab_row_bytes, tab.size(),
                           hipMemcpyDeviceToHost, s->ostream) == hipSuccess &&
            hipStreamSynchronize(s->ostream) == hipSuccess;
        if (!ok) {
            rc = SOS_EHIP;
        } else {
            unsigned bad = 0;
            for (int k = 0; k < K; ++k) {
                const unsigned char *p = tab.data() + (size_t)k * s->tab_row_bytes;
                unsigned long long w;
                std::memcpy(&w, p + 8 * HDR_STATUS, 8);
                bad |= (unsigned)w;
            }
            rc = status_of_bits(bad);
        }
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc == SOS_OK && s->stop) rc = SOS_ECLOSED;
    if (rc != SOS_OK) {
        if (K > 0) s->rows.release(row, K);
        return rc;
    }
    const int64_t sid = s->next_stream++;
    Stream &str = s->streams[sid];
    str.K = K;
    str.lane = (int)(sid % kStepLanes);
    str.row = row;
    *stream_id = sid;
    return SOS_OK;
}

int sos_stream_push(sos_server_t s, int64_t stream_id, const float *chunk, int64_t n, float *out,
                    uint64_t *ticket)
{
    if (!s || !ticket) return SOS_EINVAL;
    *ticket = 0;
    return push_many(s, 1, &stream_id, &chunk, &out, &n, ticket);
}

int sos_stream_push_many(sos_server_t s, int count, const int64_t *stream_ids,
                         const float *const *chunks, const int64_t *n, float *const *outs,
                         uint64_t *tickets)
{
    if (!s || count < 0 || (count > 0 && (!stream_ids || !chunks || !n || !outs || !tickets)))
        return SOS_EINVAL;
    if (count == 0) return SOS_OK;
    return push_many(s, count, stream_ids, chunks, outs, n, tickets);
}

int sos_stream_wait(sos_server_t s, uint64_t ticket, double *latency_s)
{
    if (!s) return SOS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SOS_EINVAL;
    s->cv_done.wait(lk, [&] { return it->second.status != kPending; });
    const int rc = it->second.status;
    if (latency_s) *latency_s = it->second.latency;
    s->reqs.erase(it);
    return rc;
}

int sos_stream_state(sos_server_t s, int64_t stream_id, float *zf_host)
{
    if (!s) return SOS_EINVAL;
    int K = 0;
    int64_t row = 0;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->streams.find(stream_id);
        if (it == s->streams.end()) return SOS_ECLOSED;
        s->cv_done.wait(lk, [&] { return it->second.outstanding == 0 || s->stop; });
        if (it->second.err != SOS_OK) return it->second.err;   // no valid state to export
        K = it->second.K;
        row = it->second.row;
    }
    if (K == 0) return SOS_OK;
    if (!zf_host) return SOS_EINVAL;
    DeviceGuard g(s->device);
    if (!g.ok) return SOS_EHIP;
    if (hipMemcpyAsync(zf_host, s->state + 2 * row, 2 * sizeof(float) * (size_t)K,
                       hipMemcpyDeviceToHost, s->ostream) != hipSuccess ||
        hipStreamSynchronize(s->ostream) != hipSuccess)
        return SOS_EHIP;
    return SOS_OK;
}

int sos_stream_close(sos_server_t s, int64_t stream_id)
{
    if (!s) return SOS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream_id);
    if (it == s->streams.end() || it->second.closing) return SOS_ECLOSED;
    it->second.closing = true;
    s->cv_done.wait(lk, [&] { return it->second.outstanding == 0 || s->stop; });
    if (it->second.K > 0) s->rows.release(it->second.row, it->second.K);
    s->streams.erase(it);
    return SOS_OK;
}

int sos_server_replay(sos_server_t s, int64_t R, const int64_t *stream_ids, const int64_t *offs,
                      const int64_t *lens, const double *arrival_s, const float *x, float *y,
                      double *latency_s, double *wall_s)
{
    if (!s || R < 0 || (R > 0 && (!stream_ids || !offs || !lens || !arrival_s || !x || !y)))
        return SOS_EINVAL;
    std::vector<uint64_t> tickets((size_t)R, 0);
    std::vector<const float *> xs;
    std::vector<float *> ys;
    std::vector<int64_t> ids, ns;
    const Clock::time_point t0 = Clock::now();
    int rc = SOS_OK;
    int64_t r = 0;
    while (r < R && rc == SOS_OK) {
        const double now = std::chrono::duration<double>(Clock::now() - t0).count();
        int64_t e = r;
        while (e < R && arrival_s[e] <= now) ++e;
        if (e == r) {
            std::this_thread::yield();
            continue;
        }
        xs.clear();
        ys.clear();
        ids.clear();
        ns.clear();
        for (int64_t i = r; i < e; ++i) {
            xs.push_back(x + offs[i]);
            ys.push_back(y + offs[i]);
            ids.push_back(stream_ids[i]);
            ns.push_back(lens[i]);
        }
        rc = push_many(s, (int)(e - r), ids.data(), xs.data(), ys.data(), ns.data(),
                       tickets.data() + r);
        r = e;
    }
    int last = SOS_OK;
    for (int64_t i = 0; i < r; ++i) {
        double lat = 0.0;
        const int w = sos_stream_wait(s, tickets[(size_t)i], &lat);
        if (latency_s) latency_s[i] = lat;
        if (w != SOS_OK && last == SOS_OK) last = w;
    }
    if (wall_s) *wall_s = std::chrono::duration<double>(Clock::now() - t0).count();
    return rc != SOS_OK ? rc : last;
}

}  // extern "C"
