/*
 * qqmc_server.cpp -- continuous-batching serving loop for parameter-sweep
 * requests (each request: one dot, one order-n integral).
 *
 * A scheduler thread owns the device work:
 *   admission   requests queue in arrival order; the head is admitted while
 *               a slot is free and its device footprint (tables unless
 *               cached, shifts, tile sums) fits in the HBM budget.  Tables
 *               are built on the device by a kernel, per-request buffers
 *               come from the stream-ordered allocator, all on an admission
 *               stream, so admission never waits for the GPU;
 *   batching    a launch takes, up to a cost budget, first the whole of
 *               every admitted request small enough to finish in it, then
 *               contiguous tile ranges of the oldest requests (first come
 *               first served), so requests that arrive while others run
 *               share the next launches; its tiles run as one batched
 *               kernel per kernel key (order, elimination tree,
 *               observable, point set);
 *   overlap     two launches are in flight on two streams, so the tail of
 *               one launch overlaps the next and the host prepares launches
 *               while the GPU runs;
 *   completion  when every tile of a request is done, its per-shift sums are
 *               reduced on the admission stream, copied to pinned host memory
 *               and its device buffers are returned to the pool.  The
 *               reduction is only queued when the launch retires: the
 *               scheduler issues the next launch first and collects the
 *               results once their event has fired (the reduction kernel
 *               waits for compute units behind the launch in flight, and
 *               waiting for it at once would leave that launch's tail
 *               alone on the GPU).
 * Green's-function tables stay on the device, shared by requests with the
 * same dot parameters (reference counted; unused ones are evicted first when
 * memory runs short).  A request is cut into the tiles qqmc_eval_order
 * uses by default, so every result equals the plain evaluation bit for bit,
 * alone or in the mix.
 */
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "qqmc_internal.h"

namespace qqmc {
namespace {

/* launches in flight: two keep the GPU fed across launch boundaries;
 * three measured 2% slower (kernels of different orders then contend for
 * the compute units), one leaves gaps */
constexpr int kSlots = 2;

struct TableEntry {
    qqmc_tables t = nullptr;
    int refs = 0;
    size_t bytes = 0;
    uint64_t last_use = 0;
};

using TableKey = std::tuple<double, double, double, double, double, int32_t, double, int32_t>;

struct Request {
    uint64_t ticket = 0;
    qqmc_dot dot{};
    ItemDesc desc{};
    std::vector<double> shifts;
    std::vector<uint32_t> sobol;     /* direction numbers + digital shifts, or empty */
    TableKey key;
    double *d_shifts = nullptr, *d_tiles = nullptr;
    uint32_t *d_sobol = nullptr;
    int64_t next_tile = 0, done_tiles = 0;
    double t_submit = 0.0, t_done = 0.0;
    bool finished = false;
    qqmc_status status = QQMC_OK;
    std::vector<double> q_shift;
    double q_mean[2] = {0.0, 0.0};
    double q_stderr = 0.0;
};

/* Pinned host staging and device buffers of one launch slot (own stream). */
struct Launch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    ItemDesc *h_items = nullptr, *d_items = nullptr;
    TileRef *h_tiles = nullptr, *d_tiles = nullptr;
    size_t cap_items = 0, cap_tiles = 0;
    std::vector<std::pair<std::shared_ptr<Request>, int64_t>> issued; /* request, #tiles */
    bool busy = false;
    uint64_t seq = 0;
};

/* Per-shift reduction of finished requests: at most one in flight (its
 * buffers are reused by the next). */
struct Completion {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    ItemDesc *h_items = nullptr, *d_items = nullptr;
    int64_t *h_base = nullptr, *d_base = nullptr;
    double *h_sums = nullptr, *d_sums = nullptr;
    size_t cap_items = 0, cap_base = 0, cap_sums = 0;
    bool pending = false;
    hipError_t error = hipSuccess;
    std::vector<std::shared_ptr<Request>> fin;
    std::vector<int64_t> base;
};

/* Grows a pinned host / device buffer pair to at least `need` elements. */
template <typename T> hipError_t grow_pair(T **h, T **d, size_t *cap, size_t need)
{
    if (need <= *cap) return hipSuccess;
    const size_t n = std::max<size_t>(need, 2 * *cap);
    if (*h) hipHostFree(*h);
    if (*d) hipFree(*d);
    *h = nullptr;
    *d = nullptr;
    hipError_t e = hipHostMalloc((void **)h, sizeof(T) * n, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void **)d, sizeof(T) * n);
    *cap = e == hipSuccess ? n : 0;
    return e;
}

} // namespace
} // namespace qqmc

struct qqmc_server_s {
    size_t budget = 0, used = 0;
    int32_t max_slots = 1;
    double launch_cost = 0.0;
    int device = 0, n_cu = 1;
    hipStream_t admit_stream = nullptr;
    hipEvent_t admitted = nullptr;   /* last admission work on admit_stream */
    bool admitted_pending = false;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1, use_clock = 0, next_seq = 1;
    std::deque<std::shared_ptr<qqmc::Request>> waiting;
    std::vector<std::shared_ptr<qqmc::Request>> active;
    std::map<uint64_t, std::shared_ptr<qqmc::Request>> all;
    std::map<qqmc::TableKey, qqmc::TableEntry> tables;
    qqmc::Launch launches[qqmc::kSlots];
    qqmc::Completion comp;
    std::thread worker;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace qqmc {
namespace {

/* the dot's tables, and a lead's dot-lead functions when it names one */
size_t table_bytes(const qqmc_dot &d)
{
    return sizeof(double) * 4 * (size_t)d.n_grid * (d.lead ? 2 : 1);
}

size_t request_bytes(const Request &r, bool need_table)
{
    return (need_table ? table_bytes(r.dot) : 0) + sizeof(double) * r.shifts.size() +
           sizeof(uint32_t) * r.sobol.size() + sizeof(double) * 2 * (size_t)r.desc.n_tiles;
}

void fail(qqmc_server_s *s, const std::shared_ptr<Request> &r, qqmc_status st)
{
    r->status = st;
    r->finished = true;
    r->t_done = s->now();
    s->cv_done.notify_all();
}

/* Frees unused cached tables (oldest first) until `need` more bytes fit. */
void evict_tables(qqmc_server_s *s, size_t need)
{
    while (s->used + need > s->budget) {
        auto victim = s->tables.end();
        for (auto it = s->tables.begin(); it != s->tables.end(); ++it)
            if (it->second.refs == 0 &&
                (victim == s->tables.end() || it->second.last_use < victim->second.last_use))
                victim = it;
        if (victim == s->tables.end()) return;
        s->used -= victim->second.bytes;
        /* no launch may still read it */
        for (auto &L : s->launches) hipStreamSynchronize(L.stream);
        hipStreamSynchronize(s->admit_stream);
        qqmc_free_tables(victim->second.t);
        s->tables.erase(victim);
    }
}

/* Admits waiting requests in arrival order (lock held). */
void admit(qqmc_server_s *s)
{
    while (!s->waiting.empty() && (int32_t)s->active.size() < s->max_slots) {
        auto r = s->waiting.front();
        auto it = s->tables.find(r->key);
        const bool need_table = it == s->tables.end();
        const size_t bytes = request_bytes(*r, need_table);
        if (s->used + bytes > s->budget) evict_tables(s, bytes);
        if (s->used + bytes > s->budget) return; /* wait for memory */
        s->waiting.pop_front();
        if (need_table) {
            qqmc_tables t = nullptr;
            qqmc_status st = qqmc_make_tables(&r->dot, s->admit_stream, &t);
            if (st != QQMC_OK) {
                fail(s, r, st);
                continue;
            }
            TableEntry e;
            e.t = t;
            e.bytes = table_bytes(r->dot);
            s->tables[r->key] = e;
            s->used += e.bytes;
            it = s->tables.find(r->key);
        }
        it->second.refs += 1;
        it->second.last_use = ++s->use_clock;
        fill_item_tables(r->desc, it->second.t);
        hipError_t e = hipMallocAsync((void **)&r->d_shifts, sizeof(double) * r->shifts.size(),
                                      s->admit_stream);
        if (e == hipSuccess)
            e = hipMallocAsync((void **)&r->d_tiles, sizeof(double) * 2 * r->desc.n_tiles, s->admit_stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->d_shifts, r->shifts.data(), sizeof(double) * r->shifts.size(),
                               hipMemcpyHostToDevice, s->admit_stream);
        if (e == hipSuccess && !r->sobol.empty()) {
            e = hipMallocAsync((void **)&r->d_sobol, sizeof(uint32_t) * r->sobol.size(),
                               s->admit_stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->d_sobol, r->sobol.data(), sizeof(uint32_t) * r->sobol.size(),
                                   hipMemcpyHostToDevice, s->admit_stream);
        }
        if (e == hipSuccess) e = hipEventRecord(s->admitted, s->admit_stream);
        if (e == hipSuccess) s->admitted_pending = true;
        if (e != hipSuccess) {
            /* release what this admission allocated before failing it */
            if (r->d_shifts) hipFreeAsync(r->d_shifts, s->admit_stream);
            if (r->d_tiles) hipFreeAsync(r->d_tiles, s->admit_stream);
            if (r->d_sobol) hipFreeAsync(r->d_sobol, s->admit_stream);
            r->d_shifts = r->d_tiles = nullptr;
            r->d_sobol = nullptr;
            it->second.refs -= 1;
            fail(s, r, hip_error(e, "server admission"));
            continue;
        }
        r->desc.shifts = r->d_shifts;
        r->desc.sobol = r->d_sobol;
        r->desc.tile_sums = r->d_tiles;
        s->used += request_bytes(*r, false);
        s->active.push_back(r);
    }
}

/* Fills and submits launch slot L with tiles of the active requests (lock
 * held).  Returns false if there was nothing to issue.  Tiles are taken in
 * two passes over the admitted requests, in admission order, up to the cost
 * budget of a launch:
 *   1. a request whose remaining work fits in a quarter of the budget is
 *      taken whole, so the many small requests of a sweep finish in the next
 *      launch instead of queueing behind large ones;
 *   2. the oldest requests' remaining tiles then fill the budget as
 *      contiguous ranges, at least enough tiles of a kernel to give every
 *      resident workgroup eight (so a launch fills the GPU), first come first
 *      served: completion follows arrival order, which bounds the tail
 *      latency, and a launch reads few tables at a time.
 * The tiles are grouped by kernel key (order, tree, observable, point set):
 * one batched launch per key, in sequence on the slot's stream; the other
 * slots' launches overlap them. */
bool issue(qqmc_server_s *s, Launch &L)
{
    const size_t na = s->active.size();
    std::vector<int64_t> take(na, 0);
    const double budget = s->launch_cost;
    double spent = 0.0;
    for (size_t i = 0; i < na && spent < budget; ++i) {
        const Request &r = *s->active[i];
        const int64_t left = r.desc.n_tiles - r.next_tile;
        if (left <= 0) continue;
        const double c = tile_cost(r.desc) * (double)left;
        if (c <= 0.25 * budget && spent + c <= budget) {
            take[i] = left;
            spent += c;
        }
    }
    for (size_t i = 0; i < na && spent < budget; ++i) {
        const Request &r = *s->active[i];
        const int64_t left = r.desc.n_tiles - r.next_tile - take[i];
        if (left <= 0) continue;
        const double tc = tile_cost(r.desc);
        const int64_t fill = 8 * (int64_t)s->n_cu * batch_blocks_per_cu(kernel_key(r.desc));
        int64_t k = tc > 0.0 ? (int64_t)std::ceil((budget - spent) / tc) : left;
        k = std::min(left, std::max(k, fill));
        take[i] += k;
        spent += tc * (double)k;
    }
    bool any = false;
    for (size_t i = 0; i < na; ++i) any = any || take[i] > 0;
    if (!any) return false;
    std::vector<std::shared_ptr<Request>> open;
    for (size_t i = 0; i < na; ++i)
        if (take[i]) open.push_back(s->active[i]);
    {
        std::vector<int64_t> t2;
        for (size_t i = 0; i < na; ++i)
            if (take[i]) t2.push_back(take[i]);
        take.swap(t2);
    }
    std::vector<ItemDesc> items;
    std::vector<std::vector<TileRef>> by(kMaxKernelKey + 1);
    L.issued.clear();
    for (size_t i = 0; i < open.size(); ++i) {
        if (!take[i]) continue;
        const int32_t idx = (int32_t)items.size();
        items.push_back(open[i]->desc);
        for (int64_t k = 0; k < take[i]; ++k) {
            TileRef t;
            t.item = idx;
            t.pad = 0;
            t.tile = open[i]->next_tile + k;
            by[kernel_key(open[i]->desc)].push_back(t);
        }
        open[i]->next_tile += take[i];
        L.issued.push_back({open[i], take[i]});
    }
    std::vector<TileRef> tiles;
    struct G {
        int32_t key;
        int64_t off, cnt;
    };
    std::vector<G> groups;
    for (int n = kMaxKernelKey; n >= 1; --n) {
        if (by[n].empty()) continue;
        groups.push_back({n, (int64_t)tiles.size(), (int64_t)by[n].size()});
        tiles.insert(tiles.end(), by[n].begin(), by[n].end());
    }
    hipError_t e = grow_pair(&L.h_items, &L.d_items, &L.cap_items, items.size());
    if (e == hipSuccess) e = grow_pair(&L.h_tiles, &L.d_tiles, &L.cap_tiles, tiles.size());
    /* launches must see every admission before them */
    if (e == hipSuccess && s->admitted_pending) e = hipStreamWaitEvent(L.stream, s->admitted, 0);
    if (e == hipSuccess) {
        std::memcpy(L.h_items, items.data(), sizeof(ItemDesc) * items.size());
        std::memcpy(L.h_tiles, tiles.data(), sizeof(TileRef) * tiles.size());
        e = hipMemcpyAsync(L.d_items, L.h_items, sizeof(ItemDesc) * items.size(), hipMemcpyHostToDevice,
                           L.stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(L.d_tiles, L.h_tiles, sizeof(TileRef) * tiles.size(), hipMemcpyHostToDevice,
                           L.stream);
    /* one workgroup per tile: the hardware dispatcher hands tiles to compute
     * units as they free up, which evens out the uneven tile costs better
     * than a fixed persistent grid */
    for (size_t g = 0; g < groups.size() && e == hipSuccess; ++g) {
        const int32_t grid = (int32_t)std::min<int64_t>(groups[g].cnt, INT32_MAX);
        e = launch_batch(groups[g].key, L.d_items, L.d_tiles + groups[g].off, groups[g].cnt, grid,
                         L.stream);
    }
    if (e == hipSuccess) e = hipEventRecord(L.done, L.stream);
    if (e != hipSuccess) {
        const qqmc_status st = hip_error(e, "server launch");
        for (auto &pr : L.issued) pr.first->status = st;
        hipEventRecord(L.done, L.stream);
    }
    L.busy = true;
    L.seq = s->next_seq++;
    return true;
}

/* Finishes the completion in flight, if any: waits for its event (lock
 * released meanwhile), then hands the per-shift results to the requests and
 * returns their budget.  Called by the scheduler thread only. */
void complete_end(qqmc_server_s *s, std::unique_lock<std::mutex> &lk)
{
    Completion &C = s->comp;
    if (!C.pending) return;
    lk.unlock();
    hipError_t e = hipEventSynchronize(C.done);
    lk.lock();
    if (C.error != hipSuccess) e = C.error;
    const qqmc_status st = e == hipSuccess ? QQMC_OK : hip_error(e, "server completion");
    const double now = s->now();
    for (size_t c = 0; c < C.fin.size(); ++c) {
        auto &r = C.fin[c];
        if (r->status == QQMC_OK && st != QQMC_OK) r->status = st;
        if (r->status == QQMC_OK) {
            const int K = r->desc.n_shifts;
            const double N = (double)r->desc.mask + 1.0;
            const double *v = C.h_sums + 2 * C.base[c];
            r->q_shift.resize(2 * (size_t)K);
            double mr = 0.0, mi = 0.0;
            for (int k = 0; k < K; ++k) {
                r->q_shift[2 * k] = v[2 * k] / N;
                r->q_shift[2 * k + 1] = v[2 * k + 1] / N;
                mr += r->q_shift[2 * k];
                mi += r->q_shift[2 * k + 1];
            }
            mr /= K;
            mi /= K;
            r->q_mean[0] = mr;
            r->q_mean[1] = mi;
            double ss = 0.0;
            for (int k = 0; k < K; ++k) ss += (r->q_shift[2 * k] - mr) * (r->q_shift[2 * k] - mr);
            r->q_stderr = K > 1 ? std::sqrt(ss / (K - 1)) / std::sqrt((double)K) : std::nan("");
        }
        s->used -= request_bytes(*r, false);
        auto it = s->tables.find(r->key);
        if (it != s->tables.end()) it->second.refs -= 1;
        r->t_done = now;
        r->finished = true;
    }
    C.fin.clear();
    C.pending = false;
    std::vector<std::shared_ptr<Request>> still;
    for (auto &r : s->active)
        if (!r->finished) still.push_back(r);
    s->active.swap(still);
    s->cv_done.notify_all();
}

/* Queues the per-shift reduction of finished requests on the completion
 * stream, the copy of the sums to pinned host memory and the release of the
 * requests' device buffers, then records the completion's event; the
 * results are taken by complete_end.  Lock held. */
void complete_begin(qqmc_server_s *s, std::vector<std::shared_ptr<Request>> &fin,
                    std::unique_lock<std::mutex> &lk)
{
    if (fin.empty()) return;
    complete_end(s, lk);
    Completion &C = s->comp;
    C.base.assign(fin.size(), 0);
    int64_t sums = 0;
    int32_t kmax = 1;
    for (size_t c = 0; c < fin.size(); ++c) {
        C.base[c] = sums;
        sums += fin[c]->desc.n_shifts;
        kmax = std::max(kmax, fin[c]->desc.n_shifts);
    }
    hipError_t e = grow_pair(&C.h_items, &C.d_items, &C.cap_items, fin.size());
    if (e == hipSuccess) e = grow_pair(&C.h_base, &C.d_base, &C.cap_base, fin.size());
    if (e == hipSuccess) e = grow_pair(&C.h_sums, &C.d_sums, &C.cap_sums, 2 * (size_t)sums);
    if (e == hipSuccess) {
        for (size_t c = 0; c < fin.size(); ++c) {
            C.h_items[c] = fin[c]->desc;
            C.h_base[c] = C.base[c];
        }
        e = hipMemcpyAsync(C.d_items, C.h_items, sizeof(ItemDesc) * fin.size(), hipMemcpyHostToDevice,
                           C.stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(C.d_base, C.h_base, sizeof(int64_t) * fin.size(), hipMemcpyHostToDevice, C.stream);
    if (e == hipSuccess)
        e = launch_shift_reduce(C.d_items, (int32_t)fin.size(), C.d_base, C.d_sums, kmax, C.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(C.h_sums, C.d_sums, sizeof(double) * 2 * sums, hipMemcpyDeviceToHost, C.stream);
    for (auto &r : fin) {
        hipFreeAsync(r->d_shifts, C.stream);
        hipFreeAsync(r->d_tiles, C.stream);
        if (r->d_sobol) hipFreeAsync(r->d_sobol, C.stream);
        r->d_shifts = r->d_tiles = nullptr;
        r->d_sobol = nullptr;
    }
    const hipError_t er = hipEventRecord(C.done, C.stream);
    C.error = e != hipSuccess ? e : er;
    C.fin.swap(fin);
    C.pending = true;
}

/* Waits for launch L (lock released meanwhile) and starts the completion
 * of the requests whose last tiles it ran. */
void retire(qqmc_server_s *s, Launch &L, std::unique_lock<std::mutex> &lk)
{
    lk.unlock();
    hipEventSynchronize(L.done);
    lk.lock();
    L.busy = false;
    std::vector<std::shared_ptr<Request>> fin;
    for (auto &pr : L.issued) {
        pr.first->done_tiles += pr.second;
        if (pr.first->done_tiles == pr.first->desc.n_tiles) fin.push_back(pr.first);
    }
    L.issued.clear();
    complete_begin(s, fin, lk);
}

void worker_loop(qqmc_server_s *s)
{
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        admit(s);
        /* results whose reduction has finished, without waiting */
        if (s->comp.pending && hipEventQuery(s->comp.done) != hipErrorNotReady) {
            complete_end(s, lk);
            continue;
        }
        int slot = -1;
        for (int i = 0; i < kSlots; ++i)
            if (!s->launches[i].busy) {
                slot = i;
                break;
            }
        if (slot >= 0 && issue(s, s->launches[slot])) continue;
        /* nothing to issue now: retire the oldest launch in flight */
        int oldest = -1;
        for (int i = 0; i < kSlots; ++i)
            if (s->launches[i].busy && (oldest < 0 || s->launches[i].seq < s->launches[oldest].seq))
                oldest = i;
        if (oldest >= 0) {
            retire(s, s->launches[oldest], lk);
            continue;
        }
        if (s->comp.pending) {
            complete_end(s, lk);
            continue;
        }
        if (s->stop && s->waiting.empty() && s->active.empty()) break;
        if (!s->waiting.empty() && s->active.empty()) {
            /* the head does not fit although nothing runs: refuse it */
            auto r = s->waiting.front();
            s->waiting.pop_front();
            fail(s, r, set_error(QQMC_EADMIT, "request cannot be admitted"));
            continue;
        }
        s->cv_work.wait(lk, [&] { return s->stop || !s->waiting.empty(); });
    }
}

} // namespace
} // namespace qqmc

using namespace qqmc;

extern "C" {

qqmc_status qqmc_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t batch_tiles,
                               qqmc_server *out)
{
    if (!out || max_slots < 1 || hbm_budget_bytes == 0 || batch_tiles < 0)
        return set_error(QQMC_EINVAL, "bad server arguments");
    auto *s = new (std::nothrow) qqmc_server_s();
    if (!s) return set_error(QQMC_ENOMEM, "host allocation failed");
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    hipGetDevice(&s->device);
    /* Three streams: the two launch slots, created first, and one for
     * admission and completion.  HIP maps a process's streams onto a few
     * hardware queues (four by default) and streams past that share one;
     * two launch streams on one queue run one after the other, which takes
     * the overlap of launch tails away (measured: one kernel in flight 97%
     * of the time instead of two, 7% longer makespan, when a fourth server
     * stream shared a queue after the caller's default stream). */
    hipError_t e = hipSuccess;
    for (int i = 0; i < kSlots && e == hipSuccess; ++i) {
        Launch &L = s->launches[i];
        e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->admit_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->admitted, hipEventDisableTiming);
    s->comp.stream = s->admit_stream;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->comp.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete s;
        return hip_error(e, "server streams");
    }
    hipDeviceProp_t prop;
    hipGetDeviceProperties(&prop, s->device);
    s->n_cu = prop.multiProcessorCount;
    /* cost budget of one launch: enough order-8 tiles of 256 indices (or
     * batch_tiles of them) to give every resident workgroup about sixteen
     * (a few milliseconds) */
    ItemDesc ref;
    std::memset(&ref, 0, sizeof(ref));
    ref.order = 8;
    ref.mode = QQMC_MODE_CHARGE;
    ref.tile_len = 256;
    ref.t_meas = 10.0;
    ref.tau = 1.0;
    const int32_t bt = batch_tiles ? batch_tiles : 16 * s->n_cu * batch_blocks_per_cu(8);
    s->launch_cost = tile_cost(ref) * bt;
    s->t0 = std::chrono::steady_clock::now();
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return QQMC_OK;
}

qqmc_status qqmc_submit(qqmc_server s, const qqmc_dot *dot, const qqmc_order *ord, uint64_t *ticket)
{
    if (!s || !dot || !ord || !ticket) return set_error(QQMC_EINVAL, "NULL argument");
    if (!(dot->gamma > 0.0) || !(dot->beta > 0.0) || !(dot->t_half > 0.0) || dot->n_grid < 2 ||
        dot->n_grid > (1 << 24))
        return set_error(QQMC_EINVAL, "bad dot parameters");
    if (dot->lead != 0 && !((dot->lead == 1 || dot->lead == 2) && finite_band(dot)))
        return set_error(QQMC_EINVAL, "lead must be 0, or 1 or 2 with a finite half_bandwidth");
    auto r = std::make_shared<Request>();
    Validated v;
    if (qqmc_status st = validate_order(ord, dot->n_grid, dot->t_half, &v)) return st;
    if (ord->mode == QQMC_MODE_CURRENT && dot->lead == 0)
        return set_error(QQMC_EINVAL, "the current needs a dot with a lead (1 or 2)");
    r->dot = *dot;
    r->desc = v.desc;
    r->shifts = v.shifts;
    r->sobol = v.sobol;
    const int64_t N = (int64_t)v.desc.mask + 1;
    /* the tile length qqmc_eval_order takes by default, so that served
     * results equal the plain evaluation bit for bit */
    r->desc.tile_len = default_tile_len(r->desc, N);
    r->desc.tiles_per_shift = (int32_t)(N / r->desc.tile_len);
    r->desc.n_tiles = (int64_t)r->desc.tiles_per_shift * r->desc.n_shifts;
    r->key = TableKey(dot->eps_d, dot->gamma, dot->beta, dot->bias_v, dot->t_half, dot->n_grid,
                      finite_band(dot) ? dot->half_bandwidth : 0.0, dot->lead);
    if (request_bytes(*r, true) > s->budget)
        return set_error(QQMC_EADMIT, "request footprint exceeds the HBM budget");
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    s->waiting.push_back(r);
    s->all[r->ticket] = r;
    *ticket = r->ticket;
    s->cv_work.notify_all();
    return QQMC_OK;
}

qqmc_status qqmc_poll(qqmc_server s, uint64_t ticket, double *q_shift, double *q_mean,
                      double *q_stderr, double *t_submit_s, double *t_done_s)
{
    if (!s) return set_error(QQMC_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(QQMC_ENOTICKET, "unknown ticket");
    auto r = it->second;
    if (!r->finished) return QQMC_PENDING;
    s->all.erase(it);
    if (r->status != QQMC_OK) return set_error(r->status, "request failed");
    if (q_shift) std::memcpy(q_shift, r->q_shift.data(), sizeof(double) * r->q_shift.size());
    if (q_mean) {
        q_mean[0] = r->q_mean[0];
        q_mean[1] = r->q_mean[1];
    }
    if (q_stderr) *q_stderr = r->q_stderr;
    if (t_submit_s) *t_submit_s = r->t_submit;
    if (t_done_s) *t_done_s = r->t_done;
    return QQMC_OK;
}

double qqmc_server_now(qqmc_server s) { return s ? s->now() : 0.0; }

qqmc_status qqmc_server_drain(qqmc_server s)
{
    if (!s) return set_error(QQMC_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->waiting.empty() && s->active.empty(); });
    return QQMC_OK;
}

void qqmc_server_destroy(qqmc_server s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &L : s->launches) {
        if (L.stream) hipStreamSynchronize(L.stream);
        if (L.done) hipEventDestroy(L.done);
        if (L.h_items) hipHostFree(L.h_items);
        if (L.d_items) hipFree(L.d_items);
        if (L.h_tiles) hipHostFree(L.h_tiles);
        if (L.d_tiles) hipFree(L.d_tiles);
        if (L.stream) hipStreamDestroy(L.stream);
    }
    Completion &C = s->comp;
    if (C.stream) hipStreamSynchronize(C.stream);
    if (C.h_items) hipHostFree(C.h_items);
    if (C.d_items) hipFree(C.d_items);
    if (C.h_base) hipHostFree(C.h_base);
    if (C.d_base) hipFree(C.d_base);
    if (C.h_sums) hipHostFree(C.h_sums);
    if (C.d_sums) hipFree(C.d_sums);
    if (s->admit_stream) hipStreamSynchronize(s->admit_stream);
    for (auto &kv : s->all) {
        auto &r = kv.second;
        if (r->d_shifts) hipFree(r->d_shifts);
        if (r->d_tiles) hipFree(r->d_tiles);
        if (r->d_sobol) hipFree(r->d_sobol);
    }
    for (auto &kv : s->tables) qqmc_free_tables(kv.second.t);
    if (C.done) hipEventDestroy(C.done);
    if (s->admitted) hipEventDestroy(s->admitted);
    if (s->admit_stream) hipStreamDestroy(s->admit_stream);
    delete s;
}

} // extern "C"
