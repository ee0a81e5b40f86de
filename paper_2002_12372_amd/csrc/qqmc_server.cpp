/*
 * qqmc_server.cpp -- continuous-batching serving loop for parameter-sweep
 * requests (each request: one dot, one order-n integral).
 *
 * A scheduler thread owns the device work:
 *   admission   requests queue in arrival order; the head is admitted while
 *               a slot is free and its device footprint (tables unless
 *               cached, shifts, tile sums) fits in the HBM budget;
 *   batching    every launch takes tiles from all admitted requests in turn
 *               (round robin, up to a per-launch cost budget), so requests
 *               that arrive while others run share the next launches;
 *   pipelining  two launches are in flight on the server's stream, so the
 *               host prepares launch k+1 while launch k runs;
 *   completion  when all tiles of a request are done its per-shift sums are
 *               reduced on the device and copied back, and its device
 *               buffers are released.
 * Green's-function tables stay on the device, shared by requests with the
 * same dot parameters (reference counted; unused ones are evicted first when
 * memory runs short).  Tiles are the same as qqmc_eval_order_async's for the
 * server's tile length, so every result equals the solo evaluation bit for
 * bit.
 */
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "qqmc_internal.h"

namespace qqmc {
namespace {

using Clock = std::chrono::steady_clock;

struct TableEntry {
    qqmc_tables t = nullptr;
    int refs = 0;
    size_t bytes = 0;
    uint64_t last_use = 0;
};

using TableKey = std::tuple<double, double, double, double, double, int32_t>;

struct Request {
    uint64_t ticket = 0;
    qqmc_dot dot{};
    ItemDesc desc{};
    std::vector<double> shifts;
    TableKey key;
    size_t footprint = 0;
    double *d_shifts = nullptr, *d_tiles = nullptr, *d_sums = nullptr;
    int64_t next_tile = 0, done_tiles = 0;
    double t_submit = 0.0, t_done = 0.0;
    bool finished = false;
    qqmc_status status = QQMC_OK;
    std::vector<double> q_shift;
    double q_mean[2] = {0.0, 0.0};
    double q_stderr = 0.0;
};

struct Launch {
    hipEvent_t done = nullptr;
    ItemDesc *d_items = nullptr;
    TileRef *d_tiles = nullptr;
    size_t cap_items = 0, cap_tiles = 0;
    std::vector<std::pair<std::shared_ptr<Request>, int64_t>> issued; /* request, #tiles */
    bool busy = false;
};

} // namespace
} // namespace qqmc

struct qqmc_server_s {
    size_t budget = 0, used = 0;
    int32_t max_slots = 1, tile_len = 1024;
    double launch_cost = 0.0;
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t grid = 0, lds = 0;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1, use_clock = 0;
    std::deque<std::shared_ptr<qqmc::Request>> waiting;
    std::vector<std::shared_ptr<qqmc::Request>> active;
    std::map<uint64_t, std::shared_ptr<qqmc::Request>> all;
    std::map<qqmc::TableKey, qqmc::TableEntry> tables;
    qqmc::Launch launches[2];
    int next_launch = 0;
    std::thread worker;
    std::string fatal;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace qqmc {
namespace {

size_t table_bytes(const qqmc_dot &d) { return sizeof(double) * 4 * (size_t)d.n_grid; }

size_t request_bytes(const Request &r, bool need_table)
{
    return (need_table ? table_bytes(r.dot) : 0) + sizeof(double) * r.shifts.size() +
           sizeof(double) * 2 * (size_t)r.desc.n_tiles + sizeof(double) * 2 * (size_t)r.desc.n_shifts;
}

/* Frees unused cached tables (oldest first) until `need` more bytes fit. */
void evict_tables(qqmc_server_s *s, size_t need)
{
    while (s->used + need > s->budget) {
        auto victim = s->tables.end();
        for (auto it = s->tables.begin(); it != s->tables.end(); ++it)
            if (it->second.refs == 0 && (victim == s->tables.end() || it->second.last_use < victim->second.last_use))
                victim = it;
        if (victim == s->tables.end()) return;
        s->used -= victim->second.bytes;
        qqmc_free_tables(victim->second.t);
        s->tables.erase(victim);
    }
}

/* Admits waiting requests in arrival order (called with the lock held). */
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
            qqmc_status st = qqmc_make_tables(&r->dot, s->stream, &t);
            if (st != QQMC_OK) {
                r->status = st;
                r->finished = true;
                r->t_done = s->now();
                s->cv_done.notify_all();
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
        hipError_t e = hipMalloc(&r->d_shifts, sizeof(double) * r->shifts.size());
        if (e == hipSuccess) e = hipMalloc(&r->d_tiles, sizeof(double) * 2 * r->desc.n_tiles);
        if (e == hipSuccess) e = hipMalloc(&r->d_sums, sizeof(double) * 2 * r->desc.n_shifts);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->d_shifts, r->shifts.data(), sizeof(double) * r->shifts.size(),
                               hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) {
            r->status = hip_error(e, "server admission");
            r->finished = true;
            r->t_done = s->now();
            it->second.refs -= 1;
            s->cv_done.notify_all();
            continue;
        }
        r->desc.shifts = r->d_shifts;
        r->desc.tile_sums = r->d_tiles;
        s->used += request_bytes(*r, false);
        s->active.push_back(r);
    }
}

void finish(qqmc_server_s *s, const std::shared_ptr<Request> &r)
{
    /* device reduction of the tile sums, then the host epilogue */
    ItemDesc *d_item = nullptr;
    int64_t *d_base = nullptr;
    const int64_t zero = 0;
    hipError_t e = hipMalloc(&d_item, sizeof(ItemDesc));
    if (e == hipSuccess) e = hipMalloc(&d_base, sizeof(int64_t));
    if (e == hipSuccess) e = hipMemcpyAsync(d_item, &r->desc, sizeof(ItemDesc), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_base, &zero, sizeof(int64_t), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = launch_shift_reduce(d_item, 1, d_base, r->d_sums, r->desc.n_shifts, s->stream);
    std::vector<double> sums(2 * (size_t)r->desc.n_shifts);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sums.data(), r->d_sums, sizeof(double) * sums.size(), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (d_item) hipFree(d_item);
    if (d_base) hipFree(d_base);
    if (e != hipSuccess) {
        r->status = hip_error(e, "server completion");
    } else {
        const int K = r->desc.n_shifts;
        const double N = (double)r->desc.mask + 1.0;
        r->q_shift.resize(2 * (size_t)K);
        double mr = 0.0, mi = 0.0;
        for (int k = 0; k < K; ++k) {
            r->q_shift[2 * k] = sums[2 * k] / N;
            r->q_shift[2 * k + 1] = sums[2 * k + 1] / N;
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
    hipFree(r->d_shifts);
    hipFree(r->d_tiles);
    hipFree(r->d_sums);
    r->d_shifts = r->d_tiles = r->d_sums = nullptr;
    s->used -= request_bytes(*r, false);
    auto it = s->tables.find(r->key);
    if (it != s->tables.end()) it->second.refs -= 1;
    r->t_done = s->now();
    r->finished = true;
}

/* Fills launch slot L with tiles of the active requests (lock held).
 * Returns false if there was nothing to issue. */
bool build_launch(qqmc_server_s *s, Launch &L, std::vector<ItemDesc> &items, std::vector<TileRef> &tiles)
{
    items.clear();
    tiles.clear();
    L.issued.clear();
    std::vector<std::shared_ptr<Request>> open;
    for (auto &r : s->active)
        if (r->next_tile < r->desc.n_tiles) open.push_back(r);
    if (open.empty()) return false;
    std::vector<double> cost(open.size());
    std::vector<int64_t> take(open.size(), 0);
    for (size_t i = 0; i < open.size(); ++i) {
        const ItemDesc &d = open[i]->desc;
        const double frac = 0.5;
        cost[i] = d.tile_len * (8.0 * d.order + frac * (48.0 * std::ldexp(1.0, d.order) + 30.0 * d.order * d.order));
    }
    /* round robin, one tile per request per pass, until the cost budget */
    double spent = 0.0;
    bool progress = true;
    while (progress && spent < s->launch_cost) {
        progress = false;
        for (size_t i = 0; i < open.size() && spent < s->launch_cost; ++i) {
            if (open[i]->next_tile + take[i] < open[i]->desc.n_tiles) {
                take[i] += 1;
                spent += cost[i];
                progress = true;
            }
        }
    }
    for (size_t i = 0; i < open.size(); ++i) {
        if (!take[i]) continue;
        const int32_t idx = (int32_t)items.size();
        items.push_back(open[i]->desc);
        for (int64_t k = 0; k < take[i]; ++k) {
            TileRef t;
            t.item = idx;
            t.pad = 0;
            t.tile = open[i]->next_tile + k;
            tiles.push_back(t);
        }
        open[i]->next_tile += take[i];
        L.issued.push_back({open[i], take[i]});
    }
    /* most expensive tiles first inside the launch */
    std::stable_sort(tiles.begin(), tiles.end(), [&](const TileRef &a, const TileRef &b) {
        return items[a.item].order > items[b.item].order;
    });
    return true;
}

hipError_t submit_launch(qqmc_server_s *s, Launch &L, const std::vector<ItemDesc> &items,
                         const std::vector<TileRef> &tiles)
{
    hipError_t e = hipSuccess;
    if (items.size() > L.cap_items) {
        if (L.d_items) hipFree(L.d_items);
        L.cap_items = std::max<size_t>(items.size(), 2 * L.cap_items);
        e = hipMalloc(&L.d_items, sizeof(ItemDesc) * L.cap_items);
    }
    if (e == hipSuccess && tiles.size() > L.cap_tiles) {
        if (L.d_tiles) hipFree(L.d_tiles);
        L.cap_tiles = std::max<size_t>(tiles.size(), 2 * L.cap_tiles);
        e = hipMalloc(&L.d_tiles, sizeof(TileRef) * L.cap_tiles);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(L.d_items, items.data(), sizeof(ItemDesc) * items.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(L.d_tiles, tiles.data(), sizeof(TileRef) * tiles.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
        int32_t grid = s->grid;
        if ((int64_t)grid > (int64_t)tiles.size()) grid = (int32_t)tiles.size();
        e = launch_batch(L.d_items, L.d_tiles, (int64_t)tiles.size(), grid, s->lds, s->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(L.done, s->stream);
    return e;
}

void retire(qqmc_server_s *s, Launch &L, std::unique_lock<std::mutex> &lk)
{
    lk.unlock();
    hipEventSynchronize(L.done);
    lk.lock();
    L.busy = false;
    for (auto &pr : L.issued) pr.first->done_tiles += pr.second;
    L.issued.clear();
    std::vector<std::shared_ptr<Request>> still;
    for (auto &r : s->active) {
        if (r->done_tiles == r->desc.n_tiles) finish(s, r);
        else still.push_back(r);
    }
    if (still.size() != s->active.size()) {
        s->active.swap(still);
        s->cv_done.notify_all();
    }
}

void worker_loop(qqmc_server_s *s)
{
    hipSetDevice(s->device);
    std::vector<ItemDesc> items;
    std::vector<TileRef> tiles;
    uint64_t seq[2] = {0, 0}, next_seq = 1;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        admit(s);
        int slot = -1;
        for (int i = 0; i < 2; ++i)
            if (!s->launches[i].busy) { slot = i; break; }
        if (slot >= 0 && build_launch(s, s->launches[slot], items, tiles)) {
            Launch &L = s->launches[slot];
            hipError_t e = submit_launch(s, L, items, tiles);
            if (e != hipSuccess) {
                s->fatal = std::string("server launch: ") + hipGetErrorString(e);
                for (auto &pr : L.issued) pr.first->status = QQMC_EDEVICE;
                hipEventRecord(L.done, s->stream);
            }
            L.busy = true;
            seq[slot] = next_seq++;
            continue;
        }
        /* nothing to issue now: retire the oldest launch in flight */
        int oldest = -1;
        for (int i = 0; i < 2; ++i)
            if (s->launches[i].busy && (oldest < 0 || seq[i] < seq[oldest])) oldest = i;
        if (oldest >= 0) {
            retire(s, s->launches[oldest], lk);
            continue;
        }
        if (s->stop && s->waiting.empty() && s->active.empty()) break;
        if (!s->waiting.empty() && s->active.empty()) {
            /* the head does not fit although nothing runs: fail it */
            auto r = s->waiting.front();
            s->waiting.pop_front();
            r->status = set_error(QQMC_EADMIT, "request cannot be admitted");
            r->finished = true;
            r->t_done = s->now();
            s->cv_done.notify_all();
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
    s->tile_len = 1024;
    hipGetDevice(&s->device);
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&s->launches[i].done, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete s;
        return hip_error(e, "server stream");
    }
    hipDeviceProp_t prop;
    hipGetDeviceProperties(&prop, s->device);
    s->lds = batch_lds_bytes(QQMC_MAX_ORDER);
    s->grid = prop.multiProcessorCount * batch_blocks_per_cu(s->lds);
    /* cost budget of one launch: enough tiles to keep every resident
     * workgroup busy for a few tiles of order 8 (or batch_tiles tiles) */
    const double c8 = 1024.0 * (64.0 + 0.5 * (48.0 * 256.0 + 30.0 * 64.0));
    const int32_t bt = batch_tiles ? batch_tiles : 4 * s->grid;
    s->launch_cost = c8 * bt;
    s->t0 = Clock::now();
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
    auto r = std::make_shared<Request>();
    Validated v;
    if (qqmc_status st = validate_order(ord, dot->n_grid, dot->t_half, &v)) return st;
    r->dot = *dot;
    r->desc = v.desc;
    r->shifts = v.shifts;
    const int64_t N = (int64_t)v.desc.mask + 1;
    r->desc.tile_len = (int32_t)std::min<int64_t>(s->tile_len, N);
    r->desc.tiles_per_shift = (int32_t)(N / r->desc.tile_len);
    r->desc.n_tiles = (int64_t)r->desc.tiles_per_shift * r->desc.n_shifts;
    r->key = TableKey(dot->eps_d, dot->gamma, dot->beta, dot->bias_v, dot->t_half, dot->n_grid);
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
    if (q_mean) { q_mean[0] = r->q_mean[0]; q_mean[1] = r->q_mean[1]; }
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
    s->cv_done.wait(lk, [&] {
        if (!s->waiting.empty() || !s->active.empty()) return false;
        return true;
    });
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
    hipStreamSynchronize(s->stream);
    for (auto &L : s->launches) {
        if (L.done) hipEventDestroy(L.done);
        if (L.d_items) hipFree(L.d_items);
        if (L.d_tiles) hipFree(L.d_tiles);
    }
    for (auto &kv : s->all) {
        auto &r = kv.second;
        if (r->d_shifts) hipFree(r->d_shifts);
        if (r->d_tiles) hipFree(r->d_tiles);
        if (r->d_sums) hipFree(r->d_sums);
    }
    for (auto &kv : s->tables) qqmc_free_tables(kv.second.t);
    if (s->stream) hipStreamDestroy(s->stream);
    delete s;
}

} // extern "C"
