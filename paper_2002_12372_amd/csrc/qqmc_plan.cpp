/*
 * qqmc_plan.cpp -- batched form: many (parameter point, order) integrals in
 * one HIP-graph launch.
 *
 * Every item is cut into the same tiles qqmc_eval_order_async uses for the
 * same tile length, so each tile sum, and therefore each per-shift sum, is
 * bitwise the one the single-order launch produces.  Tiles are grouped by
 * kernel (order, and scalar or paired elimination tree); inside a group they
 * are sorted by decreasing cost (cost model below) and dealt round robin to
 * the resident workgroups of one persistent launch of that kernel
 * (workgroup b takes entries b, b + G, ...).
 * The groups run as concurrent branches of the graph (at most four branch
 * streams, groups assigned greedily to the least loaded branch, most
 * expensive first), joined before the per-shift reduction.  This balances
 * the very uneven per-item work (2^n index vectors per point, 2^16..2^22
 * points per item) while every kernel keeps the register allocation of its
 * own order.
 *
 * The tile length and the share of resident workgroups are chosen by a small
 * autotuner when the caller passes 0: each candidate is timed on a subsample
 * of every group (every k-th tile) and the fastest per point is kept.  The
 * tile-length candidates are one length for every item (64 .. 2048) and each
 * item at its own default length (the one qqmc_eval_order takes when given
 * 0).  With
 * tile_len 0 it also picks each group's lane mapping where the kernel has
 * two (the scalar-tree charge on the lattice from order 5: the default, or
 * a depth-5 register tree at orders 5 and 6, a depth-4 one at orders 7, 8
 * and 11-14, cooperative top levels at 9 and 10), timing the group alone
 * under each.  The two mappings split
 * the eliminations differently between a lane's path and its subtree, so
 * their sums agree to rounding, not bit for bit; with the default mapping
 * kept (a fixed tile_len, or the default chosen) every tile sum is the
 * single-order launch's.
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "qqmc_internal.h"

namespace qqmc {

namespace {

constexpr int kBranches = 4;

/* Probability that the warped point lies in the domain: the sum of n
 * exponential(tau) spacings stays below t, i.e. the regularised lower
 * incomplete gamma function P(n, t/tau) (series). */
double inside_fraction(int n, double t_over_tau)
{
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 400; ++k) {
        term *= t_over_tau / (n + k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    double lg = std::lgamma((double)n + 1.0);
    return std::exp(n * std::log(t_over_tau) - t_over_tau - lg) * sum;
}

struct Buffers {
    double *shifts = nullptr, *tile_sums = nullptr, *shift_sums = nullptr;
    uint32_t *sobol = nullptr;
    ItemDesc *items = nullptr;
    int64_t *base = nullptr;
    TileRef *tiles = nullptr;
    void release()
    {
        if (shifts) hipFree(shifts);
        if (sobol) hipFree(sobol);
        if (tile_sums) hipFree(tile_sums);
        if (shift_sums) hipFree(shift_sums);
        if (items) hipFree(items);
        if (base) hipFree(base);
        if (tiles) hipFree(tiles);
        *this = Buffers();
    }
};

struct Group {
    int32_t key = 0, branch = 0, grid = 0; /* kernel key: order, paired tree */
    bool alt = false;                      /* the kernel's second lane mapping */
    int64_t offset = 0, count = 0;
    double cost = 0.0;
};

int32_t group_blocks_per_cu(const Group &g)
{
    return g.alt ? batch_blocks_per_cu_alt(key_order(g.key)) : batch_blocks_per_cu(g.key);
}

hipError_t launch_group(const Group &g, const ItemDesc *items, const TileRef *tiles, int32_t grid,
                        hipStream_t s)
{
    if (g.count <= 0) return hipSuccess;
    return g.alt ? launch_batch_alt(key_order(g.key), items, tiles, g.count, grid, s)
                 : launch_batch(g.key, items, tiles, g.count, grid, s);
}

} // namespace

/* Relative cost of one tile: warp for every point, the Keldysh sum (about
 * 140 issued FP64 operations per index vector, the tree's work plus the
 * lanes' repeated set-up, plus O(n^2) per point) for the points inside the
 * domain (the charge and the current).  Only ratios matter: it orders tiles
 * and sizes launches. */
double tile_cost(const ItemDesc &d)
{
    const bool sum = d.mode == QQMC_MODE_CHARGE || d.mode == QQMC_MODE_CURRENT;
    const double frac = sum ? inside_fraction(d.order, d.t_meas / d.tau) : 0.0;
    const double per_point = 8.0 * d.order + frac * (140.0 * std::ldexp(1.0, d.order) + 30.0 * d.order * d.order);
    return per_point * d.tile_len;
}

} // namespace qqmc

struct qqmc_plan_s {
    std::vector<qqmc::ItemDesc> items;   /* device pointers filled in */
    std::vector<std::vector<double>> shifts;
    std::vector<std::vector<uint32_t>> sobol; /* direction numbers + digital shifts, or empty */
    std::vector<int64_t> shift_base;
    std::vector<double> inv_n;
    std::vector<qqmc::TileRef> tiles;    /* grouped by order */
    std::vector<qqmc::Group> groups;
    qqmc::Buffers buf;
    int64_t n_tiles = 0, n_points = 0, total_shifts = 0;
    int32_t tile_len = 0, grid_blocks = 0, max_shifts = 0, n_cu = 1;
    double grid_share = 1.0;
    hipStream_t cap = nullptr;
    hipStream_t branch[qqmc::kBranches] = {};
    hipEvent_t fork = nullptr, join[qqmc::kBranches] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;

    void drop_graph()
    {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~qqmc_plan_s()
    {
        drop_graph();
        buf.release();
        if (fork) hipEventDestroy(fork);
        for (auto &e : join)
            if (e) hipEventDestroy(e);
        for (auto &s : branch)
            if (s) hipStreamDestroy(s);
        if (cap) hipStreamDestroy(cap);
    }
};

namespace qqmc {
namespace {

/* Groups of a tile list by kernel key, sorted within a group by decreasing
 * cost, groups assigned to branches (longest processing time first). */
void make_groups(qqmc_plan_s *p, const std::vector<std::pair<double, TileRef>> &all,
                 std::vector<TileRef> &tiles, std::vector<Group> &groups)
{
    std::vector<std::vector<std::pair<double, TileRef>>> by(kMaxKernelKey + 1);
    for (auto &c : all) by[kernel_key(p->items[c.second.item])].push_back(c);
    tiles.clear();
    groups.clear();
    for (int n = 1; n <= kMaxKernelKey; ++n) {
        auto &v = by[n];
        if (v.empty()) continue;
        std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        Group g;
        g.key = n;
        g.offset = (int64_t)tiles.size();
        g.count = (int64_t)v.size();
        for (auto &c : v) {
            g.cost += c.first;
            tiles.push_back(c.second);
        }
        groups.push_back(g);
    }
    std::vector<size_t> idx(groups.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return groups[a].cost > groups[b].cost; });
    double load[kBranches] = {0.0, 0.0, 0.0, 0.0};
    for (size_t i : idx) {
        int best = 0;
        for (int b = 1; b < kBranches; ++b)
            if (load[b] < load[best]) best = b;
        groups[i].branch = best;
        load[best] += groups[i].cost;
    }
}

/* Lays out tiles for tile length `tl` (kPerItemTiles: each item at the
 * tile length qqmc_eval_order takes by default) and (re)allocates the
 * device buffers. */
constexpr int32_t kPerItemTiles = 0;

qqmc_status layout(qqmc_plan_s *p, int32_t tl)
{
    p->buf.release();
    p->tile_len = tl;
    int64_t tile_off = 0;
    std::vector<std::pair<double, TileRef>> all;
    for (size_t i = 0; i < p->items.size(); ++i) {
        ItemDesc &d = p->items[i];
        const int64_t N = (int64_t)d.mask + 1;
        d.tile_len = tl == kPerItemTiles ? default_tile_len(d, N) : (tl < N ? tl : (int32_t)N);
        d.tiles_per_shift = (int32_t)(N / d.tile_len);
        d.n_tiles = (int64_t)d.tiles_per_shift * d.n_shifts;
        const double c = tile_cost(d);
        for (int64_t t = 0; t < d.n_tiles; ++t) {
            TileRef r;
            r.item = (int32_t)i;
            r.pad = 0;
            r.tile = t;
            all.push_back({c, r});
        }
        tile_off += d.n_tiles;
    }
    make_groups(p, all, p->tiles, p->groups);
    p->n_tiles = (int64_t)p->tiles.size();

    size_t n_shift_vals = 0, n_sobol_words = 0;
    for (auto &s : p->shifts) n_shift_vals += s.size();
    for (auto &s : p->sobol) n_sobol_words += s.size();
    hipError_t e = hipMalloc(&p->buf.shifts, sizeof(double) * (n_shift_vals ? n_shift_vals : 1));
    if (e == hipSuccess && n_sobol_words)
        e = hipMalloc(&p->buf.sobol, sizeof(uint32_t) * n_sobol_words);
    if (e == hipSuccess) e = hipMalloc(&p->buf.tile_sums, sizeof(double) * 2 * (tile_off ? tile_off : 1));
    if (e == hipSuccess) e = hipMalloc(&p->buf.shift_sums, sizeof(double) * 2 * p->total_shifts);
    if (e == hipSuccess) e = hipMalloc(&p->buf.items, sizeof(ItemDesc) * p->items.size());
    if (e == hipSuccess) e = hipMalloc(&p->buf.base, sizeof(int64_t) * p->items.size());
    if (e == hipSuccess) e = hipMalloc(&p->buf.tiles, sizeof(TileRef) * (p->n_tiles ? p->n_tiles : 1));
    if (e != hipSuccess) {
        p->buf.release();
        return hip_error(e, "plan buffers");
    }
    size_t so = 0, wo = 0;
    int64_t to = 0;
    for (size_t i = 0; i < p->items.size(); ++i) {
        ItemDesc &d = p->items[i];
        e = hipMemcpy(p->buf.shifts + so, p->shifts[i].data(), sizeof(double) * p->shifts[i].size(),
                      hipMemcpyHostToDevice);
        if (e == hipSuccess && !p->sobol[i].empty()) {
            e = hipMemcpy(p->buf.sobol + wo, p->sobol[i].data(),
                          sizeof(uint32_t) * p->sobol[i].size(), hipMemcpyHostToDevice);
            d.sobol = p->buf.sobol + wo;
            wo += p->sobol[i].size();
        }
        if (e != hipSuccess) return hip_error(e, "plan upload");
        d.shifts = p->buf.shifts + so;
        d.tile_sums = p->buf.tile_sums + 2 * to;
        so += p->shifts[i].size();
        to += d.n_tiles;
    }
    e = hipMemcpy(p->buf.items, p->items.data(), sizeof(ItemDesc) * p->items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->buf.base, p->shift_base.data(), sizeof(int64_t) * p->items.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && p->n_tiles)
        e = hipMemcpy(p->buf.tiles, p->tiles.data(), sizeof(TileRef) * p->n_tiles, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "plan upload");
    return QQMC_OK;
}

/* Fork to the branch streams, one persistent launch per order group, join,
 * then the per-shift reduction, all ordered after the work already on s. */
hipError_t enqueue(qqmc_plan_s *p, const std::vector<Group> &groups, const TileRef *d_tiles,
                   double share, hipStream_t s)
{
    hipError_t e = hipEventRecord(p->fork, s);
    bool used[kBranches] = {false, false, false, false};
    for (const Group &g : groups) {
        if (e != hipSuccess) break;
        hipStream_t b = p->branch[g.branch];
        if (!used[g.branch]) {
            e = hipStreamWaitEvent(b, p->fork, 0);
            used[g.branch] = true;
        }
        /* share > 0: that fraction of the order's resident workgroups, each
         * walking a strided share of the tiles; share 0: one workgroup per
         * tile, handed out by the hardware dispatcher */
        const int32_t grid =
            share > 0.0 ? (int32_t)std::max(1.0, share * p->n_cu * group_blocks_per_cu(g))
                        : (int32_t)std::min<int64_t>(g.count, INT32_MAX);
        if (e == hipSuccess) e = launch_group(g, p->buf.items, d_tiles + g.offset, grid, b);
    }
    for (int b = 0; b < kBranches && e == hipSuccess; ++b) {
        if (!used[b]) continue;
        e = hipEventRecord(p->join[b], p->branch[b]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join[b], 0);
    }
    if (e == hipSuccess)
        e = launch_shift_reduce(p->buf.items, (int32_t)p->items.size(), p->buf.base, p->buf.shift_sums,
                                p->max_shifts, s);
    return e;
}

qqmc_status capture(qqmc_plan_s *p)
{
    p->drop_graph();
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    hipError_t le = enqueue(p, p->groups, p->buf.tiles, p->grid_share, p->cap);
    e = hipStreamEndCapture(p->cap, &p->graph);
    if (le != hipSuccess) return hip_error(le, "plan capture launch");
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_error(e, "hipGraphInstantiate");
    return QQMC_OK;
}

/* Times the plan on a subsample (every k-th tile of each group) with the
 * given workgroup share; seconds per lattice point.  The subsample is the
 * same fraction of the work for every tile length (a quarter, less for
 * very large plans), so launch overheads weigh alike in every probe. */
double probe(qqmc_plan_s *p, double share, const std::vector<Group> &which, int64_t step = 0,
             int reps = 2)
{
    if (step <= 0) step = std::max<int64_t>(4, p->n_points / ((int64_t)1 << 26));
    std::vector<TileRef> sub;
    std::vector<Group> groups;
    double pts = 0.0;
    for (const Group &g : which) {
        Group h = g;
        h.offset = (int64_t)sub.size();
        for (int64_t t = 0; t < g.count; t += step) {
            const TileRef r = p->tiles[g.offset + t];
            sub.push_back(r);
            pts += p->items[r.item].tile_len;
        }
        h.count = (int64_t)sub.size() - h.offset;
        if (h.count) groups.push_back(h);
    }
    TileRef *d_sub = nullptr;
    if (sub.empty() || hipMalloc(&d_sub, sizeof(TileRef) * sub.size()) != hipSuccess) return 1e30;
    hipMemcpy(d_sub, sub.data(), sizeof(TileRef) * sub.size(), hipMemcpyHostToDevice);
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    double best = 1e30;
    for (int rep = 0; rep < reps; ++rep) {
        hipEventRecord(a, p->cap);
        hipError_t e = enqueue(p, groups, d_sub, share, p->cap);
        hipEventRecord(b, p->cap);
        hipStreamSynchronize(p->cap);
        float ms = 0.0f;
        hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && rep > 0) best = std::min(best, (double)ms * 1e-3 / pts);
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(d_sub);
    return best;
}

} // namespace
} // namespace qqmc

using namespace qqmc;

extern "C" {

qqmc_status qqmc_plan_create(const qqmc_batch_item *items, int32_t n_items, int32_t tile_len,
                             int32_t grid_blocks, void *stream, qqmc_plan *out)
{
    if (!items || n_items < 1 || !out) return set_error(QQMC_EINVAL, "no items");
    if (tile_len != 0 && (tile_len < 64 || (tile_len & (tile_len - 1)) != 0))
        return set_error(QQMC_EINVAL, "tile_len must be 0 or a power of two >= 64");
    if (grid_blocks < 0) return set_error(QQMC_EINVAL, "grid_blocks < 0");
    auto *p = new (std::nothrow) qqmc_plan_s();
    if (!p) return set_error(QQMC_ENOMEM, "host allocation failed");
    hipGetDevice(&p->device);
    int64_t sb = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        if (qqmc_status st = check_tables(items[i].tables)) {
            delete p;
            return st;
        }
        Validated v;
        if (items[i].order.mode == QQMC_MODE_CURRENT && !items[i].tables->d_col) {
            delete p;
            return set_error(QQMC_EINVAL, "item " + std::to_string(i) +
                                              ": the current needs tables with lead functions");
        }
        if (qqmc_status st = validate_order(&items[i].order, items[i].tables->n_grid,
                                            items[i].tables->t_half, &v)) {
            delete p;
            return set_error(st, "item " + std::to_string(i) + ": " + qqmc_last_error());
        }
        fill_item_tables(v.desc, items[i].tables);
        p->items.push_back(v.desc);
        p->shifts.push_back(v.shifts);
        p->sobol.push_back(v.sobol);
        p->shift_base.push_back(sb);
        p->inv_n.push_back(v.desc.inv_n);
        sb += v.desc.n_shifts;
        p->max_shifts = std::max(p->max_shifts, v.desc.n_shifts);
        p->n_points += (int64_t)(v.desc.mask + 1) * v.desc.n_shifts;
    }
    p->total_shifts = sb;
    hipError_t e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    for (int b = 0; b < kBranches && e == hipSuccess; ++b) {
        e = hipStreamCreateWithFlags(&p->branch[b], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    /* the items' tables may still be being built on the caller's stream: the
     * plan's own stream (uploads, autotuning probes, capture) waits for
     * everything queued there so far */
    if (e == hipSuccess) e = hipEventRecord(p->fork, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->cap, p->fork, 0);
    if (e != hipSuccess) {
        delete p;
        return hip_error(e, "plan streams");
    }
    hipDeviceProp_t prop;
    hipGetDeviceProperties(&prop, p->device);
    p->n_cu = prop.multiProcessorCount;

    /* grid_blocks given: it caps the workgroups of every order's launch,
     * expressed as a share of that order's full residency */
    /* candidates: every item at its own default length first (ties keep
     * it: its sums are then the default single launch's), then one length
     * for all */
    std::vector<int32_t> tls = tile_len ? std::vector<int32_t>{tile_len}
                                        : std::vector<int32_t>{kPerItemTiles, 64, 128, 256, 512,
                                                               1024, 2048};
    std::vector<double> shares = {1.0, 0.5, 0.0};
    if (grid_blocks) shares = {std::min(1.0, (double)grid_blocks / (p->n_cu * batch_blocks_per_cu(8)))};
    int32_t best_tl = tls[0];
    double best_share = shares[0];
    if (tls.size() * shares.size() > 1) {
        double best = 1e30;
        for (int32_t tl : tls) {
            if (qqmc_status st = layout(p, tl)) {
                delete p;
                return st;
            }
            for (double sh : shares) {
                const double v = probe(p, sh, p->groups);
                if (v < best) {
                    best = v;
                    best_tl = tl;
                    best_share = sh;
                }
            }
        }
    }
    p->grid_share = best_share;
    p->grid_blocks = best_share > 0.0
                         ? (int32_t)std::max(1.0, best_share * p->n_cu * batch_blocks_per_cu(8))
                         : 0;
    if (qqmc_status st = layout(p, best_tl)) {
        delete p;
        return st;
    }
    if (tile_len == 0) {
        /* lane mapping per group: each candidate timed on the group alone */
        for (Group &g : p->groups) {
            if (!key_has_alt(g.key)) continue;
            Group a = g, b = g;
            a.alt = false;
            b.alt = true;
            /* a group of up to 2^25 points is timed whole (a quarter of a
             * small group is mostly launch overhead), larger ones on every
             * k-th tile; best of three after a warm-up */
            int64_t pts = 0;
            for (int64_t t = 0; t < g.count; ++t) pts += p->items[p->tiles[g.offset + t].item].tile_len;
            const int64_t step = pts <= ((int64_t)1 << 25) ? 1 : 0;
            const double t0 = probe(p, best_share, {a}, step, 4);
            const double t1 = probe(p, best_share, {b}, step, 4);
            g.alt = t1 < t0;
        }
    }
    if (qqmc_status st = capture(p)) {
        delete p;
        return st;
    }
    *out = p;
    return QQMC_OK;
}

qqmc_status qqmc_plan_run(qqmc_plan p, void *stream)
{
    if (!p || !p->exec) return set_error(QQMC_EINVAL, "plan is NULL");
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    return QQMC_OK;
}

qqmc_status qqmc_plan_results(qqmc_plan p, void *stream, double *q_shift)
{
    if (!p || !q_shift) return set_error(QQMC_EINVAL, "NULL argument");
    std::vector<double> sums(2 * (size_t)p->total_shifts);
    hipError_t e = hipMemcpyAsync(sums.data(), p->buf.shift_sums, sizeof(double) * sums.size(),
                                  hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "plan results");
    for (size_t i = 0; i < p->items.size(); ++i) {
        const int64_t b = p->shift_base[i];
        for (int32_t s = 0; s < p->items[i].n_shifts; ++s) {
            q_shift[2 * (b + s)] = sums[2 * (b + s)] * p->inv_n[i];
            q_shift[2 * (b + s) + 1] = sums[2 * (b + s) + 1] * p->inv_n[i];
        }
    }
    return QQMC_OK;
}

qqmc_status qqmc_plan_info(qqmc_plan p, int64_t *n_tiles, int64_t *n_points, int32_t *tile_len,
                           int32_t *grid_blocks, int32_t *lanes_per_item, int32_t *top_levels)
{
    if (!p) return set_error(QQMC_EINVAL, "plan is NULL");
    if (n_tiles) *n_tiles = p->n_tiles;
    if (n_points) *n_points = p->n_points;
    if (tile_len) *tile_len = p->tile_len;
    if (grid_blocks) *grid_blocks = p->grid_blocks;
    int32_t lanes[QQMC_MAX_ORDER] = {}, top[QQMC_MAX_ORDER] = {};
    /* the scalar-tree charge group of an order first, else any group */
    for (int pass = 0; pass < 2; ++pass)
        for (const Group &g : p->groups) {
            const int n = key_order(g.key) - 1;
            if (lanes[n] == 0 && (pass == 1 || key_plain_scalar(g.key)))
                mapping_shape(g.key, g.alt, &lanes[n], &top[n]);
        }
    for (int n = 0; n < QQMC_MAX_ORDER; ++n) {
        if (lanes_per_item) lanes_per_item[n] = lanes[n];
        if (top_levels) top_levels[n] = top[n];
    }
    return QQMC_OK;
}

qqmc_status qqmc_plan_set_geometry(qqmc_plan p, int32_t order, int32_t lanes_per_item,
                                   int32_t top_levels)
{
    if (!p) return set_error(QQMC_EINVAL, "plan is NULL");
    for (Group &g : p->groups) {
        if (key_order(g.key) != order || !key_has_alt(g.key)) continue;
        bool alt = false;
        int32_t l0, t0, l1, t1;
        mapping_shape(g.key, false, &l0, &t0);
        mapping_shape(g.key, true, &l1, &t1);
        if (lanes_per_item == l0 && top_levels == t0) alt = false;
        else if (lanes_per_item == l1 && top_levels == t1) alt = true;
        else
            return set_error(QQMC_EINVAL, "order " + std::to_string(order) + " has no mapping with " +
                                              std::to_string(lanes_per_item) + " lanes per item and " +
                                              std::to_string(top_levels) + " top levels");
        if (alt == g.alt) return QQMC_OK;
        g.alt = alt;
        if (qqmc_status st = capture(p)) {
            g.alt = !alt;
            capture(p);
            return st;
        }
        return QQMC_OK;
    }
    return set_error(QQMC_EINVAL, "the plan has no scalar-tree charge group of order " +
                                      std::to_string(order) + " with a second lane mapping");
}

void qqmc_plan_destroy(qqmc_plan p) { delete p; }

} // extern "C"
