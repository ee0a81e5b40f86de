/*
 * qqmc_noalloc.hip -- qqmc_eval_order_noalloc: the estimate of
 * qqmc_eval_order_async without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid it).
 *
 * The per-call device memory of the asynchronous form (the item descriptor
 * and shift offset read by the per-shift reduction, the shifts, the Sobol'
 * numbers and the per-tile partial sums) lives here in one file-scope device
 * array of kScratchBytes.  Each device holds its own copy until the process
 * ends; its address is looked up once per device, with that device current,
 * on the first call there, and only that address is used from the host.
 * Every call on a device reuses the array: nothing in it has to start at
 * zero (every tile writes its own sum, the reduction writes every shift),
 * and calls that overlap on one device race on it.
 */
#include <mutex>
#include <string>

#include "qqmc_internal.h"

namespace qqmc {
namespace {

constexpr size_t kScratchBytes = (size_t)QQMC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

/* The device address of this device's scratch array (host-side name is a
 * stand-in that must not reach a kernel). */
qqmc_status scratch_on_device(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(QQMC_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return QQMC_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

} // namespace
} // namespace qqmc

using namespace qqmc;

extern "C" qqmc_status qqmc_eval_order_noalloc(qqmc_tables t, const qqmc_order *ord,
                                               int32_t tile_len, void *stream,
                                               double *shift_sums, int64_t *n_tiles_out)
{
    if (qqmc_status st = check_tables(t)) return st;
    if (!shift_sums) return set_error(QQMC_EINVAL, "shift_sums is NULL");
    Validated v;
    if (qqmc_status st = validate_order(ord, t->n_grid, t->t_half, &v)) return st;
    const int64_t N = (int64_t)1 << ord->log2_n;
    ItemDesc d = v.desc;
    fill_item_tables(d, t);
    if (d.mode == QQMC_MODE_CURRENT && !d.col)
        return set_error(QQMC_EINVAL, "the current needs tables with lead functions");
    if (tile_len == 0) tile_len = default_tile_len(d, N);
    if (tile_len < 64 || tile_len % 64 != 0 || N % tile_len != 0)
        return set_error(QQMC_EINVAL, "tile_len must be a multiple of 64 dividing N");
    d.tile_len = tile_len;
    d.tiles_per_shift = (int32_t)(N / tile_len);
    d.n_tiles = (int64_t)d.tiles_per_shift * d.n_shifts;
    /* layout: descriptor, shift offset, shifts, Sobol' numbers, tile sums */
    const size_t off_item = 0;
    const size_t off_base = off_item + round256(sizeof(ItemDesc));
    const size_t off_shifts = off_base + 256;
    const size_t off_sobol = off_shifts + round256(sizeof(double) * v.shifts.size());
    const size_t off_tiles = off_sobol + round256(sizeof(uint32_t) * v.sobol.size());
    const size_t need = off_tiles + sizeof(double) * 2 * (size_t)d.n_tiles;
    if (need > kScratchBytes)
        return set_error(QQMC_EINVAL,
                         "the no-allocation entry point holds at most " +
                             std::to_string(kScratchBytes >> 20) +
                             " MiB of per-call device data (tile sums: 16 bytes per tile); "
                             "this call needs " + std::to_string(need) +
                             " bytes: pass a longer tile_len, or use qqmc_eval_order_async");
    if (n_tiles_out) *n_tiles_out = d.n_tiles;
    double *base = nullptr;
    if (qqmc_status st = scratch_on_device(&base)) return st;
    char *sb = reinterpret_cast<char *>(base);
    hipStream_t s = (hipStream_t)stream;
    d.shifts = reinterpret_cast<const double *>(sb + off_shifts);
    d.sobol = v.sobol.empty() ? nullptr : reinterpret_cast<const uint32_t *>(sb + off_sobol);
    d.tile_sums = reinterpret_cast<double *>(sb + off_tiles);
    const int64_t zero = 0;
    hipError_t e = hipMemcpyAsync(sb + off_shifts, v.shifts.data(),
                                  sizeof(double) * v.shifts.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !v.sobol.empty())
        e = hipMemcpyAsync(sb + off_sobol, v.sobol.data(), sizeof(uint32_t) * v.sobol.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sb + off_item, &d, sizeof(ItemDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sb + off_base, &zero, sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_order(d, s);
    if (e == hipSuccess)
        e = launch_shift_reduce(reinterpret_cast<const ItemDesc *>(sb + off_item), 1,
                                reinterpret_cast<const int64_t *>(sb + off_base), shift_sums,
                                d.n_shifts, s);
    if (e != hipSuccess) return hip_error(e, "qqmc_eval_order_noalloc launch");
    return QQMC_OK;
}
