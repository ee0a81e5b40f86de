/*
 * qqmc_internal.h -- structures shared by the host API and the kernels.
 */
#ifndef QQMC_INTERNAL_H
#define QQMC_INTERNAL_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/qqmc.h"

namespace qqmc {

/* Device-side description of one order-n integral. */
struct ItemDesc {
    const double *tab;       /* device: (g^<, g^>) per grid node, 4 doubles */
    const double *shifts;    /* device: n_shifts x order                    */
    double t_half, h;        /* grid half-range and spacing                 */
    double g0x, g0y;         /* vertex diagonal g^<(0) - i alpha = i (n_sigma - alpha) */
    double t_meas, tau, tau_n, inv_n;
    uint32_t z[QQMC_MAX_ORDER]; /* Korobov generating vector a^j mod N     */
    uint32_t mask;           /* N - 1                                       */
    int32_t n_grid, order, mode, n_shifts;
    int32_t tile_len, tiles_per_shift;
    int64_t n_tiles;
    double *tile_sums;       /* device, 2 per tile, or null                 */
    const double *model_cdf; /* device: learned warp, order x (bins + 1), or null */
    int32_t model_bins;
    int32_t sobol_points;    /* 1: Sobol' points (sobol below), 0: the lattice */
    double *sample_out;      /* device: per-point Re fbar (learning pass), or null */
    double alpha;            /* interaction shift U (n_up - alpha)(n_dn - alpha) */
    const double *col;       /* device: lead functions for the current, or null */
    const uint32_t *sobol;   /* device: Sobol' direction numbers (order x 32)
                                then digital shifts (n_shifts x order), or null */
};

/* Tree selection by the vertex diagonal g0 = i (n_sigma - alpha): the
 * scalar tree divides by it at the root, so below |n_sigma - alpha| = 0.05
 * (pivot growth beyond about (0.6/0.05)^2 against the largest Green's
 * function values) the paired tree runs, whose 2x2 pivot blocks stay
 * invertible at a zero diagonal; above it the scalar tree is both cheaper
 * and better conditioned. */
constexpr double kPairDiagonal = 0.05;
inline bool needs_pair(double g0y) { return g0y < kPairDiagonal && g0y > -kPairDiagonal; }

/* Batched-kernel selector of an item, 1 .. 16 QQMC_MAX_ORDER: its order,
 * plus QQMC_MAX_ORDER when it runs the paired elimination tree, plus
 * 2 QQMC_MAX_ORDER for the current, plus 4 QQMC_MAX_ORDER on Sobol' points,
 * plus 8 QQMC_MAX_ORDER through a learned second warp (the charge only): a
 * batched kernel carries only its own variant, because a kernel holding
 * both warps measured about 2% slower on the exponential warp's tiles. */
inline int32_t kernel_key(const ItemDesc &d)
{
    return d.order + (needs_pair(d.g0y) ? QQMC_MAX_ORDER : 0) +
           (d.mode == QQMC_MODE_CURRENT ? 2 * QQMC_MAX_ORDER : 0) +
           (d.sobol_points ? 4 * QQMC_MAX_ORDER : 0) +
           (d.model_cdf ? 8 * QQMC_MAX_ORDER : 0);
}
constexpr int32_t kMaxKernelKey = 16 * QQMC_MAX_ORDER;
inline int32_t key_order(int32_t key) { return (key - 1) % QQMC_MAX_ORDER + 1; }
inline bool key_pair(int32_t key) { return ((key - 1) / QQMC_MAX_ORDER) & 1; }
inline bool key_current(int32_t key) { return ((key - 1) / (2 * QQMC_MAX_ORDER)) & 1; }
inline bool key_sobol(int32_t key) { return ((key - 1) / (4 * QQMC_MAX_ORDER)) & 1; }
inline bool key_model(int32_t key) { return (key - 1) / (8 * QQMC_MAX_ORDER) == 1; }

/* Entry of the batched tile list: which item, which tile of it. */
struct TileRef {
    int32_t item;
    int32_t pad;
    int64_t tile;
};

/* Launchers (defined in qqmc_kernels.hip).  All return hipSuccess or the
 * first launch error. */
hipError_t launch_order(const ItemDesc &it, hipStream_t s);
hipError_t launch_shift_reduce(const ItemDesc *items_dev, int32_t n_items,
                               const int64_t *shift_base_dev,
                               double *shift_sums, int32_t total_shifts,
                               hipStream_t s);
hipError_t launch_points_tree(const double *tab, const double *col, int32_t n_grid,
                              double t_half, double h, double n_sigma, double alpha,
                              int32_t order,
                              double t_meas, const double *u, int64_t n_points,
                              double *f, hipStream_t s);
hipError_t launch_points_direct(const double *tab, const double *col, int32_t n_grid,
                                double t_half, double h, double n_sigma, double alpha,
                                int32_t order, double t_meas, const double *u,
                                int64_t n_points, double *f, double *mass, hipStream_t s);
/* One persistent launch over a tile list whose items all have this kernel
 * key. */
hipError_t launch_batch(int32_t key, const ItemDesc *items_dev,
                        const TileRef *tiles_dev, int64_t n_tiles,
                        int32_t grid_blocks, hipStream_t s);
/* Learning pass: per-point Re fbar of the lattice points of tile range
 * [0, it.n_tiles) into it.sample_out. */
hipError_t launch_sample(const ItemDesc &it, hipStream_t s);
hipError_t launch_tables(double *tab, int32_t n_grid, double t_half, double eps_d,
                         double gamma, double beta, double bias_v, double n_sigma,
                         hipStream_t s);
int32_t batch_blocks_per_cu(int32_t key);
/* Lane mappings (qqmc_kernels_geo.hip): the batched scalar-tree charge
 * kernel on the lattice has a second mapping from order 5 (a depth-4
 * register tree at orders 5-8 and 11-14, cooperative top levels at 9 and
 * 10); every other key has one.  Both mappings run the same eliminations
 * per index vector, only split differently between a lane's path and its
 * subtree, so tile sums agree to rounding. */
inline bool key_plain_scalar(int32_t key)
{
    return !key_pair(key) && !key_current(key) && !key_sobol(key) && !key_model(key);
}
inline bool key_has_alt(int32_t key) { return key_order(key) >= 5 && key_plain_scalar(key); }
hipError_t launch_batch_alt(int32_t order, const ItemDesc *items_dev, const TileRef *tiles_dev,
                            int64_t n_tiles, int32_t grid_blocks, hipStream_t s);
int32_t batch_blocks_per_cu_alt(int32_t order);
/* lanes that evaluate one item together and cooperative top levels (an
 * item is one point, or one top-level index prefix of 2^top_levels per
 * point) of this key's default or alternative mapping */
void mapping_shape(int32_t key, bool alt, int32_t *lanes_per_item, int32_t *top_levels);
/* Relative cost of one tile of an item (qqmc_plan.cpp). */
double tile_cost(const ItemDesc &d);
int32_t default_tile_len(const ItemDesc &d, int64_t N);
qqmc_status check_tables(qqmc_tables t);
void fill_item_tables(ItemDesc &d, const qqmc_tables_s *t);

/* Host table builder (qqmc_tables.cpp). */
double occupation_per_spin(double eps_d, double gamma, double beta,
                           double bias_v);
void build_tables_host(double eps_d, double gamma, double beta, double bias_v,
                       int32_t n_grid, double t_half, double n_sigma,
                       double *tab /* 4*n_grid, interleaved */);
/* Semicircular leads of half-bandwidth D (|eps_d| < D - gamma): fills tab as
 * above and returns n_sigma. */
double build_tables_band(double eps_d, double gamma, double beta, double bias_v, double D,
                         int32_t n_grid, double t_half, double *tab);
/* Lead functions gamma g^<_{0i}, gamma g^>_{0i} of lead i (1: mu = -V/2,
 * 2: +V/2) on the same grid, same layout. */
void build_lead_tables(double eps_d, double gamma, double beta, double bias_v, double D,
                       int32_t lead, int32_t n_grid, double t_half, double *tab);
/* Finite bandwidth requested (0 and +infinity mean the wide band). */
inline bool finite_band(const qqmc_dot *d)
{
    return d->half_bandwidth > 0.0 && d->half_bandwidth < INFINITY;
}

/* Error reporting (qqmc_api.cpp). */
qqmc_status set_error(qqmc_status st, const std::string &msg);
qqmc_status hip_error(hipError_t e, const char *what);

struct Validated {
    ItemDesc desc;             /* pointers not yet set */
    std::vector<double> shifts;
    std::vector<uint32_t> sobol; /* direction numbers, then digital shifts */
};
qqmc_status validate_order(const qqmc_order *ord, int32_t n_grid,
                           double t_half, Validated *out);

} // namespace qqmc

struct qqmc_tables_s {
    double *d_tab = nullptr;   /* 4*n_grid doubles: (g<re, g<im, g>re, g>im) */
    double *d_col = nullptr;   /* lead functions, same layout, or null       */
    int32_t n_grid = 0;
    double t_half = 0.0, h = 0.0, n_sigma = 0.0;
    int device = 0;
};

struct qqmc_model_s {
    double *d_cdf = nullptr;   /* order x (n_bins + 1) doubles                */
    int32_t order = 0, n_bins = 0;
    std::vector<double> cdf;   /* host copy                                   */
    std::vector<double> hist;  /* projected sums of the learning sample       */
    int device = 0;
};

#endif
