/*
 * qqmc.h -- C ABI of the MI355X quantum quasi-Monte Carlo (QQMC) library.
 *
 * The library estimates the order-n coefficient Q_n of the charge
 * Q(U) = sum_n Q_n U^n of an Anderson quantum dot (arXiv:2002.12372,
 * Macek et al.): a randomly shifted rank-1 lattice (or digitally shifted
 * Sobol' points, App. B) is warped through the product-of-exponentials model
 * function (optionally followed by a learned per-coordinate warp, App. I)
 * into time-ordered interaction vertices, and at every point the Keldysh sum
 * of products of spin-up and spin-down Wick determinants is evaluated on the
 * GPU.  The same path gives the particle current into a lead (App. E), for
 * the alpha-shifted interaction U (n_up - alpha)(n_dn - alpha), with
 * wide-band leads at T > 0 or T = 0 or semicircular leads of finite
 * bandwidth; single launches, batched plans (HIP graphs) and a
 * continuous-batching server share the same kernels and the same bits.
 *
 * General conventions
 *  - All arithmetic is IEEE binary64; complex numbers are (re, im) pairs of
 *    doubles.
 *  - Pointers marked "host" are ordinary host memory; pointers marked
 *    "device" are HIP device allocations (for example torch tensors'
 *    data_ptr()).  The caller owns every buffer it passes; the library owns
 *    the memory behind the opaque handles it returns.
 *  - Streams are hipStream_t values passed as void*; NULL is the null stream.
 *    Calls that return host results synchronise the stream before returning.
 *  - Functions return a qqmc_status; on failure qqmc_last_error() gives a
 *    message (per thread).  No call throws across the ABI.
 *  - Time and energy units: Gamma sets the scale only through the caller's
 *    choice; nothing is normalised inside.
 */
#ifndef QQMC_H
#define QQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QQMC_OK = 0,
    QQMC_PENDING = 1,      /* qqmc_poll: the request has not finished      */
    QQMC_EINVAL = -1,      /* an argument is outside its documented range  */
    QQMC_ENOMEM = -2,      /* a host or device allocation failed           */
    QQMC_EDEVICE = -3,     /* a HIP runtime call failed                    */
    QQMC_EADMIT = -4,      /* qqmc_submit: the request can never fit       */
    QQMC_ENOTICKET = -5    /* qqmc_poll: unknown or already collected      */
} qqmc_status;

/* Highest perturbation order the kernels are built for. */
#define QQMC_MAX_ORDER 14

/* Anderson dot between two leads (App. E "Model"): wide band (hybridisation
 * Delta = -i Gamma) or semicircular leads of half-bandwidth D, with
 * Delta(omega) = (Gamma/D)(omega - i sqrt(D^2 - omega^2)) in the band.  The
 * Green's functions are tabulated on the uniform grid tau_j = -t_half + j*h,
 * h = 2 t_half/(n_grid-1). */
typedef struct {
    double eps_d;    /* dot level                                           */
    double gamma;    /* tunnelling rate Gamma > 0                           */
    double beta;     /* inverse temperature > 0; +INFINITY for T = 0        */
    double bias_v;   /* symmetric bias V between the two leads              */
    double t_half;   /* half-range of the table grid (>= measurement time)  */
    int32_t n_grid;  /* number of grid points, 2 .. 2^24                    */
    double half_bandwidth; /* D; 0 or +INFINITY: wide band.  A finite D
                              needs |eps_d| < D - gamma (no bound state
                              outside the band; EINVAL otherwise)        */
    int32_t lead;    /* 0; or 1 (chemical potential -V/2) / 2 (+V/2): also
                        tabulate that lead's dot-lead functions for
                        QQMC_MODE_CURRENT (needs a finite D)                */
} qqmc_dot;

typedef struct qqmc_tables_s *qqmc_tables;

/* Integrand modes of qqmc_eval_order. */
enum {
    QQMC_MODE_CHARGE = 0,   /* -2 i^{n+1} S(u) W: the charge coefficient      */
    QQMC_MODE_MODEL = 1,    /* f := p_n over the whole v-domain: every sample
                               equals C = tau^n (warp/estimator self-test)    */
    QQMC_MODE_CONSTANT = 2, /* f := 1 on the ordered simplex: t^n/n!          */
    QQMC_MODE_CURRENT = 3   /* -4 i^n S(u) W with the measurement column on
                               the lead site (tables made with dot.lead = i):
                               the real part is the order-n particle current
                               from the dot into lead i, both spins, i.e.
                               -4 Re gamma G^<_{0i}(t, t) (App. E); no
                               learned warp; in plans and the server as
                               the charge is                                  */
};

/* A learned second warp (App. I, "Learning h^(i) from the integrand"): per
 * coordinate a density q_j on [0, 1), piecewise constant on n_bins equal
 * bins, applied to the lattice point before the exponential warp
 * (w_j = F_j^{-1}(x_j), weight divided by prod_j q_j(w_j)).  Opaque handle
 * owning device memory; see qqmc_learn_model. */
typedef struct qqmc_model_s *qqmc_model;

/* One order-n integral (Eq. (warped_int2)): N = 2^log2_n points of the rank-1
 * lattice with generating vector (1, a, a^2, ...) mod N, each shifted by the
 * n_shifts rows of `shifts`, warped with h(v) = exp(-v/model_tau)
 * (Eq. (hi_expo)) towards the measurement time t_meas, optionally after a
 * learned second warp. */
typedef struct {
    int32_t order;          /* n, 1 .. QQMC_MAX_ORDER                         */
    int32_t log2_n;         /* 6 .. 24                                        */
    uint64_t lattice_a;     /* odd Korobov multiplier, 1 < a < N              */
    int32_t n_shifts;       /* K >= 1                                         */
    const double *shifts;   /* host, K x order row-major, each in [0, 1);
                               copied during the call                          */
    double model_tau;       /* tau > 0                                        */
    double t_meas;          /* measurement time t, 0 < t <= table t_half      */
    int32_t mode;           /* QQMC_MODE_*; with a model, QQMC_MODE_MODEL uses
                               the combined model p_n(u) prod_j q_j(w_j)       */
    qqmc_model model;       /* learned second warp of the same order, or NULL;
                               must stay valid until the work using it ends  */
    double alpha;           /* interaction U (n_up - alpha)(n_dn - alpha)
                               (App. E, "Model"): every vertex diagonal of the
                               Wick matrices becomes g^<(0) - i alpha, the
                               measurement diagonal stays g^<(0); the tables
                               are built at the quadratic level E_d, whose
                               one-electron energy is E_d - alpha U; finite;
                               0 = the plain interaction U n_up n_dn          */
    const uint32_t *sobol_v;      /* host, order x 32, or NULL: Sobol' points
                                     (App. B) instead of the lattice; point i
                                     has coordinates (XOR over the set bits k
                                     of i of sobol_v[j][k]) * 2^-32; lattice_a
                                     and shifts are then not used            */
    const uint32_t *sobol_shifts; /* host, n_shifts x order digital shifts
                                     (XORed into the coordinate words), with
                                     sobol_v; both copied during the call
                                     (by plans and the server at creation /
                                     submission).  The charge (with or
                                     without a learned warp) and the current
                                     run on Sobol' points everywhere the
                                     lattice runs; tiles start at multiples
                                     of 64 indices (every tile_len is a power
                                     of two >= 64)                            */
} qqmc_order;

/* ---- Green's function tables (App. E, Eq. (lesser_greater_freq) with the
 * standard Keldysh normalisation g^< = i A fbar, g^> = -i A (1 - fbar)) --- */

/* Builds g^<(tau_j), g^>(tau_j) on the current device (exact residue series
 * over the Matsubara poles, one workgroup per grid node, launched on
 * `stream`; the handle is usable by later work on the same stream) and
 * n_sigma = -i g^<(0) on the host (digamma closed form).  At T = 0
 * (beta = +INFINITY) the grid is computed on the host from the Fourier
 * integral turned off the real axis into the lower half plane (App. E,
 * "Precision calculation"): along a ray from each Fermi level plus the
 * residue of the pole it encloses; uploaded, n_sigma from the arctan closed
 * form.  With a finite half_bandwidth D (any beta) the grid is computed on
 * the host by a graded Gauss-Legendre rule over the band (theta in [0, pi],
 * omega = -D cos theta, panels refined at the Fermi levels and at eps_d),
 * n_sigma from the same rule, and uploaded.  EINVAL for gamma <= 0,
 * beta <= 0 or NaN, t_half <= 0, n_grid outside 2..2^24, a negative or NaN
 * half_bandwidth, or a finite one with |eps_d| >= D - gamma. */
qqmc_status qqmc_make_tables(const qqmc_dot *dot, void *stream,
                             qqmc_tables *out);

/* Host-only form of the same computation: fills caller arrays (2*n_grid
 * doubles each, (re, im) per node) and n_sigma without touching the GPU. */
qqmc_status qqmc_tables_compute_host(const qqmc_dot *dot, double *gl,
                                     double *gg, double *n_sigma);

/* Wraps caller-supplied tables (host arrays of 2*n_grid doubles each, same
 * grid convention) so that any Green's function can be integrated.  The data
 * are copied; the caller may free them on return. */
qqmc_status qqmc_tables_from_host(const double *gl, const double *gg,
                                  int32_t n_grid, double t_half,
                                  double n_sigma, void *stream,
                                  qqmc_tables *out);

/* Copies the tables back: gl, gg host arrays of 2*n_grid doubles (either may
 * be NULL), n_sigma host scalar (may be NULL). */
qqmc_status qqmc_tables_export(qqmc_tables t, double *gl, double *gg,
                               double *n_sigma);

/* Grid size and half-range of a table handle (either pointer may be NULL). */
qqmc_status qqmc_tables_info(qqmc_tables t, int32_t *n_grid, double *t_half);

/* Releases the handle and its device memory.  NULL is ignored. */
void qqmc_free_tables(qqmc_tables t);

/* Dot-lead functions of lead i for the current (App. E; finite bandwidth):
 * with Sigma_i = Delta/2 and the Langreth rules for g_{0i} = g_{00} gamma G_i,
 *   gamma g^<_{0i}(omega) = conj(Delta)/2 g^< + Sigma^<_i g^R,
 *   gamma g^>_{0i}(omega) = conj(Delta)/2 g^> + Sigma^>_i g^R,
 *   Sigma^<_i = -i f_i Im Delta,  Sigma^>_i = i (1 - f_i) Im Delta,
 * Fourier transformed on the dot's grid by the band rule of
 * qqmc_make_tables.  Host-only: fills cl, cg (2*n_grid doubles each).
 * EINVAL unless dot->lead is 1 or 2 and the band is finite and valid. */
qqmc_status qqmc_lead_tables_compute_host(const qqmc_dot *dot, double *cl, double *cg);

/* Attaches caller lead functions (host arrays as above, same grid as t) to
 * existing tables, replacing any there; synchronous. */
qqmc_status qqmc_tables_lead_from_host(qqmc_tables t, const double *cl, const double *cg);

/* ---- The hot path -------------------------------------------------------
 * qqmc_eval_order: estimates Q_n (Eq. (warped_int2), randomised over shifts
 * as in App. G).  Launches the integrand kernel over all N x K points on
 * `stream`, reduces on the device, copies K complex per-shift estimates
 * back and synchronises the stream.
 *   q_shift  host, 2*n_shifts doubles: Q^{(s)} = (1/N) sum_i fbar_{i,s}
 *   q_mean   host, 2 doubles: mean over shifts (may be NULL)
 *   q_stderr host, 1 double: sample standard deviation of Re Q^{(s)} over
 *            shifts / sqrt(K); NaN for K = 1 (may be NULL)
 * EINVAL on any out-of-range field, an even or out-of-range lattice_a, a
 * shift outside [0, 1), t_meas > t_half or a model of another order.  Q_n is
 * real; the imaginary part is a rounding diagnostic. */
qqmc_status qqmc_eval_order(qqmc_tables t, const qqmc_order *ord,
                            void *stream, double *q_shift, double *q_mean,
                            double *q_stderr);

/* Asynchronous form of qqmc_eval_order for callers that keep results on the
 * device: launches on `stream` and returns without synchronising.
 *   tile_len   lattice indices per work tile (a multiple of 64 dividing N),
 *              or 0 for the library's choice
 *   tile_sums  device, 2*n_tiles doubles or NULL: per-tile sums of fbar,
 *              tile k covering shift k / (N/tile_len) and lattice indices
 *              [(k % (N/tile_len)) * tile_len, ... + tile_len)
 *   shift_sums device, 2*n_shifts doubles: sum_i fbar_{i,s} (not divided
 *              by N)
 * n_tiles_out (host, may be NULL) receives the number of tiles.  The buffers
 * must stay valid until the stream reaches the end of the launch. */
qqmc_status qqmc_eval_order_async(qqmc_tables t, const qqmc_order *ord,
                                  int32_t tile_len, void *stream,
                                  double *tile_sums, double *shift_sums,
                                  int64_t *n_tiles_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): the estimate of
 * qqmc_eval_order_async without per-tile output and without any device
 * allocation.  The per-call device data (shifts, Sobol' numbers, the
 * per-tile partial sums, 16 bytes per tile, and the reduction's descriptor)
 * lives in a static device array of QQMC_NOALLOC_SCRATCH_BYTES that each
 * device holds from its first call until the process ends.  EINVAL if a call
 * needs more (pass a longer tile_len); otherwise as qqmc_eval_order_async,
 * whose per-shift sums it reproduces bit for bit for the same tile_len.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other streams, other threads) race and must be serialised by
 * the caller.  shift_sums: device, 2*n_shifts doubles, as above. */
#define QQMC_NOALLOC_SCRATCH_BYTES (4u << 20)
qqmc_status qqmc_eval_order_noalloc(qqmc_tables t, const qqmc_order *ord,
                                    int32_t tile_len, void *stream,
                                    double *shift_sums, int64_t *n_tiles_out);

/* Per-point integrand f_n(u) = -2 i^{n+1} S(u) of Eq. (integral_gf) (the
 * integrand of Q_n over the ordered simplex, without warping weight).
 *   alpha   interaction shift, as in qqmc_order (finite)
 *   observable  QQMC_OBS_CHARGE: f_n as above; QQMC_OBS_CURRENT: -4 i^n S(u)
 *           with the lead site in the measurement column (tables with lead
 *           functions)
 *   u       device, n_points x order row-major, vertex times (u_1..u_n)
 *   f       device, 2*n_points doubles (re, im)
 *   method  QQMC_METHOD_TREE: the production kernel; requires
 *           t_meas >= u_1 >= u_2 >= ... >= u_n >= 0 per row and writes NaN
 *           for rows that violate it;
 *           QQMC_METHOD_DIRECT: enumerates all 2^n Keldysh index vectors with
 *           one partially pivoted LU per determinant; any vertex times
 *           (within the table range).
 *   mass    device, n_points doubles, or NULL: the term mass of each point,
 *           |c| sum_a |det_up(a) det_dn(a)| with c the prefactor above
 *           (2 for the charge, 4 for the current), so |f| <= mass and
 *           |f| / mass measures the cancellation in the Keldysh sum (the
 *           sign problem of the expansion); direct method only (EINVAL
 *           with the tree method).
 * Asynchronous on `stream`. */
enum { QQMC_METHOD_TREE = 0, QQMC_METHOD_DIRECT = 1 };
enum { QQMC_OBS_CHARGE = 0, QQMC_OBS_CURRENT = 1 };
qqmc_status qqmc_eval_points(qqmc_tables t, int32_t order, double t_meas,
                             double alpha, int32_t observable, const double *u,
                             int64_t n_points, int32_t method, double *f, double *mass,
                             void *stream);

/* ---- Learned second warp (App. I) ---------------------------------------
 * Learning: the library evaluates the order-n integrand f~ (exponential warp
 * with model_tau, charge mode, Jacobian included) at the 2^log2_m points of
 * one shifted lattice, or of one digitally shifted Sobol' sequence (the
 * sample App. I draws), on the GPU, projects |Re f~| onto each coordinate of
 * the unit cube with n_bins equal bins, smooths each projection with the
 * Gaussian kernel exp(-(w - w')^2 / lambda^2) over the bin centres,
 * normalises it to a density, mixes in the uniform density with weight
 * floor_eps (every bin keeps a positive weight) and stores the CDF at the bin
 * edges. */
typedef struct {
    int32_t order;          /* n, 1 .. QQMC_MAX_ORDER                         */
    int32_t log2_m;         /* learning sample M = 2^log2_m, 6 .. 24          */
    uint64_t lattice_a;     /* odd Korobov multiplier of the sample lattice
                               (not used with sobol_v)                        */
    const double *shift;    /* host, order doubles in [0, 1) (not used with
                               sobol_v)                                        */
    double model_tau;       /* first (exponential) warp, > 0                  */
    double t_meas;          /* 0 < t_meas <= table t_half                     */
    int32_t n_bins;         /* 1 .. 4096                                      */
    double lambda;          /* kernel width > 0                               */
    double floor_eps;       /* uniform weight in [0, 1]                       */
    double alpha;           /* interaction shift of the learned integrand, as
                               in qqmc_order                                   */
    const uint32_t *sobol_v;     /* host, order x 32 direction numbers as in
                                    qqmc_order, or NULL (lattice sample)      */
    const uint32_t *sobol_shift; /* host, order words: the sample's digital
                                    shift; set exactly when sobol_v is         */
} qqmc_learn_params;

/* Learns a model on the current device; synchronises `stream`.  EINVAL on
 * any out-of-range field, ENOMEM / EDEVICE on allocation or HIP failure. */
qqmc_status qqmc_learn_model(qqmc_tables t, const qqmc_learn_params *p,
                             void *stream, qqmc_model *out);

/* Wraps a caller-supplied model: cdf host, order x (n_bins + 1) row-major,
 * each row non-decreasing from 0 to 1 with positive bin widths (copied). */
qqmc_status qqmc_model_from_host(int32_t order, int32_t n_bins,
                                 const double *cdf, void *stream,
                                 qqmc_model *out);

/* Copies a model back: order and n_bins (either may be NULL), cdf host
 * order x (n_bins + 1) (may be NULL), hist host order x n_bins projected
 * sums of the learning sample, zeros for a model from the host (may be
 * NULL). */
qqmc_status qqmc_model_export(qqmc_model m, int32_t *order, int32_t *n_bins,
                              double *cdf, double *hist);

/* Releases the handle and its device memory.  NULL is ignored. */
void qqmc_free_model(qqmc_model m);

/* ---- Batched form -------------------------------------------------------
 * Many (parameter point, order) integrals in one persistent launch.  Each
 * item is estimated exactly as qqmc_eval_order_async estimates it at the
 * plan's tile_len (0: at each item's default; the same tile decomposition,
 * hence the same per-shift sums bit for bit, as long as every order keeps
 * its default lane mapping: see qqmc_plan_set_geometry).  The plan owns device buffers and a captured
 * HIP graph; qqmc_plan_run replays it. */
typedef struct {
    qqmc_tables tables;
    qqmc_order order;      /* shifts are copied at plan creation */
} qqmc_batch_item;

typedef struct qqmc_plan_s *qqmc_plan;

/* tile_len: lattice indices per tile (0 = autotuned, together with each
 * order's lane mapping where there is a choice); grid_blocks:
 * persistent workgroups per order-8 launch, scaled by residency for other
 * orders (0 = autotuned, which may also choose one workgroup per tile; then
 * qqmc_plan_info reports grid_blocks 0).  Items may mix the charge, the
 * model and constant modes, and the current (whose tables must hold lead
 * functions), on the lattice or on Sobol' points, with or without a learned
 * warp (not for the current). */
/* stream: the plan's own work (uploads, autotuning probes) is ordered after
 * everything queued on it so far, e.g. the tables' construction; replays and
 * result reads must come on streams ordered after the tables too. */
qqmc_status qqmc_plan_create(const qqmc_batch_item *items, int32_t n_items,
                             int32_t tile_len, int32_t grid_blocks,
                             void *stream, qqmc_plan *out);
/* Replays the launch on `stream` (asynchronous). */
qqmc_status qqmc_plan_run(qqmc_plan p, void *stream);
/* Synchronises `stream` and copies results: q_shift host, concatenated
 * 2*n_shifts(item) doubles per item in item order (divided by N). */
qqmc_status qqmc_plan_results(qqmc_plan p, void *stream, double *q_shift);
/* Number of tiles and of lattice points (all items, all shifts), the tile
 * length (0: each item at its own default tile length, the one
 * qqmc_eval_order takes when given 0) and the workgroup count, and the lane
 * mapping of each order n at
 * index n - 1 of two arrays of QQMC_MAX_ORDER entries (either may be NULL):
 * lanes_per_item, the lanes of one wavefront that evaluate one item
 * together (64 / lanes items share a wavefront), and top_levels, the
 * levels of the elimination tree that those lanes take cooperatively before
 * each walks its own path (an item is one of the 2^top_levels top-level
 * index prefixes of a point).  Reported for the plan's scalar-tree charge
 * group of that order if it has one, else its first group of that order;
 * 0 and 0 for orders the plan does not hold. */
qqmc_status qqmc_plan_info(qqmc_plan p, int64_t *n_tiles, int64_t *n_points,
                           int32_t *tile_len, int32_t *grid_blocks, int32_t *lanes_per_item,
                           int32_t *top_levels);
/* Lane mapping of the plan's scalar-tree charge group (lattice points, no
 * learned warp) of order `order` >= 5, which has two: the default, the one
 * qqmc_eval_order uses (a depth-5 register tree: 2^(n-5) lanes per point
 * up to order 10 with no top levels, 8 lanes per item and n - 8 top levels
 * above; at orders 5 and 6 a depth-4 tree, 2^(n-4) lanes per point, two
 * waves per SIMD), and a second one -- at orders 5 and 6 the depth-5 tree,
 * at orders 7, 8 and 11-14 a depth-4 register tree (twice the lanes per
 * item, compiled for two waves per SIMD), at orders 9 and 10 n - 8
 * cooperative top levels with 8 lanes per item.  The
 * mapping is named by its (lanes_per_item, top_levels) as qqmc_plan_info
 * reports them; the graph is captured again.  The two agree to rounding.
 * EINVAL if the plan has no such group or the order has no such mapping. */
qqmc_status qqmc_plan_set_geometry(qqmc_plan p, int32_t order, int32_t lanes_per_item,
                                   int32_t top_levels);
void qqmc_plan_destroy(qqmc_plan p);

/* ---- Serving ------------------------------------------------------------
 * A background scheduler admits requests while their device footprint fits
 * in hbm_budget_bytes and a slot is free, keeps tables and partial sums on
 * the device, and launches batches that mix the pending tiles of every
 * admitted request (continuous batching: requests that arrive while others
 * run join the next batch).  A request is cut into the tiles that
 * qqmc_eval_order uses by default (tile_len 0), and its per-shift sums are
 * the same, bit for bit, as those of qqmc_eval_order on the same input.
 * A launch first takes whole every admitted request that fits in a quarter
 * of its cost budget, then contiguous tile ranges of the oldest requests
 * (first come, first served). */
typedef struct qqmc_server_s *qqmc_server;

/* max_slots: requests resident at once; batch_tiles: tiles per launch
 * (0 = default).  Uses the current device and a stream of its own. */
qqmc_status qqmc_server_create(size_t hbm_budget_bytes, int32_t max_slots,
                               int32_t batch_tiles, qqmc_server *out);
/* Queues a request; never blocks on the GPU.  EADMIT if its footprint alone
 * exceeds hbm_budget_bytes; EINVAL as for qqmc_eval_order, and for the
 * current on a dot without a lead (dot.lead names the lead; the server
 * builds and caches its dot-lead functions).  Sobol' points are served as
 * the lattice is. */
qqmc_status qqmc_submit(qqmc_server s, const qqmc_dot *dot,
                        const qqmc_order *ord, uint64_t *ticket);
/* QQMC_PENDING until done; then fills the outputs (as qqmc_eval_order, each
 * may be NULL), t_submit_s / t_done_s on the server's monotonic clock, and
 * forgets the ticket (a second poll gives ENOTICKET). */
qqmc_status qqmc_poll(qqmc_server s, uint64_t ticket, double *q_shift,
                      double *q_mean, double *q_stderr, double *t_submit_s,
                      double *t_done_s);
/* Seconds on the server's clock (the clock of t_submit_s / t_done_s). */
double qqmc_server_now(qqmc_server s);
/* Blocks until every submitted request has finished. */
qqmc_status qqmc_server_drain(qqmc_server s);
void qqmc_server_destroy(qqmc_server s);

/* Message describing the last failure on the calling thread. */
const char *qqmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QQMC_H */
