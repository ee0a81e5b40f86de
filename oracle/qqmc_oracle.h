/*
 * qqmc_oracle.h -- CPU FP64 oracle for the quantum quasi-Monte Carlo (QQMC)
 * charge integrand of arXiv:2002.12372 (Macek, Dumitrescu, Bertrand, Triggs,
 * Parcollet, Waintal).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plainly written
 * reference against which the GPU path is checked.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  The product
 * library never links, loads or calls it, and it shares no code with the
 * product (no headers, helpers, tables or constants).
 *
 * Everything is IEEE double / double complex.  Every function names the
 * passage of the paper it writes out.  Readings of passages the paper leaves
 * open are listed next to the function that takes them.
 */
#ifndef QQMC_ORACLE_H
#define QQMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Non-interacting dot Green's functions on a uniform time grid
 * (App. E "Model" and Eq. (lesser_greater_freq), wide-band limit).
 * Grid: tau_j = -t_half + j*h, h = 2*t_half/(n_grid-1), j = 0..n_grid-1.
 * gl, gg: 2*n_grid doubles each (re, im interleaved) receiving g^<(tau_j)
 * and g^>(tau_j).  n_sigma receives the occupation per spin, so that
 * g^<(0) = i*n_sigma.  Returns 0 on success, -1 on bad arguments. */
int oracle_tables(double eps_d, double gamma, double beta, double bias_v,
                  int n_grid, double t_half,
                  double *gl, double *gg, double *n_sigma);

/* Occupation per spin n_sigma (the tau = 0 value of -i g^<). */
double oracle_n_sigma(double eps_d, double gamma, double beta, double bias_v);

/* g^<(tau) and g^>(tau) evaluated directly from the residue series (no grid),
 * out[0..3] = (re g<, im g<, re g>, im g>).  Used by the table pins. */
void oracle_gf_direct(double eps_d, double gamma, double beta, double bias_v,
                      double tau, double *out);

/* Linear interpolation in a table built as above; out = (re, im). */
double oracle_n_sigma_band(double eps_d, double gamma, double beta, double bias_v, double D);

void oracle_gf_band(double eps_d, double gamma, double beta, double bias_v, double D,
                    double tau, double *out);

int oracle_tables_band(double eps_d, double gamma, double beta, double bias_v, double D,
                       int n_grid, double t_half, double *gl, double *gg, double *n_sigma);

void oracle_interp(const double *tab, int n_grid, double t_half, double tau,
                   double *out);

/* Determinant of a dense complex m x m matrix a (row-major, re/im
 * interleaved), by LU factorisation with partial pivoting. out = (re, im). */
void oracle_det(int m, const double *a, double *out);

/* The (n+1)x(n+1) Wick matrix of Eq. (integral_gf) for Keldysh indices
 * a[0..n-1] (each 0 or 1), in the paper's order: row/column 0 is the
 * measurement point, rows/columns 1..n are the vertices U_1..U_n.  The
 * n x n spin-down matrix is its lower-right block.  out: 2*(n+1)^2 doubles. */
void oracle_wick_matrix(const double *gl, const double *gg, int n_grid,
                        double t_half, double n_sigma, double alpha, double t_meas,
                        int n, const double *u, const int *a, double *out);

/* Keldysh sum S(u) = sum_a (-1)^{sum a} det_up(a) det_dn(a) over all 2^n
 * index vectors (Eq. (integral_gf)), and the term mass
 * M(u) = sum_a |det_up(a) det_dn(a)|.  u[0..n-1] = (u_1..u_n), any order.
 * S_out = (re, im). */
void oracle_keldysh_sum(const double *gl, const double *gg, int n_grid,
                        double t_half, double n_sigma, double alpha, double t_meas,
                        int n, const double *u, double *S_out, double *M_out);

/* Rank-1 (Korobov) lattice point with a random shift:
 * x_j = frac(((i * z_j) mod N)/N + shift_j), z_j = a^j mod N. */
void oracle_lattice_point(uint64_t i, int n, int log2_n, uint64_t lattice_a,
                          const double *shift, double *x);

/* Product-model warping with h(v) = exp(-v/tau) (Eqs. (warper1d),
 * (x_of_v_simple), (hi_expo)).  Gives u[0..n-1] = (u_1..u_n) and the weight
 * W = C/p_n(u) with C = tau^n.  Returns 1 if 0 < u_n (point inside the
 * integration domain), 0 otherwise. */
int oracle_warp(int n, const double *x, double model_tau, double t_meas,
                double *u, double *W);

/* Sums over lattice indices i in [i_begin, i_end) of the warped integrand for
 * each of n_shifts shifts (Eq. (warped_int2)): sums[2*s..2*s+1] receives
 * sum_i fbar_{i,s} (not yet divided by N).  mode 0: charge integrand
 * -2 i^{n+1} S(u) W; mode 1: the model function itself (f := p_n, no domain
 * cut, every sample equals C); mode 2: f := 1 on the ordered simplex.
 * n_threads <= 0 uses all OpenMP threads.  Returns 0, or -1 on bad args. */
int oracle_eval_sums(const double *gl, const double *gg, int n_grid,
                     double t_half, double n_sigma, double alpha, double t_meas,
                     int n, int log2_n, uint64_t lattice_a,
                     int n_shifts, const double *shifts, double model_tau,
                     int mode, int64_t i_begin, int64_t i_end, int n_threads,
                     double *sums);

/* Number of OpenMP threads the oracle would use for n_threads <= 0. */
int oracle_eval_mass(const double *gl, const double *gg, int n_grid,
                     double t_half, double n_sigma, double alpha, double t_meas,
                     int n, int log2_n, uint64_t lattice_a,
                     int n_shifts, const double *shifts, double model_tau,
                     int64_t i_begin, int64_t i_end, int n_threads, double *mass);

void oracle_gf_lead(double eps_d, double gamma, double beta, double bias_v, double D, int lead,
                    double tau, double *out);

int oracle_lead_tables(double eps_d, double gamma, double beta, double bias_v, double D,
                       int lead, int n_grid, double t_half, double *cl, double *cg);

void oracle_keldysh_sum_lead(const double *gl, const double *gg, const double *cl,
                             const double *cg, int n_grid, double t_half, double n_sigma,
                             double alpha, double t_meas, int n, const double *u,
                             double *S_out, double *M_out);

int oracle_eval_sums_lead(const double *gl, const double *gg, const double *cl,
                          const double *cg, int n_grid, double t_half, double n_sigma,
                          double alpha, double t_meas, int n, int log2_n, uint64_t lattice_a,
                          int n_shifts, const double *shifts, double model_tau,
                          int64_t i_begin, int64_t i_end, int n_threads, double *sums,
                          double *mass);

void oracle_sobol_point(uint64_t i, int n, const uint32_t *V, const uint32_t *dshift, double *x);

int oracle_eval_sums_sobol(const double *gl, const double *gg, int n_grid,
                           double t_half, double n_sigma, double alpha, double t_meas,
                           int n, const uint32_t *sobol_v, int n_shifts,
                           const uint32_t *sobol_shifts, double model_tau,
                           const double *cdf, int n_bins, int mode,
                           int64_t i_begin, int64_t i_end, int n_threads, double *sums);

int oracle_max_threads(void);

/* ---- Learned second warp (App. I, "Learning h^(i) from the integrand") ----
 * After the exponential warp the integrand over the unit cube is
 * f~(w) = fbar(u(w)) (Jacobian C/p_n included).  The second warp maps a
 * lattice point x to w coordinate by coordinate through the inverse CDF of a
 * density q_j on [0, 1), piecewise constant on n_bins equal bins; the weight
 * gains a factor 1/prod_j q_j(w_j).  A model is stored as its CDF at the bin
 * edges, cdf[j*(n_bins+1) + b], b = 0..n_bins, cdf[...0] = 0, cdf[...n_bins]
 * = 1.
 *
 * Readings (the appendix leaves them open): the projection bins |Re f~|
 * (a density must be non-negative; Q_n is real); bins are [b, b+1)/n_bins
 * with centres (b + 1/2)/n_bins, where the kernel smoothing is evaluated;
 * the smoothed projection is normalised to a density p_j and mixed with the
 * uniform density, q_j = (1 - floor_eps) p_j + floor_eps, so every bin keeps
 * a positive weight; an empty projection gives the uniform density. */

/* Learns a model from the lattice points i < 2^log2_m of one shift (the
 * exponential warp with model_tau as the first warp, the charge integrand of
 * mode 0): hist (n*n_bins, may be NULL) receives the projected |Re f~| sums
 * per coordinate and bin, cdf (n*(n_bins+1)) the model.  Returns 0, or -1 on
 * bad arguments. */
int oracle_learn_model(const double *gl, const double *gg, int n_grid,
                       double t_half, double n_sigma, double alpha, double t_meas,
                       int n, int log2_m, uint64_t lattice_a,
                       const double *shift, double model_tau, int n_bins,
                       double lambda, double floor_eps, int n_threads,
                       double *hist, double *cdf);

/* The same learning pass over the Sobol' points i < 2^log2_m (App. I samples
 * the cube with Sobol' points): sobol_v n x 32 direction numbers, dshift n
 * words of one digital shift. */
int oracle_learn_model_sobol(const double *gl, const double *gg, int n_grid,
                             double t_half, double n_sigma, double alpha, double t_meas,
                             int n, int log2_m, const uint32_t *sobol_v,
                             const uint32_t *dshift, double model_tau, int n_bins,
                             double lambda, double floor_eps, int n_threads,
                             double *hist, double *cdf);

/* Builds a model from given per-coordinate projections (n*n_bins values):
 * smoothing, normalisation, floor and CDF as in oracle_learn_model. */
int oracle_model_from_hist(int n, int n_bins, const double *hist, double lambda,
                           double floor_eps, double *cdf);

/* Inverse CDF of one coordinate: w = F^{-1}(x) for x in [0, 1); returns the
 * density q(w).  The bin is the last b with cdf[b] <= x. */
double oracle_model_inverse(const double *cdf, int n_bins, double x, double *w);

/* oracle_eval_sums with the learned second warp in front of the exponential
 * one (cdf == NULL: none, identical to oracle_eval_sums).  In mode 1 the
 * model function is the combined one, p_n(u) prod_j q_j(w_j), so every sample
 * still equals C. */
int oracle_eval_sums_model(const double *gl, const double *gg, int n_grid,
                           double t_half, double n_sigma, double alpha, double t_meas,
                           int n, int log2_n, uint64_t lattice_a,
                           int n_shifts, const double *shifts, double model_tau,
                           const double *cdf, int n_bins,
                           int mode, int64_t i_begin, int64_t i_end, int n_threads,
                           double *sums);

#ifdef __cplusplus
}
#endif
#endif
