/*
 * oracle.h -- plain FP64 CPU reference for TV-regularised parallel-beam tomography solved by
 * ProxSkip with the SVRG gradient estimator (ProxSVRGSkip).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no source, header, table or helper
 * with the HIP library: everything here is written out from the paper's definitions
 * (Sec. 1, Eq. 1-4; Algorithm 1 and its estimator table; Sec. 2.1, Eq. 5) and from the
 * published methods the paper cites (Beck & Teboulle's FGP; Joseph interpolation; SplitMix64).
 *
 * Precision: every floating-point value is IEEE double, built with -ffp-contract=off and no
 * fast-math.  OpenMP is used only over output elements: every output element is accumulated by
 * one thread in a fixed serial order, so results do not depend on the thread count.
 *
 * Conventions (where the paper leaves a point open, the reading taken is stated here):
 *   image x:     [nz][ny][nx] row-major, pixel (i, j) centre at (j - (nx-1)/2, i - (ny-1)/2),
 *                unit pixels; slices are independent for the projector (rotation axis = z).
 *   angles:      theta_k = k*pi/A unless an explicit table is given.
 *   detector:    bin centre s_u = (u - (B-1)/2)*du + off; ray (k, u) = {x cos + y sin = s_u}.
 *   sinogram:    [nz][A][B]; subset i holds angles {i, i+N, i+2N, ...} (interleaved, Sec. 2.1 and
 *                the data-splitting figure), stored as [nz][a_i][B] with its angles in order.
 *   dual field:  [d][nz][ny][nx], d = 2 for nz == 1 and d = 3 otherwise (3D TV couples slices).
 *
 * Parity pins: see tests/test_oracle_*.py.  The paper prints no iterate value.  The loop is
 * pinned by the algorithm's reductions (p = 1 is proximal gradient; prox = identity gives plain
 * SVRG descent) and, at p < 1 with a non-trivial prox, by its fixed point (x -> x* of the
 * reference method, h -> grad f(x*)); FGP at a finite number of inner iterations is pinned by
 * trajectories derived by hand on two- and four-pixel images.
 */
#ifndef PROXSKIP_ORACLE_H
#define PROXSKIP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny, nz;       /* image columns, rows, slices                                  */
    int n_angles;         /* A                                                            */
    int n_bins;           /* B                                                            */
    int n_subsets;        /* N >= 1                                                       */
    double du;            /* detector bin width in pixel units                            */
    double off;           /* detector centre offset in pixel units                        */
    const double *angles; /* optional table of A angles (radians); NULL => k*pi/A         */
} orc_geom;

typedef struct {
    int epochs_done, iters_done, prox_calls;
    double last_rel_change;
} orc_stats;

/* Number of angles in subset i (i = -1: all A angles). */
int orc_subset_size(const orc_geom *g, int subset);

/* Discrete Radon transform by Joseph interpolation (Sec. 2.1: "discrete Radon transform").
 * y[nz][a_i][B] = A_i x (subset = -1: all angles, y = [nz][A][B]). */
void orc_project(const orc_geom *g, int subset, const double *x, double *y);

/* Exact transpose of orc_project: x = A_i^T y (overwrites x). */
void orc_backproject(const orc_geom *g, int subset, const double *y, double *x);

/* Single rays of the full operator, for sampled checks at large sizes:
 * out[r] = (A x)(slice zs[r], angle ks[r], bin us[r]). */
void orc_project_rays(const orc_geom *g, const double *x, int n_rays, const int *zs,
                      const int *ks, const int *us, double *out);

/* Single pixels of A_i^T y by brute force over every ray of the subset:
 * out[r] = (A_i^T y)(zs[r], is[r], js[r]). */
void orc_backproject_pixels(const orc_geom *g, int subset, const double *y, int n_px,
                            const int *zs, const int *is, const int *js, double *out);

/* Subset gradient of f_i(x) = 1/2 ||A_i x - b_i||^2: out = A_i^T (A_i x - b_i); b is [nz][A][B]. */
void orc_grad_subset(const orc_geom *g, int subset, const double *x, const double *b, double *out);

/* Full gradient  grad f(x) = sum_{i=0}^{N-1} grad f_i(x), summed in increasing i. */
void orc_grad_full(const orc_geom *g, const double *x, const double *b, double *out);

/* f(x) = sum_i 1/2 ||A_i x - b_i||^2. */
double orc_data_fit(const orc_geom *g, const double *x, const double *b);

/* Lipschitz constant of grad f: L = lambda_max(A^T A) by the power method from the all-ones
 * vector; returns the final Rayleigh quotient. */
double orc_lipschitz(const orc_geom *g, int iters);

/* Isotropic TV (forward differences, Neumann boundary; 3-component when nz > 1). */
double orc_tv(int nx, int ny, int nz, const double *z);

/* z = prox_{tau (TV + I_C)}(v) by FGP (Beck & Teboulle 2009) with n_inner iterations, C = {z >= 0}
 * when nonneg != 0, else R^n.  dual: [d][nz][ny][nx] warm start in, final dual out; NULL =>
 * cold start, not returned.  tau == 0 => z = P_C(v) and the dual is untouched.  z may alias v. */
void orc_tv_prox_fgp(int nx, int ny, int nz, const double *v, double *z, double tau, int n_inner,
                     int nonneg, double *dual);

/* Unaccelerated dual projected gradient for the same prox (an independent solver, used only to
 * pin FGP).  Same conventions as orc_tv_prox_fgp. */
void orc_tv_prox_dpg(int nx, int ny, int nz, const double *v, double *z, double tau, int n_iter,
                     int nonneg, double *dual);

/* Counter-based SplitMix64 streams (Steele, Lea & Flood 2014):
 *   u(seed, j) = mix64(seed + (j + 1) * 0x9e3779b97f4a7c15)
 *   subset i_k = ((u(seed, 2k) >> 32) * N) >> 32
 *   coin theta_k = (u(seed, 2k+1) >> 11) < floor(p * 2^53)
 * for k = k0 .. k0 + count - 1. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t j);
void orc_sequences(uint64_t seed, int64_t k0, int64_t count, int n_subsets, double p,
                   int32_t *subset_out, uint8_t *coin_out);

/* ProxSkip (Algorithm 1) with the SVRG estimator, literal form:
 *   snapshot every N iterations (k mod N == 0): xs = x, gs = grad f(xs)
 *   G  = N (grad f_i(x) - grad f_i(xs)) + gs
 *   xh = x - gamma (G - h)
 *   theta = 1: x+ = prox_{(gamma/p) g}(xh - (gamma/p) h)  with g = alpha TV + I_C
 *   theta = 0: x+ = xh
 *   h+ = h + (p/gamma)(x+ - xh)
 * plain != 0 runs non-skipped ProxSVRG instead: x+ = prox_{gamma g}(x - gamma G), h untouched.
 * x, h, dual: in/out.  k0: first iteration index (a multiple of N).  tol > 0 stops at the first
 * epoch end whose relative change ||x_e - x_{e-1}|| / ||x_e|| is below tol.
 * rel_change_out (may be NULL) receives one value per completed epoch.
 * Returns 0, or -1 on invalid arguments. */
int orc_proxskip_svrg(const orc_geom *g, const double *b, double *x, double *h, double *dual,
                      double gamma, double p, double alpha, int fgp_inner, int nonneg,
                      int n_epochs, int plain, uint64_t seed, int64_t k0, double tol,
                      orc_stats *stats, double *rel_change_out);

/* Refresh coins of the loopless SVRG estimator (Sec. 1.2: the full gradient is refreshed with
 * probability 1/N in every iteration):
 *   rho_k = (u(seed, 2^62 + k) >> 11) < floor(2^53 / N)      (integer division)
 * for k = k0 .. k0 + count - 1.  The counters 2^62 + k never meet the subset and coin counters
 * 2k and 2k + 1 while k < 2^61. */
void orc_refresh_coins(uint64_t seed, int64_t k0, int64_t count, int n_subsets, uint8_t *out);

/* Gradient estimators of the table beside Algorithm 1 (Sec. 1.2). */
enum { ORC_SVRG = 0, ORC_LSVRG = 1, ORC_SAGA = 2 };

/* Algorithm 1 with estimator G_k:
 *   ORC_SVRG   G = N (grad f_i(x) - grad f_i(xs)) + grad f(xs), snapshot xs = x and
 *              grad f(xs) refreshed at every k with k mod N == 0;
 *   ORC_LSVRG  the same G, the snapshot refreshed at the run's first iteration and at every
 *              later k with refresh[t] = 1 (before G_k is formed, so G_k = grad f(x_k) there);
 *   ORC_SAGA   G = N (grad f_i(x) - v_i) + vbar, then vbar += grad f_i(x) - v_i and
 *              v_i = grad f_i(x) (Eq. 4); at the run's first iteration the table is filled with
 *              v_i = grad f_i(x) for every i and vbar = sum_i v_i (increasing i).
 * then xh = x - gamma (G - h); theta = coin[t]: x+ = prox_{(gamma/p) g}(xh - (gamma/p) h) or
 * x+ = xh; h+ = h + (p/gamma)(x+ - xh).  plain != 0: x+ = prox_{gamma g}(x - gamma G), h unused.
 * The random draws are inputs: sub[t], coin[t], refresh[t] for iteration k = k0 + t,
 * t = 0 .. n_iters - 1 (refresh may be NULL unless ORC_LSVRG; coin may be NULL when plain).
 * Epochs are the N-iteration blocks from k0 (k0 a multiple of N); at each epoch end the relative
 * change ||x_e - x_{e-1}|| / ||x_e|| goes to rel_change_out (may be NULL) and, with tol > 0, the
 * run stops at the first epoch end below tol.  table (N * n) and table_sum (n) receive the SAGA
 * state when not NULL.  Returns 0, or -1 on invalid arguments. */
int orc_proxskip(const orc_geom *g, const double *b, double *x, double *h, double *dual,
                 double gamma, double p, double alpha, int fgp_inner, int nonneg, int plain,
                 int estimator, int64_t k0, int64_t n_iters, const int32_t *sub,
                 const uint8_t *coin, const uint8_t *refresh, double tol, orc_stats *stats,
                 double *rel_change_out, double *table, double *table_sum);

/* FISTA (Beck & Teboulle 2009; the table beside Algorithm 1: ISTA with an acceleration step):
 *   x_{k+1} = prox_{gamma g}(y_k - gamma grad f(y_k)),  t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
 *   y_{k+1} = x_{k+1} + ((t_k - 1) / t_{k+1}) (x_{k+1} - x_k),   y_0 = x_0,  t_0 = 1,
 * g = alpha TV + I_C with the prox by FGP (fgp_inner warm-started iterations, dual in/out).
 * x: in x_0, out x_K.  fval_out (may be NULL) receives f(x_{k+1}) + alpha TV(x_{k+1}) for
 * k = 0 .. n_iters - 1.  Returns 0, or -1 on invalid arguments. */
int orc_fista(const orc_geom *g, const double *b, double *x, double *dual, double gamma,
              double alpha, int fgp_inner, int nonneg, int n_iters, double *fval_out);

/* High-accuracy reference x* (Sec. 2.1: "a separate primal-dual proximal method", the
 * data-splitting figure: PDHG with diagonal preconditioning, Chambolle & Pock 2011) for
 * Eq. 5, min_x 1/2 ||Ax - b||^2 + alpha TV(x) + I_C(x), written as min F(Kx) + G(x) with
 * K = [A; D], F(u, w) = 1/2 ||u - b||^2 + alpha sum_pixels ||w_pixel||_2, G = I_C:
 *   tau_j   = 1 / (sum_i |A_ij| + sum_i |D_ij|)     (column sums of |K|)
 *   sigma_i = 1 / sum_j |A_ij|  (1 where the row is zero),   sigma_D = 1/2  (row sums of |D|)
 *   x+   = P_C(x - tau (A^T y1 + D^T y2));   xbar = 2 x+ - x
 *   y1+  = (y1 + sigma (A xbar - b)) / (1 + sigma)               (prox of F1*)
 *   y2+  = each pixel's d-vector of y2 + sigma_D D xbar scaled onto the ball of radius alpha
 * x [nz][ny][nx], y1 [nz][A][B], y2 [d][nz][ny][nx]: in/out (zeros for a fresh start).
 * Returns 0, or -1 on invalid arguments. */
int orc_pdhg(const orc_geom *g, const double *b, double *x, double *y1, double *y2, double alpha,
             int nonneg, int n_iters);

/* Threads the OpenMP runtime will use (for reporting), and a new count for later calls (for
 * timing; every result is independent of the thread count: each output element is summed by one
 * thread in a fixed order). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
