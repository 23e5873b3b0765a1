/*
 * oracle.c -- plain FP64 CPU reference (test infrastructure only; see oracle.h).
 *
 * Every routine follows a definition written out in the paper or in the published method it
 * cites, in the order that definition states it.  No blocking, fusion or reordering beyond
 * that: the only parallelism is an OpenMP loop over independent output elements.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------------------------ */
/* Geometry: angles, subsets, detector bins.                                                   */
/* ------------------------------------------------------------------------------------------ */

static double angle_of(const orc_geom *g, int k)
{
    /* Uniform angles on [0, pi) unless a table is given. */
    return g->angles ? g->angles[k] : (double)k * M_PI / (double)g->n_angles;
}

int orc_subset_size(const orc_geom *g, int subset)
{
    if (subset < 0) return g->n_angles;
    /* Interleaved split (Sec. 2.1, data-splitting figure): subset i = {i, i+N, i+2N, ...}. */
    if (subset >= g->n_angles) return 0;
    return (g->n_angles - 1 - subset) / g->n_subsets + 1;
}

static int subset_angle(const orc_geom *g, int subset, int l)
{
    return subset < 0 ? l : subset + l * g->n_subsets;
}

static double bin_centre(const orc_geom *g, int u)
{
    return ((double)u - (g->n_bins - 1) / 2.0) * g->du + g->off;
}

/* Threads only pay off above some work size (small cases run serially; results are the same). */
static int par_worth(const orc_geom *g, int na)
{
    return (double)g->nz * na * g->n_bins * (g->nx > g->ny ? g->nx : g->ny) > 2.0e6;
}

/* Pixel value with zero outside the image. */
static double pix(const orc_geom *g, const double *xs, int i, int j)
{
    if (i < 0 || i >= g->ny || j < 0 || j >= g->nx) return 0.0;
    return xs[(size_t)i * g->nx + j];
}

/* ------------------------------------------------------------------------------------------ */
/* Joseph projector (discrete Radon transform, Sec. 2.1).                                      */
/*   The ray {x cos t + y sin t = s} is walked one pixel row at a time when |cos t| >= |sin t|  */
/*   (else one column at a time).  At each row the image is linearly interpolated between the  */
/*   two nearest pixel centres of that row, and the sum is scaled by the path length per row,   */
/*   1/|cos t| (1/|sin t| for columns).  Samples outside the image are zero.                     */
/* ------------------------------------------------------------------------------------------ */

static double ray_sum(const orc_geom *g, const double *xs, int k, int u)
{
    const int nx = g->nx, ny = g->ny;
    const double th = angle_of(g, k);
    const double c = cos(th), s = sin(th);
    const double su = bin_centre(g, u);
    double acc = 0.0;
    if (fabs(c) >= fabs(s)) {
        for (int i = 0; i < ny; ++i) {
            const double yi = i - (ny - 1) / 2.0;
            const double q = (su - yi * s) / c + (nx - 1) / 2.0; /* fractional column */
            const double fl = floor(q);
            const int j0 = (int)fl;
            const double w = q - fl;
            acc += (1.0 - w) * pix(g, xs, i, j0) + w * pix(g, xs, i, j0 + 1);
        }
        return acc / fabs(c);
    } else {
        for (int j = 0; j < nx; ++j) {
            const double xj = j - (nx - 1) / 2.0;
            const double q = (su - xj * c) / s + (ny - 1) / 2.0; /* fractional row */
            const double fl = floor(q);
            const int i0 = (int)fl;
            const double w = q - fl;
            acc += (1.0 - w) * pix(g, xs, i0, j) + w * pix(g, xs, i0 + 1, j);
        }
        return acc / fabs(s);
    }
}

void orc_project(const orc_geom *g, int subset, const double *x, double *y)
{
    const int na = orc_subset_size(g, subset);
    const int B = g->n_bins;
    const size_t n_img = (size_t)g->nx * g->ny;
#pragma omp parallel for collapse(3) schedule(static) if (par_worth(g, na))
    for (int z = 0; z < g->nz; ++z)
        for (int l = 0; l < na; ++l)
            for (int u = 0; u < B; ++u) {
                const int k = subset_angle(g, subset, l);
                y[((size_t)z * na + l) * B + u] = ray_sum(g, x + (size_t)z * n_img, k, u);
            }
}

void orc_project_rays(const orc_geom *g, const double *x, int n_rays, const int *zs,
                      const int *ks, const int *us, double *out)
{
    const size_t n_img = (size_t)g->nx * g->ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_rays; ++r)
        out[r] = ray_sum(g, x + (size_t)zs[r] * n_img, ks[r], us[r]);
}

/* Adjoint: the same loops as ray_sum with the assignment reversed (a scatter), so that it is
 * the transpose of the projector by construction.  A row-walked ray only touches its own row,
 * and a column-walked ray its own column, so the scatter is split into a pass over rows (for
 * the row-walked angles) and a pass over columns (for the column-walked ones); each output pixel
 * is then accumulated by a single thread, in angle order then bin order. */
void orc_backproject(const orc_geom *g, int subset, const double *y, double *x)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz, B = g->n_bins;
    const int na = orc_subset_size(g, subset);
    const size_t n_img = (size_t)nx * ny;
    memset(x, 0, sizeof(double) * n_img * nz);

#pragma omp parallel for collapse(2) schedule(static) if (par_worth(g, na))
    for (int z = 0; z < nz; ++z)
        for (int i = 0; i < ny; ++i) {
            double *row = x + (size_t)z * n_img + (size_t)i * nx;
            const double yi = i - (ny - 1) / 2.0;
            for (int l = 0; l < na; ++l) {
                const int k = subset_angle(g, subset, l);
                const double th = angle_of(g, k), c = cos(th), s = sin(th);
                if (!(fabs(c) >= fabs(s))) continue;
                const double *yl = y + ((size_t)z * na + l) * B;
                for (int u = 0; u < B; ++u) {
                    const double su = bin_centre(g, u);
                    const double q = (su - yi * s) / c + (nx - 1) / 2.0;
                    const double fl = floor(q);
                    const int j0 = (int)fl;
                    const double w = q - fl;
                    const double val = yl[u] / fabs(c);
                    if (j0 >= 0 && j0 < nx) row[j0] += (1.0 - w) * val;
                    if (j0 + 1 >= 0 && j0 + 1 < nx) row[j0 + 1] += w * val;
                }
            }
        }

#pragma omp parallel for collapse(2) schedule(static) if (par_worth(g, na))
    for (int z = 0; z < nz; ++z)
        for (int j = 0; j < nx; ++j) {
            double *img = x + (size_t)z * n_img;
            const double xj = j - (nx - 1) / 2.0;
            for (int l = 0; l < na; ++l) {
                const int k = subset_angle(g, subset, l);
                const double th = angle_of(g, k), c = cos(th), s = sin(th);
                if (fabs(c) >= fabs(s)) continue;
                const double *yl = y + ((size_t)z * na + l) * B;
                for (int u = 0; u < B; ++u) {
                    const double su = bin_centre(g, u);
                    const double q = (su - xj * c) / s + (ny - 1) / 2.0;
                    const double fl = floor(q);
                    const int i0 = (int)fl;
                    const double w = q - fl;
                    const double val = yl[u] / fabs(s);
                    if (i0 >= 0 && i0 < ny) img[(size_t)i0 * nx + j] += (1.0 - w) * val;
                    if (i0 + 1 >= 0 && i0 + 1 < ny) img[(size_t)(i0 + 1) * nx + j] += w * val;
                }
            }
        }
}

/* One pixel of A_i^T y by brute force over every ray of the subset: the weight of pixel (i, j)
 * in ray (k, u) is read off the projector's own interpolation at that row (column). */
void orc_backproject_pixels(const orc_geom *g, int subset, const double *y, int n_px,
                            const int *zs, const int *is, const int *js, double *out)
{
    const int nx = g->nx, ny = g->ny, B = g->n_bins;
    const int na = orc_subset_size(g, subset);
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_px; ++r) {
        const int z = zs[r], i = is[r], j = js[r];
        double acc = 0.0;
        for (int l = 0; l < na; ++l) {
            const int k = subset_angle(g, subset, l);
            const double th = angle_of(g, k), c = cos(th), s = sin(th);
            const double *yl = y + ((size_t)z * na + l) * B;
            for (int u = 0; u < B; ++u) {
                const double su = bin_centre(g, u);
                if (fabs(c) >= fabs(s)) {
                    const double yi = i - (ny - 1) / 2.0;
                    const double q = (su - yi * s) / c + (nx - 1) / 2.0;
                    const double fl = floor(q);
                    const int j0 = (int)fl;
                    const double w = q - fl;
                    const double val = yl[u] / fabs(c);
                    if (j0 == j) acc += (1.0 - w) * val;
                    if (j0 + 1 == j) acc += w * val;
                } else {
                    const double xj = j - (nx - 1) / 2.0;
                    const double q = (su - xj * c) / s + (ny - 1) / 2.0;
                    const double fl = floor(q);
                    const int i0 = (int)fl;
                    const double w = q - fl;
                    const double val = yl[u] / fabs(s);
                    if (i0 == i) acc += (1.0 - w) * val;
                    if (i0 + 1 == i) acc += w * val;
                }
            }
        }
        out[r] = acc;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Data fit f(x) = sum_i 1/2 ||A_i x - b_i||^2 and its gradients (Sec. 2.1).                   */
/* ------------------------------------------------------------------------------------------ */

static double *alloc_d(size_t n)
{
    double *p = (double *)calloc(n ? n : 1, sizeof(double));
    if (!p) abort();
    return p;
}

/* r = A_i x - b_i, with b_i gathered from the full sinogram b [nz][A][B]. */
static void subset_residual(const orc_geom *g, int subset, const double *x, const double *b,
                            double *r)
{
    const int na = orc_subset_size(g, subset), B = g->n_bins, A = g->n_angles;
    orc_project(g, subset, x, r);
    for (int z = 0; z < g->nz; ++z)
        for (int l = 0; l < na; ++l) {
            const int k = subset_angle(g, subset, l);
            for (int u = 0; u < B; ++u)
                r[((size_t)z * na + l) * B + u] -= b[((size_t)z * A + k) * B + u];
        }
}

void orc_grad_subset(const orc_geom *g, int subset, const double *x, const double *b, double *out)
{
    const int na = orc_subset_size(g, subset);
    double *r = alloc_d((size_t)g->nz * na * g->n_bins);
    subset_residual(g, subset, x, b, r);
    orc_backproject(g, subset, r, out);
    free(r);
}

void orc_grad_full(const orc_geom *g, const double *x, const double *b, double *out)
{
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    double *gi = alloc_d(n);
    memset(out, 0, sizeof(double) * n);
    for (int i = 0; i < g->n_subsets; ++i) {
        orc_grad_subset(g, i, x, b, gi);
        for (size_t e = 0; e < n; ++e) out[e] += gi[e];
    }
    free(gi);
}

double orc_data_fit(const orc_geom *g, const double *x, const double *b)
{
    double f = 0.0;
    for (int i = 0; i < g->n_subsets; ++i) {
        const int na = orc_subset_size(g, i);
        const size_t m = (size_t)g->nz * na * g->n_bins;
        double *r = alloc_d(m);
        subset_residual(g, i, x, b, r);
        double s = 0.0;
        for (size_t e = 0; e < m; ++e) s += r[e] * r[e];
        f += 0.5 * s;
        free(r);
    }
    return f;
}

double orc_lipschitz(const orc_geom *g, int iters)
{
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    const size_t m = (size_t)g->nz * g->n_angles * g->n_bins;
    double *v = alloc_d(n), *w = alloc_d(n), *y = alloc_d(m);
    for (size_t e = 0; e < n; ++e) v[e] = 1.0 / sqrt((double)n);
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        orc_project(g, -1, v, y);
        orc_backproject(g, -1, y, w); /* w = A^T A v */
        double vw = 0.0, ww = 0.0;
        for (size_t e = 0; e < n; ++e) { vw += v[e] * w[e]; ww += w[e] * w[e]; }
        lam = vw; /* Rayleigh quotient, ||v|| = 1 */
        const double nrm = sqrt(ww);
        if (nrm == 0.0) break;
        for (size_t e = 0; e < n; ++e) v[e] = w[e] / nrm;
    }
    free(v); free(w); free(y);
    return lam;
}

/* ------------------------------------------------------------------------------------------ */
/* Isotropic TV and its proximal operator (Sec. 2.1, Eq. 5; FGP of Beck & Teboulle 2009).      */
/*   D: forward differences with a zero last difference (Neumann boundary).                     */
/*   D^T: its exact adjoint.  ||D||^2 <= 4 d.                                                    */
/* ------------------------------------------------------------------------------------------ */

typedef struct { int nx, ny, nz, d; size_t n; } grid;

static grid make_grid(int nx, int ny, int nz)
{
    grid G = {nx, ny, nz, nz > 1 ? 3 : 2, (size_t)nx * ny * nz};
    return G;
}

/* p = D z ; p is [d][n]. */
static void op_D(const grid *G, const double *z, double *p)
{
    const int nx = G->nx, ny = G->ny, nz = G->nz;
#pragma omp parallel for collapse(2) schedule(static) if (G->n > 65536)
    for (int zz = 0; zz < nz; ++zz)
        for (int i = 0; i < ny; ++i)
            for (int j = 0; j < nx; ++j) {
                const size_t e = ((size_t)zz * ny + i) * nx + j;
                p[e] = (j < nx - 1) ? z[e + 1] - z[e] : 0.0;
                p[G->n + e] = (i < ny - 1) ? z[e + nx] - z[e] : 0.0;
                if (G->d == 3) p[2 * G->n + e] = (zz < nz - 1) ? z[e + (size_t)nx * ny] - z[e] : 0.0;
            }
}

/* out = D^T p. */
static void op_DT(const grid *G, const double *p, double *out)
{
    const int nx = G->nx, ny = G->ny, nz = G->nz;
    const size_t plane = (size_t)nx * ny;
#pragma omp parallel for collapse(2) schedule(static) if (G->n > 65536)
    for (int zz = 0; zz < nz; ++zz)
        for (int i = 0; i < ny; ++i)
            for (int j = 0; j < nx; ++j) {
                const size_t e = ((size_t)zz * ny + i) * nx + j;
                const double *px = p, *py = p + G->n;
                double tx = (j > 0 ? px[e - 1] : 0.0) - (j < nx - 1 ? px[e] : 0.0);
                double ty = (i > 0 ? py[e - nx] : 0.0) - (i < ny - 1 ? py[e] : 0.0);
                double t = tx + ty;
                if (G->d == 3) {
                    const double *pz = p + 2 * G->n;
                    t += (zz > 0 ? pz[e - plane] : 0.0) - (zz < nz - 1 ? pz[e] : 0.0);
                }
                out[e] = t;
            }
}

double orc_tv(int nx, int ny, int nz, const double *z)
{
    grid G = make_grid(nx, ny, nz);
    double *p = alloc_d(G.d * G.n);
    op_D(&G, z, p);
    double tv = 0.0;
    for (size_t e = 0; e < G.n; ++e) {
        double s = 0.0;
        for (int c = 0; c < G.d; ++c) s += p[c * G.n + e] * p[c * G.n + e];
        tv += sqrt(s);
    }
    free(p);
    return tv;
}

/* z = P_C(v - tau D^T p). */
static void primal_from_dual(const grid *G, const double *v, const double *p, double tau,
                             int nonneg, double *tmp, double *z)
{
    op_DT(G, p, tmp);
    for (size_t e = 0; e < G->n; ++e) {
        const double w = v[e] - tau * tmp[e];
        z[e] = (nonneg && w < 0.0) ? 0.0 : w;
    }
}

/* P_P: scale each pixel's d-vector onto the unit ball (isotropic TV). */
static void project_unit_ball(const grid *G, double *p)
{
    for (size_t e = 0; e < G->n; ++e) {
        double s = 0.0;
        for (int c = 0; c < G->d; ++c) s += p[c * G->n + e] * p[c * G->n + e];
        const double nrm = sqrt(s);
        if (nrm > 1.0)
            for (int c = 0; c < G->d; ++c) p[c * G->n + e] /= nrm;
    }
}

void orc_tv_prox_fgp(int nx, int ny, int nz, const double *v, double *z, double tau, int n_inner,
                     int nonneg, double *dual)
{
    grid G = make_grid(nx, ny, nz);
    const size_t n = G.n, dn = G.d * G.n;
    if (tau == 0.0) {
        for (size_t e = 0; e < n; ++e) z[e] = (nonneg && v[e] < 0.0) ? 0.0 : v[e];
        return;
    }
    double *vv = alloc_d(n), *tmp = alloc_d(n), *zk = alloc_d(n);
    double *p_prev = alloc_d(dn), *r = alloc_d(dn), *pn = alloc_d(dn), *dz = alloc_d(dn);
    memcpy(vv, v, sizeof(double) * n); /* z may alias v */
    if (dual) memcpy(p_prev, dual, sizeof(double) * dn);
    memcpy(r, p_prev, sizeof(double) * dn); /* r_1 = p_0 */
    double t = 1.0;
    const double step = 1.0 / (4.0 * G.d * tau); /* 1/(L tau^2) * tau with L = ||D||^2 <= 4d */
    for (int k = 0; k < n_inner; ++k) {
        primal_from_dual(&G, vv, r, tau, nonneg, tmp, zk); /* z_k = P_C(v - tau D^T r_k) */
        op_D(&G, zk, dz);
        for (size_t e = 0; e < dn; ++e) pn[e] = r[e] + step * dz[e]; /* dual ascent step */
        project_unit_ball(&G, pn);                                  /* p_k = P_P(...)  */
        const double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
        const double beta = (t - 1.0) / tn;
        for (size_t e = 0; e < dn; ++e) r[e] = pn[e] + beta * (pn[e] - p_prev[e]);
        memcpy(p_prev, pn, sizeof(double) * dn);
        t = tn;
    }
    primal_from_dual(&G, vv, p_prev, tau, nonneg, tmp, z);
    if (dual) memcpy(dual, p_prev, sizeof(double) * dn);
    free(vv); free(tmp); free(zk); free(p_prev); free(r); free(pn); free(dz);
}

void orc_tv_prox_dpg(int nx, int ny, int nz, const double *v, double *z, double tau, int n_iter,
                     int nonneg, double *dual)
{
    grid G = make_grid(nx, ny, nz);
    const size_t n = G.n, dn = G.d * G.n;
    if (tau == 0.0) {
        for (size_t e = 0; e < n; ++e) z[e] = (nonneg && v[e] < 0.0) ? 0.0 : v[e];
        return;
    }
    double *vv = alloc_d(n), *tmp = alloc_d(n), *zk = alloc_d(n);
    double *p = alloc_d(dn), *dz = alloc_d(dn);
    memcpy(vv, v, sizeof(double) * n);
    if (dual) memcpy(p, dual, sizeof(double) * dn);
    const double step = 1.0 / (4.0 * G.d * tau);
    for (int k = 0; k < n_iter; ++k) {
        primal_from_dual(&G, vv, p, tau, nonneg, tmp, zk);
        op_D(&G, zk, dz);
        for (size_t e = 0; e < dn; ++e) p[e] += step * dz[e];
        project_unit_ball(&G, p);
    }
    primal_from_dual(&G, vv, p, tau, nonneg, tmp, z);
    if (dual) memcpy(dual, p, sizeof(double) * dn);
    free(vv); free(tmp); free(zk); free(p); free(dz);
}

/* ------------------------------------------------------------------------------------------ */
/* Random streams: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) read at a counter.            */
/* ------------------------------------------------------------------------------------------ */

uint64_t orc_splitmix64(uint64_t seed, uint64_t j)
{
    uint64_t z = seed + (j + 1u) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

void orc_sequences(uint64_t seed, int64_t k0, int64_t count, int n_subsets, double p,
                   int32_t *subset_out, uint8_t *coin_out)
{
    const uint64_t thresh = (uint64_t)floor(p * 9007199254740992.0); /* p * 2^53 */
    for (int64_t t = 0; t < count; ++t) {
        const uint64_t k = (uint64_t)(k0 + t);
        const uint64_t us = orc_splitmix64(seed, 2u * k);
        const uint64_t uc = orc_splitmix64(seed, 2u * k + 1u);
        if (subset_out) subset_out[t] = (int32_t)(((us >> 32) * (uint64_t)n_subsets) >> 32);
        if (coin_out) coin_out[t] = (uint8_t)((uc >> 11) < thresh);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* ProxSkip with the SVRG estimator (Algorithm 1; estimator table, ProxSVRGSkip row).          */
/* ------------------------------------------------------------------------------------------ */

static double rel_change(const double *x, const double *xs, size_t n)
{
    double dd = 0.0, xx = 0.0;
    for (size_t e = 0; e < n; ++e) {
        const double d = x[e] - xs[e];
        dd += d * d;
        xx += x[e] * x[e];
    }
    return xx > 0.0 ? sqrt(dd) / sqrt(xx) : (dd > 0.0 ? INFINITY : 0.0);
}

int orc_proxskip_svrg(const orc_geom *g, const double *b, double *x, double *h, double *dual,
                      double gamma, double p, double alpha, int fgp_inner, int nonneg,
                      int n_epochs, int plain, uint64_t seed, int64_t k0, double tol,
                      orc_stats *stats, double *rel_change_out)
{
    const int N = g->n_subsets;
    if (N < 1 || gamma <= 0.0 || !(p > 0.0 && p <= 1.0) || alpha < 0.0 || fgp_inner < 0 ||
        n_epochs < 0 || k0 < 0 || k0 % N != 0)
        return -1;
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    double *xs = alloc_d(n), *gs = alloc_d(n), *gx = alloc_d(n), *gxs = alloc_d(n);
    double *G = alloc_d(n), *xh = alloc_d(n), *v = alloc_d(n), *xn = alloc_d(n);
    const int64_t K = (int64_t)n_epochs * N;
    int32_t *sub = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
    uint8_t *coin = (uint8_t *)malloc((size_t)(K > 0 ? K : 1));
    orc_sequences(seed, k0, K, N, p, sub, coin);

    orc_stats st = {0, 0, 0, 0.0};
    for (int64_t t = 0; t <= K; ++t) {
        const int64_t k = k0 + t;
        if (k % N == 0) {
            if (t > 0) { /* end of an epoch: x_e versus x_{e-1} (= the snapshot) */
                st.last_rel_change = rel_change(x, xs, n);
                if (rel_change_out) rel_change_out[st.epochs_done] = st.last_rel_change;
                st.epochs_done++;
                if (tol > 0.0 && st.last_rel_change < tol) break;
            }
            if (t == K) break;
            /* SVRG snapshot, refreshed every N iterations. */
            memcpy(xs, x, sizeof(double) * n);
            orc_grad_full(g, xs, b, gs);
        }
        const int i = sub[t];
        /* G_k = N (grad f_i(x_k) - grad f_i(xs)) + grad f(xs) */
        orc_grad_subset(g, i, x, b, gx);
        orc_grad_subset(g, i, xs, b, gxs);
        for (size_t e = 0; e < n; ++e) G[e] = (double)N * (gx[e] - gxs[e]) + gs[e];

        if (plain) {
            /* non-skipped ProxSVRG: x+ = prox_{gamma g}(x - gamma G) */
            for (size_t e = 0; e < n; ++e) v[e] = x[e] - gamma * G[e];
            orc_tv_prox_fgp(g->nx, g->ny, g->nz, v, x, gamma * alpha, fgp_inner, nonneg, dual);
            st.prox_calls++;
        } else {
            for (size_t e = 0; e < n; ++e) xh[e] = x[e] - gamma * (G[e] - h[e]);
            if (coin[t]) {
                for (size_t e = 0; e < n; ++e) v[e] = xh[e] - (gamma / p) * h[e];
                orc_tv_prox_fgp(g->nx, g->ny, g->nz, v, xn, gamma * alpha / p, fgp_inner, nonneg,
                                dual);
                st.prox_calls++;
            } else {
                memcpy(xn, xh, sizeof(double) * n);
            }
            for (size_t e = 0; e < n; ++e) h[e] = h[e] + (p / gamma) * (xn[e] - xh[e]);
            memcpy(x, xn, sizeof(double) * n);
        }
        st.iters_done++;
    }
    if (stats) *stats = st;
    free(xs); free(gs); free(gx); free(gxs); free(G); free(xh); free(v); free(xn);
    free(sub); free(coin);
    return 0;
}

void orc_refresh_coins(uint64_t seed, int64_t k0, int64_t count, int n_subsets, uint8_t *out)
{
    const uint64_t thresh = (1ULL << 53) / (uint64_t)n_subsets; /* floor(2^53 / N) */
    for (int64_t t = 0; t < count; ++t) {
        const uint64_t u = orc_splitmix64(seed, (1ULL << 62) + (uint64_t)(k0 + t));
        out[t] = (uint8_t)((u >> 11) < thresh);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Algorithm 1 with the SVRG, loopless SVRG and SAGA estimators (the table beside it).         */
/* ------------------------------------------------------------------------------------------ */

int orc_proxskip(const orc_geom *g, const double *b, double *x, double *h, double *dual,
                 double gamma, double p, double alpha, int fgp_inner, int nonneg, int plain,
                 int estimator, int64_t k0, int64_t n_iters, const int32_t *sub,
                 const uint8_t *coin, const uint8_t *refresh, double tol, orc_stats *stats,
                 double *rel_change_out, double *table, double *table_sum)
{
    const int N = g->n_subsets;
    if (N < 1 || gamma <= 0.0 || !(p > 0.0 && p <= 1.0) || alpha < 0.0 || fgp_inner < 0 ||
        n_iters < 0 || k0 < 0 || k0 % N != 0 || !sub || (!plain && !coin) ||
        estimator < ORC_SVRG || estimator > ORC_SAGA || (estimator == ORC_LSVRG && !refresh))
        return -1;
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    double *xs = alloc_d(n), *gs = alloc_d(n), *gx = alloc_d(n), *gxs = alloc_d(n);
    double *G = alloc_d(n), *xh = alloc_d(n), *v = alloc_d(n), *xn = alloc_d(n);
    double *xe = alloc_d(n);                 /* x at the last epoch end (or the start) */
    double *V = NULL, *vbar = NULL;
    if (estimator == ORC_SAGA) {
        V = table ? table : alloc_d(n * (size_t)N);
        vbar = table_sum ? table_sum : alloc_d(n);
    }
    memcpy(xe, x, sizeof(double) * n);

    orc_stats st = {0, 0, 0, 0.0};
    for (int64_t t = 0; t < n_iters; ++t) {
        const int64_t k = k0 + t;
        const int i = sub[t];
        if (estimator == ORC_SAGA) {
            if (t == 0) {
                /* table v_j = grad f_j(x_0), vbar = sum_j v_j in increasing j */
                memset(vbar, 0, sizeof(double) * n);
                for (int j = 0; j < N; ++j) {
                    double *vj = V + (size_t)j * n;
                    orc_grad_subset(g, j, x, b, vj);
                    for (size_t e = 0; e < n; ++e) vbar[e] += vj[e];
                }
            }
            /* Eq. 4: G = N (grad f_i(x) - v_i) + vbar, then the table entry i and the sum */
            double *vi = V + (size_t)i * n;
            orc_grad_subset(g, i, x, b, gx);
            for (size_t e = 0; e < n; ++e) {
                const double diff = gx[e] - vi[e];
                G[e] = (double)N * diff + vbar[e];
                vbar[e] += diff;
                vi[e] = gx[e];
            }
        } else {
            const int refresh_now = estimator == ORC_SVRG ? (k % N == 0) : (t == 0 || refresh[t]);
            if (refresh_now) {
                memcpy(xs, x, sizeof(double) * n);
                orc_grad_full(g, xs, b, gs);
            }
            orc_grad_subset(g, i, x, b, gx);
            orc_grad_subset(g, i, xs, b, gxs);
            for (size_t e = 0; e < n; ++e) G[e] = (double)N * (gx[e] - gxs[e]) + gs[e];
        }

        if (plain) {
            for (size_t e = 0; e < n; ++e) v[e] = x[e] - gamma * G[e];
            orc_tv_prox_fgp(g->nx, g->ny, g->nz, v, x, gamma * alpha, fgp_inner, nonneg, dual);
            st.prox_calls++;
        } else {
            for (size_t e = 0; e < n; ++e) xh[e] = x[e] - gamma * (G[e] - h[e]);
            if (coin[t]) {
                for (size_t e = 0; e < n; ++e) v[e] = xh[e] - (gamma / p) * h[e];
                orc_tv_prox_fgp(g->nx, g->ny, g->nz, v, xn, gamma * alpha / p, fgp_inner, nonneg,
                                dual);
                st.prox_calls++;
            } else {
                memcpy(xn, xh, sizeof(double) * n);
            }
            for (size_t e = 0; e < n; ++e) h[e] = h[e] + (p / gamma) * (xn[e] - xh[e]);
            memcpy(x, xn, sizeof(double) * n);
        }
        st.iters_done++;
        if ((k + 1) % N == 0) {
            st.last_rel_change = rel_change(x, xe, n);
            if (rel_change_out) rel_change_out[st.epochs_done] = st.last_rel_change;
            st.epochs_done++;
            memcpy(xe, x, sizeof(double) * n);
            if (tol > 0.0 && st.last_rel_change < tol) break;
        }
    }
    if (stats) *stats = st;
    if (V && V != table) free(V);
    if (vbar && vbar != table_sum) free(vbar);
    free(xs); free(gs); free(gx); free(gxs); free(G); free(xh); free(v); free(xn); free(xe);
    return 0;
}

/* FISTA: ISTA with the acceleration step of Beck & Teboulle (2009). */
int orc_fista(const orc_geom *g, const double *b, double *x, double *dual, double gamma,
              double alpha, int fgp_inner, int nonneg, int n_iters, double *fval_out)
{
    if (gamma <= 0.0 || alpha < 0.0 || fgp_inner < 0 || n_iters < 0) return -1;
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    double *y = alloc_d(n), *gy = alloc_d(n), *v = alloc_d(n), *xn = alloc_d(n);
    memcpy(y, x, sizeof(double) * n);
    double t = 1.0;
    for (int k = 0; k < n_iters; ++k) {
        orc_grad_full(g, y, b, gy);
        for (size_t e = 0; e < n; ++e) v[e] = y[e] - gamma * gy[e];
        orc_tv_prox_fgp(g->nx, g->ny, g->nz, v, xn, gamma * alpha, fgp_inner, nonneg, dual);
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        const double beta = (t - 1.0) / tn;
        for (size_t e = 0; e < n; ++e) {
            y[e] = xn[e] + beta * (xn[e] - x[e]);
            x[e] = xn[e];
        }
        t = tn;
        if (fval_out) fval_out[k] = orc_data_fit(g, x, b) + alpha * orc_tv(g->nx, g->ny, g->nz, x);
    }
    free(y); free(gy); free(v); free(xn);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Reference solution: diagonally preconditioned PDHG (Chambolle & Pock 2011).                 */
/* ------------------------------------------------------------------------------------------ */

int orc_pdhg(const orc_geom *g, const double *b, double *x, double *y1, double *y2, double alpha,
             int nonneg, int n_iters)
{
    if (alpha < 0.0 || n_iters < 0) return -1;
    grid G = make_grid(g->nx, g->ny, g->nz);
    const size_t n = G.n, dn = G.d * G.n;
    const size_t m = (size_t)g->nz * g->n_angles * g->n_bins;
    double *tau = alloc_d(n), *sig = alloc_d(m), *ones_n = alloc_d(n), *ones_m = alloc_d(m);
    double *kty = alloc_d(n), *dty = alloc_d(n), *xbar = alloc_d(n), *axb = alloc_d(m);
    double *dxb = alloc_d(dn);
    const double sig_d = 0.5;
    /* preconditioners from the row and column sums of |K| (A >= 0 entrywise) */
    for (size_t e = 0; e < n; ++e) ones_n[e] = 1.0;
    for (size_t e = 0; e < m; ++e) ones_m[e] = 1.0;
    orc_project(g, -1, ones_n, sig);     /* row sums of A    */
    orc_backproject(g, -1, ones_m, tau); /* column sums of A */
    for (size_t e = 0; e < m; ++e) sig[e] = sig[e] > 0.0 ? 1.0 / sig[e] : 1.0;
    for (int zz = 0; zz < g->nz; ++zz)
        for (int i = 0; i < g->ny; ++i)
            for (int j = 0; j < g->nx; ++j) {
                const size_t e = ((size_t)zz * g->ny + i) * g->nx + j;
                /* pixel e enters the differences of itself and of its lower neighbours */
                double cd = (j < g->nx - 1) + (j > 0) + (i < g->ny - 1) + (i > 0);
                if (G.d == 3) cd += (zz < g->nz - 1) + (zz > 0);
                tau[e] = 1.0 / (tau[e] + cd);
            }
    for (int k = 0; k < n_iters; ++k) {
        /* primal step */
        orc_backproject(g, -1, y1, kty);
        op_DT(&G, y2, dty);
        for (size_t e = 0; e < n; ++e) {
            double w = x[e] - tau[e] * (kty[e] + dty[e]);
            if (nonneg && w < 0.0) w = 0.0;
            xbar[e] = 2.0 * w - x[e];
            x[e] = w;
        }
        /* dual steps at the extrapolated point */
        orc_project(g, -1, xbar, axb);
        for (size_t e = 0; e < m; ++e) y1[e] = (y1[e] + sig[e] * (axb[e] - b[e])) / (1.0 + sig[e]);
        op_D(&G, xbar, dxb);
        for (size_t e = 0; e < n; ++e) {
            double s2 = 0.0;
            for (int c = 0; c < G.d; ++c) {
                const double v = y2[c * n + e] + sig_d * dxb[c * n + e];
                y2[c * n + e] = v;
                s2 += v * v;
            }
            const double nrm = sqrt(s2);
            if (nrm > alpha) {
                const double sc = alpha > 0.0 ? alpha / nrm : 0.0;
                for (int c = 0; c < G.d; ++c) y2[c * n + e] *= sc;
            }
        }
    }
    free(tau); free(sig); free(ones_n); free(ones_m); free(kty); free(dty); free(xbar); free(axb);
    free(dxb);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
