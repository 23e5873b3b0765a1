// solver.hip -- ProxSkip with the SVRG estimator (Algorithm 1, ProxSVRGSkip row), driven from
// the host over the projector, backprojector and FGP kernels, plus the resumable handle API.
//
// Per epoch (N iterations, one data pass):
//   k = eN      snapshot xs = x; r = A xs - b (full projection, residual fused);
//               gs = A^T r fused with the first step (G = gs because x = xs);
//   k = eN + t  y = A_i (x - xs)  (the SVRG difference: N (grad f_i(x) - grad f_i(xs)) equals
//               N A_i^T A_i (x - xs) exactly for the least-squares fit, and saves one projection
//               pair per iteration); G = N A_i^T y + gs fused into the backprojector with
//               xh = x - gamma (G - h):  theta = 0 -> x = xh;  theta = 1 -> v = xh - (gamma/p) h,
//               then FGP gives x = prox(v) and h = h + (p/gamma)(x - xh) = (p/gamma)(x - v).
//   epoch end   ||x - xs||^2 and ||x||^2 (fixed-order two-level reduction in FP64).
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "internal.h"

namespace ps {

constexpr int kNormBlocks = 1024;

// Partial sums of ||x - xs||^2 and ||x||^2 (FP64) per block; optionally xs = x afterwards.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_snapshot(const T *__restrict__ x, T *__restrict__ xs,
                                                     size_t n, int do_norm, int do_copy,
                                                     double *__restrict__ part) {
    __shared__ double sd[kBlock], sx[kBlock];
    double dd = 0.0, xx = 0.0;
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock) {
        const T xv = x[e];
        if (do_norm) {
            const double dv = static_cast<double>(xv) - static_cast<double>(xs[e]);
            dd += dv * dv;
            xx += static_cast<double>(xv) * static_cast<double>(xv);
        }
        if (do_copy) xs[e] = xv;
    }
    if (!do_norm) return;
    sd[threadIdx.x] = dd;
    sx[threadIdx.x] = xx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            sd[threadIdx.x] += sd[threadIdx.x + w];
            sx[threadIdx.x] += sx[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sd[0];
        part[2 * blockIdx.x + 1] = sx[0];
    }
}

// out[0..1] = sums of the block partials, in a fixed order.
__global__ __launch_bounds__(kBlock) void k_norm_final(const double *__restrict__ part, int nblk,
                                                       double *__restrict__ out) {
    __shared__ double sd[kBlock], sx[kBlock];
    double dd = 0.0, xx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        dd += part[2 * b];
        xx += part[2 * b + 1];
    }
    sd[threadIdx.x] = dd;
    sx[threadIdx.x] = xx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            sd[threadIdx.x] += sd[threadIdx.x + w];
            sx[threadIdx.x] += sx[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sd[0];
        out[1] = sx[0];
    }
}

static int norm_blocks(size_t n) {
    return static_cast<int>(std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, kNormBlocks)));
}

struct Layout {
    size_t xs, gs, v, sino, pws, bws, fws, npart, stats, total;
    size_t pws_bytes, bws_bytes, fws_bytes;
};

static Layout layout(const ps_geometry *g, int n_epochs) {
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    const size_t m = static_cast<size_t>(d.nz) * d.n_angles * d.n_bins;
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    L.xs = take(n * g->elem);
    L.gs = take(n * g->elem);
    L.v = take(n * g->elem);
    L.sino = take(m * g->elem);
    L.pws_bytes = std::max(proj_workspace(g, d.n_angles), proj_workspace(g, max_subset_count(g)));
    L.pws = take(L.pws_bytes);
    L.bws_bytes = back_workspace(g, -1);
    for (int i = 0; i < d.n_subsets; ++i) L.bws_bytes = std::max(L.bws_bytes, back_workspace(g, i));
    L.bws = take(L.bws_bytes);
    L.fws_bytes = fgp_workspace(g);
    L.fws = take(L.fws_bytes);
    L.npart = take(sizeof(double) * 2 * kNormBlocks);
    L.stats = take(sizeof(double) * 2 * static_cast<size_t>(std::max(n_epochs, 1)));
    L.total = off;
    return L;
}

static ps_status check_params(const ps_geometry *g, const ps_solver_params *p) {
    if (!p) return fail(PS_EINVAL, "params is null");
    if (!(p->gamma > 0.0) || !std::isfinite(p->gamma)) return fail(PS_EINVAL, "gamma must be > 0");
    if (!(p->p > 0.0 && p->p <= 1.0)) return fail(PS_EINVAL, "p must be in (0, 1]");
    if (!(p->alpha >= 0.0) || !std::isfinite(p->alpha)) return fail(PS_EINVAL, "alpha must be >= 0");
    if (p->fgp_inner < 0) return fail(PS_EINVAL, "fgp_inner must be >= 0");
    if (p->nonneg != 0 && p->nonneg != 1) return fail(PS_EINVAL, "nonneg must be 0 or 1");
    if (p->plain_prox_svrg != 0 && p->plain_prox_svrg != 1)
        return fail(PS_EINVAL, "plain_prox_svrg must be 0 or 1");
    if (p->n_epochs < 0) return fail(PS_EINVAL, "n_epochs must be >= 0");
    if (p->k0 < 0 || p->k0 % g->desc.n_subsets != 0)
        return fail(PS_EINVAL, "k0 must be a non-negative multiple of n_subsets");
    if (!(p->tol_rel_change >= 0.0)) return fail(PS_EINVAL, "tol_rel_change must be >= 0");
    return PS_OK;
}

}  // namespace ps

using namespace ps;

struct ps_solver {
    const ps_geometry *g;
    const void *b;
    void *x, *h, *dual;
    ps_solver_params prm;
    unsigned char *ws;
    Layout L;
    int64_t k;               // next iteration index
    int epochs_done;         // epochs queued
    int epochs_read;         // epochs whose norms were read back
    int prox_calls;
    double last_rel;
    bool converged, cancelled, nonfinite;
    hipStream_t stream;
    std::vector<int32_t> sub;
    std::vector<uint8_t> coin;
    std::vector<double> stats_host;
};

namespace ps {

template <typename T>
static ps_status snapshot_norms(ps_solver *s, int do_norm, int do_copy, hipStream_t st) {
    const auto &d = s->g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    const int nb = norm_blocks(n);
    double *part = reinterpret_cast<double *>(s->ws + s->L.npart);
    hipLaunchKernelGGL((k_snapshot<T>), dim3(nb), dim3(kBlock), 0, st, static_cast<const T *>(s->x),
                       reinterpret_cast<T *>(s->ws + s->L.xs), n, do_norm, do_copy, part);
    PS_LAUNCHED("k_snapshot");
    if (do_norm) {
        double *out = reinterpret_cast<double *>(s->ws + s->L.stats) + 2 * s->epochs_done;
        hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kBlock), 0, st, part, nb, out);
        PS_LAUNCHED("k_norm_final");
    }
    return PS_OK;
}

template <typename T>
static ps_status run_epoch(ps_solver *s, hipStream_t st) {
    const ps_geometry *g = s->g;
    const auto &d = g->desc;
    const auto &P = s->prm;
    const int N = d.n_subsets;
    unsigned char *w = s->ws;
    s->sub.resize(N);
    s->coin.resize(N);
    draw_sequences(P.seed, s->k, N, N, P.p, s->sub.data(), s->coin.data());

    UpdateArgs up{};
    up.x = s->x;
    up.h = s->h;
    up.gs = w + s->L.gs;
    up.vout = w + s->L.v;
    up.gamma = P.gamma;
    up.gamma_over_p = P.gamma / P.p;
    up.nsub = static_cast<double>(N);
    up.plain = P.plain_prox_svrg;

    FgpOut fo{};
    fo.x = s->x;
    fo.h = s->h;
    fo.hscale = P.p / P.gamma;
    fo.proxskip = P.plain_prox_svrg ? 2 : 1;
    const double tau = P.plain_prox_svrg ? P.gamma * P.alpha : P.gamma * P.alpha / P.p;

    PS_TRY(snapshot_norms<T>(s, 0, 1, st));  // xs = x
    for (int t = 0; t < N; ++t) {
        const int i = s->sub[t];
        const bool prox = P.plain_prox_svrg || s->coin[t];
        up.coin = s->coin[t];
        if (t == 0) {
            // r = A xs - b over all angles, then gs = A^T r fused with the step (G = gs)
            PS_TRY(launch_project(g, -1, w + s->L.xs, nullptr, s->b, w + s->L.sino, w + s->L.pws,
                                  s->L.pws_bytes, st));
            PS_TRY(launch_backproject(g, -1, w + s->L.sino, nullptr, BP_SNAPSHOT, &up, w + s->L.bws,
                                      s->L.bws_bytes, st));
        } else {
            PS_TRY(launch_project(g, i, s->x, w + s->L.xs, nullptr, w + s->L.sino, w + s->L.pws,
                                  s->L.pws_bytes, st));
            PS_TRY(launch_backproject(g, i, w + s->L.sino, nullptr, BP_SVRG, &up, w + s->L.bws,
                                      s->L.bws_bytes, st));
        }
        if (prox) {
            PS_TRY(launch_fgp(g, w + s->L.v, s->dual, tau, P.fgp_inner, P.nonneg, fo, w + s->L.fws,
                              s->L.fws_bytes, st));
            s->prox_calls++;
        }
    }
    s->k += N;
    PS_TRY(snapshot_norms<T>(s, 1, 0, st));  // ||x_e - x_{e-1}||, ||x_e||
    s->epochs_done++;
    return PS_OK;
}

// Read back the norms of the epochs queued since the last read; updates last_rel/converged.
static ps_status read_stats(ps_solver *s) {
    if (s->epochs_read >= s->epochs_done) return PS_OK;
    PS_HIP(hipStreamSynchronize(s->stream));
    const int e0 = s->epochs_read, cnt = s->epochs_done - e0;
    s->stats_host.resize(2 * static_cast<size_t>(s->epochs_done));
    PS_HIP(hipMemcpy(s->stats_host.data() + 2 * e0,
                     reinterpret_cast<double *>(s->ws + s->L.stats) + 2 * e0,
                     sizeof(double) * 2 * cnt, hipMemcpyDeviceToHost));
    for (int e = e0; e < s->epochs_done; ++e) {
        const double dd = s->stats_host[2 * e], xx = s->stats_host[2 * e + 1];
        if (!std::isfinite(dd) || !std::isfinite(xx)) s->nonfinite = true;
        s->last_rel = xx > 0.0 ? std::sqrt(dd) / std::sqrt(xx) : (dd > 0.0 ? INFINITY : 0.0);
        if (s->prm.tol_rel_change > 0.0 && s->last_rel < s->prm.tol_rel_change) {
            s->converged = true;
        }
    }
    s->epochs_read = s->epochs_done;
    if (s->nonfinite) return fail(PS_ENONFINITE, "non-finite iterate at an epoch end");
    return PS_OK;
}

static bool active(const ps_solver *s) {
    return !s->cancelled && !s->converged && !s->nonfinite && s->epochs_done < s->prm.n_epochs;
}

}  // namespace ps

extern "C" size_t proxskip_workspace_bytes(const ps_geometry *g, const ps_solver_params *p) {
    if (!g || !p) return 0;
    return layout(g, p->n_epochs).total;
}

extern "C" ps_status solver_init(const ps_geometry *g, const void *b, void *x, void *h, void *dual,
                                 const ps_solver_params *prm, void *workspace, size_t ws_bytes,
                                 ps_solver **out) {
    clear_error();
    if (!out) return fail(PS_EINVAL, "out is null");
    *out = nullptr;
    if (!g) return fail(PS_EINVAL, "geometry is null");
    PS_TRY(check_params(g, prm));
    PS_TRY(check_ready(g));
    PS_TRY(check_ptr(b, "b", g->elem));
    PS_TRY(check_ptr(x, "x", g->elem));
    PS_TRY(check_ptr(h, "h", g->elem));
    PS_TRY(check_ptr(dual, "dual", g->elem));
    PS_TRY(check_ptr(workspace, "workspace", kAlign));
    const Layout L = layout(g, prm->n_epochs);
    if (ws_bytes < L.total)
        return fail(PS_EINVAL, "solver workspace: %zu bytes given, %zu needed", ws_bytes, L.total);
    ps_solver *s = new (std::nothrow) ps_solver();
    if (!s) return fail(PS_ENOMEM, "out of host memory");
    s->g = g;
    s->b = b;
    s->x = x;
    s->h = h;
    s->dual = dual;
    s->prm = *prm;
    s->ws = static_cast<unsigned char *>(workspace);
    s->L = L;
    s->k = prm->k0;
    s->epochs_done = s->epochs_read = s->prox_calls = 0;
    s->last_rel = 0.0;
    s->converged = s->cancelled = s->nonfinite = false;
    s->stream = nullptr;
    *out = s;
    return PS_OK;
}

extern "C" ps_status solver_epochs(ps_solver *const *handles, int32_t n_handles, int32_t n_epochs,
                                   void *stream) {
    clear_error();
    if (n_handles < 0 || n_epochs < 0 || (n_handles > 0 && !handles))
        return fail(PS_EINVAL, "bad handle list or epoch count");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n_handles; ++i) {
        if (!handles[i]) return fail(PS_EINVAL, "handle %d is null", i);
        if (handles[i]->cancelled) return fail(PS_ECANCELLED, "handle %d was cancelled", i);
    }
    for (int e = 0; e < n_epochs; ++e) {
        bool any = false;
        for (int i = 0; i < n_handles; ++i) {
            ps_solver *s = handles[i];
            if (!active(s)) continue;
            s->stream = st;
            any = true;
            if (s->g->desc.dtype == PS_F64)
                PS_TRY(run_epoch<double>(s, st));
            else
                PS_TRY(run_epoch<float>(s, st));
        }
        if (!any) break;
        bool need_read = false;
        for (int i = 0; i < n_handles; ++i)
            if (handles[i]->prm.tol_rel_change > 0.0 && handles[i]->epochs_read < handles[i]->epochs_done)
                need_read = true;
        if (need_read) {
            for (int i = 0; i < n_handles; ++i) PS_TRY(read_stats(handles[i]));
        }
    }
    return PS_OK;
}

extern "C" ps_status solver_query(ps_solver *s, ps_solver_stats *out) {
    clear_error();
    if (!s) return fail(PS_EINVAL, "handle is null");
    const ps_status rs = read_stats(s);
    if (out) {
        out->epochs_done = s->epochs_done;
        out->iters_done = static_cast<int32_t>(s->k - s->prm.k0);
        out->prox_calls = s->prox_calls;
        out->last_rel_change = s->last_rel;
    }
    return rs;
}

extern "C" ps_status solver_cancel(ps_solver *s) {
    clear_error();
    if (!s) return fail(PS_EINVAL, "handle is null");
    s->cancelled = true;
    return PS_OK;
}

extern "C" void solver_free(ps_solver *s) { delete s; }

extern "C" ps_status proxskip_svrg_run(const ps_geometry *g, const void *b, void *x, void *h,
                                       void *dual, const ps_solver_params *prm,
                                       ps_solver_stats *stats_out, void *workspace, size_t ws_bytes,
                                       void *stream) {
    ps_solver *s = nullptr;
    PS_TRY(solver_init(g, b, x, h, dual, prm, workspace, ws_bytes, &s));
    ps_status st = solver_epochs(&s, 1, prm->n_epochs, stream);
    s->stream = static_cast<hipStream_t>(stream);
    if (st == PS_OK) {
        st = solver_query(s, stats_out);
    } else {
        (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    }
    solver_free(s);
    return st;
}
