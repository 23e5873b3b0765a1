// solver.hip -- ProxSkip (Algorithm 1) with the SVRG, loopless-SVRG and SAGA estimators of the
// table beside it, driven from the host over the projector, backprojector and FGP kernels, plus
// the resumable handle API and FISTA.
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
// Loopless SVRG takes the snapshot branch at iterations whose refresh coin is 1 instead of at
// epoch starts.  SAGA projects x itself (y = A_i x - b_i) and updates its table in the
// backprojector's epilogue; both keep x of the last epoch end (xe) for the epoch-end norms.
#include <algorithm>
#include <climits>
#include <cmath>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace ps {

constexpr int kNormBlocks = 1024;

// Instantiated graphs of captured epoch rounds, keyed by the round's launch topology.
struct GraphCache {
    hipStream_t capture = nullptr;   // never runs work: launches are recorded on it
    std::vector<std::pair<std::string, hipGraphExec_t>> execs;   // most recently used last
    ~GraphCache() {
        for (auto &e : execs) (void)hipGraphExecDestroy(e.second);
        if (capture) (void)hipStreamDestroy(capture);
    }
};
constexpr size_t kMaxGraphs = 64;

// Partial sums of ||x - xs||^2 and ||x||^2 (FP64) per block; optionally xs = x afterwards.
template <typename T>
struct SnapItem {
    const T *x;
    T *xs;
    double *part;
    size_t n;
    int do_norm, do_copy, blocks;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_snapshot(WorkList<SnapItem<T>> wl) {
    __shared__ double sd[kBlock], sx[kBlock];
    int local;
    const SnapItem<T> &it = wl.item[work_item(wl, local)];
    const T *__restrict__ x = it.x;
    T *__restrict__ xs = it.xs;
    const int do_norm = it.do_norm, do_copy = it.do_copy;
    double dd = 0.0, xx = 0.0;
    for (size_t e = local * static_cast<size_t>(kBlock) + threadIdx.x; e < it.n;
         e += static_cast<size_t>(it.blocks) * kBlock) {
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
        it.part[2 * local] = sd[0];
        it.part[2 * local + 1] = sx[0];
    }
}

// out[0..1] = sums of the block partials, in a fixed order (one workgroup per item).
struct NormItem {
    const double *part;
    double *out;
    int nblk;
};

__global__ __launch_bounds__(kBlock) void k_norm_final(WorkList<NormItem> wl) {
    __shared__ double sd[kBlock], sx[kBlock];
    int local;
    const NormItem &it = wl.item[work_item(wl, local)];
    double dd = 0.0, xx = 0.0;
    for (int b = threadIdx.x; b < it.nblk; b += kBlock) {
        dd += it.part[2 * b];
        xx += it.part[2 * b + 1];
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
        it.out[0] = sd[0];
        it.out[1] = sx[0];
    }
}

// tsum = sum_j tab[j] in increasing j (the SAGA table's running sum at initialisation).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_table_sum(const T *__restrict__ tab, T *__restrict__ tsum,
                                                      int nrows, size_t n) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock) {
        T acc = T(0);
        for (int j = 0; j < nrows; ++j) acc += tab[static_cast<size_t>(j) * n + e];
        tsum[e] = acc;
    }
}

// FISTA extrapolation: y = xn + beta (xn - x), then x = xn.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fista_momentum(T *__restrict__ x, const T *__restrict__ xn,
                                                           T *__restrict__ y, T beta, size_t n) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock) {
        const T a = xn[e];
        y[e] = a + beta * (a - x[e]);
        x[e] = a;
    }
}

// dx = x - xs (the SVRG difference after a prox step rewrote x).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diff(const T *__restrict__ x, const T *__restrict__ xs,
                                                 T *__restrict__ dx, size_t n) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock)
        dx[e] = x[e] - xs[e];
}

static int elementwise_blocks(size_t n) {
    return static_cast<int>(std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, 8192)));
}

static int norm_blocks(size_t n) {
    return static_cast<int>(std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, kNormBlocks)));
}

struct Layout {
    size_t xs, gs, v, xe, tab, tsum, dx, sino, pws, bws, fws, npart, stats, total;
    size_t pws_bytes, bws_bytes, fws_bytes;
    bool has_dx;   // the difference buffer dx is kept (keeps_difference)
};

// The SVRG difference dx = x - xs kept in the workspace for the subset projector, once x and xs
// together outgrow an XCD's 4 MiB L2: the projector then reads one image instead of two, which
// it would otherwise fetch from HBM for every angle's rows.  dx is written where x is written
// (the backprojector epilogue, or k_diff after a prox), with the projector's own subtraction, so
// the results are bit for bit the same either way.
static bool keeps_difference(const ps_geometry *g, int estimator) {
    return estimator != PS_EST_SAGA && solver_reads_one_image(g);
}

}  // namespace ps

bool ps::solver_reads_one_image(const ps_geometry *g) {
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    return 2 * n * g->elem > (static_cast<size_t>(4) << 20);
}

namespace ps {

static Layout layout(const ps_geometry *g, int n_epochs, int estimator) {
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    const size_t m = static_cast<size_t>(d.nz) * d.n_angles * d.n_bins;
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    if (estimator != PS_EST_SAGA) {
        L.xs = take(n * g->elem);
        L.gs = take(n * g->elem);
    }
    L.v = take(n * g->elem);
    if (estimator != PS_EST_SVRG) L.xe = take(n * g->elem);
    if (estimator == PS_EST_SAGA) {
        L.tab = take(static_cast<size_t>(d.n_subsets) * n * g->elem);
        L.tsum = take(n * g->elem);
    }
    L.has_dx = keeps_difference(g, estimator);
    if (L.has_dx) L.dx = take(n * g->elem);
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
    if (p->estimator < PS_EST_SVRG || p->estimator > PS_EST_SAGA)
        return fail(PS_EINVAL, "estimator %d is not a ps_estimator", p->estimator);
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
    std::vector<int32_t> sub;   // i_k, theta_k (and rho_k, loopless SVRG) of the current epoch
    std::vector<uint8_t> coin, refresh;
    std::vector<double> stats_host;
    // tolerance runs: the epoch-end norms travel to pinned host memory behind an event
    bool pending;
    hipEvent_t ev;
    double *pinned;
    uint64_t id;                  // unique per handle (keys of the graph cache)
    ps::GraphCache *graphs;       // executable epoch graphs of rounds this handle led, or null
};

namespace ps {

// Record an epoch's norms (dd = ||x_e - x_{e-1}||^2, xx = ||x_e||^2) on the host.
static void take_norms(ps_solver *s, int e, double dd, double xx) {
    if (!std::isfinite(dd) || !std::isfinite(xx)) s->nonfinite = true;
    s->last_rel = xx > 0.0 ? std::sqrt(dd) / std::sqrt(xx) : (dd > 0.0 ? INFINITY : 0.0);
    if (s->prm.tol_rel_change > 0.0 && s->last_rel < s->prm.tol_rel_change) s->converged = true;
    if (s->stats_host.size() < 2 * static_cast<size_t>(e + 1)) s->stats_host.resize(2 * static_cast<size_t>(e + 1));
    s->stats_host[2 * e] = dd;
    s->stats_host[2 * e + 1] = xx;
    s->epochs_read = std::max(s->epochs_read, e + 1);
}

// Read back the norms of the epochs queued since the last read; updates last_rel/converged.
static ps_status read_stats(ps_solver *s) {
    if (s->pending) {
        PS_HIP(hipEventSynchronize(s->ev));
        take_norms(s, s->epochs_done - 1, s->pinned[0], s->pinned[1]);
        s->pending = false;
    }
    if (s->epochs_read >= s->epochs_done) {
        if (s->nonfinite) return fail(PS_ENONFINITE, "non-finite iterate at an epoch end");
        return PS_OK;
    }
    PS_HIP(hipStreamSynchronize(s->stream));
    const int e0 = s->epochs_read, cnt = s->epochs_done - e0;
    std::vector<double> buf(2 * static_cast<size_t>(cnt));
    PS_HIP(hipMemcpy(buf.data(), reinterpret_cast<double *>(s->ws + s->L.stats) + 2 * e0,
                     sizeof(double) * 2 * cnt, hipMemcpyDeviceToHost));
    for (int e = 0; e < cnt; ++e) take_norms(s, e0 + e, buf[2 * e], buf[2 * e + 1]);
    if (s->nonfinite) return fail(PS_ENONFINITE, "non-finite iterate at an epoch end");
    return PS_OK;
}

static bool active(const ps_solver *s) {
    return !s->cancelled && !s->converged && !s->nonfinite && s->epochs_done < s->prm.n_epochs;
}

template <typename T>
static ps_status launch_snapshots(const std::vector<SnapItem<T>> &items, hipStream_t st) {
    ListBuilder<SnapItem<T>> lb;
    for (const auto &it : items) {
        lb.add(it, it.blocks);
        if (lb.full()) {
            hipLaunchKernelGGL((k_snapshot<T>), dim3(lb.blocks), dim3(kBlock), 0, st, lb.wl);
            PS_LAUNCHED("k_snapshot");
            lb.clear();
        }
    }
    if (!lb.empty()) {
        hipLaunchKernelGGL((k_snapshot<T>), dim3(lb.blocks), dim3(kBlock), 0, st, lb.wl);
        PS_LAUNCHED("k_snapshot");
    }
    return PS_OK;
}

// One request of snapshot_many: copy x into the workspace buffer at `dst` and/or take the
// epoch-end norms ||x - dst||^2, ||x||^2 (the copy, when both, follows the norm element-wise).
struct SnapReq {
    ps_solver *s;
    size_t dst;
    int do_norm, do_copy;
};

static ps_status snapshot_many(const std::vector<SnapReq> &reqs, hipStream_t st) {
    std::vector<SnapItem<float>> f32;
    std::vector<SnapItem<double>> f64;
    ListBuilder<NormItem> nb;
    bool any_norm = false;
    for (const SnapReq &r : reqs) {
        ps_solver *s = r.s;
        const auto &d = s->g->desc;
        const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
        const int nbk = norm_blocks(n);
        double *part = reinterpret_cast<double *>(s->ws + s->L.npart);
        any_norm = any_norm || r.do_norm;
        if (d.dtype == PS_F64) {
            f64.push_back(SnapItem<double>{static_cast<const double *>(s->x),
                                           reinterpret_cast<double *>(s->ws + r.dst), part, n,
                                           r.do_norm, r.do_copy, nbk});
        } else {
            f32.push_back(SnapItem<float>{static_cast<const float *>(s->x),
                                          reinterpret_cast<float *>(s->ws + r.dst), part, n,
                                          r.do_norm, r.do_copy, nbk});
        }
    }
    if (!f32.empty()) PS_TRY(launch_snapshots<float>(f32, st));
    if (!f64.empty()) PS_TRY(launch_snapshots<double>(f64, st));
    if (!any_norm) return PS_OK;
    for (const SnapReq &r : reqs) {
        if (!r.do_norm) continue;
        ps_solver *s = r.s;
        const auto &d = s->g->desc;
        const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
        NormItem ni{reinterpret_cast<const double *>(s->ws + s->L.npart),
                    reinterpret_cast<double *>(s->ws + s->L.stats) + 2 * s->epochs_done, norm_blocks(n)};
        nb.add(ni, 1);
        if (nb.full()) {
            hipLaunchKernelGGL(k_norm_final, dim3(nb.blocks), dim3(kBlock), 0, st, nb.wl);
            PS_LAUNCHED("k_norm_final");
            nb.clear();
        }
    }
    if (!nb.empty()) {
        hipLaunchKernelGGL(k_norm_final, dim3(nb.blocks), dim3(kBlock), 0, st, nb.wl);
        PS_LAUNCHED("k_norm_final");
    }
    return PS_OK;
}

// SAGA table at the run's first iteration: v_j = A_j^T (A_j x - b_j) for every subset j, then
// vbar = sum_j v_j in increasing j.
template <typename T>
static ps_status saga_fill_t(ps_solver *s, hipStream_t st) {
    const ps_geometry *g = s->g;
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    unsigned char *w = s->ws;
    T *tab = reinterpret_cast<T *>(w + s->L.tab);
    for (int j = 0; j < d.n_subsets; ++j) {
        PS_TRY(launch_project(g, j, s->x, nullptr, s->b, w + s->L.sino, w + s->L.pws, s->L.pws_bytes, st));
        PS_TRY(launch_backproject(g, j, w + s->L.sino, tab + static_cast<size_t>(j) * n, BP_OVERWRITE,
                                  nullptr, w + s->L.bws, s->L.bws_bytes, st));
    }
    hipLaunchKernelGGL((k_table_sum<T>), dim3(elementwise_blocks(n)), dim3(kBlock), 0, st, tab,
                       reinterpret_cast<T *>(w + s->L.tsum), d.n_subsets, n);
    PS_LAUNCHED("k_table_sum");
    return PS_OK;
}

constexpr long kBatchTiles = 2048;   // 8 gather workgroups per CU

// A subset's projection and gather backprojection with the projector's reduction pass left to
// the gather (when the plan fuses them): the projector keeps its partial sums in its workspace
// and the gather reads them there.
static void fuse_pair(ProjCall &pc, BackCall &bc, const void *b) {
    if (!gather_fused(pc.g, pc.subset)) return;
    pc.first_pass_only = true;
    bc.y = pc.ws;
    bc.psplit = proj_plan(pc.g, subset_count(pc.g, pc.subset)).split;
    bc.pb = b;
}

// Does iteration s->k take the snapshot branch (xs = x, full gradient)?
static bool snapshot_now(const ps_solver *s, int t) {
    const int est = s->prm.estimator;
    if (est == PS_EST_SVRG) return t == 0;
    if (est == PS_EST_LSVRG) return s->k == s->prm.k0 || s->refresh[t] != 0;
    return false;
}

// One iteration of every handle in `hs`, each stage one batched launch (per kernel variant):
//   snapshot copies (handles taking the snapshot branch, and x of the run's start) -> SAGA table
//   fills (first iteration) -> projections -> backprojections with the fused estimator and
//   ProxSkip step -> FGP prox (handles whose coin is heads) -> epoch-end norms.
// Every handle computes exactly what it computes alone.
static ps_status run_step(const std::vector<ps_solver *> &hs, hipStream_t st,
                          std::vector<ps_solver *> &ending) {
    std::vector<SnapReq> copies;
    std::vector<ps_solver *> fills, refresh_diff;
    std::vector<ProjCall> pc;
    std::vector<BackCall> bc;
    std::vector<FgpCall> fc;
    pc.reserve(hs.size());
    bc.reserve(hs.size());
    for (ps_solver *s : hs) {
        const ps_geometry *g = s->g;
        const auto &P = s->prm;
        const int N = g->desc.n_subsets;
        const int t = static_cast<int>(s->k % N);
        const int est = P.estimator;
        const bool first = s->k == P.k0;
        unsigned char *w = s->ws;
        if (t == 0) {
            s->sub.resize(N);
            s->coin.resize(N);
            draw_sequences(P.seed, s->k, N, N, P.p, s->sub.data(), s->coin.data());
            if (est == PS_EST_LSVRG) {
                s->refresh.resize(N);
                draw_refresh(P.seed, s->k, N, N, s->refresh.data());
            }
        }
        const bool snap = snapshot_now(s, t);
        if (snap) copies.push_back(SnapReq{s, s->L.xs, 0, 1});
        if (first && est != PS_EST_SVRG) copies.push_back(SnapReq{s, s->L.xe, 0, 1});
        if (first && est == PS_EST_SAGA) fills.push_back(s);
        const int i = s->sub[t];
        const bool prox = P.plain_prox_svrg || s->coin[t];
        UpdateArgs up{};
        up.x = s->x;
        up.h = s->h;
        up.gs = est == PS_EST_SAGA ? nullptr : w + s->L.gs;
        up.vout = w + s->L.v;
        up.gamma = P.gamma;
        up.gamma_over_p = P.gamma / P.p;
        up.nsub = static_cast<double>(N);
        up.plain = P.plain_prox_svrg;
        up.coin = s->coin[t];
        const bool diff = s->L.has_dx;
        if (diff) {
            up.xs = w + s->L.xs;
            up.dx = w + s->L.dx;
            if (prox) refresh_diff.push_back(s);   // x is rewritten by the prox: dx after it
        }
        if (est == PS_EST_SAGA) {
            // y = A_i x - b_i; G = N (A_i^T y - v_i) + vbar with the table updated in the epilogue
            const size_t n = static_cast<size_t>(g->desc.nx) * g->desc.ny * g->desc.nz;
            up.tab = w + s->L.tab + static_cast<size_t>(i) * n * g->elem;
            up.tsum = w + s->L.tsum;
            pc.push_back(ProjCall{g, i, s->x, nullptr, s->b, w + s->L.sino, w + s->L.pws, s->L.pws_bytes});
            bc.push_back(BackCall{g, i, w + s->L.sino, nullptr, BP_SAGA, up, w + s->L.bws, s->L.bws_bytes});
            fuse_pair(pc.back(), bc.back(), s->b);
        } else if (snap) {
            // r = A xs - b over all angles, then gs = A^T r fused with the step (G = gs)
            pc.push_back(ProjCall{g, -1, w + s->L.xs, nullptr, s->b, w + s->L.sino, w + s->L.pws, s->L.pws_bytes});
            bc.push_back(BackCall{g, -1, w + s->L.sino, nullptr, BP_SNAPSHOT, up, w + s->L.bws, s->L.bws_bytes});
        } else {
            if (diff)
                pc.push_back(ProjCall{g, i, w + s->L.dx, nullptr, nullptr, w + s->L.sino, w + s->L.pws, s->L.pws_bytes});
            else
                pc.push_back(ProjCall{g, i, s->x, w + s->L.xs, nullptr, w + s->L.sino, w + s->L.pws, s->L.pws_bytes});
            bc.push_back(BackCall{g, i, w + s->L.sino, nullptr, BP_SVRG, up, w + s->L.bws, s->L.bws_bytes});
            fuse_pair(pc.back(), bc.back(), nullptr);
        }
        if (prox) {
            FgpOut fo{};
            fo.x = s->x;
            fo.h = s->h;
            fo.hscale = P.p / P.gamma;
            fo.proxskip = P.plain_prox_svrg ? 2 : 1;
            const double tau = P.plain_prox_svrg ? P.gamma * P.alpha : P.gamma * P.alpha / P.p;
            fc.push_back(FgpCall{g, w + s->L.v, s->dual, tau, P.fgp_inner, P.nonneg, fo, w + s->L.fws, s->L.fws_bytes});
            s->prox_calls++;
        }
        s->k++;
        if (s->k % N == 0) ending.push_back(s);
    }
    // Handles advanced together that fill the chip between them (at least kBatchTiles gather
    // workgroups) take the tallest gather tile, 4 rows per wave: each staged ray window then
    // serves twice the pixels.  Rows per wave decide only which wave computes a pixel, never
    // the order of its sums, so every handle still gets the bits it gets alone (64 x 128^2
    // solves: 21.9k against 20.4k slice-epochs/s).
    if (hs.size() > 1) {
        long tiles = 0;
        for (const BackCall &c : bc)
            if (c.subset >= 0 && back_method(c.g, c.subset) == BP_GATHER)
                tiles += gather_tiles(c.g, c.subset, gather_rows(c.g, c.subset));
        if (tiles >= kBatchTiles)
            for (BackCall &c : bc) c.rows = 4;
    }
    if (!copies.empty()) PS_TRY(snapshot_many(copies, st));
    for (ps_solver *s : fills)
        PS_TRY(s->g->desc.dtype == PS_F64 ? saga_fill_t<double>(s, st) : saga_fill_t<float>(s, st));
    PS_TRY(launch_project_many(pc.data(), static_cast<int>(pc.size()), st));
    PS_TRY(launch_backproject_many(bc.data(), static_cast<int>(bc.size()), st));
    if (!fc.empty()) PS_TRY(launch_fgp_many(fc.data(), static_cast<int>(fc.size()), st));
    for (ps_solver *s : refresh_diff) {
        const auto &d = s->g->desc;
        const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
        if (d.dtype == PS_F64)
            hipLaunchKernelGGL((k_diff<double>), dim3(elementwise_blocks(n)), dim3(kBlock), 0, st,
                               static_cast<const double *>(s->x), reinterpret_cast<const double *>(s->ws + s->L.xs),
                               reinterpret_cast<double *>(s->ws + s->L.dx), n);
        else
            hipLaunchKernelGGL((k_diff<float>), dim3(elementwise_blocks(n)), dim3(kBlock), 0, st,
                               static_cast<const float *>(s->x), reinterpret_cast<const float *>(s->ws + s->L.xs),
                               reinterpret_cast<float *>(s->ws + s->L.dx), n);
        PS_LAUNCHED("k_diff");
    }
    if (!ending.empty()) {
        // ||x_e - x_{e-1}||, ||x_e||: x_{e-1} is the SVRG snapshot, else the kept copy xe
        std::vector<SnapReq> norms;
        for (ps_solver *s : ending)
            norms.push_back(s->prm.estimator == PS_EST_SVRG ? SnapReq{s, s->L.xs, 1, 0}
                                                            : SnapReq{s, s->L.xe, 1, 1});
        PS_TRY(snapshot_many(norms, st));
    }
    return PS_OK;
}

// After the epoch-end norms of `ended` are queued on `st`: count the epochs and send the norms of
// tolerance handles to pinned host memory behind their events.
static ps_status finish_epochs(const std::vector<ps_solver *> &ended, hipStream_t st) {
    for (ps_solver *s : ended) {
        if (s->prm.tol_rel_change > 0.0) {
            const double *src = reinterpret_cast<const double *>(s->ws + s->L.stats) + 2 * s->epochs_done;
            PS_HIP(hipMemcpyAsync(s->pinned, src, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            PS_HIP(hipEventRecord(s->ev, st));
            s->pending = true;
        }
        s->epochs_done++;
    }
    return PS_OK;
}

}  // namespace ps

extern "C" size_t proxskip_workspace_bytes(const ps_geometry *g, const ps_solver_params *p) {
    if (!g || !p) return 0;
    return layout(g, p->n_epochs, p->estimator).total;
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
    const Layout L = layout(g, prm->n_epochs, prm->estimator);
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
    s->pending = false;
    s->ev = nullptr;
    s->pinned = nullptr;
    static std::atomic<uint64_t> next_id{1};
    s->id = next_id.fetch_add(1);
    s->graphs = nullptr;
    if (prm->tol_rel_change > 0.0) {
        // pinned host memory (no device allocation) for the per-epoch tolerance checks
        if (hipHostMalloc(reinterpret_cast<void **>(&s->pinned), 2 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess) {
            if (s->pinned) (void)hipHostFree(s->pinned);
            delete s;
            return fail(PS_EHIP, "could not create the tolerance-check event or host buffer");
        }
    }
    *out = s;
    return PS_OK;
}

namespace ps {

// Lockstep driver shared by solver_epochs and solver_steps.  Handle i runs until it has done
// target[i] epochs (or met its tolerance or budget), for at most max_steps steps.  On return
// no tolerance check is left pending.
static ps_status lockstep(ps_solver *const *handles, int n_handles, const std::vector<int> &target,
                          int64_t max_steps, hipStream_t st) {
    std::vector<ps_solver *> ready;
    bool nonfinite = false;
    int64_t steps = 0;
    for (;;) {
        ready.clear();
        ps_solver *waiting = nullptr;
        for (int i = 0; i < n_handles; ++i) {
            ps_solver *s = handles[i];
            if (s->pending) {
                const hipError_t q = hipEventQuery(s->ev);
                if (q == hipSuccess) {
                    take_norms(s, s->epochs_done - 1, s->pinned[0], s->pinned[1]);
                    s->pending = false;
                    if (s->nonfinite) nonfinite = true;
                } else if (q != hipErrorNotReady) {
                    return fail(PS_EHIP, "hipEventQuery failed: %s", hipGetErrorString(q));
                } else {
                    if (!waiting) waiting = s;
                    continue;
                }
            }
            if (active(s) && s->epochs_done < target[i]) ready.push_back(s);
        }
        if (ready.empty() || steps >= max_steps) {
            if (!waiting) break;
            PS_HIP(hipEventSynchronize(waiting->ev));
            continue;
        }
        std::vector<ps_solver *> ended;
        PS_TRY(run_step(ready, st, ended));
        PS_TRY(finish_epochs(ended, st));
        ++steps;
    }
    if (nonfinite) return fail(PS_ENONFINITE, "non-finite iterate at an epoch end");
    return PS_OK;
}

static ps_status begin_call(ps_solver *const *handles, int32_t n_handles, hipStream_t st) {
    if (n_handles < 0 || (n_handles > 0 && !handles)) return fail(PS_EINVAL, "bad handle list");
    for (int i = 0; i < n_handles; ++i) {
        if (!handles[i]) return fail(PS_EINVAL, "handle %d is null", i);
        if (handles[i]->cancelled) return fail(PS_ECANCELLED, "handle %d was cancelled", i);
        for (int j = 0; j < i; ++j)
            if (handles[j] == handles[i]) return fail(PS_EINVAL, "handle %d appears twice", i);
    }
    for (int i = 0; i < n_handles; ++i) {
        ps_solver *s = handles[i];
        // a tolerance check left over from an earlier call is settled first
        if (s->pending) {
            PS_HIP(hipEventSynchronize(s->ev));
            take_norms(s, s->epochs_done - 1, s->pinned[0], s->pinned[1]);
            s->pending = false;
        }
        s->stream = st;
    }
    return PS_OK;
}

}  // namespace ps

extern "C" ps_status solver_epochs(ps_solver *const *handles, int32_t n_handles, int32_t n_epochs,
                                   void *stream) {
    clear_error();
    if (n_epochs < 0) return fail(PS_EINVAL, "n_epochs must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    PS_TRY(begin_call(handles, n_handles, st));
    std::vector<int> target(n_handles);
    for (int i = 0; i < n_handles; ++i)
        target[i] = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(handles[i]->epochs_done) + n_epochs,
                                                       handles[i]->prm.n_epochs));
    return lockstep(handles, n_handles, target, INT64_MAX, st);
}

extern "C" ps_status solver_steps(ps_solver *const *handles, int32_t n_handles, int32_t n_steps,
                                  void *stream) {
    clear_error();
    if (n_steps < 0) return fail(PS_EINVAL, "n_steps must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    PS_TRY(begin_call(handles, n_handles, st));
    std::vector<int> target(n_handles);
    for (int i = 0; i < n_handles; ++i) target[i] = handles[i]->prm.n_epochs;
    return lockstep(handles, n_handles, target, n_steps, st);
}

namespace ps {

// One round under graph capture: one epoch of every handle in `hs` (all at an epoch start),
// recorded on the cache's capture stream, instantiated (or an earlier graph of the same
// topology updated with the new kernel arguments) and launched on `st`.
static ps_status graph_round(const std::vector<ps_solver *> &hs, hipStream_t st, GraphCache *gc) {
    int steps = 0;
    std::string key;
    for (ps_solver *s : hs) {
        const int N = s->g->desc.n_subsets;
        steps = std::max(steps, N);
        std::vector<uint8_t> coin(N);
        draw_sequences(s->prm.seed, s->k, N, N, s->prm.p, nullptr, coin.data());
        key += std::to_string(s->id) + ":" + std::to_string(N) + ":";
        for (int t = 0; t < N; ++t) key += static_cast<char>('0' + (s->prm.plain_prox_svrg ? 1 : coin[t]));
        if (s->prm.estimator == PS_EST_LSVRG) {
            std::vector<uint8_t> rho(N);
            draw_refresh(s->prm.seed, s->k, N, N, rho.data());
            key += "/";
            for (int t = 0; t < N; ++t) key += static_cast<char>('0' + rho[t]);
        }
        if (s->k == s->prm.k0) key += "/first";
        key += ";";
    }
    if (!gc->capture) PS_HIP(hipStreamCreateWithFlags(&gc->capture, hipStreamNonBlocking));
    PS_HIP(hipStreamBeginCapture(gc->capture, hipStreamCaptureModeRelaxed));
    ps_status rs = PS_OK;
    std::vector<ps_solver *> ended_all, part, ended;
    for (int t = 0; t < steps && rs == PS_OK; ++t) {
        part.clear();
        for (ps_solver *s : hs)
            if (t < s->g->desc.n_subsets) part.push_back(s);
        ended.clear();
        rs = run_step(part, gc->capture, ended);
        ended_all.insert(ended_all.end(), ended.begin(), ended.end());
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(gc->capture, &graph);
    if (rs != PS_OK) {
        if (ec == hipSuccess && graph) (void)hipGraphDestroy(graph);
        return rs;
    }
    if (ec != hipSuccess) return fail(PS_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    for (size_t i = 0; i < gc->execs.size(); ++i) {
        if (gc->execs[i].first != key) continue;
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res{};
        if (hipGraphExecUpdate(gc->execs[i].second, graph, &err_node, &res) == hipSuccess &&
            res == hipGraphExecUpdateSuccess) {
            exec = gc->execs[i].second;
            std::rotate(gc->execs.begin() + i, gc->execs.begin() + i + 1, gc->execs.end());
        } else {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(gc->execs[i].second);
            gc->execs.erase(gc->execs.begin() + i);
        }
        break;
    }
    if (!exec) {
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(PS_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
        }
        if (gc->execs.size() >= kMaxGraphs) {
            (void)hipGraphExecDestroy(gc->execs.front().second);
            gc->execs.erase(gc->execs.begin());
        }
        gc->execs.emplace_back(key, exec);
    }
    (void)hipGraphDestroy(graph);
    PS_HIP(hipGraphLaunch(exec, st));
    return finish_epochs(ended_all, st);
}

}  // namespace ps

extern "C" ps_status solver_epochs_graph(ps_solver *const *handles, int32_t n_handles,
                                         int32_t n_epochs, void *stream) {
    clear_error();
    if (n_epochs < 0) return fail(PS_EINVAL, "n_epochs must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    PS_TRY(begin_call(handles, n_handles, st));
    if (n_handles == 0) return PS_OK;
    for (int i = 0; i < n_handles; ++i) {
        if (handles[i]->k % handles[i]->g->desc.n_subsets != 0)
            return fail(PS_EINVAL, "handle %d is inside an epoch (after solver_steps): finish it with solver_steps or solver_epochs first", i);
    }
    ps_solver *lead = handles[0];
    if (!lead->graphs) {
        lead->graphs = new (std::nothrow) GraphCache();
        if (!lead->graphs) return fail(PS_ENOMEM, "out of host memory");
    }
    std::vector<int> target(n_handles);
    for (int i = 0; i < n_handles; ++i)
        target[i] = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(handles[i]->epochs_done) + n_epochs,
                                                       handles[i]->prm.n_epochs));
    std::vector<ps_solver *> ready;
    bool nonfinite = false;
    for (;;) {
        // tolerance checks of the previous round decide who takes part in the next one
        ready.clear();
        for (int i = 0; i < n_handles; ++i) {
            ps_solver *s = handles[i];
            if (s->pending) {
                PS_HIP(hipEventSynchronize(s->ev));
                take_norms(s, s->epochs_done - 1, s->pinned[0], s->pinned[1]);
                s->pending = false;
                if (s->nonfinite) nonfinite = true;
            }
            if (active(s) && s->epochs_done < target[i]) ready.push_back(s);
        }
        if (ready.empty()) break;
        PS_TRY(graph_round(ready, st, lead->graphs));
    }
    for (int i = 0; i < n_handles; ++i) {
        ps_solver *s = handles[i];
        if (s->pending) {
            PS_HIP(hipEventSynchronize(s->ev));
            take_norms(s, s->epochs_done - 1, s->pinned[0], s->pinned[1]);
            s->pending = false;
            if (s->nonfinite) nonfinite = true;
        }
    }
    if (nonfinite) return fail(PS_ENONFINITE, "non-finite iterate at an epoch end");
    return PS_OK;
}

extern "C" int32_t solver_done(const ps_solver *s) {
    if (!s) return -1;
    return (!s->pending && !active(s)) ? 1 : 0;
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

extern "C" void solver_free(ps_solver *s) {
    if (!s) return;
    if (s->ev) {
        (void)hipEventSynchronize(s->ev);
        (void)hipEventDestroy(s->ev);
    }
    if (s->pinned) (void)hipHostFree(s->pinned);
    if (s->graphs) {
        // graphs launched on the handle's stream may still run
        (void)hipStreamSynchronize(s->stream);
        delete s->graphs;
    }
    delete s;
}

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

// ---------------------------------------------------------------------------------------------
// proxskip_svrg_run without a caller workspace: the solver's scratch (snapshot, its gradient, the
// prox argument, one sinogram, projector partial sums, backprojector partial images, FGP
// buffers, epoch norms) lives in a fixed device array of this file, one per GPU, for callers
// that cannot allocate device memory.  Host code never names the array in a launch or copy: its
// device address is looked up once per device (hipGetSymbolAddress, with that device current)
// and that address is what the kernels receive.  Every region of the solver workspace is written
// before it is read (the workspace entry point takes uninitialised memory too), so nothing has
// to be cleared between calls.
// ---------------------------------------------------------------------------------------------
namespace ps {

constexpr size_t kStaticScratchBytes = static_cast<size_t>(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mutex;
static unsigned char *g_scratch_ptr[kMaxDevices];

// Device address of this GPU's scratch array (the current device's), looked up on first use.
static ps_status static_scratch(unsigned char **out) {
    int dev = -1;
    PS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PS_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PS_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return PS_OK;
}

}  // namespace ps

extern "C" size_t proxskip_noalloc_max_bytes(void) { return ps::kStaticScratchBytes; }

extern "C" ps_status proxskip_svrg_run_noalloc(const ps_geometry *g, const void *b, void *x, void *h,
                                               void *dual, const ps_solver_params *prm,
                                               ps_solver_stats *stats_out, void *stream) {
    clear_error();
    if (!g) return fail(PS_EINVAL, "geometry is null");
    PS_TRY(check_params(g, prm));
    if (prm->tol_rel_change > 0.0)
        return fail(PS_EINVAL, "proxskip_svrg_run_noalloc runs a fixed number of epochs: "
                               "tol_rel_change must be 0 (the tolerance check needs pinned host memory)");
    const size_t need = layout(g, prm->n_epochs, prm->estimator).total;
    if (need > kStaticScratchBytes)
        return fail(PS_EINVAL, "proxskip_svrg_run_noalloc: this problem needs %zu bytes of scratch, "
                               "the static scratch holds %zu", need, kStaticScratchBytes);
    unsigned char *ws = nullptr;
    PS_TRY(static_scratch(&ws));
    return proxskip_svrg_run(g, b, x, h, dual, prm, stats_out, ws, kStaticScratchBytes, stream);
}

// ---------------------------------------------------------------------------------------------
// FISTA (Beck & Teboulle 2009): per iteration one all-angle projection of y with the residual
// fused (r = A y - b), one all-angle backprojection with the gradient step fused
// (v = y - gamma A^T r), the FGP prox of v into xn, and the extrapolation y = xn + beta (xn - x).
// ---------------------------------------------------------------------------------------------
namespace ps {

struct FistaLayout {
    size_t v, xn, sino, pws, bws, fws, total;
    size_t pws_bytes, bws_bytes, fws_bytes;
};

static FistaLayout fista_layout(const ps_geometry *g) {
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    const size_t m = static_cast<size_t>(d.nz) * d.n_angles * d.n_bins;
    FistaLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    L.v = take(n * g->elem);
    L.xn = take(n * g->elem);
    L.sino = take(m * g->elem);
    L.pws_bytes = proj_workspace(g, d.n_angles);
    L.pws = take(L.pws_bytes);
    L.bws_bytes = back_workspace(g, -1);
    L.bws = take(L.bws_bytes);
    L.fws_bytes = fgp_workspace(g);
    L.fws = take(L.fws_bytes);
    L.total = off;
    return L;
}

template <typename T>
static ps_status fista_momentum(void *x, const void *xn, void *y, double beta, size_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_fista_momentum<T>), dim3(elementwise_blocks(n)), dim3(kBlock), 0, st,
                       static_cast<T *>(x), static_cast<const T *>(xn), static_cast<T *>(y),
                       static_cast<T>(beta), n);
    PS_LAUNCHED("k_fista_momentum");
    return PS_OK;
}

}  // namespace ps

extern "C" size_t fista_workspace_bytes(const ps_geometry *g) {
    if (!g) return 0;
    return fista_layout(g).total;
}

extern "C" ps_status fista_run(const ps_geometry *g, const void *b, void *x, void *y, void *dual,
                               double *t_io, double gamma, double alpha, int32_t fgp_inner,
                               int32_t nonneg, int32_t n_iters, void *workspace, size_t ws_bytes,
                               void *stream) {
    clear_error();
    if (!g) return fail(PS_EINVAL, "geometry is null");
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(PS_EINVAL, "gamma must be > 0");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(PS_EINVAL, "alpha must be >= 0");
    if (fgp_inner < 0) return fail(PS_EINVAL, "fgp_inner must be >= 0");
    if (nonneg != 0 && nonneg != 1) return fail(PS_EINVAL, "nonneg must be 0 or 1");
    if (n_iters < 0) return fail(PS_EINVAL, "n_iters must be >= 0");
    if (!t_io || !(*t_io >= 1.0) || !std::isfinite(*t_io)) return fail(PS_EINVAL, "t must point to a value >= 1");
    PS_TRY(check_ready(g));
    PS_TRY(check_ptr(b, "b", g->elem));
    PS_TRY(check_ptr(x, "x", g->elem));
    PS_TRY(check_ptr(y, "y", g->elem));
    PS_TRY(check_ptr(dual, "dual", g->elem));
    PS_TRY(check_ptr(workspace, "workspace", kAlign));
    const FistaLayout L = fista_layout(g);
    if (ws_bytes < L.total)
        return fail(PS_EINVAL, "FISTA workspace: %zu bytes given, %zu needed", ws_bytes, L.total);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    unsigned char *w = static_cast<unsigned char *>(workspace);
    double t = *t_io;
    for (int k = 0; k < n_iters; ++k) {
        PS_TRY(launch_project(g, -1, y, nullptr, b, w + L.sino, w + L.pws, L.pws_bytes, st));
        UpdateArgs up{};
        up.x = y;
        up.vout = w + L.v;
        up.gamma = gamma;
        PS_TRY(launch_backproject(g, -1, w + L.sino, nullptr, BP_GRADSTEP, &up, w + L.bws, L.bws_bytes, st));
        FgpOut fo{};
        fo.z = w + L.xn;
        fo.proxskip = 0;
        PS_TRY(launch_fgp(g, w + L.v, dual, gamma * alpha, fgp_inner, nonneg, fo, w + L.fws, L.fws_bytes, st));
        const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        const double beta = (t - 1.0) / tn;
        PS_TRY(d.dtype == PS_F64 ? fista_momentum<double>(x, w + L.xn, y, beta, n, st)
                                 : fista_momentum<float>(x, w + L.xn, y, beta, n, st));
        t = tn;
    }
    *t_io = t;
    return PS_OK;
}
