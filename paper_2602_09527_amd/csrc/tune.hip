// tune.hip -- launch plans of a geometry: query, override, and the autotuner that times candidate
// plans on the device and keeps the fastest.
//
// What is tuned: the projector's ray split (partial sums over S workgroups per ray, then a fixed
// order reduction), the backprojector's method, angle groups G and strip height R (or the
// gather's tile), whether a subset gather adds the projector's partials itself, and the FGP
// tiles and inner iterations per launch (temporal blocking depth).  None of them changes what is
// computed; split and grouping change the order of floating-point sums.
#include <algorithm>
#include <array>
#include <functional>
#include <utility>
#include <vector>

#include "internal.h"

namespace ps {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tune_fill(T *__restrict__ p, size_t n) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock)
        p[e] = static_cast<T>(1.0 + 0.001 * static_cast<double>(e % 997));
}

static ps_status fill(const ps_geometry *g, void *p, size_t n, hipStream_t st) {
    const unsigned blocks = static_cast<unsigned>(std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, 4096)));
    if (g->desc.dtype == PS_F64)
        hipLaunchKernelGGL((k_tune_fill<double>), dim3(blocks), dim3(kBlock), 0, st, static_cast<double *>(p), n);
    else
        hipLaunchKernelGGL((k_tune_fill<float>), dim3(blocks), dim3(kBlock), 0, st, static_cast<float *>(p), n);
    PS_LAUNCHED("k_tune_fill");
    return PS_OK;
}

static size_t n_image(const ps_geometry *g) {
    return static_cast<size_t>(g->desc.nx) * g->desc.ny * g->desc.nz;
}

static int proj_max_split(const ps_geometry *g) {
    const ProjPlan p = proj_plan(g, g->desc.n_angles);
    return std::max(1, std::max(g->desc.nx, g->desc.ny) / (2 * p.strip));
}

// All-angle launches are tuned only when they are short (they run once per epoch, at the
// snapshot); beyond this many samples (A B max(nx, ny) nz) the automatic plan is kept and the
// scratch is sized for single subsets only.
constexpr double kFullTuneSamples = 4.0e9;
// Backprojector angle groups tried on images above this many voxels (2 x G partial images).
constexpr size_t kBigImage = static_cast<size_t>(1) << 26;

static bool tune_full(const ps_geometry *g) {
    const auto &d = g->desc;
    return static_cast<double>(d.n_angles) * d.n_bins * std::max(d.nx, d.ny) * d.nz <= kFullTuneSamples;
}

static int max_groups(const ps_geometry *g) { return n_image(g) > kBigImage ? 4 : 16; }

struct TuneLayout {
    size_t x, y, img, pws, bws, fws, dual, total;
    size_t xs, dx, h, gs, v;   // the other images a solver iteration reads or writes
    size_t pws_bytes, bws_bytes, fws_bytes;
};

static TuneLayout tune_layout(const ps_geometry *g) {
    const auto &d = g->desc;
    const size_t n = n_image(g);
    // all angles when they are tuned, or when the all-angle method is chosen (gather allowed)
    const int a_tuned = tune_full(g) || g->gather_ok ? d.n_angles : max_subset_count(g);
    const size_t m = static_cast<size_t>(d.nz) * a_tuned * d.n_bins;
    TuneLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    L.x = take(n * g->elem);
    L.y = take(m * g->elem);
    L.img = take(n * g->elem);
    // the largest split any candidate can take, for the largest call tuned
    L.pws_bytes = align_up(static_cast<size_t>(proj_max_split(g)) * m * g->elem);
    L.pws = take(L.pws_bytes);
    // 2 angle classes x the most groups tried, of partial images
    L.bws_bytes = align_up(2 * static_cast<size_t>(max_groups(g)) * n * g->elem);
    L.bws = take(L.bws_bytes);
    L.fws_bytes = fgp_workspace(g);
    L.fws = take(L.fws_bytes);
    L.dual = take(static_cast<size_t>(g->tv_dims) * n * g->elem);
    L.xs = take(n * g->elem);
    L.dx = take(n * g->elem);
    L.h = take(n * g->elem);
    L.gs = take(n * g->elem);
    L.v = take(n * g->elem);
    L.total = off;
    return L;
}

// The projection and backprojection of a solver iteration, on the tuning workspace: a subset's
// projection reads x and the snapshot xs (or the kept difference image alone, where the solver
// keeps one) and its backprojection applies the SVRG step; all angles project xs and apply the
// snapshot step.  Candidates are timed as the solver runs them, epilogue included (the gather
// applies it in its own launch, the scatter in its combine pass).  x is the image at L.img.
static ProjCall tune_projection(const ps_geometry *g, int subset, const TuneLayout &L, unsigned char *w) {
    if (subset < 0) return ProjCall{g, -1, w + L.xs, nullptr, nullptr, w + L.y, w + L.pws, L.pws_bytes};
    if (solver_reads_one_image(g)) return ProjCall{g, subset, w + L.dx, nullptr, nullptr, w + L.y, w + L.pws, L.pws_bytes};
    return ProjCall{g, subset, w + L.img, w + L.xs, nullptr, w + L.y, w + L.pws, L.pws_bytes};
}

static BackCall tune_backprojection(const ps_geometry *g, int subset, const TuneLayout &L, unsigned char *w) {
    BackCall c{};
    c.g = g;
    c.subset = subset;
    c.y = w + L.y;
    c.out = w + L.img;
    c.mode = subset < 0 ? BP_SNAPSHOT : BP_SVRG;
    c.upd.x = w + L.img;
    c.upd.h = w + L.h;
    c.upd.gs = w + L.gs;
    c.upd.vout = w + L.v;
    if (solver_reads_one_image(g)) {
        c.upd.xs = w + L.xs;
        c.upd.dx = w + L.dx;
    }
    c.upd.gamma = 1e-9;          // tiny steps: the repeated calls keep x finite
    c.upd.gamma_over_p = 1e-8;
    c.upd.nsub = static_cast<double>(g->desc.n_subsets);
    c.ws = w + L.bws;
    c.ws_bytes = L.bws_bytes;
    return c;
}

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Milliseconds per call of fn: the median of three rounds of `reps` calls, after one warm-up call.
template <typename F>
static ps_status time_calls(F &&fn, int reps, hipStream_t st, Timer &tm, float *ms) {
    PS_TRY(fn());
    float t[3];
    for (int round = 0; round < 3; ++round) {
        PS_HIP(hipEventRecord(tm.e0, st));
        for (int r = 0; r < reps; ++r) PS_TRY(fn());
        PS_HIP(hipEventRecord(tm.e1, st));
        PS_HIP(hipEventSynchronize(tm.e1));
        PS_HIP(hipEventElapsedTime(&t[round], tm.e0, tm.e1));
        t[round] /= static_cast<float>(std::max(reps, 1));
    }
    std::sort(t, t + 3);
    *ms = t[1];
    return PS_OK;
}

// A candidate replaces the automatic plan (always the first candidate timed) only when it is
// at least this much faster, so timing noise does not move plans between runs.
constexpr float kMinGain = 0.97f;

// An all-angle launch (run once per epoch, at the snapshot) longer than this keeps the automatic
// plan: timing its alternatives would cost seconds on volumes.
constexpr float kLongLaunchMs = 5.0f;

}  // namespace ps

using namespace ps;

extern "C" ps_status geometry_get_plan(const ps_geometry *g, ps_plan *out) {
    clear_error();
    if (!g || !out) return fail(PS_EINVAL, "null argument");
    const int A = g->desc.n_angles;
    out->proj_split_full = proj_plan(g, A).split;
    out->proj_split_subset = proj_plan(g, max_subset_count(g)).split;
    const BackPlan bf = back_plan(g, -1), bs = back_plan(g, 0);
    out->bp_groups_full = bf.groups;
    out->bp_groups_subset = bs.groups;
    out->bp_strip_full = bf.strip;
    out->bp_strip_subset = bs.strip;
    out->fgp_iters = fgp_iters_per_launch(g);
    out->bp_method_full = back_method(g, -1);
    out->bp_method_subset = back_method(g, 0);
    out->bp_gather_rows = gather_rows(g, 0);
    out->bp_gather_split = gather_split(g, 0);
    out->fgp_cols = fgp_cols_of(g);
    out->bp_gather_fused = gather_fused(g, 0) ? 2 : 1;
    out->fgp3d_chunk = fgp3d_chunk_of(g);
    fgp_tile_of(g, &out->fgp_waves, &out->fgp_rows);
    out->fgp3d_form = fgp3d_form_of(g);
    return PS_OK;
}

extern "C" ps_status geometry_set_plan(ps_geometry *g, const ps_plan *p) {
    clear_error();
    if (!g || !p) return fail(PS_EINVAL, "null argument");
    auto strip_ok = [](int s) { return s == 0 || s == 1 || s == 2 || s == 4 || s == 8; };
    if (p->proj_split_full < 0 || p->proj_split_full > 64 || p->proj_split_subset < 0 ||
        p->proj_split_subset > 64)
        return fail(PS_EINVAL, "projector split must be in [0, 64]");
    if (p->bp_groups_full < 0 || p->bp_groups_full > 16 || p->bp_groups_subset < 0 ||
        p->bp_groups_subset > 16)
        return fail(PS_EINVAL, "backprojector groups must be in [0, 16]");
    if (!strip_ok(p->bp_strip_full) || !strip_ok(p->bp_strip_subset))
        return fail(PS_EINVAL, "backprojector strip must be 0, 1, 2, 4 or 8");
    if (p->fgp_iters < 0 || p->fgp_iters > fgp_max_iters_of(g))
        return fail(PS_EINVAL, "fgp_iters must be in [0, %d]", fgp_max_iters_of(g));
    if (p->bp_method_full < 0 || p->bp_method_full > 2 || p->bp_method_subset < 0 || p->bp_method_subset > 2)
        return fail(PS_EINVAL, "bp_method must be 0 (automatic), 1 (scatter) or 2 (gather)");
    if (p->bp_gather_rows != 0 && p->bp_gather_rows != 2 && p->bp_gather_rows != 4)
        return fail(PS_EINVAL, "bp_gather_rows must be 0, 2 or 4");
    if (p->bp_gather_split != 0 && p->bp_gather_split != 1 && p->bp_gather_split != 2 && p->bp_gather_split != 4)
        return fail(PS_EINVAL, "bp_gather_split must be 0, 1, 2 or 4");
    if (p->fgp_cols < 0 || p->fgp_cols > 2) return fail(PS_EINVAL, "fgp_cols must be 0, 1 or 2");
    if (p->bp_gather_fused < 0 || p->bp_gather_fused > 2)
        return fail(PS_EINVAL, "bp_gather_fused must be 0, 1 or 2");
    if (p->fgp3d_chunk < 0 || p->fgp3d_chunk > 256) return fail(PS_EINVAL, "fgp3d_chunk must be in [0, 256]");
    if (p->fgp3d_form < 0 || p->fgp3d_form > kF3Forms) return fail(PS_EINVAL, "fgp3d_form must be in [0, %d]", kF3Forms);
    if (!(p->fgp_waves == 0 && p->fgp_rows == 0) && !fgp_tile_ok(p->fgp_waves, p->fgp_rows))
        return fail(PS_EINVAL, "FGP tile %d x %d: waves x rows must be 4x4, 4x8, 8x2, 8x4, 8x8, 16x2, 16x4 or 0x0",
                    p->fgp_waves, p->fgp_rows);
    g->plan = *p;
    return PS_OK;
}

extern "C" size_t geometry_autotune_workspace_bytes(const ps_geometry *g) {
    return g ? tune_layout(g).total : 0;
}

extern "C" ps_status geometry_autotune(ps_geometry *g, void *workspace, size_t ws_bytes,
                                       int32_t reps, void *stream, ps_plan *out) {
    clear_error();
    PS_TRY(check_ready(g));
    PS_TRY(check_ptr(workspace, "workspace", kAlign));
    if (reps < 1) return fail(PS_EINVAL, "reps must be >= 1");
    const TuneLayout L = tune_layout(g);
    if (ws_bytes < L.total)
        return fail(PS_EINVAL, "autotune workspace: %zu bytes given, %zu needed", ws_bytes, L.total);
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char *w = static_cast<unsigned char *>(workspace);
    const auto &d = g->desc;
    const size_t n = n_image(g);
    Timer tm;
    PS_HIP(hipEventCreate(&tm.e0));
    PS_HIP(hipEventCreate(&tm.e1));
    PS_TRY(fill(g, w + L.x, n, st));
    PS_TRY(fill(g, w + L.y, static_cast<size_t>(d.nz) * d.n_angles * d.n_bins, st));
    for (size_t off : {L.img, L.xs, L.dx, L.h, L.gs, L.v}) PS_TRY(fill(g, w + off, n, st));

    ps_plan best = g->plan;
    const ps_plan saved = g->plan;
    auto restore_on_error = [&](ps_status s) {
        if (s != PS_OK) g->plan = saved;
        return s;
    };
    const int splits[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
    const int max_split = proj_max_split(g);

    const int first_pass = tune_full(g) ? 1 : 0;
    // projector: all angles (when short), then subset 0
    for (int full = first_pass; full >= 0; --full) {
        const int subset = full ? -1 : 0;
        float best_ms = 0.f;
        int best_s = 0;
        bool have = false;
        std::vector<std::pair<float, int>> timed;   // (ms, split)
        g->plan = best;
        const int auto_split = full ? proj_plan(g, d.n_angles).split : proj_plan(g, max_subset_count(g)).split;
        std::vector<int> cand{auto_split};
        for (int s : splits)
            if (s <= max_split && s != auto_split) cand.push_back(s);
        const int r = reps;
        for (size_t c = 0; c < cand.size(); ++c) {
            ps_plan trial = best;
            (full ? trial.proj_split_full : trial.proj_split_subset) = cand[c];
            g->plan = trial;
            float ms = 0.f;
            const ProjCall pc = tune_projection(g, subset, L, w);
            PS_TRY(restore_on_error(time_calls([&] { return launch_project_many(&pc, 1, st); }, r, st, tm, &ms)));
            if (!have || ms < best_ms * (best_s == cand[0] ? kMinGain : 1.0f)) {
                best_ms = ms;
                best_s = cand[c];
                have = true;
            }
            timed.push_back({ms, cand[c]});
            if (c == 0 && full && ms > kLongLaunchMs) break;
        }
        // the pick gives way to a smaller split within 3% of its time (the timing noise): every
        // split writes one partial sum per ray, most of the launch's HBM traffic
        const float limit = best_ms / kMinGain;
        for (const auto &t : timed)
            if (t.second < best_s && t.first <= limit) best_s = t.second;
        (full ? best.proj_split_full : best.proj_split_subset) = best_s;
    }

    // backprojector: scatter with (strip, groups), or the gather, for all angles (when short)
    // then subset 0.  For subsets the fastest scatter plan and the fastest gather tile are kept
    // for the pair stage below, which decides between them.
    std::array<int, 3> sub_scatter{}, sub_gather{};
    bool have_scatter = false, have_gather = false;
    bool full_untuned = !tune_full(g);   // all-angle candidates not timed (too long)
    for (int full = first_pass; full >= 0; --full) {
        const int subset = full ? -1 : 0;
        g->plan = best;
        const int auto_method = back_method(g, subset);
        const BackPlan auto_bp = back_plan(g, subset);
        // candidate (method, strip, groups) or (gather, rows, angle split); the automatic first
        std::vector<std::array<int, 3>> cand;
        const int auto_rows = gather_rows(g, subset), auto_split = gather_split(g, subset);
        if (auto_method == BP_GATHER) cand.push_back({BP_GATHER, auto_rows, auto_split});
        cand.push_back({BP_SCATTER, auto_bp.strip, auto_bp.groups});
        for (int s : {8, 4, 2})
            for (int G : {1, 2, 4, 8, 16})
                if (G <= max_groups(g) && !(s == auto_bp.strip && G == auto_bp.groups))
                    cand.push_back({BP_SCATTER, s, G});
        if (g->gather_ok)
            for (int rows : {2, 4})
                for (int split : {1, 2, 4})
                    if (!(auto_method == BP_GATHER && rows == auto_rows && split == auto_split))
                        cand.push_back({BP_GATHER, rows, split});
        float best_ms = 0.f;
        std::array<int, 3> pick = cand[0];
        bool have = false;
        std::vector<std::pair<float, size_t>> timed;   // (ms, candidate)
        const int r = reps;
        for (size_t c = 0; c < cand.size(); ++c) {
            ps_plan trial = best;
            int &m = full ? trial.bp_method_full : trial.bp_method_subset;
            int &st_ = full ? trial.bp_strip_full : trial.bp_strip_subset;
            int &gr = full ? trial.bp_groups_full : trial.bp_groups_subset;
            m = cand[c][0];
            if (cand[c][0] == BP_SCATTER) {
                st_ = cand[c][1];
                gr = cand[c][2];
            } else {
                trial.bp_gather_rows = cand[c][1];
                trial.bp_gather_split = cand[c][2];
            }
            g->plan = trial;
            if (cand[c][0] == BP_SCATTER) {
                const BackPlan bp = back_plan(g, subset);
                // skip candidates the LDS budget or the angle count clamps to one already timed
                if (c > 0 && (bp.strip != cand[c][1] || bp.groups != cand[c][2])) continue;
                if (back_workspace(g, subset) > L.bws_bytes) continue;
            }
            float ms = 0.f;
            const BackCall bc = tune_backprojection(g, subset, L, w);
            PS_TRY(restore_on_error(time_calls([&] { return launch_backproject_many(&bc, 1, st); }, r, st, tm, &ms)));
            timed.push_back({ms, c});
            if (c == 0 && full && ms > kLongLaunchMs) {
                full_untuned = true;
                break;
            }
        }
        // the method and plan: the automatic one unless another is 3% faster, else the fastest
        for (const auto &t : timed) {
            if (!have || t.first < best_ms * (pick == cand[0] ? kMinGain : 1.0f)) {
                best_ms = t.first;
                pick = cand[t.second];
                have = true;
            }
        }
        // a scatter pick gives way to a scatter plan with fewer angle groups that is within 3%
        // of it (the timing noise): each group writes its own partial images, whose bytes are
        // most of the launch's HBM traffic
        if (pick[0] == BP_SCATTER) {
            const float limit = best_ms / kMinGain;
            for (const auto &t : timed) {
                const std::array<int, 3> &k = cand[t.second];
                if (k[0] != BP_SCATTER || t.first > limit) continue;
                if (k[2] < pick[2] || (k[2] == pick[2] && t.first < best_ms)) {
                    best_ms = t.first;
                    pick = k;
                }
            }
        }
        if (!full) {
            float sc_ms = 0.f, ga_ms = 0.f;
            for (const auto &t : timed) {
                const std::array<int, 3> &k = cand[t.second];
                if (k[0] == BP_SCATTER && (!have_scatter || t.first < sc_ms)) {
                    sc_ms = t.first;
                    sub_scatter = k;
                    have_scatter = true;
                } else if (k[0] == BP_GATHER && (!have_gather || t.first < ga_ms)) {
                    ga_ms = t.first;
                    sub_gather = k;
                    have_gather = true;
                }
            }
            for (const auto &t : timed) {   // fewer angle groups within 3%, as above
                const std::array<int, 3> &k = cand[t.second];
                if (k[0] == BP_SCATTER && t.first <= sc_ms / kMinGain && k[2] < sub_scatter[2]) sub_scatter = k;
            }
        }
        if (full) {
            best.bp_method_full = pick[0];
            if (pick[0] == BP_SCATTER) {
                best.bp_strip_full = pick[1];
                best.bp_groups_full = pick[2];
            }
        } else {
            best.bp_method_subset = pick[0];
            if (pick[0] == BP_SCATTER) {
                best.bp_strip_subset = pick[1];
                best.bp_groups_subset = pick[2];
            } else {
                best.bp_gather_rows = pick[1];   // the subset calls dominate: their tile
                best.bp_gather_split = pick[2];
            }
        }
    }

    // A subset's projection and backprojection as a solver iteration runs them (the pair), which
    // decides the subset method where the gather applies: the scatter (fastest plan above) at
    // every projector split, and the gather (fastest tile above) at every split with the
    // reduction pass or (split > 1) adding the partials itself; then, if the gather wins, every
    // gather tile (rows per wave, angle split) at the split chosen.  The plan chosen so far is
    // timed first and is the one to beat; pairs are short, so each is timed over enough calls to
    // fill about 5 ms.
    g->plan = best;
    if (have_gather) {
        // {method, projector split, fused, strip or rows, groups or angle split}
        using Pair = std::array<int, 5>;
        auto plan_of = [&](const Pair &k) {
            ps_plan t = best;
            t.bp_method_subset = k[0];
            t.proj_split_subset = k[1];
            t.bp_gather_fused = k[2];
            if (k[0] == BP_SCATTER) {
                t.bp_strip_subset = k[3];
                t.bp_groups_subset = k[4];
            } else {
                t.bp_gather_rows = k[3];
                t.bp_gather_split = k[4];
            }
            return t;
        };
        auto time_pair = [&](const Pair &k, int r, float *ms) -> ps_status {
            g->plan = plan_of(k);
            ProjCall pc = tune_projection(g, 0, L, w);
            BackCall bc = tune_backprojection(g, 0, L, w);
            if (gather_fused(g, 0)) {
                pc.first_pass_only = true;
                bc.y = w + L.pws;
                bc.psplit = proj_plan(g, subset_count(g, 0)).split;
            }
            return time_calls([&] {
                PS_TRY(launch_project_many(&pc, 1, st));
                return launch_backproject_many(&bc, 1, st);
            }, r, st, tm, ms);
        };
        const int m0 = back_method(g, 0);
        const BackPlan bp0 = back_plan(g, 0);
        const Pair first{m0, proj_plan(g, max_subset_count(g)).split, gather_fused(g, 0) ? 2 : 1,
                         m0 == BP_SCATTER ? bp0.strip : gather_rows(g, 0),
                         m0 == BP_SCATTER ? bp0.groups : gather_split(g, 0)};
        float est = 0.f;
        PS_TRY(restore_on_error(time_pair(first, reps, &est)));
        const int r = std::max(reps, std::min(100, static_cast<int>(5.0f / std::max(est, 1e-3f))));
        float best_ms = 0.f;
        Pair pick = first;
        PS_TRY(restore_on_error(time_pair(first, r, &best_ms)));
        auto consider = [&](const Pair &k) -> ps_status {
            if (k == first) return PS_OK;
            g->plan = plan_of(k);
            if (proj_plan(g, max_subset_count(g)).split != k[1]) return PS_OK;   // clamped
            if (back_method(g, 0) != k[0]) return PS_OK;
            if (k[0] == BP_SCATTER && back_workspace(g, 0) > L.bws_bytes) return PS_OK;
            float ms = 0.f;
            PS_TRY(time_pair(k, r, &ms));
            if (ms < best_ms * (pick == first ? kMinGain : 1.0f)) {
                best_ms = ms;
                pick = k;
            }
            return PS_OK;
        };
        for (int s : splits) {
            if (s > max_split) continue;
            if (have_scatter)
                PS_TRY(restore_on_error(consider({BP_SCATTER, s, 1, sub_scatter[1], sub_scatter[2]})));
            for (int f : {1, 2})
                if (f == 1 || s > 1)
                    PS_TRY(restore_on_error(consider({BP_GATHER, s, f, sub_gather[1], sub_gather[2]})));
        }
        if (pick[0] == BP_GATHER) {
            const int split_pick = pick[1];
            for (int rows : {2, 4})
                for (int as : {1, 2, 4})
                    for (int f : {1, 2})
                        if (f == 1 || split_pick > 1)
                            PS_TRY(restore_on_error(consider({BP_GATHER, split_pick, f, rows, as})));
        }
        best = plan_of(pick);
    }

    // All-angle backprojection too long to tune fully (it runs once per epoch, at the snapshot):
    // the plan's method against the gather on the tile chosen above, one timed call each.  On the
    // 1024^2 x 256 volume the gather took 356 ms against the scatter's 414.
    if (full_untuned && g->gather_ok) {
        g->plan = best;
        const int m0 = back_method(g, -1);
        float ms0 = 0.f, ms1 = 0.f;
        const BackCall b0 = tune_backprojection(g, -1, L, w);
        if (m0 == BP_GATHER || back_workspace(g, -1) <= L.bws_bytes) {
            PS_TRY(restore_on_error(time_calls([&] { return launch_backproject_many(&b0, 1, st); }, 1, st, tm, &ms0)));
            ps_plan trial = best;
            trial.bp_method_full = m0 == BP_GATHER ? BP_SCATTER : BP_GATHER;
            g->plan = trial;
            if (trial.bp_method_full == BP_GATHER || back_workspace(g, -1) <= L.bws_bytes) {
                const BackCall b1 = tune_backprojection(g, -1, L, w);
                PS_TRY(restore_on_error(time_calls([&] { return launch_backproject_many(&b1, 1, st); }, 1, st, tm, &ms1)));
                if (ms1 < ms0 * kMinGain) best.bp_method_full = trial.bp_method_full;
            }
        }
    }

    // 2D FGP tile shape and inner iterations per launch: one 50-iteration prox per timed call;
    // the automatic plan (tile and depth) is timed first and is the one to beat
    if (g->tv_dims == 2) {
        PS_TRY(fill(g, w + L.dual, 2 * n, st));
        g->plan = best;
        g->plan.fgp_waves = g->plan.fgp_rows = g->plan.fgp_iters = g->plan.fgp_cols = 0;
        int auto_w, auto_r;
        fgp_tile_of(g, &auto_w, &auto_r);
        const int auto_t = fgp_iters_per_launch(g), auto_c = fgp_cols_of(g);
        std::vector<std::array<int, 4>> cands{{auto_w, auto_r, auto_t, auto_c}};
        for (int cx : {1, 2})
            for (int w8 : {4, 8, 16})
                for (int r8 : {2, 4, 8}) {
                    if (!fgp_tile_ok(w8, r8)) continue;
                    const int cap = std::min(fgp_max_iters_of(g), w8 * r8 / 2 - 2);
                    for (int T = cap; T >= 2; --T)
                        if (!(w8 == auto_w && r8 == auto_r && T == auto_t && cx == auto_c))
                            cands.push_back({w8, r8, T, cx});
                }
        float best_ms = 0.f;
        int pick_t = 0, pick_w = 0, pick_r = 0, pick_c = 0;
        bool auto_best = true;
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            ps_plan trial = best;
            trial.fgp_waves = cands[ci][0];
            trial.fgp_rows = cands[ci][1];
            trial.fgp_iters = cands[ci][2];
            trial.fgp_cols = cands[ci][3];
            g->plan = trial;
            FgpOut o{};
            o.z = w + L.img;
            float ms = 0.f;
            PS_TRY(restore_on_error(time_calls([&] {
                return launch_fgp(g, w + L.x, w + L.dual, 1e-3, 50, 1, o, w + L.fws, L.fws_bytes, st);
            }, reps, st, tm, &ms)));
            if (ci == 0 || ms < best_ms * (auto_best ? kMinGain : 1.0f)) {
                best_ms = ms;
                pick_w = cands[ci][0];
                pick_r = cands[ci][1];
                pick_t = cands[ci][2];
                pick_c = cands[ci][3];
                auto_best = ci == 0;
            }
        }
        best.fgp_iters = pick_t;
        best.fgp_waves = pick_w;
        best.fgp_rows = pick_r;
        best.fgp_cols = pick_c;
    }
    // 3D FGP: launch form and slices per workgroup (10 inner iterations per timed call); the
    // automatic form with chunks of 16 is timed first
    if (g->tv_dims == 3) {
        PS_TRY(fill(g, w + L.dual, 3 * n, st));
        float best_ms = 0.f;
        int pick_ch = 0, pick_form = 0;
        bool auto_best = true;
        ps_plan automatic = best;
        automatic.fgp3d_form = 0;
        g->plan = automatic;
        const int auto_form = fgp3d_form_of(g);
        std::vector<std::array<int, 2>> cands{{auto_form, 16}};
        for (int form = 2; form <= kF3Forms; ++form)
            for (int ch : {8, 16, 24, 32})
                if (!(form == auto_form && ch == 16)) cands.push_back({form, ch});
        for (int ch : {4, 8, 2, 16}) cands.push_back({1, ch});
        for (const auto &fc : cands) {
            const int form = fc[0], ch = fc[1];
            ps_plan trial = best;
            trial.fgp3d_chunk = ch;
            trial.fgp3d_form = form;
            g->plan = trial;
            FgpOut o{};
            o.z = w + L.img;
            float ms = 0.f;
            PS_TRY(restore_on_error(time_calls([&] {
                return launch_fgp(g, w + L.x, w + L.dual, 1e-3, 10, 1, o, w + L.fws, L.fws_bytes, st);
            }, reps, st, tm, &ms)));
            if (pick_ch == 0 || ms < best_ms * (auto_best ? kMinGain : 1.0f)) {
                best_ms = ms;
                auto_best = pick_ch == 0;
                pick_ch = ch;
                pick_form = form;
            }
        }
        best.fgp3d_chunk = pick_ch;
        best.fgp3d_form = pick_form;
    }
    g->plan = best;
    if (out) PS_TRY(geometry_get_plan(g, out));
    return PS_OK;
}

// ---------------------------------------------------------------------------------------------
// Measurement support: one kernel class timed alone on synthetic inputs, `reps` back-to-back
// launches between two HIP events (median of three rounds), with the geometry's plan.
// ---------------------------------------------------------------------------------------------
namespace ps {

struct KtLayout {
    size_t x, y, img, pws, bws, total, pws_bytes, bws_bytes;
};

static KtLayout kt_layout(const ps_geometry *g) {
    const auto &d = g->desc;
    const size_t n = n_image(g);
    const size_t m = static_cast<size_t>(d.nz) * d.n_angles * d.n_bins;
    KtLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    L.x = take(n * g->elem);
    L.y = take(m * g->elem);
    L.img = take(n * g->elem);
    L.pws_bytes = std::max(proj_workspace(g, d.n_angles), proj_workspace(g, max_subset_count(g)));
    L.pws = take(L.pws_bytes);
    L.bws_bytes = std::max(back_workspace(g, -1), back_workspace(g, 0));
    L.bws = take(L.bws_bytes);
    L.total = off;
    return L;
}

}  // namespace ps

extern "C" size_t kernel_time_workspace_bytes(const ps_geometry *g) { return g ? kt_layout(g).total : 0; }

extern "C" ps_status kernel_time(const ps_geometry *g, int32_t kernel_class, int32_t reps,
                                 void *workspace, size_t ws_bytes, void *stream, double *us_per_launch) {
    clear_error();
    PS_TRY(check_ready(g));
    PS_TRY(check_ptr(workspace, "workspace", kAlign));
    if (!us_per_launch) return fail(PS_EINVAL, "us_per_launch is null");
    if (reps < 1) return fail(PS_EINVAL, "reps must be >= 1");
    const KtLayout L = kt_layout(g);
    if (ws_bytes < L.total)
        return fail(PS_EINVAL, "kernel_time workspace: %zu bytes given, %zu needed", ws_bytes, L.total);
    const int subset = (kernel_class == KC_BP_SCATTER_FULL || kernel_class == KC_PROJECT_FULL) ? -1 : 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char *w = static_cast<unsigned char *>(workspace);
    std::function<ps_status()> fn;
    if (kernel_class == KC_BP_SCATTER_SUBSET || kernel_class == KC_BP_SCATTER_FULL ||
        kernel_class == KC_BP_GATHER) {
        const bool gather = back_method(g, subset) == BP_GATHER;
        if (gather != (kernel_class == KC_BP_GATHER))
            return fail(PS_EINVAL, "kernel class %d: the plan backprojects %s with the %s", kernel_class,
                        subset < 0 ? "all angles" : "subsets", gather ? "gather" : "scatter");
        BackCall c{};
        c.g = g;
        c.subset = subset;
        c.y = w + L.y;
        c.out = w + L.img;
        c.mode = BP_OVERWRITE;
        c.ws = w + L.bws;
        c.ws_bytes = L.bws_bytes;
        c.partials_only = !gather;   // the scatter kernel alone, without its combine pass
        fn = [=] { return launch_backproject_many(&c, 1, st); };
    } else if (kernel_class == KC_PROJECT_SUBSET || kernel_class == KC_PROJECT_FULL) {
        // subset launches read what the solver's do: x - xs, or the one kept difference image
        const bool two = subset >= 0 && !solver_reads_one_image(g);
        ProjCall c{g, subset, w + L.x, two ? w + L.img : nullptr, nullptr, w + L.y, w + L.pws, L.pws_bytes};
        c.first_pass_only = true;    // the projector kernel alone, without the split-ray sum
        fn = [=] { return launch_project_many(&c, 1, st); };
    } else {
        return fail(PS_EINVAL, "kernel_time supports the projector and backprojector classes, not %d",
                    kernel_class);
    }
    PS_TRY(fill(g, w + L.x, n_image(g), st));
    PS_TRY(fill(g, w + L.img, n_image(g), st));
    PS_TRY(fill(g, w + L.y, static_cast<size_t>(g->desc.nz) * g->desc.n_angles * g->desc.n_bins, st));
    Timer tm;
    PS_HIP(hipEventCreate(&tm.e0));
    PS_HIP(hipEventCreate(&tm.e1));
    float ms = 0.f;
    PS_TRY(time_calls(fn, reps, st, tm, &ms));
    *us_per_launch = 1e3 * static_cast<double>(ms);
    return PS_OK;
}
