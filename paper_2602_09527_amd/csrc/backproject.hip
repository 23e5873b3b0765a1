// backproject.hip -- adjoint x = A_i^T y (K2): the projector's ray walk run backwards.
//
// Every ray deposits, at every step, its value y_u / |cos| (or / |sin|) times the two Joseph
// weights (1 - w, w) on the pixels j0, j0 + 1 it interpolates -- the same fixed-point walk as
// the projector, so A^T is the projector's transpose weight for weight.
//
// Work split.  Row-walked angles deposit along image rows, column-walked angles along columns.
// A workgroup owns a strip of R image rows (row class) or R image columns (column class) of one
// slice, and one of G groups of the subset's angles of that class.  Each of its waves keeps a
// private accumulator strip in LDS and walks whole ray chunks of its angles through the strip:
// 64 lanes = 64 rays that are P bins apart (one "pass"), so the 2 x 64 deposits of one step never
// share a pixel and a plain LDS read-add-write needs no atomics.  The workgroup then adds its
// waves' strips in a fixed order and writes one partial image per (class, group); a combine pass
// adds the 2G partials in a fixed order and applies the epilogue (overwrite, accumulate, or the
// fused SVRG / ProxSkip gradient step).  Results are bitwise reproducible.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace ps {

constexpr int kWave = 64;

BackPlan back_plan(const ps_geometry *g, int subset) {
    const auto &d = g->desc;
    BackPlan p{};
    const int ext = std::max(d.nx, d.ny);
    p.stride = ext + 4;
    p.waves = 4;
    const int forced_strip = subset < 0 ? g->plan.bp_strip_full : g->plan.bp_strip_subset;
    p.strip = forced_strip > 0 ? forced_strip : 8;
    const size_t budget = 80 * 1024;  // two workgroups per CU (160 KB of LDS)
    while (p.strip > 1 && static_cast<size_t>(p.waves) * p.strip * p.stride * g->elem > budget)
        p.strip >>= 1;
    while (p.waves > 1 && static_cast<size_t>(p.waves) * p.strip * p.stride * g->elem > budget)
        p.waves >>= 1;
    p.s_row = (d.ny + p.strip - 1) / p.strip;
    p.s_col = (d.nx + p.strip - 1) / p.strip;
    const int na = subset_count(g, subset);
    const int nrow = subset < 0 ? g->nrow_full : g->nrow_sub[subset];
    const int most = std::max(nrow, na - nrow);
    const long per_group = static_cast<long>(p.s_row + p.s_col) * d.nz;
    long G = (512 + per_group - 1) / per_group;
    const int forced_g = subset < 0 ? g->plan.bp_groups_full : g->plan.bp_groups_subset;
    if (forced_g > 0) G = forced_g;
    G = std::max(1L, std::min<long>(G, std::min(16, std::max(1, most))));
    p.groups = static_cast<int>(G);
    p.lds_bytes = static_cast<size_t>(p.waves) * p.strip * p.stride * g->elem;
    p.part_elems = static_cast<size_t>(2) * p.groups * d.nx * d.ny * d.nz;
    return p;
}

size_t back_workspace(const ps_geometry *g, int subset) {
    return align_up(back_plan(g, subset).part_elems * g->elem);
}

// One backprojector application: partial images of A_sub^T y, one per (angle class, group).
template <typename T>
struct BackItem {
    const T *y;
    T *part;
    const int32_t *order;
    AngleTab<T> tab;
    int subset, nsub, na, nx, ny, nz, nbins, strip, stride, s_row, s_col, groups, passes, nrow;
};

template <typename T, int NP, int kStrip>
__global__ __launch_bounds__(kBlock) void k_backproject(WorkList<BackItem<T>> wl) {
    extern __shared__ unsigned char smem_raw[];
    T *acc_all = reinterpret_cast<T *>(smem_raw);
    constexpr bool kFixed = std::is_same<T, float>::value;
    int local;
    const BackItem<T> &it = wl.item[work_item(wl, local)];
    const T *__restrict__ y = it.y;
    T *__restrict__ part = it.part;
    const int32_t *__restrict__ order = it.order;
    const AngleTab<T> &tab = it.tab;
    const int subset = it.subset, nsub = it.nsub, na = it.na, nx = it.nx, ny = it.ny;
    const int nbins = it.nbins, strip = it.strip, stride = it.stride, s_row = it.s_row;
    const int groups = it.groups, passes = it.passes, nrow = it.nrow;
    const int nw = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    // workgroup -> (strip index, angle group, slice), strip fastest
    const int nstrips = s_row + it.s_col;
    const int sx = local % nstrips, grp = (local / nstrips) % groups, z = local / (nstrips * groups);
    const bool rowc = sx < s_row;
    const int s = rowc ? sx : sx - s_row;
    const int nsteps = rowc ? ny : nx;   // stepping axis of this class
    const int ext = rowc ? nx : ny;      // deposit axis
    const int t_lo = s * strip;
    const int nt = min(strip, nsteps - t_lo);
    const size_t plane = static_cast<size_t>(nx) * ny;
    const T *yz = y + static_cast<size_t>(z) * na * nbins;

    // this class's angles, and this group's share of them
    const int cls_lo = rowc ? 0 : nrow, cls_cnt = rowc ? nrow : na - nrow;
    const int per = (cls_cnt + groups - 1) / groups;
    const int e_lo = cls_lo + grp * per;
    const int e_hi = cls_lo + min(cls_cnt, (grp + 1) * per);

    for (int e = threadIdx.x; e < nw * strip * stride; e += blockDim.x) acc_all[e] = T(0);
    __syncthreads();
    T *acc = acc_all + static_cast<size_t>(wave) * strip * stride;

    const int span = kWave * passes;               // rays per chunk
    const int chunks = (nbins + span - 1) / span;
    const int units = max(0, e_hi - e_lo) * chunks;
    const uint32_t lim = static_cast<uint32_t>(ext + 2);

    // ray values (y / |cos| or y / |sin|) of one work unit, for up to NP passes
    auto fetch = [&](int unit, T *yv) {
        const int e = e_lo + unit / chunks, c = unit % chunks;
        const int l = order[e];
        const int k = subset < 0 ? l : subset + l * nsub;
        const T inv = tab.inv[k];
        const T *yl = yz + static_cast<size_t>(l) * nbins;
#pragma unroll
        for (int pass = 0; pass < (NP > 0 ? NP : 1); ++pass) {
            const int u = c * span + pass + passes * lane;
            yv[pass] = u < nbins ? yl[u] * inv : T(0);
        }
    };
    // deposit one pass of one unit: rays u = c * span + pass + passes * lane
    auto deposit = [&](int unit, int pass, T y0) {
        const int e = e_lo + unit / chunks, c = unit % chunks;
        const int l = order[e];
        const int k = subset < 0 ? l : subset + l * nsub;
        const int u = c * span + pass + passes * lane;
        if constexpr (kFixed) {
            const T y1 = y0 * T(0x1p-32f);
            const int64_t q2 = tab.q2[k];
            int64_t q = tab.q0[k] + (static_cast<int64_t>(2) << 32) + static_cast<int64_t>(u) * tab.q1[k] +
                        static_cast<int64_t>(t_lo) * q2;
            if (nt == kStrip) {
                // all reads of the strip's rows first (rows never alias), then the writes
                T *cell[kStrip];
                T c0[kStrip], c1[kStrip], m[kStrip];
#pragma unroll
                for (int t = 0; t < kStrip; ++t) {
                    cell[t] = acc + t * stride + min(static_cast<uint32_t>(q >> 32), lim);
                    m[t] = static_cast<T>(static_cast<uint32_t>(q)) * y1;  // w y
                    q += q2;
                }
#pragma unroll
                for (int t = 0; t < kStrip; ++t) {
                    c0[t] = cell[t][0];
                    c1[t] = cell[t][1];
                }
#pragma unroll
                for (int t = 0; t < kStrip; ++t) {
                    cell[t][0] = c0[t] + (y0 - m[t]);
                    cell[t][1] = c1[t] + m[t];
                }
            } else {
                for (int t = 0; t < nt; ++t) {
                    const uint32_t idx = min(static_cast<uint32_t>(q >> 32), lim);
                    const T mm = static_cast<T>(static_cast<uint32_t>(q)) * y1;
                    T *cl = acc + t * stride + idx;
                    const T a = cl[0], b = cl[1];
                    cl[0] = a + (y0 - mm);
                    cl[1] = b + mm;
                    q += q2;
                }
            }
        } else {
            const T a0 = tab.a0[k], a1 = tab.a1[k], a2 = tab.a2[k];
            for (int t = 0; t < nt; ++t) {
                const T q = fma(static_cast<T>(u), a1, fma(static_cast<T>(t_lo + t), a2, a0));
                const T fl = floor(q);
                const uint32_t idx = min(static_cast<uint32_t>(static_cast<int>(fl) + 2), lim);
                const T m = (q - fl) * y0;
                T *cell = acc + t * stride + idx;
                const T c0 = cell[0], c1 = cell[1];
                cell[0] = c0 + (y0 - m);
                cell[1] = c1 + m;
            }
        }
    };

    if constexpr (NP > 0) {
        // software pipeline: the next unit's ray values are in flight while this one deposits
        T ynext[NP];
        int unit = wave;
        if (unit < units) fetch(unit, ynext);
        while (unit < units) {
            T ycur[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) ycur[q] = ynext[q];
            const int nxt = unit + nw;
            if (nxt < units) fetch(nxt, ynext);
#pragma unroll
            for (int pass = 0; pass < NP; ++pass) deposit(unit, pass, ycur[pass]);
            unit = nxt;
        }
    } else {
        for (int unit = wave; unit < units; unit += nw) {
            const int e = e_lo + unit / chunks, c = unit % chunks;
            const int l = order[e];
            const int k = subset < 0 ? l : subset + l * nsub;
            const T inv = tab.inv[k];
            const T *yl = yz + static_cast<size_t>(l) * nbins;
            for (int pass = 0; pass < passes; ++pass) {
                const int u = c * span + pass + passes * lane;
                deposit(unit, pass, u < nbins ? yl[u] * inv : T(0));
            }
        }
    }
    __syncthreads();

    // sum the waves' strips (fixed order) and write this (class, group) partial image
    T *pz = part + (static_cast<size_t>(rowc ? 0 : 1) * groups + grp) * (plane * it.nz) + z * plane;
    if (rowc) {
        for (int e = threadIdx.x; e < nt * ext; e += blockDim.x) {
            const int t = e / ext, j = e - t * ext;
            T v = T(0);
            for (int w = 0; w < nw; ++w) v += acc_all[(static_cast<size_t>(w) * strip + t) * stride + j + 2];
            pz[static_cast<size_t>(t_lo + t) * nx + j] = v;
        }
    } else {
        for (int e = threadIdx.x; e < nt * ext; e += blockDim.x) {
            const int i = e / nt, t = e - i * nt;   // nt adjacent columns of one row
            T v = T(0);
            for (int w = 0; w < nw; ++w) v += acc_all[(static_cast<size_t>(w) * strip + t) * stride + i + 2];
            pz[static_cast<size_t>(i) * nx + t_lo + t] = v;
        }
    }
}

template <typename T>
struct UpdateT {
    T *x;
    const T *h;
    T *gs;
    T *vout;
    T gamma, gamma_over_p, nsub;
    int coin, plain;
};

// d = sum of the 2G partial images (fixed order), then the epilogue of `mode`.
template <typename T>
struct CombineItem {
    const T *part;
    T *out;
    UpdateT<T> upd;
    size_t n;
    int groups, mode, blocks;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_backproject_combine(WorkList<CombineItem<T>> wl) {
    int local;
    const CombineItem<T> &it = wl.item[work_item(wl, local)];
    const T *__restrict__ part = it.part;
    T *__restrict__ out = it.out;
    const UpdateT<T> &upd = it.upd;
    const size_t n = it.n;
    const int groups = it.groups, mode = it.mode;
    for (size_t p = local * static_cast<size_t>(kBlock) + threadIdx.x; p < n;
         p += static_cast<size_t>(it.blocks) * kBlock) {
        T d = T(0);
        for (int q0 = 0; q0 < 2 * groups; q0 += 8) {
            T v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = q0 + q < 2 * groups ? part[(q0 + q) * n + p] : T(0);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q0 + q < 2 * groups) d += v[q];
        }
        if (mode == BP_OVERWRITE) {
            out[p] = d;
        } else if (mode == BP_ACCUMULATE) {
            out[p] += d;
        } else {
            T G;
            if (mode == BP_SNAPSHOT) {
                upd.gs[p] = d;
                G = d;
            } else {
                G = fma(upd.nsub, d, upd.gs[p]);
            }
            const T xv = upd.x[p];
            if (upd.plain) {
                upd.vout[p] = xv - upd.gamma * G;
            } else {
                const T hv = upd.h[p];
                const T xh = xv - upd.gamma * (G - hv);
                if (upd.coin)
                    upd.vout[p] = xh - upd.gamma_over_p * hv;
                else
                    upd.x[p] = xh;
            }
        }
    }
}

template <typename T, int NP, int S>
static ps_status launch_bp_list(const WorkList<BackItem<T>> &wl, int blocks, int waves, size_t lds,
                                hipStream_t st) {
    hipLaunchKernelGGL((k_backproject<T, NP, S>), dim3(blocks), dim3(kWave * waves), lds, st, wl);
    PS_LAUNCHED("k_backproject");
    return PS_OK;
}

template <typename T, int NP>
static ps_status launch_bp_strip(int strip, const WorkList<BackItem<T>> &wl, int blocks, int waves,
                                 size_t lds, hipStream_t st) {
    switch (strip) {
        case 8: return launch_bp_list<T, NP, 8>(wl, blocks, waves, lds, st);
        case 4: return launch_bp_list<T, NP, 4>(wl, blocks, waves, lds, st);
        default: return launch_bp_list<T, NP, 1>(wl, blocks, waves, lds, st);
    }
}

template <typename T>
static ps_status launch_bp_key(int np, int strip, const WorkList<BackItem<T>> &wl, int blocks,
                               int waves, size_t lds, hipStream_t st) {
    switch (np) {
        case 1: return launch_bp_strip<T, 1>(strip, wl, blocks, waves, lds, st);
        case 2: return launch_bp_strip<T, 2>(strip, wl, blocks, waves, lds, st);
        case 3: return launch_bp_strip<T, 3>(strip, wl, blocks, waves, lds, st);
        case 4: return launch_bp_strip<T, 4>(strip, wl, blocks, waves, lds, st);
        default: return launch_bp_strip<T, 0>(strip, wl, blocks, waves, lds, st);
    }
}

static int strip_key(int strip) { return strip == 8 || strip == 4 ? strip : 1; }
static int np_key(int passes) { return passes >= 1 && passes <= 4 ? passes : 0; }

// All calls of one dtype: scatter launches grouped by (passes, strip, waves), then the combines.
template <typename T>
static ps_status backproject_many_t(const BackCall *calls, int n, hipStream_t st) {
    std::vector<BackItem<T>> items;
    std::vector<BackPlan> plans;
    std::vector<int> call_of;
    for (int c = 0; c < n; ++c) {
        const BackCall &bc = calls[c];
        const ps_geometry *g = bc.g;
        const auto &d = g->desc;
        if (bc.mode < BP_OVERWRITE || bc.mode > BP_SNAPSHOT)
            return fail(PS_EINVAL, "backprojector mode %d", bc.mode);
        const BackPlan bp = back_plan(g, bc.subset);
        const size_t need = back_workspace(g, bc.subset);
        if (!bc.ws || bc.ws_bytes < need)
            return fail(PS_EINVAL, "backprojector workspace: %zu bytes given, %zu needed", bc.ws_bytes, need);
        const AngleTab<T> tab = angle_tab<T>(g);
        BackItem<T> it{};
        it.y = static_cast<const T *>(bc.y);
        it.part = static_cast<T *>(bc.ws);
        it.order = bc.subset < 0 ? tab.ord_full : tab.ord_sub + g->sub_off[bc.subset];
        it.tab = tab;
        it.subset = bc.subset;
        it.nsub = d.n_subsets;
        it.na = subset_count(g, bc.subset);
        it.nx = d.nx;
        it.ny = d.ny;
        it.nz = d.nz;
        it.nbins = d.n_bins;
        it.strip = bp.strip;
        it.stride = bp.stride;
        it.s_row = bp.s_row;
        it.s_col = bp.s_col;
        it.groups = bp.groups;
        it.passes = g->bp_passes;
        it.nrow = bc.subset < 0 ? g->nrow_full : g->nrow_sub[bc.subset];
        items.push_back(it);
        plans.push_back(bp);
        call_of.push_back(c);
    }
    // scatter: one list per kernel instance (passes, strip) and block size, kMaxItems at a time
    std::vector<bool> done(items.size(), false);
    for (size_t i0 = 0; i0 < items.size(); ++i0) {
        if (done[i0]) continue;
        const int np = np_key(items[i0].passes), sk = strip_key(items[i0].strip);
        const int waves = plans[i0].waves;
        ListBuilder<BackItem<T>> lb;
        size_t lds = 0;
        for (size_t i = i0; i < items.size(); ++i) {
            if (done[i] || np_key(items[i].passes) != np || strip_key(items[i].strip) != sk ||
                plans[i].waves != waves)
                continue;
            done[i] = true;
            const long blocks = static_cast<long>(plans[i].s_row + plans[i].s_col) * plans[i].groups * items[i].nz;
            if (blocks > (1L << 30)) return fail(PS_EUNSUPPORTED, "backprojector grid too large");
            lb.add(items[i], static_cast<int>(blocks));
            lds = std::max(lds, plans[i].lds_bytes);
            if (lb.full()) {
                PS_TRY(launch_bp_key<T>(np, sk, lb.wl, lb.blocks, waves, lds, st));
                lb.clear();
                lds = 0;
            }
        }
        if (!lb.empty()) PS_TRY(launch_bp_key<T>(np, sk, lb.wl, lb.blocks, waves, lds, st));
    }
    // combine + epilogue
    ListBuilder<CombineItem<T>> lb;
    for (size_t i = 0; i < items.size(); ++i) {
        const BackCall &bc = calls[call_of[i]];
        CombineItem<T> ci{};
        ci.part = items[i].part;
        ci.out = static_cast<T *>(bc.out);
        const UpdateArgs &u = bc.upd;
        ci.upd.x = static_cast<T *>(u.x);
        ci.upd.h = static_cast<const T *>(u.h);
        ci.upd.gs = static_cast<T *>(u.gs);
        ci.upd.vout = static_cast<T *>(u.vout);
        ci.upd.gamma = static_cast<T>(u.gamma);
        ci.upd.gamma_over_p = static_cast<T>(u.gamma_over_p);
        ci.upd.nsub = static_cast<T>(u.nsub);
        ci.upd.coin = u.coin;
        ci.upd.plain = u.plain;
        ci.n = static_cast<size_t>(items[i].nx) * items[i].ny * items[i].nz;
        ci.groups = items[i].groups;
        ci.mode = bc.mode;
        ci.blocks = static_cast<int>(std::max<size_t>(1, std::min<size_t>((ci.n + kBlock - 1) / kBlock, 8192)));
        lb.add(ci, ci.blocks);
        if (lb.full()) {
            hipLaunchKernelGGL((k_backproject_combine<T>), dim3(lb.blocks), dim3(kBlock), 0, st, lb.wl);
            PS_LAUNCHED("k_backproject_combine");
            lb.clear();
        }
    }
    if (!lb.empty()) {
        hipLaunchKernelGGL((k_backproject_combine<T>), dim3(lb.blocks), dim3(kBlock), 0, st, lb.wl);
        PS_LAUNCHED("k_backproject_combine");
    }
    return PS_OK;
}

ps_status launch_backproject_many(const BackCall *calls, int n, hipStream_t st) {
    std::vector<BackCall> f32, f64;
    for (int c = 0; c < n; ++c) (calls[c].g->desc.dtype == PS_F64 ? f64 : f32).push_back(calls[c]);
    if (!f32.empty()) PS_TRY(backproject_many_t<float>(f32.data(), static_cast<int>(f32.size()), st));
    if (!f64.empty()) PS_TRY(backproject_many_t<double>(f64.data(), static_cast<int>(f64.size()), st));
    return PS_OK;
}

ps_status launch_backproject(const ps_geometry *g, int subset, const void *y, void *out, int mode,
                             const UpdateArgs *upd, void *ws, size_t ws_bytes, hipStream_t st) {
    BackCall c{};
    c.g = g;
    c.subset = subset;
    c.y = y;
    c.out = out;
    c.mode = mode;
    if (upd) c.upd = *upd;
    c.ws = ws;
    c.ws_bytes = ws_bytes;
    return launch_backproject_many(&c, 1, st);
}

}  // namespace ps

using namespace ps;

extern "C" size_t backproject_workspace_bytes(const ps_geometry *g, int32_t subset) {
    if (!g || subset_count(g, subset) < 0) return 0;
    return back_workspace(g, subset);
}

extern "C" ps_status backproject_subset(const ps_geometry *g, int32_t subset, const void *y,
                                        void *x, int32_t accumulate, void *workspace,
                                        size_t ws_bytes, void *stream) {
    clear_error();
    PS_TRY(check_ready(g));
    if (subset_count(g, subset) < 0) return fail(PS_EINVAL, "subset %d out of range", subset);
    PS_TRY(check_ptr(y, "y", g->elem));
    PS_TRY(check_ptr(x, "x", g->elem));
    if (accumulate != 0 && accumulate != 1) return fail(PS_EINVAL, "accumulate must be 0 or 1");
    return launch_backproject(g, subset, y, x, accumulate ? BP_ACCUMULATE : BP_OVERWRITE, nullptr,
                              workspace, ws_bytes, static_cast<hipStream_t>(stream));
}
