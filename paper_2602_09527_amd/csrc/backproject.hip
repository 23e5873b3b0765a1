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
#include <type_traits>
#include <vector>

#include "internal.h"

namespace ps {

constexpr int kWave = 64;
constexpr int kGatherTX = 63;   // output columns per gather tile (lane 0 of a wave is a halo)

// Wave-uniform copies (readfirstlane) of values every lane holds alike, so that arithmetic on
// them runs on the scalar unit.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float uni(float v) { return __builtin_bit_cast(float, uni(__builtin_bit_cast(int, v))); }
__device__ inline int64_t uni(int64_t v) {
    const uint64_t u = static_cast<uint64_t>(v);
    return static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(uni(static_cast<int>(u >> 32)))) << 32) |
                                static_cast<uint32_t>(uni(static_cast<int>(u & 0xffffffffu))));
}
__device__ inline double uni(double v) { return __builtin_bit_cast(double, uni(__builtin_bit_cast(int64_t, v))); }

// Constants of one angle as the scatter kernel uses them, staged in LDS per workgroup.
template <typename T>
struct ScatterAngle {
    int64_t qb, q1, q2;   // FP32 path (32.32 fixed point): qb = position of bin 0 at the strip's
                          // first step, plus the two pad words
    T a0, a1, a2;         // FP64 path
    T inv;
    int l;                // index within the call's angle list (row of y)
};

constexpr int kScatterAngles = 64;   // angle records staged in LDS at a time
constexpr int kPrefetch = 4;         // work units whose ray values are loaded ahead

static size_t scatter_angle_bytes(size_t elem) {
    return elem == sizeof(double) ? sizeof(ScatterAngle<double>) : sizeof(ScatterAngle<float>);
}

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
    const int per = (std::max(1, most) + p.groups - 1) / p.groups;   // angles per workgroup
    p.lds_bytes = align_up(static_cast<size_t>(p.waves) * p.strip * p.stride * g->elem, 16) +
                  static_cast<size_t>(std::min(per, kScatterAngles)) * scatter_angle_bytes(g->elem);
    p.part_elems = static_cast<size_t>(2) * p.groups * d.nx * d.ny * d.nz;
    return p;
}

size_t back_workspace(const ps_geometry *g, int subset) {
    return align_up(back_plan(g, subset).part_elems * g->elem);
}

int back_method(const ps_geometry *g, int subset) {
    const int forced = subset < 0 ? g->plan.bp_method_full : g->plan.bp_method_subset;
    if (!g->gather_ok) return BP_SCATTER;
    if (forced == BP_SCATTER || forced == BP_GATHER) return forced;
    // automatic: the scatter (faster on the workloads measured; the autotuner may pick the gather)
    return BP_SCATTER;
}

int gather_rows(const ps_geometry *g, int subset) {
    const int forced = g->plan.bp_gather_rows;
    if (forced == 2 || forced == 4) return forced;
    // 4 rows per wave (tiles of 63 x 16) unless that leaves fewer than 512 workgroups
    const auto &d = g->desc;
    const long tiles4 = static_cast<long>((d.nx + kGatherTX - 1) / kGatherTX) * ((d.ny + 15) / 16) * d.nz;
    return tiles4 < 512 ? 2 : 4;
}

int gather_split(const ps_geometry *g, int subset) {
    const int forced = g->plan.bp_gather_split;
    if (forced == 1 || forced == 2 || forced == 4) return forced;
    // small images: split the angles until there are about 1024 workgroups (at 128^2 the 4-way
    // split cuts a subset's gather from 9.7 to 6.2 us)
    const auto &d = g->desc;
    const int rows = gather_rows(g, subset);
    const long tiles = static_cast<long>((d.nx + kGatherTX - 1) / kGatherTX) * ((d.ny + 4 * rows - 1) / (4 * rows)) * d.nz;
    return tiles < 256 ? 4 : tiles < 1024 ? 2 : 1;
}

long gather_tiles(const ps_geometry *g, int subset, int rows) {
    const auto &d = g->desc;
    const int tile_rows = (4 / gather_split(g, subset)) * rows;
    return static_cast<long>((d.nx + kGatherTX - 1) / kGatherTX) * ((d.ny + tile_rows - 1) / tile_rows) * d.nz;
}

// Automatic fusion of the projector's reduction into the subset gather: up to this many partials
// per ray value (each staged value then costs that many loads instead of one), and while all of
// them fit in the caches (the 1024^2 x 256 volume's 356 MB of subset partials, re-read from HBM
// by every tile that stages them, made its epoch 1% slower fused).
constexpr int kGatherFuseSplit = 8;
constexpr size_t kGatherFuseBytes = static_cast<size_t>(32) << 20;

bool gather_fused(const ps_geometry *g, int subset) {
    if (subset < 0 || back_method(g, subset) != BP_GATHER) return false;
    const int split = proj_plan(g, subset_count(g, subset)).split;
    const size_t bytes = proj_workspace(g, subset_count(g, subset));
    if (split <= 1 || bytes >= (static_cast<size_t>(1) << 32)) return false;
    const int forced = g->plan.bp_gather_fused;
    if (forced == 1 || forced == 2) return forced == 2;
    return split <= kGatherFuseSplit && bytes <= kGatherFuseBytes;
}

// One backprojector application: partial images of A_sub^T y, one per (angle class, group).
template <typename T>
struct BackItem {
    const T *y;
    T *part;
    const int32_t *order;
    AngleTab<T> tab;
    int subset, nsub, na, nx, ny, nz, nbins, strip, stride, s_row, s_col, groups, passes, nrow;
    int xcd;   // set on every item of a launch whose items all take all angles: XCD-ordered grid
};

template <typename T, int NP, int kStrip>
__global__ __launch_bounds__(kBlock) void k_backproject(WorkList<BackItem<T>> wl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *acc_all = reinterpret_cast<T *>(smem_raw);
    constexpr bool kFixed = std::is_same<T, float>::value;
    int local;
    // all-angle launches take their workgroups in XCD order (each XCD's L2 then fetches the rows
    // of y of its own angle groups and slices only); subset launches keep the dispatch order,
    // which measured faster for them
    const BackItem<T> &it = wl.item[wl.item[0].xcd ? work_item_xcd(wl, local) : work_item(wl, local)];
    const T *__restrict__ y = it.y;
    T *__restrict__ part = it.part;
    const int32_t *__restrict__ order = it.order;
    const AngleTab<T> &tab = it.tab;
    const int subset = it.subset, nsub = it.nsub, na = it.na, nx = it.nx, ny = it.ny;
    const int nbins = it.nbins, strip = it.strip, stride = it.stride, s_row = it.s_row;
    const int groups = it.groups, passes = it.passes, nrow = it.nrow;
    const int nw = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));
    const int lane = threadIdx.x % kWave;
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

    {
        // zero the accumulator strips with 16-byte stores, then the few words past the last
        // whole 16 bytes
        const int total = nw * strip * stride;
        const int n16 = total * static_cast<int>(sizeof(T)) / 16;
        uint4 *a16 = reinterpret_cast<uint4 *>(acc_all);
        for (int e = threadIdx.x; e < n16; e += blockDim.x) a16[e] = make_uint4(0u, 0u, 0u, 0u);
        const int done = n16 * 16 / static_cast<int>(sizeof(T));
        if (static_cast<int>(threadIdx.x) < total - done) acc_all[done + threadIdx.x] = T(0);
    }
    // this workgroup's angles, staged once (the per-unit loads would otherwise wait on L2)
    // this workgroup's angles, staged kScatterAngles at a time (per-unit loads of the tables would
    // otherwise wait on L2 inside the deposit loop)
    ScatterAngle<T> *angs = reinterpret_cast<ScatterAngle<T> *>(
        smem_raw + ((static_cast<size_t>(nw) * strip * stride * sizeof(T) + 15) / 16) * 16);
    T *acc = acc_all + static_cast<size_t>(wave) * strip * stride;

    const int span = kWave * passes;               // rays per chunk
    const int chunks = (nbins + span - 1) / span;
    const uint32_t lim = static_cast<uint32_t>(ext + 2);
    const int lp = passes * lane;                  // this lane's bin within a pass of a chunk

    // Work unit (e, c): staged angle e, rays c * span + pass + passes * lane of every pass.  The
    // waves take units round robin; e and c are wave-uniform (scalar registers).
    auto advance = [&](int &e, int &c) {
        c += nw;
        while (c >= chunks) {
            c -= chunks;
            ++e;
        }
    };
    // raw ray values of one work unit, for up to NP passes: plain loads from a clamped (always
    // valid) bin, so that nothing waits for them until they are used (scaled by ray_value)
    auto fetch = [&](int e, int c, T *yv) {
        const int l = uni(angs[e].l);
        const T *yl = yz + static_cast<size_t>(l) * nbins + c * span;
        const int last = nbins - 1 - c * span;   // >= 0: c < chunks
#pragma unroll
        for (int pass = 0; pass < (NP > 0 ? NP : 1); ++pass) yv[pass] = yl[min(pass + lp, last)];
    };
    // the deposited value y / |cos| (or y / |sin|), zero for lanes past the last bin
    auto ray_value = [&](int e, int c, int pass, T raw) {
        const T v = raw * uni(angs[e].inv);
        return pass + lp < nbins - c * span ? v : T(0);   // a select, not a branch
    };
    // deposit one ray of value y0 through the strip; FP32: q = its fixed-point position at the
    // strip's first step (plus the pad)
    auto deposit_fixed = [&](int64_t q, int64_t q2, T y0) {
        const T y1 = y0 * T(0x1p-32f);
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
    };
    auto deposit_float = [&](int e, int u, T y0) {
        const T a0 = uni(angs[e].a0), a1 = uni(angs[e].a1), a2 = uni(angs[e].a2);
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
    };
    // position of this lane's first ray of unit (e, c): qb + (c * span + passes * lane) q1
    auto lane_q = [&](int e, int c, int64_t &q1, int64_t &q2) {
        q1 = uni(angs[e].q1);
        q2 = uni(angs[e].q2);
        const uint64_t off = static_cast<uint64_t>(static_cast<uint32_t>(lp)) * static_cast<uint64_t>(q1);
        return uni(angs[e].qb) + static_cast<int64_t>(c * span) * q1 + static_cast<int64_t>(off);
    };

    for (int a0 = e_lo; a0 < e_hi; a0 += kScatterAngles) {
        const int an = min(kScatterAngles, e_hi - a0);
        __syncthreads();  // accumulators zeroed / the previous angles' records no longer read
        for (int e = threadIdx.x; e < an; e += blockDim.x) {
            ScatterAngle<T> ra;
            ra.l = order[a0 + e];
            const int k = subset < 0 ? ra.l : subset + ra.l * nsub;
            ra.q1 = tab.q1[k];
            ra.q2 = tab.q2[k];
            ra.qb = tab.q0[k] + (static_cast<int64_t>(2) << 32) + static_cast<int64_t>(t_lo) * ra.q2;
            ra.a0 = tab.a0[k];
            ra.a1 = tab.a1[k];
            ra.a2 = tab.a2[k];
            ra.inv = tab.inv[k];
            angs[e] = ra;
        }
        __syncthreads();
        int e = wave / chunks, c = wave - e * chunks;   // this wave's first unit
        if constexpr (NP > 0) {
            // software pipeline: the ray values of the next kPrefetch units are in flight while
            // this one deposits (a unit's deposits take far less time than a load that misses
            // the XCD's L2, as the values written by the previous launch on another XCD do)
            // every fetch is issued (past the last unit it reloads unit (an - 1, 0), unused), so
            // the number of loads in flight is the same on every path and a use waits only for
            // its own slot
            T ybuf[kPrefetch][NP];
            int fe = e, fc = c;   // the next unit to fetch
            auto fetch_any = [&](T *yv) {
                if (fe < an) fetch(fe, fc, yv);
                else fetch(an - 1, 0, yv);
            };
#pragma unroll
            for (int d = 0; d < kPrefetch; ++d) {
                fetch_any(ybuf[d]);
                advance(fe, fc);
            }
            while (e < an) {
#pragma unroll
                for (int d = 0; d < kPrefetch; ++d) {
                    if (e < an) {
                        T ycur[NP];
#pragma unroll
                        for (int q = 0; q < NP; ++q) ycur[q] = ray_value(e, c, q, ybuf[d][q]);
                        fetch_any(ybuf[d]);
                        advance(fe, fc);
                        if constexpr (kFixed) {
                            int64_t q1, q2;
                            int64_t q = lane_q(e, c, q1, q2);
#pragma unroll
                            for (int pass = 0; pass < NP; ++pass) {
                                deposit_fixed(q, q2, ycur[pass]);
                                q += q1;
                            }
                        } else {
#pragma unroll
                            for (int pass = 0; pass < NP; ++pass)
                                deposit_float(e, c * span + pass + lp, ycur[pass]);
                        }
                        advance(e, c);
                    }
                }
            }
        } else {
            for (; e < an; advance(e, c)) {
                const int l = uni(angs[e].l);
                const T inv = uni(angs[e].inv);
                const T *yl = yz + static_cast<size_t>(l) * nbins;
                int64_t q1 = 0, q2 = 0, q = 0;
                if constexpr (kFixed) q = lane_q(e, c, q1, q2);
                for (int pass = 0; pass < passes; ++pass) {
                    const int u = c * span + pass + lp;
                    const T y0 = u < nbins ? yl[u] * inv : T(0);
                    if constexpr (kFixed) {
                        deposit_fixed(q, q2, y0);
                        q += q1;
                    } else {
                        deposit_float(e, u, y0);
                    }
                }
            }
        }
    }
    __syncthreads();

    // sum the waves' strips (fixed order) and write this (class, group) partial image
    T *pz = part + (static_cast<size_t>(rowc ? 0 : 1) * groups + grp) * (plane * it.nz) + z * plane;
    // (no integer division per element on full strips)
    if (rowc) {
        for (int t = 0; t < nt; ++t) {
            T *prow = pz + static_cast<size_t>(t_lo + t) * nx;
            for (int j = threadIdx.x; j < ext; j += blockDim.x) {
                T v = T(0);
                for (int w = 0; w < nw; ++w) v += acc_all[(w * strip + t) * stride + j + 2];
                prow[j] = v;
            }
        }
    } else if (nt == kStrip) {
        // nt adjacent lanes write the strip's nt adjacent columns of one image row (one 16- or
        // 32-byte piece per row for the store); the row and column come from shifts
        constexpr int sh = kStrip == 8 ? 3 : kStrip == 4 ? 2 : kStrip == 2 ? 1 : 0;
        for (int e = threadIdx.x; e < nt * ext; e += blockDim.x) {
            const int i = e >> sh, t = e & (kStrip - 1);
            T v = T(0);
            for (int w = 0; w < nw; ++w) v += acc_all[(w * strip + t) * stride + i + 2];
            pz[static_cast<size_t>(i) * nx + t_lo + t] = v;
        }
    } else {
        for (int e = threadIdx.x; e < nt * ext; e += blockDim.x) {
            const int i = e / nt, t = e - i * nt;   // nt adjacent columns of one row
            T v = T(0);
            for (int w = 0; w < nw; ++w) v += acc_all[(w * strip + t) * stride + i + 2];
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
    T *tab, *tsum;
    const T *xs;
    T *dx;
    T gamma, gamma_over_p, nsub;
    int coin, plain;
    int nx, ny, nz, nonneg;
};

// (D^T y2) at pixel p of an nx x ny x nz grid (forward differences with a zero last difference;
// y2 holds d = 2 or 3 components of n values each).
template <typename T>
__device__ inline T div_at(const T *__restrict__ y2, size_t p, int nx, int ny, int nz) {
    const size_t plane = static_cast<size_t>(nx) * ny, n = plane * nz;
    const int j = static_cast<int>(p % nx), i = static_cast<int>((p / nx) % ny);
    const int z = static_cast<int>(p / plane);
    const T *yx = y2, *yy = y2 + n;
    T t = (j > 0 ? yx[p - 1] : T(0)) - (j < nx - 1 ? yx[p] : T(0));
    t += (i > 0 ? yy[p - nx] : T(0)) - (i < ny - 1 ? yy[p] : T(0));
    if (nz > 1) {
        const T *yz = y2 + 2 * n;
        t += (z > 0 ? yz[p - plane] : T(0)) - (z < nz - 1 ? yz[p] : T(0));
    }
    return t;
}

// The epilogue of a backprojection at pixel p, d = (A^T y)(p): overwrite, accumulate, or the fused
// SVRG / ProxSkip gradient step (see UpdateArgs).
template <typename T>
__device__ inline void bp_epilogue(int mode, const UpdateT<T> &upd, T *__restrict__ out, size_t p, T d) {
    if (mode == BP_OVERWRITE) {
        out[p] = d;
    } else if (mode == BP_ACCUMULATE) {
        out[p] += d;
    } else if (mode == BP_GRADSTEP) {
        upd.vout[p] = upd.x[p] - upd.gamma * d;
    } else if (mode == BP_PDHG) {
        const T xv = upd.x[p];
        T w = xv - upd.gs[p] * (d + div_at(upd.tab, p, upd.nx, upd.ny, upd.nz));
        if (upd.nonneg && w < T(0)) w = T(0);
        upd.vout[p] = T(2) * w - xv;
        upd.x[p] = w;
    } else {
        T G;
        if (mode == BP_SNAPSHOT) {
            upd.gs[p] = d;
            G = d;
        } else if (mode == BP_SAGA) {
            const T diff = d - upd.tab[p];
            const T sum = upd.tsum[p];
            G = fma(upd.nsub, diff, sum);
            upd.tsum[p] = sum + diff;
            upd.tab[p] = d;
        } else {
            G = fma(upd.nsub, d, upd.gs[p]);
        }
        const T xv = upd.x[p];
        if (upd.plain) {
            upd.vout[p] = xv - upd.gamma * G;
        } else {
            const T hv = upd.h[p];
            const T xh = xv - upd.gamma * (G - hv);
            if (upd.coin) {
                upd.vout[p] = xh - upd.gamma_over_p * hv;
            } else {
                upd.x[p] = xh;
                if (upd.dx) upd.dx[p] = xh - upd.xs[p];
            }
        }
    }
}

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
        // fixed order over the 2G partials; the loads of a batch of 8 are unconditional (clamped
        // to the last partial) so that they are all in flight before the first add
        const int np = 2 * groups;
        T d = T(0);
        for (int q0 = 0; q0 < np; q0 += 8) {
            T v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = part[static_cast<size_t>(min(q0 + q, np - 1)) * n + p];
#pragma unroll
            for (int q = 0; q < 8; ++q) d = q0 + q < np ? d + v[q] : d;
        }
        bp_epilogue(mode, upd, out, p, d);
    }
}

// ---- pixel-driven gather ---------------------------------------------------------------------
//
// A workgroup owns a tile of 63 columns x 16 rows of one slice and sums, for every pixel, the
// contributions of all the call's angles directly: no partial images, and the epilogue (the
// SVRG / ProxSkip step) is applied in the same kernel.
//   Pixel (i, j) receives from ray u of an angle the weight the projector gives it.  With p the
//   pixel's coordinate along the interpolation axis (j for row-walked angles, i for column-walked
//   ones) and s along the stepping axis, ray u's cell at step s is c = floor(q(u, s)) with weight
//   w = frac(q): the pixel gets (1 - w) y_u / |.| from the ray with c = p and w y_u / |.| from the
//   ray with c = p - 1 -- the same 32.32 fixed-point q (FP32) or FMA-evaluated q (FP64) and the
//   same products as the scatter kernel, so A^T stays the projector's transpose.
//   When adjacent rays are at least one pixel apart (|a1| >= 1) a cell holds at most one ray
//   (FP32: exact fixed point; FP64 rounding can put two in one cell, and both are taken), found
//   among the two integers around u* = (p - a0 - s a2) / a1 (each checked exactly).  Each
//   lane finds the ray of its own cell; the ray of cell p - 1 is its neighbour's: the lane to the
//   left for row-walked angles (a DPP lane shift; lane 0 is a halo column that only supplies
//   this), the lane's previous row for column-walked ones (one extra lookup per wave).  In FP32
//   the search runs once per angle and the lane then walks its rays in cell order from row to
//   row (cell_walk_start), which takes the same rays and gives the same bits.
//   The rays an angle can send into the tile form a window of at most kGatherWin consecutive
//   bins; the windows of up to kGatherChunk angles (y / |.|, zero outside [0, B)) are staged in
//   LDS at a time.
//   Inside a solver iteration the gather may also take the projector's split partial sums in
//   place of y (psplit > 1): the staging then forms each staged ray value as the projector's
//   reduction pass does -- the partials added in split order, times 1/|.|, minus b when a data
//   term is subtracted -- with the same operations, so the result has the same bits as the
//   reduction pass followed by the gather, and the iteration needs one launch fewer.
constexpr int kGatherChunk = 32;
constexpr int kGatherWin = 96;

template <typename T>
struct GatherItem {
    const T *y;       // the sinogram (nz x na x B), or with psplit > 1 the projector's partials
    T *out;
    UpdateT<T> upd;
    AngleTab<T> tab;
    const T *pb;      // psplit > 1: b (nz x A x B) subtracted from the summed rays, or null
    int subset, nsub, na, nx, ny, nbins, tiles_x, tiles_y, mode;
    int psplit, n_angles;
    uint32_t pbytes;  // psplit > 1: bytes between consecutive partials (nz na B elements)
};

template <typename T>
struct GatherAngle {
    int row;
    int cs, co;       // candidate rule: uf = cs * floor(cr * u* + 1/64) + co (see cell_ray)
    T a0, a1, a2, ia1, cr, inv;
    T csf, cof;       // cs and co as floating point
    int64_t q0, q1, q2;
};

template <typename T>
__device__ inline GatherAngle<T> uni(const GatherAngle<T> &g) {
    GatherAngle<T> r;
    r.row = uni(g.row);
    r.cs = uni(g.cs);
    r.co = uni(g.co);
    r.cr = uni(g.cr);
    r.csf = uni(g.csf);
    r.cof = uni(g.cof);
    r.inv = uni(g.inv);
    r.a0 = uni(g.a0);
    r.a1 = uni(g.a1);
    r.a2 = uni(g.a2);
    r.ia1 = uni(g.ia1);
    r.q0 = uni(g.q0);
    r.q1 = uni(g.q1);
    r.q2 = uni(g.q2);
    return r;
}

template <typename T>
__device__ inline GatherAngle<T> gather_angle(const AngleTab<T> &tab, int k) {
    GatherAngle<T> g;
    g.row = tab.row[k];
    g.a0 = tab.a0[k];
    g.a1 = tab.a1[k];
    g.a2 = tab.a2[k];
    g.ia1 = tab.ia1[k];
    g.q0 = tab.q0[k];
    g.q1 = tab.q1[k];
    g.q2 = tab.q2[k];
    g.inv = tab.inv[k];
    const bool up = g.a1 > T(0);
    g.cr = up ? T(-1) : T(1);
    g.cs = up ? -1 : 1;
    g.co = up ? 0 : -1;
    g.csf = static_cast<T>(g.cs);
    g.cof = static_cast<T>(g.co);
    return g;
}

__device__ inline float lane_from_left(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ inline double lane_from_left(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(__double2loint(v)), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(__double2hiint(v)), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// The ray of cell p at step s: its two deposits, own = (1 - w) y and next = w y (zero when the
// cell holds no ray).  c = fma(s, a2, a0) and base = q0 + s q2 are the step's constants; ub is
// the first bin of the staged window yw.
template <typename T>
__device__ inline void cell_ray(const GatherAngle<T> &ga, int p, T c, int64_t base, const T *yw, int ub,
                                int nb, T &own, T &next) {
    constexpr bool kFixed = std::is_same<T, float>::value;
    // q(u) = c + u a1 is in [p, p + 1) for the bins in [u*, u* + 1/a1) (a1 > 0) or
    // (u* + 1/a1, u*] (a1 < 0), u* = (p - c) / a1: an interval of length <= 1 holding at most the
    // integer ceil(u*) (resp. floor(u*)).  Candidates uf and uf + 1 with uf = ceil(u* - 1/64)
    // (resp. floor(u* + 1/64) - 1) contain it whatever the rounding of u* (|error| < 1e-3).
    // branch-free: ceil(u* - 1/64) = -floor(1/64 - u*)
    const T us = (static_cast<T>(p) - c) * ga.ia1;
    int u;
    T w;
    bool hit;
    if constexpr (kFixed) {
        // the candidate in floating point (an exact small integer), clamped into [0, nb]: a ray
        // outside the detector deposits nothing, so the clamp loses no contribution.  Then
        // uf * q1 needs one 32 x 32 -> 64-bit multiply-add (uf >= 0) and a 24-bit product for
        // the small high word of q1, not a full 64-bit multiply.
        const int uf = min(max(static_cast<int>(fma(ga.csf, floor(fma(us, ga.cr, T(0.015625))), ga.cof)), 0), nb);
        const uint32_t q1lo = static_cast<uint32_t>(static_cast<uint64_t>(ga.q1));
        const int q1hi = static_cast<int>(ga.q1 >> 32);
        const uint64_t prod = static_cast<uint64_t>(static_cast<uint32_t>(uf)) * q1lo +
                              (static_cast<uint64_t>(static_cast<uint32_t>(__mul24(uf, q1hi))) << 32);
        const int64_t Q0 = static_cast<int64_t>(static_cast<uint64_t>(base) + prod);
        const int64_t Q1 = Q0 + ga.q1;
        const bool h0 = static_cast<int>(Q0 >> 32) == p;
        hit = h0 || static_cast<int>(Q1 >> 32) == p;
        u = h0 ? uf : uf + 1;
        w = static_cast<T>(static_cast<uint32_t>(h0 ? Q0 : Q1));
    } else {
        const int uf = ga.cs * static_cast<int>(floor(fma(us, ga.cr, T(0.015625)))) + ga.co;
        // FP64 positions are rounded: with |a1| = 1 two adjacent rays can land in one cell (for
        // instance q = -1 - 6e-17 rounds to -1 while the next ray has q = -6e-17), so every
        // candidate in the cell contributes, as in the scatter
        own = next = T(0);
#pragma unroll
        for (int cnd = 0; cnd < 2; ++cnd) {
            const T q = fma(static_cast<T>(uf + cnd), ga.a1, c);
            const T fl = floor(q);
            if (static_cast<int>(fl) == p) {
                const T y0 = yw[min(max(uf + cnd - ub, 0), kGatherWin - 1)];
                const T m = (q - fl) * y0;
                own += y0 - m;
                next += m;
            }
        }
        return;
    }
    const int widx = min(max(u - ub, 0), kGatherWin - 1);
    const T y0 = yw[widx];
    // the scatter's products: m = lo(Q) * (y * 2^-32)
    const T m = w * (y0 * T(0x1p-32f));
    own = hit ? y0 - m : T(0);
    next = hit ? m : T(0);
}

// FP32 walk start for cell p at step c / base (as cell_ray): the first ray, in the order of
// increasing cell, whose cell is >= p.  cell_ray's candidate pair holds it (its lower member for
// a1 > 0, its upper one for a1 < 0, as the cells then fall with u), or else the next ray in cell
// order; one exact check of the first decides.  Clamped into [0, nb] + 1 like cell_ray's pair.
__device__ inline void cell_walk_start(const GatherAngle<float> &ga, int p, float c, int64_t base, int nb,
                                       int &u, int64_t &Q) {
    const float us = (static_cast<float>(p) - c) * ga.ia1;
    const int uf = min(max(static_cast<int>(fmaf(ga.csf, floorf(fmaf(us, ga.cr, 0.015625f)), ga.cof)), 0), nb);
    const int g = uf - ga.co;                          // co = 0 (a1 > 0) or -1 (a1 < 0)
    const uint32_t q1lo = static_cast<uint32_t>(static_cast<uint64_t>(ga.q1));
    const int q1hi = static_cast<int>(ga.q1 >> 32);
    const uint64_t prod = static_cast<uint64_t>(static_cast<uint32_t>(g)) * q1lo +
                          (static_cast<uint64_t>(static_cast<uint32_t>(__mul24(g, q1hi))) << 32);
    const int64_t Qg = static_cast<int64_t>(static_cast<uint64_t>(base) + prod);
    const bool first = static_cast<int>(Qg >> 32) >= p;
    const int su = -ga.cs;
    u = first ? g : g + su;
    Q = first ? Qg : Qg + (su > 0 ? ga.q1 : -ga.q1);
}

// AS waves share each block of R rows, each taking every AS-th angle of the chunk; their sums are
// added in LDS in wave order (a fixed order) before the epilogue.  A tile is 4 / AS blocks of R
// rows: splitting the angles gives small images more workgroups without shrinking the staged
// windows' reuse below R rows.  PF: the staged values are formed from the projector's split
// partials (GatherItem::psplit > 1) rather than read from a sinogram.
template <typename T, int R, int AS, bool PF>
__global__ __launch_bounds__(kBlock) void k_backproject_gather(WorkList<GatherItem<T>> wl) {
    static_assert(AS == 1 || AS == 2 || AS == 4, "angle split");
    constexpr int kGatherRows = R;                 // rows per wave
    constexpr int kRowBlocks = 4 / AS;             // row blocks per tile
    constexpr int kGatherTY = kRowBlocks * R;      // rows per tile
    __shared__ T ywin[kGatherChunk][kGatherWin];
    __shared__ int ulo[kGatherChunk];
    __shared__ GatherAngle<T> s_ang[kGatherChunk];
    __shared__ T red[AS > 1 ? (AS - 1) * kRowBlocks * R * kWave : 1];
    int local;
    const GatherItem<T> &it = wl.item[work_item(wl, local)];
    const AngleTab<T> &tab = it.tab;
    const int tx = local % it.tiles_x, ty = (local / it.tiles_x) % it.tiles_y;
    const int z = local / (it.tiles_x * it.tiles_y);
    const int lane = threadIdx.x % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));
    const int nx = it.nx, ny = it.ny, B = it.nbins;
    const int rb = wave % kRowBlocks, ag = wave / kRowBlocks;   // row block, angle group
    const int j = tx * kGatherTX - 1 + lane;           // lane 0: halo column
    const int i0 = ty * kGatherTY + rb * kGatherRows;
    const T *yz = it.y + static_cast<size_t>(z) * it.na * B;
    T acc[kGatherRows];
#pragma unroll
    for (int r = 0; r < kGatherRows; ++r) acc[r] = T(0);

    for (int c0 = 0; c0 < it.na; c0 += kGatherChunk) {
        const int cn = min(kGatherChunk, it.na - c0);
        __syncthreads();  // the previous chunk's windows are no longer read
        if (static_cast<int>(threadIdx.x) < cn) {
            // lowest bin whose ray can reach the tile: cells d_lo - 1 .. d_hi + 1 of the
            // interpolation axis, over the tile's span of the stepping axis
            const int l = c0 + threadIdx.x;
            const int k = it.subset < 0 ? l : it.subset + l * it.nsub;
            const GatherAngle<T> ga = gather_angle(tab, k);
            s_ang[threadIdx.x] = ga;   // the angle's constants, read below by every wave
            const bool row = ga.row != 0;
            const T a0 = ga.a0, a2 = ga.a2, ia1 = ga.ia1;
            const int col_lo = tx * kGatherTX - 1, col_hi = col_lo + 63;
            const int row_lo = ty * kGatherTY - 1, row_hi = row_lo + kGatherTY;
            const int d_lo = row ? col_lo : row_lo, d_hi = row ? col_hi : row_hi;
            const int s_lo = row ? row_lo : col_lo, s_hi = row ? row_hi : col_hi;
            const T qa = static_cast<T>(d_lo - 1) - a0, qb = static_cast<T>(d_hi + 1) - a0;
            const T u1 = (qa - static_cast<T>(s_lo) * a2) * ia1, u2 = (qa - static_cast<T>(s_hi) * a2) * ia1;
            const T u3 = (qb - static_cast<T>(s_lo) * a2) * ia1, u4 = (qb - static_cast<T>(s_hi) * a2) * ia1;
            ulo[threadIdx.x] = static_cast<int>(floor(min(min(u1, u2), min(u3, u4)))) - 3;
        }
        __syncthreads();
        constexpr int kWinPer = (kGatherChunk * kGatherWin + kBlock - 1) / kBlock;
        if constexpr (PF) {
            // the projector's reduction pass, element by element: partials in split order (kPb
            // of them in flight, the last one re-read past the end), times 1/|.|, minus b; then
            // the gather's own 1/|.|.  32-bit byte offsets from the plane's base, the partial's
            // included, so that the loads take the scalar-base form (the host keeps all
            // partials within 4 GiB)
            constexpr int kPb = 2;
            const int ps = it.psplit;
            uint32_t off[kWinPer];
            T acc[kWinPer];
#pragma unroll
            for (int r = 0; r < kWinPer; ++r) {
                const int e = static_cast<int>(threadIdx.x) + r * kBlock;
                const int a = min(e / kGatherWin, cn - 1), w = e - (e / kGatherWin) * kGatherWin;
                off[r] = static_cast<uint32_t>((c0 + a) * B + min(max(ulo[a] + w, 0), B - 1)) *
                         static_cast<uint32_t>(sizeof(T));
                acc[r] = T(0);
            }
#pragma unroll 1
            for (int t0 = 0; t0 < ps; t0 += kPb) {
                T v[kPb][kWinPer];
#pragma unroll
                for (int q = 0; q < kPb; ++q) {
                    const uint32_t pt = static_cast<uint32_t>(min(t0 + q, ps - 1)) * it.pbytes;
#pragma unroll
                    for (int r = 0; r < kWinPer; ++r)
                        v[q][r] = *reinterpret_cast<const T *>(reinterpret_cast<const char *>(yz) + (off[r] + pt));
                }
#pragma unroll
                for (int q = 0; q < kPb; ++q)
#pragma unroll
                    for (int r = 0; r < kWinPer; ++r) acc[r] = t0 + q < ps ? acc[r] + v[q][r] : acc[r];
            }
            const T *bz = it.pb ? it.pb + static_cast<size_t>(z) * it.n_angles * B : nullptr;
#pragma unroll
            for (int r = 0; r < kWinPer; ++r) {
                const int e = static_cast<int>(threadIdx.x) + r * kBlock;
                const int a = e / kGatherWin, w = e - a * kGatherWin;
                if (a < cn) {
                    const int u = ulo[a] + w;
                    const int l = c0 + a;
                    const int k = it.subset < 0 ? l : it.subset + l * it.nsub;
                    const T inv = s_ang[a].inv;
                    const T val = bz ? fma(acc[r], inv, -bz[static_cast<size_t>(k) * B + min(max(u, 0), B - 1)])
                                     : acc[r] * inv;
                    ywin[a][w] = (u >= 0 && u < B) ? val * inv : T(0);
                }
            }
        } else {
            // each thread's window entries: all loads first (bins clamped into range), then the
            // scaled values (zero outside the detector) go to LDS
            T raw[kWinPer];
#pragma unroll
            for (int r = 0; r < kWinPer; ++r) {
                const int e = static_cast<int>(threadIdx.x) + r * kBlock;
                const int a = min(e / kGatherWin, cn - 1), w = e - (e / kGatherWin) * kGatherWin;
                const int u = min(max(ulo[a] + w, 0), B - 1);
                raw[r] = yz[static_cast<size_t>(c0 + a) * B + u];
            }
#pragma unroll
            for (int r = 0; r < kWinPer; ++r) {
                const int e = static_cast<int>(threadIdx.x) + r * kBlock;
                const int a = e / kGatherWin, w = e - a * kGatherWin;
                if (a < cn) {
                    const int u = ulo[a] + w;
                    const T v = raw[r] * s_ang[a].inv;
                    ywin[a][w] = (u >= 0 && u < B) ? v : T(0);
                }
            }
        }
        __syncthreads();
        // the next angle's record is read while this one is processed
        GatherAngle<T> raw = s_ang[min(ag, cn - 1)];
        int raw_ub = ulo[min(ag, cn - 1)];
        for (int a = ag; a < cn; a += AS) {
            const GatherAngle<T> ga = uni(raw);
            const int ub = uni(raw_ub);
            if (a + AS < cn) {
                raw = s_ang[a + AS];
                raw_ub = ulo[a + AS];
            }
            const T *yw = ywin[a];
            if (ga.row) {
                // interpolation along the row: cell p = j; the ray of cell j - 1 is the left lane's
                bool walked = false;
                if constexpr (std::is_same<T, float>::value && kGatherRows >= 4) {
                    // FP32, 4 rows per wave: one candidate search at the first row, then the
                    // first ray (in cell order) whose cell is >= j is carried from row to row:
                    // all cells shift by q2 per row, at most one ray spacing (|a2| <= 1 <= |a1|
                    // for row-walked angles; checked), so it moves by at most one ray, backwards
                    // when q2 >= 0.  (With 2 rows the rows' independent searches are faster: the
                    // walk chains them, and small launches are latency-bound.)
                    const int su = -ga.cs;
                    const int64_t sq1 = su > 0 ? ga.q1 : -ga.q1;
                    const int64_t q2 = ga.q2;
                    if ((q2 >= 0 ? q2 : -q2) <= sq1) {
                        walked = true;
                        int u;
                        int64_t Q;
                        cell_walk_start(ga, j, fma(static_cast<T>(i0), ga.a2, ga.a0),
                                        ga.q0 + static_cast<int64_t>(i0) * q2, B, u, Q);
                        auto rows = [&](auto backwards) {
                            constexpr bool kBack = decltype(backwards)::value;
#pragma unroll
                            for (int r = 0; r < kGatherRows; ++r) {
                                if (r > 0) {
                                    Q += q2;
                                    if constexpr (kBack) {
                                        const int64_t Qb = Q - sq1;
                                        const bool back = static_cast<int>(Qb >> 32) >= j;
                                        u = back ? u - su : u;
                                        Q = back ? Qb : Q;
                                    } else {
                                        const bool on = static_cast<int>(Q >> 32) < j;
                                        u = on ? u + su : u;
                                        Q = on ? Q + sq1 : Q;
                                    }
                                }
                                const bool hit = static_cast<int>(Q >> 32) == j;
                                const T w = static_cast<T>(static_cast<uint32_t>(Q));
                                const T y0 = yw[min(max(u - ub, 0), kGatherWin - 1)];
                                const T m = w * (y0 * T(0x1p-32f));
                                acc[r] += (hit ? y0 - m : T(0)) + lane_from_left(hit ? m : T(0));
                            }
                        };
                        if (q2 >= 0)
                            rows(std::true_type{});
                        else
                            rows(std::false_type{});
                    }
                }
                if (!walked) {
#pragma unroll
                    for (int r = 0; r < kGatherRows; ++r) {
                        const int i = i0 + r;
                        const T c = fma(static_cast<T>(i), ga.a2, ga.a0);
                        const int64_t base = ga.q0 + static_cast<int64_t>(i) * ga.q2;
                        T own, next;
                        cell_ray(ga, j, c, base, yw, ub, B, own, next);
                        acc[r] += own + lane_from_left(next);
                    }
                }
            } else {
                // interpolation along the column: cell p = i; the ray of cell i - 1 is the
                // previous row's, so each wave also looks up the row above its first
                const T c = fma(static_cast<T>(j), ga.a2, ga.a0);
                const int64_t base = ga.q0 + static_cast<int64_t>(j) * ga.q2;
                if constexpr (std::is_same<T, float>::value) {
                    // FP32: the column's rays taken in the order of their cells, from the first
                    // whose cell is >= i0 - 1 (cell_walk_start); after each row the walk moves on
                    // by one ray exactly when that row's cell held the current one (at most one
                    // ray per cell), so each row costs one check instead of a candidate search
                    int u;
                    int64_t Q;
                    cell_walk_start(ga, i0 - 1, c, base, B, u, Q);
                    const int su = -ga.cs;                       // +1: cells grow with u
                    const int64_t sq1 = su > 0 ? ga.q1 : -ga.q1;   // one ray on, in cell order
                    T prev = T(0);
#pragma unroll
                    for (int r = -1; r < kGatherRows; ++r) {
                        const bool hit = static_cast<int>(Q >> 32) == i0 + r;
                        const T w = static_cast<T>(static_cast<uint32_t>(Q));
                        const T y0 = yw[min(max(u - ub, 0), kGatherWin - 1)];
                        const T m = w * (y0 * T(0x1p-32f));
                        if (r >= 0) acc[r] += (hit ? y0 - m : T(0)) + prev;
                        prev = hit ? m : T(0);
                        u += hit ? su : 0;
                        Q += hit ? sq1 : 0;
                    }
                } else {
                    T own, prev;
                    cell_ray(ga, i0 - 1, c, base, yw, ub, B, own, prev);
#pragma unroll
                    for (int r = 0; r < kGatherRows; ++r) {
                        T next;
                        cell_ray(ga, i0 + r, c, base, yw, ub, B, own, next);
                        acc[r] += own + prev;
                        prev = next;
                    }
                }
            }
        }
    }
    if constexpr (AS > 1) {
        // the angle groups' sums, added to group 0's in group order
        if (ag > 0) {
#pragma unroll
            for (int r = 0; r < kGatherRows; ++r)
                red[(((ag - 1) * kRowBlocks + rb) * kGatherRows + r) * kWave + lane] = acc[r];
        }
        __syncthreads();
        if (ag > 0) return;
#pragma unroll
        for (int q = 1; q < AS; ++q)
#pragma unroll
            for (int r = 0; r < kGatherRows; ++r)
                acc[r] += red[(((q - 1) * kRowBlocks + rb) * kGatherRows + r) * kWave + lane];
    }
    if (lane == 0 || j >= nx) return;
    const size_t plane = static_cast<size_t>(nx) * ny;
#pragma unroll
    for (int r = 0; r < kGatherRows; ++r) {
        const int i = i0 + r;
        if (i < ny) bp_epilogue(it.mode, it.upd, it.out, z * plane + static_cast<size_t>(i) * nx + j, acc[r]);
    }
}

template <typename T, int NP, int S>
static ps_status launch_bp_list(const WorkList<BackItem<T>> &wl, int blocks, int waves, size_t lds,
                                hipStream_t st) {
    const int kc = wl.item[0].subset < 0 ? KC_BP_SCATTER_FULL : KC_BP_SCATTER_SUBSET;
    timer_mark(kc, st, true);
    hipLaunchKernelGGL((k_backproject<T, NP, S>), dim3(blocks), dim3(kWave * waves), lds, st, wl);
    PS_LAUNCHED("k_backproject");
    timer_mark(kc, st, false);
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

template <typename T>
static UpdateT<T> to_update(const UpdateArgs &u) {
    UpdateT<T> r{};
    r.x = static_cast<T *>(u.x);
    r.h = static_cast<const T *>(u.h);
    r.gs = static_cast<T *>(u.gs);
    r.vout = static_cast<T *>(u.vout);
    r.tab = static_cast<T *>(u.tab);
    r.tsum = static_cast<T *>(u.tsum);
    r.xs = static_cast<const T *>(u.xs);
    r.dx = static_cast<T *>(u.dx);
    r.nx = u.nx;
    r.ny = u.ny;
    r.nz = u.nz;
    r.nonneg = u.nonneg;
    r.gamma = static_cast<T>(u.gamma);
    r.gamma_over_p = static_cast<T>(u.gamma_over_p);
    r.nsub = static_cast<T>(u.nsub);
    r.coin = u.coin;
    r.plain = u.plain;
    return r;
}

static int strip_key(int strip) { return strip == 8 || strip == 4 ? strip : 1; }
static int np_key(int passes) { return passes >= 1 && passes <= 4 ? passes : 0; }

// All calls of one dtype: scatter launches grouped by (passes, strip, waves), then the combines.
// XCD order for a scatter launch whose items all take all angles (see k_backproject).
template <typename T>
static void mark_xcd_order(WorkList<BackItem<T>> &wl) {
    bool all = true;
    for (int k = 0; k < wl.count; ++k) all = all && wl.item[k].subset < 0;
    for (int k = 0; k < wl.count; ++k) wl.item[k].xcd = all ? 1 : 0;
}

template <typename T>
static ps_status backproject_many_t(const BackCall *calls, int n, hipStream_t st) {
    std::vector<BackItem<T>> items;
    std::vector<BackPlan> plans;
    std::vector<int> call_of;
    // rows per wave {2, 4} x angle split {1, 2, 4} x (sinogram, projector partials)
    ListBuilder<GatherItem<T>> gl[12];
    auto flush_gather = [&](int which) -> ps_status {
        ListBuilder<GatherItem<T>> &b = gl[which];
        if (b.empty()) return PS_OK;
        timer_mark(KC_BP_GATHER, st, true);
        const dim3 grid(b.blocks), block(kBlock);
        switch (which) {
        case 0: hipLaunchKernelGGL((k_backproject_gather<T, 2, 1, false>), grid, block, 0, st, b.wl); break;
        case 1: hipLaunchKernelGGL((k_backproject_gather<T, 2, 2, false>), grid, block, 0, st, b.wl); break;
        case 2: hipLaunchKernelGGL((k_backproject_gather<T, 2, 4, false>), grid, block, 0, st, b.wl); break;
        case 3: hipLaunchKernelGGL((k_backproject_gather<T, 4, 1, false>), grid, block, 0, st, b.wl); break;
        case 4: hipLaunchKernelGGL((k_backproject_gather<T, 4, 2, false>), grid, block, 0, st, b.wl); break;
        case 5: hipLaunchKernelGGL((k_backproject_gather<T, 4, 4, false>), grid, block, 0, st, b.wl); break;
        case 6: hipLaunchKernelGGL((k_backproject_gather<T, 2, 1, true>), grid, block, 0, st, b.wl); break;
        case 7: hipLaunchKernelGGL((k_backproject_gather<T, 2, 2, true>), grid, block, 0, st, b.wl); break;
        case 8: hipLaunchKernelGGL((k_backproject_gather<T, 2, 4, true>), grid, block, 0, st, b.wl); break;
        case 9: hipLaunchKernelGGL((k_backproject_gather<T, 4, 1, true>), grid, block, 0, st, b.wl); break;
        case 10: hipLaunchKernelGGL((k_backproject_gather<T, 4, 2, true>), grid, block, 0, st, b.wl); break;
        default: hipLaunchKernelGGL((k_backproject_gather<T, 4, 4, true>), grid, block, 0, st, b.wl); break;
        }
        PS_LAUNCHED("k_backproject_gather");
        timer_mark(KC_BP_GATHER, st, false);
        b.clear();
        return PS_OK;
    };
    for (int c = 0; c < n; ++c) {
        const BackCall &bc = calls[c];
        const ps_geometry *g = bc.g;
        const auto &d = g->desc;
        if (bc.mode < BP_OVERWRITE || bc.mode > BP_PDHG)
            return fail(PS_EINVAL, "backprojector mode %d", bc.mode);
        if (back_method(g, bc.subset) == BP_GATHER) {
            GatherItem<T> gi{};
            gi.y = static_cast<const T *>(bc.y);
            gi.out = static_cast<T *>(bc.out);
            gi.upd = to_update<T>(bc.upd);
            gi.tab = angle_tab<T>(g);
            gi.subset = bc.subset;
            gi.nsub = d.n_subsets;
            gi.na = subset_count(g, bc.subset);
            gi.nx = d.nx;
            gi.ny = d.ny;
            gi.nbins = d.n_bins;
            const int rows = bc.rows == 2 || bc.rows == 4 ? bc.rows : gather_rows(g, bc.subset);
            const int split = gather_split(g, bc.subset);
            int which = (rows == 2 ? 0 : 3) + (split == 1 ? 0 : split == 2 ? 1 : 2);
            const int tile_rows = (4 / split) * rows;
            gi.tiles_x = (d.nx + kGatherTX - 1) / kGatherTX;
            gi.tiles_y = (d.ny + tile_rows - 1) / tile_rows;
            gi.mode = bc.mode;
            gi.psplit = 1;
            if (bc.psplit > 1) {
                if (bc.subset < 0) return fail(PS_EINVAL, "projector partials given to an all-angle gather");
                gi.psplit = bc.psplit;
                gi.pb = static_cast<const T *>(bc.pb);
                const size_t pstride = static_cast<size_t>(d.nz) * gi.na * d.n_bins * sizeof(T);
                if (pstride * bc.psplit >= (static_cast<size_t>(1) << 32))
                    return fail(PS_EUNSUPPORTED, "projector partials beyond 4 GiB given to the gather");
                gi.pbytes = static_cast<uint32_t>(pstride);
                gi.n_angles = d.n_angles;
                which += 6;
            }
            const long blocks = static_cast<long>(gi.tiles_x) * gi.tiles_y * d.nz;
            if (blocks > (1L << 30)) return fail(PS_EUNSUPPORTED, "backprojector grid too large");
            gl[which].add(gi, static_cast<int>(blocks));
            if (gl[which].full()) PS_TRY(flush_gather(which));
            continue;
        }
        if (bc.psplit > 1) return fail(PS_EINVAL, "projector partials given to the scatter backprojector");
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
                mark_xcd_order(lb.wl);
                PS_TRY(launch_bp_key<T>(np, sk, lb.wl, lb.blocks, waves, lds, st));
                lb.clear();
                lds = 0;
            }
        }
        if (!lb.empty()) {
            mark_xcd_order(lb.wl);
            PS_TRY(launch_bp_key<T>(np, sk, lb.wl, lb.blocks, waves, lds, st));
        }
    }
    // combine + epilogue
    ListBuilder<CombineItem<T>> lb;
    for (size_t i = 0; i < items.size(); ++i) {
        const BackCall &bc = calls[call_of[i]];
        if (bc.partials_only) continue;
        CombineItem<T> ci{};
        ci.part = items[i].part;
        ci.out = static_cast<T *>(bc.out);
        ci.upd = to_update<T>(bc.upd);
        ci.n = static_cast<size_t>(items[i].nx) * items[i].ny * items[i].nz;
        ci.groups = items[i].groups;
        ci.mode = bc.mode;
        ci.blocks = static_cast<int>(std::max<size_t>(1, std::min<size_t>((ci.n + kBlock - 1) / kBlock, 8192)));
        lb.add(ci, ci.blocks);
        if (lb.full()) {
            timer_mark(KC_BP_COMBINE, st, true);
            hipLaunchKernelGGL((k_backproject_combine<T>), dim3(lb.blocks), dim3(kBlock), 0, st, lb.wl);
            PS_LAUNCHED("k_backproject_combine");
            timer_mark(KC_BP_COMBINE, st, false);
            lb.clear();
        }
    }
    if (!lb.empty()) {
        timer_mark(KC_BP_COMBINE, st, true);
        hipLaunchKernelGGL((k_backproject_combine<T>), dim3(lb.blocks), dim3(kBlock), 0, st, lb.wl);
        PS_LAUNCHED("k_backproject_combine");
        timer_mark(KC_BP_COMBINE, st, false);
    }
    for (int which = 0; which < 12; ++which) PS_TRY(flush_gather(which));
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
