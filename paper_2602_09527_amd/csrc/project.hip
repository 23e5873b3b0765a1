// project.hip -- forward projector y = A_i x: ray-driven Joseph interpolation (K1).
//
// A workgroup owns one angle of one slice and every detector bin of it (each thread carries
// ceil(B/256) rays in registers).  The image is walked along the ray's stepping axis in strips
// of R rows (row-walked angles) or R columns (column-walked angles, stored transposed), staged in
// LDS with 16-byte coalesced loads, four zero words on each side of every staged row.  A ray step
// is then one two-word LDS read and six VALU operations:
//     FP32: Q += q2 (32.32 fixed point), idx = min(hi(Q), ext + 4),
//           acc_v += v0,  acc_d += lo(Q) * (v1 - v0)          (scaled by 2^-32 once at the end)
//     FP64: q = a0 + u a1 + t a2 in double, floor / fraction.
// When angles x slices cannot fill the chip, the stepping axis is split over `split`
// workgroups whose partial sums a second pass adds in a fixed order (no atomics, so results do
// not depend on timing).  A per-workgroup completion counter with a device-scope fence would
// save that launch, but on this chip such a fence writes back the XCD's L2 and costs more.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace ps {

constexpr int kPad = 4;  // zero words left of each staged row (keeps 16-byte alignment)

static int strip_rows(int stride, size_t elem) {
    // largest power of two R in [4, 16] with R staged rows within 34 KB of LDS
    int r = 16;
    while (r > 4 && static_cast<size_t>(r) * stride * elem > 34 * 1024) r >>= 1;
    return r;
}

ProjPlan proj_plan(const ps_geometry *g, int na) {
    const auto &d = g->desc;
    ProjPlan p{};
    const int ext = std::max(d.nx, d.ny);
    // words per staged row: a multiple of 4 (16-byte rows) that is 4 mod 16, so the transposed
    // stores of a column strip (4 rows x 16 image rows per wave) hit 64 distinct banks
    p.stride = (ext + 2 * kPad + 3) / 4 * 4;
    p.stride += ((4 - p.stride % 16) + 16) % 16;
    p.strip = strip_rows(p.stride, g->elem);
    p.rpt = std::max(1, (d.n_bins + kBlock - 1) / kBlock);
    const long base = static_cast<long>(std::max(na, 1)) * d.nz;
    const int max_split = std::max(1, ext / (2 * p.strip));
    const long want = (2048 + base - 1) / base;
    p.split = static_cast<int>(std::max(1L, std::min<long>(want, max_split)));
    const int forced = na == d.n_angles ? g->plan.proj_split_full : g->plan.proj_split_subset;
    if (forced > 0) p.split = std::min(forced, max_split);
    p.lds_bytes = static_cast<size_t>(p.strip) * p.stride * g->elem;
    return p;
}

size_t proj_workspace(const ps_geometry *g, int na) {
    const ProjPlan p = proj_plan(g, na);
    if (p.split <= 1) return 0;
    return align_up(static_cast<size_t>(p.split) * g->desc.nz * na * g->desc.n_bins * g->elem);
}

template <typename T>
struct Vec4 {
    T a, b, c, d;
};

template <typename T>
__device__ inline Vec4<T> load4(const T *p) {
    if constexpr (std::is_same<T, float>::value) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        return Vec4<T>{v.x, v.y, v.z, v.w};
    } else {
        return Vec4<T>{p[0], p[1], p[2], p[3]};
    }
}

template <typename T>
__device__ inline void store4(T *dst, const Vec4<T> &v) {
    if constexpr (std::is_same<T, float>::value) {
        *reinterpret_cast<float4 *>(dst) = make_float4(v.a, v.b, v.c, v.d);
    } else {
        dst[0] = v.a;
        dst[1] = v.b;
        dst[2] = v.c;
        dst[3] = v.d;
    }
}

template <typename T>
__device__ inline Vec4<T> sub4(const Vec4<T> &v, const Vec4<T> &w) {
    return Vec4<T>{v.a - w.a, v.b - w.b, v.c - w.c, v.d - w.d};
}

// 16-byte loads in flight per thread while staging: 8 of x, or 4 each of x and xs.
template <bool kDiff>
constexpr int stage_batch() { return kDiff ? 4 : 8; }

// Stage rows t0 .. t0 + nt - 1 of x (minus xs when kDiff) into LDS, row t at t * stride + kPad.
// Element e = t * (ext / 4) + c is a group of 4 columns; each thread takes every kBlock-th one.
// Every load of a batch is issued before the first subtraction or store, so their latencies
// overlap.  Elements past the end load element 0 instead (always in bounds) and are not stored.
template <bool kDiff, typename T>
__device__ inline void stage_rows(T *lds, const T *xz, const T *xsz, int t0, int nt, int ext, int nx,
                                  int stride) {
    constexpr int NB = stage_batch<kDiff>();
    const int q4 = ext / 4, cnt = nt * q4;
    // (t, c) of this thread's next element, advanced by kBlock elements without dividing
    int t = threadIdx.x / q4, c = threadIdx.x - t * q4;
    const int adv_t = kBlock / q4, adv_c = kBlock - adv_t * q4;
    for (int b0 = 0; b0 < cnt; b0 += NB * kBlock) {
        uint32_t g[NB];
        int l[NB];
        bool ok[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            ok[u] = b0 + u * kBlock + static_cast<int>(threadIdx.x) < cnt;
            g[u] = ok[u] ? static_cast<uint32_t>(t0 + t) * nx + 4 * c : 0u;
            l[u] = t * stride + kPad + 4 * c;
            t += adv_t;
            c += adv_c;
            if (c >= q4) {
                c -= q4;
                ++t;
            }
        }
        Vec4<T> v[NB], w[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) v[u] = load4(xz + g[u]);
        if constexpr (kDiff) {
#pragma unroll
            for (int u = 0; u < NB; ++u) w[u] = load4(xsz + g[u]);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u)
            if (ok[u]) store4(lds + l[u], kDiff ? sub4(v[u], w[u]) : v[u]);
    }
}

// Stage columns t0 .. t0 + nt - 1 of x (minus xs) into LDS transposed: column t0 + t at
// t * stride + kPad.  Element e is a group of 4 adjacent columns (e % (strip / 4)) of image row
// e / (strip / 4); its 4 values go to 4 staged rows.  Loads as in stage_rows.
template <bool kDiff, typename T>
__device__ inline void stage_cols(T *lds, const T *xz, const T *xsz, int t0, int nt, int ext, int nx,
                                  int stride, int strip) {
    constexpr int NB = stage_batch<kDiff>();
    const int g4 = strip / 4, g4s = __builtin_ctz(g4), cnt = ext * g4;
    for (int b0 = 0; b0 < cnt; b0 += NB * kBlock) {
        uint32_t g[NB];
        int l[NB];
        bool ok[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = b0 + u * kBlock + static_cast<int>(threadIdx.x);
            const int i = e >> g4s, cg = e & (g4 - 1);
            ok[u] = e < cnt && 4 * cg < nt;
            g[u] = ok[u] ? static_cast<uint32_t>(i) * nx + t0 + 4 * cg : 0u;
            l[u] = 4 * cg * stride + kPad + i;
        }
        Vec4<T> v[NB], w[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) v[u] = load4(xz + g[u]);
        if constexpr (kDiff) {
#pragma unroll
            for (int u = 0; u < NB; ++u) w[u] = load4(xsz + g[u]);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            if (ok[u]) {
                const Vec4<T> d = kDiff ? sub4(v[u], w[u]) : v[u];
                T *dst = lds + l[u];
                dst[0] = d.a;
                dst[stride] = d.b;
                dst[2 * stride] = d.c;
                dst[3 * stride] = d.d;
            }
        }
    }
}

// One projector application: y = inv * A_sub (x - xs) [- b_sub], or partial sums when split.
template <typename T>
struct ProjItem {
    const T *x, *xs, *b, *sig;
    T *out, *part;
    AngleTab<T> tab;
    int subset, nsub, na, nx, ny, nz, nbins, n_angles;
    int split, strip, stride, vec;
};

template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_project(WorkList<ProjItem<T>> wl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr bool kFixed = std::is_same<T, float>::value;

    int local;
    const ProjItem<T> &it = wl.item[work_item(wl, local)];
    const T *__restrict__ x = it.x;
    const T *__restrict__ xs = it.xs;
    const T *__restrict__ b = it.b;
    T *__restrict__ out = it.out;
    T *__restrict__ part = it.part;
    const AngleTab<T> &tab = it.tab;
    const int subset = it.subset, nsub = it.nsub, na = it.na, nx = it.nx, ny = it.ny;
    const int nbins = it.nbins, n_angles = it.n_angles, split = it.split, strip = it.strip;
    const int stride = it.stride, vec = it.vec;
    // workgroup -> (split s, angle l, slice z), s fastest
    const int s = local % split, l = (local / split) % na, z = local / (split * na);
    const int k = subset < 0 ? l : subset + l * nsub;
    const bool row = tab.row[k] != 0;
    const int nsteps = row ? ny : nx;
    const int ext = row ? nx : ny;
    // steps of this workgroup: a multiple of the strip, so column strips stay 16-byte aligned
    const int rb = ((nsteps + split - 1) / split + strip - 1) / strip * strip;
    const int t_lo = s * rb;
    const int t_hi = min(nsteps, t_lo + rb);
    const size_t plane = static_cast<size_t>(nx) * ny;
    const T *xz = x + z * plane;
    const T *xsz = xs ? xs + z * plane : nullptr;
    const uint32_t lim = static_cast<uint32_t>(ext + kPad);

    // zero pads: kPad words left of each row, everything right of ext
    {
        const int npad = stride - ext;  // kPad on the left, the rest on the right
        for (int e = threadIdx.x; e < strip * npad; e += kBlock) {
            const int t = e / npad, c = e - t * npad;
            lds[t * stride + (c < kPad ? c : ext + c)] = T(0);
        }
    }

    const int64_t q1 = tab.q1[k], q2 = tab.q2[k];
    const int64_t q0b = tab.q0[k] + (static_cast<int64_t>(kPad) << 32);  // hi(Q) = j0 + kPad
    const T a0 = tab.a0[k], a1 = tab.a1[k], a2 = tab.a2[k];
    T acc_v[RPT], acc_d[RPT];
    int64_t uq[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        acc_v[r] = T(0);
        acc_d[r] = T(0);
        uq[r] = static_cast<int64_t>(threadIdx.x + r * kBlock) * q1;
    }

    for (int t0 = t_lo; t0 < t_hi; t0 += strip) {
        const int nt = min(strip, t_hi - t0);
        if (vec) {
            // 16-byte loads and stores (FP32 rows are 16-byte aligned: nx % 4 == 0)
            if (row) {
                if (xsz) stage_rows<true>(lds, xz, xsz, t0, nt, ext, nx, stride);
                else stage_rows<false>(lds, xz, xsz, t0, nt, ext, nx, stride);
            } else {
                if (xsz) stage_cols<true>(lds, xz, xsz, t0, nt, ext, nx, stride, strip);
                else stage_cols<false>(lds, xz, xsz, t0, nt, ext, nx, stride, strip);
            }
        } else if (row) {
            for (int e = threadIdx.x; e < nt * ext; e += kBlock) {
                const int t = e / ext, c = e - t * ext;
                const size_t gi = static_cast<size_t>(t0 + t) * nx + c;
                lds[t * stride + kPad + c] = xsz ? xz[gi] - xsz[gi] : xz[gi];
            }
        } else {
            for (int e = threadIdx.x; e < nt * ext; e += kBlock) {
                const int i = e / nt, t = e - i * nt;
                const size_t gi = static_cast<size_t>(i) * nx + t0 + t;
                lds[t * stride + kPad + i] = xsz ? xz[gi] - xsz[gi] : xz[gi];
            }
        }
        __syncthreads();

        if constexpr (kFixed) {
            int64_t q[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) q[r] = q0b + static_cast<int64_t>(t0) * q2 + uq[r];
            for (int t = 0; t < nt; ++t) {
                const T *lrow = lds + t * stride;
                T v0[RPT], v1[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const uint32_t idx = min(static_cast<uint32_t>(q[r] >> 32), lim);
                    v0[r] = lrow[idx];
                    v1[r] = lrow[idx + 1];
                }
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    acc_v[r] += v0[r];
                    acc_d[r] = fma(static_cast<T>(static_cast<uint32_t>(q[r])), v1[r] - v0[r], acc_d[r]);
                    q[r] += q2;
                }
            }
        } else {
            for (int t = 0; t < nt; ++t) {
                const T bt = fma(static_cast<T>(t0 + t), a2, a0);
                const T *lrow = lds + t * stride;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const T q = fma(static_cast<T>(threadIdx.x + r * kBlock), a1, bt);
                    const T fl = floor(q);
                    const uint32_t idx = min(static_cast<uint32_t>(static_cast<int>(fl) + kPad), lim);
                    const T v0 = lrow[idx], v1 = lrow[idx + 1];
                    acc_v[r] += v0;
                    acc_d[r] = fma(q - fl, v1 - v0, acc_d[r]);
                }
            }
        }
        __syncthreads();
    }

    const int nz_ = it.nz;
    const T dscale = kFixed ? T(0x1p-32f) : T(1);
    const T inv = tab.inv[k];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int u = threadIdx.x + r * kBlock;
        if (u >= nbins) break;
        const T acc = fma(acc_d[r], dscale, acc_v[r]);
        if (split == 1) {
            T val = acc * inv;
            if (b) val -= b[(static_cast<size_t>(z) * n_angles + k) * nbins + u];
            const size_t o = (static_cast<size_t>(z) * na + l) * nbins + u;
            if (it.sig) {
                const T sg = it.sig[o];
                val = (out[o] + sg * val) / (T(1) + sg);
            }
            out[o] = val;
        } else {
            part[((static_cast<size_t>(s) * nz_ + z) * na + l) * nbins + u] = acc;
        }
    }
}

// y = inv_k * sum_s partial[s] (- b): fixed summation order, loads issued eight at a time.
template <typename T>
struct ReduceItem {
    const T *part, *b, *inv;
    const T *sig;   // PDHG dual step (see ProjItem), or null
    T *y;
    int subset, nsub, na, nz, nbins, split, n_angles, blocks;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_project_reduce(WorkList<ReduceItem<T>> wl) {
    int local;
    const ReduceItem<T> &it = wl.item[work_item(wl, local)];
    const T *__restrict__ part = it.part;
    const T *__restrict__ b = it.b;
    T *__restrict__ y = it.y;
    const int na = it.na, nbins = it.nbins, split = it.split;
    const size_t total = static_cast<size_t>(it.nz) * na * nbins;
    for (size_t e = local * static_cast<size_t>(kBlock) + threadIdx.x; e < total;
         e += static_cast<size_t>(it.blocks) * kBlock) {
        // (ray, angle, slice) of element e: 32-bit divisions (every sinogram here has fewer than
        // 2^32 elements; a 64-bit division is a long software sequence on this chip)
        const uint32_t e32 = static_cast<uint32_t>(e);
        const uint32_t zl = e32 / static_cast<uint32_t>(nbins);
        const int u = static_cast<int>(e32 - zl * static_cast<uint32_t>(nbins));
        const int z = static_cast<int>(zl / static_cast<uint32_t>(na));
        const int l = static_cast<int>(zl - static_cast<uint32_t>(z) * static_cast<uint32_t>(na));
        const int k = it.subset < 0 ? l : it.subset + l * it.nsub;
        // fixed order over the split partials; a batch's 8 loads are unconditional (clamped to
        // the last partial) so that they are all in flight before the first add
        T acc = T(0);
        for (int s0 = 0; s0 < split; s0 += 8) {
            T v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = part[static_cast<size_t>(min(s0 + q, split - 1)) * total + e];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc = s0 + q < split ? acc + v[q] : acc;
        }
        // one rounding with b (an explicit FMA, so that no contraction choice of the compiler
        // decides the bits: the subset gather that adds the partials itself repeats this form)
        T val = b ? fma(acc, it.inv[k], -b[(static_cast<size_t>(z) * it.n_angles + k) * nbins + u])
                  : acc * it.inv[k];
        if (it.sig) {
            const T sg = it.sig[e];
            val = (y[e] + sg * val) / (T(1) + sg);
        }
        y[e] = val;
    }
}

template <typename T, int R>
static ps_status launch_proj_list(const WorkList<ProjItem<T>> &wl, int blocks, size_t lds,
                                  hipStream_t st) {
    const int kc = wl.item[0].subset < 0 ? KC_PROJECT_FULL : KC_PROJECT_SUBSET;
    timer_mark(kc, st, true);
    hipLaunchKernelGGL((k_project<T, R>), dim3(blocks), dim3(kBlock), lds, st, wl);
    PS_LAUNCHED("k_project");
    timer_mark(kc, st, false);
    return PS_OK;
}

template <typename T>
static ps_status launch_proj_rpt(int rpt, const WorkList<ProjItem<T>> &wl, int blocks, size_t lds,
                                 hipStream_t st) {
    switch (rpt) {
        case 1: return launch_proj_list<T, 1>(wl, blocks, lds, st);
        case 2: return launch_proj_list<T, 2>(wl, blocks, lds, st);
        case 3: return launch_proj_list<T, 3>(wl, blocks, lds, st);
        case 4: return launch_proj_list<T, 4>(wl, blocks, lds, st);
        case 5: return launch_proj_list<T, 5>(wl, blocks, lds, st);
        case 6: return launch_proj_list<T, 6>(wl, blocks, lds, st);
        case 7: return launch_proj_list<T, 7>(wl, blocks, lds, st);
        case 8: return launch_proj_list<T, 8>(wl, blocks, lds, st);
        default: return fail(PS_EUNSUPPORTED, "rays per thread %d", rpt);
    }
}

// All calls of one dtype: projector launches grouped by rays per thread, then the reductions.
template <typename T>
static ps_status project_many_t(const ProjCall *calls, int n, hipStream_t st) {
    std::vector<ProjItem<T>> items;
    std::vector<ProjPlan> plans;
    std::vector<bool> reduce;   // the item's split-ray sum runs
    items.reserve(n);
    plans.reserve(n);
    for (int c = 0; c < n; ++c) {
        const ProjCall &pc = calls[c];
        const ps_geometry *g = pc.g;
        const auto &d = g->desc;
        const int na = subset_count(g, pc.subset);
        if (na <= 0) continue;
        const ProjPlan p = proj_plan(g, na);
        T *part = nullptr;
        if (p.split > 1) {
            const size_t need = proj_workspace(g, na);
            if (!pc.ws || pc.ws_bytes < need)
                return fail(PS_EINVAL, "projector workspace: %zu bytes given, %zu needed", pc.ws_bytes, need);
            part = static_cast<T *>(pc.ws);
        }
        // 16-byte staging needs rows (and column strips) that start on 16-byte boundaries
        const bool aligned = reinterpret_cast<uintptr_t>(pc.x) % 16 == 0 &&
                             (!pc.xs || reinterpret_cast<uintptr_t>(pc.xs) % 16 == 0);
        ProjItem<T> it{};
        it.x = static_cast<const T *>(pc.x);
        it.xs = static_cast<const T *>(pc.xs);
        it.b = static_cast<const T *>(pc.b);
        it.sig = static_cast<const T *>(pc.sig);
        it.out = static_cast<T *>(pc.y);
        it.part = part;
        it.tab = angle_tab<T>(g);
        it.subset = pc.subset;
        it.nsub = d.n_subsets;
        it.na = na;
        it.nx = d.nx;
        it.ny = d.ny;
        it.nz = d.nz;
        it.nbins = d.n_bins;
        it.n_angles = d.n_angles;
        it.split = p.split;
        it.strip = p.strip;
        it.stride = p.stride;
        it.vec = (d.nx % 4 == 0 && aligned && sizeof(T) == 4) ? 1 : 0;
        items.push_back(it);
        plans.push_back(p);
        reduce.push_back(!pc.first_pass_only);
    }
    // projector: one list per rays-per-thread value, flushed every kMaxItems items
    for (int rpt = 1; rpt <= 8; ++rpt) {
        ListBuilder<ProjItem<T>> lb;
        size_t lds = 0;
        for (size_t i = 0; i < items.size(); ++i) {
            if (plans[i].rpt != rpt) continue;
            const long blocks = static_cast<long>(plans[i].split) * items[i].na * items[i].nz;
            if (blocks > (1L << 30)) return fail(PS_EUNSUPPORTED, "projector grid too large");
            lb.add(items[i], static_cast<int>(blocks));
            lds = std::max(lds, plans[i].lds_bytes);
            if (lb.full()) {
                PS_TRY(launch_proj_rpt<T>(rpt, lb.wl, lb.blocks, lds, st));
                lb.clear();
                lds = 0;
            }
        }
        if (!lb.empty()) PS_TRY(launch_proj_rpt<T>(rpt, lb.wl, lb.blocks, lds, st));
    }
    // reductions of the split items
    ListBuilder<ReduceItem<T>> lb;
    for (size_t i = 0; i < items.size(); ++i) {
        if (plans[i].split <= 1 || !reduce[i]) continue;
        const ProjItem<T> &pi = items[i];
        ReduceItem<T> r{};
        r.part = pi.part;
        r.b = pi.b;
        r.sig = pi.sig;
        r.inv = pi.tab.inv;
        r.y = pi.out;
        r.subset = pi.subset;
        r.nsub = pi.nsub;
        r.na = pi.na;
        r.nz = pi.nz;
        r.nbins = pi.nbins;
        r.split = pi.split;
        r.n_angles = pi.n_angles;
        const size_t total = static_cast<size_t>(pi.nz) * pi.na * pi.nbins;
        if (total >= (static_cast<size_t>(1) << 32))
            return fail(PS_EUNSUPPORTED, "a split projection of %zu rays (at most 2^32 - 1)", total);
        r.blocks = static_cast<int>(std::min<size_t>((total + kBlock - 1) / kBlock, 65535));
        lb.add(r, r.blocks);
        if (lb.full()) {
            timer_mark(KC_PROJECT_REDUCE, st, true);
            hipLaunchKernelGGL((k_project_reduce<T>), dim3(lb.blocks), dim3(kBlock), 0, st, lb.wl);
            PS_LAUNCHED("k_project_reduce");
            timer_mark(KC_PROJECT_REDUCE, st, false);
            lb.clear();
        }
    }
    if (!lb.empty()) {
        timer_mark(KC_PROJECT_REDUCE, st, true);
        hipLaunchKernelGGL((k_project_reduce<T>), dim3(lb.blocks), dim3(kBlock), 0, st, lb.wl);
        PS_LAUNCHED("k_project_reduce");
        timer_mark(KC_PROJECT_REDUCE, st, false);
    }
    return PS_OK;
}

ps_status launch_project_many(const ProjCall *calls, int n, hipStream_t st) {
    std::vector<ProjCall> f32, f64;
    for (int c = 0; c < n; ++c) (calls[c].g->desc.dtype == PS_F64 ? f64 : f32).push_back(calls[c]);
    if (!f32.empty()) PS_TRY(project_many_t<float>(f32.data(), static_cast<int>(f32.size()), st));
    if (!f64.empty()) PS_TRY(project_many_t<double>(f64.data(), static_cast<int>(f64.size()), st));
    return PS_OK;
}

ps_status launch_project(const ps_geometry *g, int subset, const void *x, const void *xs,
                         const void *b, void *y, void *ws, size_t ws_bytes, hipStream_t st) {
    const ProjCall c{g, subset, x, xs, b, y, ws, ws_bytes};
    return launch_project_many(&c, 1, st);
}

}  // namespace ps

using namespace ps;

extern "C" size_t project_workspace_bytes(const ps_geometry *g, int32_t subset) {
    if (!g) return 0;
    const int na = subset_count(g, subset);
    return na > 0 ? proj_workspace(g, na) : 0;
}

extern "C" ps_status project_subset(const ps_geometry *g, int32_t subset, const void *x, void *y,
                                    void *workspace, size_t ws_bytes, void *stream) {
    clear_error();
    PS_TRY(check_ready(g));
    if (subset_count(g, subset) < 0) return fail(PS_EINVAL, "subset %d out of range", subset);
    PS_TRY(check_ptr(x, "x", g->elem));
    PS_TRY(check_ptr(y, "y", g->elem));
    return launch_project(g, subset, x, nullptr, nullptr, y, workspace, ws_bytes,
                          static_cast<hipStream_t>(stream));
}
