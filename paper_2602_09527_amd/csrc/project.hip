// project.hip -- forward projector y = A_i x: ray-driven Joseph interpolation (K1).
//
// One workgroup owns one angle of one slice and every detector bin of it (each thread carries
// up to 8 rays in registers).  The image is walked along the ray's stepping axis in strips that
// are staged in LDS with coalesced loads: rows for row-walked angles, and, for column-walked
// angles, column strips stored transposed, so that in both cases a ray reads two neighbouring
// LDS words per step.  When angles x slices alone cannot fill the chip, the stepping axis is
// also split over `split` workgroups whose partial sums a second pass adds in a fixed order
// (no atomics: results do not depend on the split).
#include <algorithm>

#include "internal.h"

namespace ps {

ProjPlan proj_plan(const ps_geometry *g, int na) {
    const auto &d = g->desc;
    ProjPlan p{};
    const int ext = std::max(d.nx, d.ny);
    p.stride = (ext + 4) | 1;  // odd stride: transposed column-strip stores hit distinct banks
    p.strip = static_cast<int>(std::min<size_t>(32, (64 * 1024) / (p.stride * g->elem)));
    if (p.strip < 1) p.strip = 1;
    p.rpt = d.n_bins <= 256 ? 1 : d.n_bins <= 512 ? 2 : d.n_bins <= 1024 ? 4 : 8;
    const long base = static_cast<long>(std::max(na, 1)) * d.nz;
    const int steps = std::max(d.nx, d.ny);
    const int max_split = std::max(1, steps / 16);
    long want = (2048 + base - 1) / base;
    p.split = static_cast<int>(std::max(1L, std::min<long>(want, max_split)));
    p.lds_bytes = static_cast<size_t>(p.strip) * p.stride * g->elem;
    return p;
}

size_t proj_workspace(const ps_geometry *g, int na) {
    const ProjPlan p = proj_plan(g, na);
    if (p.split <= 1) return 0;
    return align_up(static_cast<size_t>(p.split) * g->desc.nz * na * g->desc.n_bins * g->elem);
}

// Sum over the ray's steps in [s*rb, (s+1)*rb) of the interpolated samples of u = x - xs.
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_project(
    const T *__restrict__ x, const T *__restrict__ xs, AngleTab<T> tab, int subset, int nsub,
    int na, int nx, int ny, int nbins, int split, int strip, int stride,
    T *__restrict__ out, const T *__restrict__ b, int n_angles) {
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const int s = blockIdx.x, l = blockIdx.y, z = blockIdx.z;
    const int k = subset < 0 ? l : subset + l * nsub;
    const bool row = tab.row[k] != 0;
    const T a0 = tab.a0[k], a1 = tab.a1[k], a2 = tab.a2[k];
    const int nsteps = row ? ny : nx;
    const int ext = row ? nx : ny;
    const int rb = (nsteps + split - 1) / split;
    const int t_lo = s * rb;
    const int t_hi = min(nsteps, t_lo + rb);
    const size_t plane = static_cast<size_t>(nx) * ny;
    const T *xz = x + z * plane;
    const T *xsz = xs ? xs + z * plane : nullptr;

    const int64_t q0 = tab.q0[k], q1 = tab.q1[k], q2 = tab.q2[k];
    T acc[RPT];
    T uf[RPT];
    int64_t uq[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        acc[r] = T(0);
        uf[r] = static_cast<T>(threadIdx.x + r * kBlock);
        uq[r] = static_cast<int64_t>(threadIdx.x + r * kBlock) * q1;
    }

    for (int t0 = t_lo; t0 < t_hi; t0 += strip) {
        const int nt = min(strip, t_hi - t0);
        const int cnt = nt * ext;
        if (row) {
            // rows t0..t0+nt-1, contiguous in memory
            for (int e = threadIdx.x; e < cnt; e += kBlock) {
                const int t = e / ext, c = e - t * ext;
                const size_t gi = static_cast<size_t>(t0 + t) * nx + c;
                T v = xz[gi];
                if (xsz) v -= xsz[gi];
                lds[t * stride + 2 + c] = v;
            }
        } else {
            // columns t0..t0+nt-1: read row segments, store transposed (one LDS row per column)
            for (int e = threadIdx.x; e < cnt; e += kBlock) {
                const int c = e / nt, t = e - c * nt;
                const size_t gi = static_cast<size_t>(c) * nx + (t0 + t);
                T v = xz[gi];
                if (xsz) v -= xsz[gi];
                lds[t * stride + 2 + c] = v;
            }
        }
        // two zero words on each side: out-of-image samples read zeros after clamping
        for (int e = threadIdx.x; e < nt * 4; e += kBlock) {
            const int t = e >> 2, c = e & 3;
            lds[t * stride + (c < 2 ? c : ext + c)] = T(0);
        }
        __syncthreads();

        if constexpr (std::is_same<T, float>::value) {
            // exact 32.32 fixed-point walk: high word = floor(q), low word = weight
            for (int t = 0; t < nt; ++t) {
                const int64_t bt = q0 + static_cast<int64_t>(t0 + t) * q2;
                const T *lrow = lds + t * stride + 2;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int64_t q = bt + uq[r];
                    int j0 = static_cast<int>(q >> 32);
                    const float w = static_cast<float>(static_cast<uint32_t>(q) >> 8) * 0x1p-24f;
                    j0 = min(max(j0, -2), ext);
                    const T v0 = lrow[j0], v1 = lrow[j0 + 1];
                    acc[r] += fma(w, v1, (T(1) - w) * v0);
                }
            }
        } else {
            for (int t = 0; t < nt; ++t) {
                const T bt = fma(static_cast<T>(t0 + t), a2, a0);
                const T *lrow = lds + t * stride + 2;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const T q = fma(uf[r], a1, bt);
                    const T fl = floor(q);
                    const T w = q - fl;
                    int j0 = static_cast<int>(fl);
                    j0 = min(max(j0, -2), ext);
                    const T v0 = lrow[j0], v1 = lrow[j0 + 1];
                    acc[r] += fma(w, v1, (T(1) - w) * v0);
                }
            }
        }
        __syncthreads();
    }

    const int nz_ = gridDim.z;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int u = threadIdx.x + r * kBlock;
        if (u >= nbins) break;
        if (split == 1) {
            T val = acc[r] * tab.inv[k];
            if (b) val -= b[(static_cast<size_t>(z) * n_angles + k) * nbins + u];
            out[(static_cast<size_t>(z) * na + l) * nbins + u] = val;
        } else {
            out[((static_cast<size_t>(s) * nz_ + z) * na + l) * nbins + u] = acc[r];
        }
    }
}

// y = inv_k * sum_s partial[s] (- b): fixed summation order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_project_reduce(
    const T *__restrict__ part, AngleTab<T> tab, int subset, int nsub, int na, int nz, int nbins,
    int split, T *__restrict__ y, const T *__restrict__ b, int n_angles) {
    const size_t total = static_cast<size_t>(nz) * na * nbins;
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < total;
         e += static_cast<size_t>(gridDim.x) * kBlock) {
        const int u = static_cast<int>(e % nbins);
        const size_t zl = e / nbins;
        const int l = static_cast<int>(zl % na);
        const int z = static_cast<int>(zl / na);
        const int k = subset < 0 ? l : subset + l * nsub;
        T acc = T(0);
        for (int s = 0; s < split; ++s) acc += part[s * total + e];
        T val = acc * tab.inv[k];
        if (b) val -= b[(static_cast<size_t>(z) * n_angles + k) * nbins + u];
        y[e] = val;
    }
}

template <typename T>
static ps_status project_t(const ps_geometry *g, int subset, const T *x, const T *xs, const T *b,
                           T *y, void *ws, size_t ws_bytes, hipStream_t st) {
    const auto &d = g->desc;
    const int na = subset_count(g, subset);
    if (na <= 0) return PS_OK;
    const ProjPlan p = proj_plan(g, na);
    const AngleTab<T> tab = angle_tab<T>(g);
    T *out = y;
    if (p.split > 1) {
        const size_t need = proj_workspace(g, na);
        if (!ws || ws_bytes < need)
            return fail(PS_EINVAL, "projector workspace: %zu bytes given, %zu needed", ws_bytes, need);
        out = static_cast<T *>(ws);
    }
    const dim3 grid(p.split, na, d.nz);
    switch (p.rpt) {
#define PS_PROJ_CASE(R)                                                                         \
    case R:                                                                                     \
        hipLaunchKernelGGL((k_project<T, R>), grid, dim3(kBlock), p.lds_bytes, st, x, xs, tab,   \
                           subset, d.n_subsets, na, d.nx, d.ny, d.n_bins, p.split, p.strip,      \
                           p.stride, out, b, d.n_angles);                                        \
        break;
        PS_PROJ_CASE(1)
        PS_PROJ_CASE(2)
        PS_PROJ_CASE(4)
        PS_PROJ_CASE(8)
#undef PS_PROJ_CASE
        default:
            return fail(PS_EUNSUPPORTED, "rays per thread %d", p.rpt);
    }
    PS_LAUNCHED("k_project");
    if (p.split > 1) {
        const size_t total = static_cast<size_t>(d.nz) * na * d.n_bins;
        const unsigned blocks = static_cast<unsigned>(std::min<size_t>((total + kBlock - 1) / kBlock, 65535));
        hipLaunchKernelGGL((k_project_reduce<T>), dim3(blocks), dim3(kBlock), 0, st, out, tab,
                           subset, d.n_subsets, na, d.nz, d.n_bins, p.split, y, b, d.n_angles);
        PS_LAUNCHED("k_project_reduce");
    }
    return PS_OK;
}

ps_status launch_project(const ps_geometry *g, int subset, const void *x, const void *xs,
                         const void *b, void *y, void *ws, size_t ws_bytes, hipStream_t st) {
    if (g->desc.dtype == PS_F64)
        return project_t<double>(g, subset, static_cast<const double *>(x),
                                 static_cast<const double *>(xs), static_cast<const double *>(b),
                                 static_cast<double *>(y), ws, ws_bytes, st);
    return project_t<float>(g, subset, static_cast<const float *>(x), static_cast<const float *>(xs),
                            static_cast<const float *>(b), static_cast<float *>(y), ws, ws_bytes, st);
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
