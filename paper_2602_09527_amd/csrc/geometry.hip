// geometry.hip -- host side: errors, geometry validation and per-angle tables, random streams.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace ps {

static thread_local std::string g_error;

ps_status fail(ps_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

void clear_error() { g_error.clear(); }

int subset_count(const ps_geometry *g, int subset) {
    const int A = g->desc.n_angles, N = g->desc.n_subsets;
    if (subset == -1) return A;
    if (subset < 0 || subset >= N) return -1;
    // interleaved split: subset i = {i, i+N, i+2N, ...}
    return subset < A ? (A - 1 - subset) / N + 1 : 0;
}

int max_subset_count(const ps_geometry *g) { return subset_count(g, 0); }

ps_status check_ready(const ps_geometry *g) {
    if (!g) return fail(PS_EINVAL, "geometry is null");
    if (!g->dev) return fail(PS_EINVAL, "geometry tables not uploaded (call geometry_upload)");
    return PS_OK;
}

ps_status check_ptr(const void *p, const char *what, size_t align) {
    if (!p) return fail(PS_EINVAL, "%s is null", what);
    if (reinterpret_cast<uintptr_t>(p) % align)
        return fail(PS_EINVAL, "%s is not %zu-byte aligned", what, align);
    return PS_OK;
}

// SplitMix64 (Steele, Lea & Flood 2014) read at counter j: the j-th output of the generator
// whose state starts at `seed` and advances by the golden-ratio increment.
uint64_t splitmix64(uint64_t seed, uint64_t j) {
    uint64_t z = seed + (j + 1u) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

void draw_sequences(uint64_t seed, int64_t k0, int64_t count, int n_subsets, double p,
                    int32_t *subset_out, uint8_t *coin_out) {
    // theta = 1 iff a uniform 53-bit integer falls below p * 2^53 (exact for p in (0, 1]).
    const uint64_t limit = static_cast<uint64_t>(std::floor(std::ldexp(p, 53)));
    for (int64_t t = 0; t < count; ++t) {
        const uint64_t k = static_cast<uint64_t>(k0 + t);
        if (subset_out) {
            const uint64_t hi = splitmix64(seed, 2u * k) >> 32;
            subset_out[t] = static_cast<int32_t>((hi * static_cast<uint64_t>(n_subsets)) >> 32);
        }
        if (coin_out) coin_out[t] = static_cast<uint8_t>((splitmix64(seed, 2u * k + 1u) >> 11) < limit);
    }
}

void draw_refresh(uint64_t seed, int64_t k0, int64_t count, int n_subsets, uint8_t *out) {
    // rho = 1 iff a uniform 53-bit integer falls below floor(2^53 / N), from counters 2^62 + k
    const uint64_t limit = (static_cast<uint64_t>(1) << 53) / static_cast<uint64_t>(n_subsets);
    for (int64_t t = 0; t < count; ++t) {
        const uint64_t j = (static_cast<uint64_t>(1) << 62) + static_cast<uint64_t>(k0 + t);
        out[t] = static_cast<uint8_t>((splitmix64(seed, j) >> 11) < limit);
    }
}

template <typename T>
static void fill_tables(ps_geometry *g, const std::vector<double> &a0, const std::vector<double> &a1,
                        const std::vector<double> &a2, const std::vector<double> &inv,
                        const std::vector<double> &ia1, const std::vector<int32_t> &row) {
    const int A = g->desc.n_angles;
    unsigned char *b = g->host_tab.data();
    T *p0 = reinterpret_cast<T *>(b + g->off_a0), *p1 = reinterpret_cast<T *>(b + g->off_a1);
    T *p2 = reinterpret_cast<T *>(b + g->off_a2), *pi = reinterpret_cast<T *>(b + g->off_inv);
    T *pa = reinterpret_cast<T *>(b + g->off_ia1);
    int32_t *pr = reinterpret_cast<int32_t *>(b + g->off_row);
    int64_t *f0 = reinterpret_cast<int64_t *>(b + g->off_q0);
    int64_t *f1 = reinterpret_cast<int64_t *>(b + g->off_q1);
    int64_t *f2 = reinterpret_cast<int64_t *>(b + g->off_q2);
    for (int k = 0; k < A; ++k) {
        f0[k] = std::llround(std::ldexp(a0[k], 32));
        f1[k] = std::llround(std::ldexp(a1[k], 32));
        f2[k] = std::llround(std::ldexp(a2[k], 32));
        p0[k] = static_cast<T>(a0[k]);
        p1[k] = static_cast<T>(a1[k]);
        p2[k] = static_cast<T>(a2[k]);
        pi[k] = static_cast<T>(inv[k]);
        pa[k] = static_cast<T>(ia1[k]);
        pr[k] = row[k];
    }
}

}  // namespace ps

using namespace ps;

extern "C" ps_status make_geometry(const ps_geometry_desc *d, ps_geometry **out) {
    clear_error();
    if (!d || !out) return fail(PS_EINVAL, "null argument");
    *out = nullptr;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(PS_EINVAL, "image size %d x %d x %d must be positive", d->nx, d->ny, d->nz);
    if (d->nz > 65535) return fail(PS_EUNSUPPORTED, "more than 65535 slices is not supported");
    if (d->n_angles > 65535) return fail(PS_EUNSUPPORTED, "more than 65535 angles is not supported");
    if (d->nx > kMaxDim || d->ny > kMaxDim)
        return fail(PS_EUNSUPPORTED, "image side above %d is not supported", kMaxDim);
    if (d->n_angles < 1) return fail(PS_EINVAL, "n_angles must be >= 1");
    if (d->n_bins < 1) return fail(PS_EINVAL, "n_bins must be >= 1");
    if (d->n_bins > kMaxBins) return fail(PS_EUNSUPPORTED, "n_bins above %d is not supported", kMaxBins);
    if (!(d->bin_width > 0.0) || !std::isfinite(d->bin_width))
        return fail(PS_EINVAL, "bin_width must be positive and finite");
    if (!std::isfinite(d->det_offset)) return fail(PS_EINVAL, "det_offset must be finite");
    if (d->n_subsets < 1 || d->n_subsets > d->n_angles)
        return fail(PS_EINVAL, "n_subsets must be in [1, n_angles]");
    if (d->dtype != PS_F32 && d->dtype != PS_F64) return fail(PS_EINVAL, "unknown dtype");
    const double n_img = static_cast<double>(d->nx) * d->ny * d->nz;
    if (n_img * 4.0 >= 9.0e18) return fail(PS_EUNSUPPORTED, "image too large");

    ps_geometry *g = new (std::nothrow) ps_geometry();
    if (!g) return fail(PS_ENOMEM, "out of host memory");
    g->desc = *d;
    const int A = d->n_angles, B = d->n_bins, nx = d->nx, ny = d->ny;
    g->angles.resize(A);
    for (int k = 0; k < A; ++k) {
        g->angles[k] = d->angles ? d->angles[k] : static_cast<double>(k) * M_PI / A;
        if (!std::isfinite(g->angles[k])) {
            delete g;
            return fail(PS_EINVAL, "angle %d is not finite", k);
        }
    }
    g->desc.angles = g->angles.data();
    g->plan = ps_plan{};
    g->tv_dims = d->nz > 1 ? 3 : 2;
    g->elem = d->dtype == PS_F64 ? sizeof(double) : sizeof(float);
    g->dev = nullptr;

    // Per-angle constants in FP64 (see AngleTab).
    std::vector<double> a0(A), a1(A), a2(A), inv(A), ia1(A);
    std::vector<int32_t> row(A);
    const double du = d->bin_width, s_first = d->det_offset - 0.5 * (B - 1) * du;
    double min_a1 = INFINITY;
    for (int k = 0; k < A; ++k) {
        const double c = std::cos(g->angles[k]), s = std::sin(g->angles[k]);
        if (std::fabs(c) >= std::fabs(s)) {
            row[k] = 1;
            a1[k] = du / c;
            a2[k] = -s / c;
            a0[k] = (s_first + 0.5 * (ny - 1) * s) / c + 0.5 * (nx - 1);
            inv[k] = 1.0 / std::fabs(c);
        } else {
            row[k] = 0;
            a1[k] = du / s;
            a2[k] = -c / s;
            a0[k] = (s_first + 0.5 * (nx - 1) * c) / s + 0.5 * (ny - 1);
            inv[k] = 1.0 / std::fabs(s);
        }
        ia1[k] = 1.0 / a1[k];
        // every ray position q must stay well inside the 32.32 fixed-point range
        const double qmax = std::fabs(a0[k]) + std::fabs(a1[k]) * B +
                            std::fabs(a2[k]) * std::max(nx, ny);
        if (!(qmax < 1073741824.0)) {
            delete g;
            return fail(PS_EUNSUPPORTED, "detector extends too far from the image (|q| >= 2^30)");
        }
        min_a1 = std::min(min_a1, std::fabs(a1[k]));
    }
    // Backprojector passes: rays P apart in one pass are >= 2 pixels apart, so their two
    // deposits never share a pixel (checked in the fixed-point units the FP32 kernels use).
    {
        int64_t min_q1 = INT64_MAX;
        for (int k = 0; k < A; ++k) min_q1 = std::min<int64_t>(min_q1, std::llabs(std::llround(std::ldexp(a1[k], 32))));
        const int64_t two = static_cast<int64_t>(1) << 33;
        const int pass_fixed = static_cast<int>((two + min_q1 - 1) / min_q1);
        const int pass_double = static_cast<int>(std::ceil(2.000001 / min_a1));
        g->bp_passes = d->dtype == PS_F64 ? pass_double : pass_fixed;
        // pixel-driven gather: at most one ray per interpolation cell, so a pixel has at most
        // two contributing rays per angle
        g->gather_ok = d->dtype == PS_F64 ? (min_a1 >= 1.0) : (min_q1 >= (static_cast<int64_t>(1) << 32));
        if (g->bp_passes > 64) {
            delete g;
            return fail(PS_EUNSUPPORTED, "detector bins finer than 1/32 pixel are not supported");
        }
    }

    // Angle lists per subset (and for all angles): row-walked angles first, then column-walked.
    {
        const int N = d->n_subsets;
        g->order_full.clear();
        for (int k = 0; k < A; ++k) if (row[k]) g->order_full.push_back(k);
        g->nrow_full = static_cast<int>(g->order_full.size());
        for (int k = 0; k < A; ++k) if (!row[k]) g->order_full.push_back(k);
        g->order_sub.clear();
        g->sub_off.assign(N + 1, 0);
        g->nrow_sub.assign(N, 0);
        for (int i = 0; i < N; ++i) {
            g->sub_off[i] = static_cast<int>(g->order_sub.size());
            const int na = (A - 1 - i) / N + 1;
            for (int l = 0; l < na; ++l) if (row[i + l * N]) g->order_sub.push_back(l);
            g->nrow_sub[i] = static_cast<int>(g->order_sub.size()) - g->sub_off[i];
            for (int l = 0; l < na; ++l) if (!row[i + l * N]) g->order_sub.push_back(l);
        }
        g->sub_off[N] = static_cast<int>(g->order_sub.size());
    }

    // Device table layout: five T arrays and one int32 array of A entries, each 256-aligned.
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    g->off_a0 = take(A * g->elem);
    g->off_a1 = take(A * g->elem);
    g->off_a2 = take(A * g->elem);
    g->off_inv = take(A * g->elem);
    g->off_ia1 = take(A * g->elem);
    g->off_row = take(A * sizeof(int32_t));
    g->off_q0 = take(A * sizeof(int64_t));
    g->off_q1 = take(A * sizeof(int64_t));
    g->off_q2 = take(A * sizeof(int64_t));
    g->off_ord_full = take(A * sizeof(int32_t));
    g->off_ord_sub = take(A * sizeof(int32_t));
    g->tab_bytes = off;
    g->host_tab.assign(off, 0);
    if (d->dtype == PS_F64)
        fill_tables<double>(g, a0, a1, a2, inv, ia1, row);
    else
        fill_tables<float>(g, a0, a1, a2, inv, ia1, row);
    std::memcpy(g->host_tab.data() + g->off_ord_full, g->order_full.data(), A * sizeof(int32_t));
    std::memcpy(g->host_tab.data() + g->off_ord_sub, g->order_sub.data(), A * sizeof(int32_t));
    *out = g;
    return PS_OK;
}

extern "C" void free_geometry(ps_geometry *g) { delete g; }

extern "C" size_t geometry_device_bytes(const ps_geometry *g) { return g ? g->tab_bytes : 0; }

extern "C" ps_status geometry_upload(ps_geometry *g, void *dev_buf, size_t bytes, void *stream) {
    clear_error();
    if (!g) return fail(PS_EINVAL, "geometry is null");
    PS_TRY(check_ptr(dev_buf, "dev_buf", kAlign));
    if (bytes < g->tab_bytes)
        return fail(PS_EINVAL, "dev_buf holds %zu bytes, %zu needed", bytes, g->tab_bytes);
    PS_HIP(hipMemcpyAsync(dev_buf, g->host_tab.data(), g->tab_bytes, hipMemcpyHostToDevice,
                          static_cast<hipStream_t>(stream)));
    g->dev = dev_buf;
    return PS_OK;
}

extern "C" int32_t subset_size(const ps_geometry *g, int32_t subset) {
    if (!g) return -1;
    return subset_count(g, subset);
}

extern "C" ps_status sample_sequences(uint64_t seed, int64_t k0, int64_t count, int32_t n_subsets,
                                      double p, int32_t *subset_out, uint8_t *coin_out) {
    clear_error();
    if (count < 0 || k0 < 0) return fail(PS_EINVAL, "count and k0 must be >= 0");
    if (n_subsets < 1) return fail(PS_EINVAL, "n_subsets must be >= 1");
    if (!(p > 0.0 && p <= 1.0)) return fail(PS_EINVAL, "p must be in (0, 1]");
    draw_sequences(seed, k0, count, n_subsets, p, subset_out, coin_out);
    return PS_OK;
}

extern "C" ps_status sample_refresh_coins(uint64_t seed, int64_t k0, int64_t count, int32_t n_subsets,
                                          uint8_t *out) {
    clear_error();
    if (count < 0 || k0 < 0) return fail(PS_EINVAL, "count and k0 must be >= 0");
    if (n_subsets < 1) return fail(PS_EINVAL, "n_subsets must be >= 1");
    if (!out && count > 0) return fail(PS_EINVAL, "out is null");
    draw_refresh(seed, k0, count, n_subsets, out);
    return PS_OK;
}

extern "C" const char *last_error_message(void) { return g_error.c_str(); }
