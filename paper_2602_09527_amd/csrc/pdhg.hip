// pdhg.hip -- the high-accuracy reference x*: PDHG with diagonal preconditioning (Chambolle &
// Pock 2011), the primal-dual method of the reference solution of Sec. 2.1 (data-splitting
// figure), for Eq. 5 written as min F(Kx) + G(x) with K = [A; D]:
//   x+   = P_C(x - tau (A^T y1 + D^T y2))         backprojector, BP_PDHG epilogue (also xbar)
//   xbar = 2 x+ - x
//   y1+  = (y1 + sigma (A xbar - b)) / (1 + sigma)  projector with the dual step fused
//   y2+  = y2 + D xbar / 2 scaled per pixel onto the ball of radius alpha   (k_pdhg_dual)
// with tau = 1 / (column sums of |K|) and sigma = 1 / (row sums of A) (1 on empty rays), 1/2 on
// the rows of D: the preconditioning that needs no norm estimate.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace ps {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *__restrict__ p, T value, size_t n) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock)
        p[e] = value;
}

// sigma = 1 / (row sum of A), 1 where the row is empty (such rays never reach x).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pdhg_sigma(T *__restrict__ sig, size_t m) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < m;
         e += static_cast<size_t>(gridDim.x) * kBlock) {
        const T r = sig[e];
        sig[e] = r > T(0) ? T(1) / r : T(1);
    }
}

// tau = 1 / (column sum of A + column sum of |D|); a pixel enters its own forward differences
// (where they are not the zero last one) and those of its lower neighbours.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pdhg_tau(T *__restrict__ tau, int nx, int ny, int nz) {
    const size_t plane = static_cast<size_t>(nx) * ny, n = plane * nz;
    for (size_t p = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; p < n;
         p += static_cast<size_t>(gridDim.x) * kBlock) {
        const int j = static_cast<int>(p % nx), i = static_cast<int>((p / nx) % ny);
        const int z = static_cast<int>(p / plane);
        int cd = (j < nx - 1) + (j > 0) + (i < ny - 1) + (i > 0);
        if (nz > 1) cd += (z < nz - 1) + (z > 0);
        tau[p] = T(1) / (tau[p] + static_cast<T>(cd));
    }
}

// y2 = y2 + D xbar / 2, each pixel's d-vector scaled onto the ball of radius alpha.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pdhg_dual(const T *__restrict__ xb, T *__restrict__ y2,
                                                      T alpha, int nx, int ny, int nz) {
    const size_t plane = static_cast<size_t>(nx) * ny, n = plane * nz;
    for (size_t p = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; p < n;
         p += static_cast<size_t>(gridDim.x) * kBlock) {
        const int j = static_cast<int>(p % nx), i = static_cast<int>((p / nx) % ny);
        const int z = static_cast<int>(p / plane);
        const T c = xb[p];
        const T gx = j < nx - 1 ? xb[p + 1] - c : T(0);
        const T gy = i < ny - 1 ? xb[p + nx] - c : T(0);
        T v0 = y2[p] + T(0.5) * gx;
        T v1 = y2[n + p] + T(0.5) * gy;
        T v2 = T(0);
        T s2 = v0 * v0 + v1 * v1;
        if (nz > 1) {
            const T gz = z < nz - 1 ? xb[p + plane] - c : T(0);
            v2 = y2[2 * n + p] + T(0.5) * gz;
            s2 += v2 * v2;
        }
        const T nrm = sqrt(s2);
        if (nrm > alpha) {
            const T sc = alpha > T(0) ? alpha / nrm : T(0);
            v0 *= sc;
            v1 *= sc;
            v2 *= sc;
        }
        y2[p] = v0;
        y2[n + p] = v1;
        if (nz > 1) y2[2 * n + p] = v2;
    }
}

static int grid_blocks(size_t n) {
    return static_cast<int>(std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, 8192)));
}

struct PdhgLayout {
    size_t tau, sig, xbar, ones, pws, bws, total;
    size_t pws_bytes, bws_bytes;
};

static PdhgLayout pdhg_layout(const ps_geometry *g) {
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    const size_t m = static_cast<size_t>(d.nz) * d.n_angles * d.n_bins;
    PdhgLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    L.tau = take(n * g->elem);
    L.sig = take(m * g->elem);
    L.xbar = take(n * g->elem);
    L.ones = take(std::max(n, m) * g->elem);
    L.pws_bytes = proj_workspace(g, d.n_angles);
    L.pws = take(L.pws_bytes);
    L.bws_bytes = back_workspace(g, -1);
    L.bws = take(L.bws_bytes);
    L.total = off;
    return L;
}

template <typename T>
static ps_status pdhg_t(const ps_geometry *g, const void *b, void *x, void *y1, void *y2, double alpha,
                        int nonneg, int n_iters, unsigned char *w, const PdhgLayout &L, hipStream_t st) {
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    const size_t m = static_cast<size_t>(d.nz) * d.n_angles * d.n_bins;
    T *tau = reinterpret_cast<T *>(w + L.tau);
    T *sig = reinterpret_cast<T *>(w + L.sig);
    T *ones = reinterpret_cast<T *>(w + L.ones);
    // preconditioners: sigma from A 1, tau from A^T 1 and the counts of D
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_blocks(n)), dim3(kBlock), 0, st, ones, T(1), n);
    PS_LAUNCHED("k_fill");
    PS_TRY(launch_project(g, -1, ones, nullptr, nullptr, sig, w + L.pws, L.pws_bytes, st));
    hipLaunchKernelGGL((k_pdhg_sigma<T>), dim3(grid_blocks(m)), dim3(kBlock), 0, st, sig, m);
    PS_LAUNCHED("k_pdhg_sigma");
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_blocks(m)), dim3(kBlock), 0, st, ones, T(1), m);
    PS_LAUNCHED("k_fill");
    PS_TRY(launch_backproject(g, -1, ones, tau, BP_OVERWRITE, nullptr, w + L.bws, L.bws_bytes, st));
    hipLaunchKernelGGL((k_pdhg_tau<T>), dim3(grid_blocks(n)), dim3(kBlock), 0, st, tau, d.nx, d.ny, d.nz);
    PS_LAUNCHED("k_pdhg_tau");

    UpdateArgs up{};
    up.x = x;
    up.vout = w + L.xbar;
    up.gs = tau;
    up.tab = y2;
    up.nx = d.nx;
    up.ny = d.ny;
    up.nz = d.nz;
    up.nonneg = nonneg;
    ProjCall pc{g, -1, w + L.xbar, nullptr, b, y1, w + L.pws, L.pws_bytes};
    pc.sig = sig;
    for (int k = 0; k < n_iters; ++k) {
        PS_TRY(launch_backproject(g, -1, y1, nullptr, BP_PDHG, &up, w + L.bws, L.bws_bytes, st));
        PS_TRY(launch_project_many(&pc, 1, st));
        hipLaunchKernelGGL((k_pdhg_dual<T>), dim3(grid_blocks(n)), dim3(kBlock), 0, st,
                           reinterpret_cast<const T *>(w + L.xbar), static_cast<T *>(y2),
                           static_cast<T>(alpha), d.nx, d.ny, d.nz);
        PS_LAUNCHED("k_pdhg_dual");
    }
    return PS_OK;
}

}  // namespace ps

using namespace ps;

extern "C" size_t pdhg_workspace_bytes(const ps_geometry *g) {
    if (!g) return 0;
    return pdhg_layout(g).total;
}

extern "C" ps_status pdhg_run(const ps_geometry *g, const void *b, void *x, void *y1, void *y2,
                              double alpha, int32_t nonneg, int32_t n_iters, void *workspace,
                              size_t ws_bytes, void *stream) {
    clear_error();
    if (!g) return fail(PS_EINVAL, "geometry is null");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(PS_EINVAL, "alpha must be >= 0");
    if (nonneg != 0 && nonneg != 1) return fail(PS_EINVAL, "nonneg must be 0 or 1");
    if (n_iters < 0) return fail(PS_EINVAL, "n_iters must be >= 0");
    PS_TRY(check_ready(g));
    PS_TRY(check_ptr(b, "b", g->elem));
    PS_TRY(check_ptr(x, "x", g->elem));
    PS_TRY(check_ptr(y1, "y1", g->elem));
    PS_TRY(check_ptr(y2, "y2", g->elem));
    PS_TRY(check_ptr(workspace, "workspace", kAlign));
    const PdhgLayout L = pdhg_layout(g);
    if (ws_bytes < L.total)
        return fail(PS_EINVAL, "PDHG workspace: %zu bytes given, %zu needed", ws_bytes, L.total);
    unsigned char *w = static_cast<unsigned char *>(workspace);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g->desc.dtype == PS_F64) return pdhg_t<double>(g, b, x, y1, y2, alpha, nonneg, n_iters, w, L, st);
    return pdhg_t<float>(g, b, x, y1, y2, alpha, nonneg, n_iters, w, L, st);
}
