// backproject.hip -- adjoint x = A_i^T y, voxel-driven gather (K2), with the SVRG / ProxSkip
// gradient step fused into its epilogue.
//
// A workgroup owns a tx x ty pixel tile of one slice, one thread per pixel.  Angles are taken in
// chunks: for each angle of a chunk the detector bins that can touch the tile (its footprint,
// a short run of bins) are staged in LDS, already scaled by the path length 1/|cos| or 1/|sin|.
// A pixel then reads the few bins whose Joseph walk passes within one pixel of it: along the
// walk's interpolation axis the pixel's weight in ray u is the tent max(0, 1 - |q_u - j|),
// where q_u is computed with exactly the expression the projector uses, so both kernels apply
// the same interpolation weights.  Every pixel is summed by one thread in a fixed angle order.
#include <algorithm>

#include "internal.h"

namespace ps {

template <typename T>
struct UpdateT {
    T *x;
    const T *h;
    T *gs;
    T *vout;
    T gamma, gamma_over_p, nsub;
    int coin, plain;
};

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_backproject(
    const T *__restrict__ y, AngleTab<T> tab, int subset, int nsub_angles, int na, int nx, int ny,
    int nbins, int chunk, int slot, int ncand, T *__restrict__ out, UpdateT<T> upd) {
    extern __shared__ unsigned char smem_raw[];
    T *ys = reinterpret_cast<T *>(smem_raw);
    __shared__ int ulo_s[64];

    const int tx = blockDim.x, ty = blockDim.y;
    const int tid = threadIdx.y * tx + threadIdx.x;
    const int j = blockIdx.x * tx + threadIdx.x;
    const int i = blockIdx.y * ty + threadIdx.y;
    const int z = blockIdx.z;
    const int j_lo = blockIdx.x * tx, j_hi = min(j_lo + tx, nx) - 1;
    const int i_lo = blockIdx.y * ty, i_hi = min(i_lo + ty, ny) - 1;
    const bool inside = (i < ny) && (j < nx);
    const T *yz = y + static_cast<size_t>(z) * na * nbins;

    T acc = T(0);
    for (int c0 = 0; c0 < na; c0 += chunk) {
        const int nca = min(chunk, na - c0);
        if (tid < nca) {
            // footprint of the tile in detector bins for angle c0 + tid
            const int l = c0 + tid;
            const int k = subset < 0 ? l : subset + l * nsub_angles;
            const bool row = tab.row[k] != 0;
            const T a0 = tab.a0[k], a2 = tab.a2[k], ia1 = tab.ia1[k];
            const T t_lo = static_cast<T>(row ? j_lo : i_lo), t_hi = static_cast<T>(row ? j_hi : i_hi);
            const T s_lo = static_cast<T>(row ? i_lo : j_lo), s_hi = static_cast<T>(row ? i_hi : j_hi);
            const T b_lo = fma(s_lo, a2, a0), b_hi = fma(s_hi, a2, a0);
            const T u1 = (t_lo - b_lo) * ia1, u2 = (t_hi - b_lo) * ia1;
            const T u3 = (t_lo - b_hi) * ia1, u4 = (t_hi - b_hi) * ia1;
            const T umin = min(min(u1, u2), min(u3, u4));
            ulo_s[tid] = static_cast<int>(floor(umin - fabs(ia1))) - 2;
        }
        __syncthreads();
        for (int e = tid; e < nca * slot; e += tx * ty) {
            const int a = e / slot, o = e - a * slot;
            const int l = c0 + a;
            const int k = subset < 0 ? l : subset + l * nsub_angles;
            const int u = ulo_s[a] + o;
            ys[e] = (u >= 0 && u < nbins) ? yz[static_cast<size_t>(l) * nbins + u] * tab.inv[k] : T(0);
        }
        __syncthreads();
        if (inside) {
            for (int a = 0; a < nca; ++a) {
                const int l = c0 + a;
                const int k = subset < 0 ? l : subset + l * nsub_angles;
                const bool row = tab.row[k] != 0;
                const T a0 = tab.a0[k], a1 = tab.a1[k], a2 = tab.a2[k], ia1 = tab.ia1[k];
                const T along = static_cast<T>(row ? i : j);
                const T target = static_cast<T>(row ? j : i);
                const T bi = fma(along, a2, a0);
                const T ustar = (target - bi) * ia1;
                const int first = static_cast<int>(floor(ustar - fabs(ia1))) + 1;
                const T *slot_a = ys + a * slot;
                const int base = first - ulo_s[a];
                if constexpr (std::is_same<T, float>::value) {
                    // D = q(u) - target in 32.32 fixed point, exactly as the projector walks it:
                    // D in [0, 1): the pixel is the left sample (weight 1 - w); D in [-1, 0): the
                    // right sample (weight w); w = the projector's truncated low word.
                    const int64_t q1 = tab.q1[k];
                    const int64_t bt = tab.q0[k] + static_cast<int64_t>(row ? i : j) * tab.q2[k];
                    int64_t D = bt + static_cast<int64_t>(first) * q1 -
                                (static_cast<int64_t>(row ? j : i) << 32);
                    for (int c = 0; c < ncand; ++c) {
                        const int hi = static_cast<int>(D >> 32);
                        const float w = static_cast<float>(static_cast<uint32_t>(D) >> 8) * 0x1p-24f;
                        const float wt = hi == 0 ? 1.0f - w : (hi == -1 ? w : 0.0f);
                        const int o = min(max(base + c, 0), slot - 1);
                        acc = fma(wt, slot_a[o], acc);
                        D += q1;
                    }
                } else {
                    for (int c = 0; c < ncand; ++c) {
                        const int u = first + c;
                        const T q = fma(static_cast<T>(u), a1, bi);
                        const T wt = max(T(0), T(1) - fabs(q - target));
                        const int o = min(max(base + c, 0), slot - 1);
                        acc = fma(wt, slot_a[o], acc);
                    }
                }
            }
        }
        __syncthreads();
    }

    if (!inside) return;
    const size_t p = (static_cast<size_t>(z) * ny + i) * nx + j;
    if (MODE == BP_OVERWRITE) {
        out[p] = acc;
    } else if (MODE == BP_ACCUMULATE) {
        out[p] += acc;
    } else {
        T G;
        if (MODE == BP_SNAPSHOT) {
            upd.gs[p] = acc;
            G = acc;
        } else {
            G = fma(upd.nsub, acc, upd.gs[p]);
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

template <typename T>
static ps_status backproject_t(const ps_geometry *g, int subset, const T *y, T *out, int mode,
                               const UpdateArgs *u, hipStream_t st) {
    const auto &d = g->desc;
    const int na = subset_count(g, subset);
    const BackPlan &bp = g->bplan;
    const AngleTab<T> tab = angle_tab<T>(g);
    UpdateT<T> ut{};
    if (u) {
        ut.x = static_cast<T *>(u->x);
        ut.h = static_cast<const T *>(u->h);
        ut.gs = static_cast<T *>(u->gs);
        ut.vout = static_cast<T *>(u->vout);
        ut.gamma = static_cast<T>(u->gamma);
        ut.gamma_over_p = static_cast<T>(u->gamma_over_p);
        ut.nsub = static_cast<T>(u->nsub);
        ut.coin = u->coin;
        ut.plain = u->plain;
    }
    const dim3 block(bp.tx, bp.ty);
    const dim3 grid((d.nx + bp.tx - 1) / bp.tx, (d.ny + bp.ty - 1) / bp.ty, d.nz);
    const int chunk = std::min(bp.chunk, 64);
    switch (mode) {
#define PS_BP_CASE(M)                                                                           \
    case M:                                                                                     \
        hipLaunchKernelGGL((k_backproject<T, M>), grid, block, bp.lds_bytes, st, y, tab, subset,  \
                           d.n_subsets, na, d.nx, d.ny, d.n_bins, chunk, bp.slot, bp.ncand, out, \
                           ut);                                                                  \
        break;
        PS_BP_CASE(BP_OVERWRITE)
        PS_BP_CASE(BP_ACCUMULATE)
        PS_BP_CASE(BP_SVRG)
        PS_BP_CASE(BP_SNAPSHOT)
#undef PS_BP_CASE
        default:
            return fail(PS_EINVAL, "backprojector mode %d", mode);
    }
    PS_LAUNCHED("k_backproject");
    return PS_OK;
}

ps_status launch_backproject(const ps_geometry *g, int subset, const void *y, void *out, int mode,
                             const UpdateArgs *upd, hipStream_t st) {
    if (g->desc.dtype == PS_F64)
        return backproject_t<double>(g, subset, static_cast<const double *>(y),
                                     static_cast<double *>(out), mode, upd, st);
    return backproject_t<float>(g, subset, static_cast<const float *>(y), static_cast<float *>(out),
                                mode, upd, st);
}

}  // namespace ps

using namespace ps;

extern "C" ps_status backproject_subset(const ps_geometry *g, int32_t subset, const void *y,
                                        void *x, int32_t accumulate, void *stream) {
    clear_error();
    PS_TRY(check_ready(g));
    if (subset_count(g, subset) < 0) return fail(PS_EINVAL, "subset %d out of range", subset);
    PS_TRY(check_ptr(y, "y", g->elem));
    PS_TRY(check_ptr(x, "x", g->elem));
    if (accumulate != 0 && accumulate != 1) return fail(PS_EINVAL, "accumulate must be 0 or 1");
    return launch_backproject(g, subset, y, x, accumulate ? BP_ACCUMULATE : BP_OVERWRITE, nullptr,
                              static_cast<hipStream_t>(stream));
}
