// fgp.hip -- proximal operator of tau (TV + I_C) by FGP (Beck & Teboulle 2009), K4/K5.
//
// Dual form: z(p) = P_C(v - tau D^T p); ascend the dual with step 1/(4 d tau) (||D||^2 <= 4d),
// project each pixel's d-vector onto the unit ball, and extrapolate with the FISTA momentum
// r_k = p_{k-1} + c_k (p_{k-1} - p_{k-2}),  c_k = (t_{k-1} - 1)/t_k,  t_1 = 1,  r_1 = p_0.
//
// 2D (one slice): temporal blocking in registers.  A workgroup owns a 64-column x EY-row tile
// (its interior plus a halo of H = T + 1 pixels) and runs T inner iterations on it before writing
// back; every iteration reaches one pixel further, so the interior is computed exactly as one
// global iteration at a time would, whatever the tile shape.  Lane = column; each of the W waves
// keeps a contiguous block of RW = EY/W rows of (v, p, r, z) in registers, takes horizontal
// neighbours from lane shuffles and exchanges only its first and last rows through LDS.  Between
// launches the state is (p_k, r_{k+1}), the dual and its extrapolation.
// 3D (slices coupled): marching tiles over global memory, one or two whole inner iterations per
// launch (HBM-bound volumes).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

// No implicit fusing of a multiply and an add into one rounding: every fused multiply-add below is
// written as fma(), so each value is rounded the same way in every kernel and tile shape that
// forms it, and the plan's tile, depth and launch form never change results.  Left to the
// compiler, the fusing differs between template instantiations (measured: the 3D iteration on
// 16 x 2 wave tiles differed from 8 x 2 in the last bit).
#pragma clang fp contract(off)

namespace ps {

constexpr int kFgpEX = 64;          // tile width including halos (= one wave)
constexpr int kFgpWaves = 4;
// Inner iterations per 2D launch: at most 16 (FP32) or 8 (FP64), so that a work list of 16 items
// with their momentum coefficients stays within 4 KB of kernel arguments; 8 unless a plan asks.
template <typename T>
constexpr int fgp_max_iters() { return std::is_same<T, double>::value ? 8 : 16; }
constexpr int kFgpAutoIters = 8;
constexpr int kFgpAutoCols = 1;     // columns per lane unless a plan asks

template <typename T>
struct FgpCoef {
    T c[fgp_max_iters<T>()];        // c_{k+1} for the T iterations of this launch
};

template <typename T>
struct FgpFinal {
    int mode;      // 0: intermediate (write p, r), 1: z, 2: proxskip (x, h), 3: plain (x)
    T *z, *x, *h;
    T hscale;
    T *dual_out;
};

// 2D kernel tile: `waves` waves of `rows` image rows each; the tile is waves x rows high
// (halos included).  More waves per tile shorten each wave's serial chain and raise occupancy;
// taller tiles recompute less halo but give fewer workgroups.
struct FgpTile {
    int waves, rows;
    int cols = 1;   // columns per lane (the tile is 64 cols wide)
};
constexpr FgpTile kFgpTiles[] = {{4, 4}, {4, 8}, {8, 2}, {8, 4}, {8, 8}, {16, 2}, {16, 4}};

bool fgp_tile_ok(int waves, int rows) {
    for (const FgpTile &t : kFgpTiles)
        if (t.waves == waves && t.rows == rows) return true;
    return false;
}

// Whole-wave lane shifts through DPP (no LDS traffic): lane i receives lane i - 1 (shr) or
// lane i + 1 (shl); the lane with no source receives 0.
__device__ inline float lane_from_left(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ inline float lane_from_right(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
__device__ inline double lane_from_left(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(__double2loint(v)), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(__double2hiint(v)), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double lane_from_right(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(__double2loint(v)), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(__double2hiint(v)), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// One launch of one FGP solve: `iters` inner iterations on every tile of every slice.
template <typename T>
struct FgpItem {
    const T *v, *p_in, *r_in;
    T *p_out, *r_out;
    size_t ncomp;   // elements between the two dual components ([2][nz][ny][nx])
    int nx, ny, iters, halo, tiles_x, tiles_y, nonneg;
    T tau, step;
    FgpCoef<T> cf;
    FgpFinal<T> fin;
};

// CX columns per lane: the tile is 64 CX columns wide, so its halo of T + 1 columns on each side
// is a smaller share of it (T = 15: 32 of 64 columns are interior with one column per lane, 96 of
// 128 with two).  A lane's two columns are neighbours in registers; across lanes the DPP shifts
// carry the edge columns.  Every value is formed by the same expressions whatever the tile.
template <typename T, int W, int RW, int CX>
__global__ __launch_bounds__(W * kFgpEX) void k_fgp2d(WorkList<FgpItem<T>> wl) {
    static_assert(CX == 1 || CX == 2, "columns per lane");
    constexpr int EY = W * RW;
    constexpr int EX = kFgpEX * CX;
    __shared__ T xch[2][W][CX][kFgpEX];   // last-row values (down) and first-row values (up)
    int local;
    const FgpItem<T> &it = wl.item[work_item(wl, local)];
    const int nx = it.nx, ny = it.ny, halo = it.halo, iters = it.iters, nonneg = it.nonneg;
    const T tau = it.tau, step = it.step;
    const FgpFinal<T> &fin = it.fin;
    const int tx = local % it.tiles_x, ty = (local / it.tiles_x) % it.tiles_y;
    const int zsl = local / (it.tiles_x * it.tiles_y);   // slice (2D TV acts on each slice)
    const size_t n = static_cast<size_t>(nx) * ny;
    const size_t zoff = static_cast<size_t>(zsl) * n;
    const T *__restrict__ v = it.v + zoff;
    const T *__restrict__ p_in = it.p_in + zoff;
    const T *__restrict__ r_in = it.r_in + zoff;
    const int TX = EX - 2 * halo, TY = EY - 2 * halo;
    const int lane = threadIdx.x % kFgpEX, wave = threadIdx.x / kFgpEX;
    const int i0 = ty * TY - halo + wave * RW;   // image row of this wave's row 0
    const int gj0 = tx * TX - halo + CX * lane;  // image column of this lane's column 0
    bool has_left[CX], has_right[CX], col_in[CX];
#pragma unroll
    for (int c = 0; c < CX; ++c) {
        const int gj = gj0 + c;
        col_in[c] = gj >= 0 && gj < nx;
        has_left[c] = gj > 0 && (c > 0 || lane > 0);
        has_right[c] = gj < nx - 1 && (c < CX - 1 || lane < kFgpEX - 1);
    }

    T vv[RW][CX], px[RW][CX], py[RW][CX], rx[RW][CX], ry[RW][CX], zz[RW][CX];
    bool in[RW][CX];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int gi = i0 + r;
#pragma unroll
        for (int c = 0; c < CX; ++c) {
            in[r][c] = col_in[c] && gi >= 0 && gi < ny;
            if (in[r][c]) {
                const size_t q = static_cast<size_t>(gi) * nx + gj0 + c;
                vv[r][c] = v[q];
                px[r][c] = p_in[q];
                py[r][c] = p_in[q + it.ncomp];
                rx[r][c] = r_in[q];
                ry[r][c] = r_in[q + it.ncomp];
            } else {
                vv[r][c] = px[r][c] = py[r][c] = rx[r][c] = ry[r][c] = T(0);
            }
        }
    }

    for (int t = 0; t < iters; ++t) {
        // z = P_C(v - tau D^T r): needs r^x of the left neighbour and r^y of the row above
#pragma unroll
        for (int c = 0; c < CX; ++c) xch[0][wave][c][lane] = ry[RW - 1][c];
        __syncthreads();
        T ry_above[CX];
#pragma unroll
        for (int c = 0; c < CX; ++c) ry_above[c] = wave > 0 ? xch[0][wave - 1][c][lane] : T(0);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int gi = i0 + r;
            const T rxl = lane_from_left(rx[r][CX - 1]);
#pragma unroll
            for (int c = 0; c < CX; ++c) {
                const int gj = gj0 + c;
                const T rx_here = (gj < nx - 1) ? rx[r][c] : T(0);
                const T rx_left = has_left[c] ? (c == 0 ? rxl : rx[r][c > 0 ? c - 1 : 0]) : T(0);
                const T ry_here = (gi < ny - 1) ? ry[r][c] : T(0);
                const T ry_up = (gi > 0) ? (r > 0 ? ry[r > 0 ? r - 1 : 0][c] : ry_above[c]) : T(0);
                T zv = vv[r][c] - tau * ((rx_left - rx_here) + (ry_up - ry_here));
                if (nonneg && zv < T(0)) zv = T(0);
                zz[r][c] = in[r][c] ? zv : T(0);
            }
        }
        // p+ = P_P(r + step D z); r+ = p+ + c (p+ - p): needs z of the right neighbour and below
#pragma unroll
        for (int c = 0; c < CX; ++c) xch[1][wave][c][lane] = zz[0][c];
        __syncthreads();
        T z_below[CX];
#pragma unroll
        for (int c = 0; c < CX; ++c) z_below[c] = wave < W - 1 ? xch[1][wave + 1][c][lane] : T(0);
        const T cm = it.cf.c[t];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int gi = i0 + r;
            const T zrl = lane_from_right(zz[r][0]);
#pragma unroll
            for (int c = 0; c < CX; ++c) {
                const T zr = c == CX - 1 ? zrl : zz[r][c < CX - 1 ? c + 1 : 0];
                const T zb = r < RW - 1 ? zz[r < RW - 1 ? r + 1 : 0][c] : z_below[c];
                const T dzx = has_right[c] ? zr - zz[r][c] : T(0);
                const T dzy = (gi < ny - 1) ? zb - zz[r][c] : T(0);
                T ax = fma(step, dzx, rx[r][c]), ay = fma(step, dzy, ry[r][c]);
                const T n2 = fma(ax, ax, ay * ay);
                if (n2 > T(1)) {
                    if constexpr (std::is_same<T, float>::value) {
                        const T sc = __frsqrt_rn(n2);   // 1 / ||(ax, ay)||
                        ax *= sc;
                        ay *= sc;
                    } else {
                        const T nrm = sqrt(n2);
                        ax /= nrm;
                        ay /= nrm;
                    }
                }
                if (in[r][c]) {
                    rx[r][c] = fma(cm, ax - px[r][c], ax);
                    ry[r][c] = fma(cm, ay - py[r][c], ay);
                    px[r][c] = ax;
                    py[r][c] = ay;
                }
            }
        }
    }

    // write back the interior
    bool col_int[CX];
#pragma unroll
    for (int c = 0; c < CX; ++c) col_int[c] = CX * lane + c >= halo && CX * lane + c < halo + TX;
    const size_t nc = it.ncomp;
    if (fin.mode == 0) {
        T *__restrict__ p_out = it.p_out + zoff;
        T *__restrict__ r_out = it.r_out + zoff;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int ey = wave * RW + r;
#pragma unroll
            for (int c = 0; c < CX; ++c) {
                if (!in[r][c] || !col_int[c] || ey < halo || ey >= halo + TY) continue;
                const size_t q = static_cast<size_t>(i0 + r) * nx + gj0 + c;
                p_out[q] = px[r][c];
                p_out[q + nc] = py[r][c];
                r_out[q] = rx[r][c];
                r_out[q + nc] = ry[r][c];
            }
        }
        return;
    }
    // z = P_C(v - tau D^T p_K)
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CX; ++c) xch[0][wave][c][lane] = py[RW - 1][c];
    __syncthreads();
    T py_above[CX];
#pragma unroll
    for (int c = 0; c < CX; ++c) py_above[c] = wave > 0 ? xch[0][wave - 1][c][lane] : T(0);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int gi = i0 + r, ey = wave * RW + r;
        const T pxl_lane = lane_from_left(px[r][CX - 1]);
#pragma unroll
        for (int c = 0; c < CX; ++c) {
            const int gj = gj0 + c;
            const T pxl = c == 0 ? pxl_lane : px[r][c > 0 ? c - 1 : 0];
            if (!in[r][c] || !col_int[c] || ey < halo || ey >= halo + TY) continue;
            const T ph = (gj < nx - 1) ? px[r][c] : T(0);
            const T pl = (gj > 0) ? pxl : T(0);
            const T qh = (gi < ny - 1) ? py[r][c] : T(0);
            const T qu = (gi > 0) ? (r > 0 ? py[r > 0 ? r - 1 : 0][c] : py_above[c]) : T(0);
            T zv = vv[r][c] - tau * ((pl - ph) + (qu - qh));
            if (nonneg && zv < T(0)) zv = T(0);
            const size_t q = zoff + static_cast<size_t>(gi) * nx + gj;
            if (fin.mode == 1) {
                fin.z[q] = zv;
            } else {
                fin.x[q] = zv;
                if (fin.mode == 2) fin.h[q] = fin.hscale * (zv - vv[r][c]);
            }
            fin.dual_out[q] = px[r][c];
            fin.dual_out[q + nc] = py[r][c];
        }
    }
}

// ---- 3D: global-memory half-iterations ------------------------------------------------------

template <typename T>
__device__ inline T mom(const T *pa, const T *pb, size_t q, T c) {
    return fma(c, pa[q] - pb[q], pa[q]);
}

// Projection of one voxel's dual 3-vector onto the unit ball: scaled by 1/||u|| when ||u|| > 1
// (FP32: one correctly rounded reciprocal square root and three products, as the 2D kernel
// does; FP64: the square root and three divisions).
template <typename T>
__device__ inline void unit_ball3(T &ux, T &uy, T &uz) {
    const T n2 = ux * ux + uy * uy + uz * uz;
    if (n2 > T(1)) {
        if constexpr (std::is_same<T, float>::value) {
            const T sc = __frsqrt_rn(n2);
            ux *= sc;
            uy *= sc;
            uz *= sc;
        } else {
            const T nrm = sqrt(n2);
            ux /= nrm;
            uy /= nrm;
            uz /= nrm;
        }
    }
}

// zbuf = P_C(v - tau D^T r), r = pa + c (pa - pb); with c = 0 and pa = p this is z(p).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fgp3d_primal(
    const T *__restrict__ v, const T *__restrict__ pa, const T *__restrict__ pb, T c, int nx,
    int ny, int nz, T tau, int nonneg, T *__restrict__ zbuf, FgpFinal<T> fin) {
    const size_t plane = static_cast<size_t>(nx) * ny, n = plane * nz;
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock) {
        const int j = static_cast<int>(e % nx);
        const int i = static_cast<int>((e / nx) % ny);
        const int zz = static_cast<int>(e / plane);
        const T *pax = pa, *pay = pa + n, *paz = pa + 2 * n;
        const T *pbx = pb, *pby = pb + n, *pbz = pb + 2 * n;
        const T tx = ((j > 0) ? mom(pax, pbx, e - 1, c) : T(0)) - ((j < nx - 1) ? mom(pax, pbx, e, c) : T(0));
        const T ty = ((i > 0) ? mom(pay, pby, e - nx, c) : T(0)) - ((i < ny - 1) ? mom(pay, pby, e, c) : T(0));
        const T tz = ((zz > 0) ? mom(paz, pbz, e - plane, c) : T(0)) - ((zz < nz - 1) ? mom(paz, pbz, e, c) : T(0));
        T zv = v[e] - tau * ((tx + ty) + tz);
        if (nonneg && zv < T(0)) zv = T(0);
        if (fin.mode == 0) {
            zbuf[e] = zv;
        } else {
            if (fin.mode == 1) {
                fin.z[e] = zv;
            } else {
                fin.x[e] = zv;
                if (fin.mode == 2) fin.h[e] = fin.hscale * (zv - v[e]);
            }
            if (fin.dual_out) {
                fin.dual_out[e] = pa[e];
                fin.dual_out[e + n] = pa[e + n];
                fin.dual_out[e + 2 * n] = pa[e + 2 * n];
            }
        }
    }
}

// pn = P_P(r + step D z), r = pa + c (pa - pb).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fgp3d_dual(
    const T *__restrict__ zbuf, const T *__restrict__ pa, const T *__restrict__ pb, T c, int nx,
    int ny, int nz, T step, T *__restrict__ pn) {
    const size_t plane = static_cast<size_t>(nx) * ny, n = plane * nz;
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock) {
        const int j = static_cast<int>(e % nx);
        const int i = static_cast<int>((e / nx) % ny);
        const int zz = static_cast<int>(e / plane);
        const T z0 = zbuf[e];
        const T dx = (j < nx - 1) ? zbuf[e + 1] - z0 : T(0);
        const T dy = (i < ny - 1) ? zbuf[e + nx] - z0 : T(0);
        const T dz = (zz < nz - 1) ? zbuf[e + plane] - z0 : T(0);
        T px = fma(step, dx, mom(pa, pb, e, c));
        T py = fma(step, dy, mom(pa + n, pb + n, e, c));
        T pz = fma(step, dz, mom(pa + 2 * n, pb + 2 * n, e, c));
        unit_ball3(px, py, pz);
        pn[e] = px;
        pn[e + n] = py;
        pn[e + 2 * n] = pz;
    }
}

// One whole 3D FGP iteration per launch:
//     r = pa + c (pa - pb),  z = P_C(v - tau D^T r),  pn = P_unit(r + step D z)
// without storing z.  A workgroup owns a tile of 62 columns x 14 rows (plus a halo of one on
// each side: lane = column, each wave 4 rows) and marches along z over a chunk of slices (the
// plan's fgp3d_chunk, 4 by default: short chunks spread the workgroups' accesses over more
// of the volume at once, which measured faster than the halo re-reads they add),
// keeping the previous slice's r and z in registers: every voxel's 7 inputs are read once and
// its 3 outputs written once (40 B/voxel in FP32, plus the halo's re-reads from L2).
//   z at (x, y, s) needs r_x at x - 1 (DPP from the left lane), r_y at y - 1 (the previous row
//   register, or the wave above through LDS) and r_z at s - 1 (the previous step's register);
//   pn at (x, y, s - 1) needs z at x + 1 (DPP from the right lane), y + 1 and s, so the output
//   of a step is the slice before the one it computes z for.  Forward differences are zero at
//   the last index and the divergence's missing neighbours are zero, as in the 2D kernel.
constexpr int kF3Rows = 4;                    // rows per wave
constexpr int kF3TX = 62, kF3TY = 4 * kF3Rows - 2;   // output columns and rows per tile
constexpr int kF3Chunk = 4;                   // output slices per workgroup (default)

template <typename T>
struct Fgp3Args {
    const T *v, *pa, *pb;
    T *pn;
    int nx, ny, nz, tiles_x, tiles_y, chunk;
    T c, tau, step;
    int nonneg;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fgp3d_iter(Fgp3Args<T> a) {
    __shared__ T xch[2][kFgpWaves][kFgpEX];
    const int lane = threadIdx.x % kFgpEX;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kFgpEX));
    const int b = blockIdx.x;
    const int tx = b % a.tiles_x, ty = (b / a.tiles_x) % a.tiles_y, zc = b / (a.tiles_x * a.tiles_y);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t plane = static_cast<size_t>(nx) * ny, n = plane * nz;
    const int gx = tx * kF3TX - 1 + lane;                 // lane 0 and 63: halo columns
    const int gy0 = ty * kF3TY - 1 + wave * kF3Rows;      // row of this wave's first register row
    const bool col_in = gx >= 0 && gx < nx;
    const int s_lo = zc * a.chunk, s_hi = min(nz, s_lo + a.chunk);
    const T c = a.c, tau = a.tau, step = a.step;

    T rx[kF3Rows], ry[kF3Rows], rz[kF3Rows], rzp[kF3Rows], zz[kF3Rows];
    T prx[kF3Rows], pry[kF3Rows], prz[kF3Rows], pz[kF3Rows];   // slice s - 1
    bool in[kF3Rows];
#pragma unroll
    for (int r = 0; r < kF3Rows; ++r) {
        const int gy = gy0 + r;
        in[r] = col_in && gy >= 0 && gy < ny;
        rzp[r] = T(0);
        prx[r] = pry[r] = prz[r] = pz[r] = T(0);
    }
    // r_z at slice s_lo - 1 (the only component of that slice that z(s_lo) needs)
    if (s_lo > 0) {
#pragma unroll
        for (int r = 0; r < kF3Rows; ++r) {
            if (!in[r]) continue;
            const size_t e = static_cast<size_t>(s_lo - 1) * plane + static_cast<size_t>(gy0 + r) * nx + gx;
            const T pa_ = a.pa[e + 2 * n], pb_ = a.pb[e + 2 * n];
            rzp[r] = fma(c, pa_ - pb_, pa_);
        }
    }
    const T *__restrict__ pa = a.pa;
    const T *__restrict__ pb = a.pb;
    const T *__restrict__ vp = a.v;
    T *__restrict__ pn = a.pn;
    // inputs of one slice, loaded one step ahead of their use
    T lax[kF3Rows], lbx[kF3Rows], lay[kF3Rows], lby[kF3Rows], laz[kF3Rows], lbz[kF3Rows], lv[kF3Rows];
    auto load_slice = [&](int s) {
#pragma unroll
        for (int r = 0; r < kF3Rows; ++r) {
            lax[r] = lbx[r] = lay[r] = lby[r] = laz[r] = lbz[r] = lv[r] = T(0);
            if (in[r] && s < nz) {
                const size_t e = static_cast<size_t>(s) * plane + static_cast<size_t>(gy0 + r) * nx + gx;
                lax[r] = pa[e];
                lbx[r] = pb[e];
                lay[r] = pa[e + n];
                lby[r] = pb[e + n];
                laz[r] = pa[e + 2 * n];
                lbz[r] = pb[e + 2 * n];
                lv[r] = vp[e];
            }
        }
    };
    load_slice(s_lo);
    // steps s = s_lo .. s_hi (the last computes z only, for the output slice s_hi - 1)
    for (int s = s_lo; s <= s_hi; ++s) {
        const bool have = s < nz;
        // r and v at slice s, then the next slice's loads go out
        T vv[kF3Rows];
#pragma unroll
        for (int r = 0; r < kF3Rows; ++r) {
            rx[r] = fma(c, lax[r] - lbx[r], lax[r]);
            ry[r] = fma(c, lay[r] - lby[r], lay[r]);
            rz[r] = fma(c, laz[r] - lbz[r], laz[r]);
            vv[r] = lv[r];
        }
        if (s < s_hi) load_slice(s + 1);
        // z at slice s: needs r_y of the row above (previous wave's last row)
        __syncthreads();
        xch[0][wave][lane] = ry[kF3Rows - 1];
        __syncthreads();
        const T ry_above = wave > 0 ? xch[0][wave - 1][lane] : T(0);
#pragma unroll
        for (int r = 0; r < kF3Rows; ++r) {
            // D^T r: the last index's dual component has no difference to pair with
            const int gy = gy0 + r;
            const T rxl = lane_from_left(rx[r]);
            const T ryu = r > 0 ? ry[r - 1] : ry_above;
            const T rxh = gx < nx - 1 ? rx[r] : T(0);
            const T ryh = gy < ny - 1 ? ry[r] : T(0);
            const T rzh = s < nz - 1 ? rz[r] : T(0);
            T zv = vv[r] - tau * (((rxl - rxh) + (ryu - ryh)) + (rzp[r] - rzh));
            if (a.nonneg && zv < T(0)) zv = T(0);
            zz[r] = (in[r] && have) ? zv : T(0);
        }
        // pn at slice s - 1: needs z at x + 1, y + 1 (next wave's first row) and s
        if (s > s_lo) {
            xch[1][wave][lane] = pz[0];
            __syncthreads();
            const T z_below = wave < kFgpWaves - 1 ? xch[1][wave + 1][lane] : T(0);
#pragma unroll
            for (int r = 0; r < kF3Rows; ++r) {
                const int gy = gy0 + r;
                const T zr = lane_from_right(pz[r]);
                const T zb = r < kF3Rows - 1 ? pz[r + 1] : z_below;
                const T dzx = gx < nx - 1 ? zr - pz[r] : T(0);
                const T dzy = gy < ny - 1 ? zb - pz[r] : T(0);
                const T dzz = s - 1 < nz - 1 ? zz[r] - pz[r] : T(0);
                T ux = fma(step, dzx, prx[r]), uy = fma(step, dzy, pry[r]), uz = fma(step, dzz, prz[r]);
                unit_ball3(ux, uy, uz);
                const bool out = in[r] && lane >= 1 && lane <= kF3TX && gy >= ty * kF3TY &&
                                 gy < ty * kF3TY + kF3TY;
                if (out) {
                    const size_t e = static_cast<size_t>(s - 1) * plane + static_cast<size_t>(gy) * nx + gx;
                    pn[e] = ux;
                    pn[e + n] = uy;
                    pn[e + 2 * n] = uz;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kF3Rows; ++r) {
            prx[r] = rx[r];
            pry[r] = ry[r];
            prz[r] = rz[r];
            pz[r] = zz[r];
            rzp[r] = rz[r];
        }
    }
}

// Two whole 3D FGP iterations per launch.  From (pa, pb) = (p_{k-1}, p_{k-2}):
//     r_k   = pa + c1 (pa - pb),    z_k   = P_C(v - tau D^T r_k),    p_k   = P_unit(r_k + step D z_k)
//     r_k+1 = p_k + c2 (p_k - pa),  z_k+1 = P_C(v - tau D^T r_k+1),  p_k+1 = P_unit(r_k+1 + step D z_k+1)
// writing p_k (pn1) and p_{k+1} (pn2): per voxel 7 values read and 6 written for two iterations
// instead of 7 read and 3 written for each.  Every value is formed by the one-iteration kernel's
// expressions, so a launch gives the bits of two one-iteration launches.
// Tile: 64 lanes = columns and W waves of RW rows, with two halo columns and rows on each side
// (60 x (W RW - 4) outputs): each iteration's D^T reaches one voxel back and its D one forward.
// Marching up z, step s holds the loads of slice s and computes
//     A  r_k(s)      B  z_k(s)      C  p_k(s-1)      D  r_k+1(s-1)      E  z_k+1(s-1)      F  p_k+1(s-2)
// keeping slice s-1's r_k, z_k, pa, v and slice s-2's r_k+1, z_k+1 in registers; p_k(s-1) and
// p_k+1(s-2) are written when they fall in the workgroup's chunk of slices [s_lo, s_hi).  The
// steps run from s_lo - 1 to s_hi + 1 (r_k's z component at s_lo - 2 is loaded up front): values
// at slices outside the chunk are halo and are never written.  Voxels outside the volume hold
// zeros in every quantity, as the zero loads of the one-iteration kernel give it.
constexpr int kF32X = kFgpEX - 4;   // output columns per tile
// launch forms: 1 = one iteration per launch; 2..5 = two per launch on tiles of (waves x rows
// per wave) 8 x 2, 4 x 4, 16 x 2, 8 x 4
constexpr int kF32Waves[kF3Forms + 1] = {0, 0, 8, 4, 16, 8};
constexpr int kF32Rows[kF3Forms + 1] = {0, 0, 2, 4, 2, 4};

template <typename T>
struct Fgp3Args2 {
    const T *v, *pa, *pb;
    T *pn1, *pn2;
    int nx, ny, nz, tiles_x, tiles_y, chunk;
    T c1, c2, tau, step;
    int nonneg;
};

template <typename T, int W, int RW>
__global__ __launch_bounds__(W * kFgpEX) void k_fgp3d_iter2(Fgp3Args2<T> a) {
    constexpr int kTY = W * RW - 4;   // output rows per tile
    // two exchange slots per phase, alternating between the two phases of a step
    __shared__ T xch[2][3][W][kFgpEX];
    const int lane = threadIdx.x % kFgpEX;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kFgpEX));
    const int b = blockIdx.x;
    const int tx = b % a.tiles_x, ty = (b / a.tiles_x) % a.tiles_y, zc = b / (a.tiles_x * a.tiles_y);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t plane = static_cast<size_t>(nx) * ny, n = plane * nz;
    const int gx = tx * kF32X - 2 + lane;                // lanes 0, 1, 62, 63: halo columns
    const int gy0 = ty * kTY - 2 + wave * RW;            // row of this wave's first register row
    const bool col_in = gx >= 0 && gx < nx;
    const bool lane_out = lane >= 2 && lane < 2 + kF32X;
    const int s_lo = zc * a.chunk, s_hi = min(nz, s_lo + a.chunk);
    const T c1 = a.c1, c2 = a.c2, tau = a.tau, step = a.step;
    const T *__restrict__ pa = a.pa;
    const T *__restrict__ pb = a.pb;
    const T *__restrict__ vp = a.v;
    T *__restrict__ pn1 = a.pn1;
    T *__restrict__ pn2 = a.pn2;

    bool in[RW], row_out[RW];
    // slice s-1: r_k (3), z_k, pa (3), v;  slice s-2: r_k+1 (3), z_k+1
    T rkx[RW], rky[RW], rkz[RW], zk[RW], pax[RW], pay[RW], paz[RW], vv1[RW];
    T r1x[RW], r1y[RW], r1z[RW], z1[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int gy = gy0 + r;
        in[r] = col_in && gy >= 0 && gy < ny;
        row_out[r] = gy >= ty * kTY && gy < ty * kTY + kTY;
        rkx[r] = rky[r] = rkz[r] = zk[r] = pax[r] = pay[r] = paz[r] = vv1[r] = T(0);
        r1x[r] = r1y[r] = r1z[r] = z1[r] = T(0);
    }
    // r_k's z component at slice s_lo - 2 (all that z_k(s_lo - 1) needs of that slice)
    if (s_lo >= 2) {
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            if (!in[r]) continue;
            const size_t e = static_cast<size_t>(s_lo - 2) * plane + static_cast<size_t>(gy0 + r) * nx + gx;
            const T pa_ = pa[e + 2 * n], pb_ = pb[e + 2 * n];
            rkz[r] = fma(c1, pa_ - pb_, pa_);
        }
    }
    // inputs of one slice, loaded one step ahead of their use
    T lax[RW], lbx[RW], lay[RW], lby[RW], laz[RW], lbz[RW], lv[RW];
    auto load_slice = [&](int s) {
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            lax[r] = lbx[r] = lay[r] = lby[r] = laz[r] = lbz[r] = lv[r] = T(0);
            if (in[r] && s >= 0 && s < nz) {
                const size_t e = static_cast<size_t>(s) * plane + static_cast<size_t>(gy0 + r) * nx + gx;
                lax[r] = pa[e];
                lbx[r] = pb[e];
                lay[r] = pa[e + n];
                lby[r] = pb[e + n];
                laz[r] = pa[e + 2 * n];
                lbz[r] = pb[e + 2 * n];
                lv[r] = vp[e];
            }
        }
    };
    // unit-ball projection of the dual step at one voxel
    auto dual_step = [&](T ux, T uy, T uz, T &ox, T &oy, T &oz) {
        unit_ball3(ux, uy, uz);
        ox = ux;
        oy = uy;
        oz = uz;
    };
    load_slice(s_lo - 1);
    for (int s = s_lo - 1; s <= s_hi + 1; ++s) {
        const bool have0 = s >= 0 && s < nz;            // slice s
        const bool have1 = s - 1 >= 0 && s - 1 < nz;    // slice s - 1
        // A: r_k and v at slice s, then the next slice's loads go out
        T ax[RW], ay[RW], az[RW], av[RW], sax[RW], say[RW], saz[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            ax[r] = fma(c1, lax[r] - lbx[r], lax[r]);
            ay[r] = fma(c1, lay[r] - lby[r], lay[r]);
            az[r] = fma(c1, laz[r] - lbz[r], laz[r]);
            av[r] = lv[r];
            sax[r] = lax[r];
            say[r] = lay[r];
            saz[r] = laz[r];
        }
        if (s <= s_hi) load_slice(s + 1);
        // exchange 1: r_k,y(s) of the last row down, z_k(s-1) and z_k+1(s-2) of the first row up
        const int ph = 0;
        xch[ph][0][wave][lane] = ay[RW - 1];
        xch[ph][1][wave][lane] = zk[0];
        xch[ph][2][wave][lane] = z1[0];
        __syncthreads();
        const T ry_above = wave > 0 ? xch[ph][0][wave - 1][lane] : T(0);
        const T zk_below = wave < W - 1 ? xch[ph][1][wave + 1][lane] : T(0);
        const T z1_below = wave < W - 1 ? xch[ph][2][wave + 1][lane] : T(0);
        // B: z_k at slice s
        T zn[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int gy = gy0 + r;
            const T rxl = lane_from_left(ax[r]);
            const T ryu = r > 0 ? ay[r - 1] : ry_above;
            const T rxh = gx < nx - 1 ? ax[r] : T(0);
            const T ryh = gy < ny - 1 ? ay[r] : T(0);
            const T rzh = s < nz - 1 ? az[r] : T(0);
            T zv = av[r] - tau * (((rxl - rxh) + (ryu - ryh)) + (rkz[r] - rzh));
            if (a.nonneg && zv < T(0)) zv = T(0);
            zn[r] = (in[r] && have0) ? zv : T(0);
        }
        // C, D: p_k and r_k+1 at slice s - 1
        T qx[RW], qy[RW], qz[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int gy = gy0 + r;
            const T zr = lane_from_right(zk[r]);
            const T zb = r < RW - 1 ? zk[r + 1] : zk_below;
            const T dzx = gx < nx - 1 ? zr - zk[r] : T(0);
            const T dzy = gy < ny - 1 ? zb - zk[r] : T(0);
            const T dzz = s - 1 < nz - 1 ? zn[r] - zk[r] : T(0);
            T px, py, pz;
            dual_step(fma(step, dzx, rkx[r]), fma(step, dzy, rky[r]), fma(step, dzz, rkz[r]), px, py, pz);
            const bool live = in[r] && have1;
            px = live ? px : T(0);
            py = live ? py : T(0);
            pz = live ? pz : T(0);
            if (live && lane_out && row_out[r] && s - 1 >= s_lo && s - 1 < s_hi) {
                const size_t e = static_cast<size_t>(s - 1) * plane + static_cast<size_t>(gy) * nx + gx;
                pn1[e] = px;
                pn1[e + n] = py;
                pn1[e + 2 * n] = pz;
            }
            qx[r] = fma(c2, px - pax[r], px);
            qy[r] = fma(c2, py - pay[r], py);
            qz[r] = fma(c2, pz - paz[r], pz);
        }
        // exchange 2: r_k+1,y(s-1) of the last row down
        xch[1][0][wave][lane] = qy[RW - 1];
        __syncthreads();
        const T qy_above = wave > 0 ? xch[1][0][wave - 1][lane] : T(0);
        // E: z_k+1 at slice s - 1
        T z1n[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int gy = gy0 + r;
            const T rxl = lane_from_left(qx[r]);
            const T ryu = r > 0 ? qy[r - 1] : qy_above;
            const T rxh = gx < nx - 1 ? qx[r] : T(0);
            const T ryh = gy < ny - 1 ? qy[r] : T(0);
            const T rzh = s - 1 < nz - 1 ? qz[r] : T(0);
            T zv = vv1[r] - tau * (((rxl - rxh) + (ryu - ryh)) + (r1z[r] - rzh));
            if (a.nonneg && zv < T(0)) zv = T(0);
            z1n[r] = (in[r] && have1) ? zv : T(0);
        }
        // F: p_k+1 at slice s - 2
        if (s - 2 >= s_lo && s - 2 < s_hi) {
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int gy = gy0 + r;
                const T zr = lane_from_right(z1[r]);
                const T zb = r < RW - 1 ? z1[r + 1] : z1_below;
                const T dzx = gx < nx - 1 ? zr - z1[r] : T(0);
                const T dzy = gy < ny - 1 ? zb - z1[r] : T(0);
                const T dzz = s - 2 < nz - 1 ? z1n[r] - z1[r] : T(0);
                T px, py, pz;
                dual_step(fma(step, dzx, r1x[r]), fma(step, dzy, r1y[r]), fma(step, dzz, r1z[r]), px, py, pz);
                if (in[r] && lane_out && row_out[r]) {
                    const size_t e = static_cast<size_t>(s - 2) * plane + static_cast<size_t>(gy) * nx + gx;
                    pn2[e] = px;
                    pn2[e + n] = py;
                    pn2[e + 2 * n] = pz;
                }
            }
        }
        // shift: slice s becomes s - 1, slice s - 1 becomes s - 2
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            r1x[r] = qx[r];
            r1y[r] = qy[r];
            r1z[r] = qz[r];
            z1[r] = z1n[r];
            rkx[r] = ax[r];
            rky[r] = ay[r];
            rkz[r] = az[r];
            zk[r] = zn[r];
            pax[r] = sax[r];
            pay[r] = say[r];
            paz[r] = saz[r];
            vv1[r] = av[r];
        }
    }
}

// tau = 0: z = P_C(v) (and the ProxSkip outputs).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prox_identity(const T *__restrict__ v, size_t n, int nonneg,
                                                          FgpFinal<T> fin) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock) {
        const T vv = v[e];
        const T zv = (nonneg && vv < T(0)) ? T(0) : vv;
        if (fin.mode == 1) {
            fin.z[e] = zv;
        } else {
            fin.x[e] = zv;
            if (fin.mode == 2) fin.h[e] = fin.hscale * (zv - vv);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *__restrict__ p, size_t n, T val) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock)
        p[e] = val;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(T *__restrict__ dst, const T *__restrict__ src, size_t n) {
    for (size_t e = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * kBlock)
        dst[e] = src[e];
}

static unsigned grid_for(size_t n) {
    return static_cast<unsigned>(std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, 8192)));
}

// FISTA momentum coefficients c_k (k = 1..K): c_1 = c_2 = 0, c_k = (t_{k-1} - 1)/t_k.
static std::vector<double> momentum(int K) {
    std::vector<double> c(K + 1, 0.0), t(K + 1, 1.0);
    for (int k = 2; k <= K; ++k) {
        t[k] = (1.0 + std::sqrt(1.0 + 4.0 * t[k - 1] * t[k - 1])) / 2.0;
        c[k] = (t[k - 1] - 1.0) / t[k];
    }
    return c;
}

size_t fgp_workspace(const ps_geometry *g) {
    const size_t n = static_cast<size_t>(g->desc.nx) * g->desc.ny * g->desc.nz;
    const size_t dn = static_cast<size_t>(g->tv_dims) * n;
    return align_up(dn * g->elem) * 4 + align_up(n * g->elem) * 2;
}

// Inner iterations per 2D launch.  A launch recomputes a halo of T + 1 pixels around every tile,
// so fewer iterations per launch waste less arithmetic but pay the per-launch cost (loading and
// storing the tile state) more often.  8 per launch is the best depth for the automatic tiles;
// taller tiles go deeper (at 512^2 a 16 x 4 tile at 10 or 12 per launch beats every tile at 8 by
// 14%), which tuned plans choose.  Neither choice changes results.
// A tile of height EY leaves EY - 2 (T + 1) interior rows, so T is capped at EY / 2 - 2.
int fgp3d_form_of(const ps_geometry *g) {
    const int f = g->plan.fgp3d_form;
    if (f >= 1 && f <= kF3Forms) return f;
    return g->desc.dtype == PS_F64 ? 2 : 5;
}

// Slices per 3D workgroup: 4 for one iteration per launch (short chunks spread the accesses
// over more of the volume), 16 for two (their z halo of three slices is paid once per chunk).
int fgp3d_chunk_of(const ps_geometry *g) {
    if (g->plan.fgp3d_chunk > 0) return g->plan.fgp3d_chunk;
    return fgp3d_form_of(g) == 1 ? kF3Chunk : 16;
}

int fgp_max_iters_of(const ps_geometry *g) {
    return g->elem == sizeof(double) ? fgp_max_iters<double>() : fgp_max_iters<float>();
}
int fgp_cols_of(const ps_geometry *g) {
    const int c = g->plan.fgp_cols;
    return c == 1 || c == 2 ? c : kFgpAutoCols;
}
static void fgp_auto_tile(const ps_geometry *g, int *waves, int *rows) {
    // 8 x 4 (FP32), 16 x 2 (FP64): at or near the fastest from 256^2 to 512^2 alone, and the
    // best throughput measured for batches (64 x 128^2)
    *waves = g->elem == sizeof(double) ? 16 : 8;
    *rows = g->elem == sizeof(double) ? 2 : 4;
}
void fgp_tile_of(const ps_geometry *g, int *waves, int *rows) {
    if (g->plan.fgp_waves > 0) {
        *waves = g->plan.fgp_waves;
        *rows = g->plan.fgp_rows;
    } else {
        fgp_auto_tile(g, waves, rows);
    }
}
static int fgp_cap(int waves, int rows) { return waves * rows / 2 - 2; }
int fgp_iters_per_launch(const ps_geometry *g) {
    int waves, rows;
    fgp_tile_of(g, &waves, &rows);
    const int f = g->plan.fgp_iters;
    return std::min(f > 0 ? std::min(f, fgp_max_iters_of(g)) : kFgpAutoIters, fgp_cap(waves, rows));
}

// A 2D FGP solve as its sequence of launches, plus the copies around them.
template <typename T>
struct FgpProgram {
    std::vector<FgpItem<T>> launches;
    const T *pre_copy_src = nullptr;  // z aliases v: v is copied first
    T *pre_copy_dst = nullptr;
    T *pre_fill = nullptr;            // cold start: zero dual
    size_t n = 0, dn = 0;
    T *post_copy_dst = nullptr;       // final dual written to a work buffer, copied back
    const T *post_copy_src = nullptr;
    FgpTile tile{};
};

// `shared`: the solve shares its launches with other 2D solves.  The plan's tile and depth are
// tuned on one solve alone; with many workgroups in flight the automatic tile and depth
// has the better throughput (64 x 128^2: 19.8k slice-epochs/s against 16.3k with the tile tuned
// alone), so shared solves use it.  The tile never changes the bits.
template <typename T>
static ps_status fgp2d_program(const FgpCall &c, bool shared, FgpProgram<T> &prog) {
    const ps_geometry *g = c.g;
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    const size_t dn = 2 * n;
    const int K = c.n_inner;
    prog.n = n;
    prog.dn = dn;
    FgpFinal<T> fin{};
    fin.mode = c.out.proxskip == 0 ? 1 : (c.out.proxskip == 1 ? 2 : 3);
    fin.z = static_cast<T *>(c.out.z);
    fin.x = static_cast<T *>(c.out.x);
    fin.h = static_cast<T *>(c.out.h);
    fin.hscale = static_cast<T>(c.out.hscale);
    unsigned char *w = static_cast<unsigned char *>(c.ws);
    const size_t sd = align_up(dn * g->elem);
    T *buf[4] = {reinterpret_cast<T *>(w), reinterpret_cast<T *>(w + sd),
                 reinterpret_cast<T *>(w + 2 * sd), reinterpret_cast<T *>(w + 3 * sd)};
    T *vcopy = reinterpret_cast<T *>(w + 4 * sd);
    const T *v = static_cast<const T *>(c.v);
    T *dual = static_cast<T *>(c.dual);

    // z may alias v: the halo reads of v must not see finished pixels of another workgroup
    const T *vin = v;
    if (fin.mode == 1 && static_cast<const void *>(fin.z) == static_cast<const void *>(v)) {
        prog.pre_copy_src = v;
        prog.pre_copy_dst = vcopy;
        vin = vcopy;
    }
    // cold start: zero dual in the workspace, final dual discarded
    const T *dual_in = dual;
    if (!dual) {
        prog.pre_fill = buf[3];
        dual_in = buf[3];
    }
    const T tauT = static_cast<T>(c.tau);
    const T stepT = static_cast<T>(1.0 / (8.0 * c.tau));
    int tmax;
    if (shared) {
        fgp_auto_tile(g, &prog.tile.waves, &prog.tile.rows);
        prog.tile.cols = kFgpAutoCols;
        tmax = std::min(kFgpAutoIters, fgp_cap(prog.tile.waves, prog.tile.rows));
    } else {
        fgp_tile_of(g, &prog.tile.waves, &prog.tile.rows);
        prog.tile.cols = fgp_cols_of(g);
        tmax = fgp_iters_per_launch(g);
    }
    const int EY = prog.tile.waves * prog.tile.rows;
    const int launches = std::max(1, (K + tmax - 1) / tmax);
    const std::vector<double> cn = momentum(K + 1);
    int done = 0;
    const T *in_p = dual_in, *in_r = dual_in;  // r_1 = p_0
    for (int L = 0; L < launches; ++L) {
        const int iters = std::min(tmax, K - done);
        const int halo = iters + 1;
        const int TX = kFgpEX * prog.tile.cols - 2 * halo, TY = EY - 2 * halo;
        FgpItem<T> it{};
        it.v = vin;
        it.p_in = in_p;
        it.r_in = in_r;
        it.ncomp = n;
        it.nx = d.nx;
        it.ny = d.ny;
        it.iters = iters;
        it.halo = halo;
        it.tiles_x = (d.nx + TX - 1) / TX;
        it.tiles_y = (d.ny + TY - 1) / TY;
        it.nonneg = c.nonneg;
        it.tau = tauT;
        it.step = stepT;
        for (int t = 0; t < iters; ++t) it.cf.c[t] = static_cast<T>(cn[done + t + 2]);
        it.fin = fin;
        const bool last = (L == launches - 1);
        T *out_p = buf[2 * (L % 2)], *out_r = buf[2 * (L % 2) + 1];
        it.p_out = out_p;
        it.r_out = out_r;
        if (last) {
            // the final dual must not land in a buffer this launch still reads as halo
            if (!dual) {
                it.fin.dual_out = out_p;  // cold start: dual discarded
            } else if (L == 0) {
                it.fin.dual_out = out_p;  // single launch reading the caller's dual: copy after
                prog.post_copy_dst = dual;
                prog.post_copy_src = out_p;
            } else {
                it.fin.dual_out = dual;
            }
        } else {
            it.fin.mode = 0;
        }
        prog.launches.push_back(it);
        in_p = out_p;
        in_r = out_r;
        done += iters;
    }
    return PS_OK;
}

template <typename T, int W, int RW>
static void launch_fgp2d_tile(const WorkList<FgpItem<T>> &wl, int blocks, int cols, hipStream_t st) {
    timer_mark(KC_FGP2D, st, true);
    if (cols == 2)
        hipLaunchKernelGGL((k_fgp2d<T, W, RW, 2>), dim3(blocks), dim3(W * kFgpEX), 0, st, wl);
    else
        hipLaunchKernelGGL((k_fgp2d<T, W, RW, 1>), dim3(blocks), dim3(W * kFgpEX), 0, st, wl);
    timer_mark(KC_FGP2D, st, false);
}

static_assert(sizeof(WorkList<FgpItem<float>>) <= 4096 && sizeof(WorkList<FgpItem<double>>) <= 4096,
              "2D FGP work lists must fit in 4 KB of kernel arguments");

template <typename T>
static ps_status launch_fgp2d_list(const WorkList<FgpItem<T>> &wl, int blocks, FgpTile tile, hipStream_t st) {
    switch (tile.waves * 100 + tile.rows) {
    case 404: launch_fgp2d_tile<T, 4, 4>(wl, blocks, tile.cols, st); break;
    case 408: launch_fgp2d_tile<T, 4, 8>(wl, blocks, tile.cols, st); break;
    case 802: launch_fgp2d_tile<T, 8, 2>(wl, blocks, tile.cols, st); break;
    case 804: launch_fgp2d_tile<T, 8, 4>(wl, blocks, tile.cols, st); break;
    case 808: launch_fgp2d_tile<T, 8, 8>(wl, blocks, tile.cols, st); break;
    case 1602: launch_fgp2d_tile<T, 16, 2>(wl, blocks, tile.cols, st); break;
    case 1604: launch_fgp2d_tile<T, 16, 4>(wl, blocks, tile.cols, st); break;
    default: return fail(PS_EINVAL, "FGP tile %d x %d not built", tile.waves, tile.rows);
    }
    PS_LAUNCHED("k_fgp2d");
    return PS_OK;
}

// 3D (coupled slices) and tau = 0 solves run on their own.
template <typename T>
static ps_status fgp_single_t(const FgpCall &c, hipStream_t st) {
    const ps_geometry *g = c.g;
    const auto &d = g->desc;
    const size_t n = static_cast<size_t>(d.nx) * d.ny * d.nz;
    const int dims = g->tv_dims;
    const size_t dn = static_cast<size_t>(dims) * n;
    const int K = c.n_inner;
    FgpFinal<T> fin{};
    fin.mode = c.out.proxskip == 0 ? 1 : (c.out.proxskip == 1 ? 2 : 3);
    fin.z = static_cast<T *>(c.out.z);
    fin.x = static_cast<T *>(c.out.x);
    fin.h = static_cast<T *>(c.out.h);
    fin.hscale = static_cast<T>(c.out.hscale);
    const T *v = static_cast<const T *>(c.v);
    T *dual = static_cast<T *>(c.dual);
    if (c.tau == 0.0) {
        hipLaunchKernelGGL((k_prox_identity<T>), dim3(grid_for(n)), dim3(kBlock), 0, st, v, n, c.nonneg, fin);
        PS_LAUNCHED("k_prox_identity");
        return PS_OK;
    }
    unsigned char *w = static_cast<unsigned char *>(c.ws);
    const size_t sd = align_up(dn * g->elem), sn = align_up(n * g->elem);
    T *buf[4] = {reinterpret_cast<T *>(w), reinterpret_cast<T *>(w + sd),
                 reinterpret_cast<T *>(w + 2 * sd), reinterpret_cast<T *>(w + 3 * sd)};
    T *vcopy = reinterpret_cast<T *>(w + 4 * sd);
    T *zscratch = reinterpret_cast<T *>(w + 4 * sd + sn);
    const T *vin = v;
    if (fin.mode == 1 && static_cast<const void *>(fin.z) == static_cast<const void *>(v)) {
        hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(n)), dim3(kBlock), 0, st, vcopy, v, n);
        PS_LAUNCHED("k_copy");
        vin = vcopy;
    }
    const T *dual_in = dual;
    if (!dual) {
        hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(dn)), dim3(kBlock), 0, st, buf[3], dn, T(0));
        PS_LAUNCHED("k_fill");
        dual_in = buf[3];
    }
    const std::vector<double> cs = momentum(std::max(K, 1));
    const T tauT = static_cast<T>(c.tau);
    const T stepT = static_cast<T>(1.0 / (4.0 * dims * c.tau));
    const unsigned gr = grid_for(n);
    const T *pb = dual_in, *pa = dual_in;
    Fgp3Args<T> fa{};
    fa.v = vin;
    fa.nx = d.nx;
    fa.ny = d.ny;
    fa.nz = d.nz;
    fa.tiles_x = (d.nx + kF3TX - 1) / kF3TX;
    fa.tiles_y = (d.ny + kF3TY - 1) / kF3TY;
    fa.tau = tauT;
    fa.step = stepT;
    fa.nonneg = c.nonneg;
    fa.chunk = fgp3d_chunk_of(g);
    const long f3_blocks = static_cast<long>(fa.tiles_x) * fa.tiles_y * ((d.nz + fa.chunk - 1) / fa.chunk);
    if (f3_blocks > (1L << 30)) return fail(PS_EUNSUPPORTED, "3D TV grid too large");
    // launch form: 1 = one iteration per launch; 2, 3 = two per launch on 8 x 2 or 4 x 4 tiles
    const int form = fgp3d_form_of(g);
    Fgp3Args2<T> fb{};
    fb.v = vin;
    fb.nx = d.nx;
    fb.ny = d.ny;
    fb.nz = d.nz;
    fb.tau = tauT;
    fb.step = stepT;
    fb.nonneg = c.nonneg;
    fb.chunk = fa.chunk;
    const int ty2 = kF32Waves[form] * kF32Rows[form] - 4;
    fb.tiles_x = (d.nx + kF32X - 1) / kF32X;
    fb.tiles_y = (d.ny + ty2 - 1) / ty2;
    const long f32_blocks = static_cast<long>(fb.tiles_x) * fb.tiles_y * ((d.nz + fb.chunk - 1) / fb.chunk);
    if (f32_blocks > (1L << 30)) return fail(PS_EUNSUPPORTED, "3D TV grid too large");
    // dual buffers: any of the four workspace buffers that the launch does not read; the last
    // launch writes the caller's dual directly when it does not read it
    T *pool[4] = {buf[0], buf[1], buf[2], buf[3]};
    auto pick = [&](const T *x1, const T *x2, const T *x3) -> T * {
        for (T *q : pool)
            if (q != x1 && q != x2 && q != x3) return q;
        return nullptr;
    };
    for (int k = 1; k <= K;) {
        const bool last = [&] { return form == 1 ? k == K : k + 1 >= K; }();
        const bool direct = last && dual && dual != pa && dual != pb;
        if (form != 1 && k + 1 <= K) {
            T *p1 = pick(pa, pb, nullptr);
            T *p2 = direct ? dual : pick(pa, pb, p1);
            fb.pa = pa;
            fb.pb = pb;
            fb.pn1 = p1;
            fb.pn2 = p2;
            fb.c1 = static_cast<T>(cs[k]);
            fb.c2 = static_cast<T>(cs[k + 1]);
            timer_mark(KC_FGP3D, st, true);
            const dim3 grid(static_cast<unsigned>(f32_blocks));
            switch (form) {
            case 2: hipLaunchKernelGGL((k_fgp3d_iter2<T, 8, 2>), grid, dim3(8 * kFgpEX), 0, st, fb); break;
            case 3: hipLaunchKernelGGL((k_fgp3d_iter2<T, 4, 4>), grid, dim3(4 * kFgpEX), 0, st, fb); break;
            case 4: hipLaunchKernelGGL((k_fgp3d_iter2<T, 16, 2>), grid, dim3(16 * kFgpEX), 0, st, fb); break;
            default: hipLaunchKernelGGL((k_fgp3d_iter2<T, 8, 4>), grid, dim3(8 * kFgpEX), 0, st, fb); break;
            }
            PS_LAUNCHED("k_fgp3d_iter2");
            timer_mark(KC_FGP3D, st, false);
            pb = p1;
            pa = p2;
            k += 2;
        } else {
            T *pn = direct ? dual : pick(pa, pb, nullptr);
            fa.pa = pa;
            fa.pb = pb;
            fa.pn = pn;
            fa.c = static_cast<T>(cs[k]);
            timer_mark(KC_FGP3D, st, true);
            hipLaunchKernelGGL((k_fgp3d_iter<T>), dim3(static_cast<unsigned>(f3_blocks)), dim3(kBlock), 0, st, fa);
            PS_LAUNCHED("k_fgp3d_iter");
            timer_mark(KC_FGP3D, st, false);
            pb = pa;
            pa = pn;
            k += 1;
        }
    }
    // z = P_C(v - tau D^T p_K); the final dual p_K sits in `pa`
    FgpFinal<T> f = fin;
    f.dual_out = nullptr;
    hipLaunchKernelGGL((k_fgp3d_primal<T>), dim3(gr), dim3(kBlock), 0, st, vin, pa, pa, T(0), d.nx,
                       d.ny, d.nz, tauT, c.nonneg, zscratch, f);
    PS_LAUNCHED("k_fgp3d_primal(final)");
    if (dual && K > 0 && pa != dual) {
        hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(dn)), dim3(kBlock), 0, st, dual, pa, dn);
        PS_LAUNCHED("k_copy");
    }
    return PS_OK;
}

// All calls of one dtype.  2D solves advance together: launch round r holds the r-th launch of
// every solve that has one.
template <typename T>
static ps_status fgp_many_t(const FgpCall *calls, int n, hipStream_t st) {
    std::vector<FgpProgram<T>> progs;
    int n2d = 0;
    for (int i = 0; i < n; ++i) n2d += calls[i].g->tv_dims == 2 && calls[i].tau != 0.0;
    for (int i = 0; i < n; ++i) {
        const FgpCall &c = calls[i];
        const size_t need = fgp_workspace(c.g);
        if (c.tau != 0.0 && (!c.ws || c.ws_bytes < need))
            return fail(PS_EINVAL, "TV prox workspace: %zu bytes given, %zu needed", c.ws_bytes, need);
        if (c.g->tv_dims != 2 || c.tau == 0.0) {
            PS_TRY(fgp_single_t<T>(c, st));
            continue;
        }
        progs.emplace_back();
        PS_TRY(fgp2d_program<T>(c, n2d > 1, progs.back()));
    }
    size_t rounds = 0;
    for (const auto &p : progs) {
        rounds = std::max(rounds, p.launches.size());
        if (p.pre_copy_dst) {
            hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(p.n)), dim3(kBlock), 0, st, p.pre_copy_dst, p.pre_copy_src, p.n);
            PS_LAUNCHED("k_copy");
        }
        if (p.pre_fill) {
            hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(p.dn)), dim3(kBlock), 0, st, p.pre_fill, p.dn, T(0));
            PS_LAUNCHED("k_fill");
        }
    }
    // solves of one tile shape share launches
    std::vector<FgpTile> tiles;
    for (const auto &p : progs) {
        bool seen = false;
        for (const FgpTile &t : tiles)
            seen = seen || (t.waves == p.tile.waves && t.rows == p.tile.rows && t.cols == p.tile.cols);
        if (!seen) tiles.push_back(p.tile);
    }
    for (size_t r = 0; r < rounds; ++r) {
        for (const FgpTile &tile : tiles) {
            ListBuilder<FgpItem<T>> lb;
            for (const auto &p : progs) {
                if (r >= p.launches.size() || p.tile.waves != tile.waves || p.tile.rows != tile.rows ||
                    p.tile.cols != tile.cols)
                    continue;
                const FgpItem<T> &it = p.launches[r];
                const long blocks = static_cast<long>(it.tiles_x) * it.tiles_y * (it.ncomp / (static_cast<size_t>(it.nx) * it.ny));
                lb.add(it, static_cast<int>(blocks));
                if (lb.full()) {
                    PS_TRY(launch_fgp2d_list<T>(lb.wl, lb.blocks, tile, st));
                    lb.clear();
                }
            }
            if (!lb.empty()) PS_TRY(launch_fgp2d_list<T>(lb.wl, lb.blocks, tile, st));
        }
    }
    for (const auto &p : progs) {
        if (p.post_copy_dst) {
            hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(p.dn)), dim3(kBlock), 0, st, p.post_copy_dst, p.post_copy_src, p.dn);
            PS_LAUNCHED("k_copy");
        }
    }
    return PS_OK;
}

ps_status launch_fgp_many(const FgpCall *calls, int n, hipStream_t st) {
    std::vector<FgpCall> f32, f64;
    for (int c = 0; c < n; ++c) (calls[c].g->desc.dtype == PS_F64 ? f64 : f32).push_back(calls[c]);
    if (!f32.empty()) PS_TRY(fgp_many_t<float>(f32.data(), static_cast<int>(f32.size()), st));
    if (!f64.empty()) PS_TRY(fgp_many_t<double>(f64.data(), static_cast<int>(f64.size()), st));
    return PS_OK;
}

ps_status launch_fgp(const ps_geometry *g, const void *v, void *dual, double tau, int n_inner,
                     int nonneg, const FgpOut &out, void *ws, size_t ws_bytes, hipStream_t st) {
    const FgpCall c{g, v, dual, tau, n_inner, nonneg, out, ws, ws_bytes};
    return launch_fgp_many(&c, 1, st);
}

}  // namespace ps

using namespace ps;

extern "C" size_t tv_prox_workspace_bytes(const ps_geometry *g) { return g ? fgp_workspace(g) : 0; }

extern "C" ps_status tv_prox_fgp(const ps_geometry *g, const void *v, void *z, double tau,
                                 int32_t n_inner, int32_t nonneg, void *dual, void *workspace,
                                 size_t ws_bytes, void *stream) {
    clear_error();
    if (!g) return fail(PS_EINVAL, "geometry is null");
    PS_TRY(check_ptr(v, "v", g->elem));
    PS_TRY(check_ptr(z, "z", g->elem));
    if (dual) PS_TRY(check_ptr(dual, "dual", g->elem));
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(PS_EINVAL, "tau must be finite and >= 0");
    if (n_inner < 0) return fail(PS_EINVAL, "n_inner must be >= 0");
    if (nonneg != 0 && nonneg != 1) return fail(PS_EINVAL, "nonneg must be 0 or 1");
    FgpOut o{};
    o.z = z;
    o.proxskip = 0;
    return launch_fgp(g, v, dual, tau, n_inner, nonneg, o, workspace, ws_bytes,
                      static_cast<hipStream_t>(stream));
}
