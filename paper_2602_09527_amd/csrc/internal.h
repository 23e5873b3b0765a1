// internal.h -- shared declarations of the HIP library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "proxskip.h"

namespace ps {

// ---------------------------------------------------------------------------------------------
// Errors: every exported call returns a ps_status and records a message per thread.
// ---------------------------------------------------------------------------------------------
ps_status fail(ps_status s, const char *fmt, ...);
void clear_error();

#define PS_HIP(call)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::ps::fail(PS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));          \
    } while (0)

#define PS_LAUNCHED(name)                                                                       \
    do {                                                                                        \
        hipError_t e_ = hipGetLastError();                                                      \
        if (e_ != hipSuccess)                                                                   \
            return ::ps::fail(PS_EHIP, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
    } while (0)

#define PS_TRY(expr)                                                                            \
    do {                                                                                        \
        ps_status s_ = (expr);                                                                  \
        if (s_ != PS_OK) return s_;                                                             \
    } while (0)

constexpr int kBlock = 256;        // threads per block of every 1D-shaped kernel
constexpr int kMaxDim = 4096;      // largest nx, ny supported by the LDS plans
constexpr int kMaxBins = 2048;     // largest B (8 rays per thread x 256 threads)
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Per-angle constants of the Joseph walk, in the arithmetic type T.
//   row-walked angle (|cos| >= |sin|): fractional column at (bin u, row i) is
//       q = a0 + u a1 + i a2,  a1 = du/c, a2 = -s/c,
//       a0 = (off - (B-1)/2 du + (ny-1)/2 s)/c + (nx-1)/2,     inv = 1/|c|
//   column-walked angle: fractional row at (bin u, column j) is
//       q = a0 + u a1 + j a2,  a1 = du/s, a2 = -c/s,
//       a0 = (off - (B-1)/2 du + (nx-1)/2 c)/s + (ny-1)/2,     inv = 1/|s|
//   ia1 = 1/a1 (bins per unit of q), row = 1 for row-walked angles.
//   q0, q1, q2: a0, a1, a2 in signed 32.32 fixed point (round(a * 2^32)).  The FP32 kernels
//   evaluate q = q0 + u q1 + t q2 exactly in 64-bit integers: floor(q) is the high word and the
//   interpolation weight the low word, so positions keep 2^-32 resolution at any image size
//   (an FP32 q near 1000 would only resolve 6e-5).
template <typename T>
struct AngleTab {
    const T *a0, *a1, *a2, *inv, *ia1;
    const int32_t *row;
    const int64_t *q0, *q1, *q2;
    const int32_t *ord_full, *ord_sub;
};

// Launch plan of the forward projector for one subset size.
struct ProjPlan {
    int split;      // S: blocks along the ray (partial sums reduced in a second pass when > 1)
    int strip;      // steps of the image staged in LDS at a time
    int stride;     // LDS row stride (elements)
    int rpt;        // rays per thread: 1, 2, 4 or 8
    size_t lds_bytes;
};

// Launch plan of the backprojector (ray-driven scatter into LDS strips, see backproject.hip).
struct BackPlan {
    int strip;      // R: image rows (or columns) per workgroup strip
    int waves;      // waves per workgroup, each with a private accumulator strip
    int stride;     // LDS row stride (floats): max(nx, ny) + 4
    int groups;     // G: angle groups, each producing a partial image per angle class
    int s_row, s_col;  // strips of rows (row-walked angles) and of columns
    size_t lds_bytes;
    size_t part_elems;  // elements of the partial-image workspace (2 G n)
};

}  // namespace ps

struct ps_geometry {
    ps_geometry_desc desc;                // angles pointer re-pointed at `angles`
    std::vector<double> angles;           // A angles (radians)
    int tv_dims;                          // 2 or 3
    size_t elem;                          // sizeof(dtype)
    // host image of the device tables, in the dtype; offsets into it
    std::vector<unsigned char> host_tab;
    size_t off_a0, off_a1, off_a2, off_inv, off_ia1, off_row, off_q0, off_q1, off_q2, tab_bytes;
    void *dev;                            // uploaded tables (caller-owned), or null
    int bp_passes;                        // backprojector ray passes (see BackPlan)
    bool gather_ok;                       // adjacent rays >= 1 pixel apart at every angle
    // angle lists, row-walked first: all angles, and subset i at order_sub[sub_off[i]..]
    std::vector<int32_t> order_full, order_sub, sub_off, nrow_sub;
    int nrow_full;
    size_t off_ord_full, off_ord_sub;
    ps_plan plan;                         // launch-plan overrides (0 = automatic)
};

namespace ps {

int subset_count(const ps_geometry *g, int subset);  // a_i, or -1 if subset is invalid
int max_subset_count(const ps_geometry *g);
ps_status check_ready(const ps_geometry *g);
ps_status check_ptr(const void *p, const char *what, size_t align);

template <typename T>
AngleTab<T> angle_tab(const ps_geometry *g) {
    const unsigned char *b = static_cast<const unsigned char *>(g->dev);
    return AngleTab<T>{reinterpret_cast<const T *>(b + g->off_a0),
                       reinterpret_cast<const T *>(b + g->off_a1),
                       reinterpret_cast<const T *>(b + g->off_a2),
                       reinterpret_cast<const T *>(b + g->off_inv),
                       reinterpret_cast<const T *>(b + g->off_ia1),
                       reinterpret_cast<const int32_t *>(b + g->off_row),
                       reinterpret_cast<const int64_t *>(b + g->off_q0),
                       reinterpret_cast<const int64_t *>(b + g->off_q1),
                       reinterpret_cast<const int64_t *>(b + g->off_q2),
                       reinterpret_cast<const int32_t *>(b + g->off_ord_full),
                       reinterpret_cast<const int32_t *>(b + g->off_ord_sub)};
}

// ---------------------------------------------------------------------------------------------
// Work lists.  A batched launch processes up to kMaxItems independent items (one problem's
// operator application each: its own geometry, buffers and launch plan) over a 1D grid; item i
// owns workgroups [first[i], first[i+1]).  An item computes exactly what it computes alone, so
// results do not depend on what else shares the launch.  The list travels in the kernel
// arguments (no device-side descriptor memory).
// ---------------------------------------------------------------------------------------------
constexpr int kMaxItems = 16;

template <typename Item>
struct WorkList {
    int count;
    int first[kMaxItems + 1];
    Item item[kMaxItems];
};

// Index of the item that owns this workgroup, and the workgroup's index within that item.
template <typename Item>
__device__ inline int work_item(const WorkList<Item> &wl, int &local) {
    const int b = static_cast<int>(blockIdx.x);
    int i = 0;
#pragma unroll
    for (int q = 1; q < kMaxItems; ++q)
        if (q < wl.count && b >= wl.first[q]) i = q;
    local = b - wl.first[i];
    return i;
}

// XCD-aware workgroup order.  The dispatcher hands workgroup b of a launch to XCD b mod 8 (round
// robin over the chip's 8 XCDs, each with its own 4 MB L2).  xcd_order maps that dispatch index
// to a logical index such that every XCD receives one contiguous range of logical workgroups, in
// order: neighbouring tiles (halos), the strips of one angle group or one slab of slices then
// share an L2 instead of each XCD fetching all of it.  A bijection of [0, nb): it moves work
// between XCDs, it never changes what a workgroup computes.
constexpr int kXcds = 8;
__device__ inline int xcd_order(int b, int nb) {
    const int x = b % kXcds, q = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    return x * per + min(x, rem) + q;
}

// work_item over the XCD-ordered grid (the items' ranges are logical workgroup ranges).
template <typename Item>
__device__ inline int work_item_xcd(const WorkList<Item> &wl, int &local) {
    const int b = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    int i = 0;
#pragma unroll
    for (int q = 1; q < kMaxItems; ++q)
        if (q < wl.count && b >= wl.first[q]) i = q;
    local = b - wl.first[i];
    return i;
}

// Measurement support (timer.hip): classes of kernel launches whose GPU time kernel_timer_start
// asks for; launch sites mark the launch of their class before and after it.  A launch of a list
// counts in the class of its first item.
enum KernelClass {
    KC_BP_SCATTER_SUBSET = 1, KC_BP_SCATTER_FULL = 2, KC_PROJECT_SUBSET = 3, KC_PROJECT_FULL = 4,
    KC_BP_COMBINE = 5, KC_PROJECT_REDUCE = 6, KC_BP_GATHER = 7, KC_FGP2D = 8, KC_FGP3D = 9
};
void timer_mark(int kernel_class, hipStream_t st, bool begin);

// Host side: append items, launching a kernel whenever the list is full.
template <typename Item>
struct ListBuilder {
    WorkList<Item> wl{};
    int blocks = 0;
    void clear() {
        wl.count = 0;
        blocks = 0;
        wl.first[0] = 0;
    }
    ListBuilder() { clear(); }
    bool full() const { return wl.count == kMaxItems; }
    bool empty() const { return wl.count == 0; }
    void add(const Item &it, int nblocks) {
        wl.item[wl.count] = it;
        wl.first[wl.count] = blocks;
        blocks += nblocks;
        ++wl.count;
        wl.first[wl.count] = blocks;
    }
};

// ---------------------------------------------------------------------------------------------
// Projector (project.hip).
// ---------------------------------------------------------------------------------------------
ProjPlan proj_plan(const ps_geometry *g, int na);
size_t proj_workspace(const ps_geometry *g, int na);
// y = A_sub (x - xs) [ - b_sub ]: xs and b may be null.  y is [nz][na][B].
struct ProjCall {
    const ps_geometry *g;
    int subset;
    const void *x, *xs, *b;
    void *y, *ws;
    size_t ws_bytes;
    const void *sig = nullptr;   // PDHG dual step: y = (y + sig (A x - b)) / (1 + sig), per ray
    bool first_pass_only = false;   // skip the split-ray sum: the partials stay in ws (kernel
                                    // timing, or a gather that adds them itself)
};
ps_status launch_project_many(const ProjCall *calls, int n, hipStream_t st);
ps_status launch_project(const ps_geometry *g, int subset, const void *x, const void *xs,
                         const void *b, void *y, void *ws, size_t ws_bytes, hipStream_t st);

// ---------------------------------------------------------------------------------------------
// Backprojector with fused epilogues (backproject.hip).
// ---------------------------------------------------------------------------------------------
enum BackMode { BP_OVERWRITE = 0, BP_ACCUMULATE = 1, BP_SVRG = 2, BP_SNAPSHOT = 3, BP_SAGA = 4,
                BP_GRADSTEP = 5, BP_PDHG = 6 };

// Gradient-step epilogue operands (BP_SVRG, BP_SNAPSHOT, BP_SAGA, BP_GRADSTEP), all [nz][ny][nx]:
//   d = A^T y at the pixel
//   BP_SVRG:     G = nsub * d + gs
//   BP_SNAPSHOT: gs = d (stored), G = d         (iteration at the snapshot: x = xs)
//   BP_SAGA:     G = nsub * (d - tab) + tsum, then tsum += d - tab, tab = d   (Eq. 4)
//   BP_GRADSTEP: v = x - gamma d -> vout         (full-gradient step, no h)
//   BP_PDHG:     w = P_C(x - tau (d + D^T y2)), vout = 2 w - x, x = w   (PDHG primal step;
//                tau per pixel in `gs`, y2 [d][n] in `tab`, the grid in nx, ny, nz)
//   plain:       v = x - gamma G                 -> vout
//   coin = 1:    v = x - gamma (G - h) - (gamma/p) h  -> vout
//   coin = 0:    x = x - gamma (G - h)           (in place)
struct UpdateArgs {
    void *x;
    const void *h;
    void *gs;
    void *vout;
    void *tab, *tsum;   // BP_SAGA: the table row of the subset and the table's running sum
    const void *xs;     // with dx: the snapshot, and
    void *dx;           //   dx = x - xs written beside x (coin = 0 steps of BP_SVRG / BP_SNAPSHOT)
    double gamma, gamma_over_p, nsub;
    int coin, plain;
    int nx, ny, nz, nonneg;   // BP_PDHG
};
BackPlan back_plan(const ps_geometry *g, int subset);
size_t back_workspace(const ps_geometry *g, int subset);
enum BackMethod { BP_SCATTER = 1, BP_GATHER = 2 };
int back_method(const ps_geometry *g, int subset);   // BP_SCATTER or BP_GATHER
int gather_rows(const ps_geometry *g, int subset);   // rows per wave of the gather tiles: 2 or 4
int gather_split(const ps_geometry *g, int subset);  // waves sharing a gather tile's rows: 1, 2 or 4
// Does a solver iteration hand subset `subset`'s projector partials straight to the gather?
// (the gather backprojects subsets, the projector splits rays, and the plan allows it)
bool gather_fused(const ps_geometry *g, int subset);
// Workgroups of a gather call with `rows` rows per wave (and the plan's angle split).
long gather_tiles(const ps_geometry *g, int subset, int rows);
struct BackCall {
    const ps_geometry *g;
    int subset;
    const void *y;
    void *out;
    int mode;
    UpdateArgs upd;
    void *ws;
    size_t ws_bytes;
    bool partials_only = false;     // scatter: skip the combine pass (kernel timing)
    // gather of a subset only: y holds the projector's psplit (> 1) partial sums, added during
    // staging as the projector's reduction pass would (minus pb when pb is not null)
    int psplit = 0;
    const void *pb = nullptr;
    int rows = 0;   // gather: rows per wave (2 or 4) in place of the plan's; 0 = the plan's
};
ps_status launch_backproject_many(const BackCall *calls, int n, hipStream_t st);
ps_status launch_backproject(const ps_geometry *g, int subset, const void *y, void *out, int mode,
                             const UpdateArgs *upd, void *ws, size_t ws_bytes, hipStream_t st);

// ---------------------------------------------------------------------------------------------
// TV prox by FGP (fgp.hip).
// ---------------------------------------------------------------------------------------------
size_t fgp_workspace(const ps_geometry *g);
int fgp_iters_per_launch(const ps_geometry *g);
int fgp_max_iters_of(const ps_geometry *g);
bool fgp_tile_ok(int waves, int rows);                 // a built 2D FGP tile shape
void fgp_tile_of(const ps_geometry *g, int *waves, int *rows);   // the shape in effect
int fgp_cols_of(const ps_geometry *g);                            // 2D FGP columns per lane: 1 or 2
constexpr int kF3Forms = 5;                                       // 3D launch forms 1..5
int fgp3d_form_of(const ps_geometry *g);                          // 3D launch form in effect
int fgp3d_chunk_of(const ps_geometry *g);                         // 3D z chunk in effect
// The SVRG solver's subset projections read one image (the kept difference x - xs) once x and xs
// together outgrow an XCD's L2, else the two images x and xs (solver.hip).
bool solver_reads_one_image(const ps_geometry *g);
// Finalise modes: write z (FGP_Z) or the ProxSkip update x = z, h = hscale (z - v) (FGP_PROXSKIP).
struct FgpOut {
    void *z;        // FGP_Z: output image (may alias v)
    void *x, *h;    // FGP_PROXSKIP
    double hscale;  // p / gamma
    int proxskip;   // 0: z, 1: proxskip update (h written), 2: plain (x = z, h untouched)
};
struct FgpCall {
    const ps_geometry *g;
    const void *v;
    void *dual;
    double tau;
    int n_inner, nonneg;
    FgpOut out;
    void *ws;
    size_t ws_bytes;
};
ps_status launch_fgp_many(const FgpCall *calls, int n, hipStream_t st);
ps_status launch_fgp(const ps_geometry *g, const void *v, void *dual, double tau, int n_inner,
                     int nonneg, const FgpOut &out, void *ws, size_t ws_bytes, hipStream_t st);

// ---------------------------------------------------------------------------------------------
// Solver pieces (solver.hip).
// ---------------------------------------------------------------------------------------------
uint64_t splitmix64(uint64_t seed, uint64_t j);
void draw_sequences(uint64_t seed, int64_t k0, int64_t count, int n_subsets, double p,
                    int32_t *subset_out, uint8_t *coin_out);
void draw_refresh(uint64_t seed, int64_t k0, int64_t count, int n_subsets, uint8_t *out);

}  // namespace ps
