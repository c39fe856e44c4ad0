// Internal declarations shared by the translation units of libapr.so.
// gfx950 only: wave64, 4 SIMD16 per CU, 160 KB LDS per CU, 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/apr.h"

namespace apr {

constexpr int kWave = 64;
constexpr int kCell = 64;       // particles per leaf cell (one wavefront)
constexpr int kFan = 64;        // tree fan-out (one wavefront tests all children)
constexpr int kMaxLev = 6;      // tree levels above the cells
constexpr int kNumXcd = 8;      // MI355X: workgroups go round-robin over 8 XCDs
constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxDevices = 64;  // GPUs per process the allocation-free scratch table covers
constexpr int kDtParts = 1024;   // partial minima of the timestep reduction

// Status words on the device (ctx->d_status).
enum {
    ST_NOCONV = 0,        // h-rho solves that hit max_iter
    ST_RANGE = 1,         // a converged h at or beyond the periodic limit (2h < box/4)
    ST_DENS_DIRECT = 2,   // density: cells whose staged set did not fit in LDS
    ST_FORCE_DIRECT = 3,  // forces: same
    ST_SUB_DIRECT = 4,    // sub-block lists that did not fit
    ST_RESTAGE = 5,       // density: searches repeated for a larger radius
    ST_PASSES = 6,        // density: Newton passes summed over cells
    ST_WINDOWS = 7,       // staged windows summed over cells and passes
    ST_BAND = 8,          // density targets whose support-test guard band exceeds the
                          // staging slack (|t|_1 >= 126 R; none expected)
    ST_EDGE = 9,          // pair tests decided in FP64 inside the guard band
    ST_WORDS = 10
};

// A leaf cell or a tree node: centre in FP64 and conservative (rounded-up)
// FP32 half extents and largest smoothing length.
struct Geo {
    double cx, cy, cz;
    float ex, ey, ez;
    float hmax;
};

// Counts of the cell structure, written on the device by the cell build so
// that no host synchronisation is needed; kernels sized by upper bounds read
// it and retire surplus workgroups.
struct Hdr {
    int32_t ncells;
    int32_t nnode[kMaxLev + 1];  // nnode[0] = ncells
};

struct Box {
    double lo[3], L[3];
    int periodic;
};

}  // namespace apr

struct apr_ctx {
    apr_params p;
    hipStream_t stream = nullptr;
    int device = -1;               // the HIP device current at creation
    std::string err;
    struct Buf {
        std::string name;
        void *p;
        size_t bytes;
    };
    std::vector<Buf> bufs;
    int32_t *d_status = nullptr;   // apr::ST_WORDS ints
    int32_t *h_status = nullptr;   // pinned host copy
    // cell structure of the last apr_build_cells.  The cell count lives on
    // the device (Hdr); per-cell kernels stride over it, so their launch
    // grids may be any size: the host sizes them from the last count it read
    // back (asynchronously, into pinned memory) and sizes buffers by bounds
    // that always hold (at most one cell per particle).
    int64_t cells_n = -1;          // particles it was built for
    int nlev = 0;                  // tree levels above the cells (enough for n cells)
    int64_t node_cap[apr::kMaxLev + 1] = {};   // buffer bound per level (level 0: cells)
    int64_t node_grid[apr::kMaxLev + 1] = {};  // launch grid per level
    uint64_t *count_pin = nullptr; // pinned host word: (build number << 32) | cell count,
                                   // written by the cell build's last scan kernel
    uint32_t build_no = 0;         // builds so far
    uint32_t count_no = 0;         // build number of count_last
    int64_t build_n[16] = {};      // particles of the last 16 builds (by number % 16)
    int64_t count_last = 0, count_last_n = 0;  // last count read, and its n
    int64_t grid_set = 0;          // apr_set_cell_grid (0: from the count)
    // derived values of the last density / force evaluation (workspace)
    int64_t dens_n = -1;           // n of the last apr_density (for the split cap)
    int64_t force_n = -1;          // n of the last force evaluation (for the timestep)
    int64_t divv_n = -1;           // velocity divergence of the last force evaluation is in the
                                   // workspace "divv" in the current particle order (else -1)
    int64_t divv_prev_n = -1;      // the one before it, carried through the last cell build's
                                   // permutation, is in "divv_prev" (else -1)
    double dt_last = 0.0;          // dt of the last step (the spacing of those two)
    // individual timesteps: each particle's last rho, Omega, vsig and nearest
    // distance ("bn_*" workspace, the context precision) follow the state
    // while only apr_bins_init / apr_step_bins reorder it
    int64_t bins_n = -1;           // n they are valid for (else -1)
    bool in_bins = false;          // set while the step driver itself reorders
    // kernel timing: pairs of events per index, summed at read time
    bool prof = false;
    uint32_t prof_mask = ~0u;      // indices timed while prof is on (bit 1 << index)
    struct EvPair {
        int idx;
        hipEvent_t a, b;
    };
    std::vector<EvPair> ev_used, ev_free;
    double prof_ms[APR_PROF_N] = {};
    int64_t prof_cnt[APR_PROF_N] = {};
};

namespace apr {

// Grow-only named device workspace.  Contents are not kept across growth.
void *ws(apr_ctx *c, const char *name, size_t bytes);
// The same, but a growing buffer keeps its first `keep` bytes.
void *ws_keep(apr_ctx *c, const char *name, size_t bytes, size_t keep);
template <class T>
T *wsa(apr_ctx *c, const char *name, size_t count)
{
    return static_cast<T *>(ws(c, name, count * sizeof(T) + 256));
}

int fail(apr_ctx *c, int code, const std::string &msg);
int fail(apr_ctx *c, int code, const char *msg);
int hip_check(apr_ctx *c, hipError_t e, const char *what);
#define APR_HIP(ctx, call)                                        \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return apr::hip_check(ctx, e_, #call); \
    } while (0)
#define APR_LAUNCHED(ctx)                                                    \
    do {                                                                     \
        hipError_t e_ = hipGetLastError();                                   \
        if (e_ != hipSuccess) return apr::hip_check(ctx, e_, "kernel launch"); \
    } while (0)

inline Box make_box(const apr_params &p)
{
    Box b;
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = p.box_lo[k];
        b.L[k] = p.box_hi[k] - p.box_lo[k];
    }
    b.periodic = p.periodic;
    return b;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ----------------------------------------------------------------- device side
__device__ inline int lane_id() { return __lane_id(); }

__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// The wavefront's index in its workgroup, as a scalar (uniform) value.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)); }

// The value of lane (lane ^ O), for every lane of the wavefront, with no
// address register (a ds_bpermute needs one per distance, and the compiler
// keeps those live across a whole kernel): O = 1, 2 quad permutations and
// O = 8 a rotation of the 16-lane row by half its length (DPP), O = 4 the
// swizzle's xor mode, O = 16 and 32 gfx950's swaps of odd and even rows and
// of the wavefront's halves.  Every lane must be active.
template <int O>
__device__ inline int lane_xor_bits(int v)
{
    static_assert(O == 1 || O == 2 || O == 4 || O == 8 || O == 16 || O == 32, "lane distance");
    if constexpr (O == 1) {
        return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    } else if constexpr (O == 2) {
        return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else if constexpr (O == 4) {
        return __builtin_amdgcn_ds_swizzle(v, 0x101F);  // and 0x1f, or 0, xor 4
    } else if constexpr (O == 8) {
        return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else if constexpr (O == 16) {
        // the swap leaves rows (r0, r0, r2, r2) in the first result and
        // (r1, r1, r3, r3) in the second
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane_id() & 16) ? (int)p[0] : (int)p[1];
    } else {
        // halves (lo, lo) in the first result, (hi, hi) in the second
        const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane_id() & 32) ? (int)p[0] : (int)p[1];
    }
}
// For O = 16 or 32: the values of the two lanes (lane & ~O, lane | O), in
// that order, in every lane: an operation on the pair then gives partner
// lanes the same result, with one swap and no select.
template <int O>
__device__ inline void lane_pair_bits(int v, int &lo, int &hi)
{
    static_assert(O == 16 || O == 32, "row or half swap");
    const auto p = O == 16 ? __builtin_amdgcn_permlane16_swap(v, v, false, false)
                           : __builtin_amdgcn_permlane32_swap(v, v, false, false);
    lo = (int)p[0];
    hi = (int)p[1];
}
template <int O>
__device__ inline void lane_pair(float v, float &lo, float &hi)
{
    int a, b;
    lane_pair_bits<O>(__float_as_int(v), a, b);
    lo = __int_as_float(a);
    hi = __int_as_float(b);
}
template <int O>
__device__ inline void lane_pair(double v, double &lo, double &hi)
{
    const long long x = __double_as_longlong(v);
    int a0, b0, a1, b1;
    lane_pair_bits<O>((int)(x & 0xffffffffll), a0, b0);
    lane_pair_bits<O>((int)(x >> 32), a1, b1);
    lo = __longlong_as_double(((long long)a1 << 32) | (long long)(unsigned)a0);
    hi = __longlong_as_double(((long long)b1 << 32) | (long long)(unsigned)b0);
}
template <int O>
__device__ inline int lane_xor(int v) { return lane_xor_bits<O>(v); }
template <int O>
__device__ inline float lane_xor(float v) { return __int_as_float(lane_xor_bits<O>(__float_as_int(v))); }
template <int O>
__device__ inline double lane_xor(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = lane_xor_bits<O>((int)(b & 0xffffffffll)), hi = lane_xor_bits<O>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// XCD-aware mapping of a 1-D grid: workgroup b runs on XCD b % 8, so give XCD
// k a contiguous range of work items (neighbouring cells share candidates and
// hit the same L2).
__device__ inline int64_t xcd_swizzle(int64_t b, int64_t nb)
{
    int64_t per = (nb + kNumXcd - 1) / kNumXcd;
    int64_t x = b % kNumXcd, r = b / kNumXcd;
    int64_t full = nb % kNumXcd == 0 ? kNumXcd : nb % kNumXcd;  // XCDs with `per` items
    // XCDs 0..full-1 own `per` items, the rest own per-1
    int64_t base = x < full ? x * per : full * per + (x - full) * (per - 1);
    return base + r;
}

// First cell of workgroup b of a per-cell kernel launched with grid G over nc
// cells; -1 if b has no cell.  Cells from G on are the caller's.  Cells
// [0, min(nc, G)) go to the XCDs in chunks of consecutive cells (Morton order:
// a compact group whose candidates mostly share the XCD's L2), dealt in turn,
// so that every XCD samples the whole domain: the cost per cell varies in
// space (a shock front, a dense disc midplane), and one contiguous eighth per
// XCD left the XCDs with the costlier regions running up to 35 % longer.  A
// chunk holds kXcdChunk cells, or more on large sets (at most kXcdRounds
// chunks per XCD), where longer chunks cut the reads of candidates beyond
// the chunk; the cells after the last whole round of chunks go in contiguous
// ranges.
constexpr int64_t kXcdChunk = 128;
constexpr int64_t kXcdRounds = 64;
__device__ inline int64_t first_cell(int64_t b, int64_t G, int64_t nc)
{
    const int64_t m = nc < G ? nc : G;
    if (b >= m) return -1;
    int64_t ch = m / (kNumXcd * kXcdRounds);
    ch = ch > kXcdChunk ? ch : kXcdChunk;
    const int64_t full = m / (kNumXcd * ch) * (kNumXcd * ch);
    if (b < full) {
        const int64_t x = b % kNumXcd, r = b / kNumXcd;
        return (r / ch * kNumXcd + x) * ch + r % ch;
    }
    return full + xcd_swizzle(b - full, m - full);
}

// Minimum-image component of a displacement (periodic box of side L).
__device__ inline double min_image(double d, double L, int periodic)
{
    if (periodic) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

// Squared gap between two boxes (centre, half extent); the centre difference
// takes the minimum image.  Conservative for culling.
__device__ inline double gap2(const Geo &a, const Geo &b, const Box &bx)
{
    double d[3] = {min_image(a.cx - b.cx, bx.L[0], bx.periodic),
                   min_image(a.cy - b.cy, bx.L[1], bx.periodic),
                   min_image(a.cz - b.cz, bx.L[2], bx.periodic)};
    double e[3] = {(double)a.ex + (double)b.ex, (double)a.ey + (double)b.ey,
                   (double)a.ez + (double)b.ez};
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        double g = fabs(d[k]) - e[k];
        if (g > 0.0) s += g * g;
    }
    return s;
}

// Round a non-negative double up to a float that is >= it.
__device__ inline float f_up(double v)
{
    float f = (float)v;
    if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);  // next float up (v >= 0)
    return f;
}

template <class T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};
template <class T>
using vec4_t = typename Vec4<T>::type;

// ------------------------------------------------------------ host launchers
// sort.hip
int exclusive_scan_u32(apr_ctx *c, const uint32_t *in, uint32_t *out, int64_t n,
                       uint32_t *total_dev);
int exclusive_scan_i64(apr_ctx *c, const int64_t *in, int64_t *out, int64_t n,
                       int64_t *total_dev);
int radix_sort_u32(apr_ctx *c, uint32_t *keys, uint32_t *vals, int64_t n, int bits,
                   uint32_t **keys_out = nullptr, uint32_t **vals_out = nullptr);

// cells.hip
// keep_accel false: ax, ay, az, dudt are left unpermuted (the caller
// recomputes them before reading them)
int build_cells(apr_ctx *c, apr_state *s, int64_t *perm, bool keep_accel = true);
// The cells of the last build, refitted to particles that moved but kept
// their order: boxes, centres, h_max, cell-frame positions and the tree's
// boxes from the current state (no sort, no permutation).
int refit_cells(apr_ctx *c, apr_state *s);
int refit_hmax_from_cells(apr_ctx *c);   // tree nodes' hmax from the cells' hmax
int set_hmax_new(apr_ctx *c, const float *hmax_new);  // cells' hmax from hmax_new[cell], then the tree's
int cells_hmax_from(apr_ctx *c, const double *h, int64_t n);  // cells' hmax from h, then refit
const Hdr *cell_hdr(apr_ctx *c);
const int32_t *cell_start(apr_ctx *c);
Geo *cell_level(apr_ctx *c, int lev);

// density.hip / forces.hip
// active (optional, [n], state order): only those targets are solved; the
// others keep h, rho and Omega (individual timesteps).
int density(apr_ctx *c, apr_state *s, void *rho, void *omega, int32_t *nneigh, int32_t *iters,
            const uint8_t *active = nullptr);
// hmax_fresh: the cells' h_max already hold the state's h (a density pass on
// this state just ran), so the refit from h is skipped.
// active (optional): only those targets get their sums (outputs of the
// others untouched).
// npair (optional, [n]): pairs per target (b != a, r < 2 max(h_a, h_b)).
int forces(apr_ctx *c, const apr_state *s, const void *rho, const void *omega, void *ax,
           void *ay, void *az, void *dudt, void *vsig, bool hmax_fresh = false,
           const uint8_t *active = nullptr, int32_t *npair = nullptr);
// EOS pack of forces.hip: vh = (v, 1/h), th = (P/(Omega rho^2), 1/(Omega rho), c, 0)
// into the workspace buffers vh32/th32 (FP32) or vh64/th64 (FP64).
int eos_pack(apr_ctx *c, const apr_state *s, const void *rho, const void *omega);

// adjoint.hip
int vjp(apr_ctx *c, const apr_state *s, const void *rho, const void *omega, const void *rho_bar,
        const void *h_bar, const void *ax_bar, const void *ay_bar, const void *az_bar,
        const void *dudt_bar, void *xbar, void *ybar, void *zbar, void *mbar);

// bins.hip (individual timesteps)
int bins_init(apr_ctx *c, apr_state *s, int8_t *bin, const apr_sink *sinks, int nsinks,
              double dt_max, double c_cfl, int max_bin);
int step_bins(apr_ctx *c, apr_state *s, int8_t *bin, const apr_zone *zones, int nzones,
              const apr_sink *sinks, int nsinks, double dt_max, double c_cfl, int max_bin,
              int64_t step, int32_t *nsub);

// relax.hip
int relax(apr_ctx *c, apr_state *s, apr_ctx *rc, const apr_state *ref, const void *ref_rho,
          const void *ref_ax, const void *ref_ay, const void *ref_az, int32_t max_shuffles,
          double ke_frac, int32_t *n_shuffles, double *ke_first, double *ke_last);

// neighbours.hip
int neighbours(apr_ctx *c, const apr_state *s, const double *h, int mode, int64_t *counts,
               int64_t *offsets, int64_t *list, int64_t cap, int64_t *total);

// integrate.hip
// kick by dtk, then drift; with hfac_out the h prediction is stored (a
// workspace of n factors, or null when there is none) instead of applied
int kick_drift(apr_ctx *c, apr_state *s, double dtk, double dt, double **hfac_out = nullptr);
int hfac_apply(apr_ctx *c, apr_state *s, const int64_t *origin, const double *hfac);
// kick_dt != 0: also v += kick_dt a (and u) with the new accelerations
int total_accel(apr_ctx *c, apr_state *s, const void *ax, const void *ay, const void *az,
                const void *dudt, const apr_sink *sinks, int nsinks, double kick_dt = 0.0,
               const uint8_t *active = nullptr, const int8_t *bin = nullptr,
               double dt_max = 0.0);
int min_timestep(apr_ctx *c, const apr_state *s, const void *vsig, double C, double *dt);
// the same reduction into a device double, with the partial minima in the
// library's per-device scratch array: no allocation, no synchronisation
int dt_scratch_setup(apr_ctx *c);
int min_timestep_noalloc(apr_ctx *c, const apr_state *s, const void *vsig, double C,
                         double *dt_dev);
// an existing workspace buffer of at least `bytes`, or null (never allocates)
void *ws_peek(apr_ctx *c, const char *name, size_t bytes);

// splitmerge.hip
// Individual timesteps: active (optional, [n]) restricts the pass to those
// particles; origin (optional, room for capacity) receives each slot's slot
// before the pass (an appended child: its parent's); made (optional, room for
// capacity) flags what a split made or a merge kept.
int split_merge(apr_ctx *c, apr_state *s, const apr_zone *zones, int nzones, int64_t step,
                int flags, int64_t *n_split, int64_t *n_merged, int64_t *n_spare,
                const uint8_t *active = nullptr, int64_t *origin = nullptr,
                uint8_t *made = nullptr);

// kernel timing: prof_begin returns a token for prof_end (-1 when disabled)
int prof_begin(apr_ctx *c, int idx);
void prof_end(apr_ctx *c, int token);

// fill helpers (kernels, so that they can sit inside captured graphs)
int fill_i32(apr_ctx *c, int32_t *p, int32_t v, int64_t n);
int fill_u32(apr_ctx *c, uint32_t *p, uint32_t v, int64_t n);

}  // namespace apr
