// Band step: Jacobi steps of the first-order upwind update (Eq. 3-5) on the
// tiles of the band list, with the 7-point stencil staged through LDS.
//
// Work decomposition.  The band list is cut into x-runs: maximal sequences
// of consecutive tile ids in one tile row, broken at every R-th tile column,
// so a work item is a box of up to R*tx x ty x tz points whose grid rows are
// contiguous in HBM (R*tx = 32 FP32 values = 128 B by default).  A persistent
// grid of blocks walks the item list; block b takes a contiguous slice of it,
// and the slices of blocks that share an XCD (b mod 8) are adjacent, so
// neighbouring items share that XCD's L2.
//
// Ping-pong.  Step s reads buffer P[s%2] and writes P[(s+1)%2] (P[0] = phi,
// P[1] = scratch) on the band tiles only.  A neighbour point that lies in a
// tile outside the band is read from phi, which holds its (frozen) value for
// the whole call; a neighbour inside the band is read from P[s%2].
#include <algorithm>
#include <type_traits>
#include <cmath>

#include "ls_compact.h"
#include "ls_stats.h"
#include "ls_stencil.h"

namespace ls {

// One persistent block walks its slice of work items.  Per item:
//  (1) every thread issues the global loads of its own grid points (phi and
//      F, NOWN rows of the item), of its halo-row points (NHALO rows of the
//      y- and z-faces) and of at most two x-face points, all into registers;
//  (2) the values go to the LDS box; (3) after a barrier every thread
//      evaluates its own points from the box and stores them.
// Thread t owns column lx = t mod xl of rows lr + q*rp (rows enumerate (y, z)
// of a full tile, y fastest), so its row offsets are fixed for the launch.

// Tile shape of a launch: compile-time when CTX > 0 (every index below then
// folds to constants), else taken from g at run time.
template <int CTX, int CTY, int CTZ, int CR>
struct Shape {
    static constexpr bool fixed = CTX > 0;
    static constexpr int cxl = fixed ? cpow2(CR * CTX) : 0;
    __device__ static inline int tx(const StepGeom &g) { return fixed ? CTX : g.tx; }
    __device__ static inline int ty(const StepGeom &g) { return fixed ? CTY : g.ty; }
    __device__ static inline int tz(const StepGeom &g) { return fixed ? CTZ : g.tz; }
    __device__ static inline int xl(const StepGeom &g) { return fixed ? cxl : g.xl; }
    __device__ static inline int xl_log(const StepGeom &g) { return fixed ? clog2(cxl) : g.xl_log; }
    __device__ static inline int sx(const StepGeom &g) { return fixed ? CR * CTX + 2 : g.sx; }
};

template <class S, class FT, bool EXACT, int NOWN, int NHALO, class SH, int MODE>
__global__ __launch_bounds__(kBlock) void upwind_kernel(StepGeom g, StepArgs<S, FT> a) {
    using C = typename Codec<S>::C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *box = reinterpret_cast<C *>(smem);

    const int nitems = *a.nitems;
    int w0, w1;
    block_slice(0, nitems, &w0, &w1);

    const int TX = SH::tx(g), TY = SH::ty(g), TZ = SH::tz(g);
    const int lx = threadIdx.x & (SH::xl(g) - 1);
    const int lr = threadIdx.x >> SH::xl_log(g);
    const int rp = kBlock >> SH::xl_log(g);  // grid rows per pass
    const int lt = lx / TX;                  // tile of the run this column lies in
    const int sx = SH::sx(g), sxy = sx * (TY + 2);
    const int rows = TY * TZ;
    const int plane = g.ny * g.nx;      // < 2^31 (checked on the host)

    for (int w = w0; w < w1; ++w) {
        const int32_t *r = a.rec + static_cast<int64_t>(w) * kItemWords;
        const int t0 = r[0];
        if (t0 < 0 || t0 >= g.ntiles) continue;  // invalid id: skipped (uniform)
        const int len = r[1];
        const uint32_t m_ym = r[2], m_yp = r[3], m_zm = r[4], m_zp = r[5], m_x = r[6];
        const int ti0 = t0 % g.ntx;
        const int rr = t0 / g.ntx;
        const int tj = rr % g.nty, tk = rr / g.nty;
        const int x0 = ti0 * TX, y0 = tj * TY, z0 = tk * TZ;
        const int W = min(len * TX, g.nx - x0);
        const int H = min(TY, g.ny - y0);
        const int D = min(TZ, g.nz - z0);
        const int64_t base = (static_cast<int64_t>(z0) * g.ny + y0) * g.nx + x0;
        const S *cur = a.cur + base;    // item-relative (uniform) bases
        const S *orig = a.orig + base;
        const FT *Fb = MODE < kReinit ? a.F + base : nullptr;
        S *nxt = a.nxt + base;
        const bool col_ok = lx < W;

        // (1) loads, all issued before any is used ----------------------------
        S raw[NOWN];
        FT fv[NOWN];
#pragma unroll
        for (int q = 0; q < NOWN; ++q) {
            const int row = lr + q * rp;
            const int ly = row % TY, lz = row / TY;
            const int o = lz * plane + ly * g.nx + lx;
            if (col_ok && row < rows && ly < H && lz < D) {
                raw[q] = cur[o];
                if constexpr (MODE < kReinit) fv[q] = Fb[o];
            }
        }
        S hv[NHALO];
#pragma unroll
        for (int q = 0; q < NHALO; ++q) {
            const int h = lr + q * rp;
            int ly, lz;
            bool ok, in;
            if (h < 2 * TZ) {  // y-face rows, one per z
                lz = h >> 1;
                ly = (h & 1) ? H : -1;
                ok = lz < D;
                in = (((h & 1) ? m_yp : m_ym) >> lt) & 1u;
            } else {             // z-face rows, one per y
                const int hh = h - 2 * TZ;
                ly = hh >> 1;
                lz = (hh & 1) ? D : -1;
                ok = hh < 2 * TY && ly < H;
                in = (((hh & 1) ? m_zp : m_zm) >> lt) & 1u;
            }
            // clamped (Neumann) coordinates, relative to the item origin
            const int cy = min(max(y0 + ly, 0), g.ny - 1) - y0;
            const int cz = min(max(z0 + lz, 0), g.nz - 1) - z0;
            const bool inside = cy >= 0 && cy < H && cz >= 0 && cz < D;
            const int o = cz * plane + cy * g.nx + lx;
            ok = ok && col_ok;
            if (ok && (inside || in)) hv[q] = cur[o];
            if (ok && !(inside || in)) hv[q] = orig[o];
        }
        S xv[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = threadIdx.x + q * kBlock;  // x-face point e: side e&1, row e>>1
            const int row = e >> 1;
            const int ly = row % TY, lz = row / TY;
            const bool ok = row < rows && ly < H && lz < D;
            const int side = e & 1;
            const int cx = min(max(side ? x0 + W : x0 - 1, 0), g.nx - 1) - x0;
            const bool in = (cx >= 0 && cx < W) || ((m_x >> side) & 1u);
            const int o = lz * plane + ly * g.nx + cx;
            if (ok && in) xv[q] = cur[o];
            if (ok && !in) xv[q] = orig[o];
        }

        // (2) to LDS --------------------------------------------------------
#pragma unroll
        for (int q = 0; q < NOWN; ++q) {
            const int row = lr + q * rp;
            const int ly = row % TY, lz = row / TY;
            if (col_ok && row < rows && ly < H && lz < D)
                box[(lz + 1) * sxy + (ly + 1) * sx + lx + 1] = Codec<S>::load(raw[q], a.scale);
        }
#pragma unroll
        for (int q = 0; q < NHALO; ++q) {
            const int h = lr + q * rp;
            int ly, lz;
            bool ok;
            if (h < 2 * TZ) {
                lz = h >> 1;
                ly = (h & 1) ? H : -1;
                ok = lz < D;
            } else {
                const int hh = h - 2 * TZ;
                ly = hh >> 1;
                lz = (hh & 1) ? D : -1;
                ok = hh < 2 * TY && ly < H;
            }
            if (ok && col_ok)
                box[(lz + 1) * sxy + (ly + 1) * sx + lx + 1] = Codec<S>::load(hv[q], a.scale);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int row = e >> 1;
            const int ly = row % TY, lz = row / TY;
            if (row < rows && ly < H && lz < D) {
                const int lxh = (e & 1) ? W : -1;
                box[(lz + 1) * sxy + (ly + 1) * sx + lxh + 1] = Codec<S>::load(xv[q], a.scale);
            }
        }
        __syncthreads();  // box complete

        // (3) update ----------------------------------------------------------
#pragma unroll
        for (int q = 0; q < NOWN; ++q) {
            const int row = lr + q * rp;
            const int ly = row % TY, lz = row / TY;
            if (col_ok && row < rows && ly < H && lz < D) {
                const int o = (lz + 1) * sxy + (ly + 1) * sx + lx + 1;
                const C c = box[o], xm = box[o - 1], xp = box[o + 1], ym = box[o - sx],
                        yp = box[o + sx], zm = box[o - sxy], zp = box[o + sxy];
                C f = C(0);
                if constexpr (MODE < kReinit) f = static_cast<C>(fv[q]);
                f = mode_speed<MODE, C, EXACT>(f, c, xm, xp, ym, yp, zm, zp, a);
                S out = raw[q];
                if (f != C(0)) {
                    const C v = mode_finish<MODE, C, EXACT>(
                        upwind_point<C, EXACT>(c, xm, xp, ym, yp, zm, zp, f, a.dx, a.dt, a.dtdx),
                        f, a.dt, a.cut_gamma);
                    out = Codec<S>::store(v, a.scale);
                }
                nxt[lz * plane + ly * g.nx + lx] = out;
            }
        }
        __syncthreads();  // box free for the next item
    }
}

// Copies the band points of src into dst (used when nsteps is odd).
template <class S>
__global__ __launch_bounds__(kBlock) void band_copy_kernel(StepGeom g, const S *__restrict__ src,
                                                           S *__restrict__ dst,
                                                           const int32_t *rec,
                                                           const int32_t *nitems_dev) {
    const int nitems = *nitems_dev;
    int w0, w1;
    block_slice(0, nitems, &w0, &w1);
    const int lx = threadIdx.x & (g.xl - 1);
    const int lr = threadIdx.x >> g.xl_log;
    const int rp = kBlock >> g.xl_log;
    for (int w = w0; w < w1; ++w) {
        const int32_t *r = rec + static_cast<int64_t>(w) * kItemWords;
        const int t0 = r[0];
        if (t0 < 0 || t0 >= g.ntiles) continue;
        const int len = r[1];
        const int ti0 = t0 % g.ntx;
        const int rr = t0 / g.ntx;
        const int x0 = ti0 * g.tx, y0 = (rr % g.nty) * g.ty, z0 = (rr / g.nty) * g.tz;
        const int W = min(len * g.tx, g.nx - x0);
        const int H = min(g.ty, g.ny - y0);
        const int D = min(g.tz, g.nz - z0);
        if (lx >= W) continue;
        for (int row = lr; row < H * D; row += rp) {
            const int ly = row % H, lz = row / H;
            const int64_t gi = (static_cast<int64_t>(z0 + lz) * g.ny + (y0 + ly)) * g.nx + x0 + lx;
            dst[gi] = src[gi];
        }
    }
}

__global__ __launch_bounds__(kBlock) void map_set_kernel(uint8_t *map, const int32_t *tiles,
                                                         const int32_t *ntiles_dev,
                                                         int ntiles_cap) {
    const int n = min(*ntiles_dev, ntiles_cap);
    for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
        const int t = tiles[p];
        if (t >= 0 && t < ntiles_cap) map[t] = 1;
    }
}

// ---------------------------------------------------------------------------
// host side

// Process-wide launch tuning (ls_set_tuning); 0 fields mean the defaults.
static ls_tuning g_tuning = {0, 0, 0, 0, 0};
constexpr int kDefaultRunWidth = 32;
constexpr int kDefaultBlocksPerCu = 32;
// Grids whose phi exceeds this stream from HBM (beyond the Infinity Cache)
// with several work items per workgroup: the software-pipelined step pays.
constexpr int64_t kPipelineBytes = int64_t(1) << 30;

bool pipeline_forced() { return g_tuning.pipeline == 2; }
int brick_temporal_mode() { return g_tuning.temporal; }

bool use_pipeline(int64_t phi_bytes, int run_tiles) {
    if (g_tuning.pipeline == 1) return false;
    if (g_tuning.pipeline == 2) return true;
    // measured: with runs of more than 4 tiles the kernel's own loads hide the
    // latency and the second set of registers costs more than it gains
    return phi_bytes > kPipelineBytes && run_tiles <= 4;
}

static int run_width() { return g_tuning.run_width > 0 ? g_tuning.run_width : kDefaultRunWidth; }

// Tiles per work item: the run width in points, by default 128 bytes of
// stored phi (a full cache line per item row: 32 FP32, 64 FP16, 16 FP64 values).
int plan_run_tiles(const Geom &g) {
    if (g.run_tiles > 0) return std::min(kMaxRun, g.run_tiles);
    const int eb = g.elem_bytes > 0 ? g.elem_bytes : 4;
    const int width = g_tuning.run_width > 0 ? g_tuning.run_width : kDefaultRunWidth * 4 / eb;
    return std::max(1, std::min(kMaxRun, width / g.tx));
}

template <class S>
static int make_step_geom(const Geom &G, StepGeom *out, size_t *lds) {
    StepGeom s;
    s.nx = G.nx, s.ny = G.ny, s.nz = G.nz;
    s.tx = G.tx, s.ty = G.ty, s.tz = G.tz;
    s.ntx = G.ntx, s.nty = G.nty, s.ntz = G.ntz;
    s.ntiles = static_cast<int>(G.ntiles);
    s.R = plan_run_tiles(G);
    const int wbox = s.R * G.tx;
    int xl = 1, lg = 0;
    while (xl < wbox) xl <<= 1, ++lg;
    if (xl > kBlock) {
        set_error("step: tile width %d too large (max %d)", G.tx, kBlock);
        return LS_ERR_UNSUPPORTED;
    }
    s.xl = xl;
    s.xl_log = lg;
    const int rp = kBlock / xl;
    const int rows = G.ty * G.tz;
    if ((rows + rp - 1) / rp > kMaxOwn || rows > kBlock) {
        set_error("step: tile %dx%dx%d has too many rows per thread (max %d)", G.tx, G.ty, G.tz,
                  kMaxOwn);
        return LS_ERR_UNSUPPORTED;
    }
    if ((2 * (G.ty + G.tz) + rp - 1) / rp > kMaxHalo) {
        set_error("step: tile %dx%dx%d has too many halo rows per thread (max %d)", G.tx, G.ty,
                  G.tz, kMaxHalo);
        return LS_ERR_UNSUPPORTED;
    }
    if (static_cast<int64_t>(G.tz + 1) * G.ny * G.nx >= (int64_t(1) << 31)) {
        set_error("step: tile planes of %d x %d points too large", G.nx, G.ny);
        return LS_ERR_UNSUPPORTED;
    }
    s.sx = wbox + 2;
    s.sy = G.ty + 2;
    using C = typename Codec<S>::C;
    *lds = static_cast<size_t>(s.sx) * s.sy * (G.tz + 2) * sizeof(C);
    if (*lds > 64 * 1024) {
        set_error("step: tile %dx%dx%d needs %zu bytes of LDS (max 65536)", G.tx, G.ty, G.tz,
                  *lds);
        return LS_ERR_UNSUPPORTED;
    }
    *out = s;
    return LS_OK;
}

static int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <class S, class FT, bool EXACT>
using UpwindFn = void (*)(StepGeom, StepArgs<S, FT>);

using DynShape = Shape<0, 0, 0, 0>;

template <class S, class FT, bool EXACT, int NOWN, int MODE>
static UpwindFn<S, FT, EXACT> select_halo(int nhalo) {
    switch (nhalo) {
    case 1: return upwind_kernel<S, FT, EXACT, NOWN, 1, DynShape, MODE>;
    case 2: return upwind_kernel<S, FT, EXACT, NOWN, 2, DynShape, MODE>;
    case 4: return upwind_kernel<S, FT, EXACT, NOWN, 4, DynShape, MODE>;
    default: return upwind_kernel<S, FT, EXACT, NOWN, 8, DynShape, MODE>;
    }
}

// Kernel for a launch: a compile-time specialisation for the common tile
// shapes and run lengths, else the run-time-shape kernel, compiled for the
// step mode MODE (StepMode: plain, cut-off, reinitialisation).
template <class S, class FT, bool EXACT, int MODE = kPlain>
static UpwindFn<S, FT, EXACT> select_upwind_kernel(const StepGeom &sg, int nown, int nhalo,
                                                   size_t *lds, int *threads,
                                                   bool aligned = false) {
    *threads = kBlock;
    const bool whole_yz = sg.ny % sg.ty == 0 && sg.nz % sg.tz == 0;
    if constexpr (std::is_same<FT, float>::value && !EXACT) {
        // aligned rows: the vectorised form (same arithmetic, fewer memory instructions)
        if (g_tuning.vector != 1 && aligned && sg.nx % 4 == 0 && sg.tx == 8 && sg.ty == 8 &&
            sg.tz == 8 && (sg.R == 4 || sg.R == 8)) {
            if (sg.R == 4) {
                *lds = VecCfg<8, 8, 4>::lds;
                *threads = VecCfg<8, 8, 4>::NT;
                return whole_yz ? upwind_vec_kernel<S, 8, 8, 4, false, MODE>
                                : upwind_vec_kernel<S, 8, 8, 4, true, MODE>;
            }
            *lds = VecCfg<8, 8, 8>::lds;
            *threads = VecCfg<8, 8, 8>::NT;
            return whole_yz ? upwind_vec_kernel<S, 8, 8, 8, false, MODE>
                            : upwind_vec_kernel<S, 8, 8, 8, true, MODE>;
        }
    }
    const bool pipe = use_pipeline(int64_t(sg.nx) * sg.ny * sg.nz * int64_t(sizeof(S)), sg.R);
#define LS_FAST(TX_, TY_, TZ_, R_)                                                          \
    if (sg.tx == TX_ && sg.ty == TY_ && sg.tz == TZ_ && sg.R == R_) {                       \
        *lds = FastCfg<S, FT, TX_, TY_, TZ_, R_>::lds;                                      \
        *threads = FastCfg<S, FT, TX_, TY_, TZ_, R_>::NT;                                   \
        if (whole_yz)                                                                       \
            return pipe ? upwind_fast_kernel<S, FT, EXACT, TX_, TY_, TZ_, R_, false, false, true, MODE>  \
                        : upwind_fast_kernel<S, FT, EXACT, TX_, TY_, TZ_, R_, false, false, false, MODE>; \
        return pipe ? upwind_fast_kernel<S, FT, EXACT, TX_, TY_, TZ_, R_, false, true, true, MODE>        \
                    : upwind_fast_kernel<S, FT, EXACT, TX_, TY_, TZ_, R_, false, true, false, MODE>;      \
    }
    LS_FAST(8, 8, 8, 4)
    LS_FAST(8, 8, 8, 2)
    LS_FAST(8, 8, 8, 8)
    LS_FAST(16, 4, 4, 2)
    LS_FAST(16, 4, 4, 4)
    LS_FAST(32, 4, 4, 1)
    LS_FAST(32, 4, 4, 2)
    LS_FAST(16, 8, 8, 2)
    LS_FAST(4, 4, 4, 8)
#undef LS_FAST
    if (sg.tx == 8 && sg.ty == 8 && sg.tz == 8 && sg.R == 4)
        return upwind_kernel<S, FT, EXACT, 8, 4, Shape<8, 8, 8, 4>, MODE>;
    switch (nown) {
    case 1: return select_halo<S, FT, EXACT, 1, MODE>(nhalo);
    case 2: return select_halo<S, FT, EXACT, 2, MODE>(nhalo);
    case 4: return select_halo<S, FT, EXACT, 4, MODE>(nhalo);
    case 8: return select_halo<S, FT, EXACT, 8, MODE>(nhalo);
    default: return select_halo<S, FT, EXACT, 16, MODE>(nhalo);
    }
}

// The two-step kernel for this geometry when the tuning asks for it, or null:
// FP32 arithmetic on FP32 or FP16s storage, 8x8x8 tiles, whole tiles in y
// and z, nx a multiple of 4, 16-byte aligned buffers, items of 4 or 8 tiles.
// Off by default: it moves a third fewer bytes per step but measured slower
// than two one-step launches (fewer resident waves, a dependent U-map read
// before each halo load).
template <class S, class FT, bool EXACT>
static UpwindFn<S, FT, EXACT> select_upwind2_kernel(const StepGeom &sg, bool aligned, size_t *lds,
                                                    int *threads) {
    if constexpr (std::is_same<FT, float>::value && !EXACT) {
        if (g_tuning.temporal == 1 && g_tuning.vector != 1 && aligned && sg.nx % 4 == 0 &&
            sg.tx == 8 && sg.ty == 8 && sg.tz == 8 && sg.ny % 8 == 0 && sg.nz % 8 == 0) {
            if (sg.R == 4) {
                *lds = Vec2Cfg<4>::lds;
                *threads = Vec2Cfg<4>::NT;
                return upwind_vec2_kernel<S, 4>;
            }
            if (sg.R == 8) {
                *lds = Vec2Cfg<8>::lds;
                *threads = Vec2Cfg<8>::NT;
                return upwind_vec2_kernel<S, 8>;
            }
        }
    }
    return nullptr;
}

template <class K>
static int persistent_grid(K kernel, int threads, size_t lds, int *grid, int *limit = nullptr,
                           int64_t max_items = INT32_MAX) {
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != LS_OK) return rc;
    int per_cu = 0;
    LS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds));
    if (per_cu < 1) per_cu = 1;
    if (limit) *limit = per_cu;
    // Default: about one block per work item, beyond what fits at once, so the
    // dispatcher balances the uneven items (measured faster than a strictly
    // persistent grid); the blocks left without an item exit at once.
    per_cu = g_tuning.blocks_per_cu > 0 ? g_tuning.blocks_per_cu : kDefaultBlocksPerCu;
    int64_t G64 = std::min<int64_t>(int64_t(di.cus) * per_cu, max_items + 7);
    int G = static_cast<int>(std::max<int64_t>(8, G64 - G64 % 8));
    *grid = G;
    return LS_OK;
}

// Host checks shared by the step entry points and the driver.
template <class S, class FT>
static int step_args(S *phi, const FT *F, const ls_grid *grid, typename Codec<S>::C dx,
                     typename Codec<S>::C dt, int nsteps, S *scratch, void *workspace,
                     int64_t ws_bytes, Geom *G, StepGeom *sg, bool need_F = true) {
    using C = typename Codec<S>::C;
    int rc = make_geom(grid, G);
    if (rc != LS_OK) return rc;
    G->elem_bytes = static_cast<int32_t>(sizeof(S));
    if (!phi || (need_F && !F) || !scratch) {
        set_error(need_F ? "step: phi, F and scratch must be non-NULL"
                         : "step: phi and scratch must be non-NULL");
        return LS_ERR_ARG;
    }
    if (static_cast<const void *>(phi) == static_cast<const void *>(scratch)) {
        set_error("step: scratch must not alias phi");
        return LS_ERR_ARG;
    }
    if (nsteps < 0) {
        set_error("step: nsteps must be >= 0 (got %d)", nsteps);
        return LS_ERR_ARG;
    }
    if (!(dx > C(0)) || !(dx < C(INFINITY))) {
        set_error("step: dx must be positive and finite");
        return LS_ERR_ARG;
    }
    if (!(dt >= C(0)) || !(dt < C(INFINITY))) {
        set_error("step: dt must be >= 0 and finite");
        return LS_ERR_ARG;
    }
    if ((rc = check_workspace(*G, workspace, ws_bytes)) != LS_OK) return rc;
    size_t lds = 0;
    return make_step_geom<S>(*G, sg, &lds);
}

// The cut-off of Eq. 8 for a step call: off (the plain step) unless `on`.
template <class C>
struct CutOff {
    bool on = false;
    C beta = C(0), gamma = C(0);
};

template <class C>
static int check_cutoff(const CutOff<C> &cut) {
    if (cut.on && !(cut.beta > C(0) && cut.beta < cut.gamma && cut.gamma < C(INFINITY))) {
        set_error("cut-off: need 0 < beta < gamma < inf");
        return LS_ERR_ARG;
    }
    return LS_OK;
}

// What every launch sequence on the plan held by the workspace (the update
// map, the work-item records and their count) shares: the kernel's row counts
// and LDS size, whether the buffers allow the vectorised kernels, and the
// arguments of every mode (the cut-off fields zero).
template <class S, class FT>
struct StepLaunch {
    int nown, nhalo;
    size_t lds;
    int threads;
    bool aligned;
    StepArgs<S, FT> args;
};

template <class S, class FT>
static StepLaunch<S, FT> step_launch(S *phi, const FT *F, typename Codec<S>::C scale,
                                     const Geom &G, const StepGeom &sg, typename Codec<S>::C dx,
                                     typename Codec<S>::C dt, S *scratch, uint8_t *ws) {
    using C = typename Codec<S>::C;
    const Workspace w = workspace_layout(G);
    StepLaunch<S, FT> L;
    const int rp = kBlock / sg.xl;
    L.nown = pow2_at_least((G.ty * G.tz + rp - 1) / rp);
    L.nhalo = pow2_at_least((2 * (G.ty + G.tz) + rp - 1) / rp);
    L.lds = static_cast<size_t>(sg.sx) * sg.sy * (G.tz + 2) * sizeof(C);
    L.threads = kBlock;
    L.aligned = reinterpret_cast<uintptr_t>(phi) % 16 == 0 &&
                reinterpret_cast<uintptr_t>(scratch) % 16 == 0 &&
                reinterpret_cast<uintptr_t>(F) % 16 == 0;
    StepArgs<S, FT> &a = L.args;
    a.F = F;
    a.rec = reinterpret_cast<int32_t *>(ws + w.items);
    a.nitems = reinterpret_cast<int32_t *>(ws + w.counters);
    a.range = nullptr;
    a.inst = nullptr;
    a.umap = ws + w.u_map;
    a.orig = phi;
    a.dx = dx;
    a.dt = dt;
    a.dtdx = static_cast<C>(static_cast<double>(dt) / static_cast<double>(dx));
    a.scale = scale;
    a.cut_beta = C(0);
    a.cut_gamma = C(0);
    a.cut_k = C(0);
    return L;
}

// The band copied from scratch back into phi (after an odd number of launches).
template <class S, class FT>
static int copy_back(const StepGeom &sg, const StepLaunch<S, FT> &L, int nblocks, S *scratch,
                     S *phi, hipStream_t stream) {
    hipLaunchKernelGGL(band_copy_kernel<S>, dim3(nblocks), dim3(kBlock), 0, stream, sg,
                       static_cast<const S *>(scratch), phi, L.args.rec, L.args.nitems);
    LS_LAUNCH_CHECK("band_copy_kernel");
    return LS_OK;
}

// nsteps launches of the step kernel on the plan held by the workspace, then
// the copy-back of the band when nsteps is odd.  With the cut-off on, the
// kernels scale the speed by c(phi) of the centre point's step-n value.
template <class S, class FT>
static int upwind_launch(S *phi, const FT *F, typename Codec<S>::C scale, const Geom &G,
                         const StepGeom &sg, typename Codec<S>::C dx, typename Codec<S>::C dt,
                         int nsteps, S *scratch, uint8_t *ws, hipStream_t stream,
                         bool land_in_scratch = false,
                         const CutOff<typename Codec<S>::C> &cut = {}) {
    using C = typename Codec<S>::C;
    constexpr bool EXACT = sizeof(C) == 8;
    if (nsteps == 0) return LS_OK;
    StepLaunch<S, FT> L = step_launch<S, FT>(phi, F, scale, G, sg, dx, dt, scratch, ws);
    auto kernel = cut.on ? select_upwind_kernel<S, FT, EXACT, kCutoff>(
                               sg, L.nown, L.nhalo, &L.lds, &L.threads, L.aligned)
                         : select_upwind_kernel<S, FT, EXACT, kPlain>(
                               sg, L.nown, L.nhalo, &L.lds, &L.threads, L.aligned);
    int nblocks = 0;
    int rc;
    if ((rc = persistent_grid(kernel, L.threads, L.lds, &nblocks, nullptr, G.ntiles)) != LS_OK)
        return rc;
    StepArgs<S, FT> &args = L.args;
    if (cut.on) {
        args.cut_beta = cut.beta;
        args.cut_gamma = cut.gamma;
        // from the arguments' values, in FP64: (gamma - beta)^3 for the exact
        // form, 1 / (gamma - beta) for the fast form
        const double d = static_cast<double>(cut.gamma) - static_cast<double>(cut.beta);
        args.cut_k = EXACT ? static_cast<C>(std::pow(d, 3.0)) : static_cast<C>(1.0 / d);
    }
    // pairs of steps in one launch where the two-step kernel applies, then a
    // single step if one is left; one pair of timing events around them all
    size_t lds2 = 0;
    int threads2 = 0, nblocks2 = 0;
    auto kernel2 = cut.on ? nullptr : select_upwind2_kernel<S, FT, EXACT>(sg, L.aligned, &lds2,
                                                                          &threads2);
    const int pairs = (kernel2 && nsteps >= 2 && !land_in_scratch) ? nsteps / 2 : 0;
    const int singles = nsteps - 2 * pairs;
    const int launches = pairs + singles;
    if (pairs &&
        (rc = persistent_grid(kernel2, threads2, lds2, &nblocks2, nullptr, G.ntiles)) != LS_OK)
        return rc;
    int64_t slot;
    if ((rc = stats_before(LS_KERNEL_UPWIND, stream, &slot, launches)) != LS_OK) return rc;
    for (int l = 0; l < launches; ++l) {
        args.cur = (l & 1) ? scratch : phi;
        args.nxt = (l & 1) ? phi : scratch;
        if (l < pairs) {
            hipLaunchKernelGGL(kernel2, dim3(nblocks2), dim3(threads2), lds2, stream, sg, args);
            LS_LAUNCH_CHECK("upwind_vec2_kernel");
        } else {
            hipLaunchKernelGGL(kernel, dim3(nblocks), dim3(L.threads), L.lds, stream, sg, args);
            LS_LAUNCH_CHECK("upwind_kernel");
        }
    }
    if ((rc = stats_after(LS_KERNEL_UPWIND, stream, slot)) != LS_OK) return rc;
    if ((launches & 1) && !land_in_scratch) return copy_back(sg, L, nblocks, scratch, phi, stream);
    return LS_OK;
}

// Step 3 of the algorithm in Sec. 1.1 on the plan held by the workspace:
// niter reinitialisation steps (Eq. 12-13, pseudo-time step dtau) on the band,
// the last one followed by the clamp of Eq. 10 to [-gamma, gamma] when clamp
// is set; ping-pong as in upwind_launch, the band copied back into phi when
// niter is odd.  The kernels read no F.
template <class S, class FT>
static int reinit_launch(S *phi, typename Codec<S>::C scale, const Geom &G, const StepGeom &sg,
                         typename Codec<S>::C dx, typename Codec<S>::C dtau,
                         typename Codec<S>::C gamma, bool clamp, int niter, S *scratch,
                         uint8_t *ws, hipStream_t stream) {
    using C = typename Codec<S>::C;
    constexpr bool EXACT = sizeof(C) == 8;
    if (niter == 0) return LS_OK;
    StepLaunch<S, FT> L =
        step_launch<S, FT>(phi, static_cast<const FT *>(nullptr), scale, G, sg, dx, dtau, scratch,
                           ws);
    auto kernel = select_upwind_kernel<S, FT, EXACT, kReinit>(sg, L.nown, L.nhalo, &L.lds,
                                                              &L.threads, L.aligned);
    auto last = clamp ? select_upwind_kernel<S, FT, EXACT, kReinitClamp>(
                            sg, L.nown, L.nhalo, &L.lds, &L.threads, L.aligned)
                      : kernel;
    int nblocks = 0;
    int rc;
    if ((rc = persistent_grid(kernel, L.threads, L.lds, &nblocks, nullptr, G.ntiles)) != LS_OK)
        return rc;
    StepArgs<S, FT> &args = L.args;
    args.cut_gamma = gamma;
    int64_t slot;
    if ((rc = stats_before(LS_KERNEL_REINIT, stream, &slot, niter)) != LS_OK) return rc;
    for (int l = 0; l < niter; ++l) {
        args.cur = (l & 1) ? scratch : phi;
        args.nxt = (l & 1) ? phi : scratch;
        hipLaunchKernelGGL(l == niter - 1 ? last : kernel, dim3(nblocks), dim3(L.threads), L.lds,
                           stream, sg, args);
        LS_LAUNCH_CHECK("upwind_kernel (reinit)");
    }
    if ((rc = stats_after(LS_KERNEL_REINIT, stream, slot)) != LS_OK) return rc;
    if (niter & 1) return copy_back(sg, L, nblocks, scratch, phi, stream);
    return LS_OK;
}

int fill_zero(uint8_t *p, int64_t bytes, hipStream_t stream);  // ls_band.hip

// One FP32 step of the plan the workspace holds (the band of the last build),
// from phi into out: the band points of out get the step, the other points of
// out are not written (the caller keeps them equal to phi).
int plan_step_to_f32(const float *phi, float *out, const float *F, const Geom &G, float dx,
                     float dt, uint8_t *ws, hipStream_t stream) {
    StepGeom sg;
    size_t lds = 0;
    int rc = make_step_geom<float>(G, &sg, &lds);
    if (rc != LS_OK) return rc;
    return upwind_launch<float, float>(const_cast<float *>(phi), F, 1.0f, G, sg, dx, dt, 1, out,
                                       ws, stream, true);
}

// The step plan of a caller's band list: its membership map, then the work
// items, in the workspace.
static int plan_list(const Geom &G, uint8_t *ws, const int32_t *tiles, const int32_t *ntiles_dev,
                     hipStream_t stream) {
    const Workspace w = workspace_layout(G);
    uint8_t *umap = ws + w.u_map;
    int rc;
    if ((rc = fill_zero(umap, G.ntiles, stream)) != LS_OK) return rc;
    const unsigned set_blocks =
        static_cast<unsigned>(std::min<int64_t>(cdiv64(G.ntiles, kBlock), 4096));
    hipLaunchKernelGGL(map_set_kernel, dim3(set_blocks), dim3(kBlock), 0, stream, umap, tiles,
                       ntiles_dev, static_cast<int>(G.ntiles));
    LS_LAUNCH_CHECK("map_set_kernel");
    return build_plan(G, ws, nullptr, nullptr, stream);
}

template <class S, class FT>
static int upwind_step(S *phi, const FT *F, typename Codec<S>::C scale, const ls_grid *grid,
                       typename Codec<S>::C dx, typename Codec<S>::C dt, const int32_t *tiles,
                       const int32_t *ntiles_dev, int nsteps, S *scratch, void *workspace,
                       int64_t ws_bytes, hipStream_t stream,
                       const CutOff<typename Codec<S>::C> &cut = {}) {
    Geom G;
    StepGeom sg;
    int rc = step_args<S, FT>(phi, F, grid, dx, dt, nsteps, scratch, workspace, ws_bytes, &G, &sg);
    if (rc != LS_OK) return rc;
    if ((rc = check_cutoff(cut)) != LS_OK) return rc;
    if (!tiles || !ntiles_dev) {
        set_error("step: tiles and ntiles_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (nsteps == 0) return LS_OK;
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    if ((rc = plan_list(G, ws, tiles, ntiles_dev, stream)) != LS_OK) return rc;
    return upwind_launch<S, FT>(phi, F, scale, G, sg, dx, dt, nsteps, scratch, ws, stream, false,
                                cut);
}

// niter reinitialisation steps (Eq. 12-13) on the listed tiles, optionally
// followed by the clamp of Eq. 10.
template <class S, class FT>
static int reinit_step(S *phi, typename Codec<S>::C scale, const ls_grid *grid,
                       typename Codec<S>::C dx, typename Codec<S>::C dtau,
                       typename Codec<S>::C gamma, int clamp, const int32_t *tiles,
                       const int32_t *ntiles_dev, int niter, S *scratch, void *workspace,
                       int64_t ws_bytes, hipStream_t stream) {
    using C = typename Codec<S>::C;
    Geom G;
    StepGeom sg;
    int rc = step_args<S, FT>(phi, nullptr, grid, dx, dtau, niter, scratch, workspace, ws_bytes,
                              &G, &sg, false);
    if (rc != LS_OK) return rc;
    if (clamp != 0 && clamp != 1) {
        set_error("reinit: clamp must be 0 or 1");
        return LS_ERR_ARG;
    }
    if (clamp && !(gamma > C(0) && gamma < C(INFINITY))) {
        set_error("reinit: gamma must be positive and finite");
        return LS_ERR_ARG;
    }
    if (!tiles || !ntiles_dev) {
        set_error("reinit: tiles and ntiles_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (niter == 0) return LS_OK;
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    if ((rc = plan_list(G, ws, tiles, ntiles_dev, stream)) != LS_OK) return rc;
    return reinit_launch<S, FT>(phi, scale, G, sg, dx, dtau, gamma, clamp != 0, niter, scratch,
                                ws, stream);
}

template <class S, class FT>
static int launch_info(const ls_grid *grid, int32_t *blocks, int32_t *lds_bytes,
                       int32_t *run_tiles, int32_t *limit) {
    using C = typename Codec<S>::C;
    constexpr bool EXACT = sizeof(C) == 8;
    Geom G;
    int rc = make_geom(grid, &G);
    if (rc != LS_OK) return rc;
    G.elem_bytes = static_cast<int32_t>(sizeof(S));
    StepGeom sg;
    size_t lds = 0;
    if ((rc = make_step_geom<S>(G, &sg, &lds)) != LS_OK) return rc;
    const int rp = kBlock / sg.xl;
    const int nown = pow2_at_least((G.ty * G.tz + rp - 1) / rp);
    const int nhalo = pow2_at_least((2 * (G.ty + G.tz) + rp - 1) / rp);
    int threads = kBlock;
    auto kernel = select_upwind_kernel<S, FT, EXACT>(sg, nown, nhalo, &lds, &threads, true);
    int nb = 0, lim = 0;
    if ((rc = persistent_grid(kernel, threads, lds, &nb, &lim, G.ntiles)) != LS_OK) return rc;
    if (blocks) *blocks = nb;
    if (lds_bytes) *lds_bytes = static_cast<int32_t>(lds);
    if (run_tiles) *run_tiles = sg.R;
    if (limit) *limit = lim;
    return LS_OK;
}

// The windowed driver: a full band build for the first window, then an exact
// incremental rebuild from the previous window's band (every point outside
// that band is unchanged, so no tile outside it can join the tube); each
// build leaves the step plan in the workspace, so the steps need no
// preparation of their own.  The band lists alternate between the caller's
// buffer and the workspace so that the last one lands in `tiles`.  With the
// cut-off on (Eq. 8) its gamma is the band's.
template <class S, class FT>
static int band_run(S *phi, const FT *F, typename Codec<S>::C scale, const ls_grid *grid,
                    typename Codec<S>::C dx, typename Codec<S>::C dt, typename Codec<S>::C gamma,
                    int nsteps, int window, int32_t *tiles, int64_t capacity,
                    int32_t *ntiles_dev, int64_t *tile_steps_dev, S *scratch, void *workspace,
                    int64_t ws_bytes, void *stream_, const CutOff<typename Codec<S>::C> &cut = {},
                    int reinit_iters = 0, typename Codec<S>::C dtau = 0) {
    if (window <= 0) {
        set_error("band run: window must be positive (got %d)", window);
        return LS_ERR_ARG;
    }
    Geom G;
    StepGeom sg;
    int rc = step_args<S, FT>(phi, F, grid, dx, dt, nsteps, scratch, workspace, ws_bytes, &G, &sg);
    if (rc != LS_OK) return rc;
    if (!tiles || !ntiles_dev) {
        set_error("band run: tiles and ntiles_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (!(gamma == gamma)) {
        set_error("band run: gamma is NaN");
        return LS_ERR_ARG;
    }
    if ((rc = check_cutoff(cut)) != LS_OK) return rc;
    if (reinit_iters < 0 || !(dtau >= 0) || !(dtau < INFINITY)) {
        set_error("band run: reinit_iters must be >= 0 and dtau >= 0 and finite");
        return LS_ERR_ARG;
    }
    if (capacity < G.ntiles) {
        set_error("band run: capacity %lld < %lld tiles", (long long)capacity,
                  (long long)G.ntiles);
        return LS_ERR_CAPACITY;
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const Workspace w = workspace_layout(G);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    int32_t *lists[2] = {tiles, reinterpret_cast<int32_t *>(ws + w.prev_list)};
    int32_t *counts[2] = {ntiles_dev, reinterpret_cast<int32_t *>(ws + w.counters) + 1};
    const int nwin = (nsteps + window - 1) / window;
    for (int k = 0; k < nwin; ++k) {
        const int n = std::min(window, nsteps - k * window);
        const int cur = (nwin - 1 - k) & 1;  // the last window writes lists[0]
        const TileAccum acc{tile_steps_dev, n};  // band tiles x steps, counted by the build
        if (k == 0)
            rc = band_build<S>(phi, scale, grid, gamma, 1, lists[cur], capacity, counts[cur],
                               workspace, ws_bytes, stream_, acc);
        else
            rc = band_rebuild<S>(phi, scale, grid, gamma, lists[cur ^ 1], counts[cur ^ 1],
                                 lists[cur], capacity, counts[cur], workspace, ws_bytes, stream_,
                                 true, acc);
        if (rc != LS_OK) return rc;
        rc = upwind_launch<S, FT>(phi, F, scale, G, sg, dx, dt, n, scratch, ws, stream, false,
                                  cut);
        if (rc != LS_OK) return rc;
        // Step 3: reinitialisation on the same band, then the clamp to the band's gamma
        rc = reinit_launch<S, FT>(phi, scale, G, sg, dx, dtau, gamma, true, reinit_iters, scratch,
                                  ws, stream);
        if (rc != LS_OK) return rc;
    }
    return LS_OK;
}

}  // namespace ls

extern "C" {

int ls_set_tuning(const ls_tuning *t) {
    ls::clear_error();
    if (!t || t->run_width < 0 || t->blocks_per_cu < 0 || t->blocks_per_cu > 64 ||
        t->pipeline < 0 || t->pipeline > 2 || t->vector < 0 || t->vector > 1 ||
        t->temporal < 0 || t->temporal > 2) {
        ls::set_error("tuning: NULL or out-of-range field");
        return LS_ERR_ARG;
    }
    ls::g_tuning = *t;
    return LS_OK;
}

int ls_get_tuning(ls_tuning *t) {
    ls::clear_error();
    if (!t) {
        ls::set_error("tuning: NULL output");
        return LS_ERR_ARG;
    }
    t->run_width = ls::run_width();
    t->blocks_per_cu = ls::g_tuning.blocks_per_cu;
    t->pipeline = ls::g_tuning.pipeline;
    t->vector = ls::g_tuning.vector;
    t->temporal = ls::g_tuning.temporal;
    return LS_OK;
}

int ls_upwind_launch_info(const ls_grid *g, int precision, int32_t *blocks, int32_t *lds_bytes,
                          int32_t *run_tiles, int32_t *blocks_per_cu_limit) {
    ls::clear_error();
    switch (precision) {
    case 0: return ls::launch_info<float, float>(g, blocks, lds_bytes, run_tiles, blocks_per_cu_limit);
    case 1: return ls::launch_info<double, double>(g, blocks, lds_bytes, run_tiles, blocks_per_cu_limit);
    case 2: return ls::launch_info<uint16_t, float>(g, blocks, lds_bytes, run_tiles, blocks_per_cu_limit);
    default: ls::set_error("launch info: precision must be 0, 1 or 2"); return LS_ERR_ARG;
    }
}

int ls_upwind_step_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                       const int32_t *tiles, const int32_t *ntiles_dev, int nsteps,
                       float *scratch, void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::upwind_step<float, float>(phi, F, 1.0f, g, dx, dt, tiles, ntiles_dev, nsteps,
                                         scratch, workspace, workspace_bytes,
                                         static_cast<hipStream_t>(stream));
}

int ls_upwind_step_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                       const int32_t *tiles, const int32_t *ntiles_dev, int nsteps,
                       double *scratch, void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::upwind_step<double, double>(phi, F, 1.0, g, dx, dt, tiles, ntiles_dev, nsteps,
                                           scratch, workspace, workspace_bytes,
                                           static_cast<hipStream_t>(stream));
}

int ls_upwind_step_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g,
                        float dx, float dt, const int32_t *tiles, const int32_t *ntiles_dev,
                        int nsteps, uint16_t *scratch, void *workspace, int64_t workspace_bytes,
                        void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("step f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::upwind_step<uint16_t, float>(phi_h, F, scale, g, dx, dt, tiles, ntiles_dev, nsteps,
                                            scratch, workspace, workspace_bytes,
                                            static_cast<hipStream_t>(stream));
}

int ls_band_run_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt, float gamma,
                    int nsteps, int window, int32_t *tiles, int64_t capacity,
                    int32_t *ntiles_dev, int64_t *tile_steps_dev, float *scratch,
                    void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_run<float, float>(phi, F, 1.0f, g, dx, dt, gamma, nsteps, window, tiles,
                                      capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                      workspace_bytes, stream);
}

int ls_band_run_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                    double gamma, int nsteps, int window, int32_t *tiles, int64_t capacity,
                    int32_t *ntiles_dev, int64_t *tile_steps_dev, double *scratch,
                    void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_run<double, double>(phi, F, 1.0, g, dx, dt, gamma, nsteps, window, tiles,
                                        capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                        workspace_bytes, stream);
}

int ls_band_run_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g, float dx,
                     float dt, float gamma, int nsteps, int window, int32_t *tiles,
                     int64_t capacity, int32_t *ntiles_dev, int64_t *tile_steps_dev,
                     uint16_t *scratch, void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("band run f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::band_run<uint16_t, float>(phi_h, F, scale, g, dx, dt, gamma, nsteps, window, tiles,
                                         capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                         workspace_bytes, stream);
}

int ls_upwind_step_cutoff_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                              float beta, float gamma, const int32_t *tiles,
                              const int32_t *ntiles_dev, int nsteps, float *scratch,
                              void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::upwind_step<float, float>(phi, F, 1.0f, g, dx, dt, tiles, ntiles_dev, nsteps,
                                         scratch, workspace, workspace_bytes,
                                         static_cast<hipStream_t>(stream), {true, beta, gamma});
}

int ls_upwind_step_cutoff_f64(double *phi, const double *F, const ls_grid *g, double dx,
                              double dt, double beta, double gamma, const int32_t *tiles,
                              const int32_t *ntiles_dev, int nsteps, double *scratch,
                              void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::upwind_step<double, double>(phi, F, 1.0, g, dx, dt, tiles, ntiles_dev, nsteps,
                                           scratch, workspace, workspace_bytes,
                                           static_cast<hipStream_t>(stream), {true, beta, gamma});
}

int ls_upwind_step_cutoff_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g,
                               float dx, float dt, float beta, float gamma,
                               const int32_t *tiles, const int32_t *ntiles_dev, int nsteps,
                               uint16_t *scratch, void *workspace, int64_t workspace_bytes,
                               void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("step f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::upwind_step<uint16_t, float>(phi_h, F, scale, g, dx, dt, tiles, ntiles_dev, nsteps,
                                            scratch, workspace, workspace_bytes,
                                            static_cast<hipStream_t>(stream), {true, beta, gamma});
}

int ls_band_run_cutoff_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                           float beta, float gamma, int nsteps, int window, int32_t *tiles,
                           int64_t capacity, int32_t *ntiles_dev, int64_t *tile_steps_dev,
                           float *scratch, void *workspace, int64_t workspace_bytes,
                           void *stream) {
    ls::clear_error();
    return ls::band_run<float, float>(phi, F, 1.0f, g, dx, dt, gamma, nsteps, window, tiles,
                                      capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                      workspace_bytes, stream, {true, beta, gamma});
}

int ls_band_run_cutoff_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                           double beta, double gamma, int nsteps, int window, int32_t *tiles,
                           int64_t capacity, int32_t *ntiles_dev, int64_t *tile_steps_dev,
                           double *scratch, void *workspace, int64_t workspace_bytes,
                           void *stream) {
    ls::clear_error();
    return ls::band_run<double, double>(phi, F, 1.0, g, dx, dt, gamma, nsteps, window, tiles,
                                        capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                        workspace_bytes, stream, {true, beta, gamma});
}

int ls_band_run_cutoff_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g,
                            float dx, float dt, float beta, float gamma, int nsteps, int window,
                            int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                            int64_t *tile_steps_dev, uint16_t *scratch, void *workspace,
                            int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("band run f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::band_run<uint16_t, float>(phi_h, F, scale, g, dx, dt, gamma, nsteps, window, tiles,
                                         capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                         workspace_bytes, stream, {true, beta, gamma});
}

int ls_reinit_step_f32(float *phi, const ls_grid *g, float dx, float dtau, float gamma, int clamp,
                       const int32_t *tiles, const int32_t *ntiles_dev, int niter,
                       float *scratch, void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::reinit_step<float, float>(phi, 1.0f, g, dx, dtau, gamma, clamp, tiles, ntiles_dev,
                                         niter, scratch, workspace, workspace_bytes,
                                         static_cast<hipStream_t>(stream));
}

int ls_reinit_step_f64(double *phi, const ls_grid *g, double dx, double dtau, double gamma,
                       int clamp, const int32_t *tiles, const int32_t *ntiles_dev, int niter,
                       double *scratch, void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::reinit_step<double, double>(phi, 1.0, g, dx, dtau, gamma, clamp, tiles, ntiles_dev,
                                           niter, scratch, workspace, workspace_bytes,
                                           static_cast<hipStream_t>(stream));
}

int ls_reinit_step_f16s(uint16_t *phi_h, float scale, const ls_grid *g, float dx, float dtau,
                        float gamma, int clamp, const int32_t *tiles, const int32_t *ntiles_dev,
                        int niter, uint16_t *scratch, void *workspace, int64_t workspace_bytes,
                        void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("reinit f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::reinit_step<uint16_t, float>(phi_h, scale, g, dx, dtau, gamma, clamp, tiles,
                                            ntiles_dev, niter, scratch, workspace,
                                            workspace_bytes, static_cast<hipStream_t>(stream));
}

int ls_band_run_reinit_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                           float beta, float gamma, float dtau, int reinit_iters, int nsteps,
                           int window, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                           int64_t *tile_steps_dev, float *scratch, void *workspace,
                           int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_run<float, float>(phi, F, 1.0f, g, dx, dt, gamma, nsteps, window, tiles,
                                      capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                      workspace_bytes, stream, {true, beta, gamma}, reinit_iters,
                                      dtau);
}

int ls_band_run_reinit_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                           double beta, double gamma, double dtau, int reinit_iters, int nsteps,
                           int window, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                           int64_t *tile_steps_dev, double *scratch, void *workspace,
                           int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_run<double, double>(phi, F, 1.0, g, dx, dt, gamma, nsteps, window, tiles,
                                        capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                        workspace_bytes, stream, {true, beta, gamma},
                                        reinit_iters, dtau);
}

int ls_band_run_reinit_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g,
                            float dx, float dt, float beta, float gamma, float dtau,
                            int reinit_iters, int nsteps, int window, int32_t *tiles,
                            int64_t capacity, int32_t *ntiles_dev, int64_t *tile_steps_dev,
                            uint16_t *scratch, void *workspace, int64_t workspace_bytes,
                            void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("band run f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::band_run<uint16_t, float>(phi_h, F, scale, g, dx, dt, gamma, nsteps, window, tiles,
                                         capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                                         workspace_bytes, stream, {true, beta, gamma},
                                         reinit_iters, dtau);
}

}  // extern "C"
