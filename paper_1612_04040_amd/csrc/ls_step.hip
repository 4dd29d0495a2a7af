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
#include <cmath>

#include "ls_compact.h"
#include "ls_stats.h"

namespace ls {

constexpr int kMaxOwn = 16;   // grid points owned by one thread per item
constexpr int kMaxHalo = 8;   // y/z halo points loaded by one thread per item
constexpr int kMaxRun = 32;   // tiles per work item (4*kMaxRun + 2 <= kBlock)

struct StepGeom {
    int nx, ny, nz;
    int tx, ty, tz;
    int ntx, nty, ntz;
    int ntiles;  // tiles of the grid (the list capacity)
    int R;       // tiles per work item (x-run length cap)
    int xl;      // threads per grid row (power of two >= R*tx)
    int xl_log;  // log2(xl)
    int sx, sy;  // LDS box strides: sx = R*tx + 2, sy = ty + 2
};

// Fast form (f32, f16s): unscaled differences, dt/dx folded into one factor.
// Exact form (f64): the definition term by term (D = difference / dx, the
// squares summed x, then y, then z), no contraction.
template <class C, bool EXACT>
__device__ inline C upwind_point(C c, C xm, C xp, C ym, C yp, C zm, C zp, C f, C dx, C dt,
                                 C dtdx) {
    if constexpr (EXACT) {
#pragma clang fp contract(off)
        const C dmx = (c - xm) / dx, dpx = (xp - c) / dx;
        const C dmy = (c - ym) / dx, dpy = (yp - c) / dx;
        const C dmz = (c - zm) / dx, dpz = (zp - c) / dx;
        const C zero = C(0);
        auto mx = [](C a, C b) { return a > b ? a : b; };
        auto mn = [](C a, C b) { return a < b ? a : b; };
        if (f > zero) {
            const C px = mx(dmx, zero) * mx(dmx, zero) + mn(dpx, zero) * mn(dpx, zero);
            const C py = mx(dmy, zero) * mx(dmy, zero) + mn(dpy, zero) * mn(dpy, zero);
            const C pz = mx(dmz, zero) * mx(dmz, zero) + mn(dpz, zero) * mn(dpz, zero);
            const C g = sqrt((px + py) + pz);
            return c - dt * f * g;
        } else {
            const C qx = mx(dpx, zero) * mx(dpx, zero) + mn(dmx, zero) * mn(dmx, zero);
            const C qy = mx(dpy, zero) * mx(dpy, zero) + mn(dmy, zero) * mn(dmy, zero);
            const C qz = mx(dpz, zero) * mx(dpz, zero) + mn(dmz, zero) * mn(dmz, zero);
            const C g = sqrt((qx + qy) + qz);
            return c - dt * f * g;
        }
    } else {
        const bool pos = f > C(0);
        const C ax = c - xm, bx = xp - c;
        const C ay = c - ym, by = yp - c;
        const C az = c - zm, bz = zp - c;
        // upwind pair: F > 0 takes (max(D-,0), min(D+,0)); F < 0 (max(D+,0), min(D-,0))
        const C px = fmaxf(pos ? ax : bx, 0.f), qx = fminf(pos ? bx : ax, 0.f);
        const C py = fmaxf(pos ? ay : by, 0.f), qy = fminf(pos ? by : ay, 0.f);
        const C pz = fmaxf(pos ? az : bz, 0.f), qz = fminf(pos ? bz : az, 0.f);
        const C s = px * px + qx * qx + py * py + qy * qy + pz * pz + qz * qz;
        return c - (dtdx * f) * __builtin_amdgcn_sqrtf(s);
    }
}

template <class S, class FT>
struct StepArgs {
    const S *cur;
    const S *orig;
    S *nxt;
    const FT *F;
    const int32_t *rec;     // work-item records, kItemWords int32 each
    const int32_t *nitems;  // number of records (device)
    typename Codec<S>::C dx, dt, dtdx, scale;
};

// Work-item record: [0] first tile id, [1] run length (tiles), [2..5] bit l =
// "tile l of the run has its y-, y+, z-, z+ face neighbour in the band (or
// outside the grid)", [6] bit 0 / bit 1 = same for the x- / x+ neighbour.
struct EmitItem {
    int32_t *rec;
    const int32_t *tiles;
    const int32_t *ntiles_dev;
    const uint8_t *umap;
    int ntx, nty, ntz, R, cap;
    __device__ void operator()(int pos, int64_t p) const {
        const int n = min(*ntiles_dev, cap);
        const int t0 = tiles[p];
        const int ti0 = t0 % ntx;
        const int r = t0 / ntx;
        const int tj = r % nty, tk = r / nty;
        int len = 1;
        while (len < R && p + len < n && ti0 + len < ntx && tiles[p + len] == t0 + len &&
               (ti0 + len) % R != 0)
            ++len;
        uint32_t m[4] = {0, 0, 0, 0};
        for (int l = 0; l < len; ++l) {
            const int t = t0 + l;
            m[0] |= uint32_t(tj == 0 || umap[t - ntx]) << l;
            m[1] |= uint32_t(tj == nty - 1 || umap[t + ntx]) << l;
            m[2] |= uint32_t(tk == 0 || umap[t - ntx * nty]) << l;
            m[3] |= uint32_t(tk == ntz - 1 || umap[t + ntx * nty]) << l;
        }
        const uint32_t xb = uint32_t(ti0 == 0 || umap[t0 - 1]) |
                            (uint32_t(ti0 + len == ntx || umap[t0 + len]) << 1);
        int32_t *o = rec + static_cast<int64_t>(pos) * kItemWords;
        o[0] = t0;
        o[1] = len;
        o[2] = static_cast<int32_t>(m[0]);
        o[3] = static_cast<int32_t>(m[1]);
        o[4] = static_cast<int32_t>(m[2]);
        o[5] = static_cast<int32_t>(m[3]);
        o[6] = static_cast<int32_t>(xb);
        o[7] = 0;
    }
};

// Slice of the item list of this block: contiguous, XCD-aware.
__device__ inline void block_slice(int nitems, int *w0, int *w1) {
    const int G = gridDim.x;
    const int b = blockIdx.x;
    const int cb = (b & 7) * (G >> 3) + (b >> 3);
    const int per = (nitems + G - 1) / G;
    *w0 = min(cb * per, nitems);
    *w1 = min(*w0 + per, nitems);
}

// One persistent block walks its slice of work items.  Per item:
//  (1) every thread issues the global loads of its own grid points (phi and
//      F, NOWN rows of the item), of its halo-row points (NHALO rows of the
//      y- and z-faces) and of at most two x-face points, all into registers;
//  (2) the values go to the LDS box; (3) after a barrier every thread
//      evaluates its own points from the box and stores them.
// Thread t owns column lx = t mod xl of rows lr + q*rp (rows enumerate (y, z)
// of a full tile, y fastest), so its row offsets are fixed for the launch.
constexpr int cpow2(int v) { return v <= 1 ? 1 : 2 * cpow2((v + 1) / 2); }
constexpr int clog2(int v) { return v <= 1 ? 0 : 1 + clog2(v / 2); }

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

template <class S, class FT, bool EXACT, int NOWN, int NHALO, class SH>
__global__ __launch_bounds__(kBlock) void upwind_kernel(StepGeom g, StepArgs<S, FT> a) {
    using C = typename Codec<S>::C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *box = reinterpret_cast<C *>(smem);

    const int nitems = *a.nitems;
    int w0, w1;
    block_slice(nitems, &w0, &w1);

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
        const FT *Fb = a.F + base;
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
                fv[q] = Fb[o];
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
                const C c = box[o];
                const C f = static_cast<C>(fv[q]);
                S out = raw[q];
                if (f != C(0)) {
                    const C v = upwind_point<C, EXACT>(c, box[o - 1], box[o + 1], box[o - sx],
                                                       box[o + sx], box[o - sxy], box[o + sxy], f,
                                                       a.dx, a.dt, a.dtdx);
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
    block_slice(nitems, &w0, &w1);
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

__global__ __launch_bounds__(kBlock) void fill_u8_kernel(uint8_t *p, int64_t n16) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n16;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        reinterpret_cast<uint4 *>(p)[i] = make_uint4(0, 0, 0, 0);
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

// A band-list position starts a work item if its tile does not continue the
// x-run of the previous entry, or sits on a multiple-of-R tile column.
struct HeadPred {
    const int32_t *tiles;
    int ntx, R;
    __device__ bool operator()(int64_t p) const {
        const int t = tiles[p];
        if (p == 0) return true;
        if ((t % ntx) % R == 0) return true;
        return tiles[p - 1] != t - 1;
    }
};

// ---------------------------------------------------------------------------
// host side

struct Tuning {
    int run_width;  // target item width in grid points (R = run_width / tx)
};

static Tuning g_tuning = {32};

template <class S>
static int make_step_geom(const Geom &G, StepGeom *out, size_t *lds) {
    StepGeom s;
    s.nx = G.nx, s.ny = G.ny, s.nz = G.nz;
    s.tx = G.tx, s.ty = G.ty, s.tz = G.tz;
    s.ntx = G.ntx, s.nty = G.nty, s.ntz = G.ntz;
    s.ntiles = static_cast<int>(G.ntiles);
    s.R = std::max(1, std::min(kMaxRun, g_tuning.run_width / G.tx));
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

template <class S, class FT, bool EXACT, int NOWN>
static UpwindFn<S, FT, EXACT> select_halo(int nhalo) {
    switch (nhalo) {
    case 1: return upwind_kernel<S, FT, EXACT, NOWN, 1, DynShape>;
    case 2: return upwind_kernel<S, FT, EXACT, NOWN, 2, DynShape>;
    case 4: return upwind_kernel<S, FT, EXACT, NOWN, 4, DynShape>;
    default: return upwind_kernel<S, FT, EXACT, NOWN, 8, DynShape>;
    }
}

// Kernel for a launch: a compile-time specialisation for the common tile
// shapes and run lengths, else the run-time-shape kernel.
template <class S, class FT, bool EXACT>
static UpwindFn<S, FT, EXACT> select_upwind_kernel(const StepGeom &sg, int nown, int nhalo) {
    if (sg.tx == 8 && sg.ty == 8 && sg.tz == 8 && sg.R == 4)
        return upwind_kernel<S, FT, EXACT, 8, 4, Shape<8, 8, 8, 4>>;
    if (sg.tx == 8 && sg.ty == 8 && sg.tz == 8 && sg.R == 8)
        return upwind_kernel<S, FT, EXACT, 16, 8, Shape<8, 8, 8, 8>>;
    switch (nown) {
    case 1: return select_halo<S, FT, EXACT, 1>(nhalo);
    case 2: return select_halo<S, FT, EXACT, 2>(nhalo);
    case 4: return select_halo<S, FT, EXACT, 4>(nhalo);
    case 8: return select_halo<S, FT, EXACT, 8>(nhalo);
    default: return select_halo<S, FT, EXACT, 16>(nhalo);
    }
}

template <class K>
static int persistent_grid(K kernel, size_t lds, int *grid) {
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != LS_OK) return rc;
    int per_cu = 0;
    LS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, lds));
    if (per_cu < 1) per_cu = 1;
    int G = di.cus * per_cu;
    G = std::max(8, G - G % 8);
    *grid = G;
    return LS_OK;
}

template <class S, class FT>
static int upwind_step(S *phi, const FT *F, typename Codec<S>::C scale, const ls_grid *grid,
                       typename Codec<S>::C dx, typename Codec<S>::C dt, const int32_t *tiles,
                       const int32_t *ntiles_dev, int nsteps, S *scratch, void *workspace,
                       int64_t ws_bytes, hipStream_t stream) {
    using C = typename Codec<S>::C;
    constexpr bool EXACT = sizeof(C) == 8;
    Geom G;
    int rc = make_geom(grid, &G);
    if (rc != LS_OK) return rc;
    if (!phi || !F || !tiles || !ntiles_dev || !scratch) {
        set_error("step: phi, F, tiles, ntiles_dev and scratch must be non-NULL");
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
    if ((rc = check_workspace(G, workspace, ws_bytes)) != LS_OK) return rc;
    StepGeom sg;
    size_t lds = 0;
    if ((rc = make_step_geom<S>(G, &sg, &lds)) != LS_OK) return rc;
    if (nsteps == 0) return LS_OK;

    const Workspace w = workspace_layout(G);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    uint8_t *umap = ws + w.u_map;
    int32_t *blk = reinterpret_cast<int32_t *>(ws + w.blk_counts);
    int32_t *items = reinterpret_cast<int32_t *>(ws + w.items);
    int32_t *nitems = reinterpret_cast<int32_t *>(ws + w.counters);

    // band membership map and work items from the list
    const int64_t n16 = cdiv64(G.ntiles, 16);
    const unsigned fill_blocks = static_cast<unsigned>(std::min<int64_t>(cdiv64(n16, kBlock), 4096));
    hipLaunchKernelGGL(fill_u8_kernel, dim3(fill_blocks), dim3(kBlock), 0, stream, umap, n16);
    LS_LAUNCH_CHECK("fill_u8_kernel");
    const unsigned set_blocks =
        static_cast<unsigned>(std::min<int64_t>(cdiv64(G.ntiles, kBlock), 4096));
    hipLaunchKernelGGL(map_set_kernel, dim3(set_blocks), dim3(kBlock), 0, stream, umap, tiles,
                       ntiles_dev, static_cast<int>(G.ntiles));
    LS_LAUNCH_CHECK("map_set_kernel");
    rc = compact(HeadPred{tiles, G.ntx, sg.R},
                 EmitItem{items, tiles, ntiles_dev, umap, G.ntx, G.nty, G.ntz, sg.R,
                          static_cast<int>(G.ntiles)},
                 ntiles_dev, G.ntiles, nitems, blk, stream);
    if (rc != LS_OK) return rc;

    const int rp = kBlock / sg.xl;
    const int nown = pow2_at_least((G.ty * G.tz + rp - 1) / rp);
    const int nhalo = pow2_at_least((2 * (G.ty + G.tz) + rp - 1) / rp);
    auto kernel = select_upwind_kernel<S, FT, EXACT>(sg, nown, nhalo);
    int nblocks = 0;
    if ((rc = persistent_grid(kernel, lds, &nblocks)) != LS_OK) return rc;

    StepArgs<S, FT> args;
    args.F = F;
    args.rec = items;
    args.nitems = nitems;
    args.orig = phi;
    args.dx = dx;
    args.dt = dt;
    args.dtdx = static_cast<C>(static_cast<double>(dt) / static_cast<double>(dx));
    args.scale = scale;
    for (int s = 0; s < nsteps; ++s) {
        args.cur = (s & 1) ? scratch : phi;
        args.nxt = (s & 1) ? phi : scratch;
        int64_t slot;
        if ((rc = stats_before(LS_KERNEL_UPWIND, stream, &slot)) != LS_OK) return rc;
        hipLaunchKernelGGL(kernel, dim3(nblocks), dim3(kBlock), lds, stream, sg, args);
        LS_LAUNCH_CHECK("upwind_kernel");
        if ((rc = stats_after(LS_KERNEL_UPWIND, stream, slot)) != LS_OK) return rc;
    }
    if (nsteps & 1) {
        hipLaunchKernelGGL(band_copy_kernel<S>, dim3(nblocks), dim3(kBlock), 0, stream, sg,
                           static_cast<const S *>(scratch), phi,
                           static_cast<const int32_t *>(items),
                           static_cast<const int32_t *>(nitems));
        LS_LAUNCH_CHECK("band_copy_kernel");
    }
    return LS_OK;
}

// declared in ls_band.hip
template <class S>
int band_build(const S *phi, typename Codec<S>::C scale, const ls_grid *grid,
               typename Codec<S>::C gamma, int dilate, int32_t *tiles, int64_t capacity,
               int32_t *ntiles_dev, void *workspace, int64_t ws_bytes, void *stream_);

template <class S, class FT>
static int band_run(S *phi, const FT *F, typename Codec<S>::C scale, const ls_grid *grid,
                    typename Codec<S>::C dx, typename Codec<S>::C dt, typename Codec<S>::C gamma,
                    int nsteps, int window, int32_t *tiles, int64_t capacity,
                    int32_t *ntiles_dev, S *scratch, void *workspace, int64_t ws_bytes,
                    void *stream_) {
    if (window <= 0) {
        set_error("band run: window must be positive (got %d)", window);
        return LS_ERR_ARG;
    }
    if (nsteps < 0) {
        set_error("band run: nsteps must be >= 0 (got %d)", nsteps);
        return LS_ERR_ARG;
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    for (int done = 0; done < nsteps; done += window) {
        const int n = std::min(window, nsteps - done);
        int rc = band_build<S>(phi, scale, grid, gamma, 1, tiles, capacity, ntiles_dev, workspace,
                               ws_bytes, stream_);
        if (rc != LS_OK) return rc;
        rc = upwind_step<S, FT>(phi, F, scale, grid, dx, dt, tiles, ntiles_dev, n, scratch,
                                workspace, ws_bytes, stream);
        if (rc != LS_OK) return rc;
    }
    return LS_OK;
}

}  // namespace ls

extern "C" {

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
                    int32_t *ntiles_dev, float *scratch, void *workspace,
                    int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_run<float, float>(phi, F, 1.0f, g, dx, dt, gamma, nsteps, window, tiles,
                                      capacity, ntiles_dev, scratch, workspace, workspace_bytes,
                                      stream);
}

int ls_band_run_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                    double gamma, int nsteps, int window, int32_t *tiles, int64_t capacity,
                    int32_t *ntiles_dev, double *scratch, void *workspace,
                    int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_run<double, double>(phi, F, 1.0, g, dx, dt, gamma, nsteps, window, tiles,
                                        capacity, ntiles_dev, scratch, workspace,
                                        workspace_bytes, stream);
}

int ls_band_run_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g, float dx,
                     float dt, float gamma, int nsteps, int window, int32_t *tiles,
                     int64_t capacity, int32_t *ntiles_dev, uint16_t *scratch, void *workspace,
                     int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("band run f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::band_run<uint16_t, float>(phi_h, F, scale, g, dx, dt, gamma, nsteps, window, tiles,
                                         capacity, ntiles_dev, scratch, workspace,
                                         workspace_bytes, stream);
}

}  // extern "C"
