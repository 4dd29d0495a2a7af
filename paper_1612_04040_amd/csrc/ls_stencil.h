// The upwind stencil (Eq. 3-5) and the fast band-step kernel, shared by the
// single-grid step and the batched step.
#pragma once

#include "ls_internal.h"

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

// One grid of a batch, as the batched kernels read it (device memory).
struct BatchInst {
    int64_t offset;          // first element of the grid in phi / F / scratch
    int32_t nx, ny, nz;
    int32_t tx, ty, tz;
    int32_t ntx, nty, ntz;
    int32_t tile_base;       // first global tile id of the grid
    int32_t ntiles;
    int32_t R;               // tiles per work item
    int32_t slab_base;       // first global slab (tj, tk) of the grid
    int32_t vec_ok;          // x rows may be read as 16-byte vectors
    float dx, dt, dtdx, gamma;
    int32_t group;           // tile-shape group of the grid
    int32_t px;              // elements between consecutive x rows (>= nx)
    int32_t pad[2];
};
static_assert(sizeof(BatchInst) == 96, "BatchInst layout");

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
        const C ax = c - xm, bx = xp - c;
        const C ay = c - ym, by = yp - c;
        const C az = c - zm, bz = zp - c;
        // upwind pair of each axis: F > 0 takes (max(D-,0), min(D+,0)) (Eq. 4),
        // F < 0 (min(D-,0), max(D+,0)) (Eq. 5, the same two squares): the
        // median of (D-, 0, L) and of (D+, 0, -L) with L = +inf for F > 0 and
        // -inf for F < 0 selects either pair with one instruction each
        const C L = f > C(0) ? __builtin_inff() : -__builtin_inff();
        const C px = __builtin_amdgcn_fmed3f(ax, 0.f, L), qx = __builtin_amdgcn_fmed3f(bx, 0.f, -L);
        const C py = __builtin_amdgcn_fmed3f(ay, 0.f, L), qy = __builtin_amdgcn_fmed3f(by, 0.f, -L);
        const C pz = __builtin_amdgcn_fmed3f(az, 0.f, L), qz = __builtin_amdgcn_fmed3f(bz, 0.f, -L);
        // the sum and the update as explicit fused multiply-adds, so that every
        // kernel compiled from this evaluates the same roundings in the same
        // order (contraction left to the compiler may pair the terms
        // differently from one kernel to the next)
        C s = px * px;
        s = fmaf(qx, qx, s);
        s = fmaf(py, py, s);
        s = fmaf(qy, qy, s);
        s = fmaf(pz, pz, s);
        s = fmaf(qz, qz, s);
        return fmaf(-(dtdx * f), __builtin_amdgcn_sqrtf(s), c);
    }
}

// The cut-off of Eq. 8 at the centre value v: 1 for |v| <= beta, the cubic
// (|v| - gamma)^2 (2|v| + gamma - 3 beta) / (gamma - beta)^3 up to gamma, 0
// beyond it and for NaN.  Exact form: the definition term by term, divided by
// k = (gamma - beta)^3.  Fast form: the same cubic written as u^2 (3 - 2u) with
// u = (gamma - |v|) / (gamma - beta) clamped to [0, 1], k = 1 / (gamma - beta)
// (fewer live registers; exactly 1 and 0 at the ends, NaN -> 0).
template <class C, bool EXACT>
__device__ inline C cutoff(C v, C beta, C gamma, C k) {
    const C a = v < C(0) ? -v : v;
    if constexpr (EXACT) {
#pragma clang fp contract(off)
        const C m = (a - gamma) * (a - gamma);
        const C l = (C(2) * a + gamma) - C(3) * beta;
        const C mid = (m * l) / k;
        return a <= beta ? C(1) : (a <= gamma ? mid : C(0));
    } else {
        const C u = fminf(fmaxf((gamma - a) * k, C(0)), C(1));
        return u * u * (C(3) - C(2) * u);
    }
}

// The smoothed sign S of Eq. 13 at the centre value c from its six
// neighbours: c / sqrt(c^2 + |Dc|^2 dx^2), Dc the central differences; 0
// where c = 0.  Exact form: the definition term by term (the squares summed x,
// then y, then z); fast form: c / sqrt(c^2 + sum of the squared neighbour
// differences / 4), with the hardware reciprocal square root.
template <class C, bool EXACT>
__device__ inline C smoothed_sign(C c, C xm, C xp, C ym, C yp, C zm, C zp, C dx) {
    if constexpr (EXACT) {
#pragma clang fp contract(off)
        const C gx = (xp - xm) / (C(2) * dx), gy = (yp - ym) / (C(2) * dx);
        const C gz = (zp - zm) / (C(2) * dx);
        const C g2 = (gx * gx + gy * gy) + gz * gz;
        const C s = c / sqrt(c * c + g2 * (dx * dx));
        return c == C(0) ? C(0) : s;
    } else {
        const C ex = xp - xm, ey = yp - ym, ez = zp - zm;
        C t = ex * ex;  // explicit fused multiply-adds (see upwind_point)
        t = fmaf(ey, ey, t);
        t = fmaf(ez, ez, t);
        const C q = fmaf(c, c, 0.25f * t);
        return c == C(0) ? C(0) : c * __builtin_amdgcn_rsqf(q);
    }
}

// What a step launch computes (a compile-time kernel parameter).
enum StepMode : int {
    kPlain = 0,        // the step of Eq. 3-5 with the speed F
    kCutoff = 1,       // the step of Eq. 8: speed c(phi) F
    kReinit = 2,       // a step of Eq. 12: speed S(d) (Eq. 13), plus dtau S; reads no F
    kReinitClamp = 3,  // kReinit, then the clamp of Eq. 10 to [-gamma, gamma]
};

// The speed of the centre point for the mode: F, c(phi) F or S(d).
template <int MODE, class C, bool EXACT, class A>
__device__ inline C mode_speed(C f, C c, C xm, C xp, C ym, C yp, C zm, C zp, const A &a) {
    if constexpr (MODE >= kReinit)
        return smoothed_sign<C, EXACT>(c, xm, xp, ym, yp, zm, zp, a.dx);
    else if constexpr (MODE == kCutoff)
        return cutoff<C, EXACT>(c, a.cut_beta, a.cut_gamma, a.cut_k) * f;
    else
        return f;
}

// The new value for the mode from the upwind value v = c - dt f |grad|:
// v itself, or v + dt S (the -1 of Eq. 12), clamped for kReinitClamp.
template <int MODE, class C, bool EXACT>
__device__ inline C mode_finish(C v, C f, C dt, C gamma) {
    if constexpr (MODE >= kReinit) {
        C w;
        if constexpr (EXACT) {
#pragma clang fp contract(off)
            w = v + dt * f;
        } else {
            w = fmaf(dt, f, v);
        }
        if constexpr (MODE == kReinitClamp) w = w < -gamma ? -gamma : (w > gamma ? gamma : w);
        return w;
    } else {
        return v;
    }
}

template <class S, class FT>
struct StepArgs {
    const S *cur;
    const S *orig;
    S *nxt;
    const FT *F;
    const int32_t *rec;       // work-item records, kItemWords int32 each
    const int32_t *nitems;    // number of records (device)
    const int32_t *range;     // batch: [first, end) records of this launch (device), else null
    const BatchInst *inst;    // batch: grid descriptors (record word 7 = grid), else null
    const uint8_t *umap;      // single grid: U membership per tile (two-step kernel), else null
    typename Codec<S>::C dx, dt, dtdx, scale;
    // cut-off of Eq. 8 (kCutoff kernels): beta, gamma and k = (gamma - beta)^3
    // (exact form) or 1 / (gamma - beta) (fast form); the clamp of Eq. 10
    // (kReinitClamp kernels) uses cut_gamma.  F is not read by kReinit*.
    typename Codec<S>::C cut_beta, cut_gamma, cut_k;
};

// Slice [w0, w1) of the items [first, end) for this block: contiguous and
// XCD-aware.  Workgroups are dispatched to the 8 XCDs round-robin (block b
// on XCD b % 8), so XCD x gets the x-th eighth of the items and its blocks
// split that eighth into contiguous slices: neighbouring items share an L2.
__device__ inline void block_slice(int first, int end, int *w0, int *w1) {
    const int n = max(end - first, 0);
    const int x = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int gx = gridDim.x >> 3;
    const int xs = first + static_cast<int>((static_cast<int64_t>(n) * x) >> 3);
    const int xe = first + static_cast<int>((static_cast<int64_t>(n) * (x + 1)) >> 3);
    const int per = (xe - xs + gx - 1) / gx;
    *w0 = min(xs + j * per, xe);
    *w1 = min(*w0 + per, xe);
}

constexpr int cpow2(int v) { return v <= 1 ? 1 : 2 * cpow2((v + 1) / 2); }
constexpr int clog2(int v) { return v <= 1 ? 0 : 1 + clog2(v / 2); }

template <class S, class FT, int TX, int TY, int TZ, int R>
struct FastCfg {
    static constexpr int XL = cpow2(R * TX);
    // threads per workgroup: 512 for item rows of 64 points and more, so that
    // every thread keeps the same number of own points as with 32-point rows
    static constexpr int NT = XL >= 64 ? 2 * kBlock : kBlock;
    static constexpr int RP = NT / XL;          // grid rows per pass
    static constexpr int ROWS = TY * TZ;
    static constexpr int NOWN = ROWS / RP;      // own points per thread
    static constexpr int NHR = 2 * (TY + TZ);   // halo rows of the y and z faces
    static constexpr int NHALO = (NHR + RP - 1) / RP;
    static constexpr int SX = R * TX + 2, SXY = SX * (TY + 2);
    using C = typename Codec<S>::C;
    static constexpr size_t lds = sizeof(C) * SXY * (TZ + 2);
    static_assert(XL <= NT && ROWS % RP == 0, "shape does not tile the block");
    static_assert(RP % TY == 0 || TY % RP == 0, "rows per pass must divide or be divided by TY");
    static_assert(ROWS <= NT, "x-face points exceed two per thread");
};

// Fast band-step kernel for a compile-time tile shape (TX, TY, TZ) and R tiles
// per work item.  Every index is a compile-time constant, a per-thread value
// or a uniform value: global loads and stores take a uniform item base plus a
// per-thread offset, LDS accesses a per-thread base plus immediates.  Per
// item, every thread
//  (1) issues the global loads of its own points (phi and F: rows lr + q*RP of
//      the item, x = lx), of its y/z halo rows and of at most one x-face
//      point, all into registers before using any;
//  (2) stores them to the LDS box; (3) after a barrier evaluates its own
//      points from the box and stores them.
// PIPE: the loads (1) of the block's next item are issued before (3) of the
// current one, so their latency overlaps the update (software pipelining over
// the block's slice of items; it pays when blocks own several items, as on
// grids that stream from HBM, at the cost of registers).
// BATCH: the item's grid comes from the descriptor its record names (word 7);
// PARTIAL: tiles at the high y/z faces may be partial (predicated rows).
// A neighbour in a band tile is read from the current buffer, one in a tile
// outside the band from phi (its value frozen for the call), one outside the
// grid is the clamped point inside the item (zero-gradient boundary).
template <class S, class FT, bool EXACT, int TX, int TY, int TZ, int R, bool BATCH, bool PARTIAL,
          bool PIPE, int MODE = kPlain>
__global__ __launch_bounds__((FastCfg<S, FT, TX, TY, TZ, R>::NT)) void upwind_fast_kernel(
    StepGeom g, StepArgs<S, FT> a) {
    using K = FastCfg<S, FT, TX, TY, TZ, R>;
    using C = typename K::C;
    constexpr int XL = K::XL, RP = K::RP, ROWS = K::ROWS, NOWN = K::NOWN, NHALO = K::NHALO;
    constexpr int SX = K::SX, SXY = K::SXY;

    extern __shared__ __align__(16) unsigned char smem[];
    C *box = reinterpret_cast<C *>(smem);

    int first = 0, end = 0;
    if (a.range) {
        first = a.range[0];
        end = a.range[1];
    } else {
        end = *a.nitems;
    }
    int w0, w1;
    block_slice(first, end, &w0, &w1);
    if (w0 >= w1) return;  // uniform

    const int lane = threadIdx.x & 63;
    const int lx = threadIdx.x % XL;
    const int lr = threadIdx.x / XL;
    const int lt = lx / TX;
    // own points: row lr + q*RP  ->  (ly, lz) = (ly0 + dly(q), lz0 + dlz(q))
    const int ly0 = (RP % TY == 0) ? lr % TY : lr;
    const int lz0 = (RP % TY == 0) ? lr / TY : 0;
    const int lbase = (lz0 + 1) * SXY + (ly0 + 1) * SX + lx + 1;
    auto dly = [](int q) { return (RP % TY == 0) ? 0 : (q % (TY / RP)) * RP; };
    auto dlz = [](int q) { return (RP % TY == 0) ? q * (RP / TY) : q / (TY / RP); };
    // x-face point of this thread (threads below 2*ROWS): side tid & 1, row tid >> 1
    const bool xok = threadIdx.x < 2 * ROWS;
    const int xside = threadIdx.x & 1;
    const int xly = (threadIdx.x >> 1) % TY, xlz = (threadIdx.x >> 1) / TY;

    // uniform description of one item, and the registers its loads fill
    struct Item {
        bool ok;
        int nx, px, ny, plane, W, H, D;
        int64_t base;
        C dtdx, dx, dt;
    };
    struct Regs {
        S raw[NOWN];
        FT fv[NOWN];
        S hv[NHALO];
        int hlds[NHALO];
        bool hok[NHALO];
        S xv;
        bool xrow_ok;
    };

    // record of item w -> geometry, then the global loads of this thread
    auto fetch = [&](int w, Item &it, Regs &r) {
        int rv = 0;
        if (lane < kItemWords) rv = a.rec[static_cast<int64_t>(w) * kItemWords + lane];
        const int t0 = __builtin_amdgcn_readlane(rv, 0);
        const int len = __builtin_amdgcn_readlane(rv, 1);
        const uint32_t m0 = __builtin_amdgcn_readlane(rv, 2), m1 = __builtin_amdgcn_readlane(rv, 3);
        const uint32_t m2 = __builtin_amdgcn_readlane(rv, 4), m3 = __builtin_amdgcn_readlane(rv, 5);
        const uint32_t mx = __builtin_amdgcn_readlane(rv, 6);
        int nz, ntx, nty, ntiles;
        int64_t goff = 0;
        it.dtdx = a.dtdx, it.dx = a.dx, it.dt = a.dt;
        if constexpr (BATCH) {
            const BatchInst &d = a.inst[__builtin_amdgcn_readlane(rv, 7)];
            it.nx = d.nx, it.px = d.px, it.ny = d.ny, nz = d.nz, ntx = d.ntx, nty = d.nty;
            ntiles = d.ntiles;
            goff = d.offset;
            it.dtdx = static_cast<C>(d.dtdx);
            it.dx = static_cast<C>(d.dx);
            it.dt = static_cast<C>(d.dt);
        } else {
            it.nx = g.nx, it.px = g.nx, it.ny = g.ny, nz = g.nz, ntx = g.ntx, nty = g.nty;
            ntiles = g.ntiles;
        }
        it.ok = t0 >= 0 && t0 < ntiles;  // an invalid id is skipped (uniform)
        if (!it.ok) return;
        const int nx = it.nx, px = it.px, ny = it.ny;
        const int plane = ny * px;
        it.plane = plane;
        const int ti0 = t0 % ntx;
        const int rr = t0 / ntx;
        const int tj = rr % nty, tk = rr / nty;
        const int x0 = ti0 * TX, y0 = tj * TY, z0 = tk * TZ;
        const int W = min(len * TX, nx - x0);
        const int H = PARTIAL ? min(TY, ny - y0) : TY;
        const int D = PARTIAL ? min(TZ, nz - z0) : TZ;
        it.W = W, it.H = H, it.D = D;
        it.base = goff + (static_cast<int64_t>(z0) * ny + y0) * px + x0;
        const S *cur = a.cur + it.base;
        const S *orig = a.orig + it.base;
        const FT *Fb = MODE < kReinit ? a.F + it.base : nullptr;
        // faces on the domain boundary: the clamped neighbour lies in the item
        const int ebits = (y0 == 0 ? 1 : 0) | (y0 + H == ny ? 2 : 0) | (z0 == 0 ? 4 : 0) |
                          (z0 + D == nz ? 8 : 0);
        const bool col_ok = lx < W;
        const int toff = lz0 * plane + ly0 * px + lx;
#pragma unroll
        for (int q = 0; q < NOWN; ++q) {
            const bool ok = col_ok && (!PARTIAL || (ly0 + dly(q) < H && lz0 + dlz(q) < D));
            if (ok) {
                const int u = dlz(q) * plane + dly(q) * px;  // uniform
                r.raw[q] = (cur + u)[toff];
                if constexpr (MODE < kReinit) r.fv[q] = (Fb + u)[toff];
            }
        }
#pragma unroll
        for (int q = 0; q < NHALO; ++q) {
            const int h = lr + q * RP;  // y-face rows (2 per z) first, then z-face rows
            int ly, lz, lyc, lzc, face;
            bool ok;
            if (h < 2 * TZ) {
                lz = h >> 1;
                face = h & 1;
                ly = face ? H : -1;
                lyc = face ? H - 1 : 0;
                lzc = lz;
                ok = lz < D;
            } else {
                const int hh = h - 2 * TZ;
                ly = hh >> 1;
                face = 2 + (hh & 1);
                lz = (hh & 1) ? D : -1;
                lzc = (hh & 1) ? D - 1 : 0;
                lyc = ly;
                ok = hh < 2 * TY && ly < H;
            }
            ok = ok && col_ok;
            r.hok[q] = ok;
            r.hlds[q] = (lz + 1) * SXY + (ly + 1) * SX + lx + 1;
            const bool hi = face & 1, zf = face & 2;
            const bool clamp = (ebits >> (face & 3)) & 1;
            const uint32_t mk = zf ? (hi ? m3 : m2) : (hi ? m1 : m0);
            const bool in = clamp || ((mk >> lt) & 1u);
            const int o = clamp ? (lzc * plane + lyc * px + lx) : (lz * plane + ly * px + lx);
            if (ok && in) r.hv[q] = cur[o];
            if (ok && !in) r.hv[q] = orig[o];
        }
        r.xrow_ok = xok && (!PARTIAL || (xly < H && xlz < D));
        const int cx = xside ? (x0 + W < nx ? W : W - 1) : (x0 > 0 ? -1 : 0);
        const bool in = (cx >= 0 && cx < W) || ((mx >> xside) & 1u);
        const int o = xlz * plane + xly * px + cx;
        if (r.xrow_ok && in) r.xv = cur[o];
        if (r.xrow_ok && !in) r.xv = orig[o];
    };

    // (2) registers -> LDS box
    auto stage = [&](const Item &it, const Regs &r) {
        if (lx < it.W) {
#pragma unroll
            for (int q = 0; q < NOWN; ++q)
                if (!PARTIAL || (ly0 + dly(q) < it.H && lz0 + dlz(q) < it.D))
                    box[lbase + dlz(q) * SXY + dly(q) * SX] = Codec<S>::load(r.raw[q], a.scale);
        }
#pragma unroll
        for (int q = 0; q < NHALO; ++q)
            if (r.hok[q]) box[r.hlds[q]] = Codec<S>::load(r.hv[q], a.scale);
        if (r.xrow_ok)
            box[(xlz + 1) * SXY + (xly + 1) * SX + (xside ? it.W + 1 : 0)] =
                Codec<S>::load(r.xv, a.scale);
    };

    // (3) update of the own points from the box
    auto update = [&](const Item &it, const Regs &r) {
        if (lx >= it.W) return;
        S *nxt = a.nxt + it.base;
        const int toff = lz0 * it.plane + ly0 * it.px + lx;
#pragma unroll
        for (int q = 0; q < NOWN; ++q) {
            if (PARTIAL && !(ly0 + dly(q) < it.H && lz0 + dlz(q) < it.D)) continue;
            const int o = lbase + dlz(q) * SXY + dly(q) * SX;
            const C c = box[o], xm = box[o - 1], xp = box[o + 1], ym = box[o - SX],
                    yp = box[o + SX], zm = box[o - SXY], zp = box[o + SXY];
            C f = C(0);
            if constexpr (MODE < kReinit) f = static_cast<C>(r.fv[q]);
            f = mode_speed<MODE, C, EXACT>(f, c, xm, xp, ym, yp, zm, zp, a);
            const C v = mode_finish<MODE, C, EXACT>(
                upwind_point<C, EXACT>(c, xm, xp, ym, yp, zm, zp, f, it.dx, it.dt, it.dtdx), f,
                it.dt, a.cut_gamma);
            const S out = (f == C(0)) ? r.raw[q] : Codec<S>::store(v, a.scale);
            (nxt + dlz(q) * it.plane + dly(q) * it.px)[toff] = out;
        }
    };

    if constexpr (PIPE) {
        Item cur;
        Regs rc;
        fetch(w0, cur, rc);
        for (int w = w0; w < w1; ++w) {
            if (cur.ok) stage(cur, rc);
            __syncthreads();  // box complete
            Item nx;
            Regs rn;
            const bool more = w + 1 < w1;  // uniform
            if (more) fetch(w + 1, nx, rn);
            if (cur.ok) update(cur, rc);
            __syncthreads();  // box free for the next item
            if (more) {
                cur = nx;
                rc = rn;
            }
        }
    } else {
        for (int w = w0; w < w1; ++w) {
            Item cur;
            Regs rc;
            fetch(w, cur, rc);
            if (!cur.ok) continue;  // uniform
            stage(cur, rc);
            __syncthreads();  // box complete
            update(cur, rc);
            __syncthreads();  // box free for the next item
        }
    }
}

// Four consecutive stored values of a row as one vector access: 16 bytes of
// FP32, 8 bytes of scaled FP16.
template <class S>
struct Vec4;
template <>
struct Vec4<float> {
    using T = float4;
    __device__ static inline float get(const T &v, int e) {
        return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
    }
    __device__ static inline T make(const float o[4]) { return make_float4(o[0], o[1], o[2], o[3]); }
};
template <>
struct Vec4<uint16_t> {
    using T = uint2;
    __device__ static inline uint16_t get(const T &v, int e) {
        const uint32_t w = e < 2 ? v.x : v.y;
        return static_cast<uint16_t>((e & 1) ? (w >> 16) : (w & 0xffffu));
    }
    __device__ static inline T make(const uint16_t o[4]) {
        return make_uint2(uint32_t(o[0]) | (uint32_t(o[1]) << 16),
                          uint32_t(o[2]) | (uint32_t(o[3]) << 16));
    }
};

// Vectorised band step (FP32 or scaled-FP16 storage, FP32 arithmetic) for
// 8-point-wide tiles on grids with nx a multiple of 4 (aligned rows): every
// lane owns 4 consecutive x-points of a row and moves them with one vector
// access, a quarter of the memory instructions of upwind_fast_kernel, with
// the same arithmetic (bit-identical results).  Box rows are padded by 4 on
// the left so the stores of the own points into LDS are aligned 16-byte
// stores too.
template <int TY, int TZ, int R>
struct VecCfg {
    static constexpr int TX = 8, V = 4;
    static constexpr int XP = R * TX;   // points per item row
    static constexpr int XV = XP / V;   // lanes per item row
    static constexpr int NT = XP >= 64 ? 2 * kBlock : kBlock;
    static constexpr int RP = NT / XV;  // item rows per pass
    static constexpr int ROWS = TY * TZ;
    static constexpr int NOWN = ROWS / RP;
    static constexpr int NHR = 2 * (TY + TZ);
    static constexpr int NHALO = (NHR + RP - 1) / RP;
    static constexpr int PAD = 4;
    static constexpr int SX = XP + 2 * PAD, SXY = SX * (TY + 2);
    static constexpr size_t lds = sizeof(float) * SXY * (TZ + 2);
    static_assert(ROWS % RP == 0 && RP % TY == 0, "rows do not tile the block");
    static_assert(2 * ROWS <= NT, "x-face points exceed one per thread");
};

// Occupancy: the cut-off variant asks for 7 waves per SIMD (at most 72
// VGPRs), the plain kernel's; left alone it took 74 VGPRs and 6 waves, and
// ran 3 % slower.  (Asking 8 waves of the plain kernel fits 64 VGPRs without
// spilling but measured 1 % slower than its own 7.)
template <class S, int TY, int TZ, int R, bool PARTIAL, int MODE = kPlain>
__global__ __launch_bounds__((VecCfg<TY, TZ, R>::NT), (MODE == kCutoff ? 7 : 1))
void upwind_vec_kernel(
    StepGeom g, StepArgs<S, float> a) {
    using K = VecCfg<TY, TZ, R>;
    using VS = Vec4<S>;
    using VT = typename VS::T;
    constexpr int TX = K::TX, RP = K::RP, ROWS = K::ROWS, NOWN = K::NOWN, NHALO = K::NHALO;
    constexpr int SX = K::SX, SXY = K::SXY, PAD = K::PAD, XV = K::XV;
    extern __shared__ __align__(16) unsigned char smem[];
    float *box = reinterpret_cast<float *>(smem);

    int w0, w1;
    block_slice(0, *a.nitems, &w0, &w1);
    const int lane = threadIdx.x & 63;
    const int lx = (threadIdx.x % XV) * 4;
    const int lr = threadIdx.x / XV;
    const int lt = lx / TX;
    const int ly0 = lr % TY, lz0 = lr / TY;
    const int lbase = (lz0 + 1) * SXY + (ly0 + 1) * SX + PAD + lx;
    constexpr int DZ = RP / TY;  // z rows between a thread's own rows
    const bool xok = threadIdx.x < 2 * ROWS;
    const int xside = threadIdx.x & 1;
    const int xly = (threadIdx.x >> 1) % TY, xlz = (threadIdx.x >> 1) / TY;
    const int nx = g.nx, ny = g.ny, nz = g.nz, plane = ny * nx;
    const float sc = a.scale;
    auto decode = [&](const VT &v) {
        return make_float4(Codec<S>::load(VS::get(v, 0), sc), Codec<S>::load(VS::get(v, 1), sc),
                           Codec<S>::load(VS::get(v, 2), sc), Codec<S>::load(VS::get(v, 3), sc));
    };

    for (int w = w0; w < w1; ++w) {
        int rv = 0;
        if (lane < kItemWords) rv = a.rec[static_cast<int64_t>(w) * kItemWords + lane];
        const int t0 = __builtin_amdgcn_readlane(rv, 0);
        const int len = __builtin_amdgcn_readlane(rv, 1);
        const uint32_t m0 = __builtin_amdgcn_readlane(rv, 2), m1 = __builtin_amdgcn_readlane(rv, 3);
        const uint32_t m2 = __builtin_amdgcn_readlane(rv, 4), m3 = __builtin_amdgcn_readlane(rv, 5);
        const uint32_t mx = __builtin_amdgcn_readlane(rv, 6);
        if (t0 < 0 || t0 >= g.ntiles) continue;  // uniform
        const int ti0 = t0 % g.ntx, rr = t0 / g.ntx;
        const int tj = rr % g.nty, tk = rr / g.nty;
        const int x0 = ti0 * TX, y0 = tj * TY, z0 = tk * TZ;
        const int W = min(len * TX, nx - x0);  // a multiple of 4
        const int H = PARTIAL ? min(TY, ny - y0) : TY;
        const int D = PARTIAL ? min(TZ, nz - z0) : TZ;
        const int64_t base = (static_cast<int64_t>(z0) * ny + y0) * nx + x0;
        const S *cur = a.cur + base;
        const S *orig = a.orig + base;
        const float *Fb = MODE < kReinit ? a.F + base : nullptr;
        S *nxt = a.nxt + base;
        const int ebits = (y0 == 0 ? 1 : 0) | (y0 + H == ny ? 2 : 0) | (z0 == 0 ? 4 : 0) |
                          (z0 + D == nz ? 8 : 0);
        const bool col_ok = lx < W;
        const int toff = lz0 * plane + ly0 * nx + lx;

        VT raw[NOWN];
        float4 fv[NOWN];
#pragma unroll
        for (int q = 0; q < NOWN; ++q) {
            if (col_ok && (!PARTIAL || (ly0 < H && lz0 + q * DZ < D))) {
                const int u = q * DZ * plane;
                raw[q] = *reinterpret_cast<const VT *>(cur + u + toff);
                if constexpr (MODE < kReinit)
                    fv[q] = *reinterpret_cast<const float4 *>(Fb + u + toff);
            }
        }
        VT hv[NHALO];
        int hlds[NHALO];
        bool hok[NHALO];
#pragma unroll
        for (int q = 0; q < NHALO; ++q) {
            const int h = lr + q * RP;  // y-face rows (2 per z) first, then z-face rows
            int ly, lz, lyc, lzc, face;
            bool ok;
            if (h < 2 * TZ) {
                lz = h >> 1;
                face = h & 1;
                ly = face ? H : -1;
                lyc = face ? H - 1 : 0;
                lzc = lz;
                ok = lz < D;
            } else {
                const int hh = h - 2 * TZ;
                ly = hh >> 1;
                face = 2 + (hh & 1);
                lz = (hh & 1) ? D : -1;
                lzc = (hh & 1) ? D - 1 : 0;
                lyc = ly;
                ok = hh < 2 * TY && ly < H;
            }
            ok = ok && col_ok;
            hok[q] = ok;
            hlds[q] = (lz + 1) * SXY + (ly + 1) * SX + PAD + lx;
            const bool hi = face & 1, zf = face & 2;
            const bool clamp = (ebits >> (face & 3)) & 1;
            const uint32_t mk = zf ? (hi ? m3 : m2) : (hi ? m1 : m0);
            const bool in = clamp || ((mk >> lt) & 1u);
            const int o = clamp ? (lzc * plane + lyc * nx + lx) : (lz * plane + ly * nx + lx);
            if (ok) hv[q] = *reinterpret_cast<const VT *>((in ? cur : orig) + o);
        }
        S xv = S(0);
        const bool xrow_ok = xok && (!PARTIAL || (xly < H && xlz < D));
        const int cx = xside ? (x0 + W < nx ? W : W - 1) : (x0 > 0 ? -1 : 0);
        {
            const bool in = (cx >= 0 && cx < W) || ((mx >> xside) & 1u);
            const int o = xlz * plane + xly * nx + cx;
            if (xrow_ok) xv = (in ? cur : orig)[o];
        }

        if (col_ok) {
#pragma unroll
            for (int q = 0; q < NOWN; ++q)
                if (!PARTIAL || (ly0 < H && lz0 + q * DZ < D))
                    *reinterpret_cast<float4 *>(box + lbase + q * DZ * SXY) = decode(raw[q]);
        }
#pragma unroll
        for (int q = 0; q < NHALO; ++q)
            if (hok[q]) *reinterpret_cast<float4 *>(box + hlds[q]) = decode(hv[q]);
        if (xrow_ok)
            box[(xlz + 1) * SXY + (xly + 1) * SX + (xside ? PAD + W : PAD - 1)] =
                Codec<S>::load(xv, sc);
        __syncthreads();  // box complete

        if (col_ok) {
#pragma unroll
            for (int q = 0; q < NOWN; ++q) {
                if (PARTIAL && !(ly0 < H && lz0 + q * DZ < D)) continue;
                const int o0 = lbase + q * DZ * SXY;
                float f4[4] = {0.f, 0.f, 0.f, 0.f};
                if constexpr (MODE < kReinit) {
                    f4[0] = fv[q].x, f4[1] = fv[q].y, f4[2] = fv[q].z, f4[3] = fv[q].w;
                }
                S out[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int o = o0 + e;
                    const float c = box[o], xm = box[o - 1], xp = box[o + 1], ym = box[o - SX],
                                yp = box[o + SX], zm = box[o - SXY], zp = box[o + SXY];
                    const float f = mode_speed<MODE, float, false>(f4[e], c, xm, xp, ym, yp, zm,
                                                                   zp, a);
                    const float v = mode_finish<MODE, float, false>(
                        upwind_point<float, false>(c, xm, xp, ym, yp, zm, zp, f, a.dx, a.dt,
                                                   a.dtdx),
                        f, a.dt, a.cut_gamma);
                    out[e] = (f == 0.f) ? VS::get(raw[q], e) : Codec<S>::store(v, sc);
                }
                *reinterpret_cast<VT *>(nxt + q * DZ * plane + toff) = VS::make(out);
            }
        }
        __syncthreads();  // box free for the next item
    }
}

// Two steps per launch (temporal blocking) of the vectorised band step, for
// 8x8x8 tiles on grids whose y and z extents are whole tiles and nx a
// multiple of 4.  A work item loads its points with a halo two points deep
// (the y/z rows at distance 1 and 2, the four yz-edge rows, and 4-point x
// ends of its own and ring rows), computes the first step on its points and
// on the ring one point outside them (a ring point outside U keeps its
// value, as it would with one step per launch), then the second step on its
// points from those.  Every value is computed from the same inputs and with
// the same arithmetic as with two one-step launches (an intermediate FP16
// value is rounded to storage as it would be stored), so the result is
// bit-identical; the item moves its own points once per two steps.  (A
// tuning option: on the bench grids it runs slower than two one-step
// launches.)
// Membership of a halo point's tile in U (read from cur, else frozen in orig)
// comes from the U map.  A neighbour outside the grid is the point itself
// (zero-gradient boundary).
template <int R>
struct Vec2Cfg {
    static constexpr int TX = 8, TY = 8, TZ = 8, V = 4;
    static constexpr int XP = R * TX;          // own points per item row
    static constexpr int XV = XP / V;          // lanes per item row
    static constexpr int NT = XP >= 64 ? 2 * kBlock : kBlock;
    static constexpr int RP = NT / XV;         // item rows per pass
    static constexpr int ROWS = TY * TZ;       // own rows
    static constexpr int NOWN = ROWS / RP;
    static constexpr int NHR = 4 * TZ + 4 * TY + 4;  // distance-1/2 y and z rows, yz-edge rows
    static constexpr int NHP = (NHR + RP - 1) / RP;
    static constexpr int NRING = 2 * TZ + 2 * TY;    // ring rows (distance 1)
    static constexpr int NXH = 2 * (ROWS + NRING);   // 4-point x ends of own and ring rows
    static constexpr int NXR = 2 * ROWS;             // x-ring points
    static constexpr int PAD = 4;
    static constexpr int SX = XP + 2 * PAD;
    static constexpr int SXY0 = SX * (TY + 4), SXY1 = SX * (TY + 2);
    static constexpr int B0 = SXY0 * (TZ + 4), B1 = SXY1 * (TZ + 2);
    static constexpr size_t lds = sizeof(float) * (B0 + B1);
    static_assert(ROWS % RP == 0 && NRING <= RP, "rows do not tile the block");
    static_assert(NXH <= NT && NXR <= NT, "x ends exceed one per thread");
};

// (ly, lz) of halo row h: y rows at ly = -2, -1, 8, 9 for every lz, then z
// rows at lz = -2, -1, 8, 9 for every ly, then the four yz-edge rows.
__device__ inline void vec2_halo_row(int h, int *ly, int *lz) {
    if (h < 32) {
        const int k = h & 3;
        *lz = h >> 2;
        *ly = k < 2 ? k - 2 : k + 6;
    } else if (h < 64) {
        const int k = h & 3;
        *ly = (h - 32) >> 2;
        *lz = k < 2 ? k - 2 : k + 6;
    } else {
        const int k = h - 64;
        *ly = (k & 1) ? 8 : -1;
        *lz = (k & 2) ? 8 : -1;
    }
}

// (ly, lz) of ring row h: y rows at ly = -1, 8 for every lz, then z rows at
// lz = -1, 8 for every ly.
__device__ inline void vec2_ring_row(int h, int *ly, int *lz) {
    if (h < 16) {
        *lz = h >> 1;
        *ly = (h & 1) ? 8 : -1;
    } else {
        *ly = (h - 16) >> 1;
        *lz = (h & 1) ? 8 : -1;
    }
}

template <class S, int R>
__global__ __launch_bounds__((Vec2Cfg<R>::NT)) void upwind_vec2_kernel(StepGeom g,
                                                                      StepArgs<S, float> a) {
    using K = Vec2Cfg<R>;
    using VS = Vec4<S>;
    using VT = typename VS::T;
    constexpr int RP = K::RP, NOWN = K::NOWN, NHP = K::NHP, XV = K::XV;
    constexpr int SX = K::SX, SXY0 = K::SXY0, SXY1 = K::SXY1, PAD = K::PAD;
    extern __shared__ __align__(16) unsigned char smem[];
    float *box0 = reinterpret_cast<float *>(smem);  // step-n values, y/z in [-2, 9]
    float *box1 = box0 + K::B0;                     // step-n+1 values, y/z in [-1, 8]

    int w0, w1;
    block_slice(0, *a.nitems, &w0, &w1);
    const int lane = threadIdx.x & 63;
    const int lx = (threadIdx.x % XV) * 4;
    const int lr = threadIdx.x / XV;
    const int nx = g.nx, ny = g.ny, nz = g.nz, plane = ny * nx;
    const int ntx = g.ntx, nty = g.nty;
    const float sc = a.scale;
    auto o0 = [](int x, int y, int z) { return (z + 2) * SXY0 + (y + 2) * SX + PAD + x; };
    auto o1 = [](int x, int y, int z) { return (z + 1) * SXY1 + (y + 1) * SX + PAD + x; };
    auto decode = [&](const VT &v) {
        return make_float4(Codec<S>::load(VS::get(v, 0), sc), Codec<S>::load(VS::get(v, 1), sc),
                           Codec<S>::load(VS::get(v, 2), sc), Codec<S>::load(VS::get(v, 3), sc));
    };
    // the value a one-step launch would store and the next one load
    auto stored = [&](float v) { return Codec<S>::load(Codec<S>::store(v, sc), sc); };
    auto in_u = [&](int gx, int gy, int gz) {
        return a.umap[(static_cast<int64_t>(gz >> 3) * nty + (gy >> 3)) * ntx + (gx >> 3)] != 0;
    };

    for (int w = w0; w < w1; ++w) {
        int rv = 0;
        if (lane < kItemWords) rv = a.rec[static_cast<int64_t>(w) * kItemWords + lane];
        const int t0 = __builtin_amdgcn_readlane(rv, 0);
        const int len = __builtin_amdgcn_readlane(rv, 1);
        if (t0 < 0 || t0 >= g.ntiles) continue;  // uniform
        const int ti0 = t0 % ntx, rr = t0 / ntx;
        const int tj = rr % nty, tk = rr / nty;
        const int x0 = ti0 * 8, y0 = tj * 8, z0 = tk * 8;
        const int W = min(len * 8, nx - x0);  // a multiple of 4
        const int64_t base = (static_cast<int64_t>(z0) * ny + y0) * nx + x0;
        const S *cur = a.cur + base;
        const S *orig = a.orig + base;
        const float *Fb = a.F + base;
        S *nxt = a.nxt + base;
        const bool col_ok = lx < W;
        auto off = [&](int x, int y, int z) { return z * plane + y * nx + x; };
        auto inside = [&](int x, int y, int z) {
            return x0 + x >= 0 && x0 + x < nx && y0 + y >= 0 && y0 + y < ny && z0 + z >= 0 &&
                   z0 + z < nz;
        };

        // (1) global loads
        VT raw[NOWN];
        float4 fv[NOWN];
#pragma unroll
        for (int q = 0; q < NOWN; ++q) {
            const int row = lr + q * RP, ly = row & 7, lz = row >> 3;
            if (col_ok) {
                raw[q] = *reinterpret_cast<const VT *>(cur + off(lx, ly, lz));
                fv[q] = *reinterpret_cast<const float4 *>(Fb + off(lx, ly, lz));
            }
        }
        VT hv[NHP];
        bool hok[NHP];
        int hslot[NHP];
#pragma unroll
        for (int q = 0; q < NHP; ++q) {
            const int h = lr + q * RP;
            int ly = 0, lz = 0;
            if (h < K::NHR) vec2_halo_row(h, &ly, &lz);
            hok[q] = h < K::NHR && col_ok && inside(lx, ly, lz);
            hslot[q] = o0(lx, ly, lz);
            if (hok[q]) {
                const bool u = in_u(x0 + lx, y0 + ly, z0 + lz);
                hv[q] = *reinterpret_cast<const VT *>((u ? cur : orig) + off(lx, ly, lz));
            }
        }
        // ring rows: F of their points (their first step is computed by this thread)
        int rly = 0, rlz = 0;
        if (lr < K::NRING) vec2_ring_row(lr, &rly, &rlz);
        const bool rok = lr < K::NRING && col_ok && inside(lx, rly, rlz);
        const bool ru = rok && in_u(x0 + lx, y0 + rly, z0 + rlz);
        float4 rf = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ru) rf = *reinterpret_cast<const float4 *>(Fb + off(lx, rly, rlz));
        // 4-point x ends of the own and ring rows
        const int xr = threadIdx.x >> 1, xside = threadIdx.x & 1;
        int xly = 0, xlz = 0;
        if (xr < K::ROWS) {
            xly = xr & 7;
            xlz = xr >> 3;
        } else if (xr < K::ROWS + K::NRING) {
            vec2_ring_row(xr - K::ROWS, &xly, &xlz);
        }
        const int xx = xside ? W : -4;
        const bool xok = threadIdx.x < K::NXH && inside(xx, xly, xlz);
        VT xh;
        if (xok) {
            const bool u = in_u(x0 + xx, y0 + xly, z0 + xlz);
            xh = *reinterpret_cast<const VT *>((u ? cur : orig) + off(xx, xly, xlz));
        }
        // x-ring points (x = -1 or W on the own rows): F and membership
        const int cxr = xside ? W : -1;
        const bool cok = threadIdx.x < K::NXR && inside(cxr, xly, xlz);
        const bool cu = cok && in_u(x0 + cxr, y0 + xly, z0 + xlz);
        float cf = 0.f;
        if (cu) cf = Fb[off(cxr, xly, xlz)];

        // (2) the step-n box
        if (col_ok) {
#pragma unroll
            for (int q = 0; q < NOWN; ++q) {
                const int row = lr + q * RP;
                *reinterpret_cast<float4 *>(box0 + o0(lx, row & 7, row >> 3)) = decode(raw[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < NHP; ++q)
            if (hok[q]) *reinterpret_cast<float4 *>(box0 + hslot[q]) = decode(hv[q]);
        if (xok) *reinterpret_cast<float4 *>(box0 + o0(xx, xly, xlz)) = decode(xh);
        __syncthreads();

        // one step at box point (x, y, z) from box b (strides sxy), F = f
        auto step = [&](const float *b, int sxy, int o, int x, int y, int z, float f) {
            const float c = b[o];
            const float xm = x0 + x > 0 ? b[o - 1] : c, xp = x0 + x < nx - 1 ? b[o + 1] : c;
            const float ym = y0 + y > 0 ? b[o - SX] : c, yp = y0 + y < ny - 1 ? b[o + SX] : c;
            const float zm = z0 + z > 0 ? b[o - sxy] : c, zp = z0 + z < nz - 1 ? b[o + sxy] : c;
            return upwind_point<float, false>(c, xm, xp, ym, yp, zm, zp, f, a.dx, a.dt, a.dtdx);
        };

        // (3) first step: own points, ring rows, x-ring points -> box1
        if (col_ok) {
#pragma unroll
            for (int q = 0; q < NOWN; ++q) {
                const int row = lr + q * RP, ly = row & 7, lz = row >> 3;
                const float f4[4] = {fv[q].x, fv[q].y, fv[q].z, fv[q].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int oo = o0(lx + e, ly, lz);
                    const float v = step(box0, SXY0, oo, lx + e, ly, lz, f4[e]);
                    box1[o1(lx + e, ly, lz)] = f4[e] == 0.f ? box0[oo] : stored(v);
                }
            }
        }
        if (rok) {
            const float f4[4] = {rf.x, rf.y, rf.z, rf.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int oo = o0(lx + e, rly, rlz);
                float v = box0[oo];  // outside U: frozen
                if (ru && f4[e] != 0.f) v = stored(step(box0, SXY0, oo, lx + e, rly, rlz, f4[e]));
                box1[o1(lx + e, rly, rlz)] = v;
            }
        }
        if (cok) {
            const int oo = o0(cxr, xly, xlz);
            float v = box0[oo];
            if (cu && cf != 0.f) v = stored(step(box0, SXY0, oo, cxr, xly, xlz, cf));
            box1[o1(cxr, xly, xlz)] = v;
        }
        __syncthreads();

        // (4) second step on the own points -> nxt
        if (col_ok) {
#pragma unroll
            for (int q = 0; q < NOWN; ++q) {
                const int row = lr + q * RP, ly = row & 7, lz = row >> 3;
                const float f4[4] = {fv[q].x, fv[q].y, fv[q].z, fv[q].w};
                S out[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float v = step(box1, SXY1, o1(lx + e, ly, lz), lx + e, ly, lz, f4[e]);
                    out[e] = f4[e] == 0.f ? VS::get(raw[q], e) : Codec<S>::store(v, sc);
                }
                *reinterpret_cast<VT *>(nxt + off(lx, ly, lz)) = VS::make(out);
            }
        }
        __syncthreads();  // boxes free for the next item
    }
}

}  // namespace ls
