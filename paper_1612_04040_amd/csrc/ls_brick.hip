// Tile-major ("brick") storage of the band update: the grid's 8^3 tiles one
// after another in tile-id order, each tile's 512 points contiguous with x
// fastest inside the tile (point (i, j, k) of tile t at t*512 + (k%8)*64 +
// (j%8)*8 + i%8).  A work item (a run of up to 4 band tiles along x) is then
// one contiguous stretch of memory for phi, F and the result, where the
// x-fastest grid scatters it over 64 rows; the band kernels move the same
// algorithmic bytes at close to streaming efficiency.  Conversion kernels
// move fields between the layouts; the band build, the steps of every mode
// (Eq. 3-5, the cut-off of Eq. 8, the reinitialisation of Eq. 12-13 with the
// clamp of Eq. 10) and the windowed driver of Sec. 1.1 run on bricks with the
// same arithmetic as the x-fastest kernels, so their results agree bit for
// bit.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "ls_stats.h"
#include "ls_stencil.h"

namespace ls {

int band_finish(const Geom &g, uint8_t *ws, int dilate, int32_t *tiles, int32_t *ntiles_dev,
                hipStream_t stream, TileAccum accum);  // ls_band.hip

typedef float brick_f4 __attribute__((ext_vector_type(4)));
typedef unsigned short brick_h8 __attribute__((ext_vector_type(8)));

constexpr int kBrick = 512;  // points of an 8^3 tile
constexpr int kBrickRun = 4;  // tiles per work item

// One tile row (8 consecutive x points) of stored values: 32 bytes of FP32
// or 16 bytes of scaled FP16, moved as 16-byte vectors.
template <class S>
struct BrickRow;

template <>
struct BrickRow<float> {
    brick_f4 a, b;
    __device__ static BrickRow load(const float *p) {
        return {*reinterpret_cast<const brick_f4 *>(p), *reinterpret_cast<const brick_f4 *>(p + 4)};
    }
    __device__ void store(float *p) const {
        *reinterpret_cast<brick_f4 *>(p) = a;
        *reinterpret_cast<brick_f4 *>(p + 4) = b;
    }
    __device__ float value(int e, float) const { return e < 4 ? a[e] : b[e - 4]; }
    __device__ float raw(int e) const { return value(e, 1.0f); }
    __device__ void set(int e, float v) {
        if (e < 4)
            a[e] = v;
        else
            b[e - 4] = v;
    }
};

template <>
struct BrickRow<uint16_t> {
    brick_h8 h;
    __device__ static BrickRow load(const uint16_t *p) {
        return {*reinterpret_cast<const brick_h8 *>(p)};
    }
    __device__ void store(uint16_t *p) const { *reinterpret_cast<brick_h8 *>(p) = h; }
    __device__ float value(int e, float s) const {
        return Codec<uint16_t>::load(static_cast<uint16_t>(h[e]), s);
    }
    __device__ uint16_t raw(int e) const { return static_cast<uint16_t>(h[e]); }
    __device__ void set(int e, uint16_t v) { h[e] = v; }
};

// ---------------------------------------------------------------------------
// layout conversion: one block per run of 4 tiles of a tile row; thread ->
// (tile b = tid & 3, row r = tid >> 2), so that 4 neighbouring lanes move one
// 32-point stretch of a grid row

template <class S, bool TO_BRICK>
__global__ __launch_bounds__(kBlock) void brick_convert_kernel(const S *__restrict__ src,
                                                               S *__restrict__ dst, int nx, int ny,
                                                               int ntx, int nty) {
    const int g4 = blockIdx.x, tj = blockIdx.y, tk = blockIdx.z;
    const int b = threadIdx.x & 3, r = threadIdx.x >> 2;
    const int ti = g4 * 4 + b;
    if (ti >= ntx) return;
    const int z = r >> 3, y = r & 7;
    const int64_t t = (static_cast<int64_t>(tk) * nty + tj) * ntx + ti;
    const int64_t di = (static_cast<int64_t>(tk * 8 + z) * ny + (tj * 8 + y)) * nx + ti * 8;
    const int64_t bi = t * kBrick + r * 8;
    if (TO_BRICK)
        BrickRow<S>::load(src + di).store(dst + bi);
    else
        BrickRow<S>::load(src + bi).store(dst + di);
}

// ---------------------------------------------------------------------------
// tile flags (Eq. 6) on bricks: one wave per tile, lane -> one tile row

template <class S>
__global__ __launch_bounds__(kBlock) void brick_flag_kernel(
    const S *__restrict__ phi, int64_t ntiles, typename Codec<S>::C gamma, float scale,
    const int32_t *__restrict__ list, const int32_t *__restrict__ list_count,
    uint8_t *__restrict__ a_flags) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBlock / 64);
    const int64_t n = list ? std::min<int64_t>(*list_count, ntiles) : ntiles;
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6); p < n;
         p += waves) {
        const int64_t t = list ? list[p] : p;
        if (t < 0 || t >= ntiles) continue;  // uniform per wave
        const BrickRow<S> row = BrickRow<S>::load(phi + t * kBrick + lane * 8);
        bool hit = false;
#pragma unroll
        for (int e = 0; e < 8; ++e) hit |= fabsf(row.value(e, scale)) < gamma;
        const bool any = __ballot(hit) != 0;
        if (lane == 0) a_flags[t] = any ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// the band step on bricks.  Item = run of len <= 4 band tiles (the record of
// the x-fastest plan).  Thread -> tile row (b = tid >> 6, z = (tid >> 3) & 7,
// y = tid & 7) of the run: it loads that row of phi and F, threads 0..127
// also one face row of a neighbour tile (y-, y+, z-, z+ of tile tid >> 5) and
// threads 128..255 one x-face point at the ends of the run; the LDS box holds
// the run with its one-point halo (x padded by 4 so that rows are 16-byte
// aligned).  A neighbour tile in the band is read from cur, one outside it
// from orig (its values frozen for the call), a face on the domain boundary
// is the tile's own boundary row (zero-gradient boundary).

// Box pitches against LDS bank conflicts (64 banks of 4 bytes; a 16-byte read
// by 16 lanes at a time): lane (y, z) of a wave reads 16-byte pieces of its
// row at y*SX + z*SXY.  With SX = 44 the pieces of y = 0..7 fall in 8 of the
// 16 four-bank groups and, with SXY = 32 mod 64, those of z + 1 in the other
// 8, so each 16-lane read is conflict-free (SX = 40 and SXY = 12 SX or 10 SX
// put up to four pieces in one group).
constexpr int kBrickPitch = kBrickRun * 8 + 12;  // 44 floats
static_assert(kBrickPitch % 8 == 4, "row pitch 4 mod 8");
constexpr int brick_plane_pitch(int rows) {  // smallest >= rows * SX that is 32 mod 64
    return rows * kBrickPitch + ((32 - rows * kBrickPitch % 64) % 64 + 64) % 64;
}

struct BrickBox {
    static constexpr int PAD = 4, SX = kBrickPitch, SXY = brick_plane_pitch(10);
    static constexpr size_t lds = sizeof(float) * SXY * 10;
};

template <class S, int MODE>
__global__ __launch_bounds__(kBlock) void brick_step_kernel(StepGeom g, StepArgs<S, float> a) {
    constexpr int PAD = BrickBox::PAD, SX = BrickBox::SX, SXY = BrickBox::SXY;
    extern __shared__ __align__(16) unsigned char smem[];
    float *box = reinterpret_cast<float *>(smem);
    int w0, w1;
    block_slice(0, *a.nitems, &w0, &w1);
    const int tid = threadIdx.x, lane = tid & 63;
    const int ntx = g.ntx, nty = g.nty, ntz = g.ntz;
    const float sc = a.scale;
    // own row
    const int ob = tid >> 6, orow = tid & 63, oz = orow >> 3, oy = orow & 7;
    const int o_lds = (oz + 1) * SXY + (oy + 1) * SX + PAD + ob * 8;
    // face row (threads 0..127): tile fl, face ff (y-, y+, z-, z+), index k
    const int fl = (tid >> 5) & 3, ff = (tid >> 3) & 3, fk = tid & 7;
    int f_src, f_own, f_lds;
    if (ff == 0) {
        f_src = fk * 64 + 7 * 8, f_own = fk * 64, f_lds = (fk + 1) * SXY;
    } else if (ff == 1) {
        f_src = fk * 64, f_own = fk * 64 + 7 * 8, f_lds = (fk + 1) * SXY + 9 * SX;
    } else if (ff == 2) {
        f_src = 7 * 64 + fk * 8, f_own = fk * 8, f_lds = (fk + 1) * SX;
    } else {
        f_src = fk * 8, f_own = 7 * 64 + fk * 8, f_lds = 9 * SXY + (fk + 1) * SX;
    }
    f_lds += PAD + fl * 8;
    const bool frow = tid < 128;
    // x-face point (threads 128..255): side xs, row (xz, xy)
    const int xs = (tid >> 6) & 1, xr = tid & 63, xz = xr >> 3, xy = xr & 7;
    const bool xthr = tid >= 128;

    for (int w = w0; w < w1; ++w) {
        int rv = 0;
        if (lane < kItemWords) rv = a.rec[static_cast<int64_t>(w) * kItemWords + lane];
        const int t0 = __builtin_amdgcn_readlane(rv, 0);
        const int len = __builtin_amdgcn_readlane(rv, 1);
        const uint32_t m0 = __builtin_amdgcn_readlane(rv, 2), m1 = __builtin_amdgcn_readlane(rv, 3);
        const uint32_t m2 = __builtin_amdgcn_readlane(rv, 4), m3 = __builtin_amdgcn_readlane(rv, 5);
        const uint32_t mx = __builtin_amdgcn_readlane(rv, 6);
        if (t0 < 0 || t0 >= g.ntiles || len < 1 || len > kBrickRun) continue;  // uniform
        const uint32_t ut = static_cast<uint32_t>(t0);
        const uint32_t rr = ut / static_cast<uint32_t>(ntx);
        const int ti0 = static_cast<int>(ut - rr * static_cast<uint32_t>(ntx));
        const int tk = static_cast<int>(rr / static_cast<uint32_t>(nty));
        const int tj = static_cast<int>(rr) - tk * nty;
        const int64_t base = static_cast<int64_t>(t0) * kBrick;
        const bool own_ok = ob < len;

        // (1) global loads
        BrickRow<S> own;
        brick_f4 fa = {0.f, 0.f, 0.f, 0.f}, fb = fa;
        if (own_ok) {
            own = BrickRow<S>::load(a.cur + base + tid * 8);
            if constexpr (MODE < kReinit) {
                fa = *reinterpret_cast<const brick_f4 *>(a.F + base + tid * 8);
                fb = *reinterpret_cast<const brick_f4 *>(a.F + base + tid * 8 + 4);
            }
        }
        BrickRow<S> face;
        const bool fok = frow && fl < len;
        if (fok) {
            const uint32_t mk = ff == 0 ? m0 : (ff == 1 ? m1 : (ff == 2 ? m2 : m3));
            const bool edge = ff == 0 ? tj == 0
                                      : (ff == 1 ? tj == nty - 1 : (ff == 2 ? tk == 0 : tk == ntz - 1));
            const bool in = (mk >> fl) & 1u;
            const int64_t step = ff < 2 ? ntx : static_cast<int64_t>(ntx) * nty;
            const int64_t nt = static_cast<int64_t>(t0 + fl) + ((ff & 1) ? step : -step);
            face = edge ? BrickRow<S>::load(a.cur + base + fl * kBrick + f_own)
                        : BrickRow<S>::load((in ? a.cur : a.orig) + nt * kBrick + f_src);
        }
        S xv = S(0);
        if (xthr) {
            const bool edge = xs ? ti0 + len == ntx : ti0 == 0;
            const bool in = (mx >> xs) & 1u;
            if (edge)
                xv = a.cur[base + (xs ? (len - 1) * kBrick + 7 : 0) + xz * 64 + xy * 8];
            else
                xv = (in ? a.cur : a.orig)[(xs ? base + len * kBrick : base - kBrick) + xz * 64 +
                                           xy * 8 + (xs ? 0 : 7)];
        }

        // (2) the box
        if (own_ok) {
            *reinterpret_cast<brick_f4 *>(box + o_lds) =
                brick_f4{own.value(0, sc), own.value(1, sc), own.value(2, sc), own.value(3, sc)};
            *reinterpret_cast<brick_f4 *>(box + o_lds + 4) =
                brick_f4{own.value(4, sc), own.value(5, sc), own.value(6, sc), own.value(7, sc)};
        }
        if (fok) {
            *reinterpret_cast<brick_f4 *>(box + f_lds) = brick_f4{
                face.value(0, sc), face.value(1, sc), face.value(2, sc), face.value(3, sc)};
            *reinterpret_cast<brick_f4 *>(box + f_lds + 4) = brick_f4{
                face.value(4, sc), face.value(5, sc), face.value(6, sc), face.value(7, sc)};
        }
        if (xthr)
            box[(xz + 1) * SXY + (xy + 1) * SX + (xs ? PAD + len * 8 : PAD - 1)] =
                Codec<S>::load(xv, sc);
        __syncthreads();  // box complete

        // (3) the update of the thread's row, in two halves of 4 points (fewer
        // live registers); a point with zero speed keeps its stored bits
        if (own_ok) {
            float c[10];
            {
                const brick_f4 c0 = *reinterpret_cast<const brick_f4 *>(box + o_lds);
                const brick_f4 c1 = *reinterpret_cast<const brick_f4 *>(box + o_lds + 4);
                c[0] = box[o_lds - 1];
                c[9] = box[o_lds + 8];
#pragma unroll
                for (int e = 0; e < 4; ++e) c[1 + e] = c0[e], c[5 + e] = c1[e];
            }
            BrickRow<S> out;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int o = o_lds + 4 * hh;
                const brick_f4 ym = *reinterpret_cast<const brick_f4 *>(box + o - SX);
                const brick_f4 yp = *reinterpret_cast<const brick_f4 *>(box + o + SX);
                const brick_f4 zm = *reinterpret_cast<const brick_f4 *>(box + o - SXY);
                const brick_f4 zp = *reinterpret_cast<const brick_f4 *>(box + o + SXY);
                const brick_f4 f4 = hh ? fb : fa;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = 4 * hh + q;
                    const float cc = c[e + 1];
                    const float f = mode_speed<MODE, float, false>(f4[q], cc, c[e], c[e + 2],
                                                                   ym[q], yp[q], zm[q], zp[q], a);
                    const float v = mode_finish<MODE, float, false>(
                        upwind_point<float, false>(cc, c[e], c[e + 2], ym[q], yp[q], zm[q], zp[q],
                                                   f, a.dx, a.dt, a.dtdx),
                        f, a.dt, a.cut_gamma);
                    if constexpr (std::is_same<S, float>::value)
                        out.set(e, f == 0.f ? cc : v);  // the box holds the stored bits
                    else
                        out.set(e, f == 0.f ? own.raw(e) : Codec<S>::store(v, sc));
                }
            }
            out.store(a.nxt + base + tid * 8);
        }
        __syncthreads();  // box free for the next item
    }
}

// Two steps per launch on bricks (temporal blocking): the run's points after
// two steps from one pass over its data.  The box holds the run with a halo
// two points deep (x in [-2, 8 len + 1], y and z in [-2, 9]), filled with the
// step-n values wherever a point within two points of the run (in the L1
// sense) needs one: the run, two face layers of its y/z neighbour tiles, one
// row of each y-z diagonal neighbour, two x-layers at the run's ends and the
// x-ends of the ring rows.  A position outside the grid takes the value of its
// clamped position (zero-gradient boundary).  The first step is computed on
// the run and on the ring one point around it (a ring point in a tile outside
// the band keeps its value; a ring position outside the grid takes the new
// value of its clamped run point), written back into the box (rounded to the
// storage, as a one-step launch would store it), and the second step on the
// run from there.  Every point gets the arithmetic of two one-step launches
// on the same values, so the result is the same, bit for bit; the run's own
// data is read and written once per two steps.
struct Brick2Box {
    static constexpr int PAD = 4, SX = kBrickPitch, SXY = brick_plane_pitch(12);
    static constexpr size_t lds = sizeof(float) * SXY * 12;
};
static_assert(Brick2Box::PAD + kBrickRun * 8 + 2 <= Brick2Box::SX, "box row holds x in [-2, 8R+1]");
static_assert(BrickBox::SXY == 480 && Brick2Box::SXY == 544, "plane pitches 32 mod 64");

template <class S, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void brick_step2_kernel(
    StepGeom g, StepArgs<S, float> a) {
    constexpr int PAD = Brick2Box::PAD, SX = Brick2Box::SX, SXY = Brick2Box::SXY;
    extern __shared__ __align__(16) unsigned char smem[];
    float *box = reinterpret_cast<float *>(smem);
    auto bx = [](int x, int y, int z) { return (z + 2) * SXY + (y + 2) * SX + PAD + x; };
    int w0, w1;
    block_slice(0, *a.nitems, &w0, &w1);
    const int tid = threadIdx.x, lane = tid & 63;
    const int ntx = g.ntx, nty = g.nty, ntz = g.ntz;
    const int64_t sy = ntx, sz = static_cast<int64_t>(ntx) * nty;
    const float sc = a.scale;
    // own row of the thread
    const int ob = tid >> 6, oz = (tid >> 3) & 7, oy = tid & 7;
    // face-layer row: tile fl, face ff (y-, y+, z-, z+), layer (outer, inner), index k
    const int fl = tid >> 6, ff = (tid >> 4) & 3, flay = (tid >> 3) & 1, fk = tid & 7;
    const int f_y = ff == 0 ? flay - 2 : ff == 1 ? 8 + flay : fk;
    const int f_z = ff == 2 ? flay - 2 : ff == 3 ? 8 + flay : fk;
    // ring half-row (first step): tile fl, face ff, index rk, half rh
    const int rk = (tid >> 1) & 7, rh = tid & 1;
    const int r_y = ff == 0 ? -1 : ff == 1 ? 8 : rk;
    const int r_z = ff == 2 ? -1 : ff == 3 ? 8 : rk;
    const int r_x = fl * 8 + rh * 4;
    // x ring point (first step, threads 0..127): side, (y, z)
    const int xs = (tid >> 6) & 1, xy = tid & 7, xz = (tid >> 3) & 7;

    // value of stored element i of buffer p as FP32
    auto val = [&](const S *p, int64_t i) { return Codec<S>::load(p[i], sc); };
    // the first step's value as a one-step launch would store and reload it
    auto kept = [&](float v) {
        if constexpr (std::is_same<S, float>::value)
            return v;
        else
            return Codec<S>::load(Codec<S>::store(v, sc), sc);
    };
    auto point = [&](int o, float f) {
        const float c = box[o], xm = box[o - 1], xp = box[o + 1], ym = box[o - SX],
                    yp = box[o + SX], zm = box[o - SXY], zp = box[o + SXY];
        const float s = mode_speed<MODE, float, false>(f, c, xm, xp, ym, yp, zm, zp, a);
        const float v = mode_finish<MODE, float, false>(
            upwind_point<float, false>(c, xm, xp, ym, yp, zm, zp, s, a.dx, a.dt, a.dtdx), s,
            a.dt, a.cut_gamma);
        return s == 0.f ? c : v;  // zero speed: the stored value unchanged
    };
    // point()'s arithmetic on the 8 points of a box row from o (16-byte
    // aligned), every operand read as an aligned 16-byte piece (single floats
    // at the row's ends met 4-way bank conflicts); emit(e, speed, update,
    // centre) receives each point
    auto row8 = [&](int o, const float (&f8)[8], auto &&emit) {
        float c[10];
        {
            const brick_f4 c0 = *reinterpret_cast<const brick_f4 *>(box + o);
            const brick_f4 c1 = *reinterpret_cast<const brick_f4 *>(box + o + 4);
            c[0] = (*reinterpret_cast<const brick_f4 *>(box + o - 4))[3];
            c[9] = (*reinterpret_cast<const brick_f4 *>(box + o + 8))[0];
#pragma unroll
            for (int e = 0; e < 4; ++e) c[1 + e] = c0[e], c[5 + e] = c1[e];
        }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int oh = o + 4 * hh;
            const brick_f4 ym = *reinterpret_cast<const brick_f4 *>(box + oh - SX);
            const brick_f4 yp = *reinterpret_cast<const brick_f4 *>(box + oh + SX);
            const brick_f4 zm = *reinterpret_cast<const brick_f4 *>(box + oh - SXY);
            const brick_f4 zp = *reinterpret_cast<const brick_f4 *>(box + oh + SXY);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = 4 * hh + q;
                const float cc = c[e + 1];
                const float sv = mode_speed<MODE, float, false>(f8[e], cc, c[e], c[e + 2], ym[q],
                                                                yp[q], zm[q], zp[q], a);
                const float uv = mode_finish<MODE, float, false>(
                    upwind_point<float, false>(cc, c[e], c[e + 2], ym[q], yp[q], zm[q], zp[q], sv,
                                               a.dx, a.dt, a.dtdx),
                    sv, a.dt, a.cut_gamma);
                emit(e, sv, uv, cc);
            }
        }
    };

    for (int w = w0; w < w1; ++w) {
        int rv = 0;
        if (lane < kItemWords) rv = a.rec[static_cast<int64_t>(w) * kItemWords + lane];
        const int t0 = __builtin_amdgcn_readlane(rv, 0);
        const int len = __builtin_amdgcn_readlane(rv, 1);
        const uint32_t m0 = __builtin_amdgcn_readlane(rv, 2), m1 = __builtin_amdgcn_readlane(rv, 3);
        const uint32_t m2 = __builtin_amdgcn_readlane(rv, 4), m3 = __builtin_amdgcn_readlane(rv, 5);
        const uint32_t mx = __builtin_amdgcn_readlane(rv, 6);
        const uint32_t dg = __builtin_amdgcn_readlane(rv, 7);
        if (t0 < 0 || t0 >= g.ntiles || len < 1 || len > kBrickRun) continue;  // uniform
        const uint32_t ut = static_cast<uint32_t>(t0);
        const uint32_t rr = ut / static_cast<uint32_t>(ntx);
        const int ti0 = static_cast<int>(ut - rr * static_cast<uint32_t>(ntx));
        const int tk = static_cast<int>(rr / static_cast<uint32_t>(nty));
        const int tj = static_cast<int>(rr) - tk * nty;
        const int nxr = 8 * len;
        const bool ex0 = ti0 == 0, ex1 = ti0 + len == ntx;
        const bool ey0 = tj == 0, ey1 = tj == nty - 1, ez0 = tk == 0, ez1 = tk == ntz - 1;

        // membership of the tile at offset (di, dj, dk) from tile l of the run
        // (di = -1 / +1: the tile before / after the run)
        auto member = [&](int l, int di, int dj, int dk) -> bool {
            if (di != 0) {
                if (dj == 0 && dk == 0) return (mx >> (di > 0 ? 1 : 0)) & 1u;
                const uint32_t e = (dg >> (di < 0 ? 16 : 20)) & 15u;
                return (e >> (dj < 0 ? 0 : dj > 0 ? 1 : dk < 0 ? 2 : 3)) & 1u;
            }
            if (dj == 0 && dk == 0) return true;
            if (dk == 0) return ((dj < 0 ? m0 : m1) >> l) & 1u;
            if (dj == 0) return ((dk < 0 ? m2 : m3) >> l) & 1u;
            return (dg >> (4 * l + (dj > 0 ? 2 : 0) + (dk > 0 ? 1 : 0))) & 1u;
        };
        // box coordinate v in [-2, 9] along y or z -> in-tile coordinate and
        // tile offset, clamped at the domain faces
        auto clampc = [](int v, bool lo_edge, bool hi_edge, int *d) {
            if (v < 0) {
                *d = lo_edge ? 0 : -1;
                return lo_edge ? 0 : v + 8;
            }
            if (v > 7) {
                *d = hi_edge ? 0 : 1;
                return hi_edge ? 7 : v - 8;
            }
            *d = 0;
            return v;
        };
        // element of the point at box (x, y, z) (x in [-2, nxr + 1]) in cur or orig
        auto src = [&](int x, int y, int z) -> const S * {
            int dj, dk, di = 0, l;
            const int yy = clampc(y, ey0, ey1, &dj), zz = clampc(z, ez0, ez1, &dk);
            int xx;
            if (x < 0) {
                l = 0;
                di = ex0 ? 0 : -1;
                xx = ex0 ? 0 : x + 8;
            } else if (x >= nxr) {
                l = len - 1;
                di = ex1 ? 0 : 1;
                xx = ex1 ? 7 : x - nxr;
            } else {
                l = x >> 3;
                xx = x & 7;
            }
            const int64_t ts = static_cast<int64_t>(t0) + l + di + dj * sy + dk * sz;
            const S *base = member(l, di, dj, dk) ? a.cur : a.orig;
            return base + ts * kBrick + zz * 64 + yy * 8 + xx;
        };

        // (1) global loads of the step-n values and of F
        const bool own_ok = ob < len;
        const int64_t obase = static_cast<int64_t>(t0 + ob) * kBrick + oz * 64 + oy * 8;
        BrickRow<S> own, face;
        brick_f4 fa = {0.f, 0.f, 0.f, 0.f}, fb = fa, rf = fa;
        if (own_ok) {
            own = BrickRow<S>::load(a.cur + obase);
            if constexpr (MODE < kReinit) {
                fa = *reinterpret_cast<const brick_f4 *>(a.F + obase);
                fb = *reinterpret_cast<const brick_f4 *>(a.F + obase + 4);
            }
        }
        const bool face_ok = fl < len;
        if (face_ok) face = BrickRow<S>::load(src(fl * 8, f_y, f_z));
        // y-z diagonal rows (threads 0..4 len - 1)
        const bool dg_ok = tid < 4 * len;
        const int dl = tid >> 2, de = tid & 3;
        const int d_y = (de & 2) ? 8 : -1, d_z = (de & 1) ? 8 : -1;
        BrickRow<S> drow;
        if (dg_ok) drow = BrickRow<S>::load(src(dl * 8, d_y, d_z));
        // x ends of the run's rows (threads 128..255): x = -2, -1 or nxr, nxr + 1
        const bool xe_ok = tid >= 128;
        float xe0 = 0.f, xe1 = 0.f;
        if (xe_ok) {
            const int x0 = xs ? nxr : -2;
            xe0 = val(src(x0, xy, xz), 0);
            xe1 = val(src(x0 + 1, xy, xz), 0);
        }
        // x ends of the ring rows (threads 16..79): x = -1 or nxr
        const int q = tid - 16;
        const bool xr_ok = q >= 0 && q < 64;
        const int qs = (q >> 5) & 1, qe = (q >> 3) & 3, qk = q & 7;
        const int q_y = qe == 0 ? -1 : qe == 1 ? 8 : qk, q_z = qe == 2 ? -1 : qe == 3 ? 8 : qk;
        const int q_x = qs ? nxr : -1;
        float xrv = 0.f;
        if (xr_ok) xrv = val(src(q_x, q_y, q_z), 0);
        // ring half-row of the first step: updated when its tile is in the band
        int rdj, rdk;
        const int rys = clampc(r_y, false, false, &rdj), rzs = clampc(r_z, false, false, &rdk);
        const bool r_inside = !((rdj < 0 && ey0) || (rdj > 0 && ey1) || (rdk < 0 && ez0) ||
                                (rdk > 0 && ez1));
        const bool r_upd = face_ok && r_inside && member(fl, 0, rdj, rdk);
        const int64_t rbase =
            (static_cast<int64_t>(t0) + fl + rdj * sy + rdk * sz) * kBrick + rzs * 64 + rys * 8 +
            rh * 4;
        if constexpr (MODE < kReinit)
            if (r_upd) rf = *reinterpret_cast<const brick_f4 *>(a.F + rbase);
        // x ring point of the first step (threads 0..127)
        const bool xp_thr = tid < 128;
        const bool x_inside = xs ? !ex1 : !ex0;
        const bool x_upd = xp_thr && x_inside && member(xs ? len - 1 : 0, xs ? 1 : -1, 0, 0);
        float xf = 0.f;
        if constexpr (MODE < kReinit)
            if (x_upd)
                xf = a.F[(static_cast<int64_t>(t0) + (xs ? len : -1)) * kBrick + xz * 64 +
                         xy * 8 + (xs ? 0 : 7)];

        // (2) the box
        const int o_own = bx(ob * 8, oy, oz);
        auto put8 = [&](int o, const BrickRow<S> &r) {
            *reinterpret_cast<brick_f4 *>(box + o) =
                brick_f4{r.value(0, sc), r.value(1, sc), r.value(2, sc), r.value(3, sc)};
            *reinterpret_cast<brick_f4 *>(box + o + 4) =
                brick_f4{r.value(4, sc), r.value(5, sc), r.value(6, sc), r.value(7, sc)};
        };
        if (own_ok) put8(o_own, own);
        if (face_ok) put8(bx(fl * 8, f_y, f_z), face);
        if (dg_ok) put8(bx(dl * 8, d_y, d_z), drow);
        if (xe_ok) {
            const int o = bx(xs ? nxr : -2, xy, xz);
            box[o] = xe0;
            box[o + 1] = xe1;
        }
        if (xr_ok) box[bx(q_x, q_y, q_z)] = xrv;
        __syncthreads();  // step-n box complete

        // (3) first step: the run's row, the ring half-row, the x ring point
        float s_own[8], s_ring[4], s_x = 0.f;
        if (own_ok) {
            const float f8[8] = {fa[0], fa[1], fa[2], fa[3], fb[0], fb[1], fb[2], fb[3]};
            row8(o_own, f8, [&](int e, float sv, float uv, float cc) {
                s_own[e] = kept(sv == 0.f ? cc : uv);
            });
        }
        const int o_ring = bx(r_x, r_y, r_z);
        if (r_upd) {
#pragma unroll
            for (int e = 0; e < 4; ++e) s_ring[e] = kept(point(o_ring + e, rf[e]));
        }
        const int o_xr = bx(xs ? nxr : -1, xy, xz);
        if (x_upd) s_x = kept(point(o_xr, xf));
        __syncthreads();  // every step-n value read
        if (own_ok) {
#pragma unroll
            for (int e = 0; e < 8; ++e) box[o_own + e] = s_own[e];
            // ring positions outside the grid: the clamped run point's new value
            if (oy == 0 && ey0)
                for (int e = 0; e < 8; ++e) box[o_own - SX + e] = s_own[e];
            if (oy == 7 && ey1)
                for (int e = 0; e < 8; ++e) box[o_own + SX + e] = s_own[e];
            if (oz == 0 && ez0)
                for (int e = 0; e < 8; ++e) box[o_own - SXY + e] = s_own[e];
            if (oz == 7 && ez1)
                for (int e = 0; e < 8; ++e) box[o_own + SXY + e] = s_own[e];
            if (ob == 0 && ex0) box[o_own - 1] = s_own[0];
            if (ob == len - 1 && ex1) box[o_own + 8] = s_own[7];
        }
        if (r_upd) {
#pragma unroll
            for (int e = 0; e < 4; ++e) box[o_ring + e] = s_ring[e];
        }
        if (x_upd) box[o_xr] = s_x;
        __syncthreads();  // step-(n+1) box complete

        // (4) second step on the run's row
        if (own_ok) {
            const float f8[8] = {fa[0], fa[1], fa[2], fa[3], fb[0], fb[1], fb[2], fb[3]};
            BrickRow<S> out;
            row8(o_own, f8, [&](int e, float sv, float uv, float cc) {
                if constexpr (std::is_same<S, float>::value)
                    out.set(e, sv == 0.f ? cc : uv);
                else
                    out.set(e, sv == 0.f ? (f8[e] == 0.f && MODE < kReinit
                                                ? own.raw(e)
                                                : Codec<S>::store(cc, sc))
                                         : Codec<S>::store(uv, sc));
            });
            out.store(a.nxt + obase);
        }
        __syncthreads();  // box free for the next item
    }
}

// listed runs of bricks copied from src to dst (the copy-back after an odd
// number of steps): item -> len contiguous tiles
template <class S>
__global__ __launch_bounds__(kBlock) void brick_copy_kernel(const S *__restrict__ src,
                                                            S *__restrict__ dst,
                                                            const int32_t *__restrict__ rec,
                                                            const int32_t *__restrict__ nitems,
                                                            int64_t ntiles) {
    int w0, w1;
    block_slice(0, *nitems, &w0, &w1);
    for (int w = w0; w < w1; ++w) {
        const int t0 = rec[static_cast<int64_t>(w) * kItemWords];
        const int len = rec[static_cast<int64_t>(w) * kItemWords + 1];
        if (t0 < 0 || t0 + len > ntiles || len < 1 || len > kBrickRun) continue;
        const int64_t base = static_cast<int64_t>(t0) * kBrick;
        if ((threadIdx.x >> 6) < len)
            BrickRow<S>::load(src + base + threadIdx.x * 8).store(dst + base + threadIdx.x * 8);
    }
}

// ---------------------------------------------------------------------------
// host side

// Grids the brick kernels take: 8^3 tiles, whole tiles on every axis, 16-byte
// aligned buffers.
static int brick_geom(const ls_grid *grid, Geom *G, const char *what) {
    int rc = make_geom(grid, G);
    if (rc != LS_OK) return rc;
    if (G->tx != 8 || G->ty != 8 || G->tz != 8) {
        set_error("%s: brick layout needs 8x8x8 tiles (got %dx%dx%d)", what, G->tx, G->ty, G->tz);
        return LS_ERR_UNSUPPORTED;
    }
    if (G->nx % 8 || G->ny % 8 || G->nz % 8) {
        set_error("%s: brick layout needs whole tiles (dims multiples of 8, got %dx%dx%d)", what,
                  G->nx, G->ny, G->nz);
        return LS_ERR_UNSUPPORTED;
    }
    if (G->ntiles > INT32_MAX / kBrick || G->nty > 65535 || G->ntz > 65535) {
        set_error("%s: grid too large for the brick kernels", what);
        return LS_ERR_UNSUPPORTED;
    }
    // the plan of the brick kernels: runs of 4 tiles, whatever the launch tuning
    G->elem_bytes = 4;
    G->run_tiles = kBrickRun;
    return LS_OK;
}

static bool aligned16(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

template <class S>
static int brick_convert(const S *src, const ls_grid *grid, S *dst, bool to_brick, void *stream_) {
    Geom G;
    int rc = brick_geom(grid, &G, to_brick ? "bricks from dense" : "bricks to dense");
    if (rc != LS_OK) return rc;
    if (!src || !dst) {
        set_error("brick conversion: src and dst must be non-NULL");
        return LS_ERR_ARG;
    }
    if (src == dst) {
        set_error("brick conversion: src and dst must be distinct buffers");
        return LS_ERR_ARG;
    }
    if (!aligned16(src) || !aligned16(dst)) {
        set_error("brick conversion: buffers must be 16-byte aligned");
        return LS_ERR_ARG;
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const dim3 grid3(static_cast<unsigned>(cdiv64(G.ntx, 4)), G.nty, G.ntz);
    if (to_brick)
        hipLaunchKernelGGL((brick_convert_kernel<S, true>), grid3, dim3(kBlock), 0, stream, src,
                           dst, G.nx, G.ny, G.ntx, G.nty);
    else
        hipLaunchKernelGGL((brick_convert_kernel<S, false>), grid3, dim3(kBlock), 0, stream, src,
                           dst, G.nx, G.ny, G.ntx, G.nty);
    LS_LAUNCH_CHECK("brick_convert_kernel");
    return LS_OK;
}

static int flag_blocks(int64_t n) {
    DeviceInfo di;
    if (device_info(&di) != LS_OK) return -1;
    return static_cast<int>(std::max<int64_t>(
        1, std::min<int64_t>(cdiv64(n, kBlock / 64), int64_t(di.cus) * 16)));
}

// Band build (list == nullptr: full scan) or exact incremental rebuild from
// the previous list, on bricks; then the dilation, the list and the plan.
template <class S>
static int brick_band(const S *phi, float scale, const Geom &G, typename Codec<S>::C gamma,
                      int dilate, const int32_t *prev, const int32_t *prev_n, int32_t *tiles,
                      int32_t *ntiles_dev, uint8_t *ws, hipStream_t stream, TileAccum acc) {
    const Workspace w = workspace_layout(G);
    const int blocks = flag_blocks(prev ? G.ntiles : G.ntiles);
    if (blocks < 0) return LS_ERR_HIP;
    int64_t slot;
    int rc;
    if ((rc = stats_before(LS_KERNEL_BAND_FLAG, stream, &slot)) != LS_OK) return rc;
    hipLaunchKernelGGL(brick_flag_kernel<S>, dim3(blocks), dim3(kBlock), 0, stream, phi, G.ntiles,
                       gamma, scale, prev, prev_n, ws + w.a_flags);
    LS_LAUNCH_CHECK("brick_flag_kernel");
    if ((rc = stats_after(LS_KERNEL_BAND_FLAG, stream, slot)) != LS_OK) return rc;
    return band_finish(G, ws, dilate, tiles, ntiles_dev, stream, acc);
}

static StepGeom brick_step_geom(const Geom &G) {
    StepGeom s{};
    s.nx = G.nx, s.ny = G.ny, s.nz = G.nz;
    s.tx = s.ty = s.tz = 8;
    s.ntx = G.ntx, s.nty = G.nty, s.ntz = G.ntz;
    s.ntiles = static_cast<int>(G.ntiles);
    s.R = kBrickRun;
    return s;
}

// workgroups per compute unit of the step launches: 32, and 64 on grids of
// 2^21 tiles or more (1024^3), whose bands stream from HBM: there more blocks
// in flight hide more of the memory latency (1024^3 FP32: 255 against 261 us
// per launch; at 512^3, cache-resident, 64 was 2 % slower and 16 the same)
constexpr int kBrickBlocksPerCu = 32, kBrickBlocksPerCuLarge = 64;
constexpr int64_t kBrickLargeTiles = int64_t(1) << 21;

// Two steps per launch in the brick driver (ls_tuning.temporal: 1 on, 2 off;
// 0 auto: on for FP32, off for FP16s, whose two-step launch is VALU-heavier
// by the decode and re-rounding of its ring values and measured slower);
// results do not depend on it.
int brick_temporal_mode();  // ls_step.hip
template <class S>
static bool brick_two_step() {
    const int m = brick_temporal_mode();
    return m == 1 || (m == 0 && sizeof(S) == 4);
}

static int brick_grid(int64_t ntiles) {
    DeviceInfo di;
    if (device_info(&di) != LS_OK) return -1;
    const int per_cu = ntiles >= kBrickLargeTiles ? kBrickBlocksPerCuLarge : kBrickBlocksPerCu;
    const int64_t g64 = std::min<int64_t>(int64_t(di.cus) * per_cu, ntiles + 7);
    return static_cast<int>(std::max<int64_t>(8, g64 - g64 % 8));
}

// n launches of the brick step of mode MODE on the plan held by the workspace,
// ping-ponging between phi and scratch (orig = phi: the values outside the
// band are never written there), then the copy-back of the band when n is odd;
// the last launch takes mode LAST (the clamp of the reinitialisation).
template <class S, int MODE, int LAST>
static int brick_launch(S *phi, S *scratch, const float *F, float scale, const Geom &G,
                        typename Codec<S>::C dx, typename Codec<S>::C dt,
                        typename Codec<S>::C beta, typename Codec<S>::C gamma, int n,
                        uint8_t *ws, hipStream_t stream, int stats_kind) {
    using C = typename Codec<S>::C;
    if (n == 0) return LS_OK;
    const Workspace w = workspace_layout(G);
    const StepGeom sg = brick_step_geom(G);
    StepArgs<S, float> a{};
    a.orig = phi;
    a.F = F;
    a.rec = reinterpret_cast<int32_t *>(ws + w.items);
    a.nitems = reinterpret_cast<int32_t *>(ws + w.counters);
    a.dx = dx;
    a.dt = dt;
    a.dtdx = static_cast<C>(static_cast<double>(dt) / static_cast<double>(dx));
    a.scale = scale;
    a.cut_beta = beta;
    a.cut_gamma = gamma;
    if (MODE == kCutoff)
        a.cut_k = static_cast<C>(1.0 / (static_cast<double>(gamma) - static_cast<double>(beta)));
    const int nblocks = brick_grid(G.ntiles);
    if (nblocks < 0) return LS_ERR_HIP;
    // pairs of steps in one launch (temporal blocking) for every step before
    // the last one of another mode, the rest one step per launch; one pair
    // fewer where that makes the launch count even, since an odd count ends
    // in scratch and costs a copy-back of the band (at 512^3 FP32 two
    // one-step launches take 49 us, a two-step launch and the copy 61 us)
    const int body = n - (LAST != MODE ? 1 : 0);
    int pairs = brick_two_step<S>() ? body / 2 : 0;
    if (pairs > 0 && (n - pairs) % 2 != 0) --pairs;
    const int launches = n - pairs;
    int64_t slot;
    int rc;
    if ((rc = stats_before(stats_kind, stream, &slot, launches)) != LS_OK) return rc;
    for (int l = 0; l < launches; ++l) {
        a.cur = (l & 1) ? scratch : phi;
        a.nxt = (l & 1) ? phi : scratch;
        if (l < pairs)
            hipLaunchKernelGGL((brick_step2_kernel<S, MODE>), dim3(nblocks), dim3(kBlock),
                               Brick2Box::lds, stream, sg, a);
        else if (l == launches - 1)
            hipLaunchKernelGGL((brick_step_kernel<S, LAST>), dim3(nblocks), dim3(kBlock),
                               BrickBox::lds, stream, sg, a);
        else
            hipLaunchKernelGGL((brick_step_kernel<S, MODE>), dim3(nblocks), dim3(kBlock),
                               BrickBox::lds, stream, sg, a);
        LS_LAUNCH_CHECK("brick_step_kernel");
    }
    if ((rc = stats_after(stats_kind, stream, slot)) != LS_OK) return rc;
    if (launches & 1) {
        hipLaunchKernelGGL(brick_copy_kernel<S>, dim3(nblocks), dim3(kBlock), 0, stream,
                           static_cast<const S *>(scratch), phi, a.rec, a.nitems, G.ntiles);
        LS_LAUNCH_CHECK("brick_copy_kernel");
    }
    return LS_OK;
}

// The windowed driver (Steps 1-3 of Sec. 1.1) on bricks: per window a band
// build (full scan first, then the exact incremental rebuild from the
// previous band), `window` steps (plain, or with the cut-off of Eq. 8 when
// beta > 0), then reinit_iters reinitialisation steps and the clamp.
template <class S>
static int brick_run(S *phi, const float *F, float scale, const ls_grid *grid,
                     typename Codec<S>::C dx, typename Codec<S>::C dt, typename Codec<S>::C gamma,
                     int nsteps, int window, typename Codec<S>::C beta, int reinit_iters,
                     typename Codec<S>::C dtau, int32_t *tiles, int64_t capacity,
                     int32_t *ntiles_dev, int64_t *tile_steps_dev, S *scratch, void *workspace,
                     int64_t ws_bytes, void *stream_) {
    using C = typename Codec<S>::C;
    Geom G;
    int rc = brick_geom(grid, &G, "band run (bricks)");
    if (rc != LS_OK) return rc;
    if (!phi || !F || !scratch || !tiles || !ntiles_dev) {
        set_error("band run (bricks): phi, F, scratch, tiles and ntiles_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (phi == scratch) {
        set_error("band run (bricks): phi and scratch must be distinct buffers");
        return LS_ERR_ARG;
    }
    if (!aligned16(phi) || !aligned16(F) || !aligned16(scratch)) {
        set_error("band run (bricks): phi, F and scratch must be 16-byte aligned");
        return LS_ERR_ARG;
    }
    if (nsteps < 0 || window <= 0) {
        set_error("band run (bricks): need nsteps >= 0 and window > 0");
        return LS_ERR_ARG;
    }
    if (!(dx > C(0)) || !(dt >= C(0)) || !(dx < C(INFINITY)) || !(dt < C(INFINITY))) {
        set_error("band run (bricks): need dx > 0 and dt >= 0, finite");
        return LS_ERR_ARG;
    }
    if (!(gamma == gamma)) {
        set_error("band run (bricks): gamma is NaN");
        return LS_ERR_ARG;
    }
    const bool cut = beta != C(0);
    if (cut && !(beta > C(0) && beta < gamma && gamma < C(INFINITY))) {
        set_error("band run (bricks): the cut-off needs 0 < beta < gamma < inf (beta = 0: none)");
        return LS_ERR_ARG;
    }
    if (reinit_iters < 0 || !(dtau >= C(0)) || !(dtau < C(INFINITY)) ||
        (reinit_iters > 0 && !(gamma > C(0) && gamma < C(INFINITY)))) {
        set_error("band run (bricks): need reinit_iters >= 0, dtau >= 0 finite and, with "
                  "reinitialisation, a positive finite gamma");
        return LS_ERR_ARG;
    }
    if (capacity < G.ntiles) {
        set_error("band run (bricks): capacity %lld < %lld tiles", (long long)capacity,
                  (long long)G.ntiles);
        return LS_ERR_CAPACITY;
    }
    if ((rc = check_workspace(G, workspace, ws_bytes)) != LS_OK) return rc;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const Workspace w = workspace_layout(G);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    int32_t *lists[2] = {tiles, reinterpret_cast<int32_t *>(ws + w.prev_list)};
    int32_t *counts[2] = {ntiles_dev, reinterpret_cast<int32_t *>(ws + w.counters) + 1};
    const int nwin = (nsteps + window - 1) / window;
    for (int k = 0; k < nwin; ++k) {
        const int n = std::min(window, nsteps - k * window);
        const int cur = (nwin - 1 - k) & 1;  // the last window writes lists[0]
        const TileAccum acc{tile_steps_dev, n};
        rc = brick_band<S>(phi, scale, G, gamma, 1, k == 0 ? nullptr : lists[cur ^ 1],
                           k == 0 ? nullptr : counts[cur ^ 1], lists[cur], counts[cur], ws,
                           stream, acc);
        if (rc != LS_OK) return rc;
        rc = cut ? brick_launch<S, kCutoff, kCutoff>(phi, scratch, F, scale, G, dx, dt, beta,
                                                     gamma, n, ws, stream, LS_KERNEL_UPWIND)
                 : brick_launch<S, kPlain, kPlain>(phi, scratch, F, scale, G, dx, dt, C(0),
                                                   C(0), n, ws, stream, LS_KERNEL_UPWIND);
        if (rc != LS_OK) return rc;
        rc = brick_launch<S, kReinit, kReinitClamp>(phi, scratch, nullptr, scale, G, dx, dtau,
                                                    C(0), gamma, reinit_iters, ws, stream,
                                                    LS_KERNEL_REINIT);
        if (rc != LS_OK) return rc;
    }
    return LS_OK;
}

template <class S>
static int brick_build(const S *phi, float scale, const ls_grid *grid, typename Codec<S>::C gamma,
                       int dilate, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                       void *workspace, int64_t ws_bytes, void *stream_) {
    Geom G;
    int rc = brick_geom(grid, &G, "band build (bricks)");
    if (rc != LS_OK) return rc;
    if (!phi || !tiles || !ntiles_dev) {
        set_error("band build (bricks): phi, tiles and ntiles_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (!aligned16(phi)) {
        set_error("band build (bricks): phi must be 16-byte aligned");
        return LS_ERR_ARG;
    }
    if (dilate != 0 && dilate != 1) {
        set_error("band build (bricks): dilate must be 0 or 1 (got %d)", dilate);
        return LS_ERR_ARG;
    }
    if (!(gamma == gamma)) {
        set_error("band build (bricks): gamma is NaN");
        return LS_ERR_ARG;
    }
    if (capacity < G.ntiles) {
        set_error("band build (bricks): capacity %lld < %lld tiles", (long long)capacity,
                  (long long)G.ntiles);
        return LS_ERR_CAPACITY;
    }
    if ((rc = check_workspace(G, workspace, ws_bytes)) != LS_OK) return rc;
    return brick_band<S>(phi, scale, G, gamma, dilate, nullptr, nullptr, tiles, ntiles_dev,
                         static_cast<uint8_t *>(workspace), static_cast<hipStream_t>(stream_),
                         TileAccum{});
}

static int check_scale(float scale, const char *what) {
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        set_error("%s: scale must be positive and finite", what);
        return LS_ERR_ARG;
    }
    return LS_OK;
}

}  // namespace ls

extern "C" {

int ls_bricks_from_dense_f32(const float *src, const ls_grid *g, float *dst, void *stream) {
    ls::clear_error();
    return ls::brick_convert<float>(src, g, dst, true, stream);
}

int ls_bricks_to_dense_f32(const float *src, const ls_grid *g, float *dst, void *stream) {
    ls::clear_error();
    return ls::brick_convert<float>(src, g, dst, false, stream);
}

int ls_bricks_from_dense_f16s(const uint16_t *src, const ls_grid *g, uint16_t *dst,
                              void *stream) {
    ls::clear_error();
    return ls::brick_convert<uint16_t>(src, g, dst, true, stream);
}

int ls_bricks_to_dense_f16s(const uint16_t *src, const ls_grid *g, uint16_t *dst, void *stream) {
    ls::clear_error();
    return ls::brick_convert<uint16_t>(src, g, dst, false, stream);
}

int ls_band_build_bricks_f32(const float *phi_b, const ls_grid *g, float gamma, int dilate,
                             int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                             void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::brick_build<float>(phi_b, 1.0f, g, gamma, dilate, tiles, capacity, ntiles_dev,
                                  workspace, workspace_bytes, stream);
}

int ls_band_build_bricks_f16s(const uint16_t *phi_b, float scale, const ls_grid *g, float gamma,
                              int dilate, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                              void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    int rc = ls::check_scale(scale, "band build (bricks) f16s");
    if (rc != LS_OK) return rc;
    return ls::brick_build<uint16_t>(phi_b, scale, g, gamma, dilate, tiles, capacity, ntiles_dev,
                                     workspace, workspace_bytes, stream);
}

int ls_band_run_bricks_f32(float *phi_b, const float *F_b, const ls_grid *g, float dx, float dt,
                           float gamma, int nsteps, int window, float beta, int reinit_iters,
                           float dtau, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                           int64_t *tile_steps_dev, float *scratch_b, void *workspace,
                           int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::brick_run<float>(phi_b, F_b, 1.0f, g, dx, dt, gamma, nsteps, window, beta,
                                reinit_iters, dtau, tiles, capacity, ntiles_dev, tile_steps_dev,
                                scratch_b, workspace, workspace_bytes, stream);
}

int ls_band_run_bricks_f16s(uint16_t *phi_b, float scale, const float *F_b, const ls_grid *g,
                            float dx, float dt, float gamma, int nsteps, int window, float beta,
                            int reinit_iters, float dtau, int32_t *tiles, int64_t capacity,
                            int32_t *ntiles_dev, int64_t *tile_steps_dev, uint16_t *scratch_b,
                            void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    int rc = ls::check_scale(scale, "band run (bricks) f16s");
    if (rc != LS_OK) return rc;
    return ls::brick_run<uint16_t>(phi_b, F_b, scale, g, dx, dt, gamma, nsteps, window, beta,
                                   reinit_iters, dtau, tiles, capacity, ntiles_dev,
                                   tile_steps_dev, scratch_b, workspace, workspace_bytes, stream);
}

}  // extern "C"
