// Batched narrow-band update: many level-set grids of uneven size advanced in
// lockstep by the same kernels, each launch covering every grid.
//
// The grids' tile grids are concatenated into one global tile space (grid i
// owns global tiles [tile_base_i, tile_base_i + ntiles_i)), so the band build
// of all grids is one flag pass, one dilation pass and one ordered
// compaction, and the band list / work items of all grids are one list each.
// Grids are ordered by tile shape (a "group"); the items of a group are
// contiguous, and each group's step is one launch of the fast kernel compiled
// for that shape, reading each item's grid from the descriptor table.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ls_compact.h"
#include "ls_stats.h"
#include "ls_stencil.h"

namespace ls {

int plan_run_tiles(const Geom &g);                               // ls_step.hip
int fill_zero(uint8_t *p, int64_t bytes, hipStream_t stream);   // ls_band.hip

constexpr int kMaxGroups = 16;
// workgroups per CU of a group's step launch: more blocks in flight put more
// of the halo rows neighbouring blocks read in L2 (on the 256-grid batch: 32
// per CU 199.2 GLUPS, 64 206.8, 128 207.8)
constexpr int kBatchBlocksPerCu = 64;

// ---------------------------------------------------------------------------
// host layout (deterministic: the same instance array gives the same layout)

struct Shape4 {
    int tx, ty, tz, R;
    bool operator<(const Shape4 &o) const {
        return std::tie(tx, ty, tz, R) < std::tie(o.tx, o.ty, o.tz, o.R);
    }
};

static bool fast_shape(const Shape4 &s) {
    static const Shape4 ok[] = {{8, 8, 8, 4}, {8, 8, 8, 2},  {16, 4, 4, 2}, {16, 4, 4, 4},
                                {32, 4, 4, 1}, {32, 4, 4, 2}, {16, 8, 8, 2}, {4, 4, 4, 8}};
    for (const auto &k : ok)
        if (k.tx == s.tx && k.ty == s.ty && k.tz == s.tz && k.R == s.R) return true;
    return false;
}

struct Group {
    Shape4 shape;
    int first, end;  // internal instance range
    int32_t tile_base;
};

struct BatchLayout {
    std::vector<BatchInst> inst;  // internal order (by group)
    std::vector<int> given;       // internal index -> caller's index
    std::vector<Group> groups;
    int64_t total_tiles = 0, total_slabs = 0;
    int max_ntx = 0;
    int64_t max_points = 0;       // largest offset + grid size (elements)
};

static int make_layout(const ls_instance *in, int n, BatchLayout *L) {
    if (!in || n <= 0) {
        set_error("batch: need a non-NULL array of at least one instance");
        return LS_ERR_ARG;
    }
    std::vector<std::pair<Shape4, int>> key(n);
    std::vector<Geom> geo(n);
    for (int i = 0; i < n; ++i) {
        int rc = make_geom(&in[i].grid, &geo[i]);
        if (rc != LS_OK) return rc;
        if (in[i].offset < 0) {
            set_error("batch: instance %d has a negative offset", i);
            return LS_ERR_ARG;
        }
        if (!(in[i].dx > 0.f) || !(in[i].dt >= 0.f) || !(in[i].gamma == in[i].gamma) ||
            !(in[i].dx < INFINITY) || !(in[i].dt < INFINITY)) {
            set_error("batch: instance %d needs dx > 0, dt >= 0 (finite) and gamma not NaN", i);
            return LS_ERR_ARG;
        }
        const Shape4 s{geo[i].tx, geo[i].ty, geo[i].tz, plan_run_tiles(geo[i])};
        if (!fast_shape(s)) {
            set_error("batch: tile shape %dx%dx%d (run of %d tiles) of instance %d is not one "
                      "of the batched kernel shapes", s.tx, s.ty, s.tz, s.R, i);
            return LS_ERR_UNSUPPORTED;
        }
        if (in[i].pitch != 0 && in[i].pitch < geo[i].nx) {
            set_error("batch: instance %d has pitch %d < nx = %d", i, in[i].pitch, geo[i].nx);
            return LS_ERR_ARG;
        }
        const int64_t px = in[i].pitch ? in[i].pitch : geo[i].nx;
        if (static_cast<int64_t>(geo[i].tz + 1) * geo[i].ny * px >= (int64_t(1) << 31)) {
            set_error("batch: instance %d is too large", i);
            return LS_ERR_UNSUPPORTED;
        }
        key[i] = {s, i};
    }
    auto pitch_of = [&](int i) -> int64_t { return in[i].pitch ? in[i].pitch : geo[i].nx; };
    auto span_of = [&](int i) -> int64_t {
        return pitch_of(i) * geo[i].ny * static_cast<int64_t>(geo[i].nz);
    };
    // check the grids do not overlap in the buffers
    std::vector<std::pair<int64_t, int64_t>> spans(n);
    for (int i = 0; i < n; ++i) spans[i] = {in[i].offset, in[i].offset + span_of(i)};
    std::sort(spans.begin(), spans.end());
    for (int i = 1; i < n; ++i)
        if (spans[i].first < spans[i - 1].second) {
            set_error("batch: instances overlap in the phi/F buffers");
            return LS_ERR_ARG;
        }
    std::stable_sort(key.begin(), key.end(),
                     [](const auto &a, const auto &b) { return a.first < b.first; });
    L->inst.resize(n);
    L->given.resize(n);
    int64_t tiles = 0, slabs = 0;
    for (int k = 0; k < n; ++k) {
        const int i = key[k].second;
        const Geom &g = geo[i];
        if (L->groups.empty() || L->groups.back().shape < key[k].first ||
            key[k].first < L->groups.back().shape) {
            if (static_cast<int>(L->groups.size()) == kMaxGroups) {
                set_error("batch: more than %d tile shapes", kMaxGroups);
                return LS_ERR_UNSUPPORTED;
            }
            L->groups.push_back({key[k].first, k, k, static_cast<int32_t>(tiles)});
        }
        L->groups.back().end = k + 1;
        BatchInst b;
        std::memset(&b, 0, sizeof(b));
        b.offset = in[i].offset;
        b.nx = g.nx, b.ny = g.ny, b.nz = g.nz;
        b.tx = g.tx, b.ty = g.ty, b.tz = g.tz;
        b.ntx = g.ntx, b.nty = g.nty, b.ntz = g.ntz;
        b.tile_base = static_cast<int32_t>(tiles);
        b.ntiles = static_cast<int32_t>(g.ntiles);
        b.R = key[k].first.R;
        b.slab_base = static_cast<int32_t>(slabs);
        b.px = static_cast<int32_t>(pitch_of(i));
        b.vec_ok = (g.nx % 4 == 0 && b.px % 4 == 0 && in[i].offset % 4 == 0) ? 1 : 0;
        b.dx = in[i].dx;
        b.dt = in[i].dt;
        b.dtdx = static_cast<float>(static_cast<double>(in[i].dt) / static_cast<double>(in[i].dx));
        b.gamma = in[i].gamma;
        b.group = static_cast<int32_t>(L->groups.size() - 1);
        L->inst[k] = b;
        L->given[k] = i;
        tiles += g.ntiles;
        slabs += static_cast<int64_t>(g.nty) * g.ntz;
        L->max_ntx = std::max(L->max_ntx, g.ntx);
        L->max_points = std::max(L->max_points, in[i].offset + span_of(i));
        if (tiles > INT32_MAX - kCompactChunk || slabs > INT32_MAX) {
            set_error("batch: too many tiles in total");
            return LS_ERR_UNSUPPORTED;
        }
    }
    L->total_tiles = tiles;
    L->total_slabs = slabs;
    if (L->max_ntx > 65536) {
        set_error("batch: more than 65536 tiles along x unsupported");
        return LS_ERR_UNSUPPORTED;
    }
    return LS_OK;
}

static int64_t a256(int64_t v) { return (v + 255) & ~int64_t(255); }

struct BatchWs {
    int64_t inst, group_base, ranges, a_flags, u_map, blk, blk2, items, list0, list1, counters;
    int64_t total;
    int64_t nblk;
};

static BatchWs batch_ws(const BatchLayout &L) {
    BatchWs w;
    const int64_t T = L.total_tiles;
    w.nblk = cdiv64(T, kCompactChunk);
    int64_t o = 0;
    w.inst = o;       o = a256(o + sizeof(BatchInst) * L.inst.size());
    w.group_base = o; o = a256(o + 4 * (kMaxGroups + 1));
    w.ranges = o;     o = a256(o + 4 * (kMaxGroups + 1));
    w.a_flags = o;    o = a256(o + T);
    w.u_map = o;      o = a256(o + T);
    w.blk = o;        o = a256(o + 4 * (w.nblk + 1));
    w.blk2 = o;       o = a256(o + 4 * (w.nblk + 1));
    w.items = o;      o = a256(o + 4 * kItemWords * T);
    w.list0 = o;      o = a256(o + 4 * T);
    w.list1 = o;      o = a256(o + 4 * T);
    w.counters = o;   o = a256(o + 4 * 64);  // [0] nitems, [1] count of list0, [2] of list1
    w.total = o;
    return w;
}

// ---------------------------------------------------------------------------
// device helpers

// Index of the grid whose field `base` range contains key (bases ascending).
__device__ inline int find_inst(const BatchInst *inst, int n, int key, bool by_slab) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int b = by_slab ? inst[mid].slab_base : inst[mid].tile_base;
        if (b <= key) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Tile flags of every grid: one block per (grid, tj, tk) slab of grid rows.
__global__ __launch_bounds__(kBlock) void batch_flag_kernel(const float *__restrict__ phi,
                                                            const BatchInst *__restrict__ inst,
                                                            int n, uint8_t *__restrict__ a_flags) {
    extern __shared__ uint8_t sflag[];
    const int slab = blockIdx.x;
    const BatchInst &d = inst[find_inst(inst, n, slab, true)];
    const int local = slab - d.slab_base;
    const int tj = local % d.nty, tk = local / d.nty;
    for (int t = threadIdx.x; t < d.ntx; t += kBlock) sflag[t] = 0;
    __syncthreads();
    const int j0 = tj * d.ty, k0 = tk * d.tz;
    const int rows_y = min(d.ty, d.ny - j0), rows_z = min(d.tz, d.nz - k0);
    const int nrows = rows_y * rows_z;
    const float *p = phi + d.offset;
    if (d.vec_ok) {
        const int nvec = d.nx >> 2;
        for (int q = threadIdx.x; q < nrows * nvec; q += kBlock) {
            const int r = q / nvec, c = q - r * nvec;
            const int jj = r % rows_y, kk = r / rows_y;
            const float4 v = *reinterpret_cast<const float4 *>(
                p + (static_cast<int64_t>(k0 + kk) * d.ny + (j0 + jj)) * d.px + 4 * c);
            if (fabsf(v.x) < d.gamma) sflag[(4 * c) / d.tx] = 1;
            if (fabsf(v.y) < d.gamma) sflag[(4 * c + 1) / d.tx] = 1;
            if (fabsf(v.z) < d.gamma) sflag[(4 * c + 2) / d.tx] = 1;
            if (fabsf(v.w) < d.gamma) sflag[(4 * c + 3) / d.tx] = 1;
        }
    } else {
        for (int q = threadIdx.x; q < nrows * d.nx; q += kBlock) {
            const int r = q / d.nx, c = q - r * d.nx;
            const int jj = r % rows_y, kk = r / rows_y;
            const float v = p[(static_cast<int64_t>(k0 + kk) * d.ny + (j0 + jj)) * d.px + c];
            if (fabsf(v) < d.gamma) sflag[c / d.tx] = 1;
        }
    }
    __syncthreads();
    uint8_t *dst = a_flags + d.tile_base + (static_cast<int64_t>(tk) * d.nty + tj) * d.ntx;
    for (int t = threadIdx.x; t < d.ntx; t += kBlock) dst[t] = sflag[t];
}

// Tile flags of the listed (global) tiles only: one wave per tile.  Tiles
// with power-of-two x and y extents (every shape the batched step is compiled
// for) are read 512 points at a time, all eight loads of a lane issued before
// any is tested; other shapes take a plain loop.
__global__ __launch_bounds__(kBlock) void batch_flag_list_kernel(
    const float *__restrict__ phi, const BatchInst *__restrict__ inst, int n, int total_tiles,
    const int32_t *__restrict__ list, const int32_t *__restrict__ list_count,
    uint8_t *__restrict__ a_flags) {
    const int cnt = min(*list_count, total_tiles);
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (kBlock / 64);
    for (int p = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); p < cnt; p += waves) {
        const int gt = list[p];
        if (gt < 0 || gt >= total_tiles) continue;  // uniform per wave
        const BatchInst &d = inst[find_inst(inst, n, gt, false)];
        const int t = gt - d.tile_base;
        const int ti = t % d.ntx, r = t / d.ntx;
        const int tj = r % d.nty, tk = r / d.nty;
        const int x0 = ti * d.tx, y0 = tj * d.ty, z0 = tk * d.tz;
        const int W = min(d.tx, d.nx - x0), H = min(d.ty, d.ny - y0), D = min(d.tz, d.nz - z0);
        const float *ph = phi + d.offset + (static_cast<int64_t>(z0) * d.ny + y0) * d.px + x0;
        const int64_t plane = static_cast<int64_t>(d.ny) * d.px;
        bool hit = false;
        if (((d.tx & (d.tx - 1)) | (d.ty & (d.ty - 1))) == 0) {
            const int sx = __ffs(d.tx) - 1, sy = __ffs(d.ty) - 1;
            const int box = d.tx * d.ty * d.tz;
            for (int q0 = 0; q0 < box; q0 += 512) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = q0 + u * 64 + lane;
                    const int lx = q & (d.tx - 1), rr = q >> sx;
                    const int ly = rr & (d.ty - 1), lz = rr >> sy;
                    v[u] = INFINITY;
                    if (q < box && lx < W && ly < H && lz < D)
                        v[u] = ph[lz * plane + static_cast<int64_t>(ly) * d.px + lx];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) hit |= fabsf(v[u]) < d.gamma;
            }
        } else {
            for (int q = lane; q < W * H * D; q += 64) {
                const int lx = q % W, rr = q / W;
                const int ly = rr % H, lz = rr / H;
                hit |= fabsf(ph[lz * plane + static_cast<int64_t>(ly) * d.px + lx]) < d.gamma;
            }
        }
        const bool any = __ballot(hit) != 0;
        if (lane == 0) a_flags[gt] = any ? 1 : 0;
    }
}

// U = A grown by one tile in all 26 directions, inside each grid.
__global__ __launch_bounds__(kBlock) void batch_dilate_kernel(const uint8_t *__restrict__ a,
                                                              uint8_t *__restrict__ u,
                                                              const BatchInst *__restrict__ inst,
                                                              int n, int total_tiles) {
    for (int gt = blockIdx.x * kBlock + threadIdx.x; gt < total_tiles; gt += gridDim.x * kBlock) {
        const BatchInst &d = inst[find_inst(inst, n, gt, false)];
        const int t = gt - d.tile_base;
        const int ti = t % d.ntx, r = t / d.ntx;
        const int tj = r % d.nty, tk = r / d.nty;
        const uint8_t *ab = a + d.tile_base;
        uint8_t hit = 0;
        for (int dk = -1; dk <= 1; ++dk) {
            const int k = tk + dk;
            if (k < 0 || k >= d.ntz) continue;
            for (int dj = -1; dj <= 1; ++dj) {
                const int j = tj + dj;
                if (j < 0 || j >= d.nty) continue;
                const uint8_t *row = ab + (static_cast<int64_t>(k) * d.nty + j) * d.ntx;
                hit |= row[ti];
                if (ti > 0) hit |= row[ti - 1];
                if (ti + 1 < d.ntx) hit |= row[ti + 1];
            }
        }
        u[gt] = hit ? 1 : 0;
    }
}

struct BatchHeadPred {
    const uint8_t *umap;
    const BatchInst *inst;
    int n;
    __device__ bool operator()(int64_t gt) const {
        if (!umap[gt]) return false;
        const BatchInst &d = inst[find_inst(inst, n, static_cast<int>(gt), false)];
        const int ti = static_cast<int>((gt - d.tile_base) % d.ntx);
        return ti % d.R == 0 || !umap[gt - 1];
    }
};

struct EmitHeadGlobal {
    int32_t *rec;
    __device__ void operator()(int pos, int64_t gt) const {
        rec[static_cast<int64_t>(pos) * kItemWords + 7] = static_cast<int32_t>(gt);
    }
};

// First item of every group: the first record whose head tile is at or past
// the group's first global tile (records are in ascending tile order).
__global__ void batch_range_kernel(const int32_t *__restrict__ rec, const int32_t *nitems,
                                   const int32_t *__restrict__ group_base, int ngroups,
                                   int32_t *__restrict__ ranges) {
    const int g = threadIdx.x;
    const int m = *nitems;
    if (g < ngroups) {
        const int key = group_base[g];
        int lo = 0, hi = m;  // first index with head >= key
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rec[static_cast<int64_t>(mid) * kItemWords + 7] < key) lo = mid + 1; else hi = mid;
        }
        ranges[g] = lo;
    }
    if (g == 0) ranges[ngroups] = m;
}

// Record of an item in grid-local terms: [0] local first tile, [1] run length,
// [2..5] y-/y+/z-/z+ neighbour bits per tile, [6] x-/x+ bits, [7] grid index.
__global__ __launch_bounds__(kBlock) void batch_record_kernel(int32_t *__restrict__ rec,
                                                              const int32_t *nitems,
                                                              const uint8_t *__restrict__ umap,
                                                              const BatchInst *__restrict__ inst,
                                                              int n) {
    const int m = *nitems;
    for (int pos = blockIdx.x * kBlock + threadIdx.x; pos < m; pos += gridDim.x * kBlock) {
        int32_t *o = rec + static_cast<int64_t>(pos) * kItemWords;
        const int gt = o[7];
        const int i = find_inst(inst, n, gt, false);
        const BatchInst &d = inst[i];
        const uint8_t *u = umap + d.tile_base;
        const int t0 = gt - d.tile_base;
        const int ti0 = t0 % d.ntx, r = t0 / d.ntx;
        const int tj = r % d.nty, tk = r / d.nty;
        int len = 1;
        while (len < d.R && ti0 + len < d.ntx && (ti0 + len) % d.R != 0 && u[t0 + len]) ++len;
        uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
        const int pl = d.ntx * d.nty;
        for (int l = 0; l < len; ++l) {
            const int t = t0 + l;
            m0 |= uint32_t(tj == 0 || u[t - d.ntx]) << l;
            m1 |= uint32_t(tj == d.nty - 1 || u[t + d.ntx]) << l;
            m2 |= uint32_t(tk == 0 || u[t - pl]) << l;
            m3 |= uint32_t(tk == d.ntz - 1 || u[t + pl]) << l;
        }
        const uint32_t xb = uint32_t(ti0 == 0 || u[t0 - 1]) |
                            (uint32_t(ti0 + len == d.ntx || u[t0 + len]) << 1);
        o[0] = t0;
        o[1] = len;
        o[2] = static_cast<int32_t>(m0);
        o[3] = static_cast<int32_t>(m1);
        o[4] = static_cast<int32_t>(m2);
        o[5] = static_cast<int32_t>(m3);
        o[6] = static_cast<int32_t>(xb);
        o[7] = i;
    }
}

// Copies the band points of src into dst for every item (odd step counts).
__global__ __launch_bounds__(kBlock) void batch_copy_kernel(const float *__restrict__ src,
                                                            float *__restrict__ dst,
                                                            const int32_t *__restrict__ rec,
                                                            const int32_t *nitems,
                                                            const BatchInst *__restrict__ inst) {
    const int m = *nitems;
    for (int w = blockIdx.x; w < m; w += gridDim.x) {
        const int32_t *r = rec + static_cast<int64_t>(w) * kItemWords;
        const BatchInst &d = inst[r[7]];
        const int t0 = r[0], len = r[1];
        const int ti0 = t0 % d.ntx, rr = t0 / d.ntx;
        const int x0 = ti0 * d.tx, y0 = (rr % d.nty) * d.ty, z0 = (rr / d.nty) * d.tz;
        const int W = min(len * d.tx, d.nx - x0), H = min(d.ty, d.ny - y0),
                  D = min(d.tz, d.nz - z0);
        for (int q = threadIdx.x; q < W * H * D; q += kBlock) {
            const int lx = q % W, rw = q / W;
            const int ly = rw % H, lz = rw / H;
            const int64_t gi =
                d.offset + (static_cast<int64_t>(z0 + lz) * d.ny + (y0 + ly)) * d.px + x0 + lx;
            dst[gi] = src[gi];
        }
    }
}


// acc += nsteps * (in-domain points of the listed tiles): a grid-stride sum,
// one atomic add per block (integer, so the order does not matter).
__global__ __launch_bounds__(kBlock) void batch_point_count_kernel(
    int64_t *acc, const int32_t *__restrict__ list, const int32_t *count,
    const BatchInst *__restrict__ inst, int n, int total_tiles, int nsteps) {
    __shared__ int64_t red[kBlock];
    const int m = min(*count, total_tiles);
    int64_t s = 0;
    for (int p = blockIdx.x * kBlock + threadIdx.x; p < m; p += gridDim.x * kBlock) {
        const int gt = list[p];
        if (gt < 0 || gt >= total_tiles) continue;
        const BatchInst &d = inst[find_inst(inst, n, gt, false)];
        const int t = gt - d.tile_base;
        const int ti = t % d.ntx, r = t / d.ntx;
        const int tj = r % d.nty, tk = r / d.nty;
        s += static_cast<int64_t>(min(d.tx, d.nx - ti * d.tx)) * min(d.ty, d.ny - tj * d.ty) *
             min(d.tz, d.nz - tk * d.tz);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(acc),
                  static_cast<unsigned long long>(red[0] * nsteps));
}

// ---------------------------------------------------------------------------
// host side

using BatchFn = void (*)(StepGeom, StepArgs<float, float>);

bool pipeline_forced();  // ls_step.hip

static BatchFn batch_kernel(const Shape4 &s, bool pipe, size_t *lds, int *threads) {
#define LS_BFAST(TX_, TY_, TZ_, R_)                                                          \
    if (s.tx == TX_ && s.ty == TY_ && s.tz == TZ_ && s.R == R_) {                            \
        *lds = FastCfg<float, float, TX_, TY_, TZ_, R_>::lds;                                \
        *threads = FastCfg<float, float, TX_, TY_, TZ_, R_>::NT;                             \
        return pipe ? upwind_fast_kernel<float, float, false, TX_, TY_, TZ_, R_, true, true, true> \
                    : upwind_fast_kernel<float, float, false, TX_, TY_, TZ_, R_, true, true, false>; \
    }
    LS_BFAST(8, 8, 8, 4)
    LS_BFAST(8, 8, 8, 2)
    LS_BFAST(16, 4, 4, 2)
    LS_BFAST(16, 4, 4, 4)
    LS_BFAST(32, 4, 4, 1)
    LS_BFAST(32, 4, 4, 2)
    LS_BFAST(16, 8, 8, 2)
    LS_BFAST(4, 4, 4, 8)
#undef LS_BFAST
    return nullptr;
}

static int check_batch_ws(const BatchLayout &L, void *ws, int64_t bytes, BatchWs *w) {
    *w = batch_ws(L);
    if (!ws) {
        set_error("batch: workspace is NULL");
        return LS_ERR_ARG;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("batch: workspace must be 256-byte aligned");
        return LS_ERR_ARG;
    }
    if (bytes < w->total) {
        set_error("batch: workspace too small: %lld bytes given, %lld needed", (long long)bytes,
                  (long long)w->total);
        return LS_ERR_CAPACITY;
    }
    return LS_OK;
}

// Band build of every grid (full scan or rescan of the previous list), the
// list into `list` / `*count`, and the plan (records, group ranges).
static int batch_build(const BatchLayout &L, const float *phi, uint8_t *ws, const BatchWs &w,
                       const int32_t *prev, const int32_t *prev_count, int32_t *list,
                       int32_t *count, hipStream_t stream, TileAccum accum) {
    const int n = static_cast<int>(L.inst.size());
    const int T = static_cast<int>(L.total_tiles);
    const BatchInst *inst = reinterpret_cast<const BatchInst *>(ws + w.inst);
    uint8_t *a = ws + w.a_flags;
    uint8_t *u = ws + w.u_map;
    int32_t *rec = reinterpret_cast<int32_t *>(ws + w.items);
    int32_t *nitems = reinterpret_cast<int32_t *>(ws + w.counters);
    int rc;
    DeviceInfo di;
    if ((rc = device_info(&di)) != LS_OK) return rc;
    int64_t slot;
    if ((rc = stats_before(LS_KERNEL_BAND_FLAG, stream, &slot)) != LS_OK) return rc;
    if (!prev) {
        hipLaunchKernelGGL(batch_flag_kernel, dim3(static_cast<unsigned>(L.total_slabs)),
                           dim3(kBlock), static_cast<size_t>(L.max_ntx), stream, phi, inst, n, a);
        LS_LAUNCH_CHECK("batch_flag_kernel");
    } else {
        // the flags equal the previous build's A, which lies inside the previous band
        const unsigned blocks =
            static_cast<unsigned>(std::min<int64_t>(cdiv64(T, kBlock / 64), int64_t(di.cus) * 16));
        hipLaunchKernelGGL(batch_flag_list_kernel, dim3(blocks), dim3(kBlock), 0, stream, phi,
                           inst, n, T, prev, prev_count, a);
        LS_LAUNCH_CHECK("batch_flag_list_kernel");
    }
    if ((rc = stats_after(LS_KERNEL_BAND_FLAG, stream, slot)) != LS_OK) return rc;
    const unsigned tb = static_cast<unsigned>(std::min<int64_t>(cdiv64(T, kBlock), 8192));
    hipLaunchKernelGGL(batch_dilate_kernel, dim3(tb), dim3(kBlock), 0, stream,
                       static_cast<const uint8_t *>(a), u, inst, n, T);
    LS_LAUNCH_CHECK("batch_dilate_kernel");
    rc = compact2(MapPred{u}, EmitIndex{list}, count, reinterpret_cast<int32_t *>(ws + w.blk),
                  BatchHeadPred{u, inst, n}, EmitHeadGlobal{rec}, nitems,
                  reinterpret_cast<int32_t *>(ws + w.blk2), nullptr, T, stream, accum);
    if (rc != LS_OK) return rc;
    hipLaunchKernelGGL(batch_range_kernel, dim3(1), dim3(64), 0, stream,
                       static_cast<const int32_t *>(rec), static_cast<const int32_t *>(nitems),
                       reinterpret_cast<const int32_t *>(ws + w.group_base),
                       static_cast<int>(L.groups.size()), reinterpret_cast<int32_t *>(ws + w.ranges));
    LS_LAUNCH_CHECK("batch_range_kernel");
    hipLaunchKernelGGL(batch_record_kernel, dim3(tb), dim3(kBlock), 0, stream, rec,
                       static_cast<const int32_t *>(nitems), static_cast<const uint8_t *>(u), inst,
                       n);
    LS_LAUNCH_CHECK("batch_record_kernel");
    return LS_OK;
}

static int batch_steps(const BatchLayout &L, float *phi, const float *F, float *scratch,
                       uint8_t *ws, const BatchWs &w, int nsteps, hipStream_t stream) {
    if (nsteps == 0) return LS_OK;
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != LS_OK) return rc;
    const int32_t *rec = reinterpret_cast<const int32_t *>(ws + w.items);
    const int32_t *nitems = reinterpret_cast<const int32_t *>(ws + w.counters);
    const int32_t *ranges = reinterpret_cast<const int32_t *>(ws + w.ranges);
    const BatchInst *inst = reinterpret_cast<const BatchInst *>(ws + w.inst);
    StepGeom sg;
    std::memset(&sg, 0, sizeof(sg));
    StepArgs<float, float> args;
    args.F = F;
    args.rec = rec;
    args.nitems = nitems;
    args.inst = inst;
    args.umap = nullptr;
    args.orig = phi;
    args.dx = args.dt = args.dtdx = 0.f;
    args.scale = 1.f;
    const int64_t G = std::max<int64_t>(8, (int64_t(di.cus) * kBatchBlocksPerCu) & ~int64_t(7));
    // software pipelining is on only when asked for: measured slower on the
    // 256-grid batch (its predicated kernels need the registers)
    const bool pipe = pipeline_forced();
    int64_t slot;
    if ((rc = stats_before(LS_KERNEL_UPWIND, stream, &slot,
                           int64_t(nsteps) * int64_t(L.groups.size()))) != LS_OK)
        return rc;
    for (int s = 0; s < nsteps; ++s) {
        args.cur = (s & 1) ? scratch : phi;
        args.nxt = (s & 1) ? phi : scratch;
        for (size_t gi = 0; gi < L.groups.size(); ++gi) {
            size_t lds = 0;
            int threads = kBlock;
            BatchFn k = batch_kernel(L.groups[gi].shape, pipe, &lds, &threads);
            args.range = ranges + gi;
            hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(G)), dim3(threads), lds, stream, sg,
                               args);
            LS_LAUNCH_CHECK("upwind_fast_kernel (batch)");
        }
    }
    if ((rc = stats_after(LS_KERNEL_UPWIND, stream, slot)) != LS_OK) return rc;
    if (nsteps & 1) {
        hipLaunchKernelGGL(batch_copy_kernel, dim3(static_cast<unsigned>(di.cus * 8)),
                           dim3(kBlock), 0, stream, static_cast<const float *>(scratch), phi, rec,
                           nitems, inst);
        LS_LAUNCH_CHECK("batch_copy_kernel");
    }
    return LS_OK;
}

}  // namespace ls

extern "C" {

int64_t ls_batch_workspace_bytes(const ls_instance *inst, int n) {
    ls::clear_error();
    ls::BatchLayout L;
    int rc = ls::make_layout(inst, n, &L);
    if (rc != LS_OK) return rc;
    return ls::batch_ws(L).total;
}

int ls_batch_layout(const ls_instance *inst, int n, int64_t *tile_base, int64_t *total_tiles) {
    ls::clear_error();
    ls::BatchLayout L;
    int rc = ls::make_layout(inst, n, &L);
    if (rc != LS_OK) return rc;
    if (tile_base)
        for (int k = 0; k < n; ++k) tile_base[L.given[k]] = L.inst[k].tile_base;
    if (total_tiles) *total_tiles = L.total_tiles;
    return LS_OK;
}

int ls_batch_setup(const ls_instance *inst, int n, void *workspace, int64_t workspace_bytes,
                   void *stream_) {
    ls::clear_error();
    ls::BatchLayout L;
    int rc = ls::make_layout(inst, n, &L);
    if (rc != LS_OK) return rc;
    ls::BatchWs w;
    if ((rc = ls::check_batch_ws(L, workspace, workspace_bytes, &w)) != LS_OK) return rc;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    std::vector<int32_t> gb(ls::kMaxGroups + 1, 0);
    for (size_t g = 0; g < L.groups.size(); ++g) gb[g] = L.groups[g].tile_base;
    gb[L.groups.size()] = static_cast<int32_t>(L.total_tiles);
    LS_HIP_CHECK(hipMemcpyAsync(ws + w.inst, L.inst.data(), sizeof(ls::BatchInst) * L.inst.size(),
                                hipMemcpyHostToDevice, stream));
    LS_HIP_CHECK(hipMemcpyAsync(ws + w.group_base, gb.data(), 4 * gb.size(),
                                hipMemcpyHostToDevice, stream));
    LS_HIP_CHECK(hipStreamSynchronize(stream));  // the host arrays go out of scope
    return LS_OK;
}

int ls_batch_run_f32(const ls_instance *inst, int n, float *phi, const float *F, float *scratch,
                     int nsteps, int window, int64_t *tile_steps_dev, int64_t *point_steps_dev,
                     void *workspace, int64_t workspace_bytes, void *stream_) {
    ls::clear_error();
    ls::BatchLayout L;
    int rc = ls::make_layout(inst, n, &L);
    if (rc != LS_OK) return rc;
    ls::BatchWs w;
    if ((rc = ls::check_batch_ws(L, workspace, workspace_bytes, &w)) != LS_OK) return rc;
    if (!phi || !F || !scratch) {
        ls::set_error("batch run: phi, F and scratch must be non-NULL");
        return LS_ERR_ARG;
    }
    if (static_cast<const void *>(phi) == static_cast<const void *>(scratch)) {
        ls::set_error("batch run: scratch must not alias phi");
        return LS_ERR_ARG;
    }
    if (nsteps < 0 || window <= 0) {
        ls::set_error("batch run: need nsteps >= 0 and window > 0");
        return LS_ERR_ARG;
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    int32_t *lists[2] = {reinterpret_cast<int32_t *>(ws + w.list0),
                         reinterpret_cast<int32_t *>(ws + w.list1)};
    int32_t *counts[2] = {reinterpret_cast<int32_t *>(ws + w.counters) + 1,
                          reinterpret_cast<int32_t *>(ws + w.counters) + 2};
    const int nwin = (nsteps + window - 1) / window;
    for (int k = 0; k < nwin; ++k) {
        const int m = std::min(window, nsteps - k * window);
        const int cur = (nwin - 1 - k) & 1;  // the last window's band lands in list0
        rc = ls::batch_build(L, phi, ws, w, k == 0 ? nullptr : lists[cur ^ 1],
                             k == 0 ? nullptr : counts[cur ^ 1], lists[cur], counts[cur], stream,
                             ls::TileAccum{tile_steps_dev, m});
        if (rc != LS_OK) return rc;
        if (point_steps_dev) {
            const unsigned pb = static_cast<unsigned>(
                std::min<int64_t>(ls::cdiv64(L.total_tiles, ls::kBlock), 1024));
            hipLaunchKernelGGL(ls::batch_point_count_kernel, dim3(pb), dim3(ls::kBlock), 0, stream,
                               point_steps_dev, static_cast<const int32_t *>(lists[cur]),
                               static_cast<const int32_t *>(counts[cur]),
                               reinterpret_cast<const ls::BatchInst *>(ws + w.inst), n,
                               static_cast<int>(L.total_tiles), m);
            LS_LAUNCH_CHECK("batch_point_count_kernel");
        }
        if ((rc = ls::batch_steps(L, phi, F, scratch, ws, w, m, stream)) != LS_OK) return rc;
    }
    return LS_OK;
}

int ls_batch_band(const ls_instance *inst, int n, void *workspace, int64_t workspace_bytes,
                  const int32_t **tiles_dev, const int32_t **ntiles_dev) {
    ls::clear_error();
    ls::BatchLayout L;
    int rc = ls::make_layout(inst, n, &L);
    if (rc != LS_OK) return rc;
    ls::BatchWs w;
    if ((rc = ls::check_batch_ws(L, workspace, workspace_bytes, &w)) != LS_OK) return rc;
    if (!tiles_dev || !ntiles_dev) {
        ls::set_error("batch band: NULL output");
        return LS_ERR_ARG;
    }
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    *tiles_dev = reinterpret_cast<const int32_t *>(ws + w.list0);
    *ntiles_dev = reinterpret_cast<const int32_t *>(ws + w.counters) + 1;
    return LS_OK;
}

}  // extern "C"
