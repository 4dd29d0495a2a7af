// Band build: tile flags of the tube (Eq. 6), one-tile dilation (the tile
// form of the region N, Eq. 11), ordered compaction into the band list.
#include <algorithm>

#include "ls_compact.h"
#include "ls_stats.h"

namespace ls {

// ---------------------------------------------------------------------------
// step plan: work items (x-runs of band tiles broken at every R-th tile
// column) and their records, from the update map

// A tile starts a work item if it is in the band and either sits on a
// multiple-of-R tile column or its x-predecessor is not in the band.
struct HeadMapPred {
    const uint8_t *umap;
    int ntx, R;
    __device__ bool operator()(int64_t t) const {
        if (!umap[t]) return false;
        const int ti = static_cast<int>(t % ntx);
        return ti % R == 0 || !umap[t - 1];
    }
};

struct EmitHeadTile {
    int32_t *rec;
    __device__ void operator()(int pos, int64_t t) const {
        rec[static_cast<int64_t>(pos) * kItemWords + 7] = static_cast<int32_t>(t);
    }
};

// Record of item pos (word 7 holds its first tile): [0] first tile, [1] run
// length, [2..5] bit l = "tile l of the run has its y-, y+, z-, z+ face
// neighbour in the band (or outside the grid)", [6] bits 0 / 1 = same for the
// x- / x+ neighbour of the run, [7] the same for the diagonal neighbours of
// runs of at most 4 tiles (below).
struct ItemRecordFn {
    int32_t *rec;
    const uint8_t *umap;
    int ntx, nty, ntz, R;
    __device__ void operator()(int pos) const {
        int32_t *o = rec + static_cast<int64_t>(pos) * kItemWords;
        const int t0 = o[7];
        const int ti0 = t0 % ntx;
        const int r = t0 / ntx;
        const int tj = r % nty, tk = r / nty;
        int len = 1;
        while (len < R && ti0 + len < ntx && (ti0 + len) % R != 0 && umap[t0 + len]) ++len;
        uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
        for (int l = 0; l < len; ++l) {
            const int t = t0 + l;
            m0 |= uint32_t(tj == 0 || umap[t - ntx]) << l;
            m1 |= uint32_t(tj == nty - 1 || umap[t + ntx]) << l;
            m2 |= uint32_t(tk == 0 || umap[t - ntx * nty]) << l;
            m3 |= uint32_t(tk == ntz - 1 || umap[t + ntx * nty]) << l;
        }
        const uint32_t xb = uint32_t(ti0 == 0 || umap[t0 - 1]) |
                            (uint32_t(ti0 + len == ntx || umap[t0 + len]) << 1);
        // word 7 (runs of at most 4 tiles): the diagonal neighbours the
        // two-step kernel reads, 1 = in the band (or outside the grid): bits
        // 4l..4l+3 the (y-,z-), (y-,z+), (y+,z-), (y+,z+) neighbours of tile l;
        // bits 16..19 / 20..23 the y-, y+, z-, z+ neighbours of the tile
        // before / after the run
        uint32_t diag = 0;
        if (R <= 4) {
            const int64_t sy = ntx, sz = static_cast<int64_t>(ntx) * nty;
            auto in = [&](int64_t t, int dj, int dk) {
                if (tj + dj < 0 || tj + dj >= nty || tk + dk < 0 || tk + dk >= ntz) return 1u;
                return umap[t + dj * sy + dk * sz] ? 1u : 0u;
            };
            for (int l = 0; l < len; ++l) {
                const int64_t t = t0 + l;
                diag |= (in(t, -1, -1) | in(t, -1, 1) << 1 | in(t, 1, -1) << 2 | in(t, 1, 1) << 3)
                        << (4 * l);
            }
            auto ends = [&](int64_t t) {
                return in(t, -1, 0) | in(t, 1, 0) << 1 | in(t, 0, -1) << 2 | in(t, 0, 1) << 3;
            };
            diag |= (ti0 > 0 ? ends(t0 - 1) : 15u) << 16;
            diag |= (ti0 + len < ntx ? ends(t0 + len) : 15u) << 20;
        }
        o[0] = t0;
        o[1] = len;
        o[2] = static_cast<int32_t>(m0);
        o[3] = static_cast<int32_t>(m1);
        o[4] = static_cast<int32_t>(m2);
        o[5] = static_cast<int32_t>(m3);
        o[6] = static_cast<int32_t>(xb);
        o[7] = static_cast<int32_t>(diag);
    }
};

__global__ __launch_bounds__(kBlock) void item_record_kernel(ItemRecordFn f, const int32_t *nitems) {
    const int n = *nitems;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) f(i);
}

int build_plan(const Geom &g, uint8_t *ws, int32_t *list, int32_t *list_count,
               hipStream_t stream, TileAccum accum) {
    const Workspace w = workspace_layout(g);
    const uint8_t *umap = ws + w.u_map;
    int32_t *blk = reinterpret_cast<int32_t *>(ws + w.blk_counts);
    int32_t *blk2 = reinterpret_cast<int32_t *>(ws + w.blk_counts2);
    int32_t *rec = reinterpret_cast<int32_t *>(ws + w.items);
    int32_t *nitems = reinterpret_cast<int32_t *>(ws + w.counters);
    const int R = plan_run_tiles(g);
    const HeadMapPred heads{umap, g.ntx, R};
    int rc;
    if (list)
        rc = compact2(MapPred{umap}, EmitIndex{list}, list_count, blk, heads, EmitHeadTile{rec},
                      nitems, blk2, nullptr, g.ntiles, stream, accum);
    else
        rc = compact(heads, EmitHeadTile{rec}, nullptr, g.ntiles, nitems, blk, stream);
    if (rc != LS_OK) return rc;
    const unsigned rb = static_cast<unsigned>(std::min<int64_t>(cdiv64(g.ntiles, kBlock), 2048));
    hipLaunchKernelGGL(item_record_kernel, dim3(rb), dim3(kBlock), 0, stream,
                       ItemRecordFn{rec, umap, g.ntx, g.nty, g.ntz, R},
                       static_cast<const int32_t *>(nitems));
    LS_LAUNCH_CHECK("item_record_kernel");
    return LS_OK;
}

// ---------------------------------------------------------------------------
// tile flags: one block per (tj, tk) slab of ty*tz grid rows, x in 16-byte
// vectors; every thread keeps its own column's hits in registers and marks
// the tile in LDS once.

template <class S>
struct Vec16 {
    static constexpr int V = 16 / sizeof(S);
    S v[V];
};

template <class S, int V>
__global__ __launch_bounds__(kBlock) void band_flag_kernel(const S *__restrict__ phi, int nx,
                                                           int ny, int nz, int tx, int ty, int tz,
                                                           int ntx, int nty,
                                                           typename Codec<S>::C gamma,
                                                           typename Codec<S>::C scale,
                                                           uint8_t *__restrict__ a_flags) {
    extern __shared__ uint8_t sflag[];
    const int tj = blockIdx.x, tk = blockIdx.y;
    for (int t = threadIdx.x; t < ntx; t += kBlock) sflag[t] = 0;
    __syncthreads();

    const int j0 = tj * ty, k0 = tk * tz;
    const int rows_y = min(ty, ny - j0), rows_z = min(tz, nz - k0);
    const int nrows = rows_y * rows_z;
    const int nvec = nx / V;

    if (nvec <= kBlock) {
        const int rpp = kBlock / nvec;  // rows per pass
        const int col = threadIdx.x % nvec;
        const int r0 = threadIdx.x / nvec;
        if (r0 < rpp) {
            bool hit[V];
#pragma unroll
            for (int e = 0; e < V; ++e) hit[e] = false;
            int jj = r0 % rows_y, kk = r0 / rows_y;
            const int djj = rpp % rows_y, dkk = rpp / rows_y;
#pragma unroll 4
            for (int r = r0; r < nrows; r += rpp) {
                const int64_t row = (static_cast<int64_t>(k0 + kk) * ny + (j0 + jj)) * nx;
                if constexpr (V > 1) {
                    const Vec16<S> w = *reinterpret_cast<const Vec16<S> *>(phi + row + col * V);
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        hit[e] |= fabs(Codec<S>::load(w.v[e], scale)) < gamma;
                } else {
                    hit[0] |= fabs(Codec<S>::load(phi[row + col], scale)) < gamma;
                }
                jj += djj;
                kk += dkk;
                if (jj >= rows_y) {
                    jj -= rows_y;
                    ++kk;
                }
            }
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (hit[e]) sflag[(col * V + e) / tx] = 1;
        }
    } else {
        for (int r = 0; r < nrows; ++r) {
            const int jj = r % rows_y, kk = r / rows_y;
            const int64_t row = (static_cast<int64_t>(k0 + kk) * ny + (j0 + jj)) * nx;
            for (int c = threadIdx.x; c < nvec; c += kBlock) {
                if constexpr (V > 1) {
                    const Vec16<S> w = *reinterpret_cast<const Vec16<S> *>(phi + row + c * V);
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if (fabs(Codec<S>::load(w.v[e], scale)) < gamma) sflag[(c * V + e) / tx] = 1;
                } else {
                    if (fabs(Codec<S>::load(phi[row + c], scale)) < gamma) sflag[c / tx] = 1;
                }
            }
        }
    }
    __syncthreads();
    uint8_t *dst = a_flags + (static_cast<int64_t>(tk) * nty + tj) * ntx;
    for (int t = threadIdx.x; t < ntx; t += kBlock) dst[t] = sflag[t];
}

// U = A grown by one tile in all 26 directions (clipped to the tile grid),
// or U = A when dilate is 0.
__global__ __launch_bounds__(kBlock) void band_dilate_kernel(const uint8_t *__restrict__ a,
                                                             uint8_t *__restrict__ u, int ntx,
                                                             int nty, int ntz, int dilate) {
    const int ti = blockIdx.x * 64 + threadIdx.x;
    const int tj = blockIdx.y * 4 + threadIdx.y;
    const int tk = blockIdx.z;
    if (ti >= ntx || tj >= nty) return;
    const int64_t t = (static_cast<int64_t>(tk) * nty + tj) * ntx + ti;
    if (!dilate) {
        u[t] = a[t];
        return;
    }
    uint8_t hit = 0;
    for (int dk = -1; dk <= 1; ++dk) {
        const int k = tk + dk;
        if (k < 0 || k >= ntz) continue;
        for (int dj = -1; dj <= 1; ++dj) {
            const int j = tj + dj;
            if (j < 0 || j >= nty) continue;
            const uint8_t *row = a + (static_cast<int64_t>(k) * nty + j) * ntx;
            hit |= row[ti];
            if (ti > 0) hit |= row[ti - 1];
            if (ti + 1 < ntx) hit |= row[ti + 1];
        }
    }
    u[t] = hit ? 1 : 0;
}

// Tile flags of the listed tiles only (the incremental rebuild): one wave per
// listed tile at a time; every lane tests its share of the tile's points and
// the wave ORs the results with a ballot.
template <class S>
__global__ __launch_bounds__(kBlock) void band_flag_list_kernel(
    const S *__restrict__ phi, int nx, int ny, int nz, int tx, int ty, int tz, int ntx, int nty,
    int ntiles_cap, typename Codec<S>::C gamma, typename Codec<S>::C scale,
    const int32_t *__restrict__ list, const int32_t *__restrict__ list_count,
    uint8_t *__restrict__ a_flags, bool vec_rows) {
    const int n = min(*list_count, ntiles_cap);
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (kBlock / 64);
    for (int p = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); p < n; p += waves) {
        const int t = list[p];
        if (t < 0 || t >= ntiles_cap) continue;  // uniform per wave
        const int ti = t % ntx, r = t / ntx;
        const int tj = r % nty, tk = r / nty;
        const int x0 = ti * tx, y0 = tj * ty, z0 = tk * tz;
        const int W = min(tx, nx - x0), H = min(ty, ny - y0), D = min(tz, nz - z0);
        bool hit = false;
        constexpr int V = Vec16<S>::V;
        if (vec_rows && W == tx) {
            // whole 16-byte vectors along x: lane -> (row, vector of the row)
            const int vpr = tx / V;  // vectors per row
            const int nv = vpr * H * D;
            for (int q = lane; q < nv; q += 64) {
                const int c = q % vpr, rr = q / vpr;
                const int ly = rr % H, lz = rr / H;
                const int64_t gi =
                    (static_cast<int64_t>(z0 + lz) * ny + (y0 + ly)) * nx + x0 + c * V;
                const Vec16<S> v = *reinterpret_cast<const Vec16<S> *>(phi + gi);
#pragma unroll
                for (int e = 0; e < V; ++e) hit |= fabs(Codec<S>::load(v.v[e], scale)) < gamma;
            }
        } else {
            const int npts = W * H * D;
#pragma unroll 8
            for (int q = lane; q < npts; q += 64) {
                const int lx = q % W, rr = q / W;
                const int ly = rr % H, lz = rr / H;
                const int64_t gi =
                    (static_cast<int64_t>(z0 + lz) * ny + (y0 + ly)) * nx + x0 + lx;
                hit |= fabs(Codec<S>::load(phi[gi], scale)) < gamma;
            }
        }
        const bool any = __ballot(hit) != 0;
        if (lane == 0) a_flags[t] = any ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// host side

template <class S>
static int band_args(const S *phi, const ls_grid *grid, typename Codec<S>::C gamma, int dilate,
                     int32_t *tiles, int64_t capacity, int32_t *ntiles_dev, void *workspace,
                     int64_t ws_bytes, Geom *g) {
    int rc = make_geom(grid, g);
    if (rc != LS_OK) return rc;
    g->elem_bytes = static_cast<int32_t>(sizeof(S));
    if (!phi || !tiles || !ntiles_dev) {
        set_error("band build: phi, tiles and ntiles_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (dilate != 0 && dilate != 1) {
        set_error("band build: dilate must be 0 or 1 (got %d)", dilate);
        return LS_ERR_ARG;
    }
    if (!(gamma == gamma)) {
        set_error("band build: gamma is NaN");
        return LS_ERR_ARG;
    }
    if (capacity < g->ntiles) {
        set_error("band build: capacity %lld < %lld tiles", (long long)capacity,
                  (long long)g->ntiles);
        return LS_ERR_CAPACITY;
    }
    if ((rc = check_workspace(*g, workspace, ws_bytes)) != LS_OK) return rc;
    if (g->ntx > 65536) {
        set_error("band build: more than 65536 tiles along x unsupported");
        return LS_ERR_UNSUPPORTED;
    }
    if (g->nty > 65535 || g->ntz > 65535) {
        set_error("band build: more than 65535 tiles along y or z unsupported");
        return LS_ERR_UNSUPPORTED;
    }
    return LS_OK;
}

// Dilation (or copy) of the flags into the update map, then the ordered band
// list and the step plan of that list.
int band_finish(const Geom &g, uint8_t *ws, int dilate, int32_t *tiles,
                       int32_t *ntiles_dev, hipStream_t stream, TileAccum accum) {
    const Workspace w = workspace_layout(g);
    const dim3 dgrid(static_cast<unsigned>(cdiv64(g.ntx, 64)), static_cast<unsigned>(cdiv64(g.nty, 4)),
                     g.ntz);
    hipLaunchKernelGGL(band_dilate_kernel, dgrid, dim3(64, 4), 0, stream,
                       static_cast<const uint8_t *>(ws + w.a_flags), ws + w.u_map, g.ntx, g.nty,
                       g.ntz, dilate);
    LS_LAUNCH_CHECK("band_dilate_kernel");
    return build_plan(g, ws, tiles, ntiles_dev, stream, accum);
}

template <class S>
int band_build(const S *phi, typename Codec<S>::C scale, const ls_grid *grid,
               typename Codec<S>::C gamma, int dilate, int32_t *tiles, int64_t capacity,
               int32_t *ntiles_dev, void *workspace, int64_t ws_bytes, void *stream_,
               TileAccum accum) {
    Geom g;
    int rc = band_args(phi, grid, gamma, dilate, tiles, capacity, ntiles_dev, workspace, ws_bytes,
                       &g);
    if (rc != LS_OK) return rc;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const Workspace w = workspace_layout(g);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    uint8_t *a = ws + w.a_flags;

    constexpr int V = Vec16<S>::V;
    const bool vec_ok = (g.nx % V == 0) && (reinterpret_cast<uintptr_t>(phi) % 16 == 0);
    const dim3 fgrid(g.nty, g.ntz);
    const size_t lds = static_cast<size_t>(g.ntx);
    int64_t slot;
    if ((rc = stats_before(LS_KERNEL_BAND_FLAG, stream, &slot)) != LS_OK) return rc;
    if (vec_ok) {
        hipLaunchKernelGGL((band_flag_kernel<S, V>), fgrid, dim3(kBlock), lds, stream, phi, g.nx,
                           g.ny, g.nz, g.tx, g.ty, g.tz, g.ntx, g.nty, gamma, scale, a);
    } else {
        hipLaunchKernelGGL((band_flag_kernel<S, 1>), fgrid, dim3(kBlock), lds, stream, phi, g.nx,
                           g.ny, g.nz, g.tx, g.ty, g.tz, g.ntx, g.nty, gamma, scale, a);
    }
    LS_LAUNCH_CHECK("band_flag_kernel");
    if ((rc = stats_after(LS_KERNEL_BAND_FLAG, stream, slot)) != LS_OK) return rc;
    return band_finish(g, ws, dilate, tiles, ntiles_dev, stream, accum);
}

__global__ __launch_bounds__(kBlock) void fill_zero_kernel(uint8_t *p, int64_t n16) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n16;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        reinterpret_cast<uint4 *>(p)[i] = make_uint4(0, 0, 0, 0);
}

int fill_zero(uint8_t *p, int64_t bytes, hipStream_t stream) {
    const int64_t n16 = cdiv64(bytes, 16);
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(cdiv64(n16, kBlock), 4096));
    hipLaunchKernelGGL(fill_zero_kernel, dim3(std::max(1u, blocks)), dim3(kBlock), 0, stream, p,
                       n16);
    LS_LAUNCH_CHECK("fill_zero_kernel");
    return LS_OK;
}

// With flags_valid the workspace's tile flags already equal the A of the
// build that produced prev_tiles (the driver's case: every build writes A, and
// A lies inside the band it dilates to), so they need no clearing: rescanning
// the previous band overwrites every flag that can change.
template <class S>
int band_rebuild(const S *phi, typename Codec<S>::C scale, const ls_grid *grid,
                 typename Codec<S>::C gamma, const int32_t *prev_tiles,
                 const int32_t *prev_ntiles_dev, int32_t *tiles, int64_t capacity,
                 int32_t *ntiles_dev, void *workspace, int64_t ws_bytes, void *stream_,
                 bool flags_valid, TileAccum accum) {
    Geom g;
    int rc = band_args(phi, grid, gamma, 1, tiles, capacity, ntiles_dev, workspace, ws_bytes, &g);
    if (rc != LS_OK) return rc;
    if (!prev_tiles || !prev_ntiles_dev) {
        set_error("band rebuild: prev_tiles and prev_ntiles_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (static_cast<const void *>(prev_tiles) == static_cast<const void *>(tiles) ||
        static_cast<const void *>(prev_ntiles_dev) == static_cast<const void *>(ntiles_dev)) {
        set_error("band rebuild: the previous and the new list must be distinct buffers");
        return LS_ERR_ARG;
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const Workspace w = workspace_layout(g);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    if (!flags_valid && (rc = fill_zero(ws + w.a_flags, g.ntiles, stream)) != LS_OK) return rc;
    DeviceInfo di;
    if ((rc = device_info(&di)) != LS_OK) return rc;
    const unsigned blocks =
        static_cast<unsigned>(std::min<int64_t>(cdiv64(g.ntiles, kBlock / 64), int64_t(di.cus) * 16));
    // rows of whole tiles load as 16-byte vectors when every row start is aligned
    constexpr int V = Vec16<S>::V;
    const bool vec_rows = g.tx % V == 0 && g.nx % V == 0 &&
                          reinterpret_cast<uintptr_t>(phi) % 16 == 0;
    int64_t slot;
    if ((rc = stats_before(LS_KERNEL_BAND_FLAG, stream, &slot)) != LS_OK) return rc;
    hipLaunchKernelGGL(band_flag_list_kernel<S>, dim3(blocks), dim3(kBlock), 0, stream, phi, g.nx,
                       g.ny, g.nz, g.tx, g.ty, g.tz, g.ntx, g.nty, static_cast<int>(g.ntiles),
                       gamma, scale, prev_tiles, prev_ntiles_dev, ws + w.a_flags, vec_rows);
    LS_LAUNCH_CHECK("band_flag_list_kernel");
    if ((rc = stats_after(LS_KERNEL_BAND_FLAG, stream, slot)) != LS_OK) return rc;
    return band_finish(g, ws, 1, tiles, ntiles_dev, stream, accum);
}

template int band_build<float>(const float *, float, const ls_grid *, float, int, int32_t *,
                               int64_t, int32_t *, void *, int64_t, void *, TileAccum);
template int band_build<double>(const double *, double, const ls_grid *, double, int, int32_t *,
                                int64_t, int32_t *, void *, int64_t, void *, TileAccum);
template int band_build<uint16_t>(const uint16_t *, float, const ls_grid *, float, int,
                                  int32_t *, int64_t, int32_t *, void *, int64_t, void *,
                                  TileAccum);
template int band_rebuild<float>(const float *, float, const ls_grid *, float, const int32_t *,
                                 const int32_t *, int32_t *, int64_t, int32_t *, void *, int64_t,
                                 void *, bool, TileAccum);
template int band_rebuild<double>(const double *, double, const ls_grid *, double,
                                  const int32_t *, const int32_t *, int32_t *, int64_t, int32_t *,
                                  void *, int64_t, void *, bool, TileAccum);
template int band_rebuild<uint16_t>(const uint16_t *, float, const ls_grid *, float,
                                    const int32_t *, const int32_t *, int32_t *, int64_t,
                                    int32_t *, void *, int64_t, void *, bool, TileAccum);

}  // namespace ls

extern "C" {

int ls_band_build_f32(const float *phi, const ls_grid *g, float gamma, int dilate, int32_t *tiles,
                      int64_t capacity, int32_t *ntiles_dev, void *workspace,
                      int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_build<float>(phi, 1.0f, g, gamma, dilate, tiles, capacity, ntiles_dev,
                                 workspace, workspace_bytes, stream);
}

int ls_band_build_f64(const double *phi, const ls_grid *g, double gamma, int dilate,
                      int32_t *tiles, int64_t capacity, int32_t *ntiles_dev, void *workspace,
                      int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_build<double>(phi, 1.0, g, gamma, dilate, tiles, capacity, ntiles_dev,
                                  workspace, workspace_bytes, stream);
}

int ls_band_rebuild_f32(const float *phi, const ls_grid *g, float gamma,
                        const int32_t *prev_tiles, const int32_t *prev_ntiles_dev, int32_t *tiles,
                        int64_t capacity, int32_t *ntiles_dev, void *workspace,
                        int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_rebuild<float>(phi, 1.0f, g, gamma, prev_tiles, prev_ntiles_dev, tiles,
                                   capacity, ntiles_dev, workspace, workspace_bytes, stream,
                                   false);
}

int ls_band_rebuild_f64(const double *phi, const ls_grid *g, double gamma,
                        const int32_t *prev_tiles, const int32_t *prev_ntiles_dev, int32_t *tiles,
                        int64_t capacity, int32_t *ntiles_dev, void *workspace,
                        int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    return ls::band_rebuild<double>(phi, 1.0, g, gamma, prev_tiles, prev_ntiles_dev, tiles,
                                    capacity, ntiles_dev, workspace, workspace_bytes, stream,
                                    false);
}

int ls_band_rebuild_f16s(const uint16_t *phi_h, float scale, const ls_grid *g, float gamma,
                         const int32_t *prev_tiles, const int32_t *prev_ntiles_dev,
                         int32_t *tiles, int64_t capacity, int32_t *ntiles_dev, void *workspace,
                         int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("band rebuild f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::band_rebuild<uint16_t>(phi_h, scale, g, gamma, prev_tiles, prev_ntiles_dev, tiles,
                                      capacity, ntiles_dev, workspace, workspace_bytes, stream,
                                      false);
}

int ls_band_build_f16s(const uint16_t *phi_h, float scale, const ls_grid *g, float gamma,
                       int dilate, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                       void *workspace, int64_t workspace_bytes, void *stream) {
    ls::clear_error();
    if (!(scale > 0.0f) || !(scale < INFINITY)) {
        ls::set_error("band build f16s: scale must be positive and finite");
        return LS_ERR_ARG;
    }
    return ls::band_build<uint16_t>(phi_h, scale, g, gamma, dilate, tiles, capacity, ntiles_dev,
                                    workspace, workspace_bytes, stream);
}

}  // extern "C"
