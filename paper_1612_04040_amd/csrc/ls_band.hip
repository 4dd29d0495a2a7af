// Band build: tile flags of the tube (Eq. 6), one-tile dilation (the tile
// form of the region N, Eq. 11), ordered compaction into the band list.
#include "ls_compact.h"
#include "ls_stats.h"

namespace ls {

// ---------------------------------------------------------------------------
// one-block exclusive scan of the per-block counts

__global__ __launch_bounds__(1024) void compact_scan_kernel(int32_t *blk, int64_t nblk,
                                                            int32_t *count) {
    __shared__ int wave_sum[1024 / 64];
    __shared__ int carry_s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int v = i < nblk ? blk[i] : 0;
        // inclusive scan inside the wave
        int s = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(s, d, 64);
            if (lane >= d) s += t;
        }
        if (lane == 63) wave_sum[wave] = s;
        __syncthreads();
        int before = carry_s;
        for (int w = 0; w < wave; ++w) before += wave_sum[w];
        if (i < nblk) blk[i] = before + s - v;  // exclusive
        __syncthreads();
        if (threadIdx.x == 1023) carry_s = before + s;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        blk[nblk] = carry_s;
        *count = carry_s;
    }
}

int compact_map(const uint8_t *map, int64_t n, int32_t *out, int32_t *count, int32_t *blk,
                hipStream_t stream) {
    return compact(MapPred{map}, EmitIndex{out}, nullptr, n, count, blk, stream);
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

// U = A grown by one tile in all 26 directions (clipped to the tile grid).
__global__ __launch_bounds__(kBlock) void band_dilate_kernel(const uint8_t *__restrict__ a,
                                                             uint8_t *__restrict__ u, int ntx,
                                                             int nty, int ntz) {
    const int ti = blockIdx.x * 64 + threadIdx.x;
    const int tj = blockIdx.y * 4 + threadIdx.y;
    const int tk = blockIdx.z;
    if (ti >= ntx || tj >= nty) return;
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
    u[(static_cast<int64_t>(tk) * nty + tj) * ntx + ti] = hit ? 1 : 0;
}

// ---------------------------------------------------------------------------
// host side

template <class S>
int band_build(const S *phi, typename Codec<S>::C scale, const ls_grid *grid,
                      typename Codec<S>::C gamma, int dilate, int32_t *tiles, int64_t capacity,
                      int32_t *ntiles_dev, void *workspace, int64_t ws_bytes, void *stream_) {
    Geom g;
    int rc = make_geom(grid, &g);
    if (rc != LS_OK) return rc;
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
    if (capacity < g.ntiles) {
        set_error("band build: capacity %lld < %lld tiles", (long long)capacity,
                  (long long)g.ntiles);
        return LS_ERR_CAPACITY;
    }
    if ((rc = check_workspace(g, workspace, ws_bytes)) != LS_OK) return rc;
    if (g.ntx > 65536) {
        set_error("band build: more than 65536 tiles along x unsupported");
        return LS_ERR_UNSUPPORTED;
    }
    if (g.nty > 65535 || g.ntz > 65535) {
        set_error("band build: more than 65535 tiles along y or z unsupported");
        return LS_ERR_UNSUPPORTED;
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const Workspace w = workspace_layout(g);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    uint8_t *a = ws + w.a_flags;
    uint8_t *u = ws + w.u_map;
    int32_t *blk = reinterpret_cast<int32_t *>(ws + w.blk_counts);

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
    const uint8_t *map = a;
    if (dilate) {
        const dim3 dgrid(static_cast<unsigned>(cdiv64(g.ntx, 64)),
                         static_cast<unsigned>(cdiv64(g.nty, 4)), g.ntz);
        hipLaunchKernelGGL(band_dilate_kernel, dgrid, dim3(64, 4), 0, stream, a, u, g.ntx, g.nty,
                           g.ntz);
        LS_LAUNCH_CHECK("band_dilate_kernel");
        map = u;
    }
    return compact_map(map, g.ntiles, tiles, ntiles_dev, blk, stream);
}

template int band_build<float>(const float *, float, const ls_grid *, float, int, int32_t *,
                               int64_t, int32_t *, void *, int64_t, void *);
template int band_build<double>(const double *, double, const ls_grid *, double, int, int32_t *,
                                int64_t, int32_t *, void *, int64_t, void *);
template int band_build<uint16_t>(const uint16_t *, float, const ls_grid *, float, int,
                                  int32_t *, int64_t, int32_t *, void *, int64_t, void *);

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
