// Band snapshot: the values of the band tiles copied, tile by tile in list
// order, into a dense tile-major buffer (the output of Step 4 of the
// algorithm in Sec. 1.1, restricted to the band), so that one contiguous
// device-to-host copy of the first n tiles takes the snapshot off the GPU.
//
// When the rows allow 4-point vector accesses (a 16-byte FP32 or an 8-byte
// FP16 access per thread), a block gathers a chunk of G consecutive band tiles
// through LDS: it reads each grid row across the chunk's tiles together (band
// tiles that follow each other in x are adjacent in the grid, so an x-run of
// them is read as whole cache lines), then writes the chunk, tile-major, as
// one contiguous block.  Otherwise one thread moves one point.  The band count
// is read on the device, so the call needs no host synchronisation.
#include <algorithm>
#include <type_traits>

#include "ls_internal.h"
#include "ls_stats.h"

namespace ls {

struct GatherGeom {
    int32_t nx, ny, nz, tx, ty, tz, ntx, nty;
    int32_t tp;        // points per tile
    int64_t ntiles;    // tiles of the grid
    int64_t capacity;  // tiles the output holds
};

template <class S>
struct GatherQuad;
template <>
struct GatherQuad<float> {
    using T = float4;
    __device__ static inline T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <>
struct GatherQuad<uint16_t> {
    using T = uint2;
    __device__ static inline T zero() { return make_uint2(0u, 0u); }
};

// V = 4: quads of x-consecutive points (tx and nx multiples of 4); V = 1:
// single points.  Points outside the grid (partial tiles) and tiles with an
// invalid id are written as zero.
template <class S, class T, int V>
__global__ __launch_bounds__(kBlock) void band_gather_kernel(GatherGeom g, const S *__restrict__ phi,
                                                             const int32_t *__restrict__ tiles,
                                                             const int32_t *__restrict__ ntiles_dev,
                                                             S *__restrict__ out,
                                                             int32_t *__restrict__ ids_out) {
    const int64_t n = min(static_cast<int64_t>(max(*ntiles_dev, 0)), g.capacity);
    const int per_row = g.tx / V;
    const int per_tile = g.tp / V;
    const int64_t total = n * per_tile;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < total;
         q += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int64_t p = q / per_tile;
        const int r = static_cast<int>(q - p * per_tile);
        const int t = tiles[p];
        const int row = r / per_row, xq = r - row * per_row;
        const int ly = row % g.ty, lz = row / g.ty;
        T v;
        if constexpr (V == 4)
            v = GatherQuad<S>::zero();
        else
            v = T(0);
        if (t >= 0 && t < g.ntiles) {
            const int ti = t % g.ntx, rr = t / g.ntx;
            const int x = ti * g.tx + xq * V, y = (rr % g.nty) * g.ty + ly,
                      z = (rr / g.nty) * g.tz + lz;
            if (x < g.nx && y < g.ny && z < g.nz)
                v = *reinterpret_cast<const T *>(
                    phi + (static_cast<int64_t>(z) * g.ny + y) * g.nx + x);
        }
        *reinterpret_cast<T *>(out + p * g.tp + static_cast<int64_t>(r) * V) = v;
        if (ids_out && r == 0) ids_out[p] = t;
    }
}

// Chunked form: G tiles per chunk, tp / 4 quads per tile staged in LDS.
template <class S, class T>
__global__ __launch_bounds__(kBlock) void band_gather_chunk_kernel(
    GatherGeom g, int G, const S *__restrict__ phi, const int32_t *__restrict__ tiles,
    const int32_t *__restrict__ ntiles_dev, S *__restrict__ out, int32_t *__restrict__ ids_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = reinterpret_cast<T *>(smem);
    const int64_t n = min(static_cast<int64_t>(max(*ntiles_dev, 0)), g.capacity);
    const int per_row = g.tx / 4, per_tile = g.tp / 4;
    const int64_t nchunks = (n + G - 1) / G;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {  // uniform per block
        const int cnt = static_cast<int>(min(static_cast<int64_t>(G), n - c * G));
        // reads: quad xq of row `row` of chunk tile gt, xq fastest, then the tile
        for (int e = threadIdx.x; e < G * per_tile; e += kBlock) {
            const int xq = e % per_row, t2 = e / per_row, gt = t2 % G, row = t2 / G;
            if (gt >= cnt) continue;
            const int t = tiles[c * G + gt];
            T v = GatherQuad<S>::zero();
            if (t >= 0 && t < g.ntiles) {
                const int ti = t % g.ntx, rr = t / g.ntx;
                const int ly = row % g.ty, lz = row / g.ty;
                const int x = ti * g.tx + xq * 4, y = (rr % g.nty) * g.ty + ly,
                          z = (rr / g.nty) * g.tz + lz;
                if (x < g.nx && y < g.ny && z < g.nz)
                    v = *reinterpret_cast<const T *>(
                        phi + (static_cast<int64_t>(z) * g.ny + y) * g.nx + x);
            }
            lds[gt * per_tile + row * per_row + xq] = v;
        }
        __syncthreads();
        // writes: the chunk's cnt tiles, contiguous
        T *dst = reinterpret_cast<T *>(out + c * G * g.tp);
        for (int e = threadIdx.x; e < cnt * per_tile; e += kBlock) dst[e] = lds[e];
        if (ids_out)
            for (int e = threadIdx.x; e < cnt; e += kBlock) ids_out[c * G + e] = tiles[c * G + e];
        __syncthreads();  // LDS free for the next chunk
    }
}

// LDS bytes staged per chunk of the chunked form.
constexpr int kGatherChunkBytes = 16384;

template <class S>
static int band_gather(const S *phi, const ls_grid *grid, const int32_t *tiles,
                       const int32_t *ntiles_dev, S *out, int32_t *ids_out, int64_t capacity,
                       hipStream_t stream) {
    Geom G;
    int rc = make_geom(grid, &G);
    if (rc != LS_OK) return rc;
    if (!phi || !tiles || !ntiles_dev || !out) {
        set_error("gather: phi, tiles, ntiles_dev and out must be non-NULL");
        return LS_ERR_ARG;
    }
    if (capacity < 0 || capacity > G.ntiles) {
        set_error("gather: capacity must be in [0, %lld] (got %lld)", (long long)G.ntiles,
                  (long long)capacity);
        return LS_ERR_ARG;
    }
    if (capacity == 0) return LS_OK;
    const int64_t tp = int64_t(G.tx) * G.ty * G.tz;
    if (tp > INT32_MAX / 4) {
        set_error("gather: tile of %lld points too large", (long long)tp);
        return LS_ERR_UNSUPPORTED;
    }
    GatherGeom g;
    g.nx = G.nx, g.ny = G.ny, g.nz = G.nz;
    g.tx = G.tx, g.ty = G.ty, g.tz = G.tz;
    g.ntx = G.ntx, g.nty = G.nty;
    g.tp = static_cast<int32_t>(tp);
    g.ntiles = G.ntiles;
    g.capacity = capacity;
    DeviceInfo di;
    if ((rc = device_info(&di)) != LS_OK) return rc;
    int64_t slot;
    if ((rc = stats_before(LS_KERNEL_GATHER, stream, &slot)) != LS_OK) return rc;
    bool quads = false;
    if constexpr (!std::is_same<S, double>::value) {
        using T = typename GatherQuad<S>::T;
        quads = G.tx % 4 == 0 && G.nx % 4 == 0 &&
                reinterpret_cast<uintptr_t>(phi) % sizeof(T) == 0 &&
                reinterpret_cast<uintptr_t>(out) % sizeof(T) == 0;
        const int64_t chunk_tiles = kGatherChunkBytes / (tp * int64_t(sizeof(S)));
        if (quads && chunk_tiles >= 2) {
            const int chunk = static_cast<int>(chunk_tiles);
            const int64_t chunks = cdiv64(capacity, chunk);
            const unsigned blocks = static_cast<unsigned>(
                std::max<int64_t>(1, std::min<int64_t>(chunks, int64_t(di.cus) * 8)));
            const size_t lds = static_cast<size_t>(chunk) * tp * sizeof(S);
            hipLaunchKernelGGL((band_gather_chunk_kernel<S, T>), dim3(blocks), dim3(kBlock), lds,
                               stream, g, chunk, phi, tiles, ntiles_dev, out, ids_out);
            LS_LAUNCH_CHECK("band_gather_chunk_kernel");
        } else if (quads) {
            const int64_t work = capacity * (tp / 4);
            const unsigned blocks = static_cast<unsigned>(
                std::max<int64_t>(1, std::min<int64_t>(cdiv64(work, kBlock), int64_t(di.cus) * 16)));
            hipLaunchKernelGGL((band_gather_kernel<S, T, 4>), dim3(blocks), dim3(kBlock), 0, stream,
                               g, phi, tiles, ntiles_dev, out, ids_out);
            LS_LAUNCH_CHECK("band_gather_kernel");
        }
    }
    if (!quads) {
        const int64_t work = capacity * tp;
        const unsigned blocks = static_cast<unsigned>(
            std::max<int64_t>(1, std::min<int64_t>(cdiv64(work, kBlock), int64_t(di.cus) * 16)));
        hipLaunchKernelGGL((band_gather_kernel<S, S, 1>), dim3(blocks), dim3(kBlock), 0, stream, g,
                           phi, tiles, ntiles_dev, out, ids_out);
        LS_LAUNCH_CHECK("band_gather_kernel");
    }
    return stats_after(LS_KERNEL_GATHER, stream, slot);
}

// Counted copy: units [first, n) of `unit` bytes, n = min(max(*count, 0),
// max_units), moved as elements of type T (the widest width that divides the
// unit and both addresses), grid-stride; block 0's first thread stores n to
// *count_out when it is non-NULL.  The count is read on the device, so a copy
// of exactly the units a preceding kernel produced is enqueued without the
// host waiting for that kernel.
template <class T>
__global__ __launch_bounds__(kBlock) void copy_counted_kernel(T *__restrict__ dst,
                                                              const T *__restrict__ src,
                                                              const int32_t *__restrict__ count,
                                                              int64_t per_unit, int64_t first,
                                                              int64_t max_units,
                                                              int32_t *__restrict__ count_out) {
    const int64_t n = min(static_cast<int64_t>(max(*count, 0)), max_units);
    if (count_out && blockIdx.x == 0 && threadIdx.x == 0) *count_out = static_cast<int32_t>(n);
    const int64_t total = n * per_unit;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    int64_t i = first * per_unit + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    // four elements per thread and pass, all loads before the stores, so that
    // more writes to the destination (host memory over the link) are in flight
    for (; i + 3 * stride < total; i += 4 * stride) {
        T v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) dst[i + k * stride] = v[k];
    }
    for (; i < total; i += stride) dst[i] = src[i];
}

template <class T>
static int copy_counted(void *dst, const void *src, const int32_t *count, int64_t unit_bytes,
                        int64_t first, int64_t max_units, int32_t *count_out, unsigned blocks,
                        hipStream_t stream) {
    const int64_t per_unit = unit_bytes / static_cast<int64_t>(sizeof(T));
    hipLaunchKernelGGL((copy_counted_kernel<T>), dim3(blocks), dim3(kBlock), 0, stream,
                       static_cast<T *>(dst), static_cast<const T *>(src), count, per_unit, first,
                       max_units, count_out);
    LS_LAUNCH_CHECK("copy_counted_kernel");
    return LS_OK;
}

}  // namespace ls

extern "C" {

int ls_copy_counted_from(void *dst, const void *src, const int32_t *count_dev,
                         int64_t unit_bytes, int64_t first_unit, int64_t max_units,
                         int32_t *count_out, int blocks, void *stream) {
    ls::clear_error();
    if (!dst || !src || !count_dev) {
        ls::set_error("copy_counted: dst, src and count_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (unit_bytes <= 0 || max_units < 0 || max_units > INT32_MAX || blocks < 0 ||
        first_unit < 0 || first_unit > max_units) {
        ls::set_error("copy_counted: unit_bytes must be > 0, max_units in [0, 2^31), first_unit "
                      "in [0, max_units], blocks >= 0 (got %lld, %lld, %lld, %d)",
                      (long long)unit_bytes, (long long)max_units, (long long)first_unit, blocks);
        return LS_ERR_ARG;
    }
    if (max_units > INT64_MAX / unit_bytes) {
        ls::set_error("copy_counted: %lld units of %lld bytes overflow", (long long)max_units,
                      (long long)unit_bytes);
        return LS_ERR_ARG;
    }
    unsigned nb = static_cast<unsigned>(blocks);
    if (nb == 0) {
        ls::DeviceInfo di;
        const int rc = ls::device_info(&di);
        if (rc != LS_OK) return rc;
        nb = static_cast<unsigned>(di.cus) / 4;
    }
    const int64_t bytes = unit_bytes * (max_units - first_unit);
    nb = static_cast<unsigned>(
        std::max<int64_t>(1, std::min<int64_t>(nb, ls::cdiv64(bytes, 16 * ls::kBlock))));
    const uintptr_t align = reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src) |
                            static_cast<uintptr_t>(unit_bytes);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t f = first_unit;
    if (align % 16 == 0)
        return ls::copy_counted<uint4>(dst, src, count_dev, unit_bytes, f, max_units, count_out,
                                       nb, s);
    if (align % 8 == 0)
        return ls::copy_counted<uint2>(dst, src, count_dev, unit_bytes, f, max_units, count_out,
                                       nb, s);
    if (align % 4 == 0)
        return ls::copy_counted<uint32_t>(dst, src, count_dev, unit_bytes, f, max_units,
                                          count_out, nb, s);
    if (align % 2 == 0)
        return ls::copy_counted<uint16_t>(dst, src, count_dev, unit_bytes, f, max_units,
                                          count_out, nb, s);
    return ls::copy_counted<uint8_t>(dst, src, count_dev, unit_bytes, f, max_units, count_out, nb,
                                     s);
}

int ls_copy_counted(void *dst, const void *src, const int32_t *count_dev, int64_t unit_bytes,
                    int64_t max_units, int32_t *count_out, int blocks, void *stream) {
    return ls_copy_counted_from(dst, src, count_dev, unit_bytes, 0, max_units, count_out, blocks,
                                stream);
}

int ls_band_gather_f32(const float *phi, const ls_grid *g, const int32_t *tiles,
                       const int32_t *ntiles_dev, float *out, int32_t *ids_out, int64_t capacity,
                       void *stream) {
    ls::clear_error();
    return ls::band_gather<float>(phi, g, tiles, ntiles_dev, out, ids_out, capacity,
                                  static_cast<hipStream_t>(stream));
}

int ls_band_gather_f64(const double *phi, const ls_grid *g, const int32_t *tiles,
                       const int32_t *ntiles_dev, double *out, int32_t *ids_out,
                       int64_t capacity, void *stream) {
    ls::clear_error();
    return ls::band_gather<double>(phi, g, tiles, ntiles_dev, out, ids_out, capacity,
                                   static_cast<hipStream_t>(stream));
}

int ls_band_gather_f16s(const uint16_t *phi_h, const ls_grid *g, const int32_t *tiles,
                        const int32_t *ntiles_dev, uint16_t *out, int32_t *ids_out,
                        int64_t capacity, void *stream) {
    ls::clear_error();
    return ls::band_gather<uint16_t>(phi_h, g, tiles, ntiles_dev, out, ids_out, capacity,
                                     static_cast<hipStream_t>(stream));
}

}  // extern "C"
