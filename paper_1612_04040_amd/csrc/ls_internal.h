// Internal helpers of libls: error state, grid geometry, workspace layout,
// storage codecs and the ordered (ballot / mbcnt) compaction used by the band
// build and by the step's work-item list.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>

#include "ls.h"

namespace ls {

// ---------------------------------------------------------------------------
// error state

void set_error(const char *fmt, ...);
void clear_error();

#define LS_HIP_CHECK(expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::ls::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                            __FILE__, __LINE__);                                        \
            return LS_ERR_HIP;                                                          \
        }                                                                               \
    } while (0)

#define LS_LAUNCH_CHECK(what)                                                           \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess) {                                                         \
            ::ls::set_error("launch of %s failed: %s", what, hipGetErrorString(e_));    \
            return LS_ERR_HIP;                                                          \
        }                                                                               \
    } while (0)

// ---------------------------------------------------------------------------
// geometry

struct Geom {
    int32_t nx, ny, nz;
    int32_t tx, ty, tz;
    int32_t ntx, nty, ntz;
    int64_t ntiles;
    int64_t npoints;
    int32_t elem_bytes;  // bytes of a stored phi value (sets the default run width); 4 if unset
    int32_t run_tiles = 0;  // tiles per work item when > 0 (else from the run width)
};

// Validates g and fills out; returns LS_OK or a status with the message set.
int make_geom(const ls_grid *g, Geom *out);

// Threads of every kernel block in this library.
constexpr int kBlock = 256;
// Tiles examined per block by the compaction kernels (kCompactRounds rounds
// of kBlock).
constexpr int kCompactRounds = 4;
constexpr int kCompactChunk = kBlock * kCompactRounds;
// int32 words of one work-item record of the band step.
constexpr int kItemWords = 8;

// Workspace layout (byte offsets), all regions 256-byte aligned.
struct Workspace {
    int64_t a_flags;     // uint8[ntiles]   tile holds a point with |phi| < gamma
    int64_t u_map;       // uint8[ntiles]   tile is in the update set
    int64_t blk_counts;  // int32[nblk + 1] per-block counts, then offsets
    int64_t blk_counts2; // int32[nblk + 1] same, second predicate of a dual compaction
    int64_t items;       // int32[8*ntiles] work-item records of the band step
    int64_t prev_list;   // int32[ntiles]   band list of the previous window (driver)
    int64_t counters;    // int32[64]       [0] item count, [1] previous-list count
    int64_t total;
    int64_t nblk;        // compaction blocks for ntiles entries
};
Workspace workspace_layout(const Geom &g);

// Checks the workspace argument against the layout for g.
int check_workspace(const Geom &g, const void *ws, int64_t ws_bytes);

inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device properties of the current device, cached per device.
struct DeviceInfo {
    int cus;
};
int device_info(DeviceInfo *out);

// ---------------------------------------------------------------------------
// storage codecs: stored type S <-> compute type C

template <class S>
struct Codec;

template <>
struct Codec<float> {
    using C = float;
    __device__ static inline float load(float v, float) { return v; }
    __device__ static inline float store(float v, float) { return v; }
};

template <>
struct Codec<double> {
    using C = double;
    __device__ static inline double load(double v, double) { return v; }
    __device__ static inline double store(double v, double) { return v; }
};

// Scaled FP16: h = fp16(phi / s) with round to nearest even; phi = fl32(h * s).
template <>
struct Codec<uint16_t> {
    using C = float;
    __device__ static inline float load(uint16_t h, float s) {
        _Float16 v = __builtin_bit_cast(_Float16, h);
        return static_cast<float>(v) * s;
    }
    __device__ static inline uint16_t store(float v, float s) {
        _Float16 h = static_cast<_Float16>(v / s);
        return __builtin_bit_cast(uint16_t, h);
    }
};

// ---------------------------------------------------------------------------
// wave-level helpers (wave64)

// Optional accumulation by a band build of (listed tiles) x mul into a
// device counter (the tile-steps numerator of the drivers): added once the
// list is counted, in the same launch.
struct TileAccum {
    int64_t *acc = nullptr;
    int mul = 0;
};

__device__ inline int lane_prefix(uint64_t mask) {
    // number of set bits of `mask` below this lane (v_mbcnt_lo / v_mbcnt_hi)
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// ---------------------------------------------------------------------------
// host launchers (defined in ls_band.hip)

// Tiles per work item of the band step for this geometry (the launch tuning's
// run width over tx, at least 1, at most 32).
int plan_run_tiles(const Geom &g);

// The step plan of a band: from the update map u_map (one byte per tile,
// complete in the workspace) and, when list != nullptr, the ordered band list
// (count in *list_count), writes the work-item records and their count.  One
// dual ordered compaction over the tile ids plus a record kernel.
int build_plan(const Geom &g, uint8_t *ws, int32_t *list, int32_t *list_count,
               hipStream_t stream, TileAccum accum = TileAccum{});

// Band build (full scan) and exact incremental rebuild of one grid, behind
// the ls_band_build_* / ls_band_rebuild_* entry points (ls_band.hip); accum
// adds (band tiles) x accum.mul to *accum.acc in the same launches.
template <class S>
int band_build(const S *phi, typename Codec<S>::C scale, const ls_grid *grid,
               typename Codec<S>::C gamma, int dilate, int32_t *tiles, int64_t capacity,
               int32_t *ntiles_dev, void *workspace, int64_t ws_bytes, void *stream_,
               TileAccum accum = TileAccum{});
template <class S>
int band_rebuild(const S *phi, typename Codec<S>::C scale, const ls_grid *grid,
                 typename Codec<S>::C gamma, const int32_t *prev_tiles,
                 const int32_t *prev_ntiles_dev, int32_t *tiles, int64_t capacity,
                 int32_t *ntiles_dev, void *workspace, int64_t ws_bytes, void *stream_,
                 bool flags_valid, TileAccum accum = TileAccum{});

}  // namespace ls
