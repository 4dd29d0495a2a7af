// Ordered stream compaction with wavefront ballots.
//
// Indices idx in [0, n) with pred(idx) true are written in ascending order.
// Three launches: per-block counts, a one-block exclusive scan of the counts
// (also writing the total), and a scatter in which every wave ranks its lanes
// with ballot + mbcnt and the block ranks its waves through LDS.  No atomics,
// so the output order (and every bit of it) is deterministic.
#pragma once

#include "ls_internal.h"

namespace ls {

template <class Pred>
__global__ __launch_bounds__(kBlock) void compact_count_kernel(Pred pred, const int32_t *n_dev,
                                                               int64_t n_host, int32_t *blk) {
    // a device count never exceeds the capacity n_host (clamped for safety)
    const int64_t n = n_dev ? min(max(static_cast<int64_t>(*n_dev), int64_t(0)), n_host) : n_host;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kCompactChunk;
    __shared__ int wave_tot[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int my = 0;
    if (base < n) {
#pragma unroll 4
        for (int r = 0; r < kCompactRounds; ++r) {
            const int64_t idx = base + r * kBlock + threadIdx.x;
            const bool p = idx < n && pred(idx);
            const uint64_t m = __ballot(p);
            my += __popcll(m);
        }
    }
    if (lane == 0) wave_tot[wave] = my;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += wave_tot[w];
        blk[blockIdx.x] = s;
    }
}

// Exclusive scan of blk[0..nblk) in place, total to blk[nblk] and *count.
__global__ __launch_bounds__(1024) void compact_scan_kernel(int32_t *blk, int64_t nblk,
                                                            int32_t *count);

template <class Pred, class Emit>
__global__ __launch_bounds__(kBlock) void compact_scatter_kernel(Pred pred, Emit emit,
                                                                 const int32_t *n_dev,
                                                                 int64_t n_host,
                                                                 const int32_t *blk) {
    // a device count never exceeds the capacity n_host (clamped for safety)
    const int64_t n = n_dev ? min(max(static_cast<int64_t>(*n_dev), int64_t(0)), n_host) : n_host;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kCompactChunk;
    if (base >= n) return;  // uniform per block
    __shared__ int wave_cnt[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int running = blk[blockIdx.x];
    for (int r = 0; r < kCompactRounds; ++r) {
        const int64_t idx = base + r * kBlock + threadIdx.x;
        const bool p = idx < n && pred(idx);
        const uint64_t m = __ballot(p);
        if (lane == 0) wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            const int c = wave_cnt[w];
            before += (w < wave) ? c : 0;
            total += c;
        }
        if (p) emit(running + before + lane_prefix(m), idx);
        running += total;
        __syncthreads();
    }
}

// Predicate / emitter used by the band build: nonzero bytes of a tile map.
struct MapPred {
    const uint8_t *map;
    __device__ bool operator()(int64_t idx) const { return map[idx] != 0; }
};
struct EmitIndex {
    int32_t *out;
    __device__ void operator()(int pos, int64_t idx) const { out[pos] = static_cast<int32_t>(idx); }
};

template <class Pred, class Emit>
int compact(Pred pred, Emit emit, const int32_t *n_dev, int64_t n_cap, int32_t *count,
            int32_t *blk, hipStream_t stream) {
    const int64_t nblk = cdiv64(n_cap, kCompactChunk);
    if (nblk > 0) {
        hipLaunchKernelGGL(compact_count_kernel<Pred>, dim3(static_cast<unsigned>(nblk)),
                           dim3(kBlock), 0, stream, pred, n_dev, n_cap, blk);
        LS_LAUNCH_CHECK("compact_count_kernel");
    }
    hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(1024), 0, stream, blk, nblk, count);
    LS_LAUNCH_CHECK("compact_scan_kernel");
    if (nblk > 0) {
        hipLaunchKernelGGL((compact_scatter_kernel<Pred, Emit>), dim3(static_cast<unsigned>(nblk)),
                           dim3(kBlock), 0, stream, pred, emit, n_dev, n_cap,
                           static_cast<const int32_t *>(blk));
        LS_LAUNCH_CHECK("compact_scatter_kernel");
    }
    return LS_OK;
}

}  // namespace ls
