// Ordered stream compaction with wavefront ballots.
//
// Indices idx in [0, n) with pred(idx) true are written in ascending order.
// Three launches: per-block counts, an exclusive scan of the counts (also
// writing the total), and a scatter in which every wave ranks its lanes with
// ballot + mbcnt and the block ranks its waves through LDS.  No atomics, so
// the output order (and every bit of it) is deterministic.  Two predicates
// can share the launches ("dual" compaction, e.g. the band list and the heads
// of its work items in one pass over the tile ids).
#pragma once

#include "ls_internal.h"

namespace ls {

struct NullPred {
    __device__ bool operator()(int64_t) const { return false; }
};
struct NullEmit {
    __device__ void operator()(int, int64_t) const {}
};

__device__ inline int64_t compact_extent(const int32_t *n_dev, int64_t n_host) {
    // a device count never exceeds the capacity n_host (clamped for safety)
    return n_dev ? min(max(static_cast<int64_t>(*n_dev), int64_t(0)), n_host) : n_host;
}

template <class PA, class PB>
__global__ __launch_bounds__(kBlock) void compact_count_kernel(PA pa, PB pb, const int32_t *n_dev,
                                                               int64_t n_host, int32_t *blk_a,
                                                               int32_t *blk_b) {
    const int64_t n = compact_extent(n_dev, n_host);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kCompactChunk;
    __shared__ int wave_tot[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int ca = 0, cb = 0;
    if (base < n) {
#pragma unroll
        for (int r = 0; r < kCompactRounds; ++r) {
            const int64_t idx = base + r * kBlock + threadIdx.x;
            const bool in = idx < n;
            ca += __popcll(__ballot(in && pa(idx)));
            cb += __popcll(__ballot(in && pb(idx)));
        }
    }
    if (lane == 0) {
        wave_tot[0][wave] = ca;
        wave_tot[1][wave] = cb;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        int s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += wave_tot[threadIdx.x][w];
        int32_t *blk = threadIdx.x == 0 ? blk_a : blk_b;
        if (blk) blk[blockIdx.x] = s;
    }
}

// Exclusive scan of blk[0..nblk) in place, total to blk[nblk] and *count.
// Block 0 scans (blk_a, count_a), block 1 (blk_b, count_b) when blk_b is set.
__global__ __launch_bounds__(1024) void compact_scan_kernel(int32_t *blk_a, int32_t *count_a,
                                                            int32_t *blk_b, int32_t *count_b,
                                                            int64_t nblk);

template <class PA, class EA, class PB, class EB>
__global__ __launch_bounds__(kBlock) void compact_scatter_kernel(PA pa, EA ea, PB pb, EB eb,
                                                                 const int32_t *n_dev,
                                                                 int64_t n_host,
                                                                 const int32_t *blk_a,
                                                                 const int32_t *blk_b) {
    const int64_t n = compact_extent(n_dev, n_host);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kCompactChunk;
    if (base >= n) return;  // uniform per block
    __shared__ int wave_cnt[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int run_a = blk_a[blockIdx.x];
    int run_b = blk_b ? blk_b[blockIdx.x] : 0;
    for (int r = 0; r < kCompactRounds; ++r) {
        const int64_t idx = base + r * kBlock + threadIdx.x;
        const bool in = idx < n;
        const bool a = in && pa(idx);
        const bool b = in && pb(idx);
        const uint64_t ma = __ballot(a);
        const uint64_t mb = __ballot(b);
        if (lane == 0) {
            wave_cnt[0][wave] = __popcll(ma);
            wave_cnt[1][wave] = __popcll(mb);
        }
        __syncthreads();
        int before_a = 0, total_a = 0, before_b = 0, total_b = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            const int c0 = wave_cnt[0][w], c1 = wave_cnt[1][w];
            before_a += (w < wave) ? c0 : 0;
            before_b += (w < wave) ? c1 : 0;
            total_a += c0;
            total_b += c1;
        }
        if (a) ea(run_a + before_a + lane_prefix(ma), idx);
        if (b) eb(run_b + before_b + lane_prefix(mb), idx);
        run_a += total_a;
        run_b += total_b;
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

// Compacts pa (into ea, count_a) and, unless blk_b is null, pb (into eb,
// count_b) over [0, n): n = *n_dev (clamped to n_cap) or n_cap.
template <class PA, class EA, class PB = NullPred, class EB = NullEmit>
int compact2(PA pa, EA ea, int32_t *count_a, int32_t *blk_a, PB pb, EB eb, int32_t *count_b,
             int32_t *blk_b, const int32_t *n_dev, int64_t n_cap, hipStream_t stream) {
    const int64_t nblk = cdiv64(n_cap, kCompactChunk);
    if (nblk > 0) {
        hipLaunchKernelGGL((compact_count_kernel<PA, PB>), dim3(static_cast<unsigned>(nblk)),
                           dim3(kBlock), 0, stream, pa, pb, n_dev, n_cap, blk_a, blk_b);
        LS_LAUNCH_CHECK("compact_count_kernel");
    }
    hipLaunchKernelGGL(compact_scan_kernel, dim3(blk_b ? 2 : 1), dim3(1024), 0, stream, blk_a,
                       count_a, blk_b, count_b, nblk);
    LS_LAUNCH_CHECK("compact_scan_kernel");
    if (nblk > 0) {
        hipLaunchKernelGGL((compact_scatter_kernel<PA, EA, PB, EB>),
                           dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, stream, pa, ea, pb,
                           eb, n_dev, n_cap, static_cast<const int32_t *>(blk_a),
                           static_cast<const int32_t *>(blk_b));
        LS_LAUNCH_CHECK("compact_scatter_kernel");
    }
    return LS_OK;
}

template <class Pred, class Emit>
int compact(Pred pred, Emit emit, const int32_t *n_dev, int64_t n_cap, int32_t *count,
            int32_t *blk, hipStream_t stream) {
    return compact2(pred, emit, count, blk, NullPred{}, NullEmit{}, nullptr, nullptr, n_dev,
                    n_cap, stream);
}

}  // namespace ls
