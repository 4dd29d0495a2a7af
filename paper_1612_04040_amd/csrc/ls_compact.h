// Ordered stream compaction with wavefront ballots.
//
// Indices idx in [0, n) with pred(idx) true are written in ascending order.
// Two launches: per-block counts, then a scatter in which every block first
// sums the counts of the blocks before it (its output offset; the last block
// also writes the totals), every wave ranks its lanes with ballot + mbcnt and
// the block ranks its waves through LDS.  No atomics, so the output order
// (and every bit of it) is deterministic.  Two predicates can share the
// launches ("dual" compaction, e.g. the band list and the heads of its work
// items in one pass over the tile ids).
#pragma once

#include <algorithm>

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

__device__ inline int wave_sum(int v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <class PA, class EA, class PB, class EB>
__global__ __launch_bounds__(kBlock) void compact_scatter_kernel(
    PA pa, EA ea, PB pb, EB eb, const int32_t *n_dev, int64_t n_host, const int32_t *blk_a,
    const int32_t *blk_b, int32_t *count_a, int32_t *count_b, TileAccum accum, int64_t nblk) {
    const int64_t n = compact_extent(n_dev, n_host);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kCompactChunk;
    const bool last = blockIdx.x == nblk - 1;
    if (base >= n && !last) return;  // uniform per block
    __shared__ int wave_cnt[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // output offsets: the counts of the blocks before this one
    int sa = 0, sb = 0;
    for (int64_t i = threadIdx.x; i < blockIdx.x; i += kBlock) {
        sa += blk_a[i];
        if (blk_b) sb += blk_b[i];
    }
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    if (lane == 0) {
        wave_cnt[0][wave] = sa;
        wave_cnt[1][wave] = sb;
    }
    __syncthreads();
    int run_a = 0, run_b = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        run_a += wave_cnt[0][w];
        run_b += wave_cnt[1][w];
    }
    if (last && threadIdx.x == 0) {
        const int ta = run_a + blk_a[blockIdx.x];
        if (count_a) *count_a = ta;
        if (count_b) *count_b = run_b + (blk_b ? blk_b[blockIdx.x] : 0);
        if (accum.acc) *accum.acc += static_cast<int64_t>(ta) * accum.mul;
    }
    __syncthreads();  // wave_cnt is reused below
    if (base >= n) return;  // uniform: the last block past the extent
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
// count_b) over [0, n): n = *n_dev (clamped to n_cap) or n_cap.  With
// accum.acc set, *accum.acc += count_a * accum.mul.
template <class PA, class EA, class PB = NullPred, class EB = NullEmit>
int compact2(PA pa, EA ea, int32_t *count_a, int32_t *blk_a, PB pb, EB eb, int32_t *count_b,
             int32_t *blk_b, const int32_t *n_dev, int64_t n_cap, hipStream_t stream,
             TileAccum accum = TileAccum{}) {
    const int64_t nblk = std::max<int64_t>(1, cdiv64(n_cap, kCompactChunk));
    hipLaunchKernelGGL((compact_count_kernel<PA, PB>), dim3(static_cast<unsigned>(nblk)),
                       dim3(kBlock), 0, stream, pa, pb, n_dev, n_cap, blk_a, blk_b);
    LS_LAUNCH_CHECK("compact_count_kernel");
    hipLaunchKernelGGL((compact_scatter_kernel<PA, EA, PB, EB>), dim3(static_cast<unsigned>(nblk)),
                       dim3(kBlock), 0, stream, pa, ea, pb, eb, n_dev, n_cap,
                       static_cast<const int32_t *>(blk_a), static_cast<const int32_t *>(blk_b),
                       count_a, count_b, accum, nblk);
    LS_LAUNCH_CHECK("compact_scatter_kernel");
    return LS_OK;
}

template <class Pred, class Emit>
int compact(Pred pred, Emit emit, const int32_t *n_dev, int64_t n_cap, int32_t *count,
            int32_t *blk, hipStream_t stream) {
    return compact2(pred, emit, count, blk, NullPred{}, NullEmit{}, nullptr, nullptr, n_dev,
                    n_cap, stream);
}

}  // namespace ls
