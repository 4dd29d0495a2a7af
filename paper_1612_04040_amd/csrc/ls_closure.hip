// Learned closure of the coarse first-order step: a 3-layer 3^3-conv network
// (3 -> 16 -> 16 -> 1 channels, SiLU) whose output r corrects the plain coarse
// update on the active tiles, phi + delta_plain + dx * r, trained toward fine
// runs of the same scheme restricted 4x.  BF16 weights and activations, FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Every convolution is an implicit GEMM over the 8^3 tiles of a tile list:
// one block per tile stages the tile and its one-point halo (10^3 points,
// channel-last) in LDS; the 16 output channels are the MFMA rows, 16 output
// points its columns, and the reduction runs over (tap, input channel) in
// chunks of 32.  Activations outside the band count as zero; since the active
// tiles lie one tile deep inside the band and the network sees 3 points
// around a point, r on the active tiles is the same as with no band at all.
#include <algorithm>
#include <cmath>

#include "ls_compact.h"
#include "ls_stats.h"
#include "ls_stencil.h"

namespace ls {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 8;          // closure tile edge (8^3 tiles)
constexpr int kP = kT + 2;     // patch edge with the one-point halo
constexpr int kTaps = 27;
// flat parameter layout (FP32 master copy), numpy order (out, in, dz, dy, dx)
constexpr int kW0 = 0, kB0 = kW0 + 16 * 3 * 27, kW1 = kB0 + 16, kB1 = kW1 + 16 * 16 * 27,
              kW2 = kB1 + 16, kB2 = kW2 + 1 * 16 * 27, kNParams = kB2 + 1;
static_assert(kNParams == 8673, "parameter count");

__device__ inline __bf16 to_bf16(float v) { return static_cast<__bf16>(v); }
__device__ inline float from_bf16(__bf16 v) { return static_cast<float>(v); }
// SiLU with the hardware reciprocal (about 1 ulp; the result is rounded to
// BF16 or feeds a BF16-rounded product)
__device__ inline float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
// Cut-off function of Eq. 8 with beta = gamma / 2, in u = |phi| / gamma:
// 1 for u <= 1/2, 8 (u - 1)^2 (2u - 1/2) for 1/2 < u <= 1, 0 beyond.
__device__ inline float cutoff_f(float phi, float inv_gamma) {
    const float u = fabsf(phi) * inv_gamma;
    if (u <= 0.5f) return 1.0f;
    if (u <= 1.0f) return 8.0f * (u - 1.0f) * (u - 1.0f) * (2.0f * u - 0.5f);
    return 0.0f;
}
__device__ inline float silu_grad_f(float z) {
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// weight packing: the MFMA A operand of every reduction chunk, per lane.
//   CIN = 16: chunk c, k = 8*(lane/16) + j: tap 2c + k/16, input channel k%16
//   CIN = 4:  chunk c, k = 8*(lane/16) + j: tap 8c + k/4,  input channel k%4
// row (output channel) = lane % 16.  Taps >= 27, channels beyond the real
// ones and rows beyond the real outputs are zero.  `flip` packs the
// transposed, tap-reversed weights of the backward (data-gradient) conv.

template <int CIN>
constexpr int nchunk() { return CIN == 16 ? 14 : 4; }

struct PackSpec {
    int woff;       // offset of the layer's weights in the flat parameters
    int cin, cout;  // real channel counts of the layer (forward)
    int pcin;       // packed input width: 4 or 16
    bool flip;      // backward: swap in/out and reverse the taps
};

__global__ void pack_weights_kernel(const float *__restrict__ params, __bf16 *__restrict__ out,
                                    PackSpec s) {
    const int nch = s.pcin == 16 ? 14 : 4;
    const int total = nch * 64 * 8;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int c = i / 512, lane = (i / 8) % 64, j = i % 8;
        const int k = 8 * (lane / 16) + j;
        const int row = lane % 16;
        int tap, ci;
        if (s.pcin == 16) {
            tap = 2 * c + k / 16;
            ci = k % 16;
        } else {
            tap = 8 * c + k / 4;
            ci = k % 4;
        }
        float v = 0.f;
        if (tap < kTaps) {
            // forward: w[out=row][in=ci][tap]; backward: w[out=ci][in=row][26-tap]
            const int o = s.flip ? ci : row, in = s.flip ? row : ci;
            const int t = s.flip ? kTaps - 1 - tap : tap;
            if (o < s.cout && in < s.cin) v = params[s.woff + (o * s.cin + in) * kTaps + t];
        }
        out[i] = to_bf16(v);
    }
}

// ---------------------------------------------------------------------------
// the convolution kernel

struct ConvGeo {
    int nx, ny, nz;
    int ntx, nty, ntz;
};

// Input of a CIN = 4 convolution, built on the fly per patch point:
//  FEAT: (clip(phi/gamma, +-2), F / Fmax, (plain - phi)/dx, 0) of the band;
//  GRAD: (g, 0, 0, 0) with g the loss gradient w.r.t. r (FP32, dense).
struct In4 {
    const float *phi, *F, *plain, *g;
    float inv_gamma, inv_fmax, inv_dx;
};

enum { OUT_HIDDEN = 0, OUT_LAST = 1, OUT_GRAD = 2 };

// One block per listed tile.  CIN: 16 (input bf16 x16 channel-last) or 4
// (In4 source).  MODE: OUT_HIDDEN writes z (pre-activation) and a = SiLU(z),
// bf16 x16; OUT_LAST writes r = row 0 (+ bias) as FP32 and, when `apply`,
// corrects the plain step on the tile (phi_next += dx*c(phi)*r, c the cut-off
// of Eq. 8, phi from in4.phi) unless some c(phi)*r of the tile is non-finite
// or above 1/2 (then counts a fallback); OUT_GRAD
// writes acc * SiLU'(z) as bf16 x16 (z read from zin).
template <int CIN, int MODE>
__global__ __launch_bounds__(kBlock) void closure_conv_kernel(
    ConvGeo g, const int32_t *__restrict__ tiles, const int32_t *__restrict__ ntiles_dev,
    int ntiles_cap, const uint8_t *__restrict__ umap, const __bf16 *__restrict__ in16, In4 in4,
    const __bf16 *__restrict__ wpack, const float *__restrict__ bias, __bf16 *__restrict__ zout,
    __bf16 *__restrict__ aout, const __bf16 *__restrict__ zin, float *__restrict__ rout,
    float *__restrict__ phi_next, float dx, int32_t *__restrict__ fallbacks) {
    constexpr int NCH = nchunk<CIN>();
    __shared__ __align__(16) __bf16 patch[kP * kP * kP * CIN];
    __shared__ int bad_s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = min(*ntiles_dev, ntiles_cap);

    // weights of this lane: one 8-wide A operand per chunk
    bf16x8 wa[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        wa[c] = *reinterpret_cast<const bf16x8 *>(wpack + (c * 64 + lane) * 8);

    for (int p = blockIdx.x; p < n; p += gridDim.x) {
        const int t = tiles[p];
        if (t < 0 || t >= g.ntx * g.nty * g.ntz) continue;  // uniform
        const int ti = t % g.ntx, rr = t / g.ntx;
        const int tj = rr % g.nty, tk = rr / g.nty;
        const int x0 = ti * kT, y0 = tj * kT, z0 = tk * kT;

        // stage the 10^3 patch (zero outside the grid and outside the band)
        for (int q = threadIdx.x; q < kP * kP * kP; q += kBlock) {
            const int px = q % kP, py = (q / kP) % kP, pz = q / (kP * kP);
            const int gx = x0 + px - 1, gy = y0 + py - 1, gz = z0 + pz - 1;
            bool ok = gx >= 0 && gy >= 0 && gz >= 0 && gx < g.nx && gy < g.ny && gz < g.nz;
            if (ok) {
                const int nt = ((gz / kT) * g.nty + gy / kT) * g.ntx + gx / kT;
                ok = umap[nt] != 0;
            }
            const int64_t gi = (static_cast<int64_t>(gz) * g.ny + gy) * g.nx + gx;
            if constexpr (CIN == 16) {
                uint4 lo = make_uint4(0, 0, 0, 0), hi = lo;
                if (ok) {
                    const uint4 *src = reinterpret_cast<const uint4 *>(in16 + gi * 16);
                    lo = src[0];
                    hi = src[1];
                }
                uint4 *dst = reinterpret_cast<uint4 *>(patch + q * 16);
                dst[0] = lo;
                dst[1] = hi;
            } else {
                float v0 = 0.f, v1 = 0.f, v2 = 0.f;
                if (ok) {
                    if (in4.g) {
                        v0 = in4.g[gi];
                    } else {
                        const float ph = in4.phi[gi];
                        v0 = fminf(fmaxf(ph * in4.inv_gamma, -2.f), 2.f);
                        v1 = in4.F[gi] * in4.inv_fmax;
                        v2 = (in4.plain[gi] - ph) * in4.inv_dx;
                    }
                }
                patch[q * 4 + 0] = to_bf16(v0);
                patch[q * 4 + 1] = to_bf16(v1);
                patch[q * 4 + 2] = to_bf16(v2);
                patch[q * 4 + 3] = to_bf16(0.f);
            }
        }
        if (MODE == OUT_LAST && threadIdx.x == 0) bad_s = 0;
        __syncthreads();

        // 32 groups of 16 output points (x fastest), 8 per wave
        const int j = lane & 15, kq = lane >> 4;
        float rvals[8];
#pragma unroll
        for (int gi8 = 0; gi8 < 8; ++gi8) {
            const int grp = wave + 4 * gi8;
            const int pt = grp * 16 + j;
            const int lx = pt & 7, ly = (pt >> 3) & 7, lz = pt >> 6;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                bf16x8 b;
                if constexpr (CIN == 16) {
                    const int tap = 2 * c + (kq >> 1);
                    if (tap < kTaps) {
                        const int dz = tap / 9, dy = (tap / 3) % 3, dxx = tap % 3;
                        const int q = ((lz + dz) * kP + (ly + dy)) * kP + (lx + dxx);
                        b = *reinterpret_cast<const bf16x8 *>(patch + q * 16 + 8 * (kq & 1));
                    } else {
                        b = bf16x8{};
                    }
                } else {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int tap = 8 * c + 2 * kq + h;
                        if (tap < kTaps) {
                            const int dz = tap / 9, dy = (tap / 3) % 3, dxx = tap % 3;
                            const int q = ((lz + dz) * kP + (ly + dy)) * kP + (lx + dxx);
#pragma unroll
                            for (int e = 0; e < 4; ++e) b[4 * h + e] = patch[q * 4 + e];
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) b[4 * h + e] = to_bf16(0.f);
                        }
                    }
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[c], b, acc, 0, 0, 0);
            }
            // acc[i] = output channel 4*kq + i of point pt
            const int64_t gpt =
                (static_cast<int64_t>(z0 + lz) * g.ny + (y0 + ly)) * g.nx + (x0 + lx);
            if constexpr (MODE == OUT_HIDDEN) {
                __bf16 zb[4], ab[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float z = acc[i] + bias[4 * kq + i];
                    zb[i] = to_bf16(z);
                    ab[i] = to_bf16(silu_f(z));
                }
                if (zout) *reinterpret_cast<uint2 *>(zout + gpt * 16 + 4 * kq) = *reinterpret_cast<uint2 *>(zb);
                *reinterpret_cast<uint2 *>(aout + gpt * 16 + 4 * kq) = *reinterpret_cast<uint2 *>(ab);
            } else if constexpr (MODE == OUT_GRAD) {
                const uint2 zr = *reinterpret_cast<const uint2 *>(zin + gpt * 16 + 4 * kq);
                const __bf16 *zv = reinterpret_cast<const __bf16 *>(&zr);
                __bf16 ob[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) ob[i] = to_bf16(acc[i] * silu_grad_f(from_bf16(zv[i])));
                *reinterpret_cast<uint2 *>(aout + gpt * 16 + 4 * kq) = *reinterpret_cast<uint2 *>(ob);
            } else {
                rvals[gi8] = acc[0] + bias[0];
                if (kq == 0) {
                    rout[gpt] = rvals[gi8];
                    // the applied correction is c(phi) r (a NaN or inf r stays non-finite)
                    if (in4.phi) rvals[gi8] *= cutoff_f(in4.phi[gpt], in4.inv_gamma);
                    if (!(fabsf(rvals[gi8]) <= 0.5f)) atomicOr(&bad_s, 1);  // NaN fails too
                }
            }
        }
        if constexpr (MODE == OUT_LAST) {
            __syncthreads();
            const bool bad = bad_s != 0;
            if (phi_next) {
                if (!bad) {
#pragma unroll
                    for (int gi8 = 0; gi8 < 8; ++gi8) {
                        const int pt = (wave + 4 * gi8) * 16 + j;
                        const int lx = pt & 7, ly = (pt >> 3) & 7, lz = pt >> 6;
                        if (kq == 0) {
                            const int64_t gpt =
                                (static_cast<int64_t>(z0 + lz) * g.ny + (y0 + ly)) * g.nx + (x0 + lx);
                            phi_next[gpt] += dx * rvals[gi8];
                        }
                    }
                } else if (threadIdx.x == 0 && fallbacks) {
                    atomicAdd(fallbacks, 1);
                }
            }
        }
        __syncthreads();  // patch free for the next tile
    }
}

// ---------------------------------------------------------------------------
// fused inference: the whole network on one active tile per block, with the
// activations in LDS.  Layer 1 runs on the 12^3 points within 2 of the tile
// (from features of the 14^3 points within 3), layer 2 on the 10^3 points
// within 1, layer 3 on the tile.  An active tile lies one tile inside the
// band, so every point read is in the band or outside the grid (zero).
//
// The three layers advance together plane by plane in z, each wave keeping
// one layer's weights in registers: wave 0 computes layer-1 plane s in step
// s, waves 1-2 layer-2 plane s-3 (from layer-1 planes s-3..s-1), wave 3
// output plane s-6 (from layer-2 planes s-6..s-4), one barrier per step; the
// gate, the limiter and the fallback test then run on the whole tile at once.
// Layer-1 and layer-2 activations live in rings of four z-planes, so a block
// holds 52 KB of LDS and three blocks share a CU.  The arithmetic of every
// point (operands, chunk order, rounding) is that of the layer-by-layer
// kernels.

constexpr int kF0 = kT + 6, kF1 = kT + 4, kF2 = kT + 2;  // 14, 12, 10
constexpr int kPl1 = kF1 * kF1, kPl2 = kF2 * kF2;        // points of a plane
constexpr size_t kFusedIn = size_t(kF0) * kF0 * kF0 * 4;  // bf16 elements
// a ring slot: one plane as two halves of 8 channels (channels 0-7, then
// 8-15), 16 bytes per point: the 16 points of an MFMA column block read 256
// contiguous bytes, free of LDS bank conflicts
constexpr size_t kSlot1 = size_t(2) * kPl1 * 8, kSlot2 = size_t(2) * kPl2 * 8;
constexpr int kRing = 4;
constexpr size_t kFusedLds = 2 * (kFusedIn + kRing * kSlot1 + kRing * kSlot2);
constexpr int kFusedSteps = kF1 + 2;  // 14: layer 1 in steps 0-11, output in 6-13
constexpr float kCorrLimit = 0.5f;    // |correction| <= kCorrLimit * |plain increment|
constexpr int kFusedBlock = 256, kL1Waves = 1, kL2Waves = 2;
constexpr int kFusedBlocksPerCu = 3;
static_assert(kFusedBlocksPerCu * (kFusedLds + 64) <= 160 * 1024, "fused LDS per CU");

// One output group of a 16-channel layer from a ring of planes: the 14
// reduction chunks (tap 2c + (lane/16)/2, 8 channels each), chunk c's B
// operand at byte base + off[c] + the ring slot of its tap's z offset (sb0,
// sb1, sb2 for dz = 0, 1, 2; tap 2c + hi has dz 0 for c < 4, hi for c = 4, 1
// for c = 5..8, 2 beyond).  Seven operand loads are kept in flight: the
// loads of chunks 0-6 first, then each product issues the load of the chunk
// seven later into the registers it has just read.
__device__ inline f32x4 ring_conv16(const bf16x8 (&wa)[14], const unsigned char *base,
                                    const int (&off)[14], int hi, int sb0, int sb1, int sb2) {
    auto at = [&](int c) {
        const int sb = c < 4 ? sb0 : (c == 4 ? (hi ? sb1 : sb0) : (c < 9 ? sb1 : sb2));
        return *reinterpret_cast<const bf16x8 *>(base + off[c] + sb);
    };
    bf16x8 b[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) b[c] = at(c);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[c], b[c], acc, 0, 0, 0);
        b[c] = at(c + 7);
    }
#pragma unroll
    for (int c = 0; c < 7; ++c)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[c + 7], b[c], acc, 0, 0, 0);
    // the order above for the scheduler: seven LDS reads, then seven pairs
    // (product, read), then seven products (masks: 0x100 LDS read, 0x8 MFMA)
    __builtin_amdgcn_sched_group_barrier(0x100, 7, 0);
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        __builtin_amdgcn_sched_group_barrier(0x8, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x8, 7, 0);
    return acc;
}

__global__ __launch_bounds__(kFusedBlock) __attribute__((amdgpu_waves_per_eu(3))) void closure_fused_kernel(
    ConvGeo g, const int32_t *__restrict__ tiles, const int32_t *__restrict__ ntiles_dev,
    int ntiles_cap, In4 feat, const __bf16 *__restrict__ wp0, const __bf16 *__restrict__ wp1,
    const __bf16 *__restrict__ wp2, const float *__restrict__ params, float *__restrict__ rout,
    float *__restrict__ corr, float dx, int32_t *__restrict__ fallbacks) {
    extern __shared__ __align__(16) unsigned char fsm[];
    __bf16 *in = reinterpret_cast<__bf16 *>(fsm);
    __bf16 *a0 = in + kFusedIn;             // layer-1 ring
    __bf16 *a1 = a0 + kRing * kSlot1;       // layer-2 ring
    const int lane = threadIdx.x & 63;
    // wave-uniform role: 0 layer 1, 1-2 layer 2, 3 layer 3
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = lane & 15, kq = lane >> 4, hi = kq >> 1;
    const int n = min(*ntiles_dev, ntiles_cap);

    for (int p = blockIdx.x; p < n; p += gridDim.x) {
        const int t = tiles[p];
        if (t < 0 || t >= g.ntx * g.nty * g.ntz) continue;  // uniform
        const int ti = t % g.ntx, rr = t / g.ntx;
        const int x0 = ti * kT, y0 = (rr % g.nty) * kT, z0 = (rr / g.nty) * kT;
        // features of the 14^3 points (zero outside the grid), in NPARTS parts
        // of the points: every load of a part issued first, then the
        // conversions and LDS stores
        constexpr int NP0 = kF0 * kF0 * kF0;
        constexpr int NPARTS = 2;
        constexpr int NQ = (NP0 + NPARTS * kFusedBlock - 1) / (NPARTS * kFusedBlock);
#pragma unroll 1
        for (int part = 0; part < NPARTS; ++part) {
            float vph[NQ], vf[NQ], vpl[NQ];
            bool vok[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const int q = threadIdx.x + (part * NQ + k) * kFusedBlock;
                const int px = q % kF0, py = (q / kF0) % kF0, pz = q / (kF0 * kF0);
                const int gx = x0 + px - 3, gy = y0 + py - 3, gz = z0 + pz - 3;
                vok[k] = q < NP0 && gx >= 0 && gy >= 0 && gz >= 0 && gx < g.nx && gy < g.ny &&
                         gz < g.nz;
                vph[k] = vf[k] = vpl[k] = 0.f;
                if (vok[k]) {
                    const int64_t gi = (static_cast<int64_t>(gz) * g.ny + gy) * g.nx + gx;
                    vph[k] = feat.phi[gi];
                    vf[k] = feat.F[gi];
                    vpl[k] = feat.plain[gi];
                }
            }
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const int q = threadIdx.x + (part * NQ + k) * kFusedBlock;
                if (q < NP0) {
                    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
                    if (vok[k]) {
                        v0 = fminf(fmaxf(vph[k] * feat.inv_gamma, -2.f), 2.f);
                        v1 = vf[k] * feat.inv_fmax;
                        v2 = (vpl[k] - vph[k]) * feat.inv_dx;
                    }
                    __bf16 d[4] = {to_bf16(v0), to_bf16(v1), to_bf16(v2), to_bf16(0.f)};
                    *reinterpret_cast<uint2 *>(in + q * 4) = *reinterpret_cast<const uint2 *>(d);
                }
            }
        }
        __syncthreads();
        // the role's weights (A operands, from L2 after the first tile) and
        // per-chunk LDS offsets; loaded after the features' barrier, so that
        // they take no registers during the feature loads.  The lane index is
        // made opaque here so that the compiler keeps these address
        // computations in the loop instead of holding them in registers
        // across the whole kernel.
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const int lkq = ln >> 4, lhi = lkq >> 1;
        bf16x8 wa[14];
        int off[14];
        float bb[4];
        float b2 = 0.f;
        if (wave < kL1Waves) {
#pragma unroll
            for (int c = 0; c < 14; ++c) {
                wa[c] = c < 4 ? *reinterpret_cast<const bf16x8 *>(wp0 + (c * 64 + ln) * 8)
                              : bf16x8{};
                off[c] = 0;
            }
            // layer 1: the lane's two taps 8c + 2(lane/16) + h of chunk c, 4 input
            // channels each; taps past the 27th have zero weights: any point reads
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int tap = 8 * c + 2 * lkq + h;
                    off[2 * c + h] = tap < kTaps
                                         ? (((tap / 9) * kF0 + (tap / 3) % 3) * kF0 + tap % 3) * 8
                                         : 0;  // bytes
                }
#pragma unroll
            for (int i = 0; i < 4; ++i) bb[i] = params[kB0 + 4 * lkq + i];
        } else {
            const bool l2 = wave < kL1Waves + kL2Waves;
            const __bf16 *wp = l2 ? wp1 : wp2;
            const int pw = l2 ? kF1 : kF2;                       // input plane width
            const int half = (lkq & 1) * (l2 ? kPl1 : kPl2) * 8;  // channel half
#pragma unroll
            for (int c = 0; c < 14; ++c) {
                wa[c] = *reinterpret_cast<const bf16x8 *>(wp + (c * 64 + ln) * 8);
                // tap 2c + (lane/16)/2, in-plane part; the z part picks the slot
                const int tap = min(2 * c + lhi, kTaps - 1);  // tap 27: zero weights
                off[c] = ((((tap / 3) % 3) * pw + tap % 3) * 8 + half) * 2;  // bytes
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) bb[i] = l2 ? params[kB1 + 4 * lkq + i] : 0.f;
            b2 = params[kB2];
        }

        for (int s = 0; s < kFusedSteps; ++s) {
            if (wave < kL1Waves) {
                if (s < kF1) {
                    // layer-1 plane s (z offset s - 2): 144 points, 9 groups
                    const int lz = s;
                    __bf16 *dst = a0 + (s % kRing) * kSlot1 + hi * kPl1 * 8 + 4 * (kq & 1);
                    // three groups at a time, as independent chains: their 24
                    // operand reads, then their 12 products, then the three
                    // epilogues (one group's chain alone is latency-bound)
                    constexpr int NG = 3;
                    static_assert((kPl1 / 16) % NG == 0, "layer-1 groups per pass");
#pragma unroll 1
                    for (int g0 = 0; g0 < kPl1 / 16; g0 += NG) {
                        uint2 v[NG][8];
#pragma unroll
                        for (int u = 0; u < NG; ++u) {
                            const int pt = (g0 + u) * 16 + j;
                            const int lx = pt % kF1, ly = pt / kF1;
                            const unsigned char *src = reinterpret_cast<const unsigned char *>(in) +
                                                       ((lz * kF0 + ly) * kF0 + lx) * 8;
#pragma unroll
                            for (int k = 0; k < 8; ++k)
                                v[u][k] = *reinterpret_cast<const uint2 *>(src + off[k]);
                        }
                        f32x4 acc[NG];
#pragma unroll
                        for (int u = 0; u < NG; ++u) {
                            acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                const bf16x8 b = __builtin_bit_cast(
                                    bf16x8, make_uint4(v[u][2 * c].x, v[u][2 * c].y,
                                                       v[u][2 * c + 1].x, v[u][2 * c + 1].y));
                                acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[c], b, acc[u],
                                                                                 0, 0, 0);
                            }
                        }
                        __builtin_amdgcn_sched_group_barrier(0x100, 8 * NG, 0);  // LDS reads
                        __builtin_amdgcn_sched_group_barrier(0x8, 4 * NG, 0);    // products
#pragma unroll
                        for (int u = 0; u < NG; ++u) {
                            const int pt = (g0 + u) * 16 + j;
                            const int lx = pt % kF1, ly = pt / kF1;
                            const int gx = x0 + lx - 2, gy = y0 + ly - 2, gz = z0 + lz - 2;
                            const bool inside = gx >= 0 && gy >= 0 && gz >= 0 && gx < g.nx &&
                                                gy < g.ny && gz < g.nz;
                            __bf16 ab[4];
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const float av = silu_f(acc[u][i] + bb[i]);  // finite: no branch
                                ab[i] = to_bf16(inside ? av : 0.f);
                            }
                            *reinterpret_cast<uint2 *>(dst + pt * 8) =
                                *reinterpret_cast<uint2 *>(ab);
                        }
                    }
                }
            } else if (wave < kL1Waves + kL2Waves) {
                const int b = s - 3;
                if (b >= 0 && b < kF2) {
                    // layer-2 plane b (z offset b - 1) from layer-1 planes b..b+2:
                    // 100 points, 7 groups (the last one partial), alternating
                    // between the layer's waves
                    // ring slots in bytes
                    const int sb0 = (b % kRing) * kSlot1 * 2, sb1 = ((b + 1) % kRing) * kSlot1 * 2,
                              sb2 = ((b + 2) % kRing) * kSlot1 * 2;
__bf16 *dst = a1 + (b % kRing) * kSlot2 + hi * kPl2 * 8 + 4 * (kq & 1);
#pragma unroll 1
                    for (int grp = wave - kL1Waves; grp < (kPl2 + 15) / 16; grp += kL2Waves) {
                        const int pt = grp * 16 + j;
                        const int ptc = min(pt, kPl2 - 1);  // lanes past the end compute a copy
                        const int lx = ptc % kF2, ly = ptc / kF2;
                        const f32x4 acc = ring_conv16(
                            wa, reinterpret_cast<const unsigned char *>(a0) + (ly * kF1 + lx) * 16,
                            off, hi, sb0, sb1, sb2);
                        const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z0 + b - 1;
                        const bool inside = gx >= 0 && gy >= 0 && gz >= 0 && gx < g.nx &&
                                            gy < g.ny && gz < g.nz;
                        __bf16 ab[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float a = silu_f(acc[i] + bb[i]);  // finite: no branch
                            ab[i] = to_bf16(inside ? a : 0.f);
                        }
                        if (pt < kPl2)
                            *reinterpret_cast<uint2 *>(dst + pt * 8) =
                                *reinterpret_cast<uint2 *>(ab);
                    }
                }
            } else {
                const int lz = s - 6;
                if (lz >= 0 && lz < kT) {
                    // output plane lz from layer-2 planes lz..lz+2: r on 64
                    // points, 4 groups, into rout and into LDS for the pass
                    // below, at the start of the feature array: feature planes
                    // below s are no longer read (layer 1 reads planes s..s+2),
                    // and plane lz's 256 bytes end below (s - 5) * 256 <= s * 1568
                    // ring slots in bytes
                    const int sb0 = (lz % kRing) * kSlot2 * 2,
                              sb1 = ((lz + 1) % kRing) * kSlot2 * 2,
                              sb2 = ((lz + 2) % kRing) * kSlot2 * 2;
#pragma unroll 1
                    for (int grp = 0; grp < 4; ++grp) {
                        const int pt = grp * 16 + j;
                        const int lx = pt & 7, ly = pt >> 3;
                        int q0 = (ly * kF2 + lx) * 16;
                        // opaque: keeps the chunk addresses from being hoisted out
                        // of the loops into registers
                        asm volatile("" : "+v"(q0));
                        const f32x4 acc = ring_conv16(
                            wa, reinterpret_cast<const unsigned char *>(a1) + q0, off, hi, sb0,
                            sb1, sb2);
                        if (kq == 0) {
                            const int64_t gpt = (static_cast<int64_t>(z0 + lz) * g.ny +
                                                 (y0 + ly)) * g.nx + (x0 + lx);
                            const float r = acc[0] + b2;
                            if (rout) rout[gpt] = r;
                            reinterpret_cast<float *>(fsm)[lz * 64 + pt] = r;
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (corr) {
            // the gated, limited correction of the tile and its fallback test,
            // two points per thread: a tile that fails the test falls back to
            // the plain step, its corrections zero.  (They are added to the
            // plain step by a later kernel, since other blocks still read the
            // plain step around their tiles.)
            constexpr int NPT = kT * kT * kT / kFusedBlock;
            float cv[NPT];
            int64_t gp[NPT];
            bool bad = false;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int pt = threadIdx.x + k * kFusedBlock;
                gp[k] = (static_cast<int64_t>(z0 + (pt >> 6)) * g.ny + (y0 + ((pt >> 3) & 7))) *
                            g.nx + (x0 + (pt & 7));
                const float ph = feat.phi[gp[k]];
                const float r = reinterpret_cast<const float *>(fsm)[pt] *
                                cutoff_f(ph, feat.inv_gamma);
                if (!(fabsf(r) <= 0.5f)) bad = true;  // NaN fails too
                // limiter: the correction changes the plain increment by at
                // most half of it, so it never reverses or stalls the plain step
                const float lim = kCorrLimit * fabsf(feat.plain[gp[k]] - ph);
                cv[k] = fminf(fmaxf(dx * r, -lim), lim);
            }
            const bool fail = __syncthreads_or(bad);
#pragma unroll
            for (int k = 0; k < NPT; ++k) corr[gp[k]] = fail ? 0.f : cv[k];
            if (fail && threadIdx.x == 0 && fallbacks) atomicAdd(fallbacks, 1);
        }
        __syncthreads();  // LDS free for the next tile
    }
}

// out += corr on every point of the listed tiles (8^3 tiles).
__global__ __launch_bounds__(kBlock) void apply_corr_kernel(ConvGeo g,
                                                            const int32_t *__restrict__ tiles,
                                                            const int32_t *__restrict__ ntiles_dev,
                                                            int cap, const float *__restrict__ corr,
                                                            float *__restrict__ out) {
    const int n = min(*ntiles_dev, cap);
    for (int p = blockIdx.x; p < n; p += gridDim.x) {
        const int t = tiles[p];
        if (t < 0 || t >= g.ntx * g.nty * g.ntz) continue;
        const int ti = t % g.ntx, rr = t / g.ntx;
        const int x0 = ti * kT, y0 = (rr % g.nty) * kT, z0 = (rr / g.nty) * kT;
        for (int q = threadIdx.x; q < kT * kT * kT; q += kBlock) {
            const int lx = q & 7, ly = (q >> 3) & 7, lz = q >> 6;
            const int64_t gi = (static_cast<int64_t>(z0 + lz) * g.ny + (y0 + ly)) * g.nx + x0 + lx;
            out[gi] += corr[gi];
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradients: per tile, for every tap, GW[o][c] += sum_p G[p][o] X[p+tap][c]
// on the matrix cores (rows o, columns c, reduction over 32 points per
// instruction), written as per-tile partial sums; a second kernel adds the
// partials of all tiles in list order (deterministic).

template <int CIN>
__global__ __launch_bounds__(kBlock) void closure_wgrad_kernel(
    ConvGeo g, const int32_t *__restrict__ tiles, const int32_t *__restrict__ ntiles_dev,
    int ntiles_cap, const uint8_t *__restrict__ umap, const __bf16 *__restrict__ x16, In4 x4,
    const __bf16 *__restrict__ gout16, const float *__restrict__ gout_r, int cout,
    float *__restrict__ partial) {
    // partial layout per tile: [tap][o 16][c 16] followed by bias [16]
    constexpr int PART = kTaps * 256 + 16;
    __shared__ __align__(16) __bf16 xs[CIN][kP * kP * kP];  // channel-major patch
    __shared__ __align__(16) __bf16 gs[16][kT * kT * kT];    // channel-major tile gradient
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = min(*ntiles_dev, ntiles_cap);
    for (int p = blockIdx.x; p < n; p += gridDim.x) {
        const int t = tiles[p];
        float *out = partial + static_cast<int64_t>(p) * PART;
        if (t < 0 || t >= g.ntx * g.nty * g.ntz) {
            for (int i = threadIdx.x; i < PART; i += kBlock) out[i] = 0.f;
            continue;
        }
        const int ti = t % g.ntx, rr = t / g.ntx;
        const int tj = rr % g.nty, tk = rr / g.nty;
        const int x0 = ti * kT, y0 = tj * kT, z0 = tk * kT;
        for (int q = threadIdx.x; q < kP * kP * kP; q += kBlock) {
            const int px = q % kP, py = (q / kP) % kP, pz = q / (kP * kP);
            const int gx = x0 + px - 1, gy = y0 + py - 1, gz = z0 + pz - 1;
            bool ok = gx >= 0 && gy >= 0 && gz >= 0 && gx < g.nx && gy < g.ny && gz < g.nz;
            if (ok) ok = umap[((gz / kT) * g.nty + gy / kT) * g.ntx + gx / kT] != 0;
            const int64_t gi = (static_cast<int64_t>(gz) * g.ny + gy) * g.nx + gx;
            if constexpr (CIN == 16) {
#pragma unroll
                for (int c = 0; c < 16; ++c) xs[c][q] = ok ? x16[gi * 16 + c] : to_bf16(0.f);
            } else {
                float v0 = 0.f, v1 = 0.f, v2 = 0.f;
                if (ok) {
                    const float ph = x4.phi[gi];
                    v0 = fminf(fmaxf(ph * x4.inv_gamma, -2.f), 2.f);
                    v1 = x4.F[gi] * x4.inv_fmax;
                    v2 = (x4.plain[gi] - ph) * x4.inv_dx;
                }
                xs[0][q] = to_bf16(v0);
                xs[1][q] = to_bf16(v1);
                xs[2][q] = to_bf16(v2);
                xs[3][q] = to_bf16(0.f);
            }
        }
        for (int q = threadIdx.x; q < 512; q += kBlock) {
            const int lx = q & 7, ly = (q >> 3) & 7, lz = q >> 6;
            const int64_t gi = (static_cast<int64_t>(z0 + lz) * g.ny + (y0 + ly)) * g.nx + x0 + lx;
            if (gout_r) {
                gs[0][q] = to_bf16(gout_r[gi]);
                for (int o = 1; o < 16; ++o) gs[o][q] = to_bf16(0.f);
            } else {
#pragma unroll
                for (int o = 0; o < 16; ++o) gs[o][q] = gout16[gi * 16 + o];
            }
        }
        __syncthreads();
        // bias gradient: sum over the tile's points
        if (threadIdx.x < 16) {
            float s = 0.f;
            for (int q = 0; q < 512; ++q) s += from_bf16(gs[threadIdx.x][q]);
            out[kTaps * 256 + threadIdx.x] = threadIdx.x < cout ? s : 0.f;
        }
        const int row = lane & 15, kq = lane >> 4;
        for (int tap = wave; tap < kTaps; tap += 4) {
            const int dz = tap / 9, dy = (tap / 3) % 3, dxx = tap % 3;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int kc = 0; kc < 16; ++kc) {  // 16 chunks of 32 points
                bf16x8 a, b;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int q = kc * 32 + 8 * kq + e;  // point of the tile
                    const int lx = q & 7, ly = (q >> 3) & 7, lz = q >> 6;
                    a[e] = gs[row][q];
                    const int xq = ((lz + dz) * kP + (ly + dy)) * kP + (lx + dxx);
                    b[e] = row < CIN ? xs[row < CIN ? row : 0][xq] : to_bf16(0.f);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
            // acc[i] = GW[o = 4*kq + i][c = row]
#pragma unroll
            for (int i = 0; i < 4; ++i) out[tap * 256 + (4 * kq + i) * 16 + row] = acc[i];
        }
        __syncthreads();
    }
}

// grad[flat param of layer] = sum over tiles of the partials, in tile order
__global__ void closure_wgrad_reduce_kernel(const float *__restrict__ partial,
                                            const int32_t *__restrict__ ntiles_dev, int cap,
                                            int woff, int boff, int cin, int cout,
                                            float *__restrict__ grad) {
    constexpr int PART = kTaps * 256 + 16;
    const int n = min(*ntiles_dev, cap);
    const int nw = cout * cin * kTaps;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nw + cout;
         i += gridDim.x * blockDim.x) {
        int src;
        if (i < nw) {
            const int o = i / (cin * kTaps), c = (i / kTaps) % cin, tap = i % kTaps;
            src = tap * 256 + o * 16 + c;
        } else {
            src = kTaps * 256 + (i - nw);
        }
        float s = 0.f;
        for (int p = 0; p < n; ++p) s += partial[static_cast<int64_t>(p) * PART + src];
        grad[i < nw ? woff + i : boff + (i - nw)] = s;
    }
}

// ---------------------------------------------------------------------------
// restriction, loss gradient, Adam

__global__ void restrict4_kernel(const float *__restrict__ fine, int nxf, int nyf, int nzf,
                                 float *__restrict__ coarse) {
    const int nxc = nxf / 4, nyc = nyf / 4, nzc = nzf / 4;
    const int64_t total = static_cast<int64_t>(nxc) * nyc * nzc;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int I = i % nxc, J = (i / nxc) % nyc, K = i / (static_cast<int64_t>(nxc) * nyc);
        float s = 0.f;
        for (int dz = 1; dz <= 2; ++dz)
            for (int dy = 1; dy <= 2; ++dy)
                for (int dxx = 1; dxx <= 2; ++dxx)
                    s += fine[(static_cast<int64_t>(4 * K + dz) * nyf + (4 * J + dy)) * nxf +
                              (4 * I + dxx)];
        coarse[i] = s * 0.125f;
    }
}

// g = 2 (r - r*) / count on the active tiles, r* = (target - phi - delta)/dx;
// partial loss sums per tile (deterministic reduction afterwards).
__global__ __launch_bounds__(kBlock) void closure_loss_kernel(
    ConvGeo g, const int32_t *__restrict__ tiles, const int32_t *__restrict__ ntiles_dev, int cap,
    const float *__restrict__ r, const float *__restrict__ phi, const float *__restrict__ plain,
    const float *__restrict__ target, float inv_dx, float inv_gamma, float *__restrict__ gr,
    float *__restrict__ tile_loss) {
    const int n = min(*ntiles_dev, cap);
    const float inv_cnt = 1.0f / fmaxf(1.0f, static_cast<float>(n) * 512.f);
    __shared__ float red[kBlock];
    for (int p = blockIdx.x; p < n; p += gridDim.x) {
        const int t = tiles[p];
        const int ti = t % g.ntx, rr = t / g.ntx;
        const int x0 = ti * kT, y0 = (rr % g.nty) * kT, z0 = (rr / g.nty) * kT;
        float s = 0.f;
        for (int q = threadIdx.x; q < 512; q += kBlock) {
            const int lx = q & 7, ly = (q >> 3) & 7, lz = q >> 6;
            const int64_t gi = (static_cast<int64_t>(z0 + lz) * g.ny + (y0 + ly)) * g.nx + x0 + lx;
            const float rs = (target[gi] - plain[gi]) * inv_dx;
            const float c = cutoff_f(phi[gi], inv_gamma);
            const float d = c * r[gi] - rs;
            gr[gi] = 2.f * c * d * inv_cnt;
            s += d * d;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) tile_loss[p] = red[0];
        __syncthreads();
    }
}

__global__ void loss_reduce_kernel(const float *__restrict__ tile_loss, const int32_t *ntiles_dev,
                                   int cap, float *__restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int n = min(*ntiles_dev, cap);
        double s = 0.0;
        for (int p = 0; p < n; ++p) s += tile_loss[p];
        *loss = static_cast<float>(s / fmax(1.0, n * 512.0));
    }
}

__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ grad,
                            float *__restrict__ m, float *__restrict__ v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// The plain scheme as judge of the corrected run's interface: every 8^3 tile
// whose zero-crossing state (holding points of both signs, phi < 0 and
// phi >= 0, or not) differs between the corrected field x and the plain
// shadow field p takes p's values; with tau > 0 so does every tile where the
// two fronts lie more than tau dx apart (a point next to either front,
// |x| < dx or |p| < dx, with |x - p| > tau dx; both fields are distance-like
// there); *resets counts those tiles.  One block of 512 threads per tile (a
// point per thread), grid-stride over the tiles.
__global__ __launch_bounds__(512) void closure_judge_kernel(float *__restrict__ x,
                                                            const float *__restrict__ p, int nx,
                                                            int ny, int ntx, int nty, int ntiles,
                                                            float dx, float tau,
                                                            int32_t *resets) {
    const int lx = threadIdx.x & 7, ly = (threadIdx.x >> 3) & 7, lz = threadIdx.x >> 6;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int ti = t % ntx, r = t / ntx;
        const int tj = r % nty, tk = r / nty;
        const int64_t i =
            (static_cast<int64_t>(tk * 8 + lz) * ny + (tj * 8 + ly)) * nx + ti * 8 + lx;
        const float xv = x[i], pv = p[i];
        const int xneg = __syncthreads_or(xv < 0.f), xpos = __syncthreads_or(!(xv < 0.f));
        const int pneg = __syncthreads_or(pv < 0.f), ppos = __syncthreads_or(!(pv < 0.f));
        const bool near = fabsf(xv) < dx || fabsf(pv) < dx;
        const int apart =
            __syncthreads_or(tau > 0.f && near && fabsf(xv - pv) > tau * dx);
        if ((xneg && xpos) != (pneg && ppos) || apart) {  // uniform over the block
            x[i] = pv;
            if (threadIdx.x == 0) atomicAdd(resets, 1);
        }
    }
}

__global__ void zero_f32_kernel(float *p, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0.f;
}

}  // namespace ls

// ---------------------------------------------------------------------------
// host side

namespace ls {

int plan_step_to_f32(const float *phi, float *out, const float *F, const Geom &G, float dx,
                     float dt, uint8_t *ws, hipStream_t stream);                      // ls_step.hip

constexpr int kPart = kTaps * 256 + 16;  // per-tile weight-gradient partial (floats)

// Closure workspace: packed weights, activations (bf16 x16, dense), dense
// FP32 fields, the active-tile list, per-tile partial sums.
struct ClosureWs {
    int64_t wp0, wp1, wp2, bp1, bp2;
    int64_t a0, z0, a1, z1, ga;
    int64_t r, gr, plain;
    int64_t shadow, shadow_scratch;  // the judge's plain run
    int64_t active, counters;  // counters: [0] active count, [1] fallbacks (scratch), [2] resets
    int64_t partial, tile_loss;
    int64_t total;
};

static ClosureWs closure_ws(const Geom &g) {
    auto al = [](int64_t v) { return (v + 255) & ~int64_t(255); };
    const int64_t N = g.npoints, T = g.ntiles;
    ClosureWs w;
    int64_t o = 0;
    w.wp0 = o; o = al(o + 2 * 4 * 64 * 8);
    w.wp1 = o; o = al(o + 2 * 14 * 64 * 8);
    w.wp2 = o; o = al(o + 2 * 14 * 64 * 8);
    w.bp1 = o; o = al(o + 2 * 14 * 64 * 8);
    w.bp2 = o; o = al(o + 2 * 4 * 64 * 8);
    w.a0 = o; o = al(o + 2 * 16 * N);
    w.z0 = o; o = al(o + 2 * 16 * N);
    w.a1 = o; o = al(o + 2 * 16 * N);
    w.z1 = o; o = al(o + 2 * 16 * N);
    w.ga = o; o = al(o + 2 * 16 * N);
    w.r = o; o = al(o + 4 * N);
    w.gr = o; o = al(o + 4 * N);
    w.plain = o; o = al(o + 4 * N);
    w.shadow = o; o = al(o + 4 * N);
    w.shadow_scratch = o; o = al(o + 4 * N);
    w.active = o; o = al(o + 4 * T);
    w.counters = o; o = al(o + 4 * 64);
    w.partial = o; o = al(o + 4 * kPart * T);
    w.tile_loss = o; o = al(o + 4 * T);
    w.total = o;
    return w;
}

static int closure_geom(const ls_grid *grid, Geom *g) {
    int rc = make_geom(grid, g);
    if (rc != LS_OK) return rc;
    if (g->tx != kT || g->ty != kT || g->tz != kT || g->nx % kT || g->ny % kT || g->nz % kT) {
        set_error("closure: needs 8x8x8 tiles and grid dims that are multiples of 8");
        return LS_ERR_UNSUPPORTED;
    }
    if (g->npoints * 32 >= (int64_t(1) << 40)) {
        set_error("closure: grid too large");
        return LS_ERR_UNSUPPORTED;
    }
    return LS_OK;
}

static int check_cws(const Geom &g, void *cws, int64_t bytes, ClosureWs *w) {
    *w = closure_ws(g);
    if (!cws || reinterpret_cast<uintptr_t>(cws) % 256) {
        set_error("closure: closure workspace NULL or not 256-byte aligned");
        return LS_ERR_ARG;
    }
    if (bytes < w->total) {
        set_error("closure: closure workspace too small: %lld bytes given, %lld needed",
                  (long long)bytes, (long long)w->total);
        return LS_ERR_CAPACITY;
    }
    return LS_OK;
}

struct ClosureCall {
    Geom G;
    ClosureWs w;
    uint8_t *cw, *ws;
    hipStream_t s;
    unsigned blocks;
};

// Shared argument checks of the closure entry points.
static int closure_setup(const ls_grid *grid, float dx, float dt, float gamma, float fmax,
                         const float *params, void *ws, int64_t ws_bytes, void *cws,
                         int64_t cws_bytes, void *stream, ClosureCall *c) {
    int rc = closure_geom(grid, &c->G);
    if (rc != LS_OK) return rc;
    if ((rc = check_cws(c->G, cws, cws_bytes, &c->w)) != LS_OK) return rc;
    if ((rc = check_workspace(c->G, ws, ws_bytes)) != LS_OK) return rc;
    if (!params) {
        set_error("closure: params is NULL");
        return LS_ERR_ARG;
    }
    if (!(dx > 0.f) || !(dt >= 0.f) || !(gamma > 0.f) || !(fmax > 0.f) || !(dx < INFINITY) ||
        !(dt < INFINITY) || !(fmax < INFINITY)) {
        set_error("closure: need finite dx > 0, dt >= 0, gamma > 0 and fmax > 0");
        return LS_ERR_ARG;
    }
    DeviceInfo di;
    if ((rc = device_info(&di)) != LS_OK) return rc;
    c->cw = static_cast<uint8_t *>(cws);
    c->ws = static_cast<uint8_t *>(ws);
    c->s = static_cast<hipStream_t>(stream);
    c->blocks = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(c->G.ntiles,
                                                                              int64_t(di.cus) * 4)));
    return LS_OK;
}

template <class T>
static T *at(const ClosureCall &c, int64_t off) {
    return reinterpret_cast<T *>(c.cw + off);
}

static int pack_all(const ClosureCall &c, const float *params) {
    const PackSpec spec[5] = {{kW0, 3, 16, 4, false},  {kW1, 16, 16, 16, false},
                              {kW2, 16, 1, 16, false}, {kW1, 16, 16, 16, true},
                              {kW2, 16, 1, 4, true}};
    const int64_t dst[5] = {c.w.wp0, c.w.wp1, c.w.wp2, c.w.bp1, c.w.bp2};
    for (int i = 0; i < 5; ++i) {
        hipLaunchKernelGGL(pack_weights_kernel, dim3(8), dim3(256), 0, c.s, params,
                           at<__bf16>(c, dst[i]), spec[i]);
        LS_LAUNCH_CHECK("pack_weights_kernel");
    }
    return LS_OK;
}

static int zero_f32(float *p, int64_t n, hipStream_t s) {
    const unsigned b = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(cdiv64(n, 256), 4096)));
    hipLaunchKernelGGL(zero_f32_kernel, dim3(b), dim3(256), 0, s, p, n);
    LS_LAUNCH_CHECK("zero_f32_kernel");
    return LS_OK;
}

static ConvGeo conv_geo(const Geom &g) { return ConvGeo{g.nx, g.ny, g.nz, g.ntx, g.nty, g.ntz}; }

// A (into the closure workspace) and U (into tiles, with its step plan in
// the band workspace) of phi.
static int closure_bands(const ClosureCall &c, const float *phi, const ls_grid *grid, float gamma,
                         int32_t *tiles, int64_t capacity, int32_t *ntiles_dev, int64_t ws_bytes) {
    int rc = band_build<float>(phi, 1.0f, grid, gamma, 0, at<int32_t>(c, c.w.active),
                               c.G.ntiles, at<int32_t>(c, c.w.counters), c.ws, ws_bytes, c.s);
    if (rc != LS_OK) return rc;
    return band_build<float>(phi, 1.0f, grid, gamma, 1, tiles, capacity, ntiles_dev, c.ws,
                             ws_bytes, c.s);
}

// plain = one plain step of phi on the planned band; with `sync`, the points
// outside the band are first copied from phi (a dense copy), else the caller
// guarantees plain equals phi there.
static int closure_plain(const ClosureCall &c, const float *phi, float *plain, const float *F,
                         float dx, float dt, bool sync) {
    if (sync) {
        int rc = ls_copy_f32(plain, phi, c.G.npoints, c.s);
        if (rc != LS_OK) return rc;
    }
    return plan_step_to_f32(phi, plain, F, c.G, dx, dt, c.ws, c.s);
}

// The network on the band (L1, L2) and the active tiles (L3): r into the
// workspace and, with `apply`, the corrected step plain += dx * r on every
// active tile whose r passes the fallback test.
static int closure_network(const ClosureCall &c, const float *phi, const float *F,
                           const float *plain, float dx, float gamma, float fmax,
                           const int32_t *band, const int32_t *nband, const float *params,
                           bool store_z, float *apply, int32_t *fallbacks) {
    const ConvGeo cg = conv_geo(c.G);
    const int cap = static_cast<int>(c.G.ntiles);
    const uint8_t *umap = c.ws + workspace_layout(c.G).u_map;
    const int32_t *active = at<int32_t>(c, c.w.active);
    const int32_t *nactive = at<int32_t>(c, c.w.counters);
    In4 feat{phi, F, plain, nullptr, 1.0f / gamma, 1.0f / fmax, 1.0f / dx};
    In4 none{nullptr, nullptr, nullptr, nullptr, 0.f, 0.f, 0.f};
    hipLaunchKernelGGL((closure_conv_kernel<4, OUT_HIDDEN>), dim3(c.blocks), dim3(kBlock), 0, c.s,
                       cg, band, nband, cap, umap, nullptr, feat, at<const __bf16>(c, c.w.wp0),
                       params + kB0, store_z ? at<__bf16>(c, c.w.z0) : nullptr,
                       at<__bf16>(c, c.w.a0), nullptr, nullptr, nullptr, 0.f, nullptr);
    LS_LAUNCH_CHECK("closure_conv_kernel (layer 1)");
    hipLaunchKernelGGL((closure_conv_kernel<16, OUT_HIDDEN>), dim3(c.blocks), dim3(kBlock), 0,
                       c.s, cg, band, nband, cap, umap, at<const __bf16>(c, c.w.a0), none,
                       at<const __bf16>(c, c.w.wp1), params + kB1,
                       store_z ? at<__bf16>(c, c.w.z1) : nullptr, at<__bf16>(c, c.w.a1), nullptr,
                       nullptr, nullptr, 0.f, nullptr);
    LS_LAUNCH_CHECK("closure_conv_kernel (layer 2)");
    In4 gate{phi, nullptr, nullptr, nullptr, 1.0f / gamma, 0.f, 0.f};
    hipLaunchKernelGGL((closure_conv_kernel<16, OUT_LAST>), dim3(c.blocks), dim3(kBlock), 0, c.s,
                       cg, active, nactive, cap, umap, at<const __bf16>(c, c.w.a1), gate,
                       at<const __bf16>(c, c.w.wp2), params + kB2, nullptr, nullptr, nullptr,
                       at<float>(c, c.w.r), apply, dx, fallbacks);
    LS_LAUNCH_CHECK("closure_conv_kernel (layer 3)");
    return LS_OK;
}

// The fused network on the active tiles: r (raw, into rout if non-NULL) and,
// with `apply`, the corrected step apply += dx * c(phi) * r per tile (with the
// fallback test), each point's correction limited to half of its plain
// increment.
static int closure_fused(const ClosureCall &c, const float *phi, const float *F, const float *plain,
                         float dx, float gamma, float fmax, const float *params, float *rout,
                         float *apply, int32_t *fallbacks) {
    static bool lds_set = false;  // per process: the attribute is per kernel, not per device
    if (!lds_set) {
        LS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(closure_fused_kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(kFusedLds)));
        lds_set = true;
    }
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != LS_OK) return rc;
    const unsigned blocks = static_cast<unsigned>(std::max<int64_t>(
        1, std::min<int64_t>(c.G.ntiles, int64_t(di.cus) * kFusedBlocksPerCu)));
    In4 feat{phi, F, plain, nullptr, 1.0f / gamma, 1.0f / fmax, 1.0f / dx};
    // with `apply` the corrections go to the workspace's r field first
    float *corr = apply ? at<float>(c, c.w.r) : nullptr;
    int64_t slot;
    if ((rc = stats_before(LS_KERNEL_CLOSURE, c.s, &slot)) != LS_OK) return rc;
    hipLaunchKernelGGL(closure_fused_kernel, dim3(blocks), dim3(kFusedBlock), kFusedLds, c.s,
                       conv_geo(c.G), at<const int32_t>(c, c.w.active),
                       at<const int32_t>(c, c.w.counters), static_cast<int>(c.G.ntiles), feat,
                       at<const __bf16>(c, c.w.wp0), at<const __bf16>(c, c.w.wp1),
                       at<const __bf16>(c, c.w.wp2), params, rout, corr, dx, fallbacks);
    LS_LAUNCH_CHECK("closure_fused_kernel");
    if ((rc = stats_after(LS_KERNEL_CLOSURE, c.s, slot)) != LS_OK) return rc;
    if (apply) {
        hipLaunchKernelGGL(apply_corr_kernel, dim3(blocks * 4), dim3(kBlock), 0, c.s,
                           conv_geo(c.G), at<const int32_t>(c, c.w.active),
                           at<const int32_t>(c, c.w.counters), static_cast<int>(c.G.ntiles),
                           static_cast<const float *>(corr), apply);
        LS_LAUNCH_CHECK("apply_corr_kernel");
    }
    return LS_OK;
}

static int wgrad_reduce(const ClosureCall &c, const int32_t *ncount, int woff, int boff, int cin,
                        int cout, float *grad) {
    const int total = cout * cin * kTaps + cout;
    hipLaunchKernelGGL(closure_wgrad_reduce_kernel, dim3(cdiv64(total, 256)), dim3(256), 0, c.s,
                       at<const float>(c, c.w.partial), ncount, static_cast<int>(c.G.ntiles), woff,
                       boff, cin, cout, grad);
    LS_LAUNCH_CHECK("closure_wgrad_reduce_kernel");
    return LS_OK;
}

}  // namespace ls

extern "C" {

int64_t ls_closure_param_count(void) { return ls::kNParams; }

int64_t ls_closure_workspace_bytes(const ls_grid *g) {
    ls::clear_error();
    ls::Geom G;
    int rc = ls::closure_geom(g, &G);
    if (rc != LS_OK) return rc;
    return ls::closure_ws(G).total;
}

int ls_restrict4_f32(const float *fine, const ls_grid *fine_grid, float *coarse, void *stream) {
    ls::clear_error();
    ls::Geom G;
    int rc = ls::make_geom(fine_grid, &G);
    if (rc != LS_OK) return rc;
    if (!fine || !coarse) {
        ls::set_error("restrict4: NULL buffer");
        return LS_ERR_ARG;
    }
    if (G.nx % 4 || G.ny % 4 || G.nz % 4) {
        ls::set_error("restrict4: fine dims must be multiples of 4");
        return LS_ERR_ARG;
    }
    hipLaunchKernelGGL(ls::restrict4_kernel, dim3(2048), dim3(256), 0,
                       static_cast<hipStream_t>(stream), fine, G.nx, G.ny, G.nz, coarse);
    LS_LAUNCH_CHECK("restrict4_kernel");
    return LS_OK;
}

int ls_closure_forward_f32(const float *phi, const float *F, const ls_grid *g, float dx, float dt,
                           float gamma, float fmax, const float *params, float *r, float *plain,
                           int32_t *tiles, int64_t capacity, int32_t *ntiles_dev, void *ws,
                           int64_t ws_bytes, void *cws, int64_t cws_bytes, void *stream) {
    ls::clear_error();
    ls::ClosureCall c;
    int rc = ls::closure_setup(g, dx, dt, gamma, fmax, params, ws, ws_bytes, cws, cws_bytes,
                               stream, &c);
    if (rc != LS_OK) return rc;
    if (!phi || !F || !tiles || !ntiles_dev) {
        ls::set_error("closure forward: NULL argument");
        return LS_ERR_ARG;
    }
    if (capacity < c.G.ntiles) {
        ls::set_error("closure forward: capacity %lld < %lld tiles", (long long)capacity,
                      (long long)c.G.ntiles);
        return LS_ERR_CAPACITY;
    }
    float *pl = ls::at<float>(c, c.w.plain);
    float *rr = ls::at<float>(c, c.w.r);
    if ((rc = ls::closure_bands(c, phi, g, gamma, tiles, capacity, ntiles_dev, ws_bytes)) != LS_OK)
        return rc;
    if ((rc = ls::closure_plain(c, phi, pl, F, dx, dt, true)) != LS_OK) return rc;
    if ((rc = ls::pack_all(c, params)) != LS_OK) return rc;
    if ((rc = ls::zero_f32(rr, c.G.npoints, c.s)) != LS_OK) return rc;
    if ((rc = ls::closure_fused(c, phi, F, pl, dx, gamma, fmax, params, rr, nullptr, nullptr)) !=
        LS_OK)
        return rc;
    if (r && (rc = ls_copy_f32(r, rr, c.G.npoints, c.s)) != LS_OK) return rc;
    if (plain && (rc = ls_copy_f32(plain, pl, c.G.npoints, c.s)) != LS_OK) return rc;
    return LS_OK;
}

int ls_closure_backward_f32(const float *phi, const float *target, const float *F,
                            const ls_grid *g, float dx, float dt, float gamma, float fmax,
                            const float *params, float *grad, float *loss_dev, int32_t *tiles,
                            int64_t capacity, int32_t *ntiles_dev, void *ws, int64_t ws_bytes,
                            void *cws, int64_t cws_bytes, void *stream) {
    ls::clear_error();
    ls::ClosureCall c;
    int rc = ls::closure_setup(g, dx, dt, gamma, fmax, params, ws, ws_bytes, cws, cws_bytes,
                               stream, &c);
    if (rc != LS_OK) return rc;
    if (!phi || !target || !F || !grad || !tiles || !ntiles_dev) {
        ls::set_error("closure backward: NULL argument");
        return LS_ERR_ARG;
    }
    if (capacity < c.G.ntiles) {
        ls::set_error("closure backward: capacity %lld < %lld tiles", (long long)capacity,
                      (long long)c.G.ntiles);
        return LS_ERR_CAPACITY;
    }
    const ls::ConvGeo cg = ls::conv_geo(c.G);
    const int cap = static_cast<int>(c.G.ntiles);
    const uint8_t *umap = c.ws + ls::workspace_layout(c.G).u_map;
    const int32_t *active = ls::at<int32_t>(c, c.w.active);
    const int32_t *nactive = ls::at<int32_t>(c, c.w.counters);
    float *pl = ls::at<float>(c, c.w.plain);
    float *gr = ls::at<float>(c, c.w.gr);
    float *part = ls::at<float>(c, c.w.partial);
    if ((rc = ls::closure_bands(c, phi, g, gamma, tiles, capacity, ntiles_dev, ws_bytes)) != LS_OK)
        return rc;
    if ((rc = ls::closure_plain(c, phi, pl, F, dx, dt, true)) != LS_OK) return rc;
    if ((rc = ls::pack_all(c, params)) != LS_OK) return rc;
    if ((rc = ls::closure_network(c, phi, F, pl, dx, gamma, fmax, tiles, ntiles_dev, params, true,
                                  nullptr, nullptr)) != LS_OK)
        return rc;
    // loss and its gradient w.r.t. r on the active tiles (zero elsewhere)
    if ((rc = ls::zero_f32(gr, c.G.npoints, c.s)) != LS_OK) return rc;
    hipLaunchKernelGGL(ls::closure_loss_kernel, dim3(c.blocks), dim3(ls::kBlock), 0, c.s, cg,
                       active, nactive, cap, ls::at<const float>(c, c.w.r), phi,
                       static_cast<const float *>(pl), target, 1.0f / dx, 1.0f / gamma, gr,
                       ls::at<float>(c, c.w.tile_loss));
    LS_LAUNCH_CHECK("closure_loss_kernel");
    if (loss_dev) {
        hipLaunchKernelGGL(ls::loss_reduce_kernel, dim3(1), dim3(64), 0, c.s,
                           ls::at<const float>(c, c.w.tile_loss), nactive, cap, loss_dev);
        LS_LAUNCH_CHECK("loss_reduce_kernel");
    }
    ls::In4 none{nullptr, nullptr, nullptr, nullptr, 0.f, 0.f, 0.f};
    ls::In4 feat{phi, F, pl, nullptr, 1.0f / gamma, 1.0f / fmax, 1.0f / dx};
    ls::In4 gin{nullptr, nullptr, nullptr, gr, 0.f, 0.f, 0.f};
    // layer 3 weights: sum over active tiles of g(p) a1(p + tap)
    hipLaunchKernelGGL((ls::closure_wgrad_kernel<16>), dim3(c.blocks), dim3(ls::kBlock), 0, c.s, cg,
                       active, nactive, cap, umap, ls::at<const __bf16>(c, c.w.a1), none,
                       nullptr, static_cast<const float *>(gr), 1, part);
    LS_LAUNCH_CHECK("closure_wgrad_kernel (layer 3)");
    if ((rc = ls::wgrad_reduce(c, nactive, ls::kW2, ls::kB2, 16, 1, grad)) != LS_OK) return rc;
    // dL/dz1 = (W3^T g) * SiLU'(z1) on the band
    hipLaunchKernelGGL((ls::closure_conv_kernel<4, ls::OUT_GRAD>), dim3(c.blocks), dim3(ls::kBlock),
                       0, c.s, cg, static_cast<const int32_t *>(tiles),
                       static_cast<const int32_t *>(ntiles_dev), cap, umap, nullptr, gin,
                       ls::at<const __bf16>(c, c.w.bp2), nullptr, nullptr, ls::at<__bf16>(c, c.w.ga),
                       ls::at<const __bf16>(c, c.w.z1), nullptr, nullptr, 0.f, nullptr);
    LS_LAUNCH_CHECK("closure_conv_kernel (grad layer 3)");
    // layer 2 weights
    hipLaunchKernelGGL((ls::closure_wgrad_kernel<16>), dim3(c.blocks), dim3(ls::kBlock), 0, c.s, cg,
                       static_cast<const int32_t *>(tiles), static_cast<const int32_t *>(ntiles_dev),
                       cap, umap, ls::at<const __bf16>(c, c.w.a0), none,
                       ls::at<const __bf16>(c, c.w.ga), nullptr, 16, part);
    LS_LAUNCH_CHECK("closure_wgrad_kernel (layer 2)");
    if ((rc = ls::wgrad_reduce(c, ntiles_dev, ls::kW1, ls::kB1, 16, 16, grad)) != LS_OK) return rc;
    // dL/dz0 = (W2^T dL/dz1) * SiLU'(z0), into the a1 buffer (no longer needed)
    hipLaunchKernelGGL((ls::closure_conv_kernel<16, ls::OUT_GRAD>), dim3(c.blocks),
                       dim3(ls::kBlock), 0, c.s, cg, static_cast<const int32_t *>(tiles),
                       static_cast<const int32_t *>(ntiles_dev), cap, umap,
                       ls::at<const __bf16>(c, c.w.ga), none, ls::at<const __bf16>(c, c.w.bp1),
                       nullptr, nullptr, ls::at<__bf16>(c, c.w.a1), ls::at<const __bf16>(c, c.w.z0),
                       nullptr, nullptr, 0.f, nullptr);
    LS_LAUNCH_CHECK("closure_conv_kernel (grad layer 2)");
    // layer 1 weights
    hipLaunchKernelGGL((ls::closure_wgrad_kernel<4>), dim3(c.blocks), dim3(ls::kBlock), 0, c.s, cg,
                       static_cast<const int32_t *>(tiles), static_cast<const int32_t *>(ntiles_dev),
                       cap, umap, nullptr, feat, ls::at<const __bf16>(c, c.w.a1), nullptr, 16, part);
    LS_LAUNCH_CHECK("closure_wgrad_kernel (layer 1)");
    return ls::wgrad_reduce(c, ntiles_dev, ls::kW0, ls::kB0, 3, 16, grad);
}

int ls_adam_step(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                 float beta1, float beta2, float eps, int t, void *stream) {
    ls::clear_error();
    if (!params || !grad || !m || !v || n <= 0 || n > INT32_MAX || t < 1 || !(lr >= 0.f) ||
        !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
        ls::set_error("adam: bad argument (NULL buffer, n, t < 1, or hyper-parameter range)");
        return LS_ERR_ARG;
    }
    const float c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), t));
    const float c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), t));
    hipLaunchKernelGGL(ls::adam_kernel, dim3(static_cast<unsigned>(ls::cdiv64(n, 256))), dim3(256),
                       0, static_cast<hipStream_t>(stream), params, grad, m, v,
                       static_cast<int>(n), lr, beta1, beta2, eps, c1, c2);
    LS_LAUNCH_CHECK("adam_kernel");
    return LS_OK;
}

int ls_closure_run_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                       float gamma, float fmax, const float *params, int nsteps, int window,
                       int judge, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                       int32_t *fallbacks_dev, int32_t *resets_dev, void *ws, int64_t ws_bytes,
                       void *cws, int64_t cws_bytes, void *stream) {
    ls::clear_error();
    // the host checks first: nothing is launched or queried on an error
    ls::Geom G0;
    int rc = ls::closure_geom(g, &G0);
    if (rc != LS_OK) return rc;
    if (!phi || !F || !tiles || !ntiles_dev || !fallbacks_dev || (judge && !resets_dev)) {
        ls::set_error("closure run: NULL argument");
        return LS_ERR_ARG;
    }
    if (nsteps < 0 || window <= 0) {
        ls::set_error("closure run: need nsteps >= 0 and window > 0");
        return LS_ERR_ARG;
    }
    if (judge < 0 || judge > 3) {
        ls::set_error("closure run: judge must be 0, 1, 2 or 3 (got %d)", judge);
        return LS_ERR_ARG;
    }
    if (capacity < G0.ntiles) {
        ls::set_error("closure run: capacity %lld < %lld tiles", (long long)capacity,
                      (long long)G0.ntiles);
        return LS_ERR_CAPACITY;
    }
    ls::ClosureCall c;
    rc = ls::closure_setup(g, dx, dt, gamma, fmax, params, ws, ws_bytes, cws, cws_bytes, stream,
                           &c);
    if (rc != LS_OK) return rc;
    if ((rc = ls::pack_all(c, params)) != LS_OK) return rc;
    float *shadow = ls::at<float>(c, c.w.shadow);
    float *shadow_scratch = ls::at<float>(c, c.w.shadow_scratch);
    if (judge && (rc = ls_copy_f32(shadow, phi, c.G.npoints, c.s)) != LS_OK) return rc;
    // ping-pong between phi and a closure buffer; within a window the points
    // outside the band are equal in both (one dense copy per window)
    float *buf[2] = {phi, ls::at<float>(c, c.w.plain)};
    int cur = 0;
    for (int s0 = 0; s0 < nsteps; s0 += window) {
        const int k = std::min(window, nsteps - s0);
        if (judge) {
            // the shadow window first: its band build uses tiles and ws, which
            // the corrected window then rebuilds from its own field
            if ((rc = ls_band_run_f32(shadow, F, g, dx, dt, gamma, k, k, tiles, capacity,
                                      ntiles_dev, nullptr, shadow_scratch, ws, ws_bytes, c.s)) !=
                LS_OK)
                return rc;
        }
        for (int s = 0; s < k; ++s) {
            const bool first = s == 0;
            if (first && (rc = ls::closure_bands(c, buf[cur], g, gamma, tiles, capacity,
                                                 ntiles_dev, ws_bytes)) != LS_OK)
                return rc;
            float *x = buf[cur], *y = buf[cur ^ 1];
            if ((rc = ls::closure_plain(c, x, y, F, dx, dt, first)) != LS_OK) return rc;
            if ((rc = ls::closure_fused(c, x, F, y, dx, gamma, fmax, params, nullptr, y,
                                        fallbacks_dev)) != LS_OK)
                return rc;
            cur ^= 1;
        }
        if (judge) {
            const unsigned jb = static_cast<unsigned>(std::min<int64_t>(c.G.ntiles, 4096));
            // judge 2 (3): the fronts within one (half a) grid spacing of each
            // other as well
            const float tau = judge == 2 ? 1.0f : (judge == 3 ? 0.5f : 0.0f);
            hipLaunchKernelGGL(ls::closure_judge_kernel, dim3(jb), dim3(512), 0, c.s, buf[cur],
                               static_cast<const float *>(shadow), c.G.nx, c.G.ny, c.G.ntx,
                               c.G.nty, static_cast<int>(c.G.ntiles), dx, tau, resets_dev);
            LS_LAUNCH_CHECK("closure_judge_kernel");
        }
    }
    if (cur == 1 && (rc = ls_copy_f32(phi, buf[1], c.G.npoints, c.s)) != LS_OK) return rc;
    return LS_OK;
}

}  // extern "C"
