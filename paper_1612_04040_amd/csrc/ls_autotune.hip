// Tile-shape autotuner of the band update (launch tuning, not part of the
// method).  For every size bucket of 32 points it times the batched
// narrow-band driver (band build or rescan, then the steps) on a batch of
// copies of a synthetic ellipsoid of that size, enough copies for about
// kTunePoints grid points, so the measurement sees the work of a full batch
// rather than launch latency; each candidate tile shape is timed and the one
// with the shortest time per window kept (rows pitched to 128 bytes, as a
// batch lays them out): the time to advance the same fronts, which is what differs between shapes (a bigger tile updates more
// points of the same band).
//
// Results are cached in a text file, one line per (device, bucket):
//   <architecture> <compute units>cu|<bucket> <tx> <ty> <tz> <ms per window>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "ls_internal.h"

namespace ls {

constexpr int kTuneBucket = 32;
constexpr int kTuneShapes[][3] = {{8, 8, 8}, {16, 4, 4}, {32, 4, 4}, {16, 8, 8}, {4, 4, 4}};
constexpr int64_t kTunePoints = int64_t(1) << 25;
constexpr float kTuneNoise = 1.03f;  // times within 3 % of the fastest count as ties
constexpr int kTuneMaxCopies = 512;
constexpr int64_t kTuneAlign = 64;     // copy offsets in elements (256 bytes)
constexpr int kTuneRowAlign = 32;      // row pitch granule in elements (128 bytes)

// copies x (phi, F) of one n^3 grid, copy c at element c * stride, x rows px
// elements apart:
// phi = (|A^-1 (x - c)| - 1) * min(a) for the axis-aligned ellipsoid with
// semi-axes a about c (sign-correct, |grad phi| in [a_min/a_max, 1] on the
// surface); F = speed.
__global__ void tune_field_kernel(float *__restrict__ phi, float *__restrict__ F, int n, int px,
                                  int copies, int64_t stride, float dx, float cx, float cy,
                                  float cz, float ax, float ay, float az, float speed) {
    const int64_t span = static_cast<int64_t>(px) * n * n;
    const int64_t total = stride * copies;
    const float amin = fminf(ax, fminf(ay, az));
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t l = i % stride;
        if (l >= span) continue;
        const int x = static_cast<int>(l % px), y = static_cast<int>((l / px) % n);
        const int z = static_cast<int>(l / (static_cast<int64_t>(px) * n));
        if (x >= n) continue;
        const float u = ((x + 0.5f) * dx - cx) / ax, v = ((y + 0.5f) * dx - cy) / ay,
                    w = ((z + 0.5f) * dx - cz) / az;
        phi[i] = (sqrtf(u * u + v * v + w * w) - 1.0f) * amin;
        F[i] = speed;
    }
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, std::max<size_t>(bytes, 256)); }
};

struct StreamGuard {
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    ~StreamGuard() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (s) (void)hipStreamDestroy(s);
    }
};

// ms per window of the batched band driver on copies of an n^3 ellipsoid
// with tile shape t.
static int time_shape(int n, const int t[3], float *ms) {
    const float dx = 1.0f / n;
    const float speed = 0.6f;
    const float dt = static_cast<float>(0.5 * static_cast<double>(dx) / speed);
    const float gamma = static_cast<float>(6.0 * static_cast<double>(dx));
    const int64_t pts = static_cast<int64_t>(n) * n * n;
    const int px = static_cast<int>(cdiv64(n, kTuneRowAlign) * kTuneRowAlign);
    const int64_t stride = cdiv64(static_cast<int64_t>(px) * n * n, kTuneAlign) * kTuneAlign;
    const int copies =
        static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(kTuneMaxCopies, kTunePoints / pts)));
    std::vector<ls_instance> inst(copies);
    for (int c = 0; c < copies; ++c)
        inst[c] = ls_instance{ls_grid{n, n, n, t[0], t[1], t[2]}, c * stride, dx, dt, gamma, px};
    const int64_t wsb = ls_batch_workspace_bytes(inst.data(), copies);
    if (wsb < 0) return static_cast<int>(wsb);
    const int64_t total = stride * copies;
    DevBuf phi, F, scratch, ws;
    LS_HIP_CHECK(phi.alloc(4 * total));
    LS_HIP_CHECK(F.alloc(4 * total));
    LS_HIP_CHECK(scratch.alloc(4 * total));
    LS_HIP_CHECK(ws.alloc(wsb));
    StreamGuard sg;
    LS_HIP_CHECK(hipStreamCreate(&sg.s));
    LS_HIP_CHECK(hipEventCreate(&sg.a));
    LS_HIP_CHECK(hipEventCreate(&sg.b));
    int rc = ls_batch_setup(inst.data(), copies, ws.p, wsb, sg.s);
    if (rc != LS_OK) return rc;
    float *p = static_cast<float *>(phi.p), *f = static_cast<float *>(F.p);
    auto reset = [&]() -> int {
        hipLaunchKernelGGL(tune_field_kernel, dim3(2048), dim3(256), 0, sg.s, p, f, n, px, copies,
                           stride, dx, 0.5f, 0.47f, 0.53f, 0.27f, 0.19f, 0.23f, speed);
        LS_LAUNCH_CHECK("tune_field_kernel");
        return LS_OK;
    };
    constexpr int kWindow = 10, kWindows = 2, kRepeats = 3;
    auto run = [&](int nsteps) {
        return ls_batch_run_f32(inst.data(), copies, p, f, static_cast<float *>(scratch.p), nsteps,
                                kWindow, nullptr, nullptr, ws.p, wsb, sg.s);
    };
    if ((rc = reset()) != LS_OK) return rc;
    if ((rc = run(kWindow)) != LS_OK) return rc;
    // best of kRepeats timed runs: the minimum is the least disturbed by clock
    // ramps and other work on the device
    float best = INFINITY;
    for (int rep = 0; rep < kRepeats; ++rep) {
        if ((rc = reset()) != LS_OK) return rc;
        LS_HIP_CHECK(hipEventRecord(sg.a, sg.s));
        if ((rc = run(kWindows * kWindow)) != LS_OK) return rc;
        LS_HIP_CHECK(hipEventRecord(sg.b, sg.s));
        LS_HIP_CHECK(hipEventSynchronize(sg.b));
        float el = 0.f;
        LS_HIP_CHECK(hipEventElapsedTime(&el, sg.a, sg.b));
        best = std::min(best, el);
    }
    *ms = best / kWindows;
    return LS_OK;
}

struct TuneEntry {
    int t[3];
    float ms;
};

static void read_cache(const char *path, std::map<std::string, TuneEntry> *out) {
    if (!path) return;
    FILE *fh = std::fopen(path, "r");
    if (!fh) return;
    char line[512];
    while (std::fgets(line, sizeof line, fh)) {
        char *bar = std::strrchr(line, '|');
        if (!bar) continue;
        int bucket, tx, ty, tz;
        float ms;
        if (std::sscanf(bar + 1, "%d %d %d %d %f", &bucket, &tx, &ty, &tz, &ms) != 5) continue;
        std::string key(line, bar - line);
        key += "|" + std::to_string(bucket);
        (*out)[key] = TuneEntry{{tx, ty, tz}, ms};
    }
    std::fclose(fh);
}

static void write_cache(const char *path, const std::map<std::string, TuneEntry> &m) {
    if (!path) return;
    FILE *fh = std::fopen(path, "w");
    if (!fh) return;  // the cache is an optimisation: an unwritable path is not an error
    for (const auto &kv : m) {
        const size_t bar = kv.first.rfind('|');
        std::fprintf(fh, "%s|%s %d %d %d %.4f\n", kv.first.substr(0, bar).c_str(),
                     kv.first.substr(bar + 1).c_str(), kv.second.t[0], kv.second.t[1],
                     kv.second.t[2], kv.second.ms);
    }
    std::fclose(fh);
}

}  // namespace ls

extern "C" {

int ls_autotune(const int32_t *sizes, int n, int precision, const char *cache_path, ls_grid *out,
                int force) {
    ls::clear_error();
    if (!sizes || !out || n <= 0) {
        ls::set_error("autotune: need non-NULL sizes and out, n > 0");
        return LS_ERR_ARG;
    }
    if (precision != 0) {
        ls::set_error("autotune: only FP32 (precision 0) is tuned");
        return LS_ERR_UNSUPPORTED;
    }
    for (int i = 0; i < n; ++i)
        if (sizes[i] < 1 || sizes[i] > 2048) {
            ls::set_error("autotune: size %d of entry %d outside 1..2048", sizes[i], i);
            return LS_ERR_ARG;
        }
    int dev = 0;
    LS_HIP_CHECK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    LS_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    // the key names the architecture and the compute-unit count (the
    // marketing name can be empty, e.g. under a profiler)
    std::string dname = std::string(prop.gcnArchName) + " " +
                        std::to_string(prop.multiProcessorCount) + "cu";
    for (char &ch : dname)
        if (ch == '|' || ch == '\n') ch = ' ';
    std::map<std::string, ls::TuneEntry> cache;
    if (!force) ls::read_cache(cache_path, &cache);
    bool changed = false;
    for (int i = 0; i < n; ++i) {
        const int bucket = sizes[i] / ls::kTuneBucket;
        const std::string key = dname + "|" + std::to_string(bucket);
        auto it = cache.find(key);
        if (it == cache.end()) {
            const int rep = bucket * ls::kTuneBucket + ls::kTuneBucket / 2;
            constexpr int kShapes = sizeof(ls::kTuneShapes) / sizeof(ls::kTuneShapes[0]);
            float ms[kShapes];
            float fastest = INFINITY;
            for (int k = 0; k < kShapes; ++k) {
                const int rc = ls::time_shape(rep, ls::kTuneShapes[k], &ms[k]);
                if (rc != LS_OK) return rc;
                fastest = std::min(fastest, ms[k]);
            }
            // among the shapes within the timing noise of the fastest, the one
            // that reads the fewest halo points per updated point (the bytes
            // beyond the algorithmic ones)
            ls::TuneEntry best{{8, 8, 8}, INFINITY};
            double best_halo = INFINITY;
            for (int k = 0; k < kShapes; ++k) {
                const int *t = ls::kTuneShapes[k];
                if (!(ms[k] <= ls::kTuneNoise * fastest)) continue;
                const double v = double(t[0]) * t[1] * t[2];
                const double halo = (double(t[0] + 2) * (t[1] + 2) * (t[2] + 2) - v) / v;
                if (halo < best_halo) {
                    best_halo = halo;
                    best = ls::TuneEntry{{t[0], t[1], t[2]}, ms[k]};
                }
            }
            it = cache.emplace(key, best).first;
            changed = true;
        }
        out[i] = ls_grid{sizes[i], sizes[i], sizes[i], it->second.t[0], it->second.t[1],
                         it->second.t[2]};
    }
    if (changed || force) ls::write_cache(cache_path, cache);
    return LS_OK;
}

}  // extern "C"
