// Kernel timing with HIP events (measurement support).
#include <algorithm>
#include <mutex>
#include <vector>

#include "ls_stats.h"

namespace ls {

namespace {
constexpr int kKinds = 5;
constexpr int64_t kMaxPairs = 65536;

struct Record {
    std::vector<hipEvent_t> start, stop;
    std::vector<int64_t> count;  // launches between the events of a pair
    int64_t launches = 0;
    int64_t used = 0;
};

std::mutex g_mu;
bool g_on = false;
Record g_rec[kKinds];
}  // namespace

bool stats_on() { return g_on; }

int stats_before(int kind, hipStream_t stream, int64_t *slot, int64_t count) {
    *slot = -1;
    if (!g_on) return LS_OK;
    std::lock_guard<std::mutex> lock(g_mu);
    Record &r = g_rec[kind];
    r.launches += count;
    if (r.used >= kMaxPairs) return LS_OK;
    if (r.used == static_cast<int64_t>(r.start.size())) {
        hipEvent_t a, b;
        LS_HIP_CHECK(hipEventCreate(&a));
        LS_HIP_CHECK(hipEventCreate(&b));
        r.start.push_back(a);
        r.stop.push_back(b);
        r.count.push_back(0);
    }
    r.count[r.used] = count;
    *slot = r.used++;
    LS_HIP_CHECK(hipEventRecord(r.start[*slot], stream));
    return LS_OK;
}

int stats_after(int kind, hipStream_t stream, int64_t slot) {
    if (slot < 0) return LS_OK;
    std::lock_guard<std::mutex> lock(g_mu);
    LS_HIP_CHECK(hipEventRecord(g_rec[kind].stop[slot], stream));
    return LS_OK;
}

__global__ __launch_bounds__(kBlock) void copy_f32_kernel(float *__restrict__ dst,
                                                          const float *__restrict__ src,
                                                          int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        dst[i] = src[i];
}

}  // namespace ls

extern "C" {

int ls_graph_begin(void *stream) {
    ls::clear_error();
    if (!stream) {
        ls::set_error("graph: capture needs a non-NULL stream");
        return LS_ERR_ARG;
    }
    LS_HIP_CHECK(hipStreamBeginCapture(static_cast<hipStream_t>(stream),
                                       hipStreamCaptureModeThreadLocal));
    return LS_OK;
}

int ls_graph_end(void *stream, void **graph) {
    ls::clear_error();
    if (!stream || !graph) {
        ls::set_error("graph: NULL stream or output");
        return LS_ERR_ARG;
    }
    hipGraph_t g = nullptr;
    LS_HIP_CHECK(hipStreamEndCapture(static_cast<hipStream_t>(stream), &g));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        ls::set_error("graph: instantiate failed: %s", hipGetErrorString(e));
        return LS_ERR_HIP;
    }
    *graph = exec;
    return LS_OK;
}

int ls_graph_launch(void *graph, void *stream) {
    ls::clear_error();
    if (!graph) {
        ls::set_error("graph: NULL graph");
        return LS_ERR_ARG;
    }
    LS_HIP_CHECK(hipGraphLaunch(static_cast<hipGraphExec_t>(graph), static_cast<hipStream_t>(stream)));
    return LS_OK;
}

int ls_graph_destroy(void *graph) {
    ls::clear_error();
    if (!graph) return LS_OK;
    LS_HIP_CHECK(hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph)));
    return LS_OK;
}

int ls_copy_f32(float *dst, const float *src, int64_t n, void *stream) {
    ls::clear_error();
    if (!dst || !src || n < 0) {
        ls::set_error("copy: NULL pointer or negative size");
        return LS_ERR_ARG;
    }
    if (n == 0) return LS_OK;
    ls::DeviceInfo di;
    int rc = ls::device_info(&di);
    if (rc != LS_OK) return rc;
    const int64_t blocks = std::min<int64_t>(ls::cdiv64(n, ls::kBlock), int64_t(di.cus) * 16);
    hipLaunchKernelGGL(ls::copy_f32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(ls::kBlock),
                       0, static_cast<hipStream_t>(stream), dst, src, n);
    LS_LAUNCH_CHECK("copy_f32_kernel");
    return LS_OK;
}

int ls_stats_enable(int on) {
    ls::clear_error();
    std::lock_guard<std::mutex> lock(ls::g_mu);
    ls::g_on = on != 0;
    if (ls::g_on)
        for (auto &r : ls::g_rec) r.launches = 0, r.used = 0;
    return LS_OK;
}

int ls_stats_read(int which, int64_t *launches, int64_t *timed, double *total_ms) {
    ls::clear_error();
    if (which < 0 || which >= ls::kKinds || !launches || !timed || !total_ms) {
        ls::set_error("stats read: bad kernel id or NULL output");
        return LS_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(ls::g_mu);
    const ls::Record &r = ls::g_rec[which];
    double sum = 0.0;
    int64_t covered = 0;
    for (int64_t i = 0; i < r.used; ++i) {
        LS_HIP_CHECK(hipEventSynchronize(r.stop[i]));
        float ms = 0.f;
        LS_HIP_CHECK(hipEventElapsedTime(&ms, r.start[i], r.stop[i]));
        sum += ms;
        covered += r.count[i];
    }
    *launches = r.launches;
    *timed = covered;
    *total_ms = sum;
    return LS_OK;
}

}  // extern "C"
