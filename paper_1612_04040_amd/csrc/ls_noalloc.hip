// Band build with no allocation and no workspace argument: the workspace of
// the band build (tile flags, update map, compaction counts, step-plan
// records) lives in a fixed device array of this library.
#include <mutex>
#include <vector>

#include "ls_internal.h"

namespace ls {

// Largest workspace the array holds (16 MiB: grids of up to ~440 000 tiles,
// e.g. 512^3 points in 8^3 tiles, whose workspace is 9.96 MB).
constexpr int64_t kNoAllocBytes = int64_t(16) << 20;

// Each device that loads the library holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel or a copy: in
// host code it is a stand-in, not a device address; the address comes from
// hipGetSymbolAddress, once per device (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on the current device, looked up on the first
// call on that device (with it current) and kept per device.
static int scratch_ptr(void **out) {
    static std::mutex mu;
    static std::vector<void *> ptrs;
    int dev = 0;
    LS_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if (static_cast<int>(ptrs.size()) <= dev) ptrs.resize(dev + 1, nullptr);
    if (!ptrs[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("band build (no allocation): hipGetSymbolAddress of the scratch array "
                      "failed on device %d: %s", dev, hipGetErrorString(e));
            return LS_ERR_HIP;
        }
        ptrs[dev] = p;
    }
    *out = ptrs[dev];
    return LS_OK;
}

}  // namespace ls

extern "C" {

int64_t ls_band_build_noalloc_max_bytes(void) { return ls::kNoAllocBytes; }

int ls_band_build_f32_noalloc(const float *phi, const ls_grid *g, float gamma, int dilate,
                              int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                              void *stream) {
    ls::clear_error();
    ls::Geom geom;
    int rc = ls::make_geom(g, &geom);
    if (rc != LS_OK) return rc;
    geom.elem_bytes = 4;
    // the argument checks of ls_band_build_f32 that need no workspace, made
    // here so that a bad call touches no device
    if (!phi || !tiles || !ntiles_dev) {
        ls::set_error("band build (no allocation): phi, tiles and ntiles_dev must be non-NULL");
        return LS_ERR_ARG;
    }
    if (dilate != 0 && dilate != 1) {
        ls::set_error("band build (no allocation): dilate must be 0 or 1 (got %d)", dilate);
        return LS_ERR_ARG;
    }
    if (!(gamma == gamma)) {
        ls::set_error("band build (no allocation): gamma is NaN");
        return LS_ERR_ARG;
    }
    if (capacity < geom.ntiles) {
        ls::set_error("band build (no allocation): capacity %lld < %lld tiles",
                      (long long)capacity, (long long)geom.ntiles);
        return LS_ERR_CAPACITY;
    }
    const int64_t need = ls::workspace_layout(geom).total;
    if (need > ls::kNoAllocBytes) {
        ls::set_error("band build (no allocation): grid of %lld tiles needs a %lld-byte "
                      "workspace, above the fixed %lld bytes; use ls_band_build_f32",
                      (long long)geom.ntiles, (long long)need, (long long)ls::kNoAllocBytes);
        return LS_ERR_CAPACITY;
    }
    void *ws = nullptr;
    if ((rc = ls::scratch_ptr(&ws)) != LS_OK) return rc;
    // every byte the build reads is written by it first (the full scan sets
    // every tile flag, the compaction its counts): nothing to clear
    return ls::band_build<float>(phi, 1.0f, g, gamma, dilate, tiles, capacity, ntiles_dev, ws,
                                 need, stream);
}

}  // extern "C"
