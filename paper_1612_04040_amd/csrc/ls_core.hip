// Host-side core of libls: error state, argument checks, workspace layout.
#include <climits>
#include <cstring>
#include <mutex>
#include <vector>

#include "ls_internal.h"

namespace ls {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

int make_geom(const ls_grid *g, Geom *out) {
    if (!g) {
        set_error("grid is NULL");
        return LS_ERR_ARG;
    }
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) {
        set_error("grid dims must be positive (got %d x %d x %d)", g->nx, g->ny, g->nz);
        return LS_ERR_ARG;
    }
    if (g->tx <= 0 || g->ty <= 0 || g->tz <= 0) {
        set_error("tile dims must be positive (got %d x %d x %d)", g->tx, g->ty, g->tz);
        return LS_ERR_ARG;
    }
    Geom r;
    r.elem_bytes = 4;
    r.nx = g->nx, r.ny = g->ny, r.nz = g->nz;
    r.tx = g->tx, r.ty = g->ty, r.tz = g->tz;
    r.ntx = static_cast<int32_t>(cdiv64(g->nx, g->tx));
    r.nty = static_cast<int32_t>(cdiv64(g->ny, g->ty));
    r.ntz = static_cast<int32_t>(cdiv64(g->nz, g->tz));
    r.ntiles = static_cast<int64_t>(r.ntx) * r.nty * r.ntz;
    r.npoints = static_cast<int64_t>(g->nx) * g->ny * g->nz;
    if (r.ntiles > INT32_MAX - kCompactChunk) {
        set_error("too many tiles (%lld) for int32 tile ids", (long long)r.ntiles);
        return LS_ERR_UNSUPPORTED;
    }
    *out = r;
    return LS_OK;
}

static int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

Workspace workspace_layout(const Geom &g) {
    Workspace w;
    w.nblk = cdiv64(g.ntiles, kCompactChunk);
    int64_t off = 0;
    w.a_flags = off;
    off = align256(off + g.ntiles);
    w.u_map = off;
    off = align256(off + g.ntiles);
    w.blk_counts = off;
    off = align256(off + 4 * (w.nblk + 1));
    w.blk_counts2 = off;
    off = align256(off + 4 * (w.nblk + 1));
    w.items = off;
    off = align256(off + 4 * kItemWords * g.ntiles);
    w.prev_list = off;
    off = align256(off + 4 * g.ntiles);
    w.counters = off;
    off = align256(off + 4 * 64);
    w.total = off;
    return w;
}

int check_workspace(const Geom &g, const void *ws, int64_t ws_bytes) {
    const Workspace w = workspace_layout(g);
    if (!ws) {
        set_error("workspace is NULL");
        return LS_ERR_ARG;
    }
    if (ws_bytes < w.total) {
        set_error("workspace too small: %lld bytes given, %lld needed", (long long)ws_bytes,
                  (long long)w.total);
        return LS_ERR_CAPACITY;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return LS_ERR_ARG;
    }
    return LS_OK;
}

int device_info(DeviceInfo *out) {
    static std::mutex mu;
    static std::vector<int> cus;
    int dev = 0;
    LS_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if (static_cast<int>(cus.size()) <= dev) cus.resize(dev + 1, 0);
    if (cus[dev] == 0) {
        int n = 0;
        LS_HIP_CHECK(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
        cus[dev] = n > 0 ? n : 1;
    }
    out->cus = cus[dev];
    return LS_OK;
}

}  // namespace ls

extern "C" {

const char *ls_last_error(void) { return ls::g_err; }

const char *ls_version(void) { return "libls 0.1 (gfx950)"; }

int64_t ls_grid_tiles(const ls_grid *g) {
    ls::Geom geom;
    int rc = ls::make_geom(g, &geom);
    if (rc != LS_OK) return rc;
    return geom.ntiles;
}

int64_t ls_workspace_bytes(const ls_grid *g) {
    ls::Geom geom;
    int rc = ls::make_geom(g, &geom);
    if (rc != LS_OK) return rc;
    return ls::workspace_layout(geom).total;
}

}  // extern "C"
