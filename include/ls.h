/*
 * ls.h -- C-ABI of the narrow-band level-set library (libls.so) for AMD
 * MI355X (gfx950).
 *
 * What it computes: the first-order upwind update of the level-set equation
 * phi_t + F |grad phi| = 0 (Wang, arXiv 1612.04040, Sec. 1, Eq. 2-5),
 *
 *   phi^{n+1} = phi^n - dt [ max(F,0) nabla^+ + min(F,0) nabla^- ]      (Eq. 3)
 *   nabla^+ = sqrt( sum_d max(D^{-d},0)^2 + min(D^{+d},0)^2 )           (Eq. 4)
 *   nabla^- = sqrt( sum_d max(D^{+d},0)^2 + min(D^{-d},0)^2 )           (Eq. 5)
 *
 * with one-sided differences D^{-x} = (phi_i - phi_{i-1})/dx and
 * D^{+x} = (phi_{i+1} - phi_i)/dx (likewise in y, z), restricted to a narrow
 * band of tiles around the zero level set (Sec. 1.1: the tube T of Eq. 6,
 * grown as the region N of Eq. 11 so the front can move into it).
 *
 * Conventions shared by every call:
 *  - Grid: nx*ny*nz points, x fastest: idx = (k*ny + j)*nx + i (the index
 *    formula of Sec. 3).  Cell-centred spacing dx in all three axes.
 *  - Boundary: zero-gradient (Neumann) by index clamping: the difference
 *    across a domain face is 0.
 *  - Tiles: tx*ty*tz points, ceil(n/t) tiles per axis, the last tile of an
 *    axis partial when t does not divide n.  Tile id
 *    t = (tk*nty + tj)*ntx + ti, int32.
 *  - Band list: ascending tile ids, no duplicates, in device memory, with its
 *    length in a device int32 (so build -> step needs no host round trip and
 *    can be captured in a HIP graph).
 *  - Memory: every pointer argument is device memory owned by the caller
 *    (the library allocates nothing and frees nothing).  `stream` is a
 *    hipStream_t (NULL = the default stream); every call is asynchronous and
 *    stream-ordered.
 *  - Errors: arguments are checked on the host before anything is launched;
 *    a failed check returns a negative status, launches nothing and sets a
 *    thread-local message readable with ls_last_error().  A HIP launch error
 *    returns LS_ERR_HIP.  No C++ exception crosses this interface.
 *  - Not checked: the contents of device buffers (non-finite phi or F are the
 *    caller's: NaN is never in the band since |NaN| < gamma is false), the
 *    CFL condition (dt * max|F| * sqrt(3) / dx <= 1 keeps the scheme
 *    monotone), and buffer sizes beyond what the arguments state.
 */
#ifndef LS_H
#define LS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ls_grid {
    int32_t nx, ny, nz; /* points per axis, x fastest */
    int32_t tx, ty, tz; /* band tile shape (8,8,8 by default) */
} ls_grid;

enum {
    LS_OK = 0,
    LS_ERR_ARG = -1,         /* null pointer, bad size, bad scalar */
    LS_ERR_CAPACITY = -2,    /* a caller buffer is smaller than required */
    LS_ERR_HIP = -3,         /* HIP runtime or launch error */
    LS_ERR_UNSUPPORTED = -4  /* shape outside what the kernels support */
};

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *ls_last_error(void);

/* Library version string. */
const char *ls_version(void);

/* Number of tiles of the grid = the capacity a band list needs (or < 0). */
int64_t ls_grid_tiles(const ls_grid *g);

/* Bytes of the `workspace` argument the calls below need for grid g (or < 0).
 * The workspace is caller-owned device memory, needs no initialisation, and
 * holds nothing of value between calls. */
int64_t ls_workspace_bytes(const ls_grid *g);

/* ---------------------------------------------------------------------------
 * Band build (Sec. 1.1, Eq. 6; Eq. 11 in tile form).
 *
 * A = tiles holding at least one grid point with |phi| < gamma (strict; the
 * comparison is made in FP32 for the f32 and f16s calls, FP64 for f64).
 * With dilate = 1 the list is U = A grown by one tile in all 26 directions,
 * clipped to the grid (the update set of the band step); with dilate = 0 it
 * is A.  Writes the ascending ids to tiles[0 .. *ntiles_dev) and their number
 * to *ntiles_dev (device int32).  capacity (entries of `tiles`) must be at
 * least ls_grid_tiles(g).  Runs in O(nx*ny*nz): a full scan of phi.
 *
 * f16s: phi is stored as scaled FP16, h = fp16(phi / scale); the value
 * compared is fl32(h * scale).
 * ------------------------------------------------------------------------- */
int ls_band_build_f32(const float *phi, const ls_grid *g, float gamma, int dilate,
                      int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                      void *workspace, int64_t workspace_bytes, void *stream);
int ls_band_build_f64(const double *phi, const ls_grid *g, double gamma, int dilate,
                      int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                      void *workspace, int64_t workspace_bytes, void *stream);
int ls_band_build_f16s(const uint16_t *phi_h, float scale, const ls_grid *g, float gamma,
                       int dilate, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                       void *workspace, int64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Band step (Sec. 1, Eq. 3-5): nsteps Jacobi steps on every grid point of the
 * tiles listed in tiles[0 .. *ntiles_dev) (ascending, as the band build
 * writes them); every other point keeps its value bit for bit, and a point
 * with F == 0 (either sign) keeps its bits too.  On return (in stream order)
 * phi holds step n + nsteps.
 *
 * scratch: caller-owned buffer of nx*ny*nz elements of phi's type, the
 * ping-pong partner of phi; needs no initialisation, undefined on return.
 * dx > 0, dt >= 0, nsteps >= 0.  The listed ids must be ascending and below
 * ls_grid_tiles(g) (not checked: they are on the device).
 *
 * f32: FP32 storage and arithmetic.  f64: FP64 throughout.
 * f16s: phi stored as scaled FP16 h = fp16(phi / scale) (round to nearest
 * even); arithmetic, F and the upwind selection by sign(F) in FP32.
 * ------------------------------------------------------------------------- */
int ls_upwind_step_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                       const int32_t *tiles, const int32_t *ntiles_dev, int nsteps,
                       float *scratch, void *workspace, int64_t workspace_bytes, void *stream);
int ls_upwind_step_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                       const int32_t *tiles, const int32_t *ntiles_dev, int nsteps,
                       double *scratch, void *workspace, int64_t workspace_bytes, void *stream);
int ls_upwind_step_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g,
                        float dx, float dt, const int32_t *tiles, const int32_t *ntiles_dev,
                        int nsteps, uint16_t *scratch, void *workspace, int64_t workspace_bytes,
                        void *stream);

/* ---------------------------------------------------------------------------
 * Incremental band rebuild: the list ls_band_build_* (dilate = 1) would
 * return, computed by rescanning only the tiles of a previous band list
 * prev_tiles[0 .. *prev_ntiles_dev) instead of the whole grid.
 *
 * Exact under this precondition: no tile outside prev_tiles holds a point with
 * |phi| < gamma.  It holds when prev_tiles is the dilated band of an earlier
 * build or rebuild of this grid and phi has changed only on prev_tiles since
 * (the band step changes nothing else): a tile outside that band had no point
 * in the tube then (the band contains the tube's tiles) and has the same
 * values now.  prev_tiles / prev_ntiles_dev must not alias tiles /
 * ntiles_dev.  Cost O(|prev band|) instead of O(nx*ny*nz).
 * ------------------------------------------------------------------------- */
int ls_band_rebuild_f32(const float *phi, const ls_grid *g, float gamma,
                        const int32_t *prev_tiles, const int32_t *prev_ntiles_dev, int32_t *tiles,
                        int64_t capacity, int32_t *ntiles_dev, void *workspace,
                        int64_t workspace_bytes, void *stream);
int ls_band_rebuild_f64(const double *phi, const ls_grid *g, double gamma,
                        const int32_t *prev_tiles, const int32_t *prev_ntiles_dev, int32_t *tiles,
                        int64_t capacity, int32_t *ntiles_dev, void *workspace,
                        int64_t workspace_bytes, void *stream);
int ls_band_rebuild_f16s(const uint16_t *phi_h, float scale, const ls_grid *g, float gamma,
                         const int32_t *prev_tiles, const int32_t *prev_ntiles_dev,
                         int32_t *tiles, int64_t capacity, int32_t *ntiles_dev, void *workspace,
                         int64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Narrow-band driver (Steps 1-2 of the algorithm in Sec. 1.1, repeated):
 * for every window of `window` steps, rebuild the dilated band from the
 * current phi and advance `window` steps on it; the last window may be
 * shorter.  The first window builds from a full scan (ls_band_build_*), the
 * later ones rebuild incrementally from the previous window's band
 * (ls_band_rebuild_*, exact here), so the result equals calling
 * ls_band_build_* and ls_upwind_step_* window by window, bit for bit.
 * tiles / ntiles_dev receive the band of the last window.  tile_steps_dev
 * (device int64, may be NULL) is incremented by the number of band tiles
 * times the steps taken on them, summed over the windows.  One call, no host
 * synchronisation.
 * ------------------------------------------------------------------------- */
int ls_band_run_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                    float gamma, int nsteps, int window, int32_t *tiles, int64_t capacity,
                    int32_t *ntiles_dev, int64_t *tile_steps_dev, float *scratch,
                    void *workspace, int64_t workspace_bytes, void *stream);
int ls_band_run_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                    double gamma, int nsteps, int window, int32_t *tiles, int64_t capacity,
                    int32_t *ntiles_dev, int64_t *tile_steps_dev, double *scratch,
                    void *workspace, int64_t workspace_bytes, void *stream);
int ls_band_run_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g, float dx,
                     float dt, float gamma, int nsteps, int window, int32_t *tiles,
                     int64_t capacity, int32_t *ntiles_dev, int64_t *tile_steps_dev,
                     uint16_t *scratch, void *workspace, int64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Launch tuning (process-wide; used by the autotuner, not part of the method).
 *
 * run_width: target width in grid points of one work item of the band step
 * (a run of run_width / tx consecutive band tiles of one tile row, at least
 * one tile, at most 32); blocks_per_cu: workgroups launched per compute unit
 * by the band step (0 = the occupancy limit).  Zero fields select the
 * defaults (run_width 32).  Results do not depend on the tuning, only speed
 * does.  Not thread-safe against concurrent launches.
 * ------------------------------------------------------------------------- */
typedef struct ls_tuning {
    int32_t run_width;
    int32_t blocks_per_cu;
} ls_tuning;
int ls_set_tuning(const ls_tuning *t);
int ls_get_tuning(ls_tuning *t);

/* Launch configuration the band step would use for grid g on the current
 * device: precision 0 = f32, 1 = f64, 2 = f16s.  Outputs (any may be NULL):
 * workgroups, LDS bytes per workgroup, tiles per work item, and the
 * occupancy limit in workgroups per compute unit. */
int ls_upwind_launch_info(const ls_grid *g, int precision, int32_t *blocks, int32_t *lds_bytes,
                          int32_t *run_tiles, int32_t *blocks_per_cu_limit);

/* ---------------------------------------------------------------------------
 * Kernel timing (measurement support, not part of the method).
 *
 * While enabled, every launch of the kernel `which` (LS_KERNEL_UPWIND: the
 * band step kernel, LS_KERNEL_BAND_FLAG: the band build's full scan of phi)
 * is bracketed by a pair of HIP events recorded on the launch stream.
 * ls_stats_enable(1) clears the record; ls_stats_read waits for the recorded
 * events and returns the number of launches and their summed duration in ms.
 * At most 65536 launches per kernel are recorded; later ones are counted in
 * *launches but not timed (*timed tells how many were).  Do not enable it
 * while a stream is being captured into a HIP graph.
 * ------------------------------------------------------------------------- */
enum { LS_KERNEL_UPWIND = 0, LS_KERNEL_BAND_FLAG = 1 };
int ls_stats_enable(int on);
int ls_stats_read(int which, int64_t *launches, int64_t *timed, double *total_ms);

/* Plain copy dst[i] = src[i], i < n, one 4-byte load and store per lane (the
 * access width of the band step): the reference kernel against which the
 * hardware traffic counters are calibrated.  Device pointers, n >= 0. */
int ls_copy_f32(float *dst, const float *src, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LS_H */
