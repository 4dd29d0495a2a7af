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
 * Band build without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): ls_band_build_f32 with the workspace taken from a fixed
 * device array of the library instead of an argument.  Same arguments,
 * results (bit for bit), checks and errors as ls_band_build_f32 otherwise.
 *
 * The array holds ls_band_build_noalloc_max_bytes() bytes (16 MiB) on every
 * device the library runs on, until the process ends; a grid whose workspace
 * (ls_workspace_bytes) is larger returns LS_ERR_CAPACITY before anything is
 * launched (8^3 tiles: grids of up to about 440 000 tiles, e.g. 512^3).  The
 * call allocates nothing (no hipMalloc, no library allocation; keep kernel
 * timing, ls_stats_enable, off, since it creates HIP events).  Every call on
 * one device uses that device's one array and leaves its contents behind:
 * calls that overlap on one device (concurrent streams, or host threads)
 * race and must be serialised by the caller.  The array's address is looked
 * up on the first call on each device (LS_ERR_HIP if that fails).
 * ------------------------------------------------------------------------- */
int64_t ls_band_build_noalloc_max_bytes(void);
int ls_band_build_f32_noalloc(const float *phi, const ls_grid *g, float gamma, int dilate,
                              int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
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
 * Tile-major ("brick") layout.  The grid's tiles one after another in tile-id
 * order, each tile's points contiguous with x fastest inside the tile: point
 * (i, j, k) of tile t = (tk*nty + tj)*ntx + ti at element
 * t*512 + (k%8)*64 + (j%8)*8 + (i%8).  A run of band tiles along x is then
 * one contiguous stretch of memory, which the band kernels stream where the
 * x-fastest layout scatters it over 64 grid rows.  Requires 8x8x8 tiles,
 * whole tiles on every axis (nx, ny, nz multiples of 8; LS_ERR_UNSUPPORTED
 * otherwise) and 16-byte aligned buffers (LS_ERR_ARG); a brick field has as
 * many elements as the grid.
 *
 * ls_bricks_from_dense_* / ls_bricks_to_dense_*: the permutation between the
 * layouts (FP32 values, or scaled-FP16 codes moved as they are); src and dst
 * must not overlap.
 *
 * ls_band_build_bricks_*: ls_band_build_* on a brick field (same list, same
 * plan in the workspace).
 *
 * ls_band_run_bricks_*: the windowed driver of Sec. 1.1 on brick fields phi_b
 * and F_b (F_b = the speed converted with ls_bricks_from_dense_f32; FP32 for
 * both storages), with scratch_b the ping-pong partner (a brick field of
 * phi's type).  Per window of `window` steps: the band build (a full scan of
 * phi_b for the first window, the exact incremental rescan of the previous
 * band after), `window` steps of Eq. 3-5 on it (with beta > 0: the cut-off
 * steps of Eq. 8 with c(phi) of beta and the band's gamma; beta = 0: plain
 * steps), then reinit_iters reinitialisation steps of Eq. 12-13 (pseudo time
 * step dtau) on the same band, the last followed by the clamp of Eq. 10 to
 * [-gamma, gamma] (reinit_iters = 0: no Step 3).  Every value equals, bit for
 * bit, what the x-fastest calls compute (ls_band_run_*, ls_band_run_cutoff_*,
 * ls_band_run_reinit_*) on the same fields converted, since the kernels
 * evaluate the same arithmetic on the same neighbours.  tiles / ntiles_dev /
 * tile_steps_dev and the errors as for ls_band_run_*; 0 < beta < gamma < inf
 * when beta != 0, gamma positive and finite when reinit_iters > 0.
 * ------------------------------------------------------------------------- */
int ls_bricks_from_dense_f32(const float *src, const ls_grid *g, float *dst, void *stream);
int ls_bricks_to_dense_f32(const float *src, const ls_grid *g, float *dst, void *stream);
int ls_bricks_from_dense_f16s(const uint16_t *src, const ls_grid *g, uint16_t *dst,
                              void *stream);
int ls_bricks_to_dense_f16s(const uint16_t *src, const ls_grid *g, uint16_t *dst, void *stream);
int ls_band_build_bricks_f32(const float *phi_b, const ls_grid *g, float gamma, int dilate,
                             int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                             void *workspace, int64_t workspace_bytes, void *stream);
int ls_band_build_bricks_f16s(const uint16_t *phi_b, float scale, const ls_grid *g, float gamma,
                              int dilate, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                              void *workspace, int64_t workspace_bytes, void *stream);
int ls_band_run_bricks_f32(float *phi_b, const float *F_b, const ls_grid *g, float dx, float dt,
                           float gamma, int nsteps, int window, float beta, int reinit_iters,
                           float dtau, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                           int64_t *tile_steps_dev, float *scratch_b, void *workspace,
                           int64_t workspace_bytes, void *stream);
int ls_band_run_bricks_f16s(uint16_t *phi_b, float scale, const float *F_b, const ls_grid *g,
                            float dx, float dt, float gamma, int nsteps, int window, float beta,
                            int reinit_iters, float dtau, int32_t *tiles, int64_t capacity,
                            int32_t *ntiles_dev, int64_t *tile_steps_dev, uint16_t *scratch_b,
                            void *workspace, int64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Cut-off step and driver (Sec. 1.1, Eq. 7-8): the same calls as
 * ls_upwind_step_* and ls_band_run_* for the cut-off equation
 * phi_t + c(phi) F |grad phi| = 0, with
 *   c(phi) = 1                                                 |phi| <= beta
 *          = (|phi| - gamma)^2 (2|phi| + gamma - 3 beta) / (gamma - beta)^3
 *                                                beta < |phi| <= gamma
 *          = 0                                 |phi| > gamma (and NaN)
 * taken at each point's step-n value: every step is the upwind step of
 * Eq. 3-5 with the speed c(phi^n) F.  Points with |phi| >= gamma, and points
 * whose c(phi) F is zero, keep their bits.  beta and gamma are in phi's units
 * (for f16s: of phi, not of h); ls_band_run_cutoff_* uses its gamma for the
 * tube of Eq. 6 as well.  Arithmetic of c: f64 the definition term by term
 * ((gamma - beta)^3 formed on the host in FP64); f32 and f16s in FP32 as the
 * equal cubic u^2 (3 - 2u), u = (gamma - |phi|) / (gamma - beta) clamped to
 * [0, 1] (1 for |phi| <= beta and 0 from gamma on, as in f64).  Requires
 * 0 < beta < gamma < inf (LS_ERR_ARG otherwise); the other arguments, buffers
 * and errors as for the plain calls.  The two-step kernel of
 * ls_tuning.temporal is not used here.
 * ------------------------------------------------------------------------- */
int ls_upwind_step_cutoff_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                              float beta, float gamma, const int32_t *tiles,
                              const int32_t *ntiles_dev, int nsteps, float *scratch,
                              void *workspace, int64_t workspace_bytes, void *stream);
int ls_upwind_step_cutoff_f64(double *phi, const double *F, const ls_grid *g, double dx,
                              double dt, double beta, double gamma, const int32_t *tiles,
                              const int32_t *ntiles_dev, int nsteps, double *scratch,
                              void *workspace, int64_t workspace_bytes, void *stream);
int ls_upwind_step_cutoff_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g,
                               float dx, float dt, float beta, float gamma,
                               const int32_t *tiles, const int32_t *ntiles_dev, int nsteps,
                               uint16_t *scratch, void *workspace, int64_t workspace_bytes,
                               void *stream);
int ls_band_run_cutoff_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                           float beta, float gamma, int nsteps, int window, int32_t *tiles,
                           int64_t capacity, int32_t *ntiles_dev, int64_t *tile_steps_dev,
                           float *scratch, void *workspace, int64_t workspace_bytes,
                           void *stream);
int ls_band_run_cutoff_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                           double beta, double gamma, int nsteps, int window, int32_t *tiles,
                           int64_t capacity, int32_t *ntiles_dev, int64_t *tile_steps_dev,
                           double *scratch, void *workspace, int64_t workspace_bytes,
                           void *stream);
int ls_band_run_cutoff_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g,
                            float dx, float dt, float beta, float gamma, int nsteps, int window,
                            int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                            int64_t *tile_steps_dev, uint16_t *scratch, void *workspace,
                            int64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Reinitialisation (Sec. 1.1, Eq. 12-13) and clamp (Eq. 10).
 *
 * ls_reinit_step_*: niter pseudo-time steps of d_tau + S(d) (|grad d| - 1) = 0
 * on every grid point of the listed tiles (the list as for ls_upwind_step_*),
 * with the smoothed sign S(d) = d / sqrt(d^2 + |Dd|^2 dx^2) of the current
 * iterate (Dd: central differences; S = 0 where d = 0).  Each step is the
 * upwind step of Eq. 3-5 with the speed S(d) for the |grad d| term, plus
 * dtau S(d) for the -1 term:  d' = d - dtau S (|grad d|_upwind - 1).  With
 * clamp = 1 the last step's values are clamped to [-gamma, gamma] (Eq. 10;
 * gamma > 0 and finite).  Points outside the tiles keep their bits and are
 * read as frozen neighbours; the grid faces are zero-gradient; a point with
 * d == 0 keeps its bits.  No F is read.  dx > 0, dtau >= 0 (stable for
 * dtau <= dx / sqrt(3)), niter >= 0; scratch as for the step.  S and the
 * update: f64 the definition term by term; f32 and f16s in FP32 with the
 * hardware reciprocal square root for 1 / sqrt(d^2 + |Dd|^2 dx^2).
 *
 * ls_band_run_reinit_*: the narrow-band algorithm of Sec. 1.1, Steps 1-3, in
 * windows: for each window of `window` steps, build (or rebuild) the band U
 * of gamma (Eq. 6, 11; U contains the region N of Eq. 11), take the cut-off
 * steps of Eq. 8 (beta, gamma as for ls_band_run_cutoff_*) on U, then
 * reinit_iters reinitialisation steps on U, the last one clamped to the band's
 * gamma.  tile_steps_dev counts band tiles x time steps (not the
 * reinitialisation steps).  reinit_iters >= 0, dtau >= 0 and finite;
 * reinit_iters = 0 is ls_band_run_cutoff_* exactly.  Errors as for the other
 * calls.
 * ------------------------------------------------------------------------- */
int ls_reinit_step_f32(float *phi, const ls_grid *g, float dx, float dtau, float gamma, int clamp,
                       const int32_t *tiles, const int32_t *ntiles_dev, int niter,
                       float *scratch, void *workspace, int64_t workspace_bytes, void *stream);
int ls_reinit_step_f64(double *phi, const ls_grid *g, double dx, double dtau, double gamma,
                       int clamp, const int32_t *tiles, const int32_t *ntiles_dev, int niter,
                       double *scratch, void *workspace, int64_t workspace_bytes, void *stream);
int ls_reinit_step_f16s(uint16_t *phi_h, float scale, const ls_grid *g, float dx, float dtau,
                        float gamma, int clamp, const int32_t *tiles, const int32_t *ntiles_dev,
                        int niter, uint16_t *scratch, void *workspace, int64_t workspace_bytes,
                        void *stream);
int ls_band_run_reinit_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                           float beta, float gamma, float dtau, int reinit_iters, int nsteps,
                           int window, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                           int64_t *tile_steps_dev, float *scratch, void *workspace,
                           int64_t workspace_bytes, void *stream);
int ls_band_run_reinit_f64(double *phi, const double *F, const ls_grid *g, double dx, double dt,
                           double beta, double gamma, double dtau, int reinit_iters, int nsteps,
                           int window, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                           int64_t *tile_steps_dev, double *scratch, void *workspace,
                           int64_t workspace_bytes, void *stream);
int ls_band_run_reinit_f16s(uint16_t *phi_h, float scale, const float *F, const ls_grid *g,
                            float dx, float dt, float beta, float gamma, float dtau,
                            int reinit_iters, int nsteps, int window, int32_t *tiles,
                            int64_t capacity, int32_t *ntiles_dev, int64_t *tile_steps_dev,
                            uint16_t *scratch, void *workspace, int64_t workspace_bytes,
                            void *stream);

/* ---------------------------------------------------------------------------
 * Band snapshot (the output of Step 4 of the algorithm in Sec. 1.1,
 * restricted to the band): copies the values of the tiles listed in
 * tiles[0 .. n), n = min(*ntiles_dev, capacity), into out, tile by tile in
 * list order: tile p occupies out[p*tp .. (p+1)*tp), tp = tx*ty*tz, its
 * points x fastest, then y, then z within the tile; points of a partial tile
 * outside the grid, and every point of a tile whose id is not in
 * [0, ls_grid_tiles(g)), are written as zero bits.  With ids_out non-NULL,
 * ids_out[p] = tiles[p] for p < n (a copy of the list, so that the snapshot
 * outlives the next band build).  out holds capacity*tp elements of phi's type
 * (f16s: the stored FP16 codes, unscaled), ids_out capacity int32;
 * 0 <= capacity <= ls_grid_tiles(g).  Nothing is read from the host: the call
 * is stream-ordered and can be captured; a device-to-host copy of the first
 * n tiles of out (n read back from *ntiles_dev) takes the snapshot off the
 * GPU.
 * ------------------------------------------------------------------------- */
int ls_band_gather_f32(const float *phi, const ls_grid *g, const int32_t *tiles,
                       const int32_t *ntiles_dev, float *out, int32_t *ids_out, int64_t capacity,
                       void *stream);
int ls_band_gather_f64(const double *phi, const ls_grid *g, const int32_t *tiles,
                       const int32_t *ntiles_dev, double *out, int32_t *ids_out,
                       int64_t capacity, void *stream);
int ls_band_gather_f16s(const uint16_t *phi_h, const ls_grid *g, const int32_t *tiles,
                        const int32_t *ntiles_dev, uint16_t *out, int32_t *ids_out,
                        int64_t capacity, void *stream);

/* Counted copy (support of the snapshot's device-to-host transfer): copies
 * n = min(max(*count_dev, 0), max_units) units of unit_bytes bytes from src to
 * dst, the count read on the device when the kernel runs, so that a copy of
 * exactly the tiles a gather produced is enqueued without the host waiting
 * for the gather.  dst and src are device-accessible (device memory, or host
 * memory allocated pinned, e.g. hipHostMalloc / torch's pin_memory: the
 * kernel then writes host memory directly) and must not overlap; with
 * count_out non-NULL (device-accessible) the copy also stores n there.  blocks
 * is the number of workgroups (0: a quarter of the compute units), kept small
 * so that the copy shares the GPU with the compute stream.  Errors: NULL
 * pointers, unit_bytes <= 0, max_units outside [0, 2^31), blocks < 0. */
int ls_copy_counted(void *dst, const void *src, const int32_t *count_dev, int64_t unit_bytes,
                    int64_t max_units, int32_t *count_out, int blocks, void *stream);
/* The same for units [first_unit, n) only (dst and src still point at unit 0;
 * nothing is copied when n <= first_unit; count_out still receives n): the
 * tail beyond what a copy of a host-known size already moved.  Errors as
 * above, and first_unit outside [0, max_units]. */
int ls_copy_counted_from(void *dst, const void *src, const int32_t *count_dev,
                         int64_t unit_bytes, int64_t first_unit, int64_t max_units,
                         int32_t *count_out, int blocks, void *stream);

/* ---------------------------------------------------------------------------
 * Batches: many grids of uneven size, advanced in lockstep by the same
 * launches (the narrow-band driver above, applied to every grid at once).
 *
 * Each grid lives in the caller's phi / F / scratch buffers (FP32) at element
 * `offset`, x fastest, with `pitch` elements from one x row to the next
 * (pitch >= nx; 0 means nx, the dense layout above) and pitch * ny from one z
 * plane to the next: point (i, j, k) is element offset + (k*ny + j)*pitch + i.
 * The pitch padding is never read or written.  A pitch that is a multiple of
 * 32 (128 bytes) with a 128-byte aligned offset starts every row on a cache
 * line, which the step kernel's row loads are laid out for.  The grids (their
 * pitch * ny * nz spans) must not overlap.  The tile shape of
 * a grid is its own (typically picked per size by an autotuner); it must be
 * one of the shapes the batched step kernel is compiled for: 8x8x8, 16x4x4,
 * 32x4x4, 16x8x8 or 4x4x4 with the default run width, and the other shapes
 * ls_upwind_launch_info reports as having a compiled fast kernel.
 *
 * The grids' tile grids are concatenated, in an order ls_batch_layout gives,
 * into one global tile space; band lists of a batch hold global tile ids
 * (ascending), grid i owning [tile_base[i], tile_base[i] + its tile count).
 * ------------------------------------------------------------------------- */
typedef struct ls_instance {
    ls_grid grid;     /* dims and band tile shape */
    int64_t offset;   /* first element of this grid in phi, F and scratch */
    float dx, dt;     /* spacing and time step */
    float gamma;      /* band half-width */
    int32_t pitch;    /* elements between consecutive x rows (>= nx); 0 = nx */
} ls_instance;

/* Workspace bytes of a batch (device memory, caller-owned). */
int64_t ls_batch_workspace_bytes(const ls_instance *inst, int n);
/* Global tile base of every grid (host array of n) and the total tile count. */
int ls_batch_layout(const ls_instance *inst, int n, int64_t *tile_base, int64_t *total_tiles);
/* Uploads the grid descriptors into the workspace (synchronises `stream`);
 * call once before ls_batch_run_f32 with the same instance array. */
int ls_batch_setup(const ls_instance *inst, int n, void *workspace, int64_t workspace_bytes,
                   void *stream);
/* The narrow-band driver for every grid of the batch: per window one band
 * build of all grids (a full scan for the first window, the exact incremental
 * rescan of the previous bands afterwards) and `window` steps of all grids;
 * equal, grid by grid, to ls_band_run_f32 on each grid alone with its tile
 * shape, bit for bit.  tile_steps_dev as in ls_band_run_f32 (summed over the
 * grids); point_steps_dev (may be NULL) accumulates steps x in-domain points
 * of every band tile (partial tiles at the high faces count their points).  Asynchronous, no host synchronisation: capturable in a HIP graph. */
int ls_batch_run_f32(const ls_instance *inst, int n, float *phi, const float *F, float *scratch,
                     int nsteps, int window, int64_t *tile_steps_dev, int64_t *point_steps_dev,
                     void *workspace, int64_t workspace_bytes, void *stream);
/* Device pointers (inside the workspace) to the batch's last band list and
 * its length. */
int ls_batch_band(const ls_instance *inst, int n, void *workspace, int64_t workspace_bytes,
                  const int32_t **tiles_dev, const int32_t **ntiles_dev);

/* ---------------------------------------------------------------------------
 * HIP graphs: capture the library calls issued on `stream` between
 * ls_graph_begin and ls_graph_end into an executable graph, replayed with
 * ls_graph_launch.  `stream` must not be the NULL stream.  A replay repeats
 * exactly the captured launches with the captured arguments (pointers and
 * scalars); the band lists, counts and work items they use live on the
 * device, so a captured window sequence needs no host involvement.  Do not
 * enable kernel timing while capturing.  *graph is an opaque handle.
 * ------------------------------------------------------------------------- */
int ls_graph_begin(void *stream);
int ls_graph_end(void *stream, void **graph);
int ls_graph_launch(void *graph, void *stream);
int ls_graph_destroy(void *graph);

/* ---------------------------------------------------------------------------
 * Launch tuning (process-wide; used by the autotuner, not part of the method).
 *
 * run_width: target width in grid points of one work item of the band step
 * (a run of run_width / tx consecutive band tiles of one tile row, at least
 * one tile, at most 32); blocks_per_cu: workgroups launched per compute unit
 * by the band step (0 = the occupancy limit).  Zero fields select the
 * defaults (run_width 32).  pipeline: whether a workgroup issues the loads of
 * its next work item before updating the current one (software pipelining;
 * it pays on grids that stream from HBM, where workgroups own several items,
 * and costs registers).  Results do not depend on the tuning, only speed
 * does.  Not thread-safe against concurrent launches.
 * ------------------------------------------------------------------------- */
typedef struct ls_tuning {
    int32_t run_width;
    int32_t blocks_per_cu;
    int32_t pipeline; /* 0 auto (single grids: on when phi exceeds 1 GiB and a
                         work item spans at most 4 tiles; batches: off),
                         1 off, 2 on */
    int32_t vector;   /* 0 auto (FP32 and FP16s, 8x8x8 tiles, nx a multiple of
                         4, aligned buffers: the vectorised kernel), 1 off */
    int32_t temporal; /* steps per launch (bit-identical either way).  0 auto:
                         one on the x-fastest layout; on the brick layout two
                         for FP32, one for FP16s;
                         1 two (x-fastest: where the vectorised kernel runs on
                         grids of whole tiles in y and z, measured slower);
                         2 one */
} ls_tuning;
int ls_set_tuning(const ls_tuning *t);
int ls_get_tuning(ls_tuning *t);

/* Tile-shape autotuner (native): for each size in sizes[0..n) (cubic grids
 * of that many points per axis), among the tile shapes whose time per window
 * of the FP32 batched band driver is within 3 % of the shortest, the one with
 * the fewest halo points per tile point, measured once per size bucket of 32
 * points on a batch of copies of a synthetic n^3 ellipsoid (n = bucket*32 +
 * 16; about 2^25 points in all, at most 512 copies) over the shapes the
 * batched step is compiled for: 8x8x8, 16x4x4, 32x4x4, 16x8x8, 4x4x4.  out[i]
 * receives the grid (sizes[i]^3) with the chosen tile.  Results are cached in
 * the text file cache_path (NULL: no cache), keyed by device architecture,
 * compute-unit count and bucket; force != 0 re-measures every bucket asked
 * for.  Unlike every other call, the measurement allocates (and frees) its
 * own device buffers and synchronises its own stream; precision must be 0
 * (FP32). */
int ls_autotune(const int32_t *sizes, int n, int precision, const char *cache_path, ls_grid *out,
                int force);

/* Launch configuration the band step would use for grid g on the current
 * device: precision 0 = f32, 1 = f64, 2 = f16s.  Outputs (any may be NULL):
 * workgroups, LDS bytes per workgroup, tiles per work item, and the
 * occupancy limit in workgroups per compute unit, for 16-byte aligned phi, F
 * and scratch buffers (what every allocator here returns). */
int ls_upwind_launch_info(const ls_grid *g, int precision, int32_t *blocks, int32_t *lds_bytes,
                          int32_t *run_tiles, int32_t *blocks_per_cu_limit);

/* ---------------------------------------------------------------------------
 * Kernel timing (measurement support, not part of the method).
 *
 * While enabled, the launches of the kernel `which` (LS_KERNEL_UPWIND: the
 * band step kernel, LS_KERNEL_BAND_FLAG: the band build's scan of phi,
 * LS_KERNEL_REINIT: the reinitialisation steps, LS_KERNEL_GATHER: the band
 * snapshot's gather, LS_KERNEL_CLOSURE: the closure's fused network kernel)
 * are
 * bracketed by pairs of HIP events recorded on the launch stream: one pair
 * around each scan, and one pair around the back-to-back step launches of a
 * call (a window's launches), so the time per launch includes the short gaps
 * between consecutive launches but not the setup of the call.
 * ls_stats_enable(1) clears the record; ls_stats_read waits for the recorded
 * events and returns the number of launches, how many of them were timed,
 * and the summed duration of the timed ones in ms.  At most 65536 event pairs
 * per kernel are recorded.  Do not enable it while a stream is being captured
 * into a HIP graph.
 * ------------------------------------------------------------------------- */
enum {
    LS_KERNEL_UPWIND = 0,
    LS_KERNEL_BAND_FLAG = 1,
    LS_KERNEL_REINIT = 2,
    LS_KERNEL_GATHER = 3,
    LS_KERNEL_CLOSURE = 4
};
int ls_stats_enable(int on);
int ls_stats_read(int which, int64_t *launches, int64_t *timed, double *total_ms);

/* Plain copy dst[i] = src[i], i < n, one 4-byte load and store per lane (the
 * access width of the band step): the reference kernel against which the
 * hardware traffic counters are calibrated.  Device pointers, n >= 0. */
int ls_copy_f32(float *dst, const float *src, int64_t n, void *stream);

/* ---------------------------------------------------------------------------
 * Learned closure of the coarse first-order step (an addition to the method:
 * the paper has no network; the step it corrects is Eq. 3-5 on the band of
 * Eq. 6 and Eq. 11).
 *
 * A 3-layer 3x3x3 convolutional network, channels 3 -> 16 -> 16 -> 1 with
 * SiLU after the first two layers and zero padding outside the grid, maps
 * per-point features of the coarse field
 *     c0 = clip(phi / gamma, -2, 2),  c1 = F / fmax,  c2 = (plain - phi) / dx
 * (plain = phi after one plain step, Eq. 3) to a correction r, and the
 * corrected step is
 *     phi^{n+1} = plain + k,  k = dx * c(phi) * r clipped to
 *                 |k| <= |plain - phi| / 2,  on the active tiles A (Eq. 6 in
 *                                            tile form),
 *     phi^{n+1} = plain                      elsewhere in the band U,
 * with c the cut-off function of Eq. 8 for beta = gamma / 2 (1 near the
 * front, 0 from |phi| = gamma on), and the clip a limiter (the correction
 * never reverses or stalls the plain step), except that an active tile where some
 * c(phi) * r is non-finite or above 1/2 in magnitude takes the plain step (a
 * fallback, counted).  Activations outside
 * U count as zero; since A lies one tile inside U and the network sees three
 * points around a point, r on A equals the network's value with no band.
 * Weights and activations are BF16 on the matrix cores with FP32
 * accumulation; the parameters are an FP32 master vector.
 *
 * Parameters: a flat FP32 vector of ls_closure_param_count() = 8673 values,
 * in the order w0 (16,3,3,3,3), b0 (16), w1 (16,16,3,3,3), b1 (16),
 * w2 (1,16,3,3,3), b2 (1); each weight is indexed (out, in, dz, dy, dx) and
 * the layer is the cross-correlation
 *     out[o](z,y,x) = b[o] + sum_{c,dz,dy,dx} w[o,c,dz,dy,dx] in[c](z+dz-1, y+dy-1, x+dx-1).
 *
 * Grid: FP32, 8x8x8 tiles, every dimension a multiple of 8.  Every closure
 * call takes, besides the band workspace of ls_workspace_bytes, a closure
 * workspace of ls_closure_workspace_bytes(g) bytes (device, caller-owned,
 * 256-byte aligned; no initialisation needed), and the caller's band list
 * buffer (tiles, capacity >= ls_grid_tiles, ntiles_dev) into which U is
 * built from the call's phi (band half-width gamma, 26-neighbour dilation).
 * fmax > 0 is the feature scale of F (the caller's max |F|).
 * ------------------------------------------------------------------------- */
int64_t ls_closure_param_count(void);
int64_t ls_closure_workspace_bytes(const ls_grid *g);

/* Coarse field of a fine one, 4x in every axis: coarse point (I,J,K) is the
 * mean of the 2x2x2 fine points 4I+1..4I+2 (likewise J, K), which surround
 * the coarse cell centre on a cell-centred grid.  fine_grid gives the fine
 * dims (multiples of 4); coarse holds (nx/4)(ny/4)(nz/4) floats. */
int ls_restrict4_f32(const float *fine, const ls_grid *fine_grid, float *coarse, void *stream);

/* One network evaluation at phi: builds A and U from phi, the plain step into
 * `plain` (dense, may be NULL) and r into `r` (dense; zero outside A; may be
 * NULL).  phi is not modified. */
int ls_closure_forward_f32(const float *phi, const float *F, const ls_grid *g, float dx, float dt,
                           float gamma, float fmax, const float *params, float *r, float *plain,
                           int32_t *tiles, int64_t capacity, int32_t *ntiles_dev, void *ws,
                           int64_t ws_bytes, void *cws, int64_t cws_bytes, void *stream);

/* Training loss and gradient at phi toward target (the fine solution one
 * coarse step later, restricted): loss = mean over the points of A of
 * (c(phi) r - r*)^2 with r* = (target - plain) / dx, written to *loss_dev (may be
 * NULL); grad (8673 floats, overwritten) is d loss / d params, computed by
 * the backward kernels (data gradients through the transposed convolutions,
 * weight gradients as per-tile partial sums reduced in tile order). */
int ls_closure_backward_f32(const float *phi, const float *target, const float *F,
                            const ls_grid *g, float dx, float dt, float gamma, float fmax,
                            const float *params, float *grad, float *loss_dev, int32_t *tiles,
                            int64_t capacity, int32_t *ntiles_dev, void *ws, int64_t ws_bytes,
                            void *cws, int64_t cws_bytes, void *stream);

/* One Adam update (Kingma and Ba) of n FP32 parameters with step count t >= 1:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
int ls_adam_step(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                 float beta1, float beta2, float eps, int t, void *stream);

/* The corrected narrow-band driver: per window of `window` steps, A and U are
 * built from the current phi, then every step is the plain step on U plus the
 * correction on A (with the per-tile fallback).  *fallbacks_dev (int32,
 * caller-zeroed) accumulates the fallback count.
 *
 * judge != 0 makes the plain scheme the judge of the corrected run's
 * interface: a shadow copy of the initial phi (in the closure workspace) is
 * advanced by the plain narrow-band driver (ls_band_run_f32) window by window
 * beside the corrected run, and after every window each 8^3 tile whose
 * zero-crossing state (whether it holds points of both signs, phi < 0 and
 * phi >= 0) differs between the corrected field and the shadow takes the
 * shadow's values.  A correction may so move the interface but not create,
 * remove, split or merge a piece of it inside a tile against the plain run.
 * judge == 2 bounds the interface's position as well: a tile also takes the
 * shadow's values when the two fronts lie more than one grid spacing apart
 * there (a point next to either front, |phi| < dx or |shadow| < dx, where
 * |phi - shadow| > dx); judge == 3 the same with half a grid spacing
 * (|phi - shadow| > dx / 2 there); judge == 1 is the topology judge alone.
 * *resets_dev (int32, caller-zeroed; required when judging) accumulates the
 * number of tiles reset.  judge == 0: no shadow run (resets_dev may be NULL);
 * other values of judge: LS_ERR_ARG.
 *
 * On return phi holds the result; the band list of the corrected run's last
 * window is in tiles / ntiles_dev. */
int ls_closure_run_f32(float *phi, const float *F, const ls_grid *g, float dx, float dt,
                       float gamma, float fmax, const float *params, int nsteps, int window,
                       int judge, int32_t *tiles, int64_t capacity, int32_t *ntiles_dev,
                       int32_t *fallbacks_dev, int32_t *resets_dev, void *ws, int64_t ws_bytes,
                       void *cws, int64_t cws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LS_H */
