/*
 * Plain FP64 CPU reference ("the oracle") for the narrow-band first-order
 * upwind level-set update of Wang, "Parallel Level set algorithm with MPI and
 * accelerated on GPU" (arXiv 1612.04040).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or constant with the GPU library.
 *
 * Written for obviousness, not speed: every step is the definition, in the
 * order the paper states it.  Built with gcc -O2 -ffp-contract=off -fopenmp so
 * that every operation is a separately rounded IEEE double operation.
 *
 * Conventions (the paper leaves them open; the readings are listed in the
 * design notes of the repository):
 *   grid      nx*ny*nz points, x fastest: idx = (k*ny + j)*nx + i (Sec. 3,
 *             the index formula of the GPU partition).
 *   D^{-x}    (phi[i] - phi[i-1]) / dx,  D^{+x} = (phi[i+1] - phi[i]) / dx,
 *             likewise in y and z; an index outside the grid is clamped to
 *             the nearest face (zero-gradient Neumann boundary).
 *   nabla^+   sqrt( [max(D-x,0)^2 + min(D+x,0)^2] + [y terms] + [z terms] )
 *             (Eq. 4, summed x, then y, then z).
 *   nabla^-   sqrt( [max(D+x,0)^2 + min(D-x,0)^2] + [y] + [z] )  (Eq. 5).
 *   update    phi' = phi - dt*[max(F,0) nabla^+ + min(F,0) nabla^-] (Eq. 3):
 *             F > 0 -> phi - dt*F*nabla^+, F < 0 -> phi - dt*F*nabla^-,
 *             F == 0 (either sign) -> phi unchanged, bit for bit.
 *   tiles     tx*ty*tz points, ceil(n/t) tiles per axis (partial tiles at the
 *             high faces), tile id = (tk*nty + tj)*ntx + ti.
 *   band A    tiles holding at least one point with |phi| < gamma (Eq. 6,
 *             strict), the tile form of the tube T.
 *   band U    A grown by one tile in all 26 directions, clipped to the grid:
 *             the tile form of the region N of Eq. 11 (the tube grown so the
 *             front can move into it).
 *   step      Jacobi: every updated point reads only values of step n; points
 *             outside the listed tiles keep their value.
 *   storage   optionally (store_scale s > 0) the state is held in scaled FP16,
 *             an addition to the method: each new value v is stored as
 *             h = fp16(v / s), rounded to nearest with ties to even, and read
 *             back as fl32(h * s); a point whose F is zero keeps its value.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LSO_OK 0
#define LSO_ERR_ARG (-1)
#define LSO_ERR_CAPACITY (-2)
#define LSO_ERR_NOMEM (-3)

/* Threads an OpenMP region of the oracle uses (for reporting only). */
int lso_max_threads(void) { return omp_get_max_threads(); }

/* Sets the threads of the following OpenMP regions (n >= 1). */
void lso_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/*
 * x rounded to the nearest IEEE binary16 value, ties to even: 10 fraction
 * bits, so the spacing is 2^(e - 11) for |x| in [2^(e-1), 2^e), never below
 * 2^-24 (the subnormal spacing); |x| >= 65520 (halfway between the largest
 * finite value 65504 and 2^16) rounds to infinity.
 */
static double round_binary16(double x)
{
    if (x != x)
        return x;
    const double a = fabs(x);
    if (a >= 65520.0)
        return copysign(INFINITY, x);
    if (a == 0.0)
        return x;
    int e;
    frexp(a, &e); /* a = m 2^e, m in [1/2, 1) */
    int q = e - 11;
    if (q < -24)
        q = -24;
    /* a / 2^q is exact; nearbyint rounds to nearest, ties to even */
    return copysign(ldexp(nearbyint(ldexp(a, -q)), q), x);
}

/* The stored value of v in scaled FP16: fl32(fp16(v / s) * s) (the product
 * of an 11-bit and a 24-bit significand is exact in double). */
static double store_f16s(double v, double s) { return (double)(float)(round_binary16(v / s) * s); }

/* Elementwise round_binary16 (exposed so that tests can check it against an
 * independent conversion). */
void lso_round_binary16(const double *in, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = round_binary16(in[i]);
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int dims_ok(int nx, int ny, int nz, int tx, int ty, int tz)
{
    return nx > 0 && ny > 0 && nz > 0 && tx > 0 && ty > 0 && tz > 0;
}

/* Number of tiles of the tile grid (the largest possible band list). */
int64_t lso_tile_count(int nx, int ny, int nz, int tx, int ty, int tz)
{
    if (!dims_ok(nx, ny, nz, tx, ty, tz))
        return LSO_ERR_ARG;
    return cdiv(nx, tx) * cdiv(ny, ty) * cdiv(nz, tz);
}

/*
 * Band tile list (Eq. 6 for A; Eq. 11 in tile form for U when dilate != 0).
 * phi holds the stored values promoted exactly to double, gamma the same
 * scalar the device receives promoted exactly.  Writes the ascending tile ids
 * to out[0..count) and returns count, or a negative status.
 */
int64_t lso_band_tiles(const double *phi, int nx, int ny, int nz,
                       int tx, int ty, int tz, double gamma, int dilate,
                       int32_t *out, int64_t capacity)
{
    if (!phi || !out || !dims_ok(nx, ny, nz, tx, ty, tz))
        return LSO_ERR_ARG;
    const int64_t ntx = cdiv(nx, tx), nty = cdiv(ny, ty), ntz = cdiv(nz, tz);
    const int64_t nt = ntx * nty * ntz;
    unsigned char *a = calloc((size_t)nt, 1);
    unsigned char *u = calloc((size_t)nt, 1);
    if (!a || !u) {
        free(a);
        free(u);
        return LSO_ERR_NOMEM;
    }

    /* A: some point of the tile lies strictly inside the tube |phi| < gamma. */
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const double v = phi[(k * ny + j) * nx + i];
                if (fabs(v) < gamma)
                    a[((k / tz) * nty + j / ty) * ntx + i / tx] = 1;
            }

    /* U: every tile within one tile (26-neighbourhood) of a tile of A. */
    for (int64_t t = 0; t < nt; ++t) {
        if (!a[t])
            continue;
        if (!dilate) {
            u[t] = 1;
            continue;
        }
        const int64_t ti = t % ntx, tj = (t / ntx) % nty, tk = t / (ntx * nty);
        for (int64_t dk = -1; dk <= 1; ++dk)
            for (int64_t dj = -1; dj <= 1; ++dj)
                for (int64_t di = -1; di <= 1; ++di) {
                    const int64_t ni = ti + di, nj = tj + dj, nk = tk + dk;
                    if (ni < 0 || nj < 0 || nk < 0 || ni >= ntx || nj >= nty || nk >= ntz)
                        continue;
                    u[(nk * nty + nj) * ntx + ni] = 1;
                }
    }

    int64_t count = 0;
    for (int64_t t = 0; t < nt; ++t)
        if (u[t])
            ++count;
    if (count > capacity) {
        free(a);
        free(u);
        return LSO_ERR_CAPACITY;
    }
    count = 0;
    for (int64_t t = 0; t < nt; ++t)
        if (u[t])
            out[count++] = (int32_t)t;
    free(a);
    free(u);
    return count;
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

static double sq(double v) { return v * v; }
static double maxd(double a, double b) { return a > b ? a : b; }
static double mind(double a, double b) { return a < b ? a : b; }

/* Eq. 3 with Eq. 4 / Eq. 5 at one point of the array cur (step n). */
static double upwind_point(const double *cur, const double *F, int64_t nx, int64_t ny, int64_t nz,
                           int64_t i, int64_t j, int64_t k, double dx, double dt)
{
    const int64_t idx = (k * ny + j) * nx + i;
    const double c = cur[idx];
    const double f = F[idx];
    if (f == 0.0)
        return c; /* max(F,0) = min(F,0) = 0: no change, not even of the sign of zero */

    /* Neighbours, indices clamped to the grid (Neumann boundary). */
    const double xm = cur[(k * ny + j) * nx + clampi(i - 1, 0, nx - 1)];
    const double xp = cur[(k * ny + j) * nx + clampi(i + 1, 0, nx - 1)];
    const double ym = cur[(k * ny + clampi(j - 1, 0, ny - 1)) * nx + i];
    const double yp = cur[(k * ny + clampi(j + 1, 0, ny - 1)) * nx + i];
    const double zm = cur[(clampi(k - 1, 0, nz - 1) * ny + j) * nx + i];
    const double zp = cur[(clampi(k + 1, 0, nz - 1) * ny + j) * nx + i];

    /* One-sided differences D^{-} and D^{+} per axis. */
    const double dmx = (c - xm) / dx, dpx = (xp - c) / dx;
    const double dmy = (c - ym) / dx, dpy = (yp - c) / dx;
    const double dmz = (c - zm) / dx, dpz = (zp - c) / dx;

    if (f > 0.0) {
        /* Eq. 4 */
        const double px = sq(maxd(dmx, 0.0)) + sq(mind(dpx, 0.0));
        const double py = sq(maxd(dmy, 0.0)) + sq(mind(dpy, 0.0));
        const double pz = sq(maxd(dmz, 0.0)) + sq(mind(dpz, 0.0));
        const double grad_plus = sqrt((px + py) + pz);
        return c - dt * f * grad_plus;
    } else {
        /* Eq. 5 */
        const double qx = sq(maxd(dpx, 0.0)) + sq(mind(dmx, 0.0));
        const double qy = sq(maxd(dpy, 0.0)) + sq(mind(dmy, 0.0));
        const double qz = sq(maxd(dpz, 0.0)) + sq(mind(dmz, 0.0));
        const double grad_minus = sqrt((qx + qy) + qz);
        return c - dt * f * grad_minus;
    }
}

/*
 * nsteps Jacobi steps of Eq. 3 on every grid point of the listed tiles,
 * in place on phi.  Points of unlisted tiles keep their value.  The tile list
 * must be ascending and in range; returns a status.
 */
int lso_upwind_steps_stored(double *phi, const double *F, int nx, int ny, int nz,
                            double dx, double dt, int tx, int ty, int tz,
                            const int32_t *tiles, int64_t ntiles, int nsteps, double store_scale)
{
    if (!phi || !F || !dims_ok(nx, ny, nz, tx, ty, tz) || nsteps < 0 || ntiles < 0)
        return LSO_ERR_ARG;
    if (ntiles > 0 && !tiles)
        return LSO_ERR_ARG;
    const int64_t ntx = cdiv(nx, tx), nty = cdiv(ny, ty), ntz = cdiv(nz, tz);
    const int64_t nt = ntx * nty * ntz;
    for (int64_t p = 0; p < ntiles; ++p) {
        if (tiles[p] < 0 || tiles[p] >= nt)
            return LSO_ERR_ARG;
        if (p > 0 && tiles[p] <= tiles[p - 1])
            return LSO_ERR_ARG;
    }
    if (nsteps == 0 || ntiles == 0)
        return LSO_OK;

    const int64_t npts = (int64_t)nx * ny * nz;
    double *nxt = malloc((size_t)npts * sizeof(double));
    if (!nxt)
        return LSO_ERR_NOMEM;

    for (int s = 0; s < nsteps; ++s) {
        /* New values of every listed point, from step-n values only. */
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t p = 0; p < ntiles; ++p) {
            const int64_t t = tiles[p];
            const int64_t ti = t % ntx, tj = (t / ntx) % nty, tk = t / (ntx * nty);
            for (int64_t k = tk * tz; k < (tk + 1) * tz && k < nz; ++k)
                for (int64_t j = tj * ty; j < (tj + 1) * ty && j < ny; ++j)
                    for (int64_t i = ti * tx; i < (ti + 1) * tx && i < nx; ++i) {
                        const int64_t idx = (k * ny + j) * nx + i;
                        double v = upwind_point(phi, F, nx, ny, nz, i, j, k, dx, dt);
                        if (store_scale > 0.0 && F[idx] != 0.0)
                            v = store_f16s(v, store_scale);
                        nxt[idx] = v;
                    }
        }
        /* Commit them: step n+1 becomes the current step. */
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t p = 0; p < ntiles; ++p) {
            const int64_t t = tiles[p];
            const int64_t ti = t % ntx, tj = (t / ntx) % nty, tk = t / (ntx * nty);
            for (int64_t k = tk * tz; k < (tk + 1) * tz && k < nz; ++k)
                for (int64_t j = tj * ty; j < (tj + 1) * ty && j < ny; ++j)
                    for (int64_t i = ti * tx; i < (ti + 1) * tx && i < nx; ++i)
                        phi[(k * ny + j) * nx + i] = nxt[(k * ny + j) * nx + i];
        }
    }
    free(nxt);
    return LSO_OK;
}

/* lso_upwind_steps_stored with the state kept in FP64 (no storage rounding). */
int lso_upwind_steps(double *phi, const double *F, int nx, int ny, int nz,
                     double dx, double dt, int tx, int ty, int tz,
                     const int32_t *tiles, int64_t ntiles, int nsteps)
{
    return lso_upwind_steps_stored(phi, F, nx, ny, nz, dx, dt, tx, ty, tz, tiles, ntiles, nsteps,
                                   0.0);
}
