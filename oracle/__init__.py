"""The oracle: a plain, slow, obviously correct FP64 CPU reference.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  It shares no code with
the GPU library and never imports it.

Arithmetic lives in ``ls_oracle.c`` (FP64, one rounding per operation); this
module marshals numpy arrays and runs the narrow-band driver of the paper's
algorithm (Sec. 1.1, Steps 1-2): rebuild the band, then advance on it.

Parity status of each function is stated in its docstring; the pins live in
``tests/test_oracle_*.py``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_LIB_PATH = None


def use_library(path=None):
    """Load the C part from ``path`` (default: the built ``liblsoracle.so``).

    Used by the mutation tests to swap in copies with a planted mistake.
    Returns the path that was in use before.
    """
    global _LIB, _LIB_PATH
    old = _LIB_PATH
    _LIB, _LIB_PATH = None, path
    return old


def _lib():
    global _LIB
    if _LIB is None:
        path = _LIB_PATH or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        i32, i64, dbl, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.lso_max_threads.restype = i32
        lib.lso_max_threads.argtypes = []
        lib.lso_tile_count.restype = i64
        lib.lso_tile_count.argtypes = [i32] * 6
        lib.lso_band_tiles.restype = i64
        lib.lso_band_tiles.argtypes = [vp, i32, i32, i32, i32, i32, i32, dbl, i32, vp, i64]
        lib.lso_upwind_steps.restype = i32
        lib.lso_upwind_steps.argtypes = [vp, vp, i32, i32, i32, dbl, dbl, i32, i32, i32, vp, i64, i32]
        lib.lso_upwind_steps_stored.restype = i32
        lib.lso_upwind_steps_stored.argtypes = [vp, vp, i32, i32, i32, dbl, dbl, i32, i32, i32, vp,
                                                i64, i32, dbl]
        lib.lso_set_threads.restype = None
        lib.lso_set_threads.argtypes = [i32]
        lib.lso_round_binary16.restype = None
        lib.lso_round_binary16.argtypes = [vp, vp, i64]
        _LIB = lib
    return _LIB


def max_threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(_lib().lso_max_threads())


def set_threads(n):
    """Sets the OpenMP threads of the oracle's parallel loops (n >= 1)."""
    _lib().lso_set_threads(int(n))


def round_binary16(x):
    """x (float64) rounded to the nearest IEEE binary16 value, ties to even,
    as an FP64 array (the rounding of the scaled-FP16 storage)."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(a)
    _lib().lso_round_binary16(a.ctypes.data, out.ctypes.data, int(a.size))
    return out


def store_f16s(v, scale):
    """The value scaled-FP16 storage holds for v: fl32(fp16(v / s) * s), s the
    FP32 scale promoted exactly."""
    s = np.float64(np.float32(scale))
    return (round_binary16(np.asarray(v, np.float64) / s) * s).astype(np.float32).astype(
        np.float64)


def _dims(a):
    """Array shape (nz, ny, nx) -> (nx, ny, nz); x is the fastest axis."""
    nz, ny, nx = a.shape
    return int(nx), int(ny), int(nz)


def tile_count(dims, tile):
    n = _lib().lso_tile_count(*[int(v) for v in dims], *[int(v) for v in tile])
    if n < 0:
        raise ValueError("bad dims or tile shape")
    return int(n)


def dequant_f16s(h, scale):
    """Scaled-FP16 storage to its FP32 value: fl32(h * s).

    The product of an 11-bit and a 24-bit significand is exact in FP64, so
    rounding it once to FP32 is the correctly rounded FP32 product.
    """
    h = np.asarray(h, dtype=np.float16)
    s = np.float64(np.float32(scale))
    return (h.astype(np.float64) * s).astype(np.float32)


def band_tiles(phi, tile=(8, 8, 8), gamma=0.0, dilate=True):
    """Ascending band tile ids (Eq. 6; dilated by one tile, Eq. 11, if asked).

    ``phi`` is the stored field (float32 or float64, shape (nz, ny, nx)); it is
    promoted exactly to FP64 together with ``gamma`` given in the same
    precision, so the comparison result equals the one made in that precision.
    """
    phi = np.asarray(phi)
    if phi.dtype not in (np.float32, np.float64):
        raise TypeError("phi must be float32 or float64")
    gamma = float(phi.dtype.type(gamma))
    p64 = np.ascontiguousarray(phi, dtype=np.float64)
    nx, ny, nz = _dims(p64)
    cap = tile_count((nx, ny, nz), tile)
    out = np.empty(max(cap, 1), dtype=np.int32)
    n = _lib().lso_band_tiles(p64.ctypes.data, nx, ny, nz, *tile, gamma, int(bool(dilate)),
                              out.ctypes.data, cap)
    if n < 0:
        raise RuntimeError(f"lso_band_tiles failed: {n}")
    return out[:n].copy()


def all_tiles(dims, tile=(8, 8, 8)):
    """Every tile of the grid: the full-grid (no band) update set."""
    return np.arange(tile_count(dims, tile), dtype=np.int32)


def upwind_steps(phi, F, dx, dt, tiles, nsteps, tile=(8, 8, 8), store_scale=None):
    """``nsteps`` Jacobi steps of Eq. 3-5 on the listed tiles, in FP64.

    Returns a new float64 array; ``phi`` and ``F`` are promoted exactly.
    With ``store_scale`` s, every new value (of a point whose F is not zero)
    is rounded to what scaled-FP16 storage holds, fl32(fp16(v / s) * s)
    (``store_f16s``), before the next step reads it.
    Pinned by the plane, F = 0, expanding/shrinking sphere, reflection,
    monotonicity and brute-force tests; the stored form by the binary16
    rounding against numpy's conversion and by the elementwise equality of
    one stored step with the FP64 step rounded afterwards.
    """
    p = np.array(phi, dtype=np.float64, order="C", copy=True)
    f = np.ascontiguousarray(F, dtype=np.float64)
    if f.shape != p.shape:
        raise ValueError("phi and F shapes differ")
    t = np.ascontiguousarray(tiles, dtype=np.int32)
    nx, ny, nz = _dims(p)
    if store_scale is None:
        rc = _lib().lso_upwind_steps(p.ctypes.data, f.ctypes.data, nx, ny, nz, float(dx),
                                     float(dt), *tile, t.ctypes.data if t.size else None,
                                     int(t.size), int(nsteps))
    else:
        s = float(np.float32(store_scale))
        if not s > 0:
            raise ValueError("store_scale must be positive")
        rc = _lib().lso_upwind_steps_stored(p.ctypes.data, f.ctypes.data, nx, ny, nz, float(dx),
                                            float(dt), *tile, t.ctypes.data if t.size else None,
                                            int(t.size), int(nsteps), s)
    if rc != 0:
        raise RuntimeError(f"lso_upwind_steps failed: {rc}")
    return p


def cutoff(phi, beta, gamma):
    """The cut-off function c of Eq. 8: 1 for |phi| <= beta, the cubic
    (|phi| - gamma)^2 (2|phi| + gamma - 3 beta) / (gamma - beta)^3 for
    beta < |phi| <= gamma, 0 beyond (NaN -> 0).

    Pinned by its closed forms (c(beta) = 1, c(gamma) = 0, c = 1/2 midway,
    flat at both ends, non-increasing) and by hand-computed values at the
    points of a plane.
    """
    a = np.abs(np.asarray(phi, dtype=np.float64))
    mid = (a - gamma) ** 2 * (2 * a + gamma - 3 * beta) / (gamma - beta) ** 3
    return np.where(a <= beta, 1.0, np.where(a <= gamma, mid, 0.0))


def cutoff_steps(phi, F, dx, dt, tiles, nsteps, beta, gamma, tile=(8, 8, 8)):
    """``nsteps`` explicit steps of the cut-off equation of Eq. 8,
    phi_t + c(phi) F |grad phi| = 0, with the upwind scheme of Eq. 3-5 on the
    listed tiles, FP64.

    Each step takes the speed c(phi^n) F from the step-n field, then one
    Jacobi step of the plain scheme with that speed.  Pinned by the plane
    closed form, by c = 1 everywhere (the plain steps, bitwise) and by the
    frozen points |phi| >= gamma.
    """
    p = np.array(phi, dtype=np.float64, copy=True)
    f = np.asarray(F, dtype=np.float64)
    for _ in range(int(nsteps)):
        p = upwind_steps(p, cutoff(p, beta, gamma) * f, dx, dt, tiles, 1, tile)
    return p


def tile_mask(dims, tiles, tile=(8, 8, 8)):
    """Boolean (nz, ny, nx) mask of the grid points of the listed tiles."""
    nx, ny, nz = dims
    tx, ty, tz = tile
    ntx, nty = -(-nx // tx), -(-ny // ty)
    m = np.zeros((nz, ny, nx), dtype=bool)
    for t in np.asarray(tiles, dtype=np.int64):
        ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        m[tk * tz:(tk + 1) * tz, tj * ty:(tj + 1) * ty, ti * tx:(ti + 1) * tx] = True
    return m


def smoothed_sign(d, dx):
    """S of Eq. 13: d / sqrt(d^2 + |Dd|^2 dx^2), FP64.

    Dd is the central difference (d[i+1] - d[i-1]) / (2 dx) per axis with the
    zero-gradient boundary (an index outside the grid is clamped to it), the
    squares summed x, then y, then z; S = 0 where d = 0.  Pinned by hand
    values on a plane, oddness and |S| < 1.
    """
    d = np.asarray(d, dtype=np.float64)
    g2 = np.zeros_like(d)
    for axis in (2, 1, 0):  # array axes of x, y, z
        n = d.shape[axis]
        up = np.take(d, np.minimum(np.arange(n) + 1, n - 1), axis=axis)
        dn = np.take(d, np.maximum(np.arange(n) - 1, 0), axis=axis)
        g2 = g2 + ((up - dn) / (2 * dx)) ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        s = d / np.sqrt(d ** 2 + g2 * dx ** 2)
    return np.where(d == 0, 0.0, s)


def reinit_steps(d, dx, dtau, tiles, niter, tile=(8, 8, 8), gamma=None):
    """``niter`` pseudo-time steps of the reinitialisation equation of Eq. 12,
    d_tau + S(d) (|grad d| - 1) = 0, on the listed tiles, FP64; then, if
    ``gamma`` is given, the clamp of Eq. 10 to [-gamma, gamma] on them.

    Each step takes S from the current iterate (Eq. 13) and applies the upwind
    scheme of Eq. 3-5 with the speed S to the |grad d| term (one Jacobi step
    of the plain scheme), then adds dtau S for the -1 term.  Points outside
    the tiles keep their values.  Pinned by the distance plane as a fixed
    point, the convergence of a steepened plane to the distance, the sphere's
    front kept in place and the clamp.
    """
    p = np.array(d, dtype=np.float64, copy=True)
    nz, ny, nx = p.shape
    m = tile_mask((nx, ny, nz), tiles, tile)
    for _ in range(int(niter)):
        s = smoothed_sign(p, dx)
        q = upwind_steps(p, s, dx, dtau, tiles, 1, tile)
        p = np.where(m, q + dtau * s, p)
    if gamma is not None:
        p = np.where(m, np.clip(p, -gamma, gamma), p)
    return p


def gather_tiles(phi, tiles, tile=(8, 8, 8)):
    """The band snapshot: the values of the listed tiles, tile by tile in list
    order, each as a (tz, ty, tx) block (x fastest); points of a partial tile
    that lie outside the grid are 0.  The snapshot output of the algorithm in
    Sec. 1.1 (Step 4), restricted to the band.  Keeps the input dtype.
    Pinned by explicit loops on a tiny grid and the scatter round trip.
    """
    phi = np.asarray(phi)
    nz, ny, nx = phi.shape
    tx, ty, tz = tile
    ntx, nty = -(-nx // tx), -(-ny // ty)
    t = np.asarray(tiles, dtype=np.int64)
    out = np.zeros((t.size, tz, ty, tx), dtype=phi.dtype)
    for p, tid in enumerate(t):
        ti, tj, tk = tid % ntx, (tid // ntx) % nty, tid // (ntx * nty)
        blk = phi[tk * tz:(tk + 1) * tz, tj * ty:(tj + 1) * ty, ti * tx:(ti + 1) * tx]
        out[p, :blk.shape[0], :blk.shape[1], :blk.shape[2]] = blk
    return out


def decide_precision(phi64, precision, scale=None):
    """The field on which the band decision is taken, in the kernel's precision.

    Where floating point decides an integer (tile membership), both sides
    decide in the same precision: the FP64 state is rounded to the storage
    precision of the device path first ('f32' -> FP32, 'f64' -> as is,
    'f16s' -> the FP32 value scaled-FP16 storage of it would decode to,
    fl32(fp16(phi / s) * s)).
    """
    if precision == "f64":
        return phi64
    if precision == "f32":
        return phi64.astype(np.float32)
    if precision == "f16s":
        return store_f16s(phi64, scale).astype(np.float32)
    raise ValueError(precision)


def run_band(phi0, F, dx, dt, gamma, nsteps, window=10, tile=(8, 8, 8), precision="f32",
             dilate=True, record_tiles=False, beta=None, reinit=None, scale=None,
             store=False):
    """The narrow-band driver (Steps 1-3 of the algorithm in Sec. 1.1), FP64.

    Every ``window`` steps the band U is rebuilt from the current state
    (decision in ``precision``; 'f16s' needs ``scale``), then the state is
    advanced on U: by the plain steps of Eq. 3-5, or, with ``beta`` given, by
    the cut-off steps of Eq. 8 with the band's gamma.  With ``reinit = (dtau,
    niter)`` the window ends with Step 3: ``niter`` reinitialisation steps
    (Eq. 12-13) on U and the clamp of Eq. 10 to the band's gamma.  With
    ``store`` (plain steps, precision 'f16s') the state is held in scaled FP16
    storage: every step's new values are rounded to it (``upwind_steps`` with
    ``store_scale``), so the run is the FP64 scheme with FP16 stores.
    Returns the final FP64 field and, if asked, the tile list of every window.
    """
    if store and (precision != "f16s" or beta is not None or reinit is not None):
        raise ValueError("stored runs are plain steps with precision 'f16s'")
    phi = np.array(phi0, dtype=np.float64, copy=True)
    lists = []
    done = 0
    while done < nsteps:
        n = min(window, nsteps - done)
        gam = np.float32(gamma) if precision in ("f32", "f16s") else np.float64(gamma)
        tiles = band_tiles(decide_precision(phi, precision, scale), tile, gam, dilate)
        if record_tiles:
            lists.append(tiles)
        if store:
            phi = upwind_steps(phi, F, dx, dt, tiles, n, tile, store_scale=scale)
        elif beta is None:
            phi = upwind_steps(phi, F, dx, dt, tiles, n, tile)
        else:
            phi = cutoff_steps(phi, F, dx, dt, tiles, n, beta, gamma, tile)
        if reinit is not None:
            phi = reinit_steps(phi, dx, reinit[0], tiles, reinit[1], tile, gamma=float(gamma))
        done += n
    return (phi, lists) if record_tiles else phi


def run_full(phi0, F, dx, dt, nsteps, tile=(8, 8, 8)):
    """Full-grid run (every tile updated every step), FP64."""
    phi = np.asarray(phi0, dtype=np.float64)
    nz, ny, nx = phi.shape
    return upwind_steps(phi, F, dx, dt, all_tiles((nx, ny, nz), tile), nsteps, tile)
