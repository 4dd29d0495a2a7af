"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

None of these re-types the oracle's formula: they check closed forms of the
scheme (a plane is advanced exactly, Eq. 3-5 with a linear field), the
viscosity solution it converges to (the expanding and shrinking sphere), the
F = 0 identity, symmetries, the monotonicity of the scheme under its CFL
condition, and an independent per-point brute force in exact arithmetic.
"""
import decimal
import math

import numpy as np
import pytest

import oracle
from oracle import tiny
from paper_1612_04040_amd import workloads as W

# --------------------------------------------------------------------------
# (a) plane fronts: with phi = g.x - c every one-sided difference equals the
# gradient component, so nabla^+ = nabla^- = |g| and each step lowers phi by
# exactly dt*F*|g| away from the faces.

OBLIQUE = (0.48, -0.6, 0.64)  # unit length, all three components non-zero


@pytest.mark.parametrize("normal", [(1.0, 0.0, 0.0), (0.0, -1.0, 0.0), OBLIQUE, (-0.64, 0.48, -0.6)])
@pytest.mark.parametrize("speed", [0.7, -0.45])
def test_plane_advances_exactly(normal, speed):
    nx, ny, nz = 24, 20, 28
    dx = 1.0 / 32
    dt = 0.4 * dx
    n = 5
    phi0 = W.plane((nz, ny, nx), dx, normal, 0.31)
    F = np.full(phi0.shape, speed)
    out = oracle.run_full(phi0, F, dx, dt, n)
    g = math.sqrt(sum(v * v for v in normal))
    expect = phi0 - n * speed * dt * g
    inner = (slice(n + 1, nz - n - 1), slice(n + 1, ny - n - 1), slice(n + 1, nx - n - 1))
    assert np.max(np.abs(out[inner] - expect[inner])) < 1e-12
    # the front (interpolated zero crossing along the normal) moved F*dt per step
    assert abs((np.mean(out[inner] - phi0[inner])) + n * speed * dt) < 1e-12


def test_plane_one_step_variable_speed():
    """One step with F of both signs and exact zeros: phi - dt*F*|g| off the faces."""
    rng = np.random.default_rng(11)
    nx, ny, nz = 17, 13, 11
    dx = 0.05
    dt = 0.3 * dx
    phi0 = W.plane((nz, ny, nx), dx, (-0.36, 0.48, 0.8), -0.2)
    F = rng.uniform(-1, 1, size=phi0.shape)
    F[rng.random(phi0.shape) < 0.2] = 0.0
    out = oracle.run_full(phi0, F, dx, dt, 1, tile=(4, 4, 4))
    expect = phi0 - dt * F * 1.0
    inner = (slice(1, -1),) * 3
    assert np.max(np.abs(out[inner] - expect[inner])) < 1e-13
    assert np.array_equal(out[F == 0], phi0[F == 0])


def test_plane_front_in_band_window():
    """Band mode: a plane front x = x0 in 8^3 tiles, F = 1, one 10-step window.

    A point whose 10-step domain of dependence stays inside the updated tiles
    moves exactly like the full-grid plane.
    """
    n = 64
    dx = 1.0 / n
    dt = 0.5 * dx
    phi0 = W.plane((n, n, n), dx, (1.0, 0.0, 0.0), 0.4)
    F = np.ones_like(phi0)
    gamma = 6 * dx
    tiles = oracle.band_tiles(phi0, (8, 8, 8), gamma, dilate=True)
    out = oracle.upwind_steps(phi0, F, dx, dt, tiles, 10)
    # band: |x - 0.4| < 6dx -> i in [19, 31] -> tile columns 2, 3 -> U columns 1..4
    cols = sorted(set(int(t) % 8 for t in tiles))
    assert cols == [1, 2, 3, 4]
    # points with i in [8+10, 40-10) have their whole domain of dependence in U
    sl = (slice(None), slice(None), slice(18, 30))
    assert np.max(np.abs(out[sl] - (phi0[sl] - 10 * dt))) < 1e-12
    # points outside U never change
    assert np.array_equal(out[:, :, :8], phi0[:, :, :8])
    assert np.array_equal(out[:, :, 40:], phi0[:, :, 40:])


# --------------------------------------------------------------------------
# (b) F = 0 leaves phi bit-unchanged (max(F,0) = min(F,0) = 0 in Eq. 3)


def test_zero_speed_is_bitwise_identity():
    rng = np.random.default_rng(5)
    shape = (9, 11, 13)
    phi = rng.standard_normal(shape)
    phi.flat[::7] = 0.0
    phi.flat[1::7] = -0.0
    phi.flat[2::11] = 5e-324  # subnormal
    phi.flat[3::11] = -1e-310
    F = np.zeros(shape)
    F.flat[::2] = -0.0
    tiles = oracle.all_tiles((13, 11, 9), (4, 4, 4))
    out = oracle.upwind_steps(phi, F, 0.1, 0.05, tiles, 7, tile=(4, 4, 4))
    assert out.tobytes() == phi.tobytes()


# --------------------------------------------------------------------------
# (c) expanding / shrinking sphere: the viscosity solution of
# phi_t + F|grad phi| = 0 with phi0 = |x-c| - r0 and constant F has its zero
# set at radius r0 + F t (Hopf-Lax formula), so the computed front must track
# it to O(dx) with first-order convergence.


def _crossing_radii(phi, dx, center):
    """Radii of the linearly interpolated zero crossings on grid edges."""
    radii = []
    for arr_axis in range(3):  # array axes (z, y, x)
        n = phi.shape[arr_axis]
        lo = np.take(phi, np.arange(n - 1), axis=arr_axis)
        hi = np.take(phi, np.arange(1, n), axis=arr_axis)
        hit = (lo < 0) != (hi < 0)
        idx = np.nonzero(hit)
        t = lo[idx] / (lo[idx] - hi[idx])
        pos = [(idx[d] + 0.5) * dx for d in range(3)]
        pos[arr_axis] = pos[arr_axis] + t * dx
        z, y, x = pos
        radii.append(np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2))
    return np.concatenate(radii)


def _sphere_error(n, speed, r0=0.25, t=25.0 / 64):
    dx = 1.0 / n
    dt = 0.5 * dx
    steps = int(round(t / dt))
    phi0 = W.sphere((n, n, n), dx, (0.5, 0.5, 0.5), r0)
    F = np.full(phi0.shape, speed)
    out = oracle.run_full(phi0, F, dx, dt, steps)
    r = _crossing_radii(out, dx, (0.5, 0.5, 0.5))
    return r - (r0 + speed * steps * dt), dx


def test_sphere_expands_at_speed():
    err, dx = _sphere_error(64, 1.0)
    assert err.size > 1000
    assert np.max(np.abs(err)) <= 1.5 * dx


def test_sphere_shrinks_at_speed():
    err, dx = _sphere_error(64, -1.0, r0=0.45, t=20.0 / 64)
    assert err.size > 1000
    assert np.max(np.abs(err)) <= 1.5 * dx


@pytest.mark.slow
def test_sphere_first_order_convergence():
    e64, _ = _sphere_error(64, 1.0)
    e128, _ = _sphere_error(128, 1.0)
    order = math.log2(np.mean(np.abs(e64)) / np.mean(np.abs(e128)))
    assert 0.7 <= order <= 1.3, order


# --------------------------------------------------------------------------
# invariants


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_reflection_is_bitwise(axis):
    """Mirroring the grid commutes with the scheme, bit for bit (each axis
    contributes a^2 + b^2 and the pair order swaps under reflection)."""
    rng = np.random.default_rng(7 + axis)
    shape = (12, 16, 16)
    phi = rng.standard_normal(shape)
    F = rng.uniform(-1, 1, shape)
    dx, dt = 0.1, 0.02
    a = oracle.run_full(phi, F, dx, dt, 3, tile=(4, 4, 4))
    b = oracle.run_full(np.flip(phi, axis), np.flip(F, axis), dx, dt, 3, tile=(4, 4, 4))
    assert np.flip(b, axis).tobytes() == a.tobytes()


def test_monotone_under_cfl():
    """phi <= psi pointwise implies S(phi) <= S(psi) when dt*max|F|*3/dx <= 1."""
    rng = np.random.default_rng(9)
    shape = (10, 10, 10)
    dx = 0.1
    F = rng.uniform(-1, 1, shape)
    dt = dx / 3.0 / np.max(np.abs(F)) * 0.99
    for trial in range(5):
        phi = rng.standard_normal(shape)
        psi = phi + rng.uniform(0, 0.5, shape)
        a = oracle.run_full(phi, F, dx, dt, 1, tile=(5, 5, 5))
        b = oracle.run_full(psi, F, dx, dt, 1, tile=(5, 5, 5))
        assert np.all(a <= b + 1e-15)


# --------------------------------------------------------------------------
# (d) brute force on tiny grids: pure-Python floats (same IEEE rounding,
# bit for bit) and 50-digit decimals (the exact value, within a few ulp)

TINY = [(1, 1, 1), (5, 3, 2), (13, 9, 7), (8, 8, 8), (9, 9, 9)]


def _ulp(v):
    return np.spacing(np.abs(v))


@pytest.mark.parametrize("dims", TINY)
@pytest.mark.parametrize("nsteps", [1, 3])
def test_bruteforce_tiny(dims, nsteps):
    nx, ny, nz = dims
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz + nsteps)
    phi = rng.standard_normal((nz, ny, nx))
    F = rng.uniform(-1, 1, (nz, ny, nx))
    F[rng.random(F.shape) < 0.15] = 0.0
    dx, dt = 0.125, 0.03
    tile = (4, 3, 2)
    ntiles = oracle.tile_count(dims, tile)
    tiles = np.sort(rng.choice(ntiles, size=max(1, ntiles * 2 // 3), replace=False)).astype(np.int32)
    got = oracle.upwind_steps(phi, F, dx, dt, tiles, nsteps, tile=tile)
    ref_f = np.array(tiny.steps(phi.tolist(), F.tolist(), dx, dt, tiles.tolist(), tile, nsteps))
    assert got.tobytes() == ref_f.tobytes()
    ref_d = tiny.steps(phi.tolist(), F.tolist(), dx, dt, tiles.tolist(), tile, nsteps, exact=True)
    ref_d = np.array([[[float(v) for v in row] for row in plane] for plane in ref_d])
    tol = 4 * nsteps * _ulp(np.maximum(np.abs(ref_d), np.abs(phi)))
    assert np.all(np.abs(got - ref_d) <= tol)


def test_decimal_context_is_50_digits():
    assert tiny._CTX.prec == 50
    assert tiny._Dec.sqrt(decimal.Decimal(2)) == decimal.Decimal(2).sqrt(tiny._CTX)
