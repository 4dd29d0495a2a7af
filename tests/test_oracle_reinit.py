"""Pins of the oracle's reinitialisation (Eq. 12-13) and clamp (Eq. 10), and of
the full narrow-band loop (Steps 1-3 of the algorithm in Sec. 1.1).

Expected values come from hand-computed numbers, from fields whose
reinitialised form is known (a distance plane, a steepened plane, a sphere)
and from the sphere's exact front motion, not from the formulas again.
"""
import numpy as np

import oracle
from paper_1612_04040_amd import workloads as W


def _plane(offset, slope=1.0, shape=(10, 9, 48)):
    nz, ny, nx = shape
    x = np.arange(nx, dtype=np.float64) - offset
    return np.broadcast_to(slope * x[None, None, :], shape).copy()


def test_smoothed_sign_hand_values():
    """On d = x - 20 (dx = 1, central difference 1 inside, 1/2 at the x
    faces): S(d) = d / sqrt(d^2 + 1) inside, d / sqrt(d^2 + 1/4) on a face."""
    d = _plane(20.0)
    s = oracle.smoothed_sign(d, 1.0)
    row = s[3, 4]
    assert row[20] == 0.0                                    # d = 0
    assert abs(row[21] - 0.7071067811865476) < 1e-15         # 1 / sqrt(2)
    assert abs(row[22] - 0.8944271909999159) < 1e-15         # 2 / sqrt(5)
    assert abs(row[19] + 0.7071067811865476) < 1e-15         # odd
    assert abs(row[0] + 0.9996876464081228) < 1e-15          # -20 / sqrt(400.25), face
    assert np.all(np.abs(s) < 1.0)


def test_distance_plane_is_a_fixed_point():
    """A signed distance (|grad d| = 1 for every one-sided difference) does
    not move: S (|grad d| - 1) = 0 at every point, faces included."""
    d = _plane(20.5)
    tiles = oracle.all_tiles((48, 9, 10))
    out = oracle.reinit_steps(d, 1.0, 0.5, tiles, 20)
    assert np.max(np.abs(out - d)) < 1e-13


def test_one_step_hand_values():
    """One step on d = 2 (x - 20.5), dx = 1, dtau = 1/2, worked by hand.  At
    d = 1 (x = 21): central difference 2, so S = 1 / sqrt(1 + 4); the upwind
    side (S > 0) has D- = 2 and D+ = 2 (min(D+, 0) = 0), so |grad d| = 2 and
    d' = 1 - (1/2) S (2 - 1) = 1 - 1/(2 sqrt 5).  At d = 3: S = 3 / sqrt(13),
    d' = 3 - 3/(2 sqrt 13).  At d = -1 the mirror image."""
    d = _plane(20.5, slope=2.0)
    tiles = oracle.all_tiles((48, 9, 10))
    row = oracle.reinit_steps(d, 1.0, 0.5, tiles, 1)[4, 3]
    assert abs(row[21] - 0.7763932022500210) < 1e-15
    assert abs(row[22] - 2.5839748528310782) < 1e-15
    assert abs(row[20] + 0.7763932022500210) < 1e-15


def test_steepened_plane_relaxes_to_the_distance():
    """d = 2 (x - 20.5): the zero set stays between the same points (the
    field near it stays antisymmetric: characteristics leave the front), and
    within 10 points of it the iterate converges to x - 20.5."""
    d = _plane(20.5, slope=2.0)
    tiles = oracle.all_tiles((48, 9, 10))
    out = oracle.reinit_steps(d, 1.0, 0.5, tiles, 80)
    row = out[5, 4]
    assert np.all(np.abs(row[11:31] + row[11:31][::-1]) < 1e-12)
    want = np.arange(48) - 20.5
    assert np.max(np.abs(row[11:31] - want[11:31])) < 1e-6
    # not there after a few steps: the iteration really moves values
    few = oracle.reinit_steps(d, 1.0, 0.5, tiles, 3)[5, 4]
    assert np.max(np.abs(few[11:31] - want[11:31])) > 1.0


def test_sphere_front_kept_and_distance_restored():
    """phi = 3 (|x - c|^2 - r0^2) / (2 r0) has the sphere |x - c| = r0 as zero
    set and gradient ~3 near it.  After reinitialisation the front stays within
    dx / 2 of r0 and the field is within dx of the distance |x - c| - r0 on
    the shell of 4 dx around the front."""
    n, dx, r0 = 48, 1.0 / 48, 0.3
    x = (np.arange(n) + 0.5) * dx
    rr = np.sqrt((x[None, None, :] - 0.5) ** 2 + (x[None, :, None] - 0.5) ** 2
                 + (x[:, None, None] - 0.5) ** 2)
    phi = 3 * (rr ** 2 - r0 ** 2) / (2 * r0)
    tiles = oracle.all_tiles((n, n, n))
    out = oracle.reinit_steps(phi, dx, 0.5 * dx, tiles, 40)
    shell = np.abs(rr - r0) < 4 * dx
    assert np.max(np.abs(out[shell] - (rr - r0)[shell])) < dx
    assert np.max(np.abs(phi[shell] - (rr - r0)[shell])) > 3 * dx  # it was not one
    # zero crossings along the lattice lines through the centre
    line = out[n // 2, n // 2]
    i = np.nonzero(np.diff(np.sign(line)))[0]
    xc = x[i] + dx * line[i] / (line[i] - line[i + 1])
    assert np.all(np.abs(np.abs(xc - 0.5) - r0) < 0.5 * dx)


def test_clamp_on_the_listed_tiles_only():
    n, dx = 32, 1.0 / 32
    d = W.sphere((n, n, n), dx, (0.5, 0.5, 0.5), 0.2) * 1.5
    tiles = oracle.band_tiles(d, (8, 8, 8), 4 * dx, dilate=True)
    gamma = 3 * dx
    out = oracle.reinit_steps(d, dx, 0.5 * dx, tiles, 5, gamma=gamma)
    m = oracle.tile_mask((n, n, n), tiles)
    assert np.all(np.abs(out[m]) <= gamma)
    assert np.any(np.abs(out[m]) == gamma)
    assert np.array_equal(out[~m], d[~m])
    # the clamp changes nothing inside [-gamma, gamma]
    free = oracle.reinit_steps(d, dx, 0.5 * dx, tiles, 5)
    inside = m & (np.abs(free) < gamma)
    assert np.array_equal(out[inside], free[inside])


def test_full_loop_front_moves_at_speed():
    """Steps 1-3 (band, cut-off steps, reinitialisation + clamp) on an
    expanding sphere (F = 1, 64^3, beta = 3 dx, gamma = 6 dx, windows of 10
    steps of dt = dx / 2, 24 reinitialisation steps of dtau = dx / 2): the
    front travels its 20 dx to the Hopf-Lax radius within a grid point, where
    the cut-off steps alone stop at the frozen points."""
    from test_oracle_pins import _crossing_radii

    n, dx, r0 = 64, 1.0 / 64, 0.25
    phi0 = W.sphere((n, n, n), dx, (0.5, 0.5, 0.5), r0)
    F = np.ones_like(phi0)
    out = oracle.run_band(phi0, F, dx, 0.5 * dx, 6 * dx, 40, window=10, precision="f64",
                          beta=3 * dx, reinit=(0.5 * dx, 24))
    r = _crossing_radii(out, dx, (0.5, 0.5, 0.5)) - (r0 + 20 * dx)
    assert r.size > 1000
    assert np.max(np.abs(r)) < dx
    assert abs(np.mean(r)) < 0.75 * dx
