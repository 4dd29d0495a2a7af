"""The pins of the oracle's numpy parts (cut-off, reinitialisation, clamp,
snapshot, closure features) and of the interface metrics must catch
plausible mistakes in them.

Each case swaps one function for a copy with a planted mistake (the cubic's
constants exchanged, c taken from the new value, one-sided instead of
central differences, the -1 term with the wrong sign, S frozen at the start,
the clamp left out, a transposed tile block, the increment over the fine
spacing, a clip at +-1, F over its sample maximum, a judge that resets a
front moved by exactly its bound, crossings without the
half-cell offset or with the interpolation weight reversed, a one-sided
Hausdorff distance, upsampling without the centre shift) and requires at
least one of the pins of that function to fail.  Everything runs on the CPU.
"""
import numpy as np
import pytest

import oracle
import oracle.closure
import test_metrics_pins as metric_pins
import test_oracle_closure as closure_pins
import test_oracle_cutoff as cut_pins
import test_oracle_reinit as re_pins
import test_oracle_snapshot as snap_pins
from paper_1612_04040_amd import metrics

_cutoff, _smoothed_sign, _reinit_steps = oracle.cutoff, oracle.smoothed_sign, oracle.reinit_steps
_cutoff_steps, _gather = oracle.cutoff_steps, oracle.gather_tiles


def cutoff_swapped(phi, beta, gamma):
    a = np.abs(np.asarray(phi, dtype=np.float64))
    mid = (a - gamma) ** 2 * (2 * a + beta - 3 * gamma) / (gamma - beta) ** 3
    return np.where(a <= beta, 1.0, np.where(a <= gamma, mid, 0.0))


def cutoff_linear(phi, beta, gamma):
    a = np.abs(np.asarray(phi, dtype=np.float64))
    return np.clip((gamma - a) / (gamma - beta), 0.0, 1.0)


def cutoff_steps_new_value(phi, F, dx, dt, tiles, nsteps, beta, gamma, tile=(8, 8, 8)):
    p = np.array(phi, dtype=np.float64, copy=True)
    f = np.asarray(F, dtype=np.float64)
    for _ in range(int(nsteps)):
        plain = oracle.upwind_steps(p, f, dx, dt, tiles, 1, tile)
        p = oracle.upwind_steps(p, _cutoff(plain, beta, gamma) * f, dx, dt, tiles, 1, tile)
    return p


def smoothed_sign_one_sided(d, dx):
    d = np.asarray(d, dtype=np.float64)
    g2 = np.zeros_like(d)
    for axis in (2, 1, 0):
        n = d.shape[axis]
        up = np.take(d, np.minimum(np.arange(n) + 1, n - 1), axis=axis)
        g2 = g2 + ((up - d) / dx) ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        s = d / np.sqrt(d ** 2 + g2 * dx ** 2)
    return np.where(d == 0, 0.0, s)


def smoothed_sign_no_dx(d, dx):
    d = np.asarray(d, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        s = d / np.sqrt(d ** 2 + dx ** 2)
    return np.where(d == 0, 0.0, s)


def reinit_wrong_sign(d, dx, dtau, tiles, niter, tile=(8, 8, 8), gamma=None):
    p = np.array(d, dtype=np.float64, copy=True)
    nz, ny, nx = p.shape
    m = oracle.tile_mask((nx, ny, nz), tiles, tile)
    for _ in range(int(niter)):
        s = _smoothed_sign(p, dx)
        q = oracle.upwind_steps(p, s, dx, dtau, tiles, 1, tile)
        p = np.where(m, q - dtau * s, p)
    if gamma is not None:
        p = np.where(m, np.clip(p, -gamma, gamma), p)
    return p


def reinit_frozen_sign(d, dx, dtau, tiles, niter, tile=(8, 8, 8), gamma=None):
    p = np.array(d, dtype=np.float64, copy=True)
    nz, ny, nx = p.shape
    m = oracle.tile_mask((nx, ny, nz), tiles, tile)
    s0 = np.sign(p)
    for _ in range(int(niter)):
        q = oracle.upwind_steps(p, s0, dx, dtau, tiles, 1, tile)
        p = np.where(m, q + dtau * s0, p)
    if gamma is not None:
        p = np.where(m, np.clip(p, -gamma, gamma), p)
    return p


def reinit_no_clamp(d, dx, dtau, tiles, niter, tile=(8, 8, 8), gamma=None):
    return _reinit_steps(d, dx, dtau, tiles, niter, tile, gamma=None)


def gather_transposed(phi, tiles, tile=(8, 8, 8)):
    out = _gather(phi, tiles, tile)
    return np.ascontiguousarray(np.swapaxes(out, 2, 3)) if tile[0] == tile[1] else out[..., ::-1]


def features_fine_spacing(phi_c, F_c, delta, dx, gamma, fmax):
    c0 = np.clip(np.asarray(phi_c, np.float64) / gamma, -2.0, 2.0)
    c1 = np.asarray(F_c, np.float64) / fmax
    c2 = np.asarray(delta, np.float64) / (dx / 4)
    return np.stack([c0, c1, c2])


def features_clip_one(phi_c, F_c, delta, dx, gamma, fmax):
    c0 = np.clip(np.asarray(phi_c, np.float64) / gamma, -1.0, 1.0)
    c1 = np.asarray(F_c, np.float64) / fmax
    c2 = np.asarray(delta, np.float64) / dx
    return np.stack([c0, c1, c2])


def features_sample_max(phi_c, F_c, delta, dx, gamma, fmax):
    f = np.asarray(F_c, np.float64)
    c0 = np.clip(np.asarray(phi_c, np.float64) / gamma, -2.0, 2.0)
    return np.stack([c0, f / np.max(np.abs(f)), np.asarray(delta, np.float64) / dx])


def crossings_no_offset(phi, dx, origin=0.0):
    return _crossings(phi, dx, origin - 0.5 * dx)


def crossings_reversed_weight(phi, dx, origin=0.0):
    phi = np.asarray(phi, dtype=np.float64)
    pts = []
    for ax in range(3):
        n = phi.shape[ax]
        lo = np.take(phi, np.arange(n - 1), axis=ax)
        hi = np.take(phi, np.arange(1, n), axis=ax)
        idx = np.nonzero((lo < 0) != (hi < 0))
        t = hi[idx] / (hi[idx] - lo[idx])
        pos = [(idx[d] + 0.5) * dx + origin for d in range(3)]
        pos[ax] = pos[ax] + t * dx
        z, y, x = pos
        pts.append(np.stack([x, y, z], axis=1))
    return np.concatenate(pts)


def hausdorff_one_sided(a, b):
    from scipy.spatial import cKDTree
    if len(a) == 0 or len(b) == 0:
        return float("inf") if len(a) != len(b) else 0.0
    return float(cKDTree(b).query(a)[0].max())


def upsample_no_shift(phi_c, factor):
    phi_c = np.asarray(phi_c, dtype=np.float64)
    nz, ny, nx = phi_c.shape

    def coords(n):
        u = (np.arange(n * factor) + 0.5) / factor
        i0 = np.clip(np.floor(u).astype(np.int64), 0, n - 1)
        i1 = np.clip(i0 + 1, 0, n - 1)
        w = np.clip(u - np.floor(u), 0.0, 1.0)
        return i0, i1, w

    x0, x1, wx = coords(nx)
    y0, y1, wy = coords(ny)
    z0, z1, wz = coords(nz)
    t = phi_c[:, :, x0] * (1 - wx) + phi_c[:, :, x1] * wx
    t = t[:, y0, :] * (1 - wy)[None, :, None] + t[:, y1, :] * wy[None, :, None]
    return t[z0] * (1 - wz)[:, None, None] + t[z1] * wz[:, None, None]


_crossings = metrics.zero_crossings

_judge = oracle.closure.judge


def judge_non_strict(phi, shadow, tile=(8, 8, 8), dx=None, tau=0.0):
    """A move of exactly tau dx already resets."""
    return _judge(phi, shadow, tile, dx, tau * (1 - 1e-12) if tau > 0 else tau)


CASES = [
    ("cutoff", cutoff_swapped, [cut_pins.test_cutoff_hand_values]),
    ("cutoff", cutoff_linear, [cut_pins.test_cutoff_hand_values]),
    ("cutoff_steps", cutoff_steps_new_value,
     [lambda: cut_pins.test_plane_step_scaled_by_cutoff(0.8)]),
    ("smoothed_sign", smoothed_sign_one_sided, [re_pins.test_smoothed_sign_hand_values]),
    ("smoothed_sign", smoothed_sign_no_dx, [re_pins.test_smoothed_sign_hand_values]),
    ("reinit_steps", reinit_wrong_sign, [re_pins.test_distance_plane_is_a_fixed_point,
                                         re_pins.test_one_step_hand_values]),
    ("reinit_steps", reinit_frozen_sign, [re_pins.test_one_step_hand_values]),
    ("reinit_steps", reinit_no_clamp, [re_pins.test_clamp_on_the_listed_tiles_only]),
    ("gather_tiles", gather_transposed, [snap_pins.test_gather_matches_explicit_loops,
                                         snap_pins.test_scatter_round_trip]),
    ((oracle.closure, "features"), features_fine_spacing,
     [closure_pins.test_features_hand_values_on_a_plane]),
    ((oracle.closure, "features"), features_clip_one,
     [closure_pins.test_features_hand_values_on_a_plane]),
    ((oracle.closure, "features"), features_sample_max,
     [closure_pins.test_features_hand_values_on_a_plane]),
    ((oracle.closure, "judge"), judge_non_strict,
     [closure_pins.test_judge_front_position_bound]),
    ((metrics, "zero_crossings"), crossings_no_offset,
     [metric_pins.test_plane_crossings_at_known_positions,
      metric_pins.test_oblique_plane_crossings_lie_on_the_plane]),
    ((metrics, "zero_crossings"), crossings_reversed_weight,
     [metric_pins.test_plane_crossings_at_known_positions,
      metric_pins.test_oblique_plane_crossings_lie_on_the_plane]),
    ((metrics, "hausdorff"), hausdorff_one_sided,
     [metric_pins.test_hausdorff_brute_force_and_symmetry]),
    ((metrics, "upsample_trilinear"), upsample_no_shift,
     [metric_pins.test_upsample_trilinear_is_exact_on_a_linear_field,
      metric_pins.test_upsample_trilinear_hand_value]),
]


def _target(name):
    return name if isinstance(name, tuple) else (oracle, name)


def _label(name):
    mod, attr = _target(name)
    return f"{mod.__name__.split('.')[-1]}.{attr}"


@pytest.mark.parametrize("name,mutant,pins", CASES,
                         ids=[f"{_label(c[0])}-{c[1].__name__}" for c in CASES])
def test_pins_catch_the_mutant(name, mutant, pins, monkeypatch):
    mod, attr = _target(name)
    monkeypatch.setattr(mod, attr, mutant)
    failed = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed > 0, f"no pin caught the mutant {mutant.__name__} of {name}"


def test_the_pins_pass_on_the_oracle():
    for _, _, pins in CASES:
        for pin in pins:
            pin()
