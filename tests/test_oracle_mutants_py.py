"""The pins of the oracle's numpy parts (cut-off, reinitialisation, clamp,
snapshot) must catch plausible mistakes in them.

Each case swaps one oracle function for a copy with a planted mistake (the
cubic's constants exchanged, c taken from the new value, one-sided instead of
central differences, the -1 term with the wrong sign, S frozen at the start,
the clamp left out, a transposed tile block) and requires at least one of the
pins of that function to fail.  Everything runs on the CPU.
"""
import numpy as np
import pytest

import oracle
import test_oracle_cutoff as cut_pins
import test_oracle_reinit as re_pins
import test_oracle_snapshot as snap_pins

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
]


@pytest.mark.parametrize("name,mutant,pins", CASES,
                         ids=[f"{c[0]}-{c[1].__name__}" for c in CASES])
def test_pins_catch_the_mutant(name, mutant, pins, monkeypatch):
    monkeypatch.setattr(oracle, name, mutant)
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
