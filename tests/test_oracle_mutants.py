"""The pins must catch plausible mistakes in the oracle.

Each case compiles a copy of the oracle's C source with one planted mistake
(a dropped term, a wrong sign, a wrong or transposed index, the wrong upwind
branch, a non-strict band test, a short dilation, a lost F = 0 guard, a binary16
rounding with ties away from zero, an extra fraction bit or no subnormal
floor, a stored point of zero speed rounded again) into a
temporary library, swaps it in, and requires at least one pin to fail.
Everything runs on the CPU.
"""
import os

import pytest

import oracle
from oracle import build as obuild

import test_oracle_band as band_pins
import test_oracle_f16s as f16_pins
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(obuild.__file__), "ls_oracle.c")

MUTANTS = {
    "drop_min_term_eq4": ("sq(maxd(dmx, 0.0)) + sq(mind(dpx, 0.0))", "sq(maxd(dmx, 0.0))"),
    "wrong_sign_update": ("return c - dt * f * grad_plus;", "return c + dt * f * grad_plus;"),
    "wrong_index_ym": ("clampi(j - 1, 0, ny - 1)", "clampi(j + 1, 0, ny - 1)"),
    "transposed_axis": ("const double dmy = (c - ym) / dx", "const double dmy = (c - zm) / dx"),
    "upwind_branch_swapped": ("if (f > 0.0) {", "if (f < 0.0) {"),
    "max_instead_of_min_eq5": ("sq(maxd(dpz, 0.0)) + sq(mind(dmz, 0.0))", "sq(maxd(dpz, 0.0)) + sq(maxd(dmz, 0.0))"),
    "periodic_not_neumann": ("clampi(i + 1, 0, nx - 1)", "((i + 1) % nx)"),
    "lost_zero_speed_guard": ("if (f == 0.0)\n        return c;", "if (0)\n        return c;"),
    "band_not_strict": ("if (fabs(v) < gamma)", "if (fabs(v) <= gamma)"),
    "dilation_one_sided": ("for (int64_t dk = -1; dk <= 1; ++dk)", "for (int64_t dk = 0; dk <= 1; ++dk)"),
    "gauss_seidel": ("nxt[idx] = v;", "nxt[idx] = v;\n                        phi[idx] = v;"),
    "binary16_ties_away": ("nearbyint(ldexp(a, -q))", "round(ldexp(a, -q))"),
    "binary16_extra_bit": ("int q = e - 11;", "int q = e - 12;"),
    "binary16_no_subnormal_floor": ("if (q < -24)", "if (q < -34)"),
    "stored_zero_speed_rounded": ("if (store_scale > 0.0 && F[idx] != 0.0)", "if (store_scale > 0.0)"),
}


def _pins():
    """Every pin, as (name, callable)."""
    out = []
    for normal in [(1.0, 0.0, 0.0), pins.OBLIQUE]:
        for speed in (0.7, -0.45):
            out.append((f"plane{normal}{speed}", lambda n=normal, s=speed: pins.test_plane_advances_exactly(n, s)))
    out.append(("plane_var", pins.test_plane_one_step_variable_speed))
    out.append(("plane_band", pins.test_plane_front_in_band_window))
    out.append(("zero_speed", pins.test_zero_speed_is_bitwise_identity))
    out.append(("sphere_grow", pins.test_sphere_expands_at_speed))
    out.append(("sphere_shrink", pins.test_sphere_shrinks_at_speed))
    for dims in pins.TINY[1:3]:
        out.append((f"brute{dims}", lambda d=dims: pins.test_bruteforce_tiny(d, 1)))
    for tile in [(8, 8, 8), (4, 3, 2)]:
        out.append((f"band_brute{tile}", lambda t=tile: band_pins.test_band_bruteforce((13, 9, 7), t, True)))
        out.append((f"band_brute_a{tile}", lambda t=tile: band_pins.test_band_bruteforce((13, 9, 7), t, False)))
    out.append(("band_plane", lambda: band_pins.test_plane_band_closed_form(0.4, (8, 8, 8))))
    out.append(("band_f32", band_pins.test_band_f32_decision_matches_f32_compare))
    out.append(("binary16", f16_pins.test_round_binary16_equals_numpy_conversion))
    out.append(("stored_steps", f16_pins.test_stored_steps_compose_and_round_each_step))
    return out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    before, after = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(before) == 1, f"mutation anchor for {name} not unique"
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(src.replace(before, after))
    lib = obuild.compile_library([str(mutant_src)], str(tmp_path / "libmutant.so"))
    caught = []
    old = oracle.use_library(lib)
    try:
        for pin_name, pin in _pins():
            try:
                pin()
            except (AssertionError, RuntimeError, ValueError):
                caught.append(pin_name)
    finally:
        oracle.use_library(old)
    assert caught, f"no pin caught the planted mistake {name}"


def test_unmutated_oracle_passes_every_pin():
    for _, pin in _pins():
        pin()
