"""Pins of the oracle's scaled-FP16 storage (the state held as h = fp16(v / s),
rounded to nearest with ties to even, read back as fl32(h * s)).

* The binary16 rounding equals numpy's float64 -> float16 conversion (an
  independent implementation) on values spread over the whole exponent range,
  on exact ties between neighbouring binary16 values, on subnormals, signed
  zeros, overflow and NaN.
* A stored run is its own composition step by step (Jacobi with a store
  after every step), and one stored step is the FP64 step rounded to storage
  point by point, except where F = 0, which keeps the stored bits.
* A plane front with storage still advances by F dt per step, within the
  accumulated half-ulp storage rounding.
"""
import numpy as np
import pytest

import oracle
from paper_1612_04040_amd import workloads as W


def _numpy_binary16(x):
    with np.errstate(over="ignore"):
        return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def test_round_binary16_equals_numpy_conversion():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(20000) * np.exp2(rng.integers(-30, 18, 20000))
    # exact ties: midpoints of consecutive binary16 values, normal and subnormal
    h = rng.integers(0, 0x7bff, 4000, dtype=np.uint16).view(np.float16).astype(np.float64)
    nxt = np.nextafter(h.astype(np.float16), np.float16(np.inf)).astype(np.float64)
    ties = 0.5 * (h + nxt)
    special = np.array([0.0, -0.0, 65504.0, 65519.9, 65520.0, -65520.0, 1e9, 2.0 ** -24,
                        2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -14, 2.0 ** -14 - 2.0 ** -25, 1.0,
                        1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, np.inf, -np.inf])
    for v in (x, ties, -ties, special):
        got = oracle.round_binary16(v)
        want = _numpy_binary16(v)
        assert np.array_equal(got, want), v[got != want][:5]
        assert np.array_equal(np.signbit(got), np.signbit(want))
    assert np.isnan(oracle.round_binary16(np.array([np.nan]))[0])


def test_store_f16s_decodes_to_fp32_of_the_scaled_code():
    s = np.float32(6.0 / 256)
    v = np.linspace(-30 * s, 30 * s, 1001)
    code = (v / np.float64(s)).astype(np.float16)
    want = (code.astype(np.float64) * np.float64(s)).astype(np.float32).astype(np.float64)
    assert np.array_equal(oracle.store_f16s(v, s), want)


def _case(n=24, seed=5):
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    s = np.float32(6 * dx)
    phi = oracle.store_f16s(W.sphere((n, n, n), dx, (0.45, 0.5, 0.55), 0.3), s)
    F = rng.uniform(-1.0, 1.0, (n, n, n))
    F[rng.random((n, n, n)) < 0.1] = 0.0
    tiles = oracle.band_tiles(phi.astype(np.float32), (8, 8, 8), np.float32(6 * dx), True)
    return phi, F, dx, 0.4 * dx, tiles, s


def test_stored_steps_compose_and_round_each_step():
    phi, F, dx, dt, tiles, s = _case()
    two = oracle.upwind_steps(phi, F, dx, dt, tiles, 2, store_scale=s)
    one = oracle.upwind_steps(phi, F, dx, dt, tiles, 1, store_scale=s)
    assert np.array_equal(two, oracle.upwind_steps(one, F, dx, dt, tiles, 1, store_scale=s))
    exact = oracle.upwind_steps(phi, F, dx, dt, tiles, 1)
    m = oracle.tile_mask(phi.shape[::-1], tiles) & (F != 0)
    assert np.array_equal(one[m], oracle.store_f16s(exact[m], s))
    assert np.array_equal(one[~m], phi[~m])  # F = 0 and points outside the band keep their bits
    # storage changes the result (the stored values are not the FP64 ones)
    assert not np.array_equal(one[m], exact[m])
    # a point of zero speed keeps its bits even when they are not a storage value
    raw = phi + 1e-7 * dx * np.random.default_rng(1).standard_normal(phi.shape)
    kept = oracle.upwind_steps(raw, F, dx, dt, tiles, 3, store_scale=s)
    assert np.array_equal(kept[F == 0], raw[F == 0])


@pytest.mark.parametrize("speed", [0.8, -0.6])
def test_stored_plane_advances_within_the_rounding(speed):
    n, steps = 32, 12
    dx = 1.0 / n
    s = np.float32(6 * dx)
    g = np.array([0.6, 0.0, 0.8])
    phi0 = oracle.store_f16s(W.plane((n, n, n), dx, tuple(g), 0.5), s)
    F = np.full((n, n, n), speed)
    dt = 0.5 * dx
    allt = oracle.all_tiles((n, n, n))
    got = oracle.upwind_steps(phi0, F, dx, dt, allt, steps, store_scale=s)
    x = (np.arange(n) + 0.5) * dx
    exact = (g[0] * x[None, None, :] + g[2] * x[:, None, None] - 0.5) - steps * speed * dt
    # away from the inflow faces (domain of dependence), |phi| <= 1/2 there
    k = steps + 1
    inner = (slice(k, n - k), slice(None), slice(k, n - k))
    err = np.abs(got - exact)[inner]
    # each store: half an ulp of fp16(|phi| / s) (|phi| / s < 32: ulp <= 2^-6) plus
    # the FP32 decode; the initial rounding counts as one more step
    half_ulp = 2.0 ** -7 * float(s)
    assert err.max() <= (steps + 1) * (half_ulp + 2.0 ** -23)
    assert err.max() > 0  # the storage rounding is visible
