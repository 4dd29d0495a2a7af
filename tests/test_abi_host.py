"""Host-side checks of the C-ABI (no GPU needed).

The library loads and exports every entry point include/ls.h declares, and
every argument error is reported with a negative status and a message before
anything is launched (so these calls never touch a device).
"""
import ctypes
import os
import re

import pytest

from paper_1612_04040_amd import ls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ls.h")

FAKE = 0x10000  # never dereferenced: every call below fails its host checks first


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_bound_symbols():
    assert declared_symbols() == ls.exported_symbols()


def test_binding_wraps_every_declared_symbol():
    for name in declared_symbols():
        assert callable(getattr(ls, name, None)), name


def test_library_exports_every_declared_symbol():
    handle = ctypes.CDLL(ls.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(handle, name), name


def test_version_and_tiles():
    assert "gfx950" in ls.ls_version()
    g = ls.grid((512, 512, 512))
    assert ls.ls_grid_tiles(g) == 64 ** 3
    assert ls.ls_grid_tiles(ls.grid((17, 9, 8), (8, 4, 3))) == 3 * 3 * 3
    assert ls.ls_workspace_bytes(g) >= 6 * 64 ** 3


def _status(fn, *args):
    with pytest.raises(ls.LsError) as e:
        fn(*args)
    assert e.value.message
    return e.value.status


def test_grid_errors():
    assert _status(ls.ls_grid_tiles, ls.grid((0, 4, 4))) == ls.LS_ERR_ARG
    assert _status(ls.ls_grid_tiles, ls.grid((4, 4, 4), (8, 0, 8))) == ls.LS_ERR_ARG
    assert _status(ls.ls_workspace_bytes, ls.grid((-1, 4, 4))) == ls.LS_ERR_ARG
    assert "positive" in ls.ls_last_error()
    assert ls.lib().ls_grid_tiles(None) == ls.LS_ERR_ARG
    assert _status(ls.ls_grid_tiles, ls.grid((1 << 30, 1 << 30, 4), (1, 1, 1))) == \
        ls.LS_ERR_UNSUPPORTED


def _band_args(g0, **over):
    g = g0
    cap = ls.ls_grid_tiles(g)
    a = dict(phi=FAKE, g=g, gamma=0.1, dilate=1, tiles=FAKE, capacity=cap, ntiles_dev=FAKE,
             workspace=FAKE * 256, workspace_bytes=ls.ls_workspace_bytes(g), stream=0)
    a.update(over)
    return a


@pytest.mark.parametrize("fn", ["f32", "f64"])
def test_band_build_errors(fn):
    build = getattr(ls, f"ls_band_build_{fn}")
    g = ls.grid((64, 64, 64))
    cases = [
        (dict(phi=None), ls.LS_ERR_ARG),
        (dict(tiles=None), ls.LS_ERR_ARG),
        (dict(ntiles_dev=None), ls.LS_ERR_ARG),
        (dict(dilate=2), ls.LS_ERR_ARG),
        (dict(gamma=float("nan")), ls.LS_ERR_ARG),
        (dict(capacity=10), ls.LS_ERR_CAPACITY),
        (dict(workspace=None), ls.LS_ERR_ARG),
        (dict(workspace_bytes=100), ls.LS_ERR_CAPACITY),
        (dict(workspace=FAKE * 256 + 8), ls.LS_ERR_ARG),
        (dict(g=ls.grid((64, 0, 64))), ls.LS_ERR_ARG),
    ]
    for over, status in cases:
        a = _band_args(g, **over)
        assert _status(build, *a.values()) == status, over


def test_band_build_f16s_errors():
    g = ls.grid((32, 32, 32))
    a = _band_args(g)
    args = list(a.values())
    args.insert(1, 0.0)  # scale
    assert _status(ls.ls_band_build_f16s, *args) == ls.LS_ERR_ARG
    args[1] = float("inf")
    assert _status(ls.ls_band_build_f16s, *args) == ls.LS_ERR_ARG


def _step_args(g0, **over):
    g = g0
    a = dict(phi=FAKE, F=FAKE, g=g, dx=0.01, dt=0.005, tiles=FAKE, ntiles_dev=FAKE, nsteps=3,
             scratch=FAKE * 2, workspace=FAKE * 256, workspace_bytes=ls.ls_workspace_bytes(g),
             stream=0)
    a.update(over)
    return a


@pytest.mark.parametrize("fn", ["f32", "f64"])
def test_step_errors(fn):
    step = getattr(ls, f"ls_upwind_step_{fn}")
    g = ls.grid((64, 64, 64))
    cases = [
        (dict(phi=None), ls.LS_ERR_ARG),
        (dict(F=None), ls.LS_ERR_ARG),
        (dict(tiles=None), ls.LS_ERR_ARG),
        (dict(scratch=None), ls.LS_ERR_ARG),
        (dict(scratch=FAKE), ls.LS_ERR_ARG),  # aliases phi
        (dict(nsteps=-1), ls.LS_ERR_ARG),
        (dict(dx=0.0), ls.LS_ERR_ARG),
        (dict(dx=float("inf")), ls.LS_ERR_ARG),
        (dict(dt=-1e-3), ls.LS_ERR_ARG),
        (dict(dt=float("nan")), ls.LS_ERR_ARG),
        (dict(workspace_bytes=1), ls.LS_ERR_CAPACITY),
        (dict(g=ls.grid((64, 64, 64), (512, 8, 8))), ls.LS_ERR_UNSUPPORTED),
        (dict(g=ls.grid((64, 64, 64), (4, 64, 64))), ls.LS_ERR_UNSUPPORTED),
    ]
    for over, status in cases:
        a = _step_args(g, **over)
        if "g" in over:
            a["workspace_bytes"] = ls.ls_workspace_bytes(over["g"])
        assert _status(step, *a.values()) == status, over


def test_step_zero_steps_launches_nothing():
    g = ls.grid((64, 64, 64))
    a = _step_args(g, nsteps=0)
    assert ls.ls_upwind_step_f32(*a.values()) == ls.LS_OK


@pytest.mark.parametrize("fn", ["f32", "f64", "f16s"])
def test_cutoff_errors(fn):
    """The cut-off calls reject beta, gamma outside 0 < beta < gamma < inf on
    the host, after the plain calls' own checks; zero steps launch nothing."""
    g = ls.grid((64, 64, 64))
    step = getattr(ls, f"ls_upwind_step_cutoff_{fn}")
    run = getattr(ls, f"ls_band_run_cutoff_{fn}")
    cap = ls.ls_grid_tiles(g)
    ws = ls.ls_workspace_bytes(g)
    lead = [FAKE, 0.5] if fn == "f16s" else [FAKE]
    for beta, gamma in [(0.0, 0.06), (-0.01, 0.06), (0.06, 0.06), (0.07, 0.06),
                        (0.03, float("inf")), (float("nan"), 0.06), (0.03, float("nan"))]:
        a = lead + [FAKE, g, 0.01, 0.005, beta, gamma, FAKE, FAKE, 3, FAKE * 2, FAKE * 256, ws, 0]
        assert _status(step, *a) == ls.LS_ERR_ARG, (beta, gamma)
        a = lead + [FAKE, g, 0.01, 0.005, beta, gamma, 10, 5, FAKE, cap, FAKE, None, FAKE * 2,
                    FAKE * 256, ws, 0]
        assert _status(run, *a) == ls.LS_ERR_ARG, (beta, gamma)
    a = lead + [None, g, 0.01, 0.005, 0.03, 0.06, FAKE, FAKE, 3, FAKE * 2, FAKE * 256, ws, 0]
    assert _status(step, *a) == ls.LS_ERR_ARG  # F NULL, before the cut-off check
    a = lead + [FAKE, g, 0.01, 0.005, 0.03, 0.06, FAKE, FAKE, 0, FAKE * 2, FAKE * 256, ws, 0]
    assert step(*a) == ls.LS_OK


@pytest.mark.parametrize("fn", ["f32", "f64", "f16s"])
def test_reinit_errors(fn):
    """Reinitialisation calls: bad clamp flag, gamma with the clamp, dtau,
    NULL pointers and negative counts are rejected on the host; zero steps
    launch nothing."""
    g = ls.grid((64, 64, 64))
    step = getattr(ls, f"ls_reinit_step_{fn}")
    run = getattr(ls, f"ls_band_run_reinit_{fn}")
    cap = ls.ls_grid_tiles(g)
    ws = ls.ls_workspace_bytes(g)
    lead = [FAKE, 0.5] if fn == "f16s" else [FAKE]

    def step_args(**o):
        a = dict(g=g, dx=0.01, dtau=0.005, gamma=0.06, clamp=1, tiles=FAKE, n=FAKE, niter=3,
                 scratch=FAKE * 2, ws=FAKE * 256, wsb=ws, stream=0)
        a.update(o)
        return lead + list(a.values())

    for over in [dict(clamp=2), dict(clamp=-1), dict(gamma=0.0), dict(gamma=float("inf")),
                 dict(dtau=float("nan")), dict(dtau=-1.0), dict(dx=0.0), dict(niter=-1),
                 dict(tiles=None), dict(scratch=None), dict(scratch=FAKE)]:
        assert _status(step, *step_args(**over)) == ls.LS_ERR_ARG, over
    assert step(*step_args(gamma=0.0, clamp=0, niter=0)) == ls.LS_OK
    assert step(*step_args(niter=0)) == ls.LS_OK

    def run_args(**o):
        a = dict(F=FAKE, g=g, dx=0.01, dt=0.005, beta=0.03, gamma=0.06, dtau=0.005, iters=4,
                 nsteps=10, window=5, tiles=FAKE, cap=cap, n=FAKE, acc=None, scratch=FAKE * 2,
                 ws=FAKE * 256, wsb=ws, stream=0)
        a.update(o)
        return lead + list(a.values())

    for over in [dict(iters=-1), dict(dtau=float("nan")), dict(dtau=-0.1), dict(beta=0.07),
                 dict(F=None), dict(window=0)]:
        assert _status(run, *run_args(**over)) == ls.LS_ERR_ARG, over
    assert _status(run, *run_args(cap=cap - 1)) == ls.LS_ERR_CAPACITY


@pytest.mark.parametrize("fn", ["f32", "f64", "f16s"])
def test_gather_errors(fn):
    g = ls.grid((40, 24, 16))
    cap = ls.ls_grid_tiles(g)
    gather = getattr(ls, f"ls_band_gather_{fn}")
    base = dict(phi=FAKE, g=g, tiles=FAKE, n=FAKE, out=FAKE * 2, ids=None, cap=cap, stream=0)
    for over in [dict(phi=None), dict(tiles=None), dict(n=None), dict(out=None),
                 dict(cap=-1), dict(cap=cap + 1), dict(g=ls.grid((40, 24, 0)))]:
        a = dict(base)
        a.update(over)
        assert _status(gather, *a.values()) == ls.LS_ERR_ARG, over
    a = dict(base)
    a.update(cap=0)
    assert gather(*a.values()) == ls.LS_OK


def test_run_errors():
    g = ls.grid((32, 32, 32))
    cap = ls.ls_grid_tiles(g)
    ws = ls.ls_workspace_bytes(g)
    base = [FAKE, FAKE, g, 0.1, 0.05, 0.2, 10, 0, FAKE, cap, FAKE, None, FAKE * 2, FAKE * 256, ws,
            0]
    assert _status(ls.ls_band_run_f32, *base) == ls.LS_ERR_ARG  # window 0
    bad = list(base)
    bad[6] = -5
    bad[7] = 10
    assert _status(ls.ls_band_run_f32, *bad) == ls.LS_ERR_ARG  # nsteps < 0
    bad = list(base)
    bad[7] = 10
    bad[9] = cap - 1
    assert _status(ls.ls_band_run_f32, *bad) == ls.LS_ERR_CAPACITY
    bad[9] = cap
    bad[5] = float("nan")
    assert _status(ls.ls_band_run_f32, *bad) == ls.LS_ERR_ARG


def test_rebuild_errors():
    g = ls.grid((32, 32, 32))
    cap = ls.ls_grid_tiles(g)
    ws = ls.ls_workspace_bytes(g)
    base = [FAKE, g, 0.1, FAKE * 3, FAKE * 4, FAKE * 5, cap, FAKE * 6, FAKE * 256, ws, 0]
    for i, status in [(3, ls.LS_ERR_ARG), (4, ls.LS_ERR_ARG), (5, ls.LS_ERR_ARG)]:
        bad = list(base)
        bad[i] = None
        assert _status(ls.ls_band_rebuild_f32, *bad) == status
    bad = list(base)
    bad[3] = bad[5]  # previous list aliases the new one
    assert _status(ls.ls_band_rebuild_f32, *bad) == ls.LS_ERR_ARG
    bad = list(base)
    bad[6] = 3
    assert _status(ls.ls_band_rebuild_f32, *bad) == ls.LS_ERR_CAPACITY


def test_batch_layout_host():
    """Layout: grids ordered by tile shape, tile bases cumulative; errors."""
    items = [((20, 20, 20), (16, 4, 4), 0, 0.05, 0.02, 0.3),
             ((17, 9, 8), (8, 8, 8), 8000, 0.05, 0.02, 0.3),
             ((33, 33, 33), (16, 4, 4), 9280, 0.03, 0.01, 0.2)]
    inst = ls.instances(items)
    base, total = ls.ls_batch_layout(inst, 3)
    t = [ls.ls_grid_tiles(ls.grid(d, tl)) for d, tl, *_ in items]
    assert total == sum(t)
    # 8x8x8 sorts before 16x4x4: grid 1 first, then grids 0 and 2 in order
    assert base == [t[1], 0, t[1] + t[0]]
    assert ls.ls_batch_workspace_bytes(inst, 3) > 0
    bad = ls.instances([items[0], (items[1][0], items[1][1], 10, 0.05, 0.02, 0.3)])
    with pytest.raises(ls.LsError):  # overlapping grids
        ls.ls_batch_layout(bad, 2)
    bad = ls.instances([((20, 20, 20), (5, 3, 2), 0, 0.05, 0.02, 0.3)])
    with pytest.raises(ls.LsError) as e:  # no batched kernel for this shape
        ls.ls_batch_layout(bad, 1)
    assert e.value.status == ls.LS_ERR_UNSUPPORTED
    assert ls.lib().ls_graph_begin(None) == ls.LS_ERR_ARG


def test_batch_pitch_host():
    """Row pitch: a grid spans pitch * ny * nz elements (overlap checks use
    that span); a pitch below nx is rejected; 0 means dense rows."""
    dense = ls.instances([((20, 20, 20), (8, 8, 8), 0, 0.05, 0.02, 0.3),
                          ((20, 20, 20), (8, 8, 8), 8000, 0.05, 0.02, 0.3)])
    assert ls.ls_batch_layout(dense, 2)[1] == 2 * 27
    # pitch 32: grid 0 spans 32 * 400 = 12800 elements, so grid 1 at 8000 overlaps
    over = ls.instances([((20, 20, 20), (8, 8, 8), 0, 0.05, 0.02, 0.3, 32),
                         ((20, 20, 20), (8, 8, 8), 8000, 0.05, 0.02, 0.3, 32)])
    with pytest.raises(ls.LsError) as e:
        ls.ls_batch_layout(over, 2)
    assert e.value.status == ls.LS_ERR_ARG
    ok = ls.instances([((20, 20, 20), (8, 8, 8), 0, 0.05, 0.02, 0.3, 32),
                       ((20, 20, 20), (8, 8, 8), 12800, 0.05, 0.02, 0.3, 32)])
    assert ls.ls_batch_layout(ok, 2)[1] == 2 * 27
    small = ls.instances([((20, 20, 20), (8, 8, 8), 0, 0.05, 0.02, 0.3, 19)])
    with pytest.raises(ls.LsError) as e:
        ls.ls_batch_layout(small, 1)
    assert e.value.status == ls.LS_ERR_ARG and "pitch" in str(e.value)


def test_closure_parameter_layout_and_cases():
    """The flat parameter vector holds the layers in the documented order and
    the library agrees on its length; closure problems are deterministic and
    their speed bound covers every sample."""
    import numpy as np
    from oracle import closure as CL
    from paper_1612_04040_amd import closure as C
    from paper_1612_04040_amd import workloads as W

    assert ls.ls_closure_param_count() == C.NPARAMS == 8673
    p = CL.init_params(np.random.default_rng(0), scale=0.5)
    back = C.unflatten(C.flatten(p))
    for k, shape in C.PARAM_SHAPES:
        assert back[k].shape == shape
        assert np.array_equal(back[k], p[k].astype(np.float32))
    a, b = W.ClosureCase(7, n_fine=64), W.ClosureCase(7, n_fine=64)
    assert np.array_equal(a.phi(16), b.phi(16))
    assert float(np.max(np.abs(a.F(64)))) <= a.fmax
    assert a.dt_coarse == 4 * a.dt_fine
    g = ls.grid((64, 64, 64))
    assert ls.ls_closure_workspace_bytes(g) > 0
    with pytest.raises(ls.LsError):
        ls.ls_closure_workspace_bytes(ls.grid((60, 64, 64)))


def test_closure_run_errors():
    """Argument errors of the corrected driver come from the host checks,
    before any device call (so they hold without a GPU)."""
    g = ls.grid((32, 32, 32))
    cap = ls.ls_grid_tiles(g)
    ws, cws = ls.ls_workspace_bytes(g), ls.ls_closure_workspace_bytes(g)

    def call(**over):
        a = dict(phi=FAKE, F=FAKE, g=g, dx=0.1, dt=0.05, gamma=0.3, fmax=1.0, params=FAKE,
                 nsteps=10, window=10, judge=1, tiles=FAKE, capacity=cap, ntiles_dev=FAKE,
                 fallbacks_dev=FAKE, resets_dev=FAKE, ws=FAKE * 256, ws_bytes=ws, cws=FAKE * 512,
                 cws_bytes=cws, stream=0)
        a.update(over)
        return _status(ls.ls_closure_run_f32, *a.values())

    assert call(resets_dev=None) == ls.LS_ERR_ARG  # the judge needs its counter
    assert call(fallbacks_dev=None) == ls.LS_ERR_ARG
    assert call(phi=None) == ls.LS_ERR_ARG
    assert call(nsteps=-1) == ls.LS_ERR_ARG
    assert call(window=0) == ls.LS_ERR_ARG
    assert call(capacity=cap - 1) == ls.LS_ERR_CAPACITY
    assert call(g=ls.grid((36, 32, 32))) == ls.LS_ERR_UNSUPPORTED  # dims must be multiples of 8


def test_copy_counted_errors():
    ok = dict(dst=FAKE, src=FAKE, count_dev=FAKE, unit_bytes=16, max_units=4, count_out=None,
              blocks=1, stream=0)
    for over in (dict(dst=None), dict(src=None), dict(count_dev=None), dict(unit_bytes=0),
                 dict(unit_bytes=-4), dict(max_units=-1), dict(max_units=1 << 31),
                 dict(blocks=-1), dict(unit_bytes=1 << 40, max_units=1 << 30)):
        a = dict(ok, **over)
        assert _status(ls.ls_copy_counted, *a.values()) == ls.LS_ERR_ARG, over


def test_copy_counted_from_errors():
    ok = dict(dst=FAKE, src=FAKE, count_dev=FAKE, unit_bytes=16, first_unit=0, max_units=4,
              count_out=None, blocks=1, stream=0)
    for over in (dict(dst=None), dict(src=None), dict(count_dev=None), dict(unit_bytes=0),
                 dict(max_units=-1), dict(max_units=1 << 31), dict(blocks=-1),
                 dict(first_unit=-1), dict(first_unit=5), dict(unit_bytes=1 << 40, max_units=1 << 30)):
        a = dict(ok, **over)
        assert _status(ls.ls_copy_counted_from, *a.values()) == ls.LS_ERR_ARG, over


def test_band_build_noalloc_errors():
    """The allocation-free build rejects bad arguments and grids whose
    workspace exceeds its fixed array, before touching a device."""
    cap_bytes = ls.ls_band_build_noalloc_max_bytes()
    assert cap_bytes == 16 << 20
    g = ls.grid((64, 64, 64))
    ok = dict(phi=FAKE, g=g, gamma=0.1, dilate=1, tiles=FAKE, capacity=ls.ls_grid_tiles(g),
              ntiles_dev=FAKE, stream=0)
    cases = [
        (dict(phi=None), ls.LS_ERR_ARG),
        (dict(tiles=None), ls.LS_ERR_ARG),
        (dict(ntiles_dev=None), ls.LS_ERR_ARG),
        (dict(dilate=-1), ls.LS_ERR_ARG),
        (dict(gamma=float("nan")), ls.LS_ERR_ARG),
        (dict(capacity=10), ls.LS_ERR_CAPACITY),
        (dict(g=ls.grid((64, 0, 64))), ls.LS_ERR_ARG),
    ]
    for over, status in cases:
        a = dict(ok, **over)
        assert _status(ls.ls_band_build_f32_noalloc, *a.values()) == status, over
    # 512^3 in 8^3 tiles fits the array; 1024^3 does not
    assert ls.ls_workspace_bytes(ls.grid((512, 512, 512))) <= cap_bytes
    big = ls.grid((1024, 1024, 1024))
    assert ls.ls_workspace_bytes(big) > cap_bytes
    a = dict(ok, g=big, capacity=ls.ls_grid_tiles(big))
    assert _status(ls.ls_band_build_f32_noalloc, *a.values()) == ls.LS_ERR_CAPACITY
    assert "fixed" in ls.ls_last_error()


def test_brick_errors():
    """The brick calls reject shapes and arguments they do not take, on the host."""
    g = ls.grid((64, 64, 64))
    cases = [
        (lambda: ls.ls_bricks_from_dense_f32(FAKE, ls.grid((60, 64, 64)), FAKE * 2, 0),
         ls.LS_ERR_UNSUPPORTED),
        (lambda: ls.ls_bricks_from_dense_f32(FAKE, ls.grid((64, 64, 64), (8, 4, 8)), FAKE * 2, 0),
         ls.LS_ERR_UNSUPPORTED),
        (lambda: ls.ls_bricks_to_dense_f32(None, g, FAKE, 0), ls.LS_ERR_ARG),
        (lambda: ls.ls_bricks_to_dense_f16s(FAKE, g, FAKE, 0), ls.LS_ERR_ARG),  # same buffer
        (lambda: ls.ls_bricks_from_dense_f16s(FAKE + 2, g, FAKE * 2, 0), ls.LS_ERR_ARG),
        (lambda: ls.ls_band_build_bricks_f32(FAKE, g, 0.1, 2, FAKE, ls.ls_grid_tiles(g), FAKE,
                                             FAKE * 256, ls.ls_workspace_bytes(g), 0),
         ls.LS_ERR_ARG),
        (lambda: ls.ls_band_build_bricks_f16s(FAKE, 0.0, g, 0.1, 1, FAKE, ls.ls_grid_tiles(g),
                                              FAKE, FAKE * 256, ls.ls_workspace_bytes(g), 0),
         ls.LS_ERR_ARG),
    ]
    run = dict(phi_b=FAKE, F_b=FAKE * 2, g=g, dx=0.01, dt=0.005, gamma=0.06, nsteps=10,
               window=10, beta=0.0, reinit_iters=0, dtau=0.0, tiles=FAKE,
               capacity=ls.ls_grid_tiles(g), ntiles_dev=FAKE, tile_steps_dev=None,
               scratch_b=FAKE * 3, workspace=FAKE * 256,
               workspace_bytes=ls.ls_workspace_bytes(g), stream=0)
    for over, status in [(dict(window=0), ls.LS_ERR_ARG), (dict(beta=0.07), ls.LS_ERR_ARG),
                         (dict(beta=-0.01), ls.LS_ERR_ARG), (dict(scratch_b=FAKE), ls.LS_ERR_ARG),
                         (dict(dx=0.0), ls.LS_ERR_ARG), (dict(capacity=5), ls.LS_ERR_CAPACITY),
                         (dict(workspace_bytes=64), ls.LS_ERR_CAPACITY),
                         (dict(reinit_iters=-1), ls.LS_ERR_ARG),
                         (dict(g=ls.grid((64, 64, 60))), ls.LS_ERR_UNSUPPORTED)]:
        a = dict(run, **over)
        cases.append((lambda a=a: ls.ls_band_run_bricks_f32(*a.values()), status))
    for fn, status in cases:
        with pytest.raises(ls.LsError) as e:
            fn()
        assert e.value.status == status, (e.value.message, status)
        assert e.value.message


def test_closure_run_rejects_unknown_judge_modes():
    g = ls.grid((64, 64, 64))
    for judge in (-1, 4):
        with pytest.raises(ls.LsError) as e:
            ls.ls_closure_run_f32(FAKE, FAKE, g, 0.01, 0.005, 0.06, 1.0, FAKE, 10, 10, judge, FAKE,
                                  ls.ls_grid_tiles(g), FAKE, FAKE, FAKE, FAKE * 256, 1 << 20,
                                  FAKE * 256, 1 << 20, 0)
        assert e.value.status == ls.LS_ERR_ARG
        assert "judge" in e.value.message
