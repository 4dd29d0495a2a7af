"""ctypes binding of libls (include/ls.h): argument marshalling only.

Each ``ls_*`` function here has the name and argument order of the C entry
point.  Pointer arguments accept a torch tensor (its ``data_ptr()``), a plain
integer address or None; ``stream`` accepts a torch stream, a raw
hipStream_t integer or None (the current torch stream).  A negative status
raises :class:`LsError` carrying the status and ``ls_last_error()``.

The library must have been built (``python -m paper_1612_04040_amd.build``);
there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libls.so")

LS_OK = 0
LS_ERR_ARG = -1
LS_ERR_CAPACITY = -2
LS_ERR_HIP = -3
LS_ERR_UNSUPPORTED = -4


class LsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libls status {status}: {message}")
        self.status = status
        self.message = message


class ls_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tx", ctypes.c_int32), ("ty", ctypes.c_int32), ("tz", ctypes.c_int32)]


class ls_tuning(ctypes.Structure):
    _fields_ = [("run_width", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("pipeline", ctypes.c_int32), ("vector", ctypes.c_int32),
                ("temporal", ctypes.c_int32)]


class ls_instance(ctypes.Structure):
    _fields_ = [("grid", ls_grid), ("offset", ctypes.c_int64), ("dx", ctypes.c_float),
                ("dt", ctypes.c_float), ("gamma", ctypes.c_float), ("pitch", ctypes.c_int32)]


def instances(items):
    """ctypes array of ls_instance from (dims, tile, offset, dx, dt, gamma[, pitch])
    tuples (pitch 0 or absent: dense rows)."""
    arr = (ls_instance * len(items))()
    for k, it in enumerate(items):
        dims, tile, offset, dx, dt, gamma = it[:6]
        pitch = int(it[6]) if len(it) > 6 else 0
        arr[k] = ls_instance(grid(dims, tile), int(offset), float(dx), float(dt), float(gamma),
                             pitch)
    return arr


def grid(dims, tile=(8, 8, 8)):
    """ls_grid for dims = (nx, ny, nz) and tile = (tx, ty, tz)."""
    nx, ny, nz = (int(v) for v in dims)
    tx, ty, tz = (int(v) for v in tile)
    return ls_grid(nx, ny, nz, tx, ty, tz)


_LIB = None

_I32, _I64, _F32, _F64, _VP = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double,
                               ctypes.c_void_p)
_G = ctypes.POINTER(ls_grid)

_SIGNATURES = {
    "ls_last_error": (ctypes.c_char_p, []),
    "ls_version": (ctypes.c_char_p, []),
    "ls_grid_tiles": (_I64, [_G]),
    "ls_workspace_bytes": (_I64, [_G]),
    "ls_band_build_f32": (_I32, [_VP, _G, _F32, _I32, _VP, _I64, _VP, _VP, _I64, _VP]),
    "ls_band_build_f64": (_I32, [_VP, _G, _F64, _I32, _VP, _I64, _VP, _VP, _I64, _VP]),
    "ls_band_build_f16s": (_I32, [_VP, _F32, _G, _F32, _I32, _VP, _I64, _VP, _VP, _I64, _VP]),
    "ls_bricks_from_dense_f32": (_I32, [_VP, _G, _VP, _VP]),
    "ls_bricks_to_dense_f32": (_I32, [_VP, _G, _VP, _VP]),
    "ls_bricks_from_dense_f16s": (_I32, [_VP, _G, _VP, _VP]),
    "ls_bricks_to_dense_f16s": (_I32, [_VP, _G, _VP, _VP]),
    "ls_band_build_bricks_f32": (_I32, [_VP, _G, _F32, _I32, _VP, _I64, _VP, _VP, _I64, _VP]),
    "ls_band_build_bricks_f16s": (_I32, [_VP, _F32, _G, _F32, _I32, _VP, _I64, _VP, _VP, _I64,
                                         _VP]),
    "ls_band_run_bricks_f32": (_I32, [_VP, _VP, _G, _F32, _F32, _F32, _I32, _I32, _F32, _I32,
                                      _F32, _VP, _I64, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_run_bricks_f16s": (_I32, [_VP, _F32, _VP, _G, _F32, _F32, _F32, _I32, _I32, _F32,
                                       _I32, _F32, _VP, _I64, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_build_noalloc_max_bytes": (_I64, []),
    "ls_band_build_f32_noalloc": (_I32, [_VP, _G, _F32, _I32, _VP, _I64, _VP, _VP]),
    "ls_upwind_step_f32": (_I32, [_VP, _VP, _G, _F32, _F32, _VP, _VP, _I32, _VP, _VP, _I64, _VP]),
    "ls_upwind_step_f64": (_I32, [_VP, _VP, _G, _F64, _F64, _VP, _VP, _I32, _VP, _VP, _I64, _VP]),
    "ls_upwind_step_f16s": (_I32, [_VP, _F32, _VP, _G, _F32, _F32, _VP, _VP, _I32, _VP, _VP, _I64,
                                   _VP]),
    "ls_band_rebuild_f32": (_I32, [_VP, _G, _F32, _VP, _VP, _VP, _I64, _VP, _VP, _I64, _VP]),
    "ls_band_rebuild_f64": (_I32, [_VP, _G, _F64, _VP, _VP, _VP, _I64, _VP, _VP, _I64, _VP]),
    "ls_band_rebuild_f16s": (_I32, [_VP, _F32, _G, _F32, _VP, _VP, _VP, _I64, _VP, _VP, _I64,
                                    _VP]),
    "ls_band_run_f32": (_I32, [_VP, _VP, _G, _F32, _F32, _F32, _I32, _I32, _VP, _I64, _VP, _VP,
                               _VP, _VP, _I64, _VP]),
    "ls_band_run_f64": (_I32, [_VP, _VP, _G, _F64, _F64, _F64, _I32, _I32, _VP, _I64, _VP, _VP,
                               _VP, _VP, _I64, _VP]),
    "ls_band_run_f16s": (_I32, [_VP, _F32, _VP, _G, _F32, _F32, _F32, _I32, _I32, _VP, _I64, _VP,
                                _VP, _VP, _VP, _I64, _VP]),
    "ls_upwind_step_cutoff_f32": (_I32, [_VP, _VP, _G, _F32, _F32, _F32, _F32, _VP, _VP, _I32,
                                         _VP, _VP, _I64, _VP]),
    "ls_upwind_step_cutoff_f64": (_I32, [_VP, _VP, _G, _F64, _F64, _F64, _F64, _VP, _VP, _I32,
                                         _VP, _VP, _I64, _VP]),
    "ls_upwind_step_cutoff_f16s": (_I32, [_VP, _F32, _VP, _G, _F32, _F32, _F32, _F32, _VP, _VP,
                                          _I32, _VP, _VP, _I64, _VP]),
    "ls_band_run_cutoff_f32": (_I32, [_VP, _VP, _G, _F32, _F32, _F32, _F32, _I32, _I32, _VP, _I64,
                                      _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_run_cutoff_f64": (_I32, [_VP, _VP, _G, _F64, _F64, _F64, _F64, _I32, _I32, _VP, _I64,
                                      _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_run_cutoff_f16s": (_I32, [_VP, _F32, _VP, _G, _F32, _F32, _F32, _F32, _I32, _I32,
                                       _VP, _I64, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_reinit_step_f32": (_I32, [_VP, _G, _F32, _F32, _F32, _I32, _VP, _VP, _I32, _VP, _VP, _I64,
                                  _VP]),
    "ls_reinit_step_f64": (_I32, [_VP, _G, _F64, _F64, _F64, _I32, _VP, _VP, _I32, _VP, _VP, _I64,
                                  _VP]),
    "ls_reinit_step_f16s": (_I32, [_VP, _F32, _G, _F32, _F32, _F32, _I32, _VP, _VP, _I32, _VP,
                                   _VP, _I64, _VP]),
    "ls_band_run_reinit_f32": (_I32, [_VP, _VP, _G, _F32, _F32, _F32, _F32, _F32, _I32, _I32,
                                      _I32, _VP, _I64, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_run_reinit_f64": (_I32, [_VP, _VP, _G, _F64, _F64, _F64, _F64, _F64, _I32, _I32,
                                      _I32, _VP, _I64, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_run_reinit_f16s": (_I32, [_VP, _F32, _VP, _G, _F32, _F32, _F32, _F32, _F32, _I32,
                                       _I32, _I32, _VP, _I64, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_gather_f32": (_I32, [_VP, _G, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_gather_f64": (_I32, [_VP, _G, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_band_gather_f16s": (_I32, [_VP, _G, _VP, _VP, _VP, _VP, _I64, _VP]),
    "ls_set_tuning": (_I32, [ctypes.c_void_p]),
    "ls_get_tuning": (_I32, [ctypes.c_void_p]),
    "ls_upwind_launch_info": (_I32, [_G, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                     ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "ls_batch_workspace_bytes": (_I64, [_VP, _I32]),
    "ls_batch_layout": (_I32, [_VP, _I32, _VP, _VP]),
    "ls_batch_setup": (_I32, [_VP, _I32, _VP, _I64, _VP]),
    "ls_batch_run_f32": (_I32, [_VP, _I32, _VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _I64,
                                _VP]),
    "ls_batch_band": (_I32, [_VP, _I32, _VP, _I64, _VP, _VP]),
    "ls_graph_begin": (_I32, [_VP]),
    "ls_graph_end": (_I32, [_VP, _VP]),
    "ls_graph_launch": (_I32, [_VP, _VP]),
    "ls_graph_destroy": (_I32, [_VP]),
    "ls_stats_enable": (_I32, [_I32]),
    "ls_copy_f32": (_I32, [_VP, _VP, _I64, _VP]),
    "ls_copy_counted": (_I32, [_VP, _VP, _VP, _I64, _I64, _VP, _I32, _VP]),
    "ls_copy_counted_from": (_I32, [_VP, _VP, _VP, _I64, _I64, _I64, _VP, _I32, _VP]),
    "ls_stats_read": (_I32, [_I32, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                             ctypes.POINTER(_F64)]),
    "ls_autotune": (_I32, [_VP, _I32, _I32, ctypes.c_char_p, _VP, _I32]),
    "ls_closure_param_count": (_I64, []),
    "ls_closure_workspace_bytes": (_I64, [_G]),
    "ls_restrict4_f32": (_I32, [_VP, _G, _VP, _VP]),
    "ls_closure_forward_f32": (_I32, [_VP, _VP, _G, _F32, _F32, _F32, _F32, _VP, _VP, _VP, _VP,
                                      _I64, _VP, _VP, _I64, _VP, _I64, _VP]),
    "ls_closure_backward_f32": (_I32, [_VP, _VP, _VP, _G, _F32, _F32, _F32, _F32, _VP, _VP, _VP,
                                       _VP, _I64, _VP, _VP, _I64, _VP, _I64, _VP]),
    "ls_adam_step": (_I32, [_VP, _VP, _VP, _VP, _I64, _F32, _F32, _F32, _F32, _I32, _VP]),
    "ls_closure_run_f32": (_I32, [_VP, _VP, _G, _F32, _F32, _F32, _F32, _VP, _I32, _I32, _I32,
                                  _VP, _I64, _VP, _VP, _VP, _VP, _I64, _VP, _I64, _VP]),
}

LS_KERNEL_UPWIND = 0
LS_KERNEL_BAND_FLAG = 1
LS_KERNEL_REINIT = 2
LS_KERNEL_GATHER = 3
LS_KERNEL_CLOSURE = 4


def lib():
    """The loaded libls.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1612_04040_amd.build` (no fallback exists)")
        # torch first: its HIP runtime is then the one libls binds to (loading
        # libls first would bring in a second runtime that sees no device once
        # torch initialises its own)
        import torch  # noqa: F401
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = handle
    return _LIB


def exported_symbols():
    return sorted(_SIGNATURES)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError(f"cannot pass {type(x).__name__} as a device pointer")


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(status):
    if status < 0:
        raise LsError(int(status), lib().ls_last_error().decode())
    return status


def _g(g):
    return ctypes.byref(g)


def ls_last_error():
    return lib().ls_last_error().decode()


def ls_version():
    return lib().ls_version().decode()


def ls_grid_tiles(g):
    return _check(lib().ls_grid_tiles(_g(g)))


def ls_workspace_bytes(g):
    return _check(lib().ls_workspace_bytes(_g(g)))


def ls_band_build_f32(phi, g, gamma, dilate, tiles, capacity, ntiles_dev, workspace,
                      workspace_bytes, stream=None):
    return _check(lib().ls_band_build_f32(_ptr(phi), _g(g), gamma, dilate, _ptr(tiles), capacity,
                                          _ptr(ntiles_dev), _ptr(workspace), workspace_bytes,
                                          _stream(stream)))


def ls_bricks_from_dense_f32(src, g, dst, stream=None):
    return _check(lib().ls_bricks_from_dense_f32(_ptr(src), _g(g), _ptr(dst), _stream(stream)))


def ls_bricks_to_dense_f32(src, g, dst, stream=None):
    return _check(lib().ls_bricks_to_dense_f32(_ptr(src), _g(g), _ptr(dst), _stream(stream)))


def ls_bricks_from_dense_f16s(src, g, dst, stream=None):
    return _check(lib().ls_bricks_from_dense_f16s(_ptr(src), _g(g), _ptr(dst), _stream(stream)))


def ls_bricks_to_dense_f16s(src, g, dst, stream=None):
    return _check(lib().ls_bricks_to_dense_f16s(_ptr(src), _g(g), _ptr(dst), _stream(stream)))


def ls_band_build_bricks_f32(phi_b, g, gamma, dilate, tiles, capacity, ntiles_dev, workspace,
                             workspace_bytes, stream=None):
    return _check(lib().ls_band_build_bricks_f32(_ptr(phi_b), _g(g), gamma, dilate, _ptr(tiles),
                                                 capacity, _ptr(ntiles_dev), _ptr(workspace),
                                                 workspace_bytes, _stream(stream)))


def ls_band_build_bricks_f16s(phi_b, scale, g, gamma, dilate, tiles, capacity, ntiles_dev,
                              workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_build_bricks_f16s(_ptr(phi_b), scale, _g(g), gamma, dilate,
                                                  _ptr(tiles), capacity, _ptr(ntiles_dev),
                                                  _ptr(workspace), workspace_bytes,
                                                  _stream(stream)))


def ls_band_run_bricks_f32(phi_b, F_b, g, dx, dt, gamma, nsteps, window, beta, reinit_iters,
                           dtau, tiles, capacity, ntiles_dev, tile_steps_dev, scratch_b,
                           workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_run_bricks_f32(
        _ptr(phi_b), _ptr(F_b), _g(g), dx, dt, gamma, nsteps, window, beta, reinit_iters, dtau,
        _ptr(tiles), capacity, _ptr(ntiles_dev), _ptr(tile_steps_dev), _ptr(scratch_b),
        _ptr(workspace), workspace_bytes, _stream(stream)))


def ls_band_run_bricks_f16s(phi_b, scale, F_b, g, dx, dt, gamma, nsteps, window, beta,
                            reinit_iters, dtau, tiles, capacity, ntiles_dev, tile_steps_dev,
                            scratch_b, workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_run_bricks_f16s(
        _ptr(phi_b), scale, _ptr(F_b), _g(g), dx, dt, gamma, nsteps, window, beta, reinit_iters,
        dtau, _ptr(tiles), capacity, _ptr(ntiles_dev), _ptr(tile_steps_dev), _ptr(scratch_b),
        _ptr(workspace), workspace_bytes, _stream(stream)))


def ls_band_build_noalloc_max_bytes():
    return _check(lib().ls_band_build_noalloc_max_bytes())


def ls_band_build_f32_noalloc(phi, g, gamma, dilate, tiles, capacity, ntiles_dev, stream=None):
    return _check(lib().ls_band_build_f32_noalloc(_ptr(phi), _g(g), gamma, dilate, _ptr(tiles),
                                                  capacity, _ptr(ntiles_dev), _stream(stream)))


def ls_band_build_f64(phi, g, gamma, dilate, tiles, capacity, ntiles_dev, workspace,
                      workspace_bytes, stream=None):
    return _check(lib().ls_band_build_f64(_ptr(phi), _g(g), gamma, dilate, _ptr(tiles), capacity,
                                          _ptr(ntiles_dev), _ptr(workspace), workspace_bytes,
                                          _stream(stream)))


def ls_band_build_f16s(phi_h, scale, g, gamma, dilate, tiles, capacity, ntiles_dev, workspace,
                       workspace_bytes, stream=None):
    return _check(lib().ls_band_build_f16s(_ptr(phi_h), scale, _g(g), gamma, dilate, _ptr(tiles),
                                           capacity, _ptr(ntiles_dev), _ptr(workspace),
                                           workspace_bytes, _stream(stream)))


def ls_upwind_step_f32(phi, F, g, dx, dt, tiles, ntiles_dev, nsteps, scratch, workspace,
                       workspace_bytes, stream=None):
    return _check(lib().ls_upwind_step_f32(_ptr(phi), _ptr(F), _g(g), dx, dt, _ptr(tiles),
                                           _ptr(ntiles_dev), nsteps, _ptr(scratch),
                                           _ptr(workspace), workspace_bytes, _stream(stream)))


def ls_upwind_step_f64(phi, F, g, dx, dt, tiles, ntiles_dev, nsteps, scratch, workspace,
                       workspace_bytes, stream=None):
    return _check(lib().ls_upwind_step_f64(_ptr(phi), _ptr(F), _g(g), dx, dt, _ptr(tiles),
                                           _ptr(ntiles_dev), nsteps, _ptr(scratch),
                                           _ptr(workspace), workspace_bytes, _stream(stream)))


def ls_upwind_step_f16s(phi_h, scale, F, g, dx, dt, tiles, ntiles_dev, nsteps, scratch,
                        workspace, workspace_bytes, stream=None):
    return _check(lib().ls_upwind_step_f16s(_ptr(phi_h), scale, _ptr(F), _g(g), dx, dt,
                                            _ptr(tiles), _ptr(ntiles_dev), nsteps, _ptr(scratch),
                                            _ptr(workspace), workspace_bytes, _stream(stream)))


def ls_band_rebuild_f32(phi, g, gamma, prev_tiles, prev_ntiles_dev, tiles, capacity, ntiles_dev,
                        workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_rebuild_f32(_ptr(phi), _g(g), gamma, _ptr(prev_tiles),
                                            _ptr(prev_ntiles_dev), _ptr(tiles), capacity,
                                            _ptr(ntiles_dev), _ptr(workspace), workspace_bytes,
                                            _stream(stream)))


def ls_band_rebuild_f64(phi, g, gamma, prev_tiles, prev_ntiles_dev, tiles, capacity, ntiles_dev,
                        workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_rebuild_f64(_ptr(phi), _g(g), gamma, _ptr(prev_tiles),
                                            _ptr(prev_ntiles_dev), _ptr(tiles), capacity,
                                            _ptr(ntiles_dev), _ptr(workspace), workspace_bytes,
                                            _stream(stream)))


def ls_band_rebuild_f16s(phi_h, scale, g, gamma, prev_tiles, prev_ntiles_dev, tiles, capacity,
                         ntiles_dev, workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_rebuild_f16s(_ptr(phi_h), scale, _g(g), gamma, _ptr(prev_tiles),
                                             _ptr(prev_ntiles_dev), _ptr(tiles), capacity,
                                             _ptr(ntiles_dev), _ptr(workspace), workspace_bytes,
                                             _stream(stream)))


def ls_band_run_f32(phi, F, g, dx, dt, gamma, nsteps, window, tiles, capacity, ntiles_dev,
                    tile_steps_dev, scratch, workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_run_f32(_ptr(phi), _ptr(F), _g(g), dx, dt, gamma, nsteps, window,
                                        _ptr(tiles), capacity, _ptr(ntiles_dev),
                                        _ptr(tile_steps_dev), _ptr(scratch), _ptr(workspace),
                                        workspace_bytes, _stream(stream)))


def ls_band_run_f64(phi, F, g, dx, dt, gamma, nsteps, window, tiles, capacity, ntiles_dev,
                    tile_steps_dev, scratch, workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_run_f64(_ptr(phi), _ptr(F), _g(g), dx, dt, gamma, nsteps, window,
                                        _ptr(tiles), capacity, _ptr(ntiles_dev),
                                        _ptr(tile_steps_dev), _ptr(scratch), _ptr(workspace),
                                        workspace_bytes, _stream(stream)))


def ls_band_run_f16s(phi_h, scale, F, g, dx, dt, gamma, nsteps, window, tiles, capacity,
                     ntiles_dev, tile_steps_dev, scratch, workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_run_f16s(_ptr(phi_h), scale, _ptr(F), _g(g), dx, dt, gamma,
                                         nsteps, window, _ptr(tiles), capacity, _ptr(ntiles_dev),
                                         _ptr(tile_steps_dev), _ptr(scratch), _ptr(workspace),
                                         workspace_bytes, _stream(stream)))


def ls_upwind_step_cutoff_f32(phi, F, g, dx, dt, beta, gamma, tiles, ntiles_dev, nsteps, scratch,
                              workspace, workspace_bytes, stream=None):
    return _check(lib().ls_upwind_step_cutoff_f32(_ptr(phi), _ptr(F), _g(g), dx, dt, beta, gamma,
                                                  _ptr(tiles), _ptr(ntiles_dev), nsteps,
                                                  _ptr(scratch), _ptr(workspace),
                                                  workspace_bytes, _stream(stream)))


def ls_upwind_step_cutoff_f64(phi, F, g, dx, dt, beta, gamma, tiles, ntiles_dev, nsteps, scratch,
                              workspace, workspace_bytes, stream=None):
    return _check(lib().ls_upwind_step_cutoff_f64(_ptr(phi), _ptr(F), _g(g), dx, dt, beta, gamma,
                                                  _ptr(tiles), _ptr(ntiles_dev), nsteps,
                                                  _ptr(scratch), _ptr(workspace),
                                                  workspace_bytes, _stream(stream)))


def ls_upwind_step_cutoff_f16s(phi_h, scale, F, g, dx, dt, beta, gamma, tiles, ntiles_dev, nsteps,
                               scratch, workspace, workspace_bytes, stream=None):
    return _check(lib().ls_upwind_step_cutoff_f16s(_ptr(phi_h), scale, _ptr(F), _g(g), dx, dt,
                                                   beta, gamma, _ptr(tiles), _ptr(ntiles_dev),
                                                   nsteps, _ptr(scratch), _ptr(workspace),
                                                   workspace_bytes, _stream(stream)))


def ls_band_run_cutoff_f32(phi, F, g, dx, dt, beta, gamma, nsteps, window, tiles, capacity,
                           ntiles_dev, tile_steps_dev, scratch, workspace, workspace_bytes,
                           stream=None):
    return _check(lib().ls_band_run_cutoff_f32(_ptr(phi), _ptr(F), _g(g), dx, dt, beta, gamma,
                                               nsteps, window, _ptr(tiles), capacity,
                                               _ptr(ntiles_dev), _ptr(tile_steps_dev),
                                               _ptr(scratch), _ptr(workspace), workspace_bytes,
                                               _stream(stream)))


def ls_band_run_cutoff_f64(phi, F, g, dx, dt, beta, gamma, nsteps, window, tiles, capacity,
                           ntiles_dev, tile_steps_dev, scratch, workspace, workspace_bytes,
                           stream=None):
    return _check(lib().ls_band_run_cutoff_f64(_ptr(phi), _ptr(F), _g(g), dx, dt, beta, gamma,
                                               nsteps, window, _ptr(tiles), capacity,
                                               _ptr(ntiles_dev), _ptr(tile_steps_dev),
                                               _ptr(scratch), _ptr(workspace), workspace_bytes,
                                               _stream(stream)))


def ls_band_run_cutoff_f16s(phi_h, scale, F, g, dx, dt, beta, gamma, nsteps, window, tiles,
                            capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                            workspace_bytes, stream=None):
    return _check(lib().ls_band_run_cutoff_f16s(_ptr(phi_h), scale, _ptr(F), _g(g), dx, dt, beta,
                                                gamma, nsteps, window, _ptr(tiles), capacity,
                                                _ptr(ntiles_dev), _ptr(tile_steps_dev),
                                                _ptr(scratch), _ptr(workspace), workspace_bytes,
                                                _stream(stream)))


def ls_reinit_step_f32(phi, g, dx, dtau, gamma, clamp, tiles, ntiles_dev, niter, scratch,
                       workspace, workspace_bytes, stream=None):
    return _check(lib().ls_reinit_step_f32(_ptr(phi), _g(g), dx, dtau, gamma, clamp, _ptr(tiles),
                                           _ptr(ntiles_dev), niter, _ptr(scratch),
                                           _ptr(workspace), workspace_bytes, _stream(stream)))


def ls_reinit_step_f64(phi, g, dx, dtau, gamma, clamp, tiles, ntiles_dev, niter, scratch,
                       workspace, workspace_bytes, stream=None):
    return _check(lib().ls_reinit_step_f64(_ptr(phi), _g(g), dx, dtau, gamma, clamp, _ptr(tiles),
                                           _ptr(ntiles_dev), niter, _ptr(scratch),
                                           _ptr(workspace), workspace_bytes, _stream(stream)))


def ls_reinit_step_f16s(phi_h, scale, g, dx, dtau, gamma, clamp, tiles, ntiles_dev, niter,
                        scratch, workspace, workspace_bytes, stream=None):
    return _check(lib().ls_reinit_step_f16s(_ptr(phi_h), scale, _g(g), dx, dtau, gamma, clamp,
                                            _ptr(tiles), _ptr(ntiles_dev), niter, _ptr(scratch),
                                            _ptr(workspace), workspace_bytes, _stream(stream)))


def ls_band_run_reinit_f32(phi, F, g, dx, dt, beta, gamma, dtau, reinit_iters, nsteps, window,
                           tiles, capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                           workspace_bytes, stream=None):
    return _check(lib().ls_band_run_reinit_f32(_ptr(phi), _ptr(F), _g(g), dx, dt, beta, gamma,
                                               dtau, reinit_iters, nsteps, window, _ptr(tiles),
                                               capacity, _ptr(ntiles_dev), _ptr(tile_steps_dev),
                                               _ptr(scratch), _ptr(workspace), workspace_bytes,
                                               _stream(stream)))


def ls_band_run_reinit_f64(phi, F, g, dx, dt, beta, gamma, dtau, reinit_iters, nsteps, window,
                           tiles, capacity, ntiles_dev, tile_steps_dev, scratch, workspace,
                           workspace_bytes, stream=None):
    return _check(lib().ls_band_run_reinit_f64(_ptr(phi), _ptr(F), _g(g), dx, dt, beta, gamma,
                                               dtau, reinit_iters, nsteps, window, _ptr(tiles),
                                               capacity, _ptr(ntiles_dev), _ptr(tile_steps_dev),
                                               _ptr(scratch), _ptr(workspace), workspace_bytes,
                                               _stream(stream)))


def ls_band_run_reinit_f16s(phi_h, scale, F, g, dx, dt, beta, gamma, dtau, reinit_iters, nsteps,
                            window, tiles, capacity, ntiles_dev, tile_steps_dev, scratch,
                            workspace, workspace_bytes, stream=None):
    return _check(lib().ls_band_run_reinit_f16s(_ptr(phi_h), scale, _ptr(F), _g(g), dx, dt, beta,
                                                gamma, dtau, reinit_iters, nsteps, window,
                                                _ptr(tiles), capacity, _ptr(ntiles_dev),
                                                _ptr(tile_steps_dev), _ptr(scratch),
                                                _ptr(workspace), workspace_bytes,
                                                _stream(stream)))


def _gather(name, phi, g, tiles, ntiles_dev, out, ids_out, capacity, stream):
    return _check(getattr(lib(), name)(_ptr(phi), _g(g), _ptr(tiles), _ptr(ntiles_dev),
                                       _ptr(out), _ptr(ids_out), capacity, _stream(stream)))


def ls_band_gather_f32(phi, g, tiles, ntiles_dev, out, ids_out, capacity, stream=None):
    return _gather("ls_band_gather_f32", phi, g, tiles, ntiles_dev, out, ids_out, capacity,
                   stream)


def ls_band_gather_f64(phi, g, tiles, ntiles_dev, out, ids_out, capacity, stream=None):
    return _gather("ls_band_gather_f64", phi, g, tiles, ntiles_dev, out, ids_out, capacity,
                   stream)


def ls_band_gather_f16s(phi_h, g, tiles, ntiles_dev, out, ids_out, capacity, stream=None):
    return _gather("ls_band_gather_f16s", phi_h, g, tiles, ntiles_dev, out, ids_out, capacity,
                   stream)


def ls_copy_counted(dst, src, count_dev, unit_bytes, max_units, count_out=None, blocks=0,
                    stream=None):
    return _check(lib().ls_copy_counted(_ptr(dst), _ptr(src), _ptr(count_dev), int(unit_bytes),
                                        int(max_units), _ptr(count_out), int(blocks),
                                        _stream(stream)))


def ls_copy_counted_from(dst, src, count_dev, unit_bytes, first_unit, max_units, count_out=None,
                         blocks=0, stream=None):
    return _check(lib().ls_copy_counted_from(_ptr(dst), _ptr(src), _ptr(count_dev),
                                             int(unit_bytes), int(first_unit), int(max_units),
                                             _ptr(count_out), int(blocks), _stream(stream)))


def ls_stats_enable(on):
    return _check(lib().ls_stats_enable(1 if on else 0))


def ls_stats_read(which):
    """(launches, timed launches, summed duration in ms) of kernel `which`."""
    launches, timed, ms = _I64(), _I64(), _F64()
    _check(lib().ls_stats_read(which, ctypes.byref(launches), ctypes.byref(timed),
                               ctypes.byref(ms)))
    return launches.value, timed.value, ms.value


def ls_set_tuning(run_width=0, blocks_per_cu=0, pipeline=0, vector=0, temporal=0):
    t = ls_tuning(int(run_width), int(blocks_per_cu), int(pipeline), int(vector), int(temporal))
    return _check(lib().ls_set_tuning(ctypes.byref(t)))


def ls_get_tuning():
    """(run_width, blocks_per_cu, pipeline, vector, temporal)."""
    t = ls_tuning()
    _check(lib().ls_get_tuning(ctypes.byref(t)))
    return t.run_width, t.blocks_per_cu, t.pipeline, t.vector, t.temporal


PRECISION_ID = {"f32": 0, "f64": 1, "f16s": 2}


def ls_upwind_launch_info(g, precision):
    """dict(blocks, lds_bytes, run_tiles, blocks_per_cu_limit) for grid g."""
    out = [_I32() for _ in range(4)]
    _check(lib().ls_upwind_launch_info(_g(g), PRECISION_ID.get(precision, precision),
                                       *[ctypes.byref(v) for v in out]))
    return dict(zip(("blocks", "lds_bytes", "run_tiles", "blocks_per_cu_limit"),
                    (v.value for v in out)))


def ls_copy_f32(dst, src, n, stream=None):
    return _check(lib().ls_copy_f32(_ptr(dst), _ptr(src), int(n), _stream(stream)))


def ls_batch_workspace_bytes(inst, n):
    return _check(lib().ls_batch_workspace_bytes(ctypes.addressof(inst), n))


def ls_batch_layout(inst, n):
    """(tile_base list, total tiles) of the batch layout."""
    base = (ctypes.c_int64 * n)()
    total = ctypes.c_int64()
    _check(lib().ls_batch_layout(ctypes.addressof(inst), n, ctypes.addressof(base),
                                 ctypes.byref(total)))
    return list(base), total.value


def ls_batch_setup(inst, n, workspace, workspace_bytes, stream=None):
    return _check(lib().ls_batch_setup(ctypes.addressof(inst), n, _ptr(workspace), workspace_bytes,
                                       _stream(stream)))


def ls_batch_run_f32(inst, n, phi, F, scratch, nsteps, window, tile_steps_dev, point_steps_dev,
                     workspace, workspace_bytes, stream=None):
    return _check(lib().ls_batch_run_f32(ctypes.addressof(inst), n, _ptr(phi), _ptr(F),
                                         _ptr(scratch), nsteps, window, _ptr(tile_steps_dev),
                                         _ptr(point_steps_dev), _ptr(workspace), workspace_bytes,
                                         _stream(stream)))


def ls_batch_band(inst, n, workspace, workspace_bytes):
    """(device address of the last band list, device address of its length)."""
    t, c = ctypes.c_void_p(), ctypes.c_void_p()
    _check(lib().ls_batch_band(ctypes.addressof(inst), n, _ptr(workspace), workspace_bytes,
                               ctypes.byref(t), ctypes.byref(c)))
    return t.value, c.value


def ls_graph_begin(stream):
    return _check(lib().ls_graph_begin(_stream(stream)))


def ls_graph_end(stream):
    h = ctypes.c_void_p()
    _check(lib().ls_graph_end(_stream(stream), ctypes.byref(h)))
    return h.value


def ls_graph_launch(graph, stream=None):
    return _check(lib().ls_graph_launch(graph, _stream(stream)))


def ls_graph_destroy(graph):
    return _check(lib().ls_graph_destroy(graph))


def ls_closure_param_count():
    return int(lib().ls_closure_param_count())


def ls_closure_workspace_bytes(g):
    return _check(lib().ls_closure_workspace_bytes(_g(g)))


def ls_restrict4_f32(fine, fine_grid, coarse, stream=None):
    return _check(lib().ls_restrict4_f32(_ptr(fine), _g(fine_grid), _ptr(coarse), _stream(stream)))


def ls_closure_forward_f32(phi, F, g, dx, dt, gamma, fmax, params, r, plain, tiles, capacity,
                           ntiles_dev, ws, ws_bytes, cws, cws_bytes, stream=None):
    return _check(lib().ls_closure_forward_f32(
        _ptr(phi), _ptr(F), _g(g), dx, dt, gamma, fmax, _ptr(params), _ptr(r), _ptr(plain),
        _ptr(tiles), capacity, _ptr(ntiles_dev), _ptr(ws), ws_bytes, _ptr(cws), cws_bytes,
        _stream(stream)))


def ls_closure_backward_f32(phi, target, F, g, dx, dt, gamma, fmax, params, grad, loss_dev, tiles,
                            capacity, ntiles_dev, ws, ws_bytes, cws, cws_bytes, stream=None):
    return _check(lib().ls_closure_backward_f32(
        _ptr(phi), _ptr(target), _ptr(F), _g(g), dx, dt, gamma, fmax, _ptr(params), _ptr(grad),
        _ptr(loss_dev), _ptr(tiles), capacity, _ptr(ntiles_dev), _ptr(ws), ws_bytes, _ptr(cws),
        cws_bytes, _stream(stream)))


def ls_adam_step(params, grad, m, v, n, lr, beta1, beta2, eps, t, stream=None):
    return _check(lib().ls_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(n), lr,
                                     beta1, beta2, eps, int(t), _stream(stream)))


def ls_closure_run_f32(phi, F, g, dx, dt, gamma, fmax, params, nsteps, window, judge, tiles,
                       capacity, ntiles_dev, fallbacks_dev, resets_dev, ws, ws_bytes, cws,
                       cws_bytes, stream=None):
    return _check(lib().ls_closure_run_f32(
        _ptr(phi), _ptr(F), _g(g), dx, dt, gamma, fmax, _ptr(params), int(nsteps), int(window),
        int(judge), _ptr(tiles), capacity, _ptr(ntiles_dev), _ptr(fallbacks_dev),
        _ptr(resets_dev), _ptr(ws), ws_bytes, _ptr(cws), cws_bytes, _stream(stream)))


def ls_autotune(sizes, cache_path=None, force=False, precision=0):
    """Tile shape per size (list of (tx, ty, tz)), measured or from the cache."""
    n = len(sizes)
    arr = (ctypes.c_int32 * n)(*[int(v) for v in sizes])
    out = (ls_grid * n)()
    path = cache_path.encode() if cache_path else None
    _check(lib().ls_autotune(ctypes.addressof(arr), n, precision, path, ctypes.addressof(out),
                             1 if force else 0))
    return [(g.tx, g.ty, g.tz) for g in out]
