"""Device buffers for one level-set grid, and thin wrappers over the C-ABI.

``BandGrid`` owns (through torch's allocator) the band list, its device
count, the workspace and the ping-pong scratch buffer of one grid; its
methods only marshal arguments to the ``ls_*`` entry points.  All arithmetic
runs in libls's HIP kernels.
"""
import torch

from . import ls

_STORAGE = {"f32": torch.float32, "f64": torch.float64, "f16s": torch.float16}


class BandGrid:
    def __init__(self, dims, tile=(8, 8, 8), precision="f32", device="cuda"):
        if precision not in _STORAGE:
            raise ValueError(f"precision must be one of {sorted(_STORAGE)}")
        self.dims = tuple(int(v) for v in dims)
        self.tile = tuple(int(v) for v in tile)
        self.precision = precision
        self.device = torch.device(device)
        self.g = ls.grid(self.dims, self.tile)
        self.capacity = ls.ls_grid_tiles(self.g)
        self.ws_bytes = ls.ls_workspace_bytes(self.g)
        self.tiles = torch.empty(self.capacity, dtype=torch.int32, device=self.device)
        self.ntiles = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off:off + self.ws_bytes]
        nx, ny, nz = self.dims
        self.scratch = torch.empty((nz, ny, nx), dtype=_STORAGE[precision], device=self.device)

    # -- band -----------------------------------------------------------------
    def build(self, phi, gamma, dilate=True, scale=None, stream=None):
        d = 1 if dilate else 0
        if self.precision == "f32":
            ls.ls_band_build_f32(phi, self.g, gamma, d, self.tiles, self.capacity, self.ntiles,
                                 self.ws, self.ws_bytes, stream)
        elif self.precision == "f64":
            ls.ls_band_build_f64(phi, self.g, gamma, d, self.tiles, self.capacity, self.ntiles,
                                 self.ws, self.ws_bytes, stream)
        else:
            ls.ls_band_build_f16s(phi, scale, self.g, gamma, d, self.tiles, self.capacity,
                                  self.ntiles, self.ws, self.ws_bytes, stream)

    def band_list(self):
        """The current band list as a host tensor (synchronises)."""
        n = int(self.ntiles.item())
        return self.tiles[:n].cpu()

    # -- steps ----------------------------------------------------------------
    def step(self, phi, F, dx, dt, nsteps, scale=None, tiles=None, ntiles=None, stream=None,
             cutoff=None):
        """nsteps band steps; ``cutoff=(beta, gamma)`` takes the cut-off steps of Eq. 8."""
        t = self.tiles if tiles is None else tiles
        n = self.ntiles if ntiles is None else ntiles
        if cutoff is not None:
            b, c = cutoff
            if self.precision == "f32":
                ls.ls_upwind_step_cutoff_f32(phi, F, self.g, dx, dt, b, c, t, n, nsteps,
                                             self.scratch, self.ws, self.ws_bytes, stream)
            elif self.precision == "f64":
                ls.ls_upwind_step_cutoff_f64(phi, F, self.g, dx, dt, b, c, t, n, nsteps,
                                             self.scratch, self.ws, self.ws_bytes, stream)
            else:
                ls.ls_upwind_step_cutoff_f16s(phi, scale, F, self.g, dx, dt, b, c, t, n, nsteps,
                                              self.scratch, self.ws, self.ws_bytes, stream)
            return
        if self.precision == "f32":
            ls.ls_upwind_step_f32(phi, F, self.g, dx, dt, t, n, nsteps, self.scratch, self.ws,
                                  self.ws_bytes, stream)
        elif self.precision == "f64":
            ls.ls_upwind_step_f64(phi, F, self.g, dx, dt, t, n, nsteps, self.scratch, self.ws,
                                  self.ws_bytes, stream)
        else:
            ls.ls_upwind_step_f16s(phi, scale, F, self.g, dx, dt, t, n, nsteps, self.scratch,
                                   self.ws, self.ws_bytes, stream)

    def reinit(self, phi, dx, dtau, niter, gamma=None, scale=None, tiles=None, ntiles=None,
               stream=None):
        """niter reinitialisation steps (Eq. 12-13) on the band list; with
        gamma the last is clamped to [-gamma, gamma] (Eq. 10)."""
        t = self.tiles if tiles is None else tiles
        n = self.ntiles if ntiles is None else ntiles
        clamp, g = (0, 0.0) if gamma is None else (1, gamma)
        if self.precision == "f32":
            ls.ls_reinit_step_f32(phi, self.g, dx, dtau, g, clamp, t, n, niter, self.scratch,
                                  self.ws, self.ws_bytes, stream)
        elif self.precision == "f64":
            ls.ls_reinit_step_f64(phi, self.g, dx, dtau, g, clamp, t, n, niter, self.scratch,
                                  self.ws, self.ws_bytes, stream)
        else:
            ls.ls_reinit_step_f16s(phi, scale, self.g, dx, dtau, g, clamp, t, n, niter,
                                   self.scratch, self.ws, self.ws_bytes, stream)

    def gather(self, phi, out, ids=None, capacity=None, tiles=None, ntiles=None, stream=None):
        """The band snapshot: the listed tiles' values into out (tile-major; see
        ls_band_gather_*), their ids into ids."""
        t = self.tiles if tiles is None else tiles
        n = self.ntiles if ntiles is None else ntiles
        cap = self.capacity if capacity is None else capacity
        fn = {"f32": ls.ls_band_gather_f32, "f64": ls.ls_band_gather_f64,
              "f16s": ls.ls_band_gather_f16s}[self.precision]
        fn(phi, self.g, t, n, out, ids, cap, stream)

    def rebuild(self, phi, gamma, prev_tiles, prev_ntiles, scale=None, stream=None):
        """Incremental rebuild from a previous band (see ls_band_rebuild_*)."""
        if self.precision == "f32":
            ls.ls_band_rebuild_f32(phi, self.g, gamma, prev_tiles, prev_ntiles, self.tiles,
                                   self.capacity, self.ntiles, self.ws, self.ws_bytes, stream)
        elif self.precision == "f64":
            ls.ls_band_rebuild_f64(phi, self.g, gamma, prev_tiles, prev_ntiles, self.tiles,
                                   self.capacity, self.ntiles, self.ws, self.ws_bytes, stream)
        else:
            ls.ls_band_rebuild_f16s(phi, scale, self.g, gamma, prev_tiles, prev_ntiles,
                                    self.tiles, self.capacity, self.ntiles, self.ws,
                                    self.ws_bytes, stream)

    def run(self, phi, F, dx, dt, gamma, nsteps, window=10, scale=None, tile_steps=None,
            stream=None, beta=None, reinit=None):
        """The windowed driver; with ``beta`` the cut-off steps of Eq. 8 (with gamma); with
        ``reinit = (dtau, iters)`` as well, Step 3 (reinitialisation and clamp) ends each
        window."""
        if reinit is not None:
            if beta is None:
                raise ValueError("the reinitialising driver takes the cut-off steps: give beta")
            dtau, iters = reinit
            if self.precision == "f32":
                ls.ls_band_run_reinit_f32(phi, F, self.g, dx, dt, beta, gamma, dtau, iters,
                                          nsteps, window, self.tiles, self.capacity, self.ntiles,
                                          tile_steps, self.scratch, self.ws, self.ws_bytes,
                                          stream)
            elif self.precision == "f64":
                ls.ls_band_run_reinit_f64(phi, F, self.g, dx, dt, beta, gamma, dtau, iters,
                                          nsteps, window, self.tiles, self.capacity, self.ntiles,
                                          tile_steps, self.scratch, self.ws, self.ws_bytes,
                                          stream)
            else:
                ls.ls_band_run_reinit_f16s(phi, scale, F, self.g, dx, dt, beta, gamma, dtau,
                                           iters, nsteps, window, self.tiles, self.capacity,
                                           self.ntiles, tile_steps, self.scratch, self.ws,
                                           self.ws_bytes, stream)
            return
        if beta is not None:
            if self.precision == "f32":
                ls.ls_band_run_cutoff_f32(phi, F, self.g, dx, dt, beta, gamma, nsteps, window,
                                          self.tiles, self.capacity, self.ntiles, tile_steps,
                                          self.scratch, self.ws, self.ws_bytes, stream)
            elif self.precision == "f64":
                ls.ls_band_run_cutoff_f64(phi, F, self.g, dx, dt, beta, gamma, nsteps, window,
                                          self.tiles, self.capacity, self.ntiles, tile_steps,
                                          self.scratch, self.ws, self.ws_bytes, stream)
            else:
                ls.ls_band_run_cutoff_f16s(phi, scale, F, self.g, dx, dt, beta, gamma, nsteps,
                                           window, self.tiles, self.capacity, self.ntiles,
                                           tile_steps, self.scratch, self.ws, self.ws_bytes,
                                           stream)
            return
        if self.precision == "f32":
            ls.ls_band_run_f32(phi, F, self.g, dx, dt, gamma, nsteps, window, self.tiles,
                               self.capacity, self.ntiles, tile_steps, self.scratch, self.ws,
                               self.ws_bytes, stream)
        elif self.precision == "f64":
            ls.ls_band_run_f64(phi, F, self.g, dx, dt, gamma, nsteps, window, self.tiles,
                               self.capacity, self.ntiles, tile_steps, self.scratch, self.ws,
                               self.ws_bytes, stream)
        else:
            ls.ls_band_run_f16s(phi, scale, F, self.g, dx, dt, gamma, nsteps, window, self.tiles,
                                self.capacity, self.ntiles, tile_steps, self.scratch, self.ws,
                                self.ws_bytes, stream)

    # -- tile-major ("brick") layout -------------------------------------------
    def to_bricks(self, src, dst, stream=None):
        """src (x-fastest) -> dst (tile-major); FP32 values or scaled-FP16 codes."""
        if self.precision == "f32" or src.dtype == torch.float32:
            ls.ls_bricks_from_dense_f32(src, self.g, dst, stream)
        else:
            ls.ls_bricks_from_dense_f16s(src, self.g, dst, stream)

    def from_bricks(self, src, dst, stream=None):
        """src (tile-major) -> dst (x-fastest)."""
        if self.precision == "f32" or src.dtype == torch.float32:
            ls.ls_bricks_to_dense_f32(src, self.g, dst, stream)
        else:
            ls.ls_bricks_to_dense_f16s(src, self.g, dst, stream)

    def build_bricks(self, phi_b, gamma, dilate=True, scale=None, stream=None):
        d = 1 if dilate else 0
        if self.precision == "f32":
            ls.ls_band_build_bricks_f32(phi_b, self.g, gamma, d, self.tiles, self.capacity,
                                        self.ntiles, self.ws, self.ws_bytes, stream)
        elif self.precision == "f16s":
            ls.ls_band_build_bricks_f16s(phi_b, scale, self.g, gamma, d, self.tiles,
                                         self.capacity, self.ntiles, self.ws, self.ws_bytes,
                                         stream)
        else:
            raise ValueError("the brick layout takes f32 or f16s storage")

    def run_bricks(self, phi_b, F_b, dx, dt, gamma, nsteps, window=10, scale=None,
                   tile_steps=None, stream=None, beta=None, reinit=None):
        """The windowed driver on tile-major fields (phi_b in this grid's storage, F_b FP32,
        both converted with to_bricks); the scratch buffer serves as the brick ping-pong
        partner.  ``beta``: the cut-off steps of Eq. 8; ``reinit = (dtau, iters)``: Step 3
        ends each window."""
        b = 0.0 if beta is None else float(beta)
        dtau, iters = (0.0, 0) if reinit is None else (float(reinit[0]), int(reinit[1]))
        if self.precision == "f32":
            ls.ls_band_run_bricks_f32(phi_b, F_b, self.g, dx, dt, gamma, nsteps, window, b, iters,
                                      dtau, self.tiles, self.capacity, self.ntiles, tile_steps,
                                      self.scratch, self.ws, self.ws_bytes, stream)
        elif self.precision == "f16s":
            ls.ls_band_run_bricks_f16s(phi_b, scale, F_b, self.g, dx, dt, gamma, nsteps, window,
                                       b, iters, dtau, self.tiles, self.capacity, self.ntiles,
                                       tile_steps, self.scratch, self.ws, self.ws_bytes, stream)
        else:
            raise ValueError("the brick layout takes f32 or f16s storage")
