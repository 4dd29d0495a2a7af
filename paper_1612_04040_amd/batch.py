"""Device buffers of a batch of uneven grids, and thin wrappers over the batch
C-ABI (argument marshalling only; the computation runs in libls)."""
import numpy as np
import torch

from . import ls

ALIGN = 64  # grid offsets in elements (256 bytes)
ROW_ALIGN = 32  # default row pitch granule in elements: every x row starts a 128-byte line


class Batch:
    """Grids (n_i^3 or any dims) packed into one phi / F / scratch buffer each.

    ``specs`` is a list of (dims, tile, dx, dt, gamma); grid i starts at
    element ``offsets[i]`` of the buffers, its x rows ``pitches[i]`` elements
    apart (nx rounded up to ``row_align``; 1 gives dense rows).
    """

    def __init__(self, specs, device="cuda", row_align=ROW_ALIGN):
        self.device = torch.device(device)
        self.specs = [(tuple(int(v) for v in d), tuple(int(v) for v in t), float(dx), float(dt),
                       float(gm)) for d, t, dx, dt, gm in specs]
        self.offsets, self.pitches = [], []
        off = 0
        for (nx, ny, nz), *_ in self.specs:
            px = -(-nx // row_align) * row_align
            self.offsets.append(off)
            self.pitches.append(px)
            off += -(-px * ny * nz // ALIGN) * ALIGN
        self.total = off
        self.n = len(self.specs)
        self.inst = ls.instances([(d, t, o, dx, dt, g, px) for (d, t, dx, dt, g), o, px
                                  in zip(self.specs, self.offsets, self.pitches)])
        self.tile_base, self.total_tiles = ls.ls_batch_layout(self.inst, self.n)
        self.ws_bytes = ls.ls_batch_workspace_bytes(self.inst, self.n)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        a = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[a:a + self.ws_bytes]
        self.phi = torch.zeros(self.total, dtype=torch.float32, device=self.device)
        self.F = torch.zeros(self.total, dtype=torch.float32, device=self.device)
        self.scratch = torch.empty(self.total, dtype=torch.float32, device=self.device)
        ls.ls_batch_setup(self.inst, self.n, self.ws, self.ws_bytes)

    def view(self, buf, i):
        """(nz, ny, nx) view of grid i in a batch buffer (strided when pitched)."""
        nx, ny, nz = self.specs[i][0]
        o, px = self.offsets[i], self.pitches[i]
        return buf[o:o + px * ny * nz].view(nz, ny, px)[:, :, :nx]

    def load(self, phis, Fs):
        for i, (p, f) in enumerate(zip(phis, Fs)):
            self.view(self.phi, i).copy_(torch.from_numpy(np.ascontiguousarray(p, np.float32)))
            self.view(self.F, i).copy_(torch.from_numpy(np.ascontiguousarray(f, np.float32)))

    def run(self, nsteps, window=10, tile_steps=None, phi=None, stream=None, point_steps=None):
        ls.ls_batch_run_f32(self.inst, self.n, self.phi if phi is None else phi, self.F,
                            self.scratch, nsteps, window, tile_steps, point_steps, self.ws,
                            self.ws_bytes, stream)

    def ntiles(self, i):
        (nx, ny, nz), (tx, ty, tz) = self.specs[i][0], self.specs[i][1]
        return -(-nx // tx) * -(-ny // ty) * -(-nz // tz)

    def band_lists(self):
        """Last band list of every grid, in grid-local tile ids (synchronises)."""
        t, c = ls.ls_batch_band(self.inst, self.n, self.ws, self.ws_bytes)
        torch.cuda.synchronize(self.device)
        base = self.ws.data_ptr()
        cnt = int(self.ws[c - base:c - base + 4].view(torch.int32).item())
        lst = self.ws[t - base:t - base + 4 * cnt].view(torch.int32).cpu().numpy()
        out = []
        for i in range(self.n):
            lo = self.tile_base[i]
            hi = lo + self.ntiles(i)
            out.append(lst[(lst >= lo) & (lst < hi)] - lo)
        return out
