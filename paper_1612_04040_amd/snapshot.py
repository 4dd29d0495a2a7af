"""Asynchronous band snapshots of a running field.

The output of the narrow-band algorithm (Sec. 1.1, Step 4) taken off the GPU
while it keeps computing: ``take`` enqueues, on the compute stream, the band
gather (``ls_band_gather_*``: the band tiles' values, tile-major, and their
ids) into one of two device staging buffers plus a device copy of the band
count, then, on a separate copy stream that waits for the gather, the copy of
the tiles and ids into pinned host memory: a DMA copy of a size the host knows
(the band count of the last snapshot the host has read, with a margin of
1/8 + 64 tiles), then the library's counted copy (``ls_copy_counted_from``)
of the tiles beyond it, if any, the count read on the device (the first
snapshot, with no count known yet, goes by the counted copy alone unless the
caller gave an estimate).  The host
never waits: ``take`` returns as soon as the work is enqueued, and the caller
enqueues the next windows while the copy runs.  Gather k + 2 reuses the
staging buffer of snapshot k and waits, on the GPU, for that buffer's copy to
finish; the host buffer of snapshot k is reused by snapshot k + 2, so a
snapshot must be waited for before two more are taken, and the arrays
``wait`` returns are views of the pinned buffers, valid until then
(``wait(copy=True)`` returns owned copies, at the cost of a host copy of the
whole snapshot, which stalls the thread that enqueues the GPU work).
``close`` waits for the copies in flight and releases the buffers, streams
and events (call it before the process ends).

Streams, events and pinned buffers are torch's; the gather and the copy are
the library's kernels.
"""
import numpy as np
import torch

from . import ls

_DTYPES = {"f32": torch.float32, "f64": torch.float64, "f16s": torch.float16}


class Snapshot:
    """A snapshot in flight; ``wait`` returns (tile ids, values (n, tz, ty, tx))."""

    def __init__(self, owner, slot, serial):
        self._owner, self._slot, self._serial = owner, slot, serial
        self._result = None

    def wait(self, copy=False):
        if self._result is None:
            self._result = self._owner._finish(self._slot, self._serial)
        ids, vals = self._result
        return (ids.copy(), vals.copy()) if copy else (ids, vals)


class Snapshots:
    """Snapshots of the fields of one BandGrid.  capacity: the most band tiles a
    snapshot holds (default: every tile of the grid; a band beyond it is cut to
    its first capacity tiles); two device staging buffers and two pinned host
    buffers of that size are allocated up front.  copy_blocks: workgroups of
    each counted copy (0: the library's default, a quarter of the compute
    units).  expected: an estimate of the band count (tiles), taken as the
    host-known count until a snapshot has been read (None: the first
    snapshots go by the counted copy alone)."""

    def __init__(self, bg, capacity=None, copy_blocks=0, expected=None):
        self.bg = bg
        dev = bg.tiles.device
        self.tile = bg.tile
        self.tp = int(np.prod(self.tile))
        self.cap = bg.capacity if capacity is None else int(capacity)
        dt = _DTYPES[bg.precision]
        self.stage = [torch.empty(self.cap * self.tp, dtype=dt, device=dev) for _ in range(2)]
        self.stage_ids = [torch.empty(self.cap, dtype=torch.int32, device=dev) for _ in range(2)]
        self.host = [torch.empty(self.cap * self.tp, dtype=dt).pin_memory() for _ in range(2)]
        self.host_ids = [torch.empty(self.cap, dtype=torch.int32).pin_memory() for _ in range(2)]
        self.stage_count = [torch.zeros(1, dtype=torch.int32, device=dev) for _ in range(2)]
        self.count = torch.zeros(2, dtype=torch.int32).pin_memory()
        self.copy_stream = torch.cuda.Stream(dev)
        self.gathered = [torch.cuda.Event() for _ in range(2)]
        self.copied = [torch.cuda.Event() for _ in range(2)]
        self.serial = [-1, -1]       # snapshot held by each slot
        self.consumed = [True, True]
        self.taken = 0
        self.copy_blocks = int(copy_blocks)
        # band count of the last snapshot read on the host
        self.known = None if expected is None else int(expected)
        self.closed = False

    def take(self, phi, stream=None):
        """Snapshot of phi on the band the BandGrid holds, enqueued on `stream`."""
        if self.closed:
            raise RuntimeError("snapshots closed")
        s = torch.cuda.current_stream(self.bg.tiles.device) if stream is None else stream
        i = self.taken % 2
        if not self.consumed[i]:
            raise RuntimeError("snapshot buffers full: wait() on the snapshot taken two "
                               "takes ago before taking another")
        if self.serial[i] >= 0:
            s.wait_event(self.copied[i])  # its staging buffer is free once copied
        self.bg.gather(phi, self.stage[i], ids=self.stage_ids[i], capacity=self.cap, stream=s)
        with torch.cuda.stream(s):
            # the band count as of this gather (the next build overwrites the grid's)
            self.stage_count[i].copy_(self.bg.ntiles[:1], non_blocking=True)
        self.gathered[i].record(s)
        self.copy_stream.wait_event(self.gathered[i])
        esize = self.stage[i].element_size()
        # tiles moved by DMA: a host-known bound on the count; the counted
        # copy takes whatever lies beyond it
        b = 0 if self.known is None else min(self.cap, self.known + self.known // 8 + 64)
        if b > 0:
            with torch.cuda.stream(self.copy_stream):
                self.host[i][: b * self.tp].copy_(self.stage[i][: b * self.tp], non_blocking=True)
                self.host_ids[i][:b].copy_(self.stage_ids[i][:b], non_blocking=True)
        ls.ls_copy_counted_from(self.host[i], self.stage[i], self.stage_count[i],
                                self.tp * esize, b, self.cap, count_out=self.count[i:i + 1],
                                blocks=self.copy_blocks, stream=self.copy_stream)
        ls.ls_copy_counted_from(self.host_ids[i], self.stage_ids[i], self.stage_count[i], 4, b,
                                self.cap, blocks=self.copy_blocks, stream=self.copy_stream)
        self.copied[i].record(self.copy_stream)
        self.serial[i] = self.taken
        self.consumed[i] = False
        snap = Snapshot(self, i, self.taken)
        self.taken += 1
        return snap

    def _finish(self, i, serial):
        if self.serial[i] != serial:
            raise RuntimeError("snapshot overwritten before it was read")
        self.copied[i].synchronize()
        n = min(int(self.count[i]), self.cap)
        self.known = n
        ids = self.host_ids[i][:n].numpy()
        vals = self.host[i][: n * self.tp].numpy()
        tx, ty, tz = self.tile
        self.consumed[i] = True
        return ids, vals.reshape(n, tz, ty, tx)

    def close(self):
        """Waits for the copies in flight, then releases the staging and pinned
        buffers (torch's pinned-memory cache is emptied too), the copy stream
        and the events.  Snapshots not yet waited for are lost."""
        if self.closed:
            return
        self.copy_stream.synchronize()
        torch.cuda.synchronize(self.bg.tiles.device)
        self.stage = self.stage_ids = self.stage_count = None
        self.host = self.host_ids = self.count = None
        self.gathered = self.copied = None
        self.copy_stream = None
        self.closed = True
        empty = getattr(torch._C, "_host_emptyCache", None)
        if empty is not None:
            empty()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False
