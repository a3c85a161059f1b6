"""Row slabs: the share of one device when an L x L lattice is split into G
horizontal slabs of h = L/G rows (Sec. 3: the checkerboard update needs only
the rows next to a slab, so each half sweep exchanges one halo row per side).

``Slabs`` holds every slab of such a split on one device and runs the
protocol a row-sharded run follows on each of its devices: before every half
sweep, copy the neighbouring slabs' edge rows into the halo rows; then sweep
each slab with ``potts_slab_half_sweep``.  The copies stand in for the
point-to-point transfers between devices.  Since the random words are keyed
by global (x, y, t), the result is the bits of ``Lattice.sweep`` for any G.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._native import check, load


def slab_half_sweep(slab_ptr: int, L: int, h: int, y0: int, q: int, seed: int, t: int, colour: int,
                    thr, ring_ptr: int, ring_slots: int, stream_ptr: int) -> None:
    """potts_slab_half_sweep on device pointers (argument marshalling only)."""
    th = np.ascontiguousarray(thr, dtype=np.uint32)
    check(load().potts_slab_half_sweep(ctypes.c_void_p(slab_ptr), int(L), int(h), int(y0), int(q), int(seed),
                                       int(t), int(colour), th.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                       ctypes.c_void_p(ring_ptr), int(ring_slots), ctypes.c_void_p(stream_ptr)))


class Slabs:
    """G row slabs of one L x L lattice, each stored as (h+2) x L bytes with its
    halos, and one record ring per slab (records summed over slabs on read)."""

    def __init__(self, L: int, q: int, seed: int = 1, start: int = 1, nslabs: int = 2,
                 ring_slots: int = 64, device="cuda"):
        import torch

        from . import Lattice

        if nslabs < 1 or L % nslabs or (L // nslabs) % 2:
            raise ValueError("L must split into nslabs slabs of an even number of rows")
        if ring_slots < 2 or ring_slots & (ring_slots - 1):
            raise ValueError("ring_slots must be a power of two >= 2")
        self.L, self.q, self.seed, self.G, self.h = int(L), int(q), int(seed), int(nslabs), int(L) // int(nslabs)
        self.slots = int(ring_slots)
        self.t = 0
        h = self.h
        with Lattice.from_torch(L, q, seed, start, device=device) as lat:
            a, b, _ = lat._keep
            cur = a if lat.device_ptr() == a.data_ptr() else b
            torch.cuda.current_stream(a.device).synchronize()
            grid = cur.view(L, L)
            self.buf = []
            for g in range(self.G):
                s = torch.empty((h + 2, L), dtype=torch.uint8, device=device)
                s[1:h + 1].copy_(grid[g * h:(g + 1) * h])
                self.buf.append(s)
            torch.cuda.current_stream(a.device).synchronize()
        # the G rings one after another, as potts_slab_records reads them
        self.ring_store = torch.zeros((self.G, self.slots, q + 1), dtype=torch.int64, device=device)
        self.rings = [self.ring_store[g] for g in range(self.G)]

    def _exchange(self) -> None:
        G, h = self.G, self.h
        for g in range(G):
            self.buf[g][0].copy_(self.buf[(g - 1) % G][h])
            self.buf[g][h + 1].copy_(self.buf[(g + 1) % G][1])

    def sweep(self, beta: float, nsweeps: int = 1, thr=None) -> None:
        import torch

        from . import threshold_table

        th = threshold_table(beta) if thr is None else np.ascontiguousarray(thr, dtype=np.uint32)
        stream = torch.cuda.current_stream(self.buf[0].device).cuda_stream
        for _ in range(int(nsweeps)):
            for colour in (0, 1):
                self._exchange()
                for g in range(self.G):
                    slab_half_sweep(self.buf[g].data_ptr(), self.L, self.h, g * self.h, self.q, self.seed,
                                    self.t, colour, th, self.rings[g].data_ptr(), self.slots, stream)
            self.t += 1

    def records(self, t0: int, n: int) -> np.ndarray:
        """Records of sweeps t0 .. t0+n-1, summed over the slabs by
        potts_slab_records (the last ring_slots - 1 sweeps are kept)."""
        import torch

        if t0 < max(0, self.t - self.slots + 1) or t0 + n > self.t:
            raise ValueError("records not in the rings")
        out = torch.empty((n, self.q + 1), dtype=torch.int64, device=self.ring_store.device)
        stream = torch.cuda.current_stream(out.device).cuda_stream
        check(load().potts_slab_records(ctypes.c_void_p(self.ring_store.data_ptr()), self.G, self.slots, self.q,
                                        int(t0), int(n), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
        return out.cpu().numpy()

    def spins(self) -> np.ndarray:
        import torch

        return torch.cat([b[1:self.h + 1] for b in self.buf]).cpu().numpy()
