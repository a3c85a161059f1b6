"""MI355X-native checkerboard Metropolis Monte Carlo for the 2D q-state Potts model.

Thin Python layer over the C ABI of ``libpotts.so`` (include/potts.h).  Every
step of a sweep runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch is optional plumbing: ``Lattice.from_torch`` runs a state
on torch-allocated device buffers and a torch stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from ._native import (PottsBatchOpts, PottsError, PottsJob, PottsJobResult, PottsNnnObs, PottsObs, PottsRequest,
                      PottsServed, PottsServerCfg, PottsSummary, check, load)

ORDERED = 0
RANDOM = 1

__all__ = ["Lattice", "Cube", "NnnLattice", "Batch", "Server", "Slabs", "slab_half_sweep", "sweep_static", "PottsError", "threshold_table",
           "threshold_table6", "nnn_table", "ORDERED", "RANDOM", "load"]


def sweep_static(spins_ptr: int, L: int, q: int, seed: int, t0: int, thr, nsweeps: int, records_ptr: int,
                 stream_ptr: int = 0) -> None:
    """potts_sweep_static on device pointers (argument marshalling only): the
    allocation-free sweeps of a caller-owned row-major lattice, records of
    sweeps t0 .. t0+nsweeps-1 into the caller's nsweeps x (1+q) int64 buffer."""
    th = np.ascontiguousarray(thr, dtype=np.uint32)
    check(load().potts_sweep_static(ctypes.c_void_p(spins_ptr), int(L), int(q), int(seed), int(t0),
                                    th.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), int(nsweeps),
                                    ctypes.c_void_p(records_ptr), ctypes.c_void_p(stream_ptr)))


def threshold_table(beta: float) -> np.ndarray:
    """thr[d-1] = min(floor(exp(-beta d) 2^32), 2^32-1), d = 1..4 (host FP64)."""
    thr = np.zeros(4, dtype=np.uint32)
    check(load().potts_threshold_table(float(beta), thr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return thr


class Lattice:
    """One L x L Potts lattice resident on the GPU (a potts_state)."""

    def __init__(self, L: int, q: int, seed: int = 1, start: int = RANDOM, _handle=None, _keep=None):
        self._lib = load()
        self._h = ctypes.c_void_p()
        self._keep = _keep
        if _handle is not None:
            self._h = _handle
        else:
            check(self._lib.potts_init(int(L), int(q), int(seed), int(start), ctypes.byref(self._h)))
        self.L = int(L)
        self.q = int(q)
        self.seed = int(seed)

    @classmethod
    def from_torch(cls, L: int, q: int, seed: int = 1, start: int = RANDOM, device="cuda",
                   stream=None, records_capacity: int = 0) -> "Lattice":
        import torch

        a = torch.empty(L * L, dtype=torch.uint8, device=device)
        b = torch.empty(L * L, dtype=torch.uint8, device=device)
        st = stream if stream is not None else torch.cuda.current_stream(a.device)
        h = ctypes.c_void_p()
        check(load().potts_init_ex(L, q, seed, start, ctypes.c_void_p(a.data_ptr()),
                                   ctypes.c_void_p(b.data_ptr()), L * L,
                                   ctypes.c_void_p(st.cuda_stream), int(records_capacity),
                                   ctypes.byref(h)))
        return cls(L, q, seed, start, _handle=h, _keep=(a, b, st))

    @classmethod
    def on_stream(cls, L: int, q: int, seed: int = 1, start: int = RANDOM, stream=None,
                  records_capacity: int = 0) -> "Lattice":
        """A state whose buffers the library owns, working on a caller's stream
        (a torch.cuda.Stream, or None for the current one)."""
        import torch

        st = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check(load().potts_init_ex(L, q, seed, start, None, None, 0, ctypes.c_void_p(st.cuda_stream),
                                   int(records_capacity), ctypes.byref(h)))
        return cls(L, q, seed, start, _handle=h, _keep=(st,))

    @classmethod
    def load_checkpoint(cls, path: str) -> "Lattice":
        h = ctypes.c_void_p()
        check(load().potts_load(os.fsencode(path), ctypes.byref(h)))
        obj = cls.__new__(cls)
        obj._lib = load()
        obj._h = h
        obj._keep = None
        obs = PottsObs()
        check(obj._lib.potts_measure(h, ctypes.byref(obs)))
        obj.L, obj.q, obj.seed = int(obs.L), int(obs.q), -1
        return obj

    # -- sweeps -----------------------------------------------------------------
    def sweep(self, beta: float, nsweeps: int = 1) -> None:
        check(self._lib.potts_sweep(self._h, float(beta), int(nsweeps)))

    def sweep_heatbath(self, beta: float, nsweeps: int = 1) -> None:
        """Heat-bath sweeps (potts_sweep_heatbath); shares t and records with sweep()."""
        check(self._lib.potts_sweep_heatbath(self._h, float(beta), int(nsweeps)))

    def sweep_heatbath_thr(self, thr, nsweeps: int = 1) -> None:
        t = np.ascontiguousarray(thr, dtype=np.uint32)
        check(self._lib.potts_sweep_heatbath_thr(self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                                 int(nsweeps)))

    def sweep_thr(self, thr, nsweeps: int = 1) -> None:
        t = np.ascontiguousarray(thr, dtype=np.uint32)
        check(self._lib.potts_sweep_thr(self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), int(nsweeps)))

    def tune(self, kernel: int = 0, strip_rows: int = 0, max_groups: int = 0) -> None:
        """Launch shape (0 = automatic); results are identical for every choice."""
        check(self._lib.potts_tune(self._h, int(kernel), int(strip_rows), int(max_groups)))

    def tune_occupancy(self, waves_per_simd: int) -> None:
        """Colour-split kernel occupancy: 0 (compiler's choice) or 8 waves per SIMD."""
        check(self._lib.potts_tune_occupancy(self._h, int(waves_per_simd)))

    def tune_tiles(self, tx: int = 0, ty: int = 0, sweeps: int = 0) -> None:
        """Multi-sweep tile kernel (kernel 5) shape: tx x ty tiles, sweeps per
        launch (0 = automatic); results are identical for every shape."""
        check(self._lib.potts_tune_tiles(self._h, int(tx), int(ty), int(sweeps)))

    def tune_graph(self, sweeps: int) -> None:
        """Replay colour-split sweeps from a captured graph of `sweeps` sweeps (0: off)."""
        check(self._lib.potts_tune_graph(self._h, int(sweeps)))

    def tune_band(self, rows: int = 0, block: int = 0) -> None:
        """Band kernel (kernel 7) shape: rows per band and lanes per workgroup
        (0 = automatic); results are identical for every shape."""
        check(self._lib.potts_tune_band(self._h, int(rows), int(block)))

    @property
    def t(self) -> int:
        return int(self._lib.potts_time(self._h))

    # -- observables ------------------------------------------------------------
    def _obs(self, fn) -> dict:
        o = PottsObs()
        check(fn(self._h, ctypes.byref(o)))
        return {"t": o.t, "e_sat": o.e_sat, "nmax": o.nmax,
                "hist": np.array(o.hist[: self.q], dtype=np.int64)}

    def observables(self) -> dict:
        return self._obs(self._lib.potts_observables)

    def measure(self) -> dict:
        return self._obs(self._lib.potts_measure)

    def records(self, t0: int, n: int) -> np.ndarray:
        out = np.zeros((n, 1 + self.q), dtype=np.int64)
        check(self._lib.potts_records(self._h, int(t0), int(n), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return out

    def stats(self, t0: int, n: int, beta: float) -> dict:
        s = PottsSummary()
        check(self._lib.potts_stats(self._h, int(t0), int(n), float(beta), ctypes.byref(s)))
        return {"n": s.n, "e": s.e, "C": s.C, "V_L": s.V_L, "m": s.m, "chi": s.chi}

    def reweight(self, t0: int, n: int, beta0: float, betas) -> list:
        """Observables at each of `betas` from the records of sweeps t0 .. t0+n-1
        sampled at beta0 (temperature reweighting)."""
        b = np.ascontiguousarray(betas, dtype=np.float64)
        out = (PottsSummary * len(b))()
        check(self._lib.potts_reweight(self._h, int(t0), int(n), float(beta0),
                                       b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(b), out))
        return [{"n": s.n, "e": s.e, "C": s.C, "V_L": s.V_L, "m": s.m, "chi": s.chi} for s in out]

    def reserve_records(self, capacity: int) -> None:
        check(self._lib.potts_reserve_records(self._h, int(capacity)))

    def ramp(self, betas, t_equil: int, t_meas: int) -> list:
        """Runs t_equil + t_meas sweeps at each beta in turn (state carried over)
        and returns the derived statistics of each point's last t_meas sweeps."""
        b = np.ascontiguousarray(betas, dtype=np.float64)
        out = (PottsSummary * len(b))()
        check(self._lib.potts_ramp(self._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(b),
                                   int(t_equil), int(t_meas), out))
        return [{"n": o.n, "e": o.e, "C": o.C, "V_L": o.V_L, "m": o.m, "chi": o.chi} for o in out]

    # -- lattice access -----------------------------------------------------------
    def spins(self) -> np.ndarray:
        out = np.zeros(self.L * self.L, dtype=np.uint8)
        check(self._lib.potts_get_spins(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out.reshape(self.L, self.L)

    def set_spins(self, spins: np.ndarray, t: int) -> None:
        a = np.ascontiguousarray(spins, dtype=np.uint8).ravel()
        if a.size != self.L * self.L:
            raise ValueError("lattice size mismatch")
        check(self._lib.potts_set_spins(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(t)))

    def device_ptr(self) -> int:
        return int(self._lib.potts_device_spins(self._h) or 0)

    def stream_ptr(self) -> int:
        """The state's hipStream_t as an integer."""
        return int(self._lib.potts_stream(self._h) or 0)

    def save(self, path: str) -> None:
        check(self._lib.potts_save(self._h, os.fsencode(path)))

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            self._lib.potts_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def threshold_table6(beta: float) -> np.ndarray:
    """thr[d-1] = min(floor(exp(-beta d) 2^32), 2^32-1), d = 1..6: the table of
    the simple-cubic lattice (host FP64)."""
    thr = np.zeros(6, dtype=np.uint32)
    check(load().potts3d_threshold_table(float(beta), thr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return thr


class Cube:
    """One L x L x L simple-cubic Potts lattice on the GPU (a potts3d_state):
    the checkerboard Metropolis sweep with colour (x + y + z) & 1 and six
    neighbours, records and statistics as for Lattice with N = L^3."""

    def __init__(self, L: int, q: int, seed: int = 1, start: int = RANDOM):
        self._lib = load()
        self._h = ctypes.c_void_p()
        check(self._lib.potts3d_init(int(L), int(q), int(seed), int(start), ctypes.byref(self._h)))
        self.L = int(L)
        self.q = int(q)
        self.seed = int(seed)

    def sweep(self, beta: float, nsweeps: int = 1) -> None:
        check(self._lib.potts3d_sweep(self._h, float(beta), int(nsweeps)))

    def sweep_thr(self, thr, nsweeps: int = 1) -> None:
        t = np.ascontiguousarray(thr, dtype=np.uint32)
        if t.size != 6:
            raise ValueError("the cubic table has six entries")
        check(self._lib.potts3d_sweep_thr(self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                          int(nsweeps)))

    def tune(self, kernel: int = 0, rows: int = 0) -> None:
        """0 automatic, 1 colour-split (L % 32 == 0), 2 chunk; results are identical."""
        check(self._lib.potts3d_tune(self._h, int(kernel), int(rows)))

    @property
    def t(self) -> int:
        return int(self._lib.potts3d_time(self._h))

    def stream_handle(self) -> int:
        """The state's hipStream_t as an integer (for torch.cuda.ExternalStream)."""
        return int(self._lib.potts3d_stream(self._h) or 0)

    def observables(self) -> dict:
        o = PottsObs()
        check(self._lib.potts3d_observables(self._h, ctypes.byref(o)))
        return {"t": o.t, "e_sat": o.e_sat, "nmax": o.nmax,
                "hist": np.array(o.hist[: self.q], dtype=np.int64)}

    def records(self, t0: int, n: int) -> np.ndarray:
        out = np.zeros((n, 1 + self.q), dtype=np.int64)
        check(self._lib.potts3d_records(self._h, int(t0), int(n),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return out

    def stats(self, t0: int, n: int, beta: float) -> dict:
        s = PottsSummary()
        check(self._lib.potts3d_stats(self._h, int(t0), int(n), float(beta), ctypes.byref(s)))
        return {"n": s.n, "e": s.e, "C": s.C, "V_L": s.V_L, "m": s.m, "chi": s.chi}

    def spins(self) -> np.ndarray:
        """The lattice as an array indexed [z, y, x]."""
        out = np.zeros(self.L ** 3, dtype=np.uint8)
        check(self._lib.potts3d_get_spins(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out.reshape(self.L, self.L, self.L)

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            self._lib.potts3d_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def nnn_table(beta: float, j2: float) -> np.ndarray:
    """The 81 acceptance entries of the first-plus-second-neighbour lattice,
    index (d1 + 4) * 9 + (d2 + 4) (host FP64)."""
    thr = np.zeros(81, dtype=np.uint64)
    check(load().potts_nnn_table(float(beta), float(j2), thr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return thr


class NnnLattice:
    """One L x L lattice with nearest (coupling 1) and diagonal (coupling j2)
    neighbours on the GPU (a potts_nnn_state): nine colour passes per sweep,
    records {e1, e2, hist}."""

    def __init__(self, L: int, q: int, seed: int = 1, start: int = RANDOM):
        self._lib = load()
        self._h = ctypes.c_void_p()
        check(self._lib.potts_nnn_init(int(L), int(q), int(seed), int(start), ctypes.byref(self._h)))
        self.L = int(L)
        self.q = int(q)
        self.seed = int(seed)

    def sweep(self, beta: float, j2: float, nsweeps: int = 1) -> None:
        check(self._lib.potts_nnn_sweep(self._h, float(beta), float(j2), int(nsweeps)))

    def sweep_thr(self, thr, nsweeps: int = 1) -> None:
        t = np.ascontiguousarray(thr, dtype=np.uint64)
        if t.size != 81:
            raise ValueError("the table has 81 entries")
        check(self._lib.potts_nnn_sweep_thr(self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                            int(nsweeps)))

    def tune(self, kernel: int = 0) -> None:
        """0 automatic, 1 row class staged in LDS (L <= 16380), 2 one launch
        per colour; all give identical results."""
        check(self._lib.potts_nnn_tune(self._h, int(kernel)))

    @property
    def t(self) -> int:
        return int(self._lib.potts_nnn_time(self._h))

    def stream_handle(self) -> int:
        return int(self._lib.potts_nnn_stream(self._h) or 0)

    def observables(self) -> dict:
        o = PottsNnnObs()
        check(self._lib.potts_nnn_observables(self._h, ctypes.byref(o)))
        return {"t": o.t, "e1": o.e1, "e2": o.e2, "nmax": o.nmax,
                "hist": np.array(o.hist[: self.q], dtype=np.int64)}

    def records(self, t0: int, n: int) -> np.ndarray:
        out = np.zeros((n, 2 + self.q), dtype=np.int64)
        check(self._lib.potts_nnn_records(self._h, int(t0), int(n),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return out

    def spins(self) -> np.ndarray:
        out = np.zeros(self.L * self.L, dtype=np.uint8)
        check(self._lib.potts_nnn_get_spins(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out.reshape(self.L, self.L)

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            self._lib.potts_nnn_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many independent lattices swept together (potts_batch_*).  jobs: dicts
    with L, q, seed, start, beta, nsweeps.  Each job gives exactly the bits it
    gives alone."""

    def __init__(self, jobs, graph: bool = True, tune: bool = True, window: int = 0, strip_rows: int = 0,
                 stream=None, tune_cache: Optional[str] = None):
        self._lib = load()
        arr = (PottsJob * len(jobs))()
        for a, j in zip(arr, jobs):
            a.L, a.q, a.seed, a.start = int(j["L"]), int(j["q"]), int(j["seed"]), int(j["start"])
            a.beta, a.nsweeps = float(j["beta"]), int(j["nsweeps"])
        self.jobs = [dict(j) for j in jobs]
        self._cache = os.fsencode(tune_cache) if tune_cache else None  # kept alive for the library
        opts = PottsBatchOpts(int(graph), int(tune), int(window), int(strip_rows),
                              ctypes.c_void_p(stream.cuda_stream) if stream is not None else None, self._cache)
        self._h = ctypes.c_void_p()
        check(self._lib.potts_batch_create(arr, len(jobs), ctypes.byref(opts), ctypes.byref(self._h)))

    def run(self) -> float:
        """Runs every job for its nsweeps (more) sweeps; returns the device time in ms."""
        check(self._lib.potts_batch_run(self._h))
        return float(self._lib.potts_batch_elapsed_ms(self._h))

    def results(self) -> list:
        out = (PottsJobResult * len(self.jobs))()
        check(self._lib.potts_batch_results(self._h, out))
        return [{"t": r.t, "e_sat": r.e_sat, "nmax": r.nmax, "e": r.stats.e, "C": r.stats.C,
                 "V_L": r.stats.V_L, "m": r.stats.m, "chi": r.stats.chi, "n": r.stats.n} for r in out]

    def records(self, job: int, t0: int, n: int) -> np.ndarray:
        q = int(self.jobs[job]["q"])
        out = np.zeros((n, 1 + q), dtype=np.int64)
        check(self._lib.potts_batch_records(self._h, int(job), int(t0), int(n),
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return out

    def spins(self, job: int) -> np.ndarray:
        L = int(self.jobs[job]["L"])
        out = np.zeros(L * L, dtype=np.uint8)
        check(self._lib.potts_batch_spins(self._h, int(job), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out.reshape(L, L)

    def tuning(self) -> str:
        return (self._lib.potts_batch_tuning(self._h) or b"").decode()

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            self._lib.potts_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Serving loop with continuous batching (potts_server_*): submit jobs (a
    beta schedule each) while earlier ones run; results are bit-identical to
    the same job run alone."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 0, quantum: int = 0, stream=None,
                 tune: bool = False, tune_cache: Optional[str] = None):
        self._lib = load()
        self._cache = os.fsencode(tune_cache) if tune_cache else None  # kept alive for the library
        cfg = PottsServerCfg(int(hbm_budget), int(max_slots), int(quantum),
                             ctypes.c_void_p(stream.cuda_stream) if stream is not None else None,
                             int(tune), 0, self._cache)
        self._h = ctypes.c_void_p()
        check(self._lib.potts_server_start(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._npoints = {}
        self._L = {}

    def submit(self, L: int, q: int, seed: int, start: int, betas, sweeps, keep_spins: bool = False,
               checkpoint: Optional[str] = None, resume_from: Optional[str] = None) -> int:
        """Queues a job; `checkpoint`: a file the server rewrites after each
        completed point; `resume_from`: such a file of the same job, to
        continue from."""
        b = np.ascontiguousarray(betas, dtype=np.float64)
        n = np.ascontiguousarray(sweeps, dtype=np.int64)
        if b.size != n.size:
            raise ValueError("one sweep count per beta")
        req = PottsRequest(int(L), int(q), int(seed), int(start), int(b.size),
                           b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(keep_spins), 0,
                           os.fsencode(checkpoint) if checkpoint else None,
                           os.fsencode(resume_from) if resume_from else None)
        t = ctypes.c_int64()
        check(self._lib.potts_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._npoints[t.value] = int(b.size)
        self._L[t.value] = int(L)
        return int(t.value)

    def wait(self, max_n: int = 256, timeout_ms: int = -1) -> list:
        buf = (ctypes.c_int64 * max_n)()
        n = ctypes.c_int32()
        check(self._lib.potts_server_wait(self._h, buf, int(max_n), int(timeout_ms), ctypes.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def inject_fault(self, ticket: int, at_sweep: int) -> None:
        """Makes the job fail (status EDEVICE) before it runs sweep at_sweep
        (host-side failure injection for recovery tests); ticket 0: the next
        job submitted, attached at its submission."""
        check(self._lib.potts_server_inject_fault(self._h, int(ticket), int(at_sweep)))

    def collect(self, ticket: int, spins: bool = False) -> dict:
        """A finished job's results; a job that failed is returned with its
        negative status (an unknown ticket raises)."""
        info = PottsServed()
        npts = self._npoints.pop(ticket)
        L = self._L.pop(ticket)
        pts = (PottsSummary * npts)()
        sp = np.zeros(L * L, dtype=np.uint8) if spins else None
        rc = self._lib.potts_server_collect(self._h, int(ticket), ctypes.byref(info), pts,
                                            sp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if spins else None)
        if rc != 0 and info.ticket != ticket:
            check(rc)
        return {"ticket": info.ticket, "L": info.L, "q": info.q, "status": info.status, "sweeps": info.sweeps,
                "t_submit": info.t_submit, "t_admit": info.t_admit, "t_done": info.t_done,
                "e_sat": info.e_sat, "nmax": info.nmax,
                "points": [{"n": p.n, "e": p.e, "C": p.C, "V_L": p.V_L, "m": p.m, "chi": p.chi} for p in pts],
                "spins": sp.reshape(L, L) if spins else None}

    def drain(self, timeout_ms: int = -1) -> None:
        check(self._lib.potts_server_drain(self._h, int(timeout_ms)))

    def now(self) -> float:
        return float(self._lib.potts_server_now(self._h))

    def iterations(self) -> int:
        return int(self._lib.potts_server_iterations(self._h))

    def tuning(self) -> str:
        """The launch shapes in use (timed by this server or read from its cache)."""
        buf = ctypes.create_string_buffer(4096)
        check(self._lib.potts_server_tuning(self._h, buf, len(buf)))
        return buf.value.decode()

    def stop(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            rc = self._lib.potts_server_stop(self._h)
            self._h = ctypes.c_void_p()
            check(rc)

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


from .slabs import Slabs, slab_half_sweep  # noqa: E402
