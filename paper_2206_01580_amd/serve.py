"""Continuous batching of energy + force requests.

The paper's prediction timings show that batching many configurations raises
GPU utilisation by orders of magnitude (Timings section: one ethanol
configuration vs 1000 in one call); single small molecules leave most of the
device idle. This module serves a stream of requests of uneven size:

* requests (atoms' representations, element ids, Jacobian blocks) are staged
  in device memory before the clock starts;
* the scheduler admits arrived requests in FIFO order while the memory budget
  for in-flight work allows, packs a contiguous run of them into one CSR batch
  (zero-copy views of the staged pool) and launches ``sorf_predict`` on one of
  several streams without waiting; completions are detected by polling;
* the plain reference path runs one molecule per launch sequence, in arrival
  order, on one stream.

The scheduler is independent of the executor so that its admission and
accounting logic can be tested on the CPU with a mock executor.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np


# --------------------------------------------------------------------------
# Scheduler (device independent)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class ServeStats:
    latency_s: np.ndarray          # completion - arrival, per request
    completion_s: np.ndarray       # completion time since the trace start
    batches: List[tuple]           # (first request, last request + 1) per launch
    wall_s: float                  # trace start to last completion
    atoms: int
    rejected: List[int]            # requests that can never fit the budget
    inflight_at_launch: List[int] = dataclasses.field(default_factory=list)
    # batches already on the device when each launch was made (continuous
    # batching admits new work while earlier batches run)

    def summary(self, warmup_s: float = 0.0, arrivals: Optional[np.ndarray] = None) -> dict:
        lat = self.latency_s
        keep = np.ones(len(lat), bool)
        if arrivals is not None and warmup_s > 0:
            keep = arrivals >= warmup_s
        lat = lat[keep & np.isfinite(lat)]
        return {
            "requests": int(keep.sum()),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
            "mean_ms": float(lat.mean() * 1e3) if len(lat) else None,
            "atoms_per_s": self.atoms / self.wall_s if self.wall_s > 0 else None,
            "launches": len(self.batches),
            "mean_batch_requests": float(np.mean([b - a for a, b in self.batches])) if self.batches else 0.0,
            "rejected": len(self.rejected),
            "launches_beside_inflight": int(sum(1 for c in self.inflight_at_launch if c > 0)),
        }


class BatchingScheduler:
    """FIFO admission into contiguous batches under an in-flight memory budget.

    executor.submit(first, last) starts requests [first, last) and returns a
    handle with ``done() -> bool``; executor.bytes_for(first, last) is the
    device memory the batch holds until it completes."""

    def __init__(self, executor, max_batch_atoms: int, max_inflight: int, mem_budget: int,
                 clock: Callable[[], float] = time.perf_counter, idle: Callable[[], None] = None,
                 max_batch_requests: Optional[int] = None):
        self.ex = executor
        self.max_batch_atoms = max_batch_atoms
        self.max_inflight = max_inflight
        self.mem_budget = mem_budget
        self.max_batch_requests = max_batch_requests
        self.clock = clock
        self.idle = idle or (lambda: None)

    def run(self, arrivals: Sequence[float], sizes: Sequence[int]) -> ServeStats:
        arrivals = np.asarray(arrivals, dtype=np.float64)
        sizes = np.asarray(sizes, dtype=np.int64)
        R = len(arrivals)
        completion = np.full(R, np.nan)
        pending = collections.deque()
        inflight = collections.deque()       # (handle, first, last, bytes)
        used = 0
        batches, rejected, beside = [], [], []
        nxt = 0
        t0 = self.clock()
        finished = 0
        while finished + len(rejected) < R:
            now = self.clock() - t0
            while nxt < R and arrivals[nxt] <= now:
                pending.append(nxt)
                nxt += 1
            # retire completed batches (in launch order per stream is not
            # required: any finished batch frees its memory)
            progressed = False
            for _ in range(len(inflight)):
                h, a, b, nbytes = inflight.popleft()
                if h.done():
                    t = self.clock() - t0
                    completion[a:b] = t
                    used -= nbytes
                    finished += b - a
                    progressed = True
                else:
                    inflight.append((h, a, b, nbytes))
            # admit a contiguous FIFO run
            if pending and len(inflight) < self.max_inflight:
                first = pending[0]
                if self.ex.bytes_for(first, first + 1) > self.mem_budget:
                    pending.popleft()          # can never be admitted
                    rejected.append(first)
                    completion[first] = np.inf
                    continue
                last = first
                atoms = 0
                while pending and pending[0] == last:
                    n = int(sizes[last])
                    if last > first and atoms + n > self.max_batch_atoms:
                        break
                    if self.max_batch_requests is not None and last - first >= self.max_batch_requests:
                        break
                    if used + self.ex.bytes_for(first, last + 1) > self.mem_budget:
                        break
                    atoms += n
                    pending.popleft()
                    last += 1
                if last > first:
                    nbytes = self.ex.bytes_for(first, last)
                    beside.append(len(inflight))
                    h = self.ex.submit(first, last)
                    inflight.append((h, first, last, nbytes))
                    used += nbytes
                    batches.append((first, last))
                    progressed = True
            if not progressed:
                self.idle()
        wall = np.nanmax(completion[np.isfinite(completion)]) if np.isfinite(completion).any() else 0.0
        lat = completion - arrivals
        done_atoms = int(sizes[np.isfinite(completion)].sum())
        return ServeStats(lat, completion, batches, float(wall), done_atoms, rejected, beside)


class PlainRunner:
    """One molecule per launch sequence, FIFO, one stream: submit, wait, next."""

    def __init__(self, executor, clock: Callable[[], float] = time.perf_counter,
                 idle: Callable[[], None] = None):
        self.ex = executor
        self.clock = clock
        self.idle = idle or (lambda: None)

    def run(self, arrivals, sizes) -> ServeStats:
        arrivals = np.asarray(arrivals, dtype=np.float64)
        sizes = np.asarray(sizes, dtype=np.int64)
        R = len(arrivals)
        completion = np.full(R, np.nan)
        t0 = self.clock()
        for r in range(R):
            while self.clock() - t0 < arrivals[r]:
                self.idle()
            h = self.ex.submit(r, r + 1)
            while not h.done():
                self.idle()
            completion[r] = self.clock() - t0
        wall = float(completion[-1]) if R else 0.0
        return ServeStats(completion - arrivals, completion, [(r, r + 1) for r in range(R)], wall,
                          int(sizes.sum()), [])


# --------------------------------------------------------------------------
# GPU executor
# --------------------------------------------------------------------------

class RequestPool:
    """Staged requests: x [A, d], element [A], per-request atom offsets and
    Jacobian block offsets into a device buffer J (blocks [N, d, 3N])."""

    def __init__(self, x, element, sizes, J, J_off, device="cuda"):
        import torch
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.atom_ptr = np.zeros(len(sizes) + 1, dtype=np.int64)
        np.cumsum(self.sizes, out=self.atom_ptr[1:])
        self.x = x if isinstance(x, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(device)
        self.element = element if isinstance(element, torch.Tensor) else \
            torch.from_numpy(np.ascontiguousarray(element, np.int32)).to(device)
        self.J = J
        self.J_off = np.asarray(J_off, dtype=np.int64)   # float offset of each request's block
        self.d = int(self.x.shape[1])


class _Handle:
    def __init__(self, event, slot, ex):
        self.event, self.slot, self.ex = event, slot, ex
        self._done = False

    def done(self) -> bool:
        if not self._done and self.event.query():
            self._done = True
            self.ex._release(self.slot)
        return self._done


class GpuExecutor:
    """Launches sorf_predict (energies and forces) for a contiguous run of
    staged requests on one of ``n_slots`` streams. Each slot owns pinned host
    and device buffers sized for ``max_batch_atoms`` / ``max_batch_reqs``."""

    def __init__(self, model, alpha, pool: RequestPool, max_batch_atoms: int,
                 max_batch_reqs: int, n_slots: int, device="cuda", copy_back: bool = True):
        import torch
        from . import sorf
        self.torch, self.sorf = torch, sorf
        self.model, self.alpha, self.pool = model, alpha, pool
        self.copy_back = copy_back
        self.slots = []
        for _ in range(n_slots):
            st = torch.cuda.Stream(device=device)       # default priority
            slot = dict(
                stream=st,
                ptr_h=torch.empty(max_batch_reqs + 1, dtype=torch.int64, pin_memory=True),
                jptr_h=torch.empty(max_batch_reqs + 1, dtype=torch.int64, pin_memory=True),
                ptr_d=torch.empty(max_batch_reqs + 1, dtype=torch.int64, device=device),
                jptr_d=torch.empty(max_batch_reqs + 1, dtype=torch.int64, device=device),
                E=torch.empty(max_batch_reqs, dtype=torch.float32, device=device),
                F=torch.empty(3 * max_batch_atoms, dtype=torch.float32, device=device),
                E_h=torch.empty(max_batch_reqs, dtype=torch.float32, pin_memory=True),
                F_h=torch.empty(3 * max_batch_atoms, dtype=torch.float32, pin_memory=True),
                pred=sorf.Predictor(model, device),
                event=torch.cuda.Event(),
            )
            with torch.cuda.stream(st):
                slot["pred"]._workspace(max_batch_atoms, max_batch_reqs)   # allocate once
            self.slots.append(slot)
        self.free = collections.deque(range(n_slots))
        self.ws_per_atom = 4 * (pool.d + 1) + 12
        self.results = {}

    def bytes_for(self, first: int, last: int) -> int:
        n = int(self.pool.atom_ptr[last] - self.pool.atom_ptr[first])
        return n * self.ws_per_atom + 4 * (last - first)

    def _release(self, s):
        slot = self.slots[s]
        if slot.get("pending") is not None:
            a, b = slot["pending"]
            if self.copy_back:
                self.results[(a, b)] = (slot["E_h"][: b - a].numpy().copy(),
                                        slot["F_h"][: 3 * int(self.pool.atom_ptr[b] - self.pool.atom_ptr[a])].numpy().copy())
            slot["pending"] = None
        self.free.append(s)

    def submit(self, first: int, last: int) -> _Handle:
        torch, sorf, pool = self.torch, self.sorf, self.pool
        while not self.free:           # the scheduler never asks for more slots than exist
            for s in self.slots:
                if s.get("handle") is not None:
                    s["handle"].done()
        s = self.free.popleft()
        slot = self.slots[s]
        a0, a1 = int(pool.atom_ptr[first]), int(pool.atom_ptr[last])
        nreq, nat = last - first, a1 - a0
        slot["ptr_h"][: nreq + 1] = torch.from_numpy(pool.atom_ptr[first:last + 1] - a0)
        # J block offsets of the batch, relative to the first request's block
        jo = pool.J_off[first:last]
        jsz = pool.sizes[first:last] * pool.d * 3 * pool.sizes[first:last]
        base = int(jo.min()) if nreq else 0
        jptr = np.empty(nreq + 1, dtype=np.int64)
        jptr[:-1] = jo - base
        jptr[-1] = int((jo + jsz).max()) - base
        slot["jptr_h"][: nreq + 1] = torch.from_numpy(jptr)
        st = slot["stream"]
        with torch.cuda.stream(st):
            slot["ptr_d"][: nreq + 1].copy_(slot["ptr_h"][: nreq + 1], non_blocking=True)
            slot["jptr_d"][: nreq + 1].copy_(slot["jptr_h"][: nreq + 1], non_blocking=True)
            batch = sorf.Batch(pool.x[a0:a1], pool.element[a0:a1], slot["ptr_d"][: nreq + 1])
            Jview = pool.J[base:]
            slot["pred"](batch, self.alpha, Jview, slot["jptr_d"][: nreq + 1],
                         E=slot["E"][:nreq], F=slot["F"][: 3 * nat])
            if self.copy_back:
                slot["E_h"][:nreq].copy_(slot["E"][:nreq], non_blocking=True)
                slot["F_h"][: 3 * nat].copy_(slot["F"][: 3 * nat], non_blocking=True)
            slot["event"].record(st)
        slot["pending"] = (first, last)
        h = _Handle(slot["event"], s, self)
        slot["handle"] = h
        return h


def request_results(executor: GpuExecutor, sizes) -> dict:
    """Per-request (E, F) from the batches an executor completed."""
    out = {}
    for (a, b), (E, F) in executor.results.items():
        off = 0
        for r in range(a, b):
            n = int(sizes[r])
            out[r] = (float(E[r - a]), F[3 * off: 3 * (off + n)].copy())
            off += n
    return out


# --------------------------------------------------------------------------
# Native executor: the library's persistent serving kernel
# --------------------------------------------------------------------------

class _ServerHandle:
    def __init__(self, server, ticket, first, last):
        self.server, self.ticket, self.first, self.last = server, ticket, first, last
        self._done = False

    def done(self) -> bool:
        if not self._done:
            q = self.server.lib.sorf_server_query(self.server.h, self.ticket)
            if q < 0:
                raise RuntimeError(f"serving kernel exited before batch {self.ticket} (query {q})")
            if q == 1:
                self.server._collect(self)
                self._done = True
        return self._done


class NativeServer:
    """Executor over sorf_server_*: one persistent kernel resident on the GPU
    takes batches from a ring in host-coherent memory (a descriptor write per
    batch, no launch, copy or event) and writes energies and forces straight
    into host-coherent result slots. Batches are runs of contiguous requests
    of the staged pool, as the scheduler forms them; at most ``ring_slots``
    are in flight and each holds at most 64 requests."""

    MAX_REQUESTS = 64

    def __init__(self, model, alpha, pool: RequestPool, max_batch_atoms: int, ring_slots: int = 8,
                 idle_timeout_s: float = 60.0, device="cuda", copy_back: bool = True):
        import ctypes
        import torch
        from . import _lib
        self.ctypes, self.lib, self._lib = ctypes, _lib.load(), _lib
        self.pool, self.copy_back = pool, copy_back
        self.ring_slots = ring_slots
        self.max_batch_atoms = max_batch_atoms
        cfg = _lib.SorfServerConfig(max_batch_atoms, ring_slots, idle_timeout_s)
        m = model.c_struct()
        nbytes = self.lib.sorf_server_workspace_bytes(ctypes.byref(m), ctypes.byref(cfg))
        if nbytes == 0:
            raise ValueError("invalid model or server configuration")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ws = self.ws.data_ptr() + ((-self.ws.data_ptr()) % 256)
        self.stream = torch.cuda.Stream(device=device)     # default priority
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _lib.check("sorf_server_start", self.lib.sorf_server_start(
            ctypes.byref(m), alpha.data_ptr(), pool.x.data_ptr(), pool.element.data_ptr(),
            pool.J.data_ptr(), ctypes.byref(cfg), ws, nbytes, self.stream.cuda_stream,
            ctypes.byref(h)))
        self.h = h
        self._keep = (model, alpha, pool)
        self.results = {}
        self._ticket = ctypes.c_int64()

    def bytes_for(self, first: int, last: int) -> int:
        """Result-slot bytes a batch holds until it is collected."""
        n = int(self.pool.atom_ptr[last] - self.pool.atom_ptr[first])
        return 12 * n + 4 * (last - first)

    def slot_bytes(self) -> int:
        return 12 * self.max_batch_atoms + 4 * self.MAX_REQUESTS

    def submit(self, first: int, last: int) -> _ServerHandle:
        ctypes, pool = self.ctypes, self.pool
        ao = np.ascontiguousarray(pool.atom_ptr[first:last + 1], dtype=np.int64)
        jo = np.ascontiguousarray(pool.J_off[first:last], dtype=np.int64)
        rc = self.lib.sorf_server_submit(self.h, last - first, ao.ctypes.data, jo.ctypes.data,
                                         ctypes.byref(self._ticket))
        self._lib.check("sorf_server_submit", rc)
        return _ServerHandle(self, self._ticket.value, first, last)

    def _collect(self, hnd: _ServerHandle):
        if not self.copy_back:
            return
        n_req = hnd.last - hnd.first
        n_at = int(self.pool.atom_ptr[hnd.last] - self.pool.atom_ptr[hnd.first])
        e = self.lib.sorf_server_energies(self.h, hnd.ticket)
        f = self.lib.sorf_server_forces(self.h, hnd.ticket)
        self.results[(hnd.first, hnd.last)] = (np.ctypeslib.as_array(e, shape=(n_req,)).copy(),
                                              np.ctypeslib.as_array(f, shape=(3 * n_at,)).copy())

    def stop(self) -> int:
        """Stops the kernel (after the published batches); returns its exit state."""
        if self.h is None:
            return 0
        st = self.ctypes.c_int32(0)
        rc = self.lib.sorf_server_stop(self.h, self.ctypes.byref(st))
        self.h = None
        self._lib.check("sorf_server_stop", rc)
        return int(st.value)
