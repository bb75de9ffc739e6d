"""Continuous-batching request loop over the batched Yee stepper.

Requests (one workload each) arrive over time.  Between replays of the
batched stepper (``steps_per_replay`` leapfrog steps of every admitted grid,
replayed from a HIP graph) the server
  * retires finished requests (results copied to the host),
  * admits waiting requests that have arrived, in arrival order, as long as a
    slot is free, the sum of admitted workspace footprints stays within the
    HBM budget and, if ``max_active_cells`` is set, the cells of the admitted
    grids stay within it (a request is always admitted when nothing runs).
    The cell cap bounds how many grids share the device, so a large request
    is not slowed by many concurrent ones while small ones still batch.
Field state stays resident on the device for the life of a request.  A
request may carry initial fields.  When it finishes, the run's health is
checked (``yee_status_flags``: a non-finite value, an FP16 overflow); a
failing request gets ``status`` and ``error`` set and does not disturb the
others.

Between replays the server also
  * cancels requests (``cancel(rid)``, or a ``deadline`` in seconds after
    arrival that has passed): a running one is retired at once and its slot
    freed, a waiting one is dropped;
  * every ``checkpoint_every`` replays, saves the state of each running
    request (``yee_save_state``) into a device buffer of its own;
  * after a device reset (simulated from the host by destroying the batch and
    every in-flight context, ``reset_after_replays``), re-queues the
    in-flight requests at the front of the queue; each resumes from its last
    checkpoint (``yee_load_state``), or from the start if it has none.  A
    resumed request's fields and probe series equal those of an
    uninterrupted run bitwise.
The plain alternative, :func:`serve_one_at_a_time`, solves requests first
come first served with one ``yee_step`` call each.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import _lib
from .solver import YeeSolver
from .workloads import Workload


# Default cap on the cells of the grids admitted at once: about two of the
# largest serving requests (160^3 = 4.1 M cells), which keeps the device busy
# while bounding how many requests share it (measured best of 4 M, 8 M, 16 M
# and no cap for p50 and p99 latency at 0.8x and 1.2x the one-at-a-time
# capacity).
DEFAULT_ACTIVE_CELLS = 8_000_000


@dataclass
class Request:
    wl: Workload
    arrival: float = 0.0                      # seconds after the start of the run
    rid: int = 0
    admitted: Optional[float] = None
    finished: Optional[float] = None
    series: Optional[np.ndarray] = None
    dft: Optional[np.ndarray] = None
    fields: dict = field(default_factory=dict)
    init: Optional[dict] = None               # component -> initial field [nx, ny, nz]
    status: int = 0                           # 0, or YEE_ENUMERIC / YEE_EOVERFLOW, YEE_EINVAL (precision)
    error: Optional[str] = None
    deadline: Optional[float] = None          # seconds after arrival; cancelled once passed
    cancelled: bool = False
    requeued: int = 0                         # times re-queued after a device reset
    _resume: Optional[tuple] = field(default=None, repr=False)   # (state tensor, steps done)

    @property
    def failed(self) -> bool:
        return self.status != 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def _set_initial(req: Request, solver: YeeSolver):
    for comp, arr in (req.init or {}).items():
        solver.set_field(comp, arr)


def _check_health(req: Request, solver: YeeSolver):
    st, flags, msg = solver.status()
    if st:
        req.status = st
        req.error = f"{_lib.STATUS_NAMES.get(st, st)} (flags {flags:#x}): {msg}"


class BatchServer:
    def __init__(self, max_slots: int = 32, hbm_budget: int = 4 << 30, steps_per_replay: int = 64,
                 device: str = "cuda:0", keep_fields=(), max_active_cells: Optional[int] = DEFAULT_ACTIVE_CELLS,
                 checkpoint_every: int = 0, precision: str = "f32", solo: bool = True):
        """precision: storage precision of every request this server takes
        ("f32", "f64" or "f16"); a request of another precision fails.
        solo: while a single request runs, step it with yee_step in its own
        launch shape (the batch picks it up again from its current step when
        others join); its results are the same bits."""
        import torch
        self.torch = torch
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.K = int(steps_per_replay)
        self.keep_fields = tuple(keep_fields)
        self.max_slots = int(max_slots)
        self.hbm_budget = int(hbm_budget)
        self.max_active_cells = max_active_cells
        self.checkpoint_every = int(checkpoint_every)
        if precision not in _lib.PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(_lib.PRECISIONS)}")
        self.precision = precision
        self.solo = bool(solo)
        self.solo_runs = 0                # replays taken by a lone request with yee_step
        self.replays = 0
        self.resets = 0
        self._cancel = set()
        self.batch = None
        self._make_batch()

    def _make_batch(self):
        b = C.c_void_p()
        _lib.check(self.lib.yee_batch_create(self.max_slots, self.hbm_budget, self.K, C.byref(b)), "yee_batch_create")
        self.batch = b
        _lib.check(self.lib.yee_batch_set_precision(b, _lib.PRECISIONS[self.precision]), "yee_batch_set_precision")
        nb = C.c_int64()
        _lib.check(self.lib.yee_batch_footprint(self.max_slots, C.byref(nb)), "yee_batch_footprint")
        self.table = self.torch.empty(nb.value + 256, dtype=self.torch.uint8, device=self.device)
        base = (self.table.data_ptr() + 255) & ~255
        _lib.check(self.lib.yee_batch_bind_workspace(b, C.c_void_p(base), nb.value), "yee_batch_bind_workspace")

    def cancel(self, rid: int):
        """Cancel request `rid` at the next replay boundary (running or waiting)."""
        self._cancel.add(rid)

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _collect(self, req: Request, solver: YeeSolver, t0: float):
        _check_health(req, solver)
        if req.wl.probes:
            req.series = solver.series(solver.steps_done - req.wl.steps + 1, req.wl.steps) \
                if req.wl.steps <= solver.desc.series_len else None
            req.dft = solver.dft()
        for c in self.keep_fields:
            req.fields[c] = solver.field(c)
        req.finished = time.perf_counter() - t0

    def _due(self, req: Request, now: float) -> bool:
        return req.rid in self._cancel or (req.deadline is not None and now > req.arrival + req.deadline)

    def _retire_cancelled(self, req: Request, now: float, done: List[Request]):
        req.cancelled = True
        req.error = "cancelled" if req.rid in self._cancel else f"deadline of {req.deadline} s passed"
        req.finished = now
        req._resume = None
        done.append(req)

    def serve(self, requests: List[Request], t0: Optional[float] = None,
              reset_after_replays: Optional[int] = None) -> List[Request]:
        """Serve requests with the given arrival offsets (seconds from t0).

        reset_after_replays: simulate a device reset after that many replays
        (the batch and every in-flight context are destroyed; see the module
        documentation)."""
        lib = self.lib
        t0 = time.perf_counter() if t0 is None else t0
        waiting = sorted(requests, key=lambda r: r.arrival)
        running = {}                      # slot -> (request, solver)
        done: List[Request] = []
        while waiting or running:
            now = time.perf_counter() - t0
            # cancellations and deadlines (a boundary between replays)
            for slot in [q for q, (r, _) in running.items() if self._due(r, now)]:
                req, solver = running.pop(slot)
                _lib.check(lib.yee_batch_release(self.batch, slot), "yee_batch_release")
                solver.close()
                self._retire_cancelled(req, now, done)
            for req in [r for r in waiting if self._due(r, now)]:
                waiting.remove(req)
                self._retire_cancelled(req, now, done)
            if not waiting and not running:
                break
            # admit arrived requests while slots, budget and the cell cap allow
            active = sum(r.wl.cells for r, _ in running.values())
            while waiting and waiting[0].arrival <= now:
                req = waiting[0]
                if req.wl.precision != self.precision:
                    # the batch takes one storage precision: this request fails alone
                    waiting.pop(0)
                    req.status = -1
                    req.error = f"YEE_EINVAL: precision {req.wl.precision}, the server runs {self.precision}"
                    req.finished = now
                    done.append(req)
                    continue
                if (self.max_active_cells is not None and running
                        and active + req.wl.cells > self.max_active_cells):
                    break
                solver = YeeSolver(req.wl, device=str(self.device),
                                   series_len=max(self.K, req.wl.steps if req.wl.probes else 1))
                left = req.wl.steps
                if req._resume is not None:
                    state, done_steps = req._resume
                    solver.load_state(state)
                    left = req.wl.steps - done_steps
                else:
                    _set_initial(req, solver)
                slot = C.c_int32()
                st = lib.yee_batch_admit(self.batch, solver.ctx, int(left), C.byref(slot))
                if st == -6:              # YEE_EAGAIN: wait for a slot or for memory
                    solver.close()
                    if not running:
                        raise RuntimeError(f"request {req.rid} ({req.wl.name}) does not fit the batch's "
                                           f"HBM budget even with nothing else admitted")
                    break
                _lib.check(st, "yee_batch_admit")
                if req.admitted is None:
                    req.admitted = time.perf_counter() - t0
                running[slot.value] = (req, solver)
                active += req.wl.cells
                waiting.pop(0)
            if not running:
                # nothing to run: wait for the next arrival
                time.sleep(max(0.0, min(0.001, waiting[0].arrival - now)))
                continue
            if self.solo and len(running) == 1:
                # a lone request: its own launch shape is faster than the batch's
                (req, solver), = running.values()
                solver.step(min(self.K, req.wl.steps - solver.steps_done))
                self.solo_runs += 1
            else:
                _lib.check(lib.yee_batch_run(self.batch, self._stream()), "yee_batch_run")
            self.replays += 1
            ndone = C.c_int32()
            buf = (C.c_int32 * self.max_slots)()
            _lib.check(lib.yee_batch_poll(self.batch, buf, self.max_slots, C.byref(ndone)), "yee_batch_poll")
            if ndone.value:
                self.torch.cuda.current_stream(self.device).synchronize()
            for q in range(ndone.value):
                slot = buf[q]
                req, solver = running.pop(slot)
                self._collect(req, solver, t0)
                _lib.check(lib.yee_batch_release(self.batch, slot), "yee_batch_release")
                solver.close()
                req._resume = None
                done.append(req)
            if self.checkpoint_every and self.replays % self.checkpoint_every == 0:
                for req, solver in running.values():
                    buf_t = req._resume[0] if req._resume is not None else None
                    state = solver.save_state(buf_t)
                    req._resume = (state, solver.steps_done)
            if reset_after_replays is not None and self.replays == reset_after_replays:
                # simulated device reset: everything in flight is lost except
                # the saved states; the requests go back to the front of the queue
                self.torch.cuda.current_stream(self.device).synchronize()
                lost = [r for r, _ in running.values()]
                self.close()
                for _, solver in running.values():
                    solver.close()
                running = {}
                self._make_batch()
                self.resets += 1
                for req in lost:
                    req.requeued += 1
                waiting = sorted(lost, key=lambda r: r.arrival) + waiting
        return done

    def close(self):
        if getattr(self, "batch", None):
            self.lib.yee_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_one_at_a_time(requests: List[Request], device: str = "cuda:0", keep_fields=(),
                        t0: Optional[float] = None) -> List[Request]:
    """First come, first served: one plain ``yee_step`` solve per request."""
    import torch
    t0 = time.perf_counter() if t0 is None else t0
    out = []
    for req in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        req.admitted = time.perf_counter() - t0
        solver = YeeSolver(req.wl, device=device, series_len=max(1, req.wl.steps))
        _set_initial(req, solver)
        solver.step(req.wl.steps)
        torch.cuda.current_stream().synchronize()
        _check_health(req, solver)
        if req.wl.probes:
            req.series = solver.series(1, req.wl.steps)
            req.dft = solver.dft()
        for c in keep_fields:
            req.fields[c] = solver.field(c)
        req.finished = time.perf_counter() - t0
        solver.close()
        out.append(req)
    return out
