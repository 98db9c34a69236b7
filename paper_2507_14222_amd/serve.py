"""Continuous-batching scoring server over a device-resident IG model.

Requests (arrays of flow codes) arrive at any time through ``Server.submit``.
A dispatcher thread admits waiting requests into free *slots* -- one HIP stream
each, with pinned staging and device buffers -- as long as the flows in flight
stay within the memory budget; requests admitted together form one
micro-batch (one ``ig_score`` launch, Eq. 4 of the paper).  While one slot's
batch runs on the GPU, the next slot copies and launches the following batch,
so copies, kernels and host work overlap.  Completion is observed by event
query; each request gets back exactly the rows of its own flows.

Scores are integers and every flow is scored independently (no state is shared
between flows), so a request's result is identical whether it is served alone
or mixed with others.

This module is host-side plumbing: every score comes from libig's kernels.  The
device work sits behind a small executor interface so that the scheduling can
be exercised on the CPU with a stand-in executor.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Deque, List, Optional, Sequence

import numpy as np

from . import ig


@dataclass
class _Request:
    codes: np.ndarray
    future: Future
    t_arrival: float
    t_admit: float = 0.0
    t_done: float = 0.0


@dataclass
class _Slot:
    handle: object                          # executor-owned buffers and stream
    requests: List[_Request] = field(default_factory=list)
    flows: int = 0


class GpuExecutor:
    """Slots on the current GPU: a HIP stream, pinned staging and device buffers."""

    def __init__(self, model: ig.Model, cap: int, d: int):
        self.model = model
        self.cap = cap
        self.d = d

    def new_slot(self):
        import torch
        h = {
            "stream": torch.cuda.Stream(),
            "done": torch.cuda.Event(),
            "h_codes": torch.empty((self.cap, self.d), dtype=torch.int16, pin_memory=True),
            "h_out": torch.empty((self.cap, 2), dtype=torch.int64, pin_memory=True),
            "d_codes": torch.empty((self.cap, self.d), dtype=torch.int16, device="cuda"),
            "d_out": torch.empty((self.cap, 2), dtype=torch.int64, device="cuda"),
        }
        # one copy on the new stream now: its first launch sets the stream up (a
        # few ms), which would otherwise fall on the first request it serves
        with torch.cuda.stream(h["stream"]):
            h["d_out"][:1].copy_(h["h_out"][:1], non_blocking=True)
        h["stream"].synchronize()
        return h

    def staging(self, h) -> np.ndarray:
        return h["h_codes"].numpy().view(np.uint16)

    def launch(self, h, n: int) -> None:
        import torch
        with torch.cuda.stream(h["stream"]):
            h["d_codes"][:n].copy_(h["h_codes"][:n], non_blocking=True)
            ig.score(self.model, h["d_codes"][:n], out=h["d_out"][:n], stream=h["stream"])
            h["h_out"][:n].copy_(h["d_out"][:n], non_blocking=True)
            h["done"].record(h["stream"])

    def ready(self, h) -> bool:
        return h["done"].query()

    def results(self, h, n: int) -> np.ndarray:
        return h["h_out"][:n].numpy()


# Interpreter settings held while any server runs, restored when the last one closes.
_settings_lock = threading.Lock()
_settings = {"servers": 0, "freezers": 0, "switch": None}


def _hold_settings(freeze: bool) -> None:
    import gc
    import sys
    with _settings_lock:
        if freeze:
            gc.collect()
            gc.freeze()
            _settings["freezers"] += 1
        if _settings["servers"] == 0:
            # the dispatcher shares the interpreter with the callers: hand the lock over often
            _settings["switch"] = sys.getswitchinterval()
            if _settings["switch"] > 0.0005:
                sys.setswitchinterval(0.0005)
        _settings["servers"] += 1


def _release_settings(freeze: bool) -> None:
    import gc
    import sys
    with _settings_lock:
        if freeze:
            _settings["freezers"] -= 1
            if _settings["freezers"] == 0:
                gc.unfreeze()
        _settings["servers"] -= 1
        if _settings["servers"] == 0:
            sys.setswitchinterval(_settings["switch"])


class Server:
    """Serve scoring requests against ``model`` with continuous batching.

    n_slots          concurrent micro-batches (one HIP stream each)
    max_batch_flows  flows per micro-batch (a larger request is rejected)
    mem_budget_bytes bytes of flows in flight (codes + results); 0 = what the slots hold
    freeze_gc        move every object that exists when the server starts out of the
                     cyclic collector's scans (gc.freeze, process-wide): a full
                     collection otherwise walks the whole process -- torch included --
                     and stalls the dispatcher for tens of ms at a time; undone
                     (gc.unfreeze) when the last server that froze closes
    """

    def __init__(self, model: Optional[ig.Model], n_slots: int = 4, max_batch_flows: int = 16384,
                 mem_budget_bytes: int = 0, d: Optional[int] = None, executor=None, freeze_gc: bool = True):
        _hold_settings(freeze_gc)
        self._freeze = freeze_gc
        self._held = True
        try:
            self._setup(model, n_slots, max_batch_flows, mem_budget_bytes, d, executor)
        except BaseException:
            self._held = False
            _release_settings(freeze_gc)
            raise

    def _setup(self, model, n_slots, max_batch_flows, mem_budget_bytes, d, executor) -> None:
        if model is not None:
            info = model.info()
            if info.d == 0:
                raise ig.IGError(ig.IG_E_INVAL, "the server scores flows given as codes; model has no bins")
            d = int(info.d)
        if d is None:
            raise ValueError("d is needed without a model")
        self.d = int(d)
        self.cap = int(max_batch_flows)
        self.bytes_per_flow = 2 * self.d + 16
        self.budget = int(mem_budget_bytes) if mem_budget_bytes else n_slots * self.cap * self.bytes_per_flow
        self.exe = executor if executor is not None else GpuExecutor(model, self.cap, self.d)
        self.slots = [_Slot(self.exe.new_slot()) for _ in range(n_slots)]
        self._free: Deque[_Slot] = collections.deque(self.slots)
        self._busy: Deque[_Slot] = collections.deque()
        self._queue: Deque[_Request] = collections.deque()
        self._in_flight_bytes = 0
        self.max_in_flight_bytes = 0
        self._cv = threading.Condition()
        self._stop = False
        self.completed: List[_Request] = []
        self.batches = 0
        self.error: Optional[BaseException] = None
        self._thread = threading.Thread(target=self._run, name="ig-serve", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------ client side
    def submit(self, codes: np.ndarray, t_arrival: Optional[float] = None) -> Future:
        """Queue one request; the future resolves to an int64 array [n, 2] = (A, N)."""
        codes = np.ascontiguousarray(codes, dtype=np.uint16)
        if codes.ndim != 2 or codes.shape[1] != self.d or codes.shape[0] == 0:
            raise ig.IGError(ig.IG_E_INVAL, f"request codes must be [n >= 1, {self.d}]")
        if codes.shape[0] > self.cap or codes.shape[0] * self.bytes_per_flow > self.budget:
            raise ig.IGError(ig.IG_E_INVAL, f"request of {codes.shape[0]} flows exceeds the batch capacity")
        fut: Future = Future()
        req = _Request(codes, fut, time.perf_counter() if t_arrival is None else t_arrival)
        with self._cv:
            if self._stop:
                raise RuntimeError("server stopped")
            if self.error is not None:
                raise RuntimeError(f"server failed: {self.error}")
            self._queue.append(req)
            self._cv.notify()
        return fut

    def close(self) -> None:
        with self._cv:
            self._stop = True
            self._cv.notify()
        self._thread.join()
        if self._held:
            self._held = False
            _release_settings(self._freeze)
        if self.error is not None:
            raise RuntimeError(f"server failed: {self.error}")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ dispatcher
    def _retire(self) -> bool:
        """Hand back the results of finished slots, in launch order."""
        any_done = False
        while self._busy and self.exe.ready(self._busy[0].handle):
            slot = self._busy.popleft()
            out = self.exe.results(slot.handle, slot.flows)
            now = time.perf_counter()
            at = 0
            for r in slot.requests:
                n = r.codes.shape[0]
                r.t_done = now
                if not r.future.cancelled():
                    r.future.set_result(np.array(out[at:at + n], copy=True))
                at += n
                self.completed.append(r)
            with self._cv:
                self._in_flight_bytes -= slot.flows * self.bytes_per_flow
            slot.requests = []
            slot.flows = 0
            self._free.append(slot)
            any_done = True
        return any_done

    def _admit(self) -> bool:
        """Pack the waiting requests at the head of the queue into one free slot."""
        if not self._free:
            return False
        batch: List[_Request] = []
        flows = 0
        with self._cv:
            while self._queue:
                r = self._queue[0]
                if r.future.cancelled():
                    self._queue.popleft()
                    continue
                n = r.codes.shape[0]
                if flows + n > self.cap or self._in_flight_bytes + (flows + n) * self.bytes_per_flow > self.budget:
                    break
                batch.append(self._queue.popleft())
                flows += n
            if not batch:
                return False
            self._in_flight_bytes += flows * self.bytes_per_flow
            self.max_in_flight_bytes = max(self.max_in_flight_bytes, self._in_flight_bytes)
        slot = self._free.popleft()
        now = time.perf_counter()
        h = self.exe.staging(slot.handle)
        at = 0
        for r in batch:
            n = r.codes.shape[0]
            h[at:at + n] = r.codes
            r.t_admit = now
            at += n
        slot.requests = batch
        slot.flows = flows
        self._busy.append(slot)          # before the launch, so a failure reaches these requests
        self.exe.launch(slot.handle, flows)
        self.batches += 1
        return True

    def _fail(self, e: BaseException) -> None:
        with self._cv:
            self.error = e
            pending = list(self._queue)
            self._queue.clear()
        for s in list(self._busy):
            pending += s.requests
        for r in pending:
            if not r.future.done():
                r.future.set_exception(e)

    def _run(self) -> None:
        try:
            while True:
                progressed = self._retire()
                progressed |= self._admit()
                with self._cv:
                    if self._stop and not self._queue and not self._busy:
                        return
                    if not progressed:
                        # nothing to launch: sleep until a request arrives or a slot may finish
                        self._cv.wait(timeout=0.0001 if self._busy else 0.005)
        except BaseException as e:  # a failing launch fails every outstanding request
            self._fail(e)


def drive(server: Server, requests: Sequence[np.ndarray], arrivals: Sequence[float]):
    """Open-loop load: submit request i at time arrivals[i] (seconds from now).
    Returns (futures, t0); latency of i = completion - (t0 + arrivals[i])."""
    t0 = time.perf_counter()
    futs = []
    for codes, ta in zip(requests, arrivals):
        target = t0 + ta
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            # sleep rather than spin: a spinning thread would hold the interpreter
            # lock against the dispatcher for a whole switch interval
            time.sleep(min(target - now, 0.0002))
        futs.append(server.submit(codes, t_arrival=target))
    return futs, t0


def serve_one_at_a_time(model: ig.Model, requests: Sequence[np.ndarray], arrivals: Sequence[float]):
    """Baseline: each request copied, scored and copied back alone, in arrival
    order, once it has arrived.  Returns (results, latencies in seconds)."""
    import torch

    d = int(model.info().d)
    cap = max(r.shape[0] for r in requests)
    exe = GpuExecutor(model, cap, d)
    h = exe.new_slot()
    t0 = time.perf_counter()
    res, lat = [], []
    for codes, ta in zip(requests, arrivals):
        while time.perf_counter() - t0 < ta:
            pass
        n = codes.shape[0]
        exe.staging(h)[:n] = codes
        exe.launch(h, n)
        h["stream"].synchronize()
        res.append(np.array(exe.results(h, n), copy=True))
        lat.append(time.perf_counter() - t0 - ta)
    torch.cuda.synchronize()
    return res, lat
