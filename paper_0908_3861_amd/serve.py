"""Continuous-batching server for the adaptive box-spline filter.

Requests (image, scale field, order, path) arrive at any time.  A scheduler thread

* admits waiting requests in arrival order while the HBM budget (image + scales +
  output bytes of every admitted request), the slot count and the tile capacity of one
  launch allow;
* uploads each admitted request from pinned host memory into device buffers that stay
  resident until its result is back;
* launches every group of newly admitted requests on the next idle one of several
  streams, as a replay of that stream's captured batch plan (``bsf_batch_plan_run``: one
  HIP graph holding the persistent tile kernels of every order/path variant, which read the
  group's descriptors from device memory), so groups admitted while others are still on
  the GPU run concurrently and no launch is planned or issued kernel by kernel;
* polls completion events, reads each request's own error word (written by the kernels,
  fetched by the graph), copies each result back (asynchronously, into pinned host
  memory), frees the request's budget and slot, and resolves its future -- with the
  library's error for a request whose kernels reported one.

``graphs=False`` launches each group with ``bsf_filter_batched`` instead (one context per
stream, so an error is traced to its group, not to the request).  The server owns its
contexts: no other thread shares them.  Latency is measured from arrival (``submit``) to
the moment the result is on the host.  The device work itself is the library's; this
module only schedules it.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import binding

TILE = 16


@dataclass
class Request:
    img: object            # torch tensor [H, W] (u8/f32/f64), ideally pinned host memory
    scales: object         # torch tensor [H, W, 4] float32
    order: int
    path: str = "f64"
    border: str = "clamp"
    a_max: float = 0.0     # bound on every scale (0: the server's bound)
    rid: int = 0
    t_arrival: float = 0.0
    future: Future = field(default_factory=Future)

    @property
    def pixels(self) -> int:
        return int(self.img.shape[0] * self.img.shape[1])

    @property
    def tiles(self) -> int:
        H, W = int(self.img.shape[0]), int(self.img.shape[1])
        return ((H + TILE - 1) // TILE) * ((W + TILE - 1) // TILE)

    def footprint(self) -> int:
        """Device bytes the request holds while admitted."""
        out_bytes = 8 if self.path == "f64" else 4
        return self.pixels * (self.img.element_size() + 16 + out_bytes) + 4096


class AdmissionError(ValueError):
    pass


class Admission:
    """FIFO admission by device-memory footprint, slot count and the tiles one launch holds
    (no request overtakes an earlier one, so a large request cannot starve)."""

    def __init__(self, budget_bytes: int, slots: int):
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.used = 0
        self.busy = 0

    def fits(self, footprint: int) -> bool:
        return self.busy < self.slots and self.used + footprint <= self.budget

    def take(self, footprint: int):
        self.used += footprint
        self.busy += 1

    def release(self, footprint: int):
        self.used -= footprint
        self.busy -= 1

    def admit(self, pending: collections.deque, max_group: int, footprint=lambda r: r.footprint(),
              max_tiles: int | None = None, tiles=lambda r: r.tiles) -> list:
        group, group_tiles = [], 0
        while pending and len(group) < max_group and self.fits(footprint(pending[0])):
            if max_tiles is not None and group_tiles + tiles(pending[0]) > max_tiles:
                break
            r = pending.popleft()
            self.take(footprint(r))
            if max_tiles is not None:
                group_tiles += tiles(r)
            group.append(r)
        return group


class Server:
    def __init__(self, budget_bytes: int = 32 << 30, slots: int = 64, streams: int = 4, device: int = 0,
                 max_group: int = 64, a_max: float = 8.0, graphs: bool = True, max_tiles: int = 1 << 20):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.max_group = int(max_group)
        self.a_max = float(a_max)
        self.graphs = bool(graphs)
        self.max_tiles = int(max_tiles)
        with torch.cuda.device(self.device):
            self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
            # the server's own contexts (one per stream without graphs, so that a device
            # error word belongs to one group)
            self.ctx = binding.Context(device)
            if self.graphs:
                self.plans = [binding.BatchPlan(self.ctx, self.max_group, self.max_tiles, self.a_max)
                              for _ in range(streams)]
                self.stream_ctx = [self.ctx] * streams
            else:
                self.plans = None
                self.stream_ctx = [binding.Context(device) for _ in range(streams)]
        self._busy = [False] * streams
        self._arrivals: queue.Queue = queue.Queue()
        self._pending: collections.deque = collections.deque()
        self._inflight: list = []
        self.admission = Admission(self.budget, self.slots)
        self._stop = threading.Event()
        self._wake = threading.Event()
        self._thread = threading.Thread(target=self._loop, name="bsf-scheduler", daemon=True)
        self.latencies: list[float] = []
        self.completed_pixels = 0
        self.failed = 0
        self.launches = 0
        self.errors: list[BaseException] = []
        self._rid = 0
        self._thread.start()

    # ------------------------------------------------------------------ client side
    def submit(self, img, scales, order: int, path: str = "f64", border: str = "clamp",
               a_max: float = 0.0) -> Future:
        a_max = float(a_max) or self.a_max
        if a_max > self.a_max:
            raise AdmissionError(f"a_max {a_max} exceeds the server's bound {self.a_max}")
        req = Request(img, scales, int(order), path, border, a_max)
        if req.footprint() > self.budget:
            raise AdmissionError(f"request needs {req.footprint()} B, more than the whole budget {self.budget} B")
        if req.tiles > self.max_tiles:
            raise AdmissionError(f"request has {req.tiles} tiles, more than one launch holds ({self.max_tiles})")
        self._rid += 1
        req.rid = self._rid
        req.t_arrival = time.perf_counter()
        self._arrivals.put(req)
        self._wake.set()
        return req.future

    def close(self, wait: bool = True):
        if wait:
            while True:
                with_work = (not self._arrivals.empty()) or self._pending or self._inflight
                if not with_work:
                    break
                time.sleep(0.001)
        self._stop.set()
        self._wake.set()
        self._thread.join()
        self.torch.cuda.synchronize(self.device)
        for p in self.plans or []:
            p.close()
        for c in set(self.stream_ctx):
            c.close()
        self.ctx.close()

    def stats(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return {"completed": len(self.latencies), "failed": self.failed,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "pixels": self.completed_pixels, "launches": self.launches,
                "graphs": self.graphs}

    # ------------------------------------------------------------------ scheduler
    def _loop(self):
        torch = self.torch
        torch.cuda.set_device(self.device)
        while not self._stop.is_set():
            progressed = False
            while True:
                try:
                    self._pending.append(self._arrivals.get_nowait())
                except queue.Empty:
                    break
            progressed |= self._retire()
            progressed |= self._admit_and_launch()
            if not progressed:
                self._wake.wait(timeout=0.0005)
                self._wake.clear()

    def _admit_and_launch(self) -> bool:
        idle = [i for i, b in enumerate(self._busy) if not b]
        if not idle or not self._pending:
            return False
        group = self.admission.admit(self._pending, self.max_group, max_tiles=self.max_tiles)
        if not group:
            return False
        torch = self.torch
        si = idle[0]
        stream = self.streams[si]
        try:
            with torch.cuda.stream(stream):
                items, host_outs = [], []
                for req in group:
                    dimg = req.img.to(self.device, non_blocking=True)
                    dsc = req.scales.to(self.device, non_blocking=True)
                    items.append(dict(img=dimg, scales=dsc, order=req.order, path=req.path, border=req.border,
                                      a_max=req.a_max))
                if self.graphs:
                    outs = self.plans[si].run(items, stream=stream)
                else:
                    outs = binding.filter_batched(items, ctx=self.stream_ctx[si], stream=stream)
                for o in outs:
                    h = torch.empty(o.shape, dtype=o.dtype, pin_memory=True)
                    h.copy_(o, non_blocking=True)
                    host_outs.append(h)
                ev = torch.cuda.Event()
                ev.record(stream)
            # keep the device buffers alive until the event has passed
            self._busy[si] = True
            self.launches += 1
            self._inflight.append((si, ev, group, items, outs, host_outs))
        except BaseException as exc:  # launch failed: fail the whole group
            for req in group:
                self.admission.release(req.footprint())
                req.future.set_exception(exc)
            self.errors.append(exc)
        return True

    def _statuses(self, si: int, n: int) -> list[int]:
        if self.graphs:
            return self.plans[si].job_status()
        st = self.stream_ctx[si].device_error(self.streams[si])
        return [st] * n

    def _retire(self) -> bool:
        done_any = False
        keep = []
        for entry in self._inflight:
            si, ev, group, items, outs, host_outs = entry
            if not ev.query():
                keep.append(entry)
                continue
            statuses = self._statuses(si, len(group))
            t = time.perf_counter()
            for req, h, st in zip(group, host_outs, statuses):
                self.admission.release(req.footprint())
                if st != 0:
                    self.failed += 1
                    req.future.set_exception(binding.BsfError(st, f"request {req.rid}"))
                    continue
                self.latencies.append(t - req.t_arrival)
                self.completed_pixels += req.pixels
                req.future.set_result(h)
            self._busy[si] = False
            done_any = True
        self._inflight = keep
        return done_any
