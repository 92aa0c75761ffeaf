"""Serving SRTM smoothing requests that arrive over time, with continuous batching.

A `Server` owns one device arena of `hbm_budget` bytes and a few streams. A request brings its
model and measurements (host arrays) and receives device-resident smoothed outputs. At every
`step`, completed batches are retired (their arena ranges freed) and, while a stream is free,
the waiting requests that fit in the remaining arena (inputs, outputs, the per-request scan
workspace and the batch table) are admitted in arrival order and launched together as one
batched library call on that stream. Requests that arrive while others are on the GPU are
therefore admitted as streams and memory free up, and batches on different streams overlap
on the device. Latency is measured from a request's arrival to the host observing its batch's
completion event. All arithmetic is in libsrtm's kernels.
"""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import srtm

ALIGN = 256


class Arena:
    """First-fit allocator of 256-byte-aligned ranges in one device byte buffer."""

    def __init__(self, nbytes: int, device):
        self.size = (int(nbytes) // ALIGN) * ALIGN
        self.buf = torch.empty(self.size, device=device, dtype=torch.uint8)
        self.free: List[List[int]] = [[0, self.size]]   # sorted [offset, length]
        self.used = 0

    @staticmethod
    def rounded(n: int) -> int:
        return ((int(n) + ALIGN - 1) // ALIGN) * ALIGN

    def alloc(self, n: int) -> Optional[int]:
        n = self.rounded(n)
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = [off + n, ln - n]
                self.used += n
                return off
        return None

    def release(self, off: int, n: int):
        n = self.rounded(n)
        self.used -= n
        i = bisect.bisect_left(self.free, [off, 0])
        self.free.insert(i, [off, n])
        # coalesce with the neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i][1] += self.free.pop(i + 1)[1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1][1] += self.free.pop(i)[1]

    def tensor(self, off: int, nbytes: int) -> torch.Tensor:
        return self.buf[off:off + nbytes]


@dataclass
class Request:
    rid: int
    arrival: float             # seconds on the server's clock
    F: np.ndarray
    Q: np.ndarray
    H: np.ndarray
    R: np.ndarray
    L: int
    m0: np.ndarray
    P0: np.ndarray
    y: np.ndarray              # [N][ny]
    fast: bool = True
    done: Optional[float] = None
    outputs: Dict[str, torch.Tensor] = field(default_factory=dict)
    info: int = 0
    batch: int = -1            # index of the launch that carried the request


class _Flight:
    """One launched batch: its requests, arena ranges, stream and completion event."""

    def __init__(self, reqs, ranges, stream, event, batch):
        self.reqs, self.ranges, self.stream, self.event, self.batch = reqs, ranges, stream, event, batch


class Server:
    def __init__(self, nx: int, ny: int, dtype=torch.float32, *, hbm_budget: int = 8 << 30, streams: int = 4,
                 max_batch: int = 64, device="cuda", keep_outputs: bool = True):
        self.nx, self.ny, self.dtype = nx, ny, dtype
        self.device = torch.device(device)
        self.esz = torch.tensor([], dtype=dtype).element_size()
        self.arena = Arena(hbm_budget, self.device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(streams)]
        self.free_streams = list(range(streams))
        self.max_batch = max_batch
        self.keep_outputs = keep_outputs
        self.waiting: List[Request] = []
        self.flights: List[_Flight] = []
        self.finished: List[Request] = []
        self.t0 = time.perf_counter()
        self.batches_launched = 0
        self._models: Dict[tuple, Dict[str, torch.Tensor]] = {}   # device copies of repeated models

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -------------------------------------------------------------- sizes
    def _model(self, r: Request) -> Dict[str, torch.Tensor]:
        """Device copy of the request's model, shared by every request that passes the same
        host arrays (outside the request arena: models are few and small)."""
        key = tuple(id(getattr(r, k)) for k in ("F", "Q", "H", "R", "m0", "P0"))
        dev = self._models.get(key)
        if dev is None:
            dev = {k: torch.as_tensor(np.asarray(getattr(r, k), dtype=np.float64)).to(self.device, self.dtype)
                   .contiguous() for k in ("F", "Q", "H", "R", "m0", "P0")}
            # batches on every stream read it: finish the upload before any of them is enqueued
            torch.cuda.current_stream(self.device).synchronize()
            # keep the host arrays alive so that their ids stay unique while cached
            dev["_host"] = tuple(getattr(r, k) for k in ("F", "Q", "H", "R", "m0", "P0"))
            self._models[key] = dev
        return dev

    def footprint(self, r: Request) -> int:
        nx, ny, N, L, e = self.nx, self.ny, r.y.shape[0], r.L, self.esz
        a = Arena.rounded
        inputs = a(N * ny * e)
        outs = (a(N * L * nx * e) + a(N * L * nx * nx * e) if r.fast else 0) + a(N * nx * e) + a(N * nx * nx * e)
        ws = a(srtm.workspace_size(nx, ny, L, N, self.dtype, True))
        table = a(256 + (N + 255) // 256 * 4)   # descriptor + its tiles in the batch table (upper bound)
        return inputs + outs + ws + table + 2 * ALIGN

    def submit(self, r: Request):
        if r.y.ndim != 2 or r.y.shape[1] != self.ny or r.F.shape != (self.nx, self.nx):
            raise srtm.SrtmError("request shapes do not match the server")
        if self.footprint(r) > self.arena.size:
            raise srtm.SrtmError(f"request {r.rid} needs more than the whole HBM budget")
        self.waiting.append(r)

    # -------------------------------------------------------------- scheduling
    def _retire(self):
        still = []
        for f in self.flights:
            if f.event.query():
                t = self.now()
                # read back on the batch's own stream (already complete), and finish with the
                # arena ranges before they are released to other streams
                with torch.cuda.stream(f.stream):
                    info = f.batch.info.cpu().tolist()
                    for r, inf in zip(f.reqs, info):
                        r.done, r.info = t, int(inf)
                        r.outputs = {k: v.clone() for k, v in r.outputs.items()} if self.keep_outputs else {}
                        self.finished.append(r)
                if self.keep_outputs:
                    f.stream.synchronize()
                for off, n in f.ranges:
                    self.arena.release(off, n)
                self.free_streams.append(self.streams.index(f.stream))
            else:
                still.append(f)
        self.flights = still

    def _launch(self):
        while self.waiting and self.free_streams:
            take, budget_left = [], self.arena.size - self.arena.used
            for r in self.waiting:
                if len(take) >= self.max_batch:
                    break
                need = self.footprint(r)
                if need > budget_left:
                    break                 # keep arrival order: no overtaking
                take.append(r)
                budget_left -= need
            if not take:
                return
            ranges, ok = [], True

            def get(n):
                nonlocal ok
                off = self.arena.alloc(n)
                if off is None:
                    ok = False
                    return torch.empty(max(int(n), 1), device=self.device, dtype=torch.uint8)[:0]
                ranges.append((off, n))
                return self.arena.tensor(off, Arena.rounded(n))[:n]

            s = self.streams[self.free_streams[-1]]
            with torch.cuda.stream(s):
                problems, outputs = [], []
                for r in take:
                    dev = {k: v for k, v in self._model(r).items() if k != "_host"}
                    h = torch.empty(r.y.shape, dtype=self.dtype, pin_memory=True)
                    h.numpy()[...] = r.y            # one host pass: convert into pinned memory
                    t = get(h.numel() * self.esz).view(self.dtype).view(h.shape)
                    t.copy_(h, non_blocking=True)
                    dev["y"] = t
                    N, nx, L = r.y.shape[0], self.nx, r.L
                    o = {}
                    if r.fast:
                        o["ms_fast"] = get(N * L * nx * self.esz).view(self.dtype).view(N, L, nx)
                        o["Ps_fast"] = get(N * L * nx * nx * self.esz).view(self.dtype).view(N, L, nx, nx)
                    o["ms_slow"] = get(N * nx * self.esz).view(self.dtype).view(N, nx)
                    o["Ps_slow"] = get(N * nx * nx * self.esz).view(self.dtype).view(N, nx, nx)
                    r.outputs = o
                    problems.append((dev["F"], dev["Q"], dev["H"], dev["R"], L, dev["m0"], dev["P0"], dev["y"]))
                    outputs.append(o)
                if not ok:   # fragmentation: give the ranges back and wait for completions
                    for off, n in ranges:
                        self.arena.release(off, n)
                    return
                b = srtm.Batch(problems, fast=True, slow=True, outputs=outputs, alloc=get)
                if not ok:
                    for off, n in ranges:
                        self.arena.release(off, n)
                    return
                b.launch(s.cuda_stream)
                ev = torch.cuda.Event()
                ev.record(s)
            for r in take:
                r.batch = self.batches_launched
            self.free_streams.pop()
            self.waiting = self.waiting[len(take):]
            self.flights.append(_Flight(take, ranges, s, ev, b))
            self.batches_launched += 1

    def step(self):
        self._retire()
        self._launch()

    def busy(self) -> bool:
        return bool(self.waiting or self.flights)

    def drain(self):
        while self.busy():
            self.step()


def serve(server: Server, requests: List[Request], *, spin_s: float = 50e-6) -> Dict:
    """Releases `requests` (sorted by arrival, times relative to the start of this call) to the
    server at their arrival times and runs it until all are finished. Returns latency and
    throughput statistics."""
    import gc
    gc_was = gc.isenabled()
    gc.disable()   # no collector pauses inside the arrival loop
    server.t0 = time.perf_counter()
    i, n = 0, len(requests)
    while i < n or server.busy():
        now = server.now()
        while i < n and requests[i].arrival <= now:
            server.submit(requests[i])
            i += 1
        server.step()
        if i < n and not server.busy():
            wait = requests[i].arrival - server.now()
            if wait > 0:
                time.sleep(min(wait, 1e-3))
        elif spin_s:
            time.sleep(spin_s)
    torch.cuda.synchronize(server.device)
    if gc_was:
        gc.enable()
    lat = np.array([r.done - r.arrival for r in requests])
    span = max(r.done for r in requests) - min(r.arrival for r in requests)
    fast_states = sum(r.y.shape[0] * r.L for r in requests)
    return dict(requests=n, batches=server.batches_launched,
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3), max_ms=float(lat.max() * 1e3), span_s=float(span),
                fast_states=int(fast_states), fast_states_per_s=float(fast_states / span),
                failed=[r.rid for r in requests if r.info])
