"""Running many independent SRTM smoothing problems on one GPU.

A `BatchRunner` either puts every problem into one mixed batch (`mixed=True`: one set of six
launches whatever the mix of state/measurement sizes, inputs and per-window models; each
workgroup dispatches on its sequence) or groups the problems by (nx, ny) with one batched call
per group (kernels compiled for that pair alone). Either way it can split the work into
`segments` sub-batches of similar size, run the sub-batches on one stream or a stream each, and
record the whole launch sequence once as a HIP graph (through the library's graph entry points)
to replay it. `autotune` times the candidate configurations on the actual problems and keeps
the fastest. All arithmetic is in libsrtm's kernels.
"""
from __future__ import annotations

import itertools
import time
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import srtm


def _balanced_split(idx: List[int], weights: List[float], parts: int) -> List[List[int]]:
    """Greedy split of `idx` into at most `parts` lists of similar total weight (largest first)."""
    parts = max(1, min(parts, len(idx)))
    bins: List[List[int]] = [[] for _ in range(parts)]
    load = [0.0] * parts
    for j in sorted(idx, key=lambda i: -weights[i]):
        b = min(range(parts), key=lambda q: load[q])
        bins[b].append(j)
        load[b] += weights[j]
    return [sorted(b) for b in bins if b]


def _sizes(pr) -> Tuple[int, int]:
    """(nx, ny) of a problem tuple (F [.., nx, nx], Q, H [.., ny, nx], ...)."""
    return int(pr[0].shape[-1]), int(pr[2].shape[-2])


def _plain(pr) -> bool:
    """Time-invariant model without inputs (what the per-pair batch entry point takes)."""
    return len(pr) == 8 and pr[0].dim() == 2


class BatchRunner:
    """problems: tuples (F, Q, H, R, L, m0, P0, y), or (F, Q, H, R, L, m0, P0, y, B, u) with known
    inputs, of device tensors (one dtype and device); F, Q, H, R of shape [N, ...] give a
    per-window model."""

    def __init__(self, problems: Sequence[tuple], *, fast: bool = True, slow: bool = True, segments: int = 1,
                 multi_stream: bool = False, graph: bool = False, mixed: bool = False,
                 outputs: Optional[List[Dict]] = None):
        self.problems = list(problems)
        self.fast, self.slow = fast, slow
        self.segments, self.multi_stream, self.use_graph = int(segments), bool(multi_stream), bool(graph)
        self.mixed = bool(mixed)
        if not self.problems:
            raise srtm.SrtmError("no problems")
        self.device = self.problems[0][7].device
        groups: Dict[Tuple[int, int], List[int]] = {}
        for j, pr in enumerate(self.problems):
            groups.setdefault((0, 0) if self.mixed else _sizes(pr), []).append(j)
        work = []
        for pr in self.problems:
            nx = _sizes(pr)[0]
            work.append(float(pr[7].shape[0] * pr[4] * (nx + nx * nx)))
        self.outputs: List[Dict] = outputs if outputs is not None else [None] * len(self.problems)
        self.batches: List = []
        self.members: List[List[int]] = []
        for key in sorted(groups):
            for part in _balanced_split(groups[key], work, self.segments):
                outs = None if outputs is None else [outputs[j] for j in part]
                probs = [self.problems[j] for j in part]
                if not self.mixed and all(_plain(pr) for pr in probs):
                    b = srtm.Batch(probs, fast=fast, slow=slow, outputs=outs)
                else:
                    b = srtm.BatchEx(probs, fast=fast, slow=slow, outputs=outs)
                self.batches.append(b)
                self.members.append(part)
                for j, o in zip(part, b.outputs):
                    self.outputs[j] = o
        self.streams = [torch.cuda.Stream(self.device) for _ in self.batches] if self.multi_stream else []
        self.graph: Optional[srtm.Graph] = None

    def _enqueue(self):
        if not self.multi_stream:
            for b in self.batches:
                b.launch()
            return
        main = torch.cuda.current_stream(self.device)
        start = torch.cuda.Event()
        start.record(main)
        ends = []
        for b, s in zip(self.batches, self.streams):
            s.wait_event(start)
            b.launch(s.cuda_stream)
            e = torch.cuda.Event()
            e.record(s)
            ends.append(e)
        for e in ends:
            main.wait_event(e)

    def capture(self):
        """Record the launch sequence once (warmed up eagerly first) as a HIP graph."""
        self._enqueue()
        torch.cuda.synchronize(self.device)
        g = srtm.Graph(self.device)
        g.record(self._enqueue)
        self.graph = g

    def run(self):
        """Enqueue one smoothing pass over every problem on the current stream."""
        if self.use_graph:
            if self.graph is None:
                self.capture()
            self.graph.replay()
        else:
            self._enqueue()

    def zero_info(self):
        for b in self.batches:
            b.info.zero_()

    def check(self):
        for b in self.batches:
            b.check()

    def describe(self) -> dict:
        """The configuration; `calls` batched library calls, `launches` kernel launches per pass."""
        return dict(segments=self.segments, multi_stream=self.multi_stream, graph=self.use_graph, mixed=self.mixed,
                    calls=len(self.batches), launches=6 * len(self.batches))


def time_runner(r: BatchRunner, reps: int = 5, warmup: int = 2) -> float:
    """Median seconds of one pass."""
    for _ in range(warmup):
        r.run()
    torch.cuda.synchronize(r.device)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r.run()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    ts.sort()
    return ts[len(ts) // 2]


_CACHE: Dict[tuple, dict] = {}


def signature(problems) -> tuple:
    pairs = tuple(sorted({_sizes(pr) for pr in problems}))
    kinds = tuple(sorted({(len(pr), pr[0].dim()) for pr in problems}))
    fast = sum(pr[7].shape[0] * pr[4] for pr in problems)
    return (len(problems), pairs, kinds, int(fast).bit_length(), str(problems[0][7].dtype))


def autotune(problems, *, fast: bool = True, slow: bool = True, segments=(1, 2, 4), reps: int = 5,
             log: Optional[list] = None) -> BatchRunner:
    """Times every (mixed, segments, multi_stream, graph) candidate on these problems, all writing
    the same output tensors, and returns the fastest runner. Results are cached per workload
    signature (count, sizes, kinds, magnitude of the work, dtype) for the process."""
    sig = signature(problems)
    outputs = None
    if sig in _CACHE:
        cfg = _CACHE[sig]
        return BatchRunner(problems, fast=fast, slow=slow, **cfg)
    groups = len({_sizes(pr) for pr in problems})
    best, best_t = None, float("inf")
    for mx, seg, ms, gr in itertools.product((True, False), segments, (False, True), (False, True)):
        if mx and groups == 1:
            continue  # one (nx, ny) group: its own kernels (register and LDS use sized for it) cover it
        if seg == 1 and ms and (mx or groups == 1):
            continue  # a single call: a stream per call changes nothing
        r = BatchRunner(problems, fast=fast, slow=slow, segments=seg, multi_stream=ms, graph=gr, mixed=mx,
                        outputs=outputs)
        outputs = r.outputs
        t = time_runner(r, reps=reps)
        if log is not None:
            log.append(dict(r.describe(), seconds=t))
        if t < best_t:
            best, best_t = r, t
    _CACHE[sig] = dict(segments=best.segments, multi_stream=best.multi_stream, graph=best.use_graph, mixed=best.mixed)
    return best
