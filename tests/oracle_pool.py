"""Float64 reference runs for many independent sequences in worker processes (test
infrastructure: only the GPU parity tests use it).

Each job runs oracle.srtm_smoother on one sequence, with one BLAS thread per worker, and
compares it per fast state (conftest.rel_errors) with the GPU outputs passed in, returning
only the largest errors, so that the reference outputs never travel back. Workers are spawned
fresh: they import numpy, threadpoolctl and the reference only, never the GPU runtime.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

PAIRS = (("ms_fast", "Ps_fast", "ms_fast", "Ps_fast"), ("ms_slow", "Ps_slow", "ms_slow", "Ps_slow"),
         ("mf_fast", "Pf_fast", "m_fast", "P_fast"), ("mf_slow", "Pf_slow", "m_slow", "P_slow"))


def _job(args):
    model, y, gpu = args
    from threadpoolctl import threadpool_limits

    import oracle
    from conftest import rel_errors
    A, Q, C, R, L, m0, P0 = model
    with_filter = any("mf_fast" in o for o in gpu.values())
    with threadpool_limits(limits=1):
        ref = oracle.srtm_smoother(A, Q, C, R, L, m0, P0, y, with_filter=with_filter)
    res = {}
    for tag, outs in gpu.items():
        e = {}
        for mk, pk, rm, rp in PAIRS:
            if mk in outs:
                em, ep = rel_errors(outs[mk], outs[pk], ref[rm], ref[rp])
                e[mk] = (float(em.max()), float(ep.max()))
        res[tag] = e
    return res


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def smoother_errors(jobs):
    """jobs: list of (model (A, Q, C, R, L, m0, P0) as float64 arrays, y, {tag: {output name: array}}).
    Returns, per job, {tag: {output: (max mean error, max covariance error)}}, in job order."""
    order = sorted(range(len(jobs)), key=lambda j: -jobs[j][1].shape[0] * jobs[j][0][4])   # largest first
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers(), mp_context=ctx) as ex:
        got = list(ex.map(_job, [jobs[j] for j in order], chunksize=1))
    out = [None] * len(jobs)
    for j, r in zip(order, got):
        out[j] = r
    return out
