"""Pins of the reference with a time-varying (per-window) model (CPU only).

* Brute force: filter and smoother marginals and the log-likelihood from one dense joint
  Gaussian whose transition products and noise blocks follow each step's window model
  (tests/brute_force.py).
* A per-window model whose windows are all equal reproduces the time-invariant reference.
* Planted mistakes (the smoother predicting with the current window's model instead of the
  next one's, the wrong window's measurement noise, ...) are caught by the brute force.
"""
import os
import types

import numpy as np
import pytest

import oracle
from paper_2410_00627_amd import workloads as wl
from brute_force import posteriors
from conftest import rel_errors

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "srtm_oracle.py")


@pytest.fixture(scope="module", params=[(3, 2, 4, 6, 301, True), (2, 1, 1, 9, 302, True), (4, 2, 3, 5, 303, False),
                                        (2, 2, 5, 4, 304, True)],
                ids=["gen_nx3ny2L4", "gen_nx2ny1L1", "drift_nx4ny2L3", "gen_nx2ny2L5"])
def case(request):
    nx, ny, L, N, seed, general = request.param
    m = wl.time_varying_model(nx, ny, L, N, seed, general=general)
    y = wl.simulate_tv(m, seed + 1)
    bf = posteriors(m.A, m.Q, m.C, m.R, L, m.m0, m.P0, y)
    return m, y, bf


def _worst(mod, m, y, bf):
    args = (m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y)
    f = mod.srtm_filter_tv(*args)
    s = mod.srtm_smoother_tv(*args)
    errs = [*rel_errors(f["m_fast"], f["P_fast"], bf["m_fast"], bf["P_fast"]),
            *rel_errors(s["ms_fast"], s["Ps_fast"], bf["ms_fast"], bf["Ps_fast"])]
    worst = max(float(np.nanmax(e)) if np.all(np.isfinite(e)) else np.inf for e in errs)
    return max(worst, abs(f["loglik"] - bf["loglik"]) / max(1.0, abs(bf["loglik"])))


def test_time_varying_matches_bruteforce(case):
    m, y, bf = case
    assert _worst(oracle.srtm_oracle, m, y, bf) < 1e-9


def test_constant_windows_equal_time_invariant():
    m = wl.random_general_model(3, 2, 4, 311)
    y = wl.simulate(m, 7, 312)
    N = y.shape[0]
    rep = lambda X: np.repeat(X[None], N, axis=0)  # noqa: E731
    a = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, with_filter=True)
    b = oracle.srtm_smoother_tv(rep(m.A), rep(m.Q), rep(m.C), rep(m.R), m.L, m.m0, m.P0, y, with_filter=True)
    for k in ("ms_fast", "Ps_fast", "m_fast", "P_fast", "m_slow", "P_slow"):
        assert np.allclose(a[k], b[k], rtol=0, atol=1e-13), k
    assert abs(a["loglik"] - b["loglik"]) < 1e-10


TV_MUTATIONS = [
    ("smoother predicts with the current window's A",
     "Ahat = np.hstack([np.zeros((nx, (L - 1) * nx)), A[k + 1]])", "Ahat = np.hstack([np.zeros((nx, (L - 1) * nx)), A[k]])"),
    ("smoother predicts with the current window's Q", "(Q[k + 1] if tv else Q)", "(Q[k] if tv else Q)"),
    ("IMKF update with the next window's R", "Rk = R[k] if tv else R", "Rk = R[min(k + 1, len(R) - 1)] if tv else R"),
    ("IMKF uses the first window's model throughout", "sr = slow_rate_model(A[k], Q[k], C[k], L)",
     "sr = slow_rate_model(A[0], Q[0], C[0], L)"),
    ("window filter with the first window's model", "            bm = batch_model(A[k], Q[k], C[k], L)\n        M_f, P_f = fast_filter_window(bm, R[k] if tv else R, mp, Pp, y[k], None if B is None else u[k])\n        if with_filter:",
     "            bm = batch_model(A[0], Q[0], C[0], L)\n        M_f, P_f = fast_filter_window(bm, R[k] if tv else R, mp, Pp, y[k], None if B is None else u[k])\n        if with_filter:"),
]


@pytest.mark.parametrize("name,old,new", TV_MUTATIONS, ids=[m[0] for m in TV_MUTATIONS])
def test_planted_tv_mistake_is_caught(case, name, old, new):
    m, y, bf = case
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {old!r}"
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    assert _worst(mod, m, y, bf) > 1e-6, f"pins did not catch: {name}"
