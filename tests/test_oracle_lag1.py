"""Lag-one smoothed cross-covariances of the CPU reference (run on the CPU only).

Cov(x_{k,i}, x_{k,i-1} | y_{1:N}), with x_{k,0} = x_{k-1,l} and x_{1,0} = x_0, against the
off-diagonal blocks of the brute-force joint posterior, for time-invariant models (l = 1
included, where every pair crosses a window boundary), known inputs and per-window models; and
planted mistakes in the three places the reference forms them are each caught.
"""
import os
import types

import numpy as np
import pytest

import oracle
from paper_2410_00627_amd import workloads as wl
from brute_force import posteriors

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "srtm_oracle.py")


def lag1_error(C, Cref, Pref):
    """Max over fast steps of |C - Cref|_F / sqrt(|P_t|_F |P_{t-1}|_F), with P_{t-1} the
    smoothed covariance of the earlier state (the prior's P0 is not in Pref: its own block)."""
    N, L = C.shape[:2]
    flat = Pref.reshape(N * L, *Pref.shape[2:])
    worst = 0.0
    for t in range(N * L):
        prev = np.linalg.norm(flat[t - 1]) if t > 0 else np.linalg.norm(flat[0])
        scale = np.sqrt(np.linalg.norm(flat[t]) * prev)
        worst = max(worst, float(np.linalg.norm(C.reshape(N * L, *C.shape[2:])[t] -
                                                Cref.reshape(N * L, *Cref.shape[2:])[t]) / scale))
    return worst


CASES = [("stable", 2, 1, 3, 4), ("general", 3, 2, 4, 3), ("general", 2, 2, 1, 6), ("stable", 4, 2, 2, 3)]


@pytest.mark.parametrize("kind,nx,ny,L,N", CASES, ids=[f"{c[0]}-nx{c[1]}ny{c[2]}L{c[3]}N{c[4]}" for c in CASES])
def test_lag1_matches_brute_force(kind, nx, ny, L, N):
    m = (wl.random_stable_model if kind == "stable" else wl.random_general_model)(nx, ny, L, 11 + nx + L)
    y = wl.simulate(m, N, 12 + nx)
    bf = posteriors(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y)
    s = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, lag1=True)
    assert lag1_error(s["Cs_fast"], bf["Cs_fast"], bf["Ps_fast"]) < 1e-9


def test_lag1_with_inputs_matches_brute_force():
    m = wl.random_general_model(3, 1, 3, 21)
    N = 4
    B, u = wl.random_inputs(3, 2, 3, N, 22)
    y = wl.simulate(m, N, 23, B=B, u=u)
    bf = posteriors(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, B, u)
    s = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, B=B, u=u, lag1=True)
    assert lag1_error(s["Cs_fast"], bf["Cs_fast"], bf["Ps_fast"]) < 1e-9


def test_lag1_per_window_model_matches_brute_force():
    m = wl.time_varying_model(2, 1, 3, 4, 31, general=True)
    y = wl.simulate_tv(m, 32)
    bf = posteriors(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y)
    s = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, lag1=True)
    assert lag1_error(s["Cs_fast"], bf["Cs_fast"], bf["Ps_fast"]) < 1e-9


MUTATIONS = [
    ("boundary term not transposed", "Cs_fast[k + 1, 0] = (G @ Ps1)[(L - 1) * nx:, :].T",
     "Cs_fast[k + 1, 0] = (G @ Ps1)[(L - 1) * nx:, :]"),
    ("boundary term from the first block row", "Cs_fast[k + 1, 0] = (G @ Ps1)[(L - 1) * nx:, :].T",
     "Cs_fast[k + 1, 0] = (G @ Ps1)[:nx, :].T"),
    ("within-window block one step off", "Cs_fast[k, i] = P_s[i * nx:(i + 1) * nx, (i - 1) * nx:i * nx]",
     "Cs_fast[k, i] = P_s[i * nx:(i + 1) * nx, i * nx:(i + 1) * nx]"),
    ("prior step without Q", "P_one = A1 @ P0 @ A1.T + Q1", "P_one = A1 @ P0 @ A1.T"),
    ("prior gain transposed", "Cs_fast[0, 0] = (G0 @ Ps_fast[0, 0]).T", "Cs_fast[0, 0] = G0 @ Ps_fast[0, 0]"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_lag1_planted_mistake_is_caught(name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {old!r}"
    mod = types.ModuleType("oracle_lag1_mutant")
    exec(compile(src.replace(old, new), "oracle_lag1_mutant", "exec"), mod.__dict__)
    m = wl.random_general_model(3, 2, 4, 41)
    y = wl.simulate(m, 3, 42)
    bf = posteriors(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y)
    s = mod.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, lag1=True)
    assert lag1_error(s["Cs_fast"], bf["Cs_fast"], bf["Ps_fast"]) > 1e-6, f"not caught: {name}"
