"""Pins of the reference with inputs (x_t = A x_{t-1} + B u_{t-1} + w_{t-1}).

* Brute force: filter and smoother marginals and the log-likelihood from one dense joint
  Gaussian whose prior mean carries the input response (tests/brute_force.py).
* Zero inputs reproduce the input-free results.
* Planted mistakes in the input terms are caught by the brute-force comparison.
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


@pytest.fixture(scope="module", params=[(3, 2, 4, 2, 6, 201), (2, 1, 1, 1, 9, 202), (4, 2, 3, 3, 5, 203)],
                ids=["nx3ny2L4nu2", "nx2ny1L1nu1", "nx4ny2L3nu3"])
def case(request):
    nx, ny, L, nu, N, seed = request.param
    m = wl.random_general_model(nx, ny, L, seed)
    B, u = wl.random_inputs(nx, nu, L, N, seed + 1)
    y = wl.simulate(m, N, seed + 2, B=B, u=u)
    bf = posteriors(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, B, u)
    return m, B, u, y, bf


def _worst(mod, m, B, u, y, bf):
    args = (m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y)
    f = mod.srtm_filter(*args, B=B, u=u)
    s = mod.srtm_smoother(*args, B=B, u=u)
    errs = [*rel_errors(f["m_fast"], f["P_fast"], bf["m_fast"], bf["P_fast"]),
            *rel_errors(s["ms_fast"], s["Ps_fast"], bf["ms_fast"], bf["Ps_fast"])]
    worst = max(float(np.nanmax(e)) if np.all(np.isfinite(e)) else np.inf for e in errs)
    worst = max(worst, abs(f["loglik"] - bf["loglik"]) / max(1.0, abs(bf["loglik"])))
    return worst


def test_inputs_match_bruteforce(case):
    m, B, u, y, bf = case
    assert _worst(oracle.srtm_oracle, m, B, u, y, bf) < 1e-9


def test_zero_inputs_equal_input_free():
    m = wl.random_general_model(3, 2, 4, 211)
    y = wl.simulate(m, 7, 212)
    B, _ = wl.random_inputs(3, 2, 4, 7, 213)
    a = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, with_filter=True)
    b = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, with_filter=True, B=B, u=np.zeros((7, 4, 2)))
    for k in ("ms_fast", "Ps_fast", "m_fast", "P_fast", "m_slow", "P_slow"):
        assert np.allclose(a[k], b[k], rtol=0, atol=1e-13)


INPUT_MUTATIONS = [
    ("smoother prediction drops the boundary input",
     "m_pred = Ahat @ M_f + (0.0 if B is None else B @ np.asarray(u[k + 1][0], dtype=float))",
     "m_pred = Ahat @ M_f"),
    ("smoother prediction uses the window's own first input",
     "B @ np.asarray(u[k + 1][0], dtype=float)", "B @ np.asarray(u[k][0], dtype=float)"),
    ("IMKF prediction drops B_bar u", "m_pred = Abar @ m + (0.0 if ub is None else sr[\"Bbar\"] @ ub)",
     "m_pred = Abar @ m"),
    ("IMKF innovation drops D_bar u", "innov = y[k] - Cbar @ m - (0.0 if ub is None else sr[\"Dbar\"] @ ub)",
     "innov = y[k] - Cbar @ m"),
    ("window input stacked in reverse", "M_pred = M_pred + bm[\"calB\"] @ np.asarray(uk, dtype=float).reshape(-1)",
     "M_pred = M_pred + bm[\"calB\"] @ np.asarray(uk, dtype=float)[::-1].reshape(-1)"),
    ("B_bar without the powers of A", "out.update(Bbar=Gbar @ Btilde, Dbar=Mbar @ Btilde)",
     "out.update(Bbar=np.hstack([B] * L), Dbar=Mbar @ Btilde)"),
    ("D_bar with the wrong sign", "out.update(Bbar=Gbar @ Btilde, Dbar=Mbar @ Btilde)",
     "out.update(Bbar=Gbar @ Btilde, Dbar=-(Mbar @ Btilde))"),
]


@pytest.mark.parametrize("name,old,new", INPUT_MUTATIONS, ids=[m[0] for m in INPUT_MUTATIONS])
def test_planted_input_mistake_is_caught(case, name, old, new):
    m, B, u, y, bf = case
    if m.L == 1 and ("reverse" in name or "powers" in name):
        pytest.skip("one step per window: the mistake does not change the arithmetic")
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {old!r}"
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    assert _worst(mod, m, B, u, y, bf) > 1e-6, f"pins did not catch: {name}"
