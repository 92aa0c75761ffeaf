"""Planted mistakes in the CPU reference must be caught by its pins (run on the CPU only).

Each case edits one expression of oracle/srtm_oracle.py in memory (a dropped term, a
wrong sign, a wrong index or a transposed operand), loads the edited source as a
throw-away module, and checks that the brute-force posteriors or the closed-form
constants then disagree with it. The committed oracle is never modified.
"""
import os
import types

import numpy as np
import pytest

from paper_2410_00627_amd import workloads as wl
from brute_force import posteriors, one_window_moments
from conftest import rel_errors

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "srtm_oracle.py")

MUTATIONS = [
    ("drop IMKF cross term", "cross = Abar @ P @ Cbar.T + Gbar @ Qt @ Mbar.T", "cross = Abar @ P @ Cbar.T"),
    ("drop M_bar noise in S", "S = Cbar @ P @ Cbar.T + Mbar @ Qt @ Mbar.T + R", "S = Cbar @ P @ Cbar.T + R"),
    ("innovation from predicted mean", "innov = y[k] - Cbar @ m", "innov = y[k] - Cbar @ m_pred"),
    ("G_bar index off by one", "Gbar = np.hstack([_mpow(A, L - 1 - j) for j in range(L)])",
     "Gbar = np.hstack([_mpow(A, L - j) for j in range(L)])"),
    ("C_bar sum from 0", "Cbar = (C / L) @ sum(_mpow(A, i) for i in range(1, L + 1))",
     "Cbar = (C / L) @ sum(_mpow(A, i) for i in range(0, L))"),
    ("M_bar blocks reversed", "for j in range(L)])\n    out = dict(Abar",
     "for j in reversed(range(L))])\n    out = dict(Abar"),
    ("calG transposed", "P_pred = calA @ P_prev @ calA.T + calG @ Qt @ calG.T",
     "P_pred = calA @ P_prev @ calA.T + calG.T @ Qt @ calG"),
    ("fast update sign", "M_f = M_pred + gain @ (yk - calH @ M_pred)", "M_f = M_pred - gain @ (yk - calH @ M_pred)"),
    ("calA starts at A^0", "calA = np.vstack([_mpow(A, i) for i in range(1, L + 1)])",
     "calA = np.vstack([_mpow(A, i) for i in range(0, L)])"),
    ("A_hat picks first block", "Ahat = np.hstack([np.zeros((nx, (L - 1) * nx)), A])",
     "Ahat = np.hstack([A, np.zeros((nx, (L - 1) * nx))])"),
    ("smoother gain sign", "M_s = M_f + G @ (ms1 - m_pred)", "M_s = M_f - G @ (ms1 - m_pred)"),
    ("smoother drops Q", "P_pred = Ahat @ P_f @ Ahat.T + (Q[k + 1] if tv else Q)\n", "P_pred = Ahat @ P_f @ Ahat.T\n"),
    ("smoother covariance correction sign", "P_s = _sym(P_f + G @ (Ps1 - P_pred) @ G.T)",
     "P_s = _sym(P_f + G @ (P_pred - Ps1) @ G.T)"),
    ("IMKF prediction with A_bar transposed", "P_pred = Abar @ P @ Abar.T + Qbar",
     "P_pred = Abar.T @ P @ Abar + Qbar"),
    ("smoother restarts from filtered block 1", "ms1, Ps1 = ms_fast[k, 0].copy(), Ps_fast[k, 0].copy()",
     "ms1, Ps1 = M_f[:nx].copy(), P_f[:nx, :nx].copy()"),
]


def _load_mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {old!r}"
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    return mod


@pytest.fixture(scope="module")
def case():
    m = wl.random_general_model(3, 2, 4, 77)
    y = wl.simulate(m, 6, 78)
    return m, y, posteriors(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y)


def _worst(mod, m, y, bf):
    args = (m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y)
    f = mod.srtm_filter(*args)
    s = mod.srtm_smoother(*args)
    errs = [*rel_errors(f["m_fast"], f["P_fast"], bf["m_fast"], bf["P_fast"]),
            *rel_errors(s["ms_fast"], s["Ps_fast"], bf["ms_fast"], bf["Ps_fast"])]
    worst = max(float(np.nanmax(e)) if np.all(np.isfinite(e)) else np.inf for e in errs)
    sr = mod.slow_rate_model(m.A, m.Q, m.C, m.L)
    Abar, Cbar, Qbar, Syx, Rx = one_window_moments(m.A, m.Q, m.C, m.R, m.L)
    for a, b in ((sr["Abar"], Abar), (sr["Cbar"], Cbar), (sr["Qbar"], Qbar),
                 (sr["Gbar"] @ sr["Qtilde"] @ sr["Mbar"].T, Syx)):
        worst = max(worst, float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)))
    return worst


def test_unmutated_reference_passes(case):
    m, y, bf = case
    assert _worst(_load_mutant("import numpy as np", "import numpy as np"), m, y, bf) < 1e-9


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(case, name, old, new):
    m, y, bf = case
    assert _worst(_load_mutant(old, new), m, y, bf) > 1e-6, f"pins did not catch: {name}"
