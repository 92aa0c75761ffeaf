import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def rel_errors(m, P, m_ref, P_ref):
    """Per-state relative errors: e_m = |m - m_ref| / max(|m_ref|, sqrt(tr P_ref)),
    e_P = |P - P_ref|_F / |P_ref|_F. Arrays are [..., nx] and [..., nx, nx]."""
    m = np.asarray(m, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    dm = np.linalg.norm(m - m_ref, axis=-1)
    scale = np.maximum(np.linalg.norm(m_ref, axis=-1),
                       np.sqrt(np.maximum(np.trace(P_ref, axis1=-2, axis2=-1), 0.0)))
    scale = np.maximum(scale, 1e-300)
    dP = np.linalg.norm((P - P_ref).reshape(P.shape[:-2] + (-1,)), axis=-1)
    sP = np.maximum(np.linalg.norm(P_ref.reshape(P_ref.shape[:-2] + (-1,)), axis=-1), 1e-300)
    return dm / scale, dP / sP


def assert_close_states(m, P, m_ref, P_ref, tol, what=""):
    em, eP = rel_errors(m, P, m_ref, P_ref)
    assert np.all(np.isfinite(em)) and np.all(np.isfinite(eP)), f"{what}: non-finite"
    assert em.max() <= tol and eP.max() <= tol, (
        f"{what}: max mean err {em.max():.3e} at {np.unravel_index(em.argmax(), em.shape)}, "
        f"max cov err {eP.max():.3e} at {np.unravel_index(eP.argmax(), eP.shape)} (tol {tol:g})")
    return em.max(), eP.max()
