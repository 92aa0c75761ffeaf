"""The sequential comparator (srtm_smooth_sequential: IMKF forwards and the sequential SRTM smoother
backwards on one GPU lane, no scan) against the float64 CPU reference, at 1e-8 (float64) and 1e-3
(float32, reference on the rounded inputs), and against the parallel path on the same inputs.
"""
import numpy as np
import pytest

import oracle
from paper_2410_00627_amd import workloads as wl
from conftest import assert_close_states

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-8, torch.float32: 1e-3}


def _srtm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_00627_amd import srtm
    srtm.lib()
    return srtm


def _r(a, dtype):
    a = np.asarray(a, dtype=np.float64)
    return a if dtype == torch.float64 else a.astype(np.float32).astype(np.float64)


CASES = [("wna", 2, 1, 10, 100), ("stable", 4, 2, 16, 600), ("general", 3, 2, 4, 257), ("stable", 2, 1, 1, 300),
         ("stable", 6, 1, 5, 200), ("general", 4, 1, 7, 1), ("general", 4, 2, 20, 2)]
PARAMS = [(c, d) for c in CASES for d in (torch.float64, torch.float32)]


@pytest.mark.parametrize("case,dtype", PARAMS, ids=[f"{'f64' if d == torch.float64 else 'f32'}-{c[0]}-nx{c[1]}"
                                                    f"ny{c[2]}L{c[3]}N{c[4]}" for c, d in PARAMS])
def test_sequential_against_reference(case, dtype):
    srtm = _srtm()
    kind, nx, ny, L, N = case
    if kind == "wna":
        m = wl.wna_model()
    else:
        make = wl.random_stable_model if kind == "stable" else wl.random_general_model
        m = make(nx, ny, L, 400 + N)
    y = wl.simulate(m, N, 401 + N)
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", dtype)
    yt = torch.as_tensor(y, dtype=torch.float64).to("cuda", dtype)
    print(f"[gpu] sequential {kind} nx={nx} ny={ny} L={L} N={N} {dtype}", flush=True)
    seq = srtm.smooth_sequential(F, Q, H, R, m.L, m0, P0, yt)
    par = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt)
    torch.cuda.synchronize()
    g = {k: v.double().cpu().numpy() for k, v in seq.items()}
    p = {k: v.double().cpu().numpy() for k, v in par.items()}
    ref = oracle.srtm_smoother(_r(m.A, dtype), _r(m.Q, dtype), _r(m.C, dtype), _r(m.R, dtype), m.L,
                               _r(m.m0, dtype), _r(m.P0, dtype), _r(y, dtype))
    tol = TOL[dtype]
    assert int(g["info"][0]) == 0
    assert_close_states(g["ms_fast"], g["Ps_fast"], ref["ms_fast"], ref["Ps_fast"], tol, "sequential fast")
    assert_close_states(g["ms_slow"], g["Ps_slow"], ref["ms_slow"], ref["Ps_slow"], tol, "sequential slow")
    assert_close_states(g["ms_fast"], g["Ps_fast"], p["ms_fast"], p["Ps_fast"], 2 * tol, "sequential vs parallel")
    assert np.array_equal(g["Ps_fast"], np.swapaxes(g["Ps_fast"], -1, -2))


def test_sequential_long_sequence():
    """20,000 windows of the long-sequence model (nx=4, ny=2, L=20), float64, every window against
    the reference."""
    srtm = _srtm()
    m = wl.headline_model()
    N = 20000
    y = wl.simulate(m, N, seed=2033)
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", torch.float64)
    yt = torch.as_tensor(y, device="cuda")
    print(f"[gpu] sequential long N={N}", flush=True)
    g = {k: v.cpu().numpy() for k, v in srtm.smooth_sequential(F, Q, H, R, m.L, m0, P0, yt).items()}
    ref = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y)
    assert_close_states(g["ms_fast"], g["Ps_fast"], ref["ms_fast"], ref["Ps_fast"], 1e-8, "sequential long")
