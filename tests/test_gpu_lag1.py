"""GPU parity of the lag-one smoothed cross-covariances (srtm_smooth_lag1) against the float64
CPU reference, Cs_fast[k, i-1] = Cov(x_{k,i}, x_{k,i-1} | y_{1:N}) with x_{k,0} = x_{k-1,L} and
x_{1,0} = x_0.

Metric: per fast state |C - C_ref|_F / sqrt(|P_t|_F |P_{t-1}|_F) with the reference's smoothed
covariances; 1e-8 (float64) and 1e-3 (float32, reference on the rounded inputs).
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


def _rounded(m, y, dtype):
    if dtype == torch.float64:
        return m, y
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    return wl.Model(r(m.A), r(m.Q), r(m.C), r(m.R), m.L, r(m.m0), r(m.P0), m.name), r(y)


def lag1_error(C, Cref, Pref):
    N, L = C.shape[:2]
    nx = C.shape[-1]
    C, Cref, Pref = (np.asarray(a).reshape(N * L, nx, nx) for a in (C, Cref, Pref))
    nP = np.linalg.norm(Pref, axis=(1, 2))
    prev = np.concatenate([nP[:1], nP[:-1]])
    return float((np.linalg.norm(C - Cref, axis=(1, 2)) / np.sqrt(nP * prev)).max())


def _run(srtm, m, y, dtype):
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", dtype)
    yt = torch.as_tensor(y, dtype=torch.float64).to("cuda", dtype)
    print(f"[gpu] smooth_lag1 nx={m.nx} ny={m.ny} L={m.L} N={y.shape[0]} {dtype}", flush=True)
    out = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, lag1=True)
    ref = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt)
    torch.cuda.synchronize()
    return ({k: v.double().cpu().numpy() for k, v in out.items()},
            {k: v.double().cpu().numpy() for k, v in ref.items()})


CASES = [("stable", 4, 2, 20, 600, 1), ("stable", 2, 1, 3, 300, 2), ("general", 3, 2, 1, 513, 3),
         ("general", 4, 2, 4, 300, 4), ("stable", 1, 1, 5, 257, 5), ("stable", 6, 1, 2, 260, 6)]
PARAMS = [(c, d) for c in CASES for d in (torch.float64, torch.float32)]


@pytest.mark.parametrize("case,dtype", PARAMS,
                         ids=[f"{'f64' if d == torch.float64 else 'f32'}-{c[0]}-nx{c[1]}ny{c[2]}L{c[3]}N{c[4]}"
                              for c, d in PARAMS])
def test_lag1_parity(case, dtype):
    kind, nx, ny, L, N, seed = case
    srtm = _srtm()
    make = wl.random_stable_model if kind == "stable" else wl.random_general_model
    m = make(nx, ny, L, 90 + seed)
    y = wl.simulate(m, N, 91 + seed)
    o, plain = _run(srtm, m, y, dtype)
    assert int(o["info"][0]) == 0
    mr, yr = _rounded(m, y, dtype)
    ref = oracle.srtm_smoother(mr.A, mr.Q, mr.C, mr.R, L, mr.m0, mr.P0, yr, lag1=True)
    err = lag1_error(o["Cs_fast"], ref["Cs_fast"], ref["Ps_fast"])
    print(f"[gpu] lag1 max err {err:.2e}", flush=True)
    assert err < TOL[dtype]
    for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):   # the same recovery as srtm_smooth
        assert np.array_equal(o[k], plain[k]), k


def test_lag1_edge_lengths():
    srtm = _srtm()
    for N in (1, 2, 255, 256, 257):
        m = wl.random_general_model(3, 2, 4, 80 + N)
        y = wl.simulate(m, N, 81 + N)
        o, _ = _run(srtm, m, y, torch.float64)
        ref = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, lag1=True)
        assert lag1_error(o["Cs_fast"], ref["Cs_fast"], ref["Ps_fast"]) < 1e-8, f"N={N}"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_lag1_full_size(dtype):
    """The long-sequence shape (nx=4, ny=2, L=20, N=2^17, 512 tiles): every window's lag-one
    cross-covariances and smoothed blocks against the reference smoother over the whole sequence
    (float32: reference on the rounded inputs), and the smoothed blocks equal to srtm_smooth's."""
    from threadpoolctl import threadpool_limits
    srtm = _srtm()
    m = wl.headline_model()
    N = wl.HEADLINE_N
    y = wl.simulate(m, N, seed=2032)
    o, plain = _run(srtm, m, y, dtype)
    assert int(o["info"][0]) == 0
    mr, yr = _rounded(m, y, dtype)
    with threadpool_limits(limits=1):
        ref = oracle.srtm_smoother(mr.A, mr.Q, mr.C, mr.R, m.L, mr.m0, mr.P0, yr, lag1=True)
    err = lag1_error(o["Cs_fast"], ref["Cs_fast"], ref["Ps_fast"])
    print(f"[gpu] lag1 full size {dtype}: max err {err:.2e}", flush=True)
    assert err < TOL[dtype]
    assert_close_states(o["ms_fast"], o["Ps_fast"], ref["ms_fast"], ref["Ps_fast"], TOL[dtype], "smoothed, all windows")
    for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
        assert np.array_equal(o[k], plain[k]), k


def test_lag1_refuses_inputs_and_filter_outputs():
    srtm = _srtm()
    m = wl.random_stable_model(2, 1, 3, 7)
    y = wl.simulate(m, 20, 8)
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", torch.float64)
    yt = torch.as_tensor(y, device="cuda")
    with pytest.raises(srtm.SrtmError):
        srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, lag1=True, with_filter=True)
