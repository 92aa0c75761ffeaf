"""GPU parity with known inputs (x_t = A x_{t-1} + B u_{t-1} + w_{t-1}) through the *_inputs
entry points, against the float64 CPU reference with the same inputs.

Tolerances as in test_gpu_parity: 1e-8 (float64), 1e-3 (float32, reference on rounded inputs).
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


def _round(a, dtype):
    return a if dtype == torch.float64 else np.asarray(a, dtype=np.float32).astype(np.float64)


def _case(nx, ny, L, N, nu, seed, dtype):
    m = wl.random_stable_model(nx, ny, L, seed)
    B, u = wl.random_inputs(nx, nu, L, N, seed + 7)
    y = wl.simulate(m, N, seed + 50, B=B, u=u)
    r = lambda a: _round(a, dtype)  # noqa: E731
    mr = wl.Model(r(m.A), r(m.Q), r(m.C), r(m.R), m.L, r(m.m0), r(m.P0), m.name)
    return m, B, u, y, mr, r(B), r(u), r(y)


def _gpu(srtm, m, B, u, y, dtype):
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", dtype)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to("cuda", dtype)  # noqa: E731
    return F, Q, H, R, m0, P0, t(y), t(B), t(u)


CASES = [
    # nx, ny, L, N, nu, seed -- several 256-window tiles with a ragged tail
    (4, 2, 20, 845, 2, 1),
    (2, 1, 10, 600, 1, 2),
    (3, 2, 7, 300, 3, 3),
    (1, 1, 3, 513, 1, 4),
    (2, 2, 1, 700, 2, 5),     # l = 1
    (6, 1, 5, 300, 4, 6),     # nx > 4, largest nu
]


@pytest.mark.parametrize("nx,ny,L,N,nu,seed", CASES, ids=[f"nx{c[0]}ny{c[1]}L{c[2]}N{c[3]}nu{c[4]}" for c in CASES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_smooth_inputs_parity(nx, ny, L, N, nu, seed, dtype):
    srtm = _srtm()
    m, B, u, y, mr, Br, ur, yr = _case(nx, ny, L, N, nu, seed, dtype)
    F, Q, H, R, m0, P0, yt, Bt, ut = _gpu(srtm, m, B, u, y, dtype)
    print(f"[gpu] smooth_inputs nx={nx} ny={ny} L={L} N={N} nu={nu} {dtype}", flush=True)
    out = srtm.smooth(F, Q, H, R, L, m0, P0, yt, with_filter=True, B=Bt, u=ut)
    torch.cuda.synchronize()
    o = {k: v.double().cpu().numpy() for k, v in out.items()}
    ref = oracle.srtm_smoother(mr.A, mr.Q, mr.C, mr.R, L, mr.m0, mr.P0, yr, with_filter=True, B=Br, u=ur)
    tol = TOL[dtype]
    assert int(o["info"][0]) == 0
    assert_close_states(o["ms_fast"], o["Ps_fast"], ref["ms_fast"], ref["Ps_fast"], tol, "smoothed fast")
    assert_close_states(o["ms_slow"], o["Ps_slow"], ref["ms_slow"], ref["Ps_slow"], tol, "smoothed slow")
    assert_close_states(o["mf_fast"], o["Pf_fast"], ref["m_fast"], ref["P_fast"], tol, "filtered fast")
    assert_close_states(o["mf_slow"], o["Pf_slow"], ref["m_slow"], ref["P_slow"], tol, "filtered slow")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_filter_and_loglik_inputs_parity(dtype):
    srtm = _srtm()
    m, B, u, y, mr, Br, ur, yr = _case(4, 2, 20, 845, 2, 11, dtype)
    F, Q, H, R, m0, P0, yt, Bt, ut = _gpu(srtm, m, B, u, y, dtype)
    print(f"[gpu] filter_inputs / loglik_inputs {dtype}", flush=True)
    f = srtm.filter(F, Q, H, R, m.L, m0, P0, yt, B=Bt, u=ut)
    ll = srtm.loglik(F, Q, H, R, m.L, m0, P0, yt, B=Bt, u=ut)
    torch.cuda.synchronize()
    ref = oracle.srtm_filter(mr.A, mr.Q, mr.C, mr.R, m.L, mr.m0, mr.P0, yr, B=Br, u=ur)
    tol = TOL[dtype]
    g = {k: v.double().cpu().numpy() for k, v in f.items()}
    assert_close_states(g["m_fast"], g["P_fast"], ref["m_fast"], ref["P_fast"], tol, "filter fast")
    assert_close_states(g["m_slow"], g["P_slow"], ref["m_slow"], ref["P_slow"], tol, "filter slow")
    assert abs(float(ll) - ref["loglik"]) <= tol * max(1.0, abs(ref["loglik"]))


def test_inputs_change_the_result_and_zero_inputs_do_not():
    """The input path with u = 0 reproduces the input-free path; nonzero inputs move the means."""
    srtm = _srtm()
    m, B, u, y, *_ = _case(3, 2, 7, 600, 2, 21, torch.float64)
    F, Q, H, R, m0, P0, yt, Bt, ut = _gpu(srtm, m, B, u, y, torch.float64)
    a = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, with_filter=True)
    z = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, with_filter=True, B=Bt, u=torch.zeros_like(ut))
    b = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, with_filter=True, B=Bt, u=ut)
    torch.cuda.synchronize()
    for k in ("ms_fast", "Ps_fast", "mf_fast", "Pf_fast", "ms_slow", "Ps_slow"):
        x, w = a[k].cpu().numpy(), z[k].cpu().numpy()
        assert np.allclose(x, w, rtol=1e-12, atol=1e-12 * np.abs(x).max()), k
    # covariances do not depend on the inputs, means do
    assert np.allclose(a["Ps_fast"].cpu().numpy(), b["Ps_fast"].cpu().numpy(), rtol=1e-12, atol=1e-14)
    assert not np.allclose(a["ms_fast"].cpu().numpy(), b["ms_fast"].cpu().numpy(), rtol=1e-3)


def test_inputs_edge_lengths():
    srtm = _srtm()
    for N in (1, 2, 255, 256, 257):
        m, B, u, y, *_ = _case(3, 2, 4, N, 2, 30 + N, torch.float64)
        F, Q, H, R, m0, P0, yt, Bt, ut = _gpu(srtm, m, B, u, y, torch.float64)
        print(f"[gpu] smooth_inputs N={N}", flush=True)
        o = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, with_filter=True, B=Bt, u=ut)
        torch.cuda.synchronize()
        ref = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, with_filter=True, B=B, u=u)
        o = {k: v.cpu().numpy() for k, v in o.items()}
        assert_close_states(o["ms_fast"], o["Ps_fast"], ref["ms_fast"], ref["Ps_fast"], 1e-8, f"N={N} smoothed")
        assert_close_states(o["mf_fast"], o["Pf_fast"], ref["m_fast"], ref["P_fast"], 1e-8, f"N={N} filtered")


def test_inputs_full_size_slow_filter():
    """nx=4, ny=2, L=20, N=2^17 with two inputs: the slow-rate filter at every window against the
    sequential IMKF with inputs, and the smoother over the last 24 windows against the dense
    smoother started from the IMKF carry."""
    srtm = _srtm()
    m = wl.headline_model()
    N = wl.HEADLINE_N
    B, u = wl.random_inputs(m.nx, 2, m.L, N, 2025)
    y = wl.simulate(m, N, 2026, B=B, u=u)
    F, Q, H, R, m0, P0, yt, Bt, ut = _gpu(srtm, m, B, u, y, torch.float64)
    print("[gpu] smooth_inputs headline size", flush=True)
    o = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, with_filter=True, B=Bt, u=ut)
    torch.cuda.synchronize()
    o = {k: v.cpu().numpy() for k, v in o.items()}
    assert int(o["info"][0]) == 0
    ms, Ps, _ = oracle.imkf(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, B, u)
    assert_close_states(o["mf_slow"], o["Pf_slow"], ms, Ps, 1e-8, "IMKF with inputs, all windows")
    n = 24
    tail = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, m.L, ms[N - n - 1], Ps[N - n - 1], y[N - n:], B=B, u=u[N - n:])
    assert_close_states(o["ms_fast"][N - n:], o["Ps_fast"][N - n:], tail["ms_fast"], tail["Ps_fast"], 1e-8,
                        "smoother tail with inputs")


def test_gradient_pass_log_likelihood_with_inputs_equals_loglik():
    """The gradient pass with inputs (both scans, then the statistics kernel) returns the same
    log-likelihood as the filter-only srtm_loglik_inputs, to rounding (the gradient itself is
    checked against finite differences in test_gpu_loglik.py)."""
    srtm = _srtm()
    m, B, u, y, *_ = _case(2, 1, 4, 50, 1, 41, torch.float64)
    F, Q, H, R, m0, P0, yt, Bt, ut = _gpu(srtm, m, B, u, y, torch.float64)
    ll_g = float(srtm.loglik_grad(F, Q, H, R, m.L, m0, P0, yt, B=Bt, u=ut)[0])
    ll = float(srtm.loglik(F, Q, H, R, m.L, m0, P0, yt, B=Bt, u=ut))
    assert abs(ll_g - ll) <= 1e-11 * max(1.0, abs(ll))
