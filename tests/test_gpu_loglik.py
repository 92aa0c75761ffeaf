"""Log-likelihood and its gradient on the GPU (srtm_loglik, srtm_loglik_grad, autograd).

The log-likelihood is compared with the float64 IMKF reference; the gradient with central
finite differences of that reference (h = 1e-6), including the parameterisation
theta = (log q, log r, entries of F) with Q = q I and R = r I.
"""
import numpy as np
import pytest

import oracle
from paper_2410_00627_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _srtm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_00627_amd import srtm
    srtm.lib()
    return srtm


def _t(a, dtype):
    return torch.as_tensor(np.asarray(a, dtype=np.float64)).to("cuda", dtype).contiguous()


def _rounded(a, dtype):
    a = np.asarray(a, dtype=np.float64)
    return a if dtype == torch.float64 else a.astype(np.float32).astype(np.float64)


CASES = [(2, 1, 3, 60, 81), (4, 2, 5, 150, 82), (4, 1, 10, 120, 83), (3, 2, 1, 80, 84)]


@pytest.mark.parametrize("nx,ny,L,N,seed", CASES, ids=[f"nx{c[0]}ny{c[1]}L{c[2]}N{c[3]}" for c in CASES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_loglik_and_gradient_against_finite_differences(nx, ny, L, N, seed, dtype):
    srtm = _srtm()
    m = wl.random_general_model(nx, ny, L, seed)
    y = wl.simulate(m, N, seed + 1)
    args = [_t(x, dtype) for x in (m.A, m.Q, m.C, m.R)] + [L] + [_t(x, dtype) for x in (m.m0, m.P0, y)]
    print(f"[gpu] loglik_grad nx={nx} ny={ny} L={L} N={N} {dtype}", flush=True)
    ll, dF, dQ, dR = srtm.loglik_grad(*args)
    ll_only = srtm.loglik(*args)
    torch.cuda.synchronize()
    r = {k: _rounded(v, dtype) for k, v in dict(A=m.A, Q=m.Q, C=m.C, R=m.R, m0=m.m0, P0=m.P0, y=y).items()}
    ref_ll = oracle.imkf(r["A"], r["Q"], r["C"], r["R"], L, r["m0"], r["P0"], r["y"])[2]
    tol_ll = 1e-10 if dtype == torch.float64 else 2e-5
    assert abs(float(ll) - ref_ll) <= tol_ll * max(1.0, abs(ref_ll))
    assert abs(float(ll_only) - ref_ll) <= tol_ll * max(1.0, abs(ref_ll))
    gA, gQ, gR = oracle.loglik_grad_fd(r["A"], r["Q"], r["C"], r["R"], L, r["m0"], r["P0"], r["y"])
    tol = 1e-6 if dtype == torch.float64 else 1e-3
    for name, got, want in (("F", dF, gA), ("Q", dQ, gQ), ("R", dR, gR)):
        got = got.double().cpu().numpy()
        scale = max(1.0, np.max(np.abs(want)))
        err = np.max(np.abs(got - want)) / scale
        print(f"[gpu]   d/d{name}: max rel err {err:.2e} (scale {scale:.3g})", flush=True)
        assert err <= tol, f"d/d{name}: {err:.3e}"


def test_autograd_log_parameters_match_finite_differences():
    """theta = (log q, log r, vec F) with Q = q I, R = r I, through torch.autograd."""
    srtm = _srtm()
    nx, ny, L, N = 4, 1, 10, 200
    m = wl.random_stable_model(nx, ny, L, 91, rho=0.99, q=0.01, r=0.1)
    y = wl.simulate(m, N, 92)
    dt = torch.float64
    logq = torch.tensor(np.log(0.01), dtype=dt, device="cuda", requires_grad=True)
    logr = torch.tensor(np.log(0.1), dtype=dt, device="cuda", requires_grad=True)
    F = _t(m.A, dt).requires_grad_(True)
    eye_x = torch.eye(nx, dtype=dt, device="cuda")
    eye_y = torch.eye(ny, dtype=dt, device="cuda")
    ll = srtm.log_likelihood(F, torch.exp(logq) * eye_x, torch.exp(logr) * eye_y, _t(m.C, dt), L, _t(m.m0, dt),
                             _t(m.P0, dt), _t(y, dt))
    ll.backward()

    def ref(theta):
        A = theta[2:].reshape(nx, nx)
        return oracle.imkf(A, np.exp(theta[0]) * np.eye(nx), m.C, np.exp(theta[1]) * np.eye(ny), L, m.m0, m.P0,
                           y)[2]

    th = np.concatenate([[np.log(0.01), np.log(0.1)], m.A.ravel()])
    fd = np.zeros_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = 1e-6
        fd[i] = (ref(th + e) - ref(th - e)) / 2e-6
    got = np.concatenate([[logq.grad.item(), logr.grad.item()], F.grad.cpu().numpy().ravel()])
    assert abs(ll.item() - ref(th)) <= 1e-10 * abs(ref(th))
    err = np.max(np.abs(got - fd)) / max(1.0, np.max(np.abs(fd)))
    print(f"[gpu] autograd theta grad max rel err {err:.2e}", flush=True)
    assert err <= 1e-6


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batched_gradient_equals_single_calls(dtype):
    srtm = _srtm()
    specs = [(4, 1, 10, 50, 101), (4, 1, 10, 300, 102), (4, 1, 5, 1, 103), (4, 1, 10, 257, 104), (4, 1, 20, 900, 105)]
    probs = []
    for nx, ny, L, N, seed in specs:
        m = wl.random_stable_model(nx, ny, L, seed, rho=0.99, q=0.01, r=0.1)
        y = wl.simulate(m, N, seed + 1)
        probs.append(tuple(_t(x, dtype) for x in (m.A, m.Q, m.C, m.R)) + (L,) +
                     tuple(_t(x, dtype) for x in (m.m0, m.P0, y)))
    b = srtm.Batch(probs, grad=True)
    b.launch()
    torch.cuda.synchronize()
    b.check()
    for j, pr in enumerate(probs):
        ll, dF, dQ, dR = srtm.loglik_grad(*pr)
        o = b.outputs[j]
        for got, want in ((o["ll"][0], ll), (o["dF"], dF), (o["dQ"], dQ), (o["dR"], dR)):
            assert torch.equal(got, want), f"sequence {j}"


IN_CASES = [(4, 2, 5, 150, 2, 131), (2, 1, 10, 300, 1, 132), (3, 1, 4, 90, 3, 133)]


@pytest.mark.parametrize("nx,ny,L,N,nu,seed", IN_CASES, ids=[f"nx{c[0]}ny{c[1]}L{c[2]}N{c[3]}nu{c[4]}" for c in IN_CASES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_gradient_with_inputs_against_finite_differences(nx, ny, L, N, nu, seed, dtype):
    """srtm_loglik_grad_inputs: the log-likelihood against the IMKF with inputs and the gradient
    against central differences of it (h = 1e-6), at the tolerances of the input-free test."""
    srtm = _srtm()
    m = wl.random_general_model(nx, ny, L, seed)
    B, u = wl.random_inputs(nx, nu, L, N, seed + 2)
    y = wl.simulate(m, N, seed + 1, B=B, u=u)
    args = [_t(x, dtype) for x in (m.A, m.Q, m.C, m.R)] + [L] + [_t(x, dtype) for x in (m.m0, m.P0, y)]
    print(f"[gpu] loglik_grad with inputs nx={nx} ny={ny} L={L} N={N} nu={nu} {dtype}", flush=True)
    ll, dF, dQ, dR = srtm.loglik_grad(*args, B=_t(B, dtype), u=_t(u, dtype))
    torch.cuda.synchronize()
    r = {k: _rounded(v, dtype) for k, v in dict(A=m.A, Q=m.Q, C=m.C, R=m.R, m0=m.m0, P0=m.P0, y=y, B=B, u=u).items()}
    ref_ll = oracle.imkf(r["A"], r["Q"], r["C"], r["R"], L, r["m0"], r["P0"], r["y"], B=r["B"], u=r["u"])[2]
    tol_ll = 1e-10 if dtype == torch.float64 else 2e-5
    assert abs(float(ll) - ref_ll) <= tol_ll * max(1.0, abs(ref_ll))
    gA, gQ, gR = oracle.loglik_grad_fd(r["A"], r["Q"], r["C"], r["R"], L, r["m0"], r["P0"], r["y"], B=r["B"], u=r["u"])
    tol = 1e-6 if dtype == torch.float64 else 1e-3
    for name, got, want in (("F", dF, gA), ("Q", dQ, gQ), ("R", dR, gR)):
        got = got.double().cpu().numpy()
        scale = max(1.0, np.max(np.abs(want)))
        err = np.max(np.abs(got - want)) / scale
        print(f"[gpu]   d/d{name}: max rel err {err:.2e} (scale {scale:.3g})", flush=True)
        assert err <= tol, f"d/d{name}: {err:.3e}"


def test_gradient_with_zero_inputs_equals_gradient_without():
    """u = 0 makes the input path reproduce the input-free gradient to rounding."""
    srtm = _srtm()
    nx, ny, L, N = 4, 2, 5, 400
    m = wl.random_stable_model(nx, ny, L, 141)
    y = wl.simulate(m, N, 142)
    dt = torch.float64
    args = [_t(x, dt) for x in (m.A, m.Q, m.C, m.R)] + [L] + [_t(x, dt) for x in (m.m0, m.P0, y)]
    B = torch.randn(nx, 2, dtype=dt, device="cuda")
    u = torch.zeros(N, L, 2, dtype=dt, device="cuda")
    a = srtm.loglik_grad(*args)
    b = srtm.loglik_grad(*args, B=B, u=u)
    for x, z in zip(a, b):
        assert torch.allclose(x, z, rtol=1e-12, atol=1e-12)


def test_autograd_with_inputs_matches_finite_differences():
    """theta = (log q, log r, vec F) through torch.autograd with known inputs as constants."""
    srtm = _srtm()
    nx, ny, L, N, nu = 3, 1, 5, 150, 2
    m = wl.random_stable_model(nx, ny, L, 151, rho=0.99, q=0.01, r=0.1)
    B, u = wl.random_inputs(nx, nu, L, N, 152)
    y = wl.simulate(m, N, 153, B=B, u=u)
    dt = torch.float64
    logq = torch.tensor(np.log(0.01), dtype=dt, device="cuda", requires_grad=True)
    logr = torch.tensor(np.log(0.1), dtype=dt, device="cuda", requires_grad=True)
    F = _t(m.A, dt).requires_grad_(True)
    ll = srtm.log_likelihood(F, torch.exp(logq) * torch.eye(nx, dtype=dt, device="cuda"),
                             torch.exp(logr) * torch.eye(ny, dtype=dt, device="cuda"), _t(m.C, dt), L, _t(m.m0, dt),
                             _t(m.P0, dt), _t(y, dt), B=_t(B, dt), u=_t(u, dt))
    ll.backward()

    def ref(theta):
        A = theta[2:].reshape(nx, nx)
        return oracle.imkf(A, np.exp(theta[0]) * np.eye(nx), m.C, np.exp(theta[1]) * np.eye(ny), L, m.m0, m.P0, y,
                           B=B, u=u)[2]

    th = np.concatenate([[np.log(0.01), np.log(0.1)], m.A.ravel()])
    fd = np.zeros_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = 1e-6
        fd[i] = (ref(th + e) - ref(th - e)) / 2e-6
    got = np.concatenate([[logq.grad.item(), logr.grad.item()], F.grad.cpu().numpy().ravel()])
    assert abs(ll.item() - ref(th)) <= 1e-10 * abs(ref(th))
    err = np.max(np.abs(got - fd)) / max(1.0, np.max(np.abs(fd)))
    print(f"[gpu] autograd theta grad with inputs max rel err {err:.2e}", flush=True)
    assert err <= 1e-6
