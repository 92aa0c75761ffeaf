"""Parity at the full sizes of the batched and gradient workloads, in the launch configurations
bench.py times, on outputs the float64 CPU reference can compute one by one.

* Batched: the 256-sequence workload (nx in {2, 4, 6}, L in {5, 10, 20}, N = round(2^U(8,14)),
  ny = 1), float32, in the tuned configuration (two segments per size group, one stream each,
  captured in a HIP graph). Checked: the float64 path on the same (rounded) inputs agrees to
  1e-3 everywhere; for sampled sequences, the float64 path matches the reference on the last
  windows (dense smoother started from the IMKF carry) and at sampled windows (one step of the
  sequential smoother from the GPU's smoothed state of the next window reproduces the window).
* Gradient: 64 sequences of N = 2^14 windows (nx = 4, ny = 1, L = 10), float32, batched; the
  log-likelihood of two sequences against the IMKF; for one sequence the float64 gradient against
  central finite differences of the float64 reference (1e-6) and the float32 gradient against the
  float64 one within the float32 conditioning bound of a gradient that is a small difference of
  large sums (near the data's own parameters it nearly vanishes).
"""
import numpy as np
import pytest

import oracle
from paper_2410_00627_amd import workloads as wl
from conftest import assert_close_states, rel_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _srtm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_00627_amd import srtm
    srtm.lib()
    return srtm


def _r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _smoother_step_check(mr, yr, ms_slow_next, Ps_slow_next, m_prev, P_prev, k, got_m, got_P, tol, what):
    """One step of the sequential smoother (eq. seq-smoothing-all) for window k from the GPU's
    smoothed slow state of window k+1 and the reference's filtered window k."""
    nx, L = mr.A.shape[0], mr.L
    bm = oracle.batch_model(mr.A, mr.Q, mr.C, L)
    M_f, P_f = oracle.fast_filter_window(bm, mr.R, m_prev, P_prev, yr[k])
    Ahat = np.hstack([np.zeros((nx, (L - 1) * nx)), mr.A])
    mpr = Ahat @ M_f
    Ppr = Ahat @ P_f @ Ahat.T + mr.Q
    G = np.linalg.solve(Ppr.T, (P_f @ Ahat.T).T).T
    M_s = M_f + G @ (ms_slow_next - mpr)
    P_s = P_f + G @ (Ps_slow_next - Ppr) @ G.T
    ms = M_s.reshape(L, nx)
    Ps = np.stack([P_s[i * nx:(i + 1) * nx, i * nx:(i + 1) * nx] for i in range(L)])
    assert_close_states(got_m, got_P, ms, Ps, tol, what)


def test_batched_workload_full_size():
    srtm = _srtm()
    from paper_2410_00627_amd import batching
    specs = wl.batched_specs()
    models, ys, p32 = [], [], []
    for nx, L, N, seed in specs:
        m = wl.batched_model(nx, L, seed)
        y = wl.simulate(m, N, seed + 1)
        F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", torch.float32)
        p32.append((F, Q, H, R, L, m0, P0, torch.as_tensor(y, dtype=torch.float64).to("cuda", torch.float32)))
        models.append(m)
        ys.append(y)
    print(f"[gpu] batched workload: {len(specs)} sequences, {sum(s[2] for s in specs)} windows", flush=True)
    r32 = batching.BatchRunner(p32, segments=2, multi_stream=True, graph=True)
    r32.zero_info()
    r32.run()
    torch.cuda.synchronize()
    r32.check()
    p64 = [tuple(t.double() if isinstance(t, torch.Tensor) else t for t in pr) for pr in p32]
    r64 = batching.BatchRunner(p64)
    r64.zero_info()
    r64.run()
    torch.cuda.synchronize()
    r64.check()
    worst = 0.0
    for j in range(len(specs)):
        a, b = r32.outputs[j], r64.outputs[j]
        for mk, pk in (("ms_fast", "Ps_fast"), ("ms_slow", "Ps_slow")):
            em, ep = rel_errors(a[mk].double().cpu().numpy(), a[pk].double().cpu().numpy(),
                                b[mk].cpu().numpy(), b[pk].cpu().numpy())
            worst = max(worst, float(em.max()), float(ep.max()))
    print(f"[gpu] float32 vs float64 path, all 256 sequences: max rel err {worst:.2e}", flush=True)
    assert worst <= 1e-3
    # reference checks of the float64 path on sampled sequences (inputs rounded as for float32)
    Ns = [s[2] for s in specs]
    pick = {int(np.argmin(Ns)), int(np.argmax(Ns))}
    for nxv in (2, 4, 6):
        pick.add(next(j for j, s in enumerate(specs) if s[0] == nxv))
    rng = np.random.default_rng(5)
    for j in sorted(pick):
        m, y = models[j], ys[j]
        mr = wl.Model(_r32(m.A), _r32(m.Q), _r32(m.C), _r32(m.R), m.L, _r32(m.m0), _r32(m.P0), m.name)
        yr = _r32(y)
        N, L = y.shape[0], m.L
        o = {k: v.cpu().numpy() for k, v in r64.outputs[j].items()}
        ms, Ps, _ = oracle.imkf(mr.A, mr.Q, mr.C, mr.R, L, mr.m0, mr.P0, yr)
        n = min(12, N - 1)
        tail = oracle.srtm_smoother(mr.A, mr.Q, mr.C, mr.R, L, ms[N - n - 1], Ps[N - n - 1], yr[N - n:])
        assert_close_states(o["ms_fast"][N - n:], o["Ps_fast"][N - n:], tail["ms_fast"], tail["Ps_fast"], 1e-8,
                            f"seq {j} (nx={m.nx} L={L} N={N}) smoother tail")
        for k in sorted(set(rng.integers(0, N - 1, 6).tolist()) | {0, N - 2}):
            mp, Pp = (mr.m0, mr.P0) if k == 0 else (ms[k - 1], Ps[k - 1])
            _smoother_step_check(mr, yr, o["ms_slow"][k + 1], o["Ps_slow"][k + 1], mp, Pp, k,
                                 o["ms_fast"][k], o["Ps_fast"][k], 1e-7, f"seq {j} window {k}")
        print(f"[gpu] sequence {j} (nx={m.nx} L={L} N={N}) matches the reference", flush=True)


def test_gradient_workload_full_size():
    srtm = _srtm()
    probs, models, ys = [], [], []
    for j in range(64):
        m = wl.random_stable_model(4, 1, 10, 5000 + j, rho=0.99, q=0.01, r=0.1)
        y = wl.simulate(m, 1 << 14, 6000 + j)
        conv = lambda a: torch.as_tensor(a, dtype=torch.float64).to("cuda", torch.float32).contiguous()  # noqa: E731
        probs.append((conv(m.A), conv(m.Q), conv(m.C), conv(m.R), 10, conv(m.m0), conv(m.P0), conv(y)))
        models.append(m)
        ys.append(y)
    print("[gpu] gradient workload: 64 x 2^14 windows, float32", flush=True)
    b = srtm.Batch(probs, grad=True)
    b.launch()
    torch.cuda.synchronize()
    b.check()
    for j in (0, 37):
        m = models[j]
        r = {k: _r32(v) for k, v in dict(A=m.A, Q=m.Q, C=m.C, R=m.R, m0=m.m0, P0=m.P0, y=ys[j]).items()}
        ref_ll = oracle.imkf(r["A"], r["Q"], r["C"], r["R"], 10, r["m0"], r["P0"], r["y"])[2]
        got = float(b.outputs[j]["ll"][0])
        print(f"[gpu] sequence {j}: ll {got:.6f} reference {ref_ll:.6f}", flush=True)
        assert abs(got - ref_ll) <= 2e-5 * max(1.0, abs(ref_ll))
        if j == 0:
            # float64 path on the same (rounded) inputs against the reference's central differences
            t64 = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()  # noqa: E731
            ll64, dF64, dQ64, dR64 = srtm.loglik_grad(t64(r["A"]), t64(r["Q"]), t64(r["C"]), t64(r["R"]), 10,
                                                      t64(r["m0"]), t64(r["P0"]), t64(r["y"]))
            gA, gQ, gR = oracle.loglik_grad_fd(r["A"], r["Q"], r["C"], r["R"], 10, r["m0"], r["P0"], r["y"])
            o = b.outputs[j]
            T, Nw = 10 << 14, 1 << 14
            eps = float(np.finfo(np.float32).eps)
            ex = 1.0  # bound on the entries of E[x x^T] of this stable model (stationary variance 0.5)
            iq = np.linalg.norm(np.linalg.inv(r["Q"]), 2)
            ir = np.linalg.norm(np.linalg.inv(r["R"]), 2)
            # float32 conditioning: the gradients are differences of sums of T second moments, each
            # carried with relative error ~eps, scaled by Q^{-1} (F), Q^{-1}..Q^{-1} (Q), R^{-1}..R^{-1} (R)
            bound32 = {"F": iq * T * eps * ex, "Q": 0.5 * iq * iq * T * eps * ex, "R": 0.5 * ir * ir * Nw * eps * ex}
            for name, g32, g64, want in (("F", o["dF"], dF64, gA), ("Q", o["dQ"], dQ64, gQ), ("R", o["dR"], dR64, gR)):
                g32 = g32.double().cpu().numpy()
                g64 = g64.cpu().numpy()
                scale = max(1.0, np.max(np.abs(want)))
                e64 = np.max(np.abs(g64 - want)) / scale
                e32 = np.max(np.abs(g32 - g64))
                print(f"[gpu]   d/d{name}: float64 vs differences {e64:.2e} (scale {scale:.3g}); "
                      f"float32 vs float64 {e32:.3g} (bound {bound32[name]:.3g})", flush=True)
                assert e64 <= 1e-6, f"d/d{name} float64: {e64:.3e}"
                assert e32 <= bound32[name], f"d/d{name} float32: {e32:.3e} > {bound32[name]:.3e}"
