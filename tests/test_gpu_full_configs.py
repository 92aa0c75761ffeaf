"""Parity at the full sizes of the batched and gradient workloads, in the launch configurations
bench.py times, on outputs the float64 CPU reference can compute one by one.

* Batched: the 256-sequence workload (nx in {2, 4, 6}, L in {5, 10, 20}, N = round(2^U(8,14)),
  ny = 1), float32, in the tuned configuration (two segments per size group, one stream each,
  captured in a HIP graph), and the float64 check run on the same rounded inputs: every window
  of every sequence against the reference smoother (1e-3 and 1e-8).
* Gradient: 64 sequences of N = 2^14 windows (nx = 4, ny = 1, L = 10), float32, batched; the
  log-likelihood of two sequences against the IMKF; for one sequence the float32 gradient (from
  the batch) and the float64 one against central finite differences of the float64 reference on
  the rounded inputs (h = 1e-6), relative to the largest entry: 1e-3 (float32), 1e-6 (float64).
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


def _r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def test_batched_workload_full_size():
    """All 256 sequences of the batched workload, element by element, against the reference's
    sequential smoother (run per sequence in worker processes, on the float32-rounded inputs):
    the float32 path in the tuned launch configuration (two segments per size group, one stream
    each, HIP-graph replay) at 1e-3, and the float64 check run on the same rounded inputs at 1e-8."""
    import oracle_pool
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
    jobs = []
    for j, m in enumerate(models):
        model = (_r32(m.A), _r32(m.Q), _r32(m.C), _r32(m.R), m.L, _r32(m.m0), _r32(m.P0))
        gpu = {"f32": {k: v.double().cpu().numpy() for k, v in r32.outputs[j].items()},
               "f64": {k: v.cpu().numpy() for k, v in r64.outputs[j].items()}}
        jobs.append((model, _r32(ys[j]), gpu))
    print(f"[gpu] reference runs on {oracle_pool.workers()} worker processes", flush=True)
    errs = oracle_pool.smoother_errors(jobs)
    worst = {"f32": 0.0, "f64": 0.0}
    for j, e in enumerate(errs):
        for tag, tol in (("f32", 1e-3), ("f64", 1e-8)):
            for k, (em, ep) in e[tag].items():
                worst[tag] = max(worst[tag], em, ep)
                assert em <= tol and ep <= tol, (
                    f"sequence {j} (nx={models[j].nx} L={models[j].L} N={ys[j].shape[0]}) {tag} {k}: "
                    f"mean err {em:.3e}, cov err {ep:.3e} (tol {tol:g})")
    print(f"[gpu] all 256 sequences against the reference: max rel err float32 {worst['f32']:.2e}, "
          f"float64 {worst['f64']:.2e}", flush=True)


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
            # float64 and float32 paths (same rounded inputs) against the reference's central differences
            t64 = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()  # noqa: E731
            ll64, dF64, dQ64, dR64 = srtm.loglik_grad(t64(r["A"]), t64(r["Q"]), t64(r["C"]), t64(r["R"]), 10,
                                                      t64(r["m0"]), t64(r["P0"]), t64(r["y"]))
            gA, gQ, gR = oracle.loglik_grad_fd(r["A"], r["Q"], r["C"], r["R"], 10, r["m0"], r["P0"], r["y"])
            o = b.outputs[j]
            for name, g32, g64, want in (("F", o["dF"], dF64, gA), ("Q", o["dQ"], dQ64, gQ), ("R", o["dR"], dR64, gR)):
                scale = max(1.0, np.max(np.abs(want)))
                e64 = np.max(np.abs(g64.cpu().numpy() - want)) / scale
                e32 = np.max(np.abs(g32.double().cpu().numpy() - want)) / scale
                print(f"[gpu]   d/d{name}: max rel err vs differences: float64 {e64:.2e}, float32 {e32:.2e} "
                      f"(scale {scale:.3g})", flush=True)
                assert e64 <= 1e-6, f"d/d{name} float64: {e64:.3e}"
                assert e32 <= 1e-3, f"d/d{name} float32: {e32:.3e}"
