"""Serving loop: requests of different lengths arriving over time, admitted against an HBM
budget and launched in continuous batches on several streams. Each request's result must be
the same alone and in the mix: bitwise equal to srtm_smooth on it alone (the same kernels run
on the same tiles), and equal to the float64 CPU reference within 1e-8 for small requests.
"""
import numpy as np
import pytest

import oracle
from paper_2410_00627_amd import workloads as wl
from conftest import assert_close_states

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_00627_amd import serving, srtm
    srtm.lib()
    return serving, srtm


def _requests(serving, n, seed, *, burst=8, gap_s=2e-4, max_n=2500, L=10):
    rng = np.random.default_rng(seed)
    model = wl.random_stable_model(4, 2, L, 2024, rho=0.99, q=0.01, r=0.05)
    pool = wl.simulate(model, max_n, seed + 1)
    reqs, t = [], 0.0
    for j in range(n):
        if j >= burst:                      # the first `burst` arrive together, then Poisson
            t += rng.exponential(gap_s)
        N = int(rng.integers(1, max_n + 1))
        off = int(rng.integers(0, max_n - N + 1))
        reqs.append(serving.Request(rid=j, arrival=t, F=model.A, Q=model.Q, H=model.C, R=model.R, L=L,
                                    m0=model.m0, P0=model.P0, y=pool[off:off + N].copy()))
    return model, reqs


def _alone(srtm, r, dtype):
    conv = lambda a: torch.as_tensor(a, dtype=torch.float64).to("cuda", dtype).contiguous()  # noqa: E731
    return srtm.smooth(conv(r.F), conv(r.Q), conv(r.H), conv(r.R), r.L, conv(r.m0), conv(r.P0), conv(r.y))


def _r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


CASES = [(512, 3, torch.float64), (24, 2, torch.float64), (512, 3, torch.float32), (12, 2, torch.float32)]


@pytest.mark.parametrize("budget_mb,streams,dtype", CASES,
                         ids=["roomy-f64", "tight-f64", "roomy-f32", "tight-f32"])
def test_serving_results_same_alone_and_in_mix(budget_mb, streams, dtype):
    import oracle_pool
    serving, srtm = _need()
    model, reqs = _requests(serving, 36, 5 + budget_mb + (dtype == torch.float32))
    srv = serving.Server(4, 2, dtype, hbm_budget=budget_mb << 20, streams=streams, max_batch=8)
    print(f"[gpu] serving {len(reqs)} requests, budget {budget_mb} MB, {streams} streams, {dtype}", flush=True)
    stats = serving.serve(srv, reqs)
    print(f"[gpu] serving stats {stats}", flush=True)
    assert stats["failed"] == [] and all(r.done is not None for r in reqs)
    assert srv.arena.used == 0 and srv.arena.free == [[0, srv.arena.size]]
    assert stats["batches"] < len(reqs)       # some requests shared a launch
    for r in reqs:
        alone = _alone(srtm, r, dtype)
        for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
            assert torch.equal(r.outputs[k], alone[k]), f"request {r.rid}: {k} differs from the request alone"
    rnd = (lambda a: np.asarray(a, dtype=np.float64)) if dtype == torch.float64 else _r32
    jobs = [((rnd(r.F), rnd(r.Q), rnd(r.H), rnd(r.R), r.L, rnd(r.m0), rnd(r.P0)), rnd(r.y),
             {"gpu": {k: v.double().cpu().numpy() for k, v in r.outputs.items()}}) for r in reqs]
    tol = 1e-8 if dtype == torch.float64 else 1e-3
    worst = 0.0
    for r, e in zip(reqs, oracle_pool.smoother_errors(jobs)):
        for k, (em, ep) in e["gpu"].items():
            worst = max(worst, em, ep)
            assert em <= tol and ep <= tol, f"request {r.rid} (N={r.y.shape[0]}) {k}: {em:.2e} {ep:.2e}"
    print(f"[gpu] every request against the reference: max rel err {worst:.2e} (tol {tol:g})", flush=True)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_serving_nan_request_fails_alone(dtype):
    """One request of a burst carries a NaN measurement: it is reported failed (info bit 8),
    and every other request, including those launched in the same batch, is bitwise equal to
    its result alone."""
    serving, srtm = _need()
    model, reqs = _requests(serving, 12, 77, burst=12, max_n=1500)
    bad = reqs[3]
    bad.y = bad.y.copy()
    bad.y[bad.y.shape[0] // 2, 0] = np.nan
    srv = serving.Server(4, 2, dtype, hbm_budget=256 << 20, streams=2, max_batch=8)
    print(f"[gpu] serving with a NaN request, {dtype}", flush=True)
    stats = serving.serve(srv, reqs)
    assert stats["failed"] == [bad.rid], stats["failed"]
    assert bad.info & 8
    shared = [r for r in reqs if r is not bad and r.batch == bad.batch]
    assert len(shared) >= 1, "the NaN request did not share its launch"
    for r in reqs:
        if r is bad:
            continue
        assert r.info == 0
        alone = _alone(srtm, r, dtype)
        for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
            assert torch.equal(r.outputs[k], alone[k]), f"request {r.rid}: {k} changed by the NaN request"


def test_serving_rejects_a_request_larger_than_the_budget():
    serving, srtm = _need()
    _, reqs = _requests(serving, 1, 9, max_n=2000)
    reqs[0].y = np.zeros((200000, 2))
    srv = serving.Server(4, 2, torch.float32, hbm_budget=8 << 20, streams=1)
    with pytest.raises(srtm.SrtmError):
        srv.submit(reqs[0])
