"""Many independent sequences in one batched call (srtm_batch_plan + srtm_smooth_batch).

Each sequence of a batch must give bitwise the results of srtm_smooth on it alone (the same
kernels run on the same tiles), and match the float64 CPU reference to 1e-8 (float64) / 1e-3
(float32, reference on the rounded inputs).
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


def _problems(srtm, specs, dtype):
    probs, models, ys = [], [], []
    for nx, ny, L, N, seed in specs:
        m = wl.random_stable_model(nx, ny, L, seed)
        y = wl.simulate(m, N, seed + 1000)
        F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", dtype)
        yt = torch.as_tensor(y, dtype=torch.float64).to("cuda", dtype)
        probs.append((F, Q, H, R, L, m0, P0, yt))
        models.append(m)
        ys.append(y)
    return probs, models, ys


def _rounded(m, y, dtype):
    if dtype == torch.float64:
        return m, y
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    return wl.Model(r(m.A), r(m.Q), r(m.C), r(m.R), m.L, r(m.m0), r(m.P0), m.name), r(y)


def _check_batch(specs, dtype, oracle_max_n=1200):
    srtm = _srtm()
    probs, models, ys = _problems(srtm, specs, dtype)
    print(f"[gpu] batch of {len(specs)} sequences dtype={dtype}", flush=True)
    outs = srtm.smooth_batch(probs)
    torch.cuda.synchronize()
    for j, (pr, m, y) in enumerate(zip(probs, models, ys)):
        alone = srtm.smooth(*pr)
        torch.cuda.synchronize()
        for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
            assert torch.equal(outs[j][k], alone[k]), f"sequence {j}: {k} differs from the single call"
        if y.shape[0] <= oracle_max_n:
            mr, yr = _rounded(m, y, dtype)
            ref = oracle.srtm_smoother(mr.A, mr.Q, mr.C, mr.R, mr.L, mr.m0, mr.P0, yr)
            got = {k: v.double().cpu().numpy() for k, v in outs[j].items()}
            assert_close_states(got["ms_fast"], got["Ps_fast"], ref["ms_fast"], ref["Ps_fast"], TOL[dtype],
                                f"batch seq {j} fast")
            assert_close_states(got["ms_slow"], got["Ps_slow"], ref["ms_slow"], ref["Ps_slow"], TOL[dtype],
                                f"batch seq {j} slow")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batch_uneven_lengths(dtype):
    specs = [(4, 2, 20, 1, 1), (4, 2, 5, 300, 2), (4, 2, 10, 256, 3), (4, 2, 3, 257, 4), (4, 2, 20, 1100, 5),
             (4, 2, 7, 40, 6)]
    _check_batch(specs, dtype)


def test_batch_small_state():
    specs = [(2, 1, 10, 600, 11), (2, 1, 5, 33, 12), (2, 1, 20, 513, 13)]
    _check_batch(specs, torch.float64)


def test_batch_many_short_sequences():
    rng = np.random.default_rng(7)
    specs = [(3, 1, int(rng.choice([5, 10, 20])), int(rng.integers(1, 700)), 100 + j) for j in range(48)]
    _check_batch(specs, torch.float64, oracle_max_n=60)


def test_batch_long_and_short_with_multi_chunk_tile_scans():
    """A sequence of 70000 windows (274 tiles: two tiles per lane in both tile-level scans)
    next to short ones."""
    specs = [(2, 2, 4, 70000, 21), (2, 2, 6, 100, 22), (2, 2, 4, 1, 23)]
    _check_batch(specs, torch.float64, oracle_max_n=200)


def test_batch_repeated_launch_and_slow_only_outputs():
    srtm = _srtm()
    specs = [(4, 1, 5, 700, 31), (4, 1, 8, 90, 32)]
    probs, _, _ = _problems(srtm, specs, torch.float64)
    b = srtm.Batch(probs, fast=False, slow=True)
    b.launch()
    torch.cuda.synchronize()
    first = [{k: v.clone() for k, v in o.items()} for o in b.outputs]
    b.launch()
    torch.cuda.synchronize()
    b.check()
    for j, pr in enumerate(probs):
        alone = srtm.smooth(*pr, fast=False)
        for k in ("ms_slow", "Ps_slow"):
            assert torch.equal(b.outputs[j][k], alone[k])
            assert torch.equal(b.outputs[j][k], first[j][k])
        assert "ms_fast" not in b.outputs[j]


def test_batch_state_six_float32():
    specs = [(6, 1, 5, 400, 41), (6, 1, 20, 90, 42), (6, 1, 10, 257, 43)]
    _check_batch(specs, torch.float32)


def test_batch_runner_graph_replays_match_eager():
    """The captured launch sequence (multi-stream, two segments per size group) replayed three
    times, with unrelated eager work and synchronisations between replays, reproduces the
    eager results bitwise every time."""
    srtm = _srtm()
    from paper_2410_00627_amd import batching
    specs = [(2, 1, 5, 300, 51), (4, 1, 10, 700, 52), (2, 1, 20, 90, 53), (4, 1, 5, 1, 54), (4, 1, 7, 260, 55)]
    probs, _, _ = _problems(srtm, specs, torch.float64)
    eager = batching.BatchRunner(probs, segments=2, multi_stream=True, graph=False)
    eager.run()
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in eager.outputs]
    g = batching.BatchRunner(probs, segments=2, multi_stream=True, graph=True)
    for rep in range(3):
        for o in g.outputs:
            for v in o.values():
                v.fill_(float("nan"))
        x = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        (x @ x).sum().item()
        print(f"[gpu] graph replay {rep}", flush=True)
        g.run()
        torch.cuda.synchronize()
        for j, o in enumerate(g.outputs):
            for k in ref[j]:
                assert torch.equal(o[k], ref[j][k]), f"replay {rep}, sequence {j}, {k}"
    g.check()


def test_graph_record_error_leaves_the_stream_usable():
    """An exception raised while a graph is being recorded ends the capture: the same Graph then
    records the batch normally, and its replay matches the eager call bitwise."""
    srtm = _srtm()
    specs = [(4, 1, 10, 300, 61), (4, 1, 5, 40, 62)]
    probs, _, _ = _problems(srtm, specs, torch.float64)
    b = srtm.Batch(probs)
    b.launch()
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in b.outputs]
    g = srtm.Graph(torch.device("cuda"))

    def failing():
        b.launch()
        raise RuntimeError("planted failure while recording")

    with pytest.raises(RuntimeError, match="planted failure"):
        g.record(failing)
    assert g.exec is None
    print("[gpu] capture ended after the planted failure; recording again", flush=True)
    g.record(b.launch)
    for o in b.outputs:
        for v in o.values():
            v.fill_(float("nan"))
    g.replay()
    torch.cuda.synchronize()
    for j, o in enumerate(b.outputs):
        for k in ref[j]:
            assert torch.equal(o[k], ref[j][k]), f"sequence {j}, {k}"


def test_autotune_picks_a_configuration_with_identical_results():
    srtm = _srtm()
    from paper_2410_00627_amd import batching
    specs = [(2, 1, 5, 400, 61), (4, 1, 10, 300, 62), (6, 1, 5, 120, 63), (2, 1, 20, 50, 64)]
    probs, _, _ = _problems(srtm, specs, torch.float32)
    log = []
    r = batching.autotune(probs, segments=(1, 2), reps=2, log=log)
    assert len(log) >= 4 and all(e["seconds"] > 0 for e in log)
    r.run()
    torch.cuda.synchronize()
    r.check()
    for j, pr in enumerate(probs):
        alone = srtm.smooth(*pr)
        for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
            assert torch.equal(r.outputs[j][k], alone[k])


def _mixed_problems(srtm, dtype):
    """Sequences of six (nx, ny) pairs and all three kinds: time-invariant, known inputs and
    per-window models, with one-window, ragged and multi-tile lengths."""
    specs = [  # nx, ny, L, N, seed, kind
        (2, 1, 5, 300, 71, "plain"), (4, 2, 10, 700, 72, "plain"), (6, 1, 5, 120, 73, "plain"),
        (1, 1, 20, 90, 74, "plain"), (3, 2, 7, 257, 75, "plain"), (4, 2, 20, 1, 76, "plain"),
        (4, 1, 10, 400, 77, "inputs"), (2, 2, 3, 530, 78, "inputs"),
        (2, 1, 5, 300, 79, "tv"), (4, 2, 10, 260, 80, "tv"), (3, 1, 4, 1100, 81, "plain")]
    conv = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64)).to("cuda", dtype).contiguous()  # noqa: E731
    probs, refs = [], []
    for nx, ny, L, N, seed, kind in specs:
        if kind == "tv":
            m = wl.time_varying_model(nx, ny, L, N, seed)
            y = wl.simulate_tv(m, seed + 1)
            probs.append((conv(m.A), conv(m.Q), conv(m.C), conv(m.R), L, conv(m.m0), conv(m.P0), conv(y)))
            refs.append((kind, m, y, None, None))
        else:
            m = wl.random_stable_model(nx, ny, L, seed)
            B = u = None
            if kind == "inputs":
                B, u = wl.random_inputs(nx, 2, L, N, seed + 2)
            y = wl.simulate(m, N, seed + 1, B=B, u=u)
            pr = (conv(m.A), conv(m.Q), conv(m.C), conv(m.R), L, conv(m.m0), conv(m.P0), conv(y))
            probs.append(pr + ((conv(B), conv(u)) if kind == "inputs" else ()))
            refs.append((kind, m, y, B, u))
    return probs, refs


def _alone_any(srtm, pr):
    if len(pr) == 10:
        return srtm.smooth(*pr[:8], B=pr[8], u=pr[9])
    return srtm.smooth(*pr)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_mixed_batch_one_launch_set(dtype):
    """Six (nx, ny) pairs, inputs and per-window models in ONE srtm_smooth_batch_ex call (six
    launches): every sequence bitwise equal to its own single call, and equal to the float64
    reference (on the rounded inputs) within 1e-8 / 1e-3."""
    srtm = _srtm()
    probs, refs = _mixed_problems(srtm, dtype)
    b = srtm.BatchEx(probs)
    print(f"[gpu] mixed batch of {b.nseq} sequences, {b.ntiles} tiles, {dtype}", flush=True)
    b.launch()
    torch.cuda.synchronize()
    b.check()
    r = (lambda a: a) if dtype == torch.float64 else (
        lambda a: None if a is None else np.asarray(a, dtype=np.float32).astype(np.float64))
    for j, (pr, (kind, m, y, B, u)) in enumerate(zip(probs, refs)):
        alone = _alone_any(srtm, pr)
        torch.cuda.synchronize()
        for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
            assert torch.equal(b.outputs[j][k], alone[k]), f"sequence {j} ({kind}): {k} differs from the single call"
        if kind == "tv":
            ref = oracle.srtm_smoother_tv(r(m.A), r(m.Q), r(m.C), r(m.R), m.L, r(m.m0), r(m.P0), r(y))
        else:
            ref = oracle.srtm_smoother(r(m.A), r(m.Q), r(m.C), r(m.R), m.L, r(m.m0), r(m.P0), r(y), B=r(B), u=r(u))
        got = {k: v.double().cpu().numpy() for k, v in b.outputs[j].items()}
        assert_close_states(got["ms_fast"], got["Ps_fast"], ref["ms_fast"], ref["Ps_fast"], TOL[dtype],
                            f"mixed seq {j} ({kind}) fast")
        assert_close_states(got["ms_slow"], got["Ps_slow"], ref["ms_slow"], ref["Ps_slow"], TOL[dtype],
                            f"mixed seq {j} ({kind}) slow")


def test_mixed_runner_graph_replays_match_eager():
    """BatchRunner(mixed=True): two segments on two streams recorded once as a HIP graph through
    the library's graph entry points and replayed three times (eager work between replays):
    bitwise the eager results every time; the grouped runner gives the same results."""
    srtm = _srtm()
    from paper_2410_00627_amd import batching
    probs, _ = _mixed_problems(srtm, torch.float64)
    eager = batching.BatchRunner(probs, segments=2, multi_stream=True, mixed=True)
    eager.run()
    torch.cuda.synchronize()
    eager.check()
    assert eager.describe()["launches"] == 12
    ref = [{k: v.clone() for k, v in o.items()} for o in eager.outputs]
    grouped = batching.BatchRunner(probs)
    grouped.run()
    torch.cuda.synchronize()
    for j, o in enumerate(grouped.outputs):
        for k in ref[j]:
            assert torch.equal(o[k], ref[j][k]), f"grouped runner, sequence {j}, {k}"
    g = batching.BatchRunner(probs, segments=2, multi_stream=True, graph=True, mixed=True)
    for rep in range(3):
        for o in g.outputs:
            for v in o.values():
                v.fill_(float("nan"))
        x = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        (x @ x).sum().item()
        print(f"[gpu] mixed graph replay {rep}", flush=True)
        g.run()
        torch.cuda.synchronize()
        for j, o in enumerate(g.outputs):
            for k in ref[j]:
                assert torch.equal(o[k], ref[j][k]), f"replay {rep}, sequence {j}, {k}"
    g.check()


def test_mixed_batch_nan_sequence_fails_alone():
    """A NaN measurement in one sequence of a mixed batch sets only that sequence's info word
    (non-finite bit) and leaves every other sequence bitwise equal to its single call."""
    srtm = _srtm()
    probs, _ = _mixed_problems(srtm, torch.float64)
    bad = 3
    y = probs[bad][7].clone()
    y[y.shape[0] // 2, 0] = float("nan")
    probs[bad] = probs[bad][:7] + (y,) + probs[bad][8:]
    b = srtm.BatchEx(probs)
    b.launch()
    torch.cuda.synchronize()
    info = b.info.cpu().tolist()
    assert info[bad] & 8 and all(v == 0 for j, v in enumerate(info) if j != bad), info
    for j, pr in enumerate(probs):
        if j == bad:
            continue
        alone = _alone_any(srtm, pr)
        for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
            assert torch.equal(b.outputs[j][k], alone[k]), f"sequence {j}: {k} changed by the NaN sequence"
